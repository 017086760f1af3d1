"""Benchmark: Lasso solves/s to duality gap 1e-6 on one MI355X, screened vs plain.

Headline workload (one step): a 2000 x 10000 Gaussian dictionary with unit-norm atoms
stored in FP32, one Bernoulli(0.02)-Gaussian signal at 20 dB SNR (unit norm), solved for
lambda / lambda_* in {0.1, 0.3, 0.5, 0.7, 0.9} by FISTA with dynamic DST3 screening
until the duality-gap certificate is <= 1e-6 ||y||^2.  Inputs are resident in HBM
before the timed region; every solve runs through the C-ABI (lasso kernels in HIP).

Batched workload (reported under "batched"): the same dictionary rounded to bfloat16,
256 signals from the same generator with lambda / lambda_* uniform in [0.1, 0.9], all
solved together by the matrix-core path to the same gap.

Printed JSON line: solves/s (value), the same solves without screening (plain), p50/p99
latency per solve, the HBM roofline of the dominant kernel (the screened correlation
GEMV) from HIP events, the batched leg with the matrix-core roofline of its Z = D^T Theta
GEMM, and the FP64 oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1412_4080_amd import datagen  # noqa: E402  (seeded input generators only)

N, K = 2000, 10000
RATIOS = (0.1, 0.3, 0.5, 0.7, 0.9)
GAP_TOL = 1e-6
HBM_PEAK_GBS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0
NB = 256  # signals of the batched leg
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_corr_lasso_2000x10000_traffic.json")


def _dev(D32, y32):
    import torch
    Dd = torch.from_numpy(np.ascontiguousarray(D32.T).astype(np.float32)).cuda().T
    yd = torch.from_numpy(y32.astype(np.float32)).cuda()
    return Dd, yd


def run_steps(binding, Dd, ys, steps, test, L, lat=None, step="constant", iters=None,
              rule="fista", bb_memory=0):
    import torch
    n = 0
    for s in range(steps):
        yd = ys[s % len(ys)]
        for r in RATIOS:
            t0 = time.perf_counter()
            own_step = step != "constant" or rule == "sparsa"   # CP takes L (its default steps)
            x, info, _, _ = binding.solve_one(Dd, yd, r, rule=rule, test=test,
                                              step_L=0.0 if own_step else L,
                                              gap_tol=GAP_TOL, max_iter=20000, trace=False,
                                              screened=False, step=step, bb_memory=bb_memory)
            if lat is not None:
                lat.append(time.perf_counter() - t0)
            if info["status"] != 0:
                raise RuntimeError(f"solve did not converge: {info}")
            if iters is not None:
                iters.append(info["iters"])
            n += 1
    torch.cuda.synchronize()
    return n


def columns_of(ys):
    """Each signal repeated once per lambda ratio: the N x 5 column-major right-hand sides of
    one step's lasso_solve call (built before any timed region, resident in HBM)."""
    return [y.reshape(-1, 1).repeat(1, len(RATIOS)).T.contiguous().T for y in ys]


def run_steps_concurrent(binding, Dd, Ys, steps, test, L):
    """One step = one signal at the five lambda ratios through one lasso_solve call: the five
    independent single-signal solves run concurrently on the library's solve lanes."""
    import torch
    n = 0
    for s in range(steps):
        _, infos = binding.solve(Dd, Ys[s % len(Ys)], RATIOS, rule="fista", test=test,
                                 step_L=L, gap_tol=GAP_TOL, max_iter=20000)
        bad = [i for i in infos if i["status"] != 0]
        if bad:
            raise RuntimeError(f"solve did not converge: {bad[0]}")
        n += len(infos)
    torch.cuda.synchronize()
    return n


def batched_setup(binding, D):
    import torch
    Dbf = datagen.to_storage(D, "bf16")
    Dd = torch.from_numpy(np.ascontiguousarray(Dbf.T)).to(device="cuda", dtype=torch.bfloat16).T
    ys = np.stack([datagen.to_storage(datagen.lasso_signal(D, j)[0], "f32") for j in range(NB)])
    Y = torch.from_numpy(ys.astype(np.float32)).cuda().T
    ratios = datagen.lambda_ratios(NB, 0.1, 0.9, datagen.LAMBDA_SEED0)
    L = binding.spectral_norm_sq(Dd, 300)

    def one():
        X, infos = binding.solve(Dd, Y, ratios, step_L=L, gap_tol=GAP_TOL, max_iter=20000)
        if any(i["status"] != 0 for i in infos):
            raise RuntimeError("batched solve did not converge")
        return X, infos
    return one


STREAM_SIGNALS = 1024


def batched_stream_leg(binding, D, steps=2):
    """Continuous batching: 1024 signals of the batched workload's generator through the
    default 512 resident slots of the bfloat16 path (a finished signal's slot takes the next
    waiting one), lambda / lambda_* uniform in [0.1, 0.9], gap 1e-6: solves/s."""
    import torch
    Dbf = datagen.to_storage(D, "bf16")
    Dd = torch.from_numpy(np.ascontiguousarray(Dbf.T)).to(device="cuda", dtype=torch.bfloat16).T
    ys = np.stack([datagen.to_storage(datagen.lasso_signal(D, j)[0], "f32")
                   for j in range(STREAM_SIGNALS)])
    Y = torch.from_numpy(ys.astype(np.float32)).cuda().T
    ratios = datagen.lambda_ratios(STREAM_SIGNALS, 0.1, 0.9, datagen.LAMBDA_SEED0)
    L = binding.spectral_norm_sq(Dd, 300)

    def one():
        _, infos = binding.solve(Dd, Y, ratios, step_L=L, gap_tol=GAP_TOL, max_iter=20000)
        if any(i["status"] != 0 for i in infos):
            raise RuntimeError("streamed batched solve did not converge")
        return infos
    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = one()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it = [i["iters"] for i in infos]
    return {"workload": "lasso_fista_dst3_gaussian_2000x10000_bf16_stream1024_slots512",
            "signals": STREAM_SIGNALS, "slots": 512,
            "solves_per_s": round(STREAM_SIGNALS * steps / dt, 2),
            "ms_per_stream": round(dt * 1e3 / steps, 3),
            "iterations": {"max": int(max(it)), "mean": round(float(np.mean(it)), 1)}}


def served_batched_leg(binding, D, n_sat=1024, n_open=1500, warm=200, seed=datagen.ARRIVAL_SEED):
    """Requests for the batched workload's dictionary (2000 x 10000, stored in bfloat16;
    signals of its generator, lambda / lambda_* uniform in [0.1, 0.9], FISTA + DST3 to gap
    1e-6) through the server: with a batched engine of 512 resident signals (requests join
    it as slots free up) and with the eight single-signal workers alone.  Saturation (all
    requests submitted at once), then Poisson arrivals at 0.5 x and 0.9 x the engine's
    saturation rate: solves/s and p50/p99 latency (submit to result, server clock)."""
    import torch
    rng = np.random.default_rng(seed + 1)
    ys = [datagen.to_storage(datagen.lasso_signal(D, j)[0], "f32").astype(np.float32)
          for j in range(256)]
    Dd = torch.from_numpy(np.ascontiguousarray(datagen.to_storage(D, "f32").T)).to(
        device="cuda", dtype=torch.float32).T

    def draw(n):
        return [(int(rng.integers(len(ys))), float(rng.uniform(0.1, 0.9))) for _ in range(n)]

    def run(S, did, reqs, gaps=None, skip=0):
        pending, done = {}, []

        def drain():
            for rid in list(pending):
                got = S.poll(rid, did)
                if got is not None:
                    if got[1]["status"] != 0:
                        raise RuntimeError(f"served solve did not converge: {got[1]}")
                    if pending[rid]:
                        done.append(got[1])
                    del pending[rid]
        t_next = t_start = time.perf_counter()
        for k, (j, r) in enumerate(reqs):
            if gaps is not None:
                t_next += gaps[k]
                while time.perf_counter() < t_next:
                    drain()
            if k == skip:
                t_start = time.perf_counter()
            rid = S.submit(did, ys[j], r, test="dst3", gap_tol=GAP_TOL, max_iter=20000)
            pending[rid] = k >= skip
        while pending:
            drain()
            time.sleep(0.0002)
        return done, time.perf_counter() - t_start

    def summary(done, dt):
        lat = np.array([i["queue_ms"] + i["run_ms"] for i in done])
        return {"solves_per_s": round(len(done) / dt, 1), "requests": len(done),
                "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                               "p99": round(float(np.percentile(lat, 99)), 3)}}

    out = {"workload": "serving_lasso_fista_dst3_gaussian_2000x10000_bf16",
           "requests_saturation": n_sat}
    sat_rate = None
    for name, bslots in (("batched_engine", 512), ("workers_only", 0)):
        S = binding.Server(max_slots=8, hbm_budget_bytes=24 << 30, max_queue=1 << 14,
                           batch_slots=bslots)
        did = S.add_dict(Dd, store="bf16")
        torch.cuda.synchronize()
        run(S, did, draw(64))                     # warm-up (autotuner, graph, workspaces)
        done, dt = run(S, did, draw(n_sat))
        leg = {"batch_slots": bslots, "worker_slots": 8, "saturation": summary(done, dt)}
        if sat_rate is None:
            sat_rate = len(done) / dt
        opens = []
        for frac in (0.5, 0.9):
            reqs = draw(warm + n_open)
            gaps = rng.exponential(1.0 / (frac * sat_rate), size=len(reqs))
            done, dt = run(S, did, reqs, gaps, skip=warm)
            opens.append(dict(offered_per_s=round(frac * sat_rate, 1), **summary(done, dt)))
        leg["open_loop"] = opens
        S.close()
        out[name] = leg
    out["saturation_engine_over_workers"] = round(
        out["batched_engine"]["saturation"]["solves_per_s"] /
        out["workers_only"]["saturation"]["solves_per_s"], 2)
    return out


def batched_roofline(binding, one):
    """One instrumented batched solve: matrix-core roofline of the Z = D^T Theta GEMM."""
    binding.stats_reset()
    binding.stats_enable(True)
    one()
    binding.stats_enable(False)
    st = binding.stats_read()
    z, th = st[binding.STAT_BATCH], st[binding.STAT_BATCH_THETA]
    z_ms = z["ms"] / max(z["launches"], 1)
    z_flops = z["flops"] / max(z["launches"], 1)
    achieved = z_flops / (z_ms * 1e-3) / 1e12 if z_ms > 0 else 0.0
    k, ta, ts = binding.batch_shape()
    return {"bound": "mfma", "kernel": "k_b_zgemm", "block": f"{ta} atoms x {ts} signals",
            "block_shape_index": k, "achieved": round(achieved, 2),
            "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / BF16_MFMA_PEAK_TFLOPS, 4), "traffic": None,
            "avg_launch_us": round(z_ms * 1e3, 3),
            "event_avg_launch_us": round(z["ms_event"] / max(z["launches"], 1) * 1e3, 3),
            "algorithmic_flops_per_launch": round(z_flops, 1),
            "launches": z["launches"],
            "theta_gather_event_avg_us": round(th["ms"] / max(th["launches"], 1) * 1e3, 3)}


def batched_leg(binding, D, steps, warmup):
    """256 signals solved together on the bfloat16 matrix-core path, `steps` times."""
    import torch
    one = batched_setup(binding, D)
    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        X, infos = one()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    dt = time.perf_counter() - t0
    iters = [i["iters"] for i in infos]
    ratios = datagen.lambda_ratios(NB, 0.1, 0.9, datagen.LAMBDA_SEED0)
    return {
        "workload": "lasso_fista_dst3_gaussian_2000x10000_bf16_batch256",
        "signals": NB, "solves_per_s": round(NB * steps / dt, 2),
        "ms_per_batch": round(dt * 1e3 / steps, 3),
        "batch_latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                             "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
        "iterations": {"max": int(max(iters)), "mean": round(float(np.mean(iters)), 1)},
        "roofline": batched_roofline(binding, one),
        "precision": batched_precision(binding, D, infos, X, ratios),
    }


def batched_groups_leg(binding, D, steps=2, n_plain=8):
    """The Group-Lasso on the bfloat16 matrix-core path: the group workload's dictionary
    (2000 x 10000, 1000 contiguous groups of 10, w_g = sqrt(10)) stored in bfloat16, 256
    signals of its generator with lambda / lambda_* uniform in [0.1, 0.9], FISTA + DGST3 to
    gap 1e-6: solves/s, against the same solves one at a time on the FP32 single-signal
    path without screening (a sample of n_plain of them)."""
    import torch
    gp = datagen.contiguous_groups(K, 10)
    Dbf = datagen.to_storage(D, "bf16")
    Dd = torch.from_numpy(np.ascontiguousarray(Dbf.T)).to(device="cuda", dtype=torch.bfloat16).T
    ys = np.stack([datagen.to_storage(datagen.group_signal(D, gp, j)[0], "f32") for j in range(NB)])
    Y = torch.from_numpy(ys.astype(np.float32)).cuda().T
    ratios = datagen.lambda_ratios(NB, 0.1, 0.9, datagen.LAMBDA_SEED0)
    L = binding.spectral_norm_sq(Dd, 300)

    def one():
        X, infos = binding.solve(Dd, Y, ratios, group_ptr=gp, rule="fista", test="dst3",
                                 step_L=L, gap_tol=GAP_TOL, max_iter=20000)
        if any(i["status"] != 0 for i in infos):
            raise RuntimeError("batched group solve did not converge")
        return infos
    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos = one()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    it = [i["iters"] for i in infos]
    # plain single-signal FP32 solves of a sample of the same signals
    D32 = torch.from_numpy(np.ascontiguousarray(datagen.to_storage(D, "f32").T)).to(
        device="cuda", dtype=torch.float32).T
    L32 = binding.spectral_norm_sq(D32, 300)
    yd = [torch.from_numpy(ys[j].astype(np.float32)).cuda() for j in range(n_plain)]
    binding.solve_one(D32, yd[0], float(ratios[0]), group_ptr=gp, rule="fista", test="none",
                      step_L=L32, gap_tol=GAP_TOL, max_iter=50000, trace=False, screened=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for j in range(n_plain):
        binding.solve_one(D32, yd[j], float(ratios[j]), group_ptr=gp, rule="fista", test="none",
                          step_L=L32, gap_tol=GAP_TOL, max_iter=50000, trace=False, screened=False)
    torch.cuda.synchronize()
    plain = n_plain / (time.perf_counter() - t1)
    sps = NB * steps / dt
    return {"workload": "group_lasso_fista_dgst3_gaussian_2000x10000_bf16_groups10_batch256",
            "signals": NB, "solves_per_s": round(sps, 2), "ms_per_batch": round(dt * 1e3 / steps, 3),
            "iterations": {"max": int(max(it)), "mean": round(float(np.mean(it)), 1)},
            "plain_single_fp32_solves_per_s": round(plain, 2),
            "over_plain_single": round(sps / plain, 2)}


INSTR_SIGNALS = 6   # signals of the instrumented pass (x 5 ratios), whatever --steps is
A_BUCKETS = (0, 1000, 2500, 5000, 7500, 10001)


def single_roofline(binding, Dd, ys, L):
    """Instrumented pass over a fixed sample (INSTR_SIGNALS signals x RATIOS, one iteration
    per chunk so that no launch runs past a solve's stop): HBM roofline of the correlation
    kernel from the device-clock spans of every launch, and per range of active atoms."""
    binding.stats_reset()
    binding.stats_enable(True)
    run_steps(binding, Dd, ys[:INSTR_SIGNALS], INSTR_SIGNALS, "dst3", L)
    binding.stats_enable(False)
    st = binding.stats_read()[binding.STAT_CORR]
    allrecs = binding.stats_launches()
    recs = [r for r in allrecs if r["kernel"] == binding.STAT_CORR]
    rres = [r for r in allrecs if r["kernel"] == binding.STAT_RESID]
    rit = [r for r in allrecs if r["kernel"] == binding.STAT_ITER]
    avg_ms = st["ms"] / max(st["launches"], 1)
    ev_ms = st["ms_event"] / max(st["launches"], 1)
    bytes_per = st["bytes"] / max(st["launches"], 1)
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    buckets = []
    for lo, hi in zip(A_BUCKETS[:-1], A_BUCKETS[1:]):
        sel = [r for r in recs if lo <= r["n_atoms"] < hi]
        if sel:
            b = sum(r["bytes"] for r in sel)
            t = sum(r["ms"] for r in sel) * 1e-3
            row = {"active_atoms": [lo, hi - 1], "launches": len(sel),
                   "avg_launch_us": round(t / len(sel) * 1e6, 3),
                   "achieved": round(b / t / 1e9, 1), "frac": round(b / t / 1e9 / HBM_PEAK_GBS, 4)}
            # the iteration: the correlation and the residual pass after it (HIP event times
            # of the two dispatches, which include the dispatch overhead)
            sr = [r["ms"] for r in rres if lo <= r["n_atoms"] < hi]
            si = [r["ms"] for r in rit if lo <= r["n_atoms"] < hi]
            if sr and si:
                row["resid_event_us"] = round(float(np.mean(sr)) * 1e3, 3)
                row["iteration_event_us"] = round(float(np.mean(si)) * 1e3, 3)
            buckets.append(row)
    out = {"bound": "hbm", "kernel": "k_corr_lasso",
           "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
           "avg_launch_us": round(avg_ms * 1e3, 3),
           "event_avg_launch_us": round(ev_ms * 1e3, 3),
           "algorithmic_bytes_per_launch": round(bytes_per, 1),
           "launches": st["launches"],
           "sample": f"{INSTR_SIGNALS} signals x {len(RATIOS)} lambda ratios, one iteration per chunk",
           "by_active_atoms": buckets}
    prof = profile_record()
    if prof is not None:
        # counters and rocprof durations of the same sample (profiles/): HBM bytes per launch
        # next to that run's own algorithmic bytes, and the frac from rocprof's average
        out["traffic"] = prof["traffic_bytes_per_launch"]
        out["traffic_run_algorithmic_bytes_per_launch"] = prof["algorithmic_bytes_per_launch"]
        out["traffic_over_algorithmic"] = round(prof["traffic_bytes_per_launch"] /
                                                prof["algorithmic_bytes_per_launch"], 4)
        r_us = prof["rocprof_avg_launch_us"]
        out["rocprof_avg_launch_us"] = r_us
        out["rocprof_frac"] = round(prof["algorithmic_bytes_per_launch"] / (r_us * 1e-6) / 1e9
                                    / HBM_PEAK_GBS, 4)
    return out


# Serving mix: (N, K, group size or 0, stored dtype) of the eight resident dictionaries.
SERVE_DICTS = ((256, 1000, 0, "f32"), (256, 5000, 10, "bf16"), (1024, 5000, 0, "bf16"),
               (1024, 20000, 10, "f32"), (2048, 20000, 0, "f32"), (2048, 40000, 10, "bf16"),
               (4096, 20000, 0, "bf16"), (4096, 40000, 10, "f32"))
SERVE_POOL = 16  # signals per dictionary, reused round-robin by the requests


def serve_inputs(seed=datagen.DICT_SEED):
    """Unit-norm Gaussian dictionaries and pools of unit-norm observations (2% active atoms
    or groups with N(0,1) coefficients, 20 dB noise), drawn on the device from seeded
    generators: the serving mix is too large to draw on the host in the bench's time."""
    import torch
    g = torch.Generator(device="cuda")
    out = []
    for k, (n, kk, gs, dt) in enumerate(SERVE_DICTS):
        g.manual_seed(seed * 1000 + k)
        D = torch.randn(kk, n, generator=g, device="cuda")
        D /= D.norm(dim=1, keepdim=True)
        Dt = D.T                                   # N x K column-major view
        units = kk // gs if gs else kk
        mask = torch.rand(SERVE_POOL, units, generator=g, device="cuda") < 0.02
        mask[:, 0] |= ~mask.any(dim=1)             # at least one active unit
        if gs:
            mask = mask.repeat_interleave(gs, dim=1)
        X0 = torch.randn(SERVE_POOL, kk, generator=g, device="cuda") * mask
        Yc = X0 @ D                                # SERVE_POOL x N clean signals
        noise = torch.randn(Yc.shape, generator=g, device="cuda")
        noise *= (Yc.norm(dim=1, keepdim=True) / noise.norm(dim=1, keepdim=True)) * 10 ** (-20 / 20)
        Y = Yc + noise
        Y /= Y.norm(dim=1, keepdim=True)
        gp = np.arange(0, kk + 1, gs, dtype=np.int64) if gs else None
        out.append((Dt, gp, dt, Y.cpu().numpy().astype(np.float32)))
    torch.cuda.synchronize()
    return out


def served_leg(binding, n_closed=320, n_open=1000, warm=100, slots=8, n_plain=96,
               seed=datagen.ARRIVAL_SEED, batch_slots=0):
    """Closed-loop saturation, then open-loop Poisson arrivals at 0.5x and 0.9x of it; the
    baseline is requests of the same mix solved one at a time without screening.  With
    batch_slots > 0 the two bfloat16 Lasso dictionaries of the mix run on batched engines
    (the baseline is then not repeated)."""
    inputs = serve_inputs()
    rng = np.random.default_rng(seed)

    def draw(n, g=rng):
        return [(int(g.integers(len(inputs))), int(g.integers(SERVE_POOL)),
                 float(g.uniform(0.1, 0.9))) for _ in range(n)]

    def server(nslots, bslots=0):
        S = binding.Server(max_slots=nslots, hbm_budget_bytes=24 << 30, max_queue=1 << 14,
                           batch_slots=bslots)
        return S, [S.add_dict(Dt, group_ptr=gp, store=dt) for (Dt, gp, dt, _) in inputs]

    def drain(S, ids, pending, done):
        for rid in list(pending):
            d = pending[rid]
            got = S.poll(rid, ids[d])
            if got is not None:
                if got[1]["status"] != 0:
                    raise RuntimeError(f"served solve did not converge: {got[1]}")
                done.append((d, got[1]))
                del pending[rid]

    def run(S, ids, reqs, gaps=None, skip=0, test="dst3"):
        """Submit reqs (all at once, or with the given inter-arrival gaps) and wait."""
        pending, done = {}, []
        t_next = t_start = time.perf_counter()
        for k, (d, j, r) in enumerate(reqs):
            if gaps is not None:
                t_next += gaps[k]
                while time.perf_counter() < t_next:
                    drain(S, ids, pending, done)
            if k == skip:
                t_start = time.perf_counter()
                done.clear()
            rid = S.submit(ids[d], inputs[d][3][j], r, test=test, gap_tol=GAP_TOL, max_iter=20000)
            pending[rid] = d
        while pending:
            drain(S, ids, pending, done)
            time.sleep(0.0002)
        return done, time.perf_counter() - t_start

    def summary(done, dt):
        lat = np.array([i["queue_ms"] + i["run_ms"] for _, i in done])
        return {"solves_per_s": round(len(done) / dt, 1), "requests": len(done),
                "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                               "p99": round(float(np.percentile(lat, 99)), 3)}}

    S, ids = server(slots, batch_slots)
    if batch_slots:
        run(S, ids, draw(64, np.random.default_rng(seed + 7)))   # warm-up of the engines
    done, dt = run(S, ids, draw(n_closed))
    sat = len(done) / dt
    per_dict = []
    for d, (n, k, g, dtp) in enumerate(SERVE_DICTS):
        infos = [i for dd, i in done if dd == d]
        if infos:
            per_dict.append({"dict": f"{n}x{k}{'g' + str(g) if g else ''}_{dtp}", "requests": len(infos),
                             "mean_run_ms": round(float(np.mean([i["run_ms"] for i in infos])), 3),
                             "mean_iters": round(float(np.mean([i["iters"] for i in infos])), 1)})
    opens = []
    for frac in (0.5, 0.9):
        reqs = draw(warm + n_open)
        gaps = rng.exponential(1.0 / (frac * sat), size=len(reqs))
        done, dt = run(S, ids, reqs, gaps, skip=warm)
        opens.append(dict(offered_per_s=round(frac * sat, 1), **summary(done, dt)))
    S.close()
    if batch_slots:
        return {"slots": slots, "batch_slots": batch_slots,
                "saturation_solves_per_s": round(sat, 1), "open_loop": opens,
                "per_dict_closed_loop": per_dict}
    # baseline: the plain (unscreened) single-signal path, one request at a time
    P, pids = server(1)
    pdone, pdt = [], 0.0
    for q in draw(n_plain):
        done, dt = run(P, pids, [q], test="none")
        pdone += done
        pdt += dt
    P.close()
    plain = len(pdone) / pdt
    return {"workload": "serving_mix_8_dicts_lasso_group_f32_bf16", "slots": slots,
            "dictionaries": [f"{n}x{k}{'g' + str(g) if g else ''}_{dt}" for n, k, g, dt in SERVE_DICTS],
            "saturation_solves_per_s": round(sat, 1),
            "plain_one_at_a_time_solves_per_s": round(plain, 1),
            "saturation_over_plain": round(sat / plain, 2),
            "open_loop": opens, "per_dict_closed_loop": per_dict}


def backtracking_leg(binding, Dd, ys, steps):
    """The headline workload with the step rule Table 1 gives FISTA (backtracking, L_0 the
    largest squared atom norm, eta = 2): screened and plain solves/s, iterations per solve."""
    import torch
    out = {"step": "backtracking", "eta": 2.0, "L0": "largest squared atom norm"}
    for test in ("dst3", "none"):
        run_steps(binding, Dd, ys, 1, test, 0.0, step="backtracking")   # warm-up
        it = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = run_steps(binding, Dd, ys, steps, test, 0.0, step="backtracking", iters=it)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = "screened" if test == "dst3" else "plain"
        out[f"{key}_solves_per_s"] = round(n / dt, 3)
        out[f"{key}_mean_iters"] = round(float(np.mean(it)), 1)
    out["screened_over_plain"] = round(out["screened_solves_per_s"] / out["plain_solves_per_s"], 4)
    return out


def dome_leg(binding, Dd, ys, steps, L):
    """The headline workload (FISTA, constant step) with the dynamic Dome test in place of
    DST3: solves/s and the mean number of atoms still active after 10 iterations."""
    import torch
    run_steps(binding, Dd, ys, 1, "dome", L)   # warm-up
    it = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = run_steps(binding, Dd, ys, steps, "dome", L, iters=it)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    act = {}
    for test in ("dst3", "dome"):
        a10 = []
        for r in RATIOS:
            _, _, _, tr = binding.solve_one(Dd, ys[0], r, rule="fista", test=test, step_L=L,
                                            gap_tol=0.0, max_iter=10, screened=False)
            a10.append(tr[-1]["n_active"])
        act[test] = round(float(np.mean(a10)), 1)
    return {"test": "dome", "solves_per_s": round(n / dt, 3),
            "mean_iters": round(float(np.mean(it)), 1),
            "mean_active_after_10_iters": act}


def cp_leg(binding, Dd, ys, steps, L):
    """The headline workload with the Chambolle-Pock update of Table 1 (gamma = 0,
    tau_0 = 1/sqrt(L), sigma_0 = 1/(tau_0 L), L the headline's bound on ||D||_2^2): screened
    (DST3) and plain solves/s and iterations per solve."""
    import torch
    out = {"rule": "cp", "gamma": 0.0, "tau0": "1/sqrt(L)", "sigma0": "1/(tau0 L)"}
    for test in ("dst3", "none"):
        run_steps(binding, Dd, ys, 1, test, L, rule="cp")   # warm-up
        it = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = run_steps(binding, Dd, ys, steps, test, L, iters=it, rule="cp")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = "screened" if test == "dst3" else "plain"
        out[f"{key}_solves_per_s"] = round(n / dt, 3)
        out[f"{key}_mean_iters"] = round(float(np.mean(it)), 1)
    return out


def sparsa_leg(binding, Dd, ys, steps):
    """The headline workload with SpaRSA (Table 1: ISTA with the Barzilai-Borwein step;
    L_0 the largest squared atom norm, eta = 2, sigma = 1e-5), monotone (memory 0) and
    with a memory of 5 iterates: screened and plain solves/s, iterations per solve."""
    import torch
    out = {"rule": "sparsa", "eta": 2.0, "sigma": 1e-5, "L0": "largest squared atom norm"}
    for mem in (0, 5):
        for test in ("dst3", "none"):
            run_steps(binding, Dd, ys, 1, test, 0.0, rule="sparsa", bb_memory=mem)  # warm-up
            it = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            n = run_steps(binding, Dd, ys, steps, test, 0.0, iters=it, rule="sparsa",
                          bb_memory=mem)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            key = f"memory{mem}_" + ("screened" if test == "dst3" else "plain")
            out[f"{key}_solves_per_s"] = round(n / dt, 3)
            out[f"{key}_mean_iters"] = round(float(np.mean(it)), 1)
    return out


# The largest dictionary of the serving mix: 4096 x 40000 FP32 is 655 MB, more than the
# 256 MB last-level cache, so every correlation pass streams it from HBM.
LARGE = (4096, 40000)
LARGE_RATIOS = (0.3, 0.5, 0.7)


def large_inputs(group, seed=datagen.DICT_SEED):
    """Unit-norm Gaussian 4096 x 40000 FP32 dictionary and one unit-norm observation (2%
    active atoms, or groups of 10, with N(0,1) coefficients, 20 dB noise), drawn on the
    device from a seeded generator (655 MB is slow to draw on the host)."""
    import torch
    n, kk = LARGE
    g = torch.Generator(device="cuda")
    g.manual_seed(seed * 1000 + 100 + int(group))
    D = torch.randn(kk, n, generator=g, device="cuda")
    D /= D.norm(dim=1, keepdim=True)
    gs = 10 if group else 0
    units = kk // gs if gs else kk
    mask = torch.rand(units, generator=g, device="cuda") < 0.02
    mask[0] |= ~mask.any()
    if gs:
        mask = mask.repeat_interleave(gs)
    x0 = torch.randn(kk, generator=g, device="cuda") * mask
    yc = x0 @ D
    noise = torch.randn(n, generator=g, device="cuda")
    noise *= yc.norm() / noise.norm() * 10 ** (-20 / 20)
    y = yc + noise
    y /= y.norm()
    gp = np.arange(0, kk + 1, gs, dtype=np.int64) if gs else None
    torch.cuda.synchronize()
    return D.T, y.contiguous(), gp


def large_leg(binding):
    """HBM roofline of the correlation kernel where the dictionary cannot stay in the
    last-level cache: one signal on 4096 x 40000 FP32, Lasso (FISTA + DST3) and
    Group-Lasso (groups of 10, FISTA + DGST3), lambda / lambda_* in LARGE_RATIOS, gap 1e-6.
    Kernel spans from the device wall clock, algorithmic bytes as in the headline."""
    out = {}
    for group in (False, True):
        Dt, y, gp = large_inputs(group)
        L = binding.spectral_norm_sq(Dt, 300)
        binding.stats_reset()
        binding.stats_enable(True)
        iters = []
        for r in LARGE_RATIOS:
            _, info, _, _ = binding.solve_one(Dt, y, r, group_ptr=gp, rule="fista", test="dst3",
                                              step_L=L, gap_tol=GAP_TOL, max_iter=20000,
                                              trace=False, screened=False)
            if info["status"] != 0:
                raise RuntimeError(f"large solve did not converge: {info}")
            iters.append(info["iters"])
        binding.stats_enable(False)
        st = binding.stats_read()[binding.STAT_CORR]
        n = max(st["launches"], 1)
        avg_ms = st["ms"] / n
        achieved = st["bytes"] / max(st["ms"] * 1e-3, 1e-12) / 1e9
        name = "group" if group else "lasso"
        out[name] = {"kernel": f"k_corr_{name}",
                     "workload": f"{name}_fista_{'dgst3' if group else 'dst3'}_gaussian_"
                                 f"{LARGE[0]}x{LARGE[1]}_f32",
                     "lambda_ratios": list(LARGE_RATIOS), "iters": iters,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "avg_launch_us": round(avg_ms * 1e3, 3),
                     "algorithmic_bytes_per_launch": round(st["bytes"] / n, 1),
                     "launches": st["launches"]}
        del Dt, y
    return out


# ---------------------------------------------------------------- the paper's experiments
# Flops model of the experiments section ("How to evaluate"), from the per-iteration trace
# of a solve (|I^c_t| = the atoms the update of iteration t used, ||x_t||_0 = the non-zeros
# of its result).  Bookkeeping only; tests check it against the oracle's statement of it.
def flops_none(trace, n, k, n_groups=0):
    """flops_N: sum_t [(K + ||x_t||_0) N + 4 K + N (+ 3 |G|)]."""
    return sum((k + t["nnz"]) * n + 4 * k + n + 3 * n_groups for t in trace)


def flops_static(trace, n, k, n_kept, n_groups=0):
    """flops_S: K N + sum_t [(|I^c_0| + ||x_t||_0) N + 4 |I^c_0| + N (+ 3 |G|)]."""
    return k * n + sum((n_kept + t["nnz"]) * n + 4 * n_kept + n + 3 * n_groups for t in trace)


def flops_dynamic(trace, n, n_groups=0):
    """flops_D: sum_t [(|I^c_t| + ||x_t||_0) N + 6 |I^c_t| + 5 N] (Lasso), or with
    7 |I^c_t| and + 5 |G| (Group-Lasso)."""
    c = 7 if n_groups else 6
    return sum((t["n_active"] + t["nnz"]) * n + c * t["n_active"] + 5 * n + 5 * n_groups
               for t in trace)


# The experiments' stopping rule: t > 200 or a relative objective change below 1e-7.
PAPER_MAX_ITER = 200
PAPER_OBJ_TOL = 1e-7
PAPER_RUNS = 30
PAPER_RATIOS = (0.1, 0.3, 0.5, 0.7, 0.9)
PAPER_RULES = ("ista", "fista", "sparsa", "cp")


def _quantiles(v):
    v = np.asarray(v, dtype=np.float64)
    return {"median": round(float(np.median(v)), 4), "p25": round(float(np.percentile(v, 25)), 4),
            "p75": round(float(np.percentile(v, 75)), 4)}


def paper_runs(binding, Dd, ys, L, rules, ratios, group_ptr=None, test="dst3"):
    """No screening, static and dynamic screening (the given test) for every observation,
    rule and ratio, under the experiments' stopping rule; normalised flops and times of
    every run, summarised by the median and the 25 / 75 % percentiles."""
    import torch
    n, k = Dd.shape
    n_groups = 0 if group_ptr is None else group_ptr.size - 1

    def run(y, r, rule, tst, screening):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, _, tr = binding.solve_one(Dd, y, r, rule=rule, test=tst, group_ptr=group_ptr,
                                           step_L=0.0 if rule == "sparsa" else L, gap_tol=0.0,
                                           obj_tol=PAPER_OBJ_TOL, max_iter=PAPER_MAX_ITER,
                                           trace=True, screened=False, screening=screening)
        torch.cuda.synchronize()
        return tr, time.perf_counter() - t0

    for rule in rules:  # untimed warm-up of every kernel instantiation
        for tst, scr in ((test, "dynamic"), (test, "static"), ("none", "dynamic")):
            run(ys[0], ratios[0], rule, tst, scr)
    out = {}
    for rule in rules:
        rows = []
        for r in ratios:
            fd, fs, td, ts, iters = [], [], [], [], []
            for y in ys:
                trn, tn = run(y, r, rule, "none", "dynamic")
                trd, td_ = run(y, r, rule, test, "dynamic")
                trs, ts_ = run(y, r, rule, test, "static")
                kept = trs[1]["n_active"] if len(trs) > 1 else k
                fnone = flops_none(trn, n, k, n_groups)
                fd.append(flops_dynamic(trd, n, n_groups) / fnone)
                fs.append(flops_static(trs, n, k, kept, n_groups) / fnone)
                td.append(td_ / tn)
                ts.append(ts_ / tn)
                iters.append(len(trn))
            rows.append({"lambda_ratio": r, "flops_dynamic_over_none": _quantiles(fd),
                         "flops_static_over_none": _quantiles(fs),
                         "time_dynamic_over_none": _quantiles(td),
                         "time_static_over_none": _quantiles(ts),
                         "iterations": _quantiles(iters)})
        out[rule] = rows
    return out


def paper_lasso_leg(binding, runs=PAPER_RUNS):
    """The Lasso experiment (the paper's normalised running times and flops on Pnoise): the
    2000 x 10000 FP32 Pnoise dictionary, observations drawn from the atoms' distribution,
    ISTA, FISTA, SpaRSA and Chambolle-Pock with no / static / dynamic ST3 screening, the
    experiments' stopping rule, medians and percentiles over `runs` observations."""
    Dp = datagen.pnoise_dictionary(N, K, datagen.DICT_SEED)
    D32 = datagen.to_storage(Dp, "f32")
    ys_h = [datagen.to_storage(datagen.atom_like_observation(N, j, "pnoise"), "f32")
            for j in range(runs)]
    Dd, _ = _dev(D32, ys_h[0])
    import torch
    ys = [torch.from_numpy(y.astype(np.float32)).cuda() for y in ys_h]
    L = binding.spectral_norm_sq(Dd, 300)
    return {"workload": "lasso_pnoise_2000x10000_f32_atomlike_observations",
            "runs": runs, "stop": f"t > {PAPER_MAX_ITER} or relative objective change < "
                                  f"{PAPER_OBJ_TOL:g}", "test": "dst3",
            "per_rule": paper_runs(binding, Dd, ys, L, PAPER_RULES, PAPER_RATIOS)}


GROUP_SIZES = (5, 10, 50, 100)


def paper_group_leg(binding, runs=PAPER_RUNS):
    """The Group-Lasso experiment: FISTA with no / static / dynamic DGST3 on the 2000 x 10000
    FP32 Pnoise dictionary in groups of 5, 10, 50 and 100 atoms (w_g = sqrt(|g|)), each
    group active with probability 0.05 (Gaussian coefficients, 20 dB noise, unit y), the
    experiments' stopping rule, medians and percentiles over `runs` observations.  The atoms
    are i.i.d., so contiguous groups are a uniformly random equal-size partition."""
    import torch
    Dp = datagen.pnoise_dictionary(N, K, datagen.DICT_SEED)
    D32 = datagen.to_storage(Dp, "f32")
    Dd, _ = _dev(D32, np.zeros(N))
    L = binding.spectral_norm_sq(Dd, 300)
    out = {}
    for gs in GROUP_SIZES:
        gp = datagen.contiguous_groups(K, gs)
        ys = [torch.from_numpy(datagen.to_storage(datagen.group_signal(Dp, gp, j, p=0.05)[0],
                                                  "f32").astype(np.float32)).cuda()
              for j in range(runs)]
        out[str(gs)] = paper_runs(binding, Dd, ys, L, ("fista",), PAPER_RATIOS,
                                  group_ptr=gp)["fista"]
    return {"workload": "group_lasso_fista_pnoise_2000x10000_f32", "runs": runs,
            "stop": f"t > {PAPER_MAX_ITER} or relative objective change < {PAPER_OBJ_TOL:g}",
            "test": "dgst3", "per_group_size": out}


FIG1 = (5000, 50000)


def paper_illustration_leg(binding):
    """The introduction's illustration: ISTA with the dynamic SAFE test against plain ISTA,
    atoms and observation uniform on the unit sphere in dimension 5000, K = 50000 atoms
    (1 GB in FP32, drawn on the device from a seeded generator), lambda = 0.75 lambda_*,
    solved to gap 1e-6: the screened dictionary's size per iteration and the times."""
    import torch
    n, k = FIG1
    g = torch.Generator(device="cuda")
    g.manual_seed(datagen.DICT_SEED * 1000 + 200)
    D = torch.randn(k, n, generator=g, device="cuda")
    D /= D.norm(dim=1, keepdim=True)
    y = torch.randn(n, generator=g, device="cuda")
    y /= y.norm()
    Dt = D.T
    L = binding.spectral_norm_sq(Dt, 300)
    res = {}
    for test in ("safe", "none"):
        binding.solve_one(Dt, y, 0.75, rule="ista", test=test, step_L=L, gap_tol=GAP_TOL,
                          max_iter=5, trace=False, screened=False)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, _, tr = binding.solve_one(Dt, y, 0.75, rule="ista", test=test, step_L=L,
                                           gap_tol=GAP_TOL, max_iter=20000, trace=True,
                                           screened=False)
        torch.cuda.synchronize()
        res[test] = (time.perf_counter() - t0, info, tr)
    t_s, info_s, tr_s = res["safe"]
    t_n, info_n, tr_n = res["none"]
    act = [t["n_active"] for t in tr_s]
    first = next((i + 1 for i, a in enumerate(act) if a < k), None)
    five = next((i + 1 for i, a in enumerate(act) if a <= 0.05 * k), None)
    marks = sorted({1, 10, 20, 25, 30, 40, 50, 100, len(act)} & set(range(1, len(act) + 1)))
    del D, Dt
    return {"workload": "lasso_ista_safe_sphere_5000x50000_f32", "lambda_ratio": 0.75,
            "iters": info_s["iters"], "iters_unscreened": info_n["iters"],
            "ms_dynamic_safe": round(t_s * 1e3, 3), "ms_unscreened": round(t_n * 1e3, 3),
            "time_dynamic_over_none": round(t_s / t_n, 4),
            "flops_dynamic_over_none": round(flops_dynamic(tr_s, n) / flops_none(tr_n, n, k), 4),
            "first_iteration_screening": first, "first_iteration_at_5_percent": five,
            "dictionary_size_at": {str(t): act[t - 1] for t in marks},
            "paper_context": "4.6 s screened vs 11.8 s unscreened (0.39), Python, hardware unstated"}


SEEDS = 30


def seeds_leg(binding, D, Dd, L, seeds=SEEDS):
    """The headline workload per lambda / lambda_* over `seeds` signals: screened (DST3) and
    plain solves timed one by one; median and 25 / 75 % percentiles of the solve time, of
    the plain / screened time ratio and of the iterations."""
    import torch
    ys = [torch.from_numpy(datagen.to_storage(datagen.lasso_signal(D, j)[0], "f32")
                           .astype(np.float32)).cuda() for j in range(seeds)]

    def timed(y, r, test):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, _, _ = binding.solve_one(Dd, y, r, rule="fista", test=test, step_L=L,
                                          gap_tol=GAP_TOL, max_iter=20000, trace=False,
                                          screened=False)
        torch.cuda.synchronize()
        if info["status"] != 0:
            raise RuntimeError(f"solve did not converge: {info}")
        return time.perf_counter() - t0, info["iters"]

    timed(ys[0], RATIOS[0], "dst3")
    timed(ys[0], RATIOS[0], "none")
    rows = []
    for r in RATIOS:
        ts, tp, it = [], [], []
        for y in ys:
            a, n_it = timed(y, r, "dst3")
            b, _ = timed(y, r, "none")
            ts.append(a * 1e3)
            tp.append(b * 1e3)
            it.append(n_it)
        rows.append({"lambda_ratio": r, "screened_ms": _quantiles(ts), "plain_ms": _quantiles(tp),
                     "plain_over_screened": _quantiles(np.array(tp) / np.array(ts)),
                     "iterations": _quantiles(it)})
    return {"workload": "lasso_fista_dst3_gaussian_2000x10000_f32", "signals": seeds,
            "per_ratio": rows}


def small_fp64_leg(binding, reps=20):
    """The small FP64 configuration: 100 x 500, ISTA + dynamic SAFE, lambda = 0.5 lambda_*,
    exactly 500 iterations; microseconds per iteration (whole solve / 500, median)."""
    import torch
    c = datagen.lasso_small_fp64()
    Dd = torch.from_numpy(np.ascontiguousarray(c["D"].T)).cuda().T
    yd = torch.from_numpy(c["y"]).cuda()
    L = binding.spectral_norm_sq(Dd, 300)
    ts = []
    for k in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, _, _ = binding.solve_one(Dd, yd, 0.5, rule="ista", test="safe", step_L=L,
                                          gap_tol=0.0, max_iter=500, trace=False,
                                          screened=False)
        torch.cuda.synchronize()
        if k:
            ts.append(time.perf_counter() - t0)
    return {"workload": "lasso_ista_safe_gaussian_100x500_f64_500_iterations",
            "us_per_iteration": round(float(np.median(ts)) / 500 * 1e6, 3),
            "ms_per_solve": round(float(np.median(ts)) * 1e3, 3), "solves": reps,
            "n_active_final": info["n_active"]}


GROUP_RATIOS = (0.3, 0.7)


def groups_leg(binding, D, Dd, L, signals=5):
    """The Group-Lasso workload: 2000 x 10000 FP32, 1000 contiguous groups of 10, w_g =
    sqrt(10), 2 % active groups, ISTA with dynamic DGST3, GSAFE or no screening, lambda /
    lambda_* in {0.3, 0.7}, gap 1e-6: solves/s and iterations per test."""
    import torch
    gp = datagen.contiguous_groups(K, 10)
    ys = [torch.from_numpy(datagen.to_storage(datagen.group_signal(D, gp, j)[0], "f32")
                           .astype(np.float32)).cuda() for j in range(signals)]
    out = {"workload": "group_lasso_ista_gaussian_2000x10000_f32_groups10", "signals": signals,
           "lambda_ratios": list(GROUP_RATIOS)}
    for test in ("dgst3", "gsafe", "none"):
        binding.solve_one(Dd, ys[0], GROUP_RATIOS[0], group_ptr=gp, rule="ista", test=test,
                          step_L=L, gap_tol=GAP_TOL, max_iter=50000, trace=False, screened=False)
        it = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = 0
        for y in ys:
            for r in GROUP_RATIOS:
                _, info, _, _ = binding.solve_one(Dd, y, r, group_ptr=gp, rule="ista", test=test,
                                                  step_L=L, gap_tol=GAP_TOL, max_iter=50000,
                                                  trace=False, screened=False)
                if info["status"] != 0:
                    raise RuntimeError(f"group solve did not converge: {info}")
                it.append(info["iters"])
                n += 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[test] = {"solves_per_s": round(n / dt, 3), "mean_iters": round(float(np.mean(it)), 1)}
    out["dgst3_over_none"] = round(out["dgst3"]["solves_per_s"] / out["none"]["solves_per_s"], 4)
    out["gsafe_over_none"] = round(out["gsafe"]["solves_per_s"] / out["none"]["solves_per_s"], 4)
    return out


def batched_precision(binding, D, infos, X, ratios, sample=16):
    """Per result, the error of the bfloat16-instance solution against the optimum of the
    unrounded dictionary, which the device's FP64 single-signal path computes to a gap of
    1e-12 ||y||^2 (that path matches the FP64 oracle to 1e-10): relative objective error
    P_D(x) / P*_D - 1 and relative iterate error ||x - x*||_inf / ||x*||_inf."""
    import torch
    D64 = torch.from_numpy(np.ascontiguousarray(D.T)).cuda().T
    L64 = binding.spectral_norm_sq(D64, 300)
    idx = np.random.default_rng(11).choice(len(infos), sample, replace=False)
    rel_obj, rel_it = [], []
    for j in idx:
        y = torch.from_numpy(datagen.to_storage(datagen.lasso_signal(D, int(j))[0], "f32")).cuda()
        lam = infos[j]["lambda_"]
        xs, info, _, _ = binding.solve_one(D64, y, lam, lambda_relative=False, rule="fista",
                                           test="dst3", step_L=L64, gap_tol=1e-12,
                                           max_iter=200000, trace=False, screened=False)
        x = X[:, int(j)].to(torch.float64)
        r = D64 @ x - y
        p = 0.5 * float(r @ r) + lam * float(x.abs().sum())
        rel_obj.append((p - info["primal"]) / info["primal"])
        rel_it.append(float((x - xs).abs().max() / xs.abs().max().clamp_min(1e-300)))
    del D64
    return {"reference": "FP64 solve of the unrounded dictionary on the device, gap 1e-12",
            "signals": sample, "rel_objective_error": _quantiles(rel_obj) | {"max": float(max(rel_obj))},
            "rel_iterate_error": _quantiles(rel_it) | {"max": float(max(rel_it))}}


def kernel_source_sha(paths):
    """sha256 over the concatenated sources a kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profile_record():
    """The committed counter and rocprof record of the instrumented sample (HBM bytes per
    launch from FETCH_SIZE and WRITE_SIZE, rocprof's average duration, the run's algorithmic
    bytes per launch), or None when the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        sha = kernel_source_sha(rec["sources"])
        ok = sha == rec["sources_sha256"]
        need = ("traffic_bytes_per_launch", "algorithmic_bytes_per_launch", "rocprof_avg_launch_us")
        return rec if ok and all(k in rec for k in need) else None
    except (OSError, KeyError, ValueError):
        return None


def _oracle_sweeps(D, D32, L, budget_s, max_signals):
    import oracle
    n = 0
    sig = 0
    dt = 0.0  # oracle time only (signal generation excluded)
    while True:
        y = datagen.to_storage(datagen.lasso_signal(D, sig)[0], "f32")
        t0 = time.perf_counter()
        for r in RATIOS:
            oracle.solve_lasso(D32, y, lam_ratio=r, rule="fista", test="dst3", L=L,
                               max_iter=20000, gap_tol=GAP_TOL)
            n += 1
        dt += time.perf_counter() - t0
        sig += 1
        if dt > budget_s or sig >= max_signals:
            break
    return n, sig, dt


def cpu_baseline(D, D32, L, budget_s=20.0, max_signals=30, one_thread_budget_s=8.0):
    """FP64 oracle on the host cores: whole sweeps of consecutive signals until ~budget;
    then the same with one BLAS thread (a shorter budget)."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count()
    n, sig, dt = _oracle_sweeps(D, D32, L, budget_s, max_signals)
    out = {"value": n / dt, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
           "sample": f"{sig} signal(s) x {len(RATIOS)} lambda ratios of the same workload, "
                     f"FP64 NumPy, FISTA + DST3 to gap {GAP_TOL:g}, {dt:.1f} s"}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            n1, sig1, dt1 = _oracle_sweeps(D, D32, L, one_thread_budget_s, max_signals)
        out["one_thread"] = {"value": n1 / dt1, "unit": "solves/s", "cores": 1,
                             "sample": f"{sig1} signal(s) x {len(RATIOS)} lambda ratios, {dt1:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--legs", default="single,seeds,small,groups,batched,batched_groups,served,"
                                      "served_batched,"
                                      "paper_lasso,paper_group,paper_illustration,large,"
                                      "backtracking,sparsa,dome,cp",
                    help="comma list of legs: single (headline), seeds (the headline per lambda "
                         "over 30 signals), small (100 x 500 FP64, microseconds per iteration), "
                         "groups (groups of 10, ISTA + DGST3 / GSAFE), batched, batched_groups (256 signals of "
                         "the group workload on the bfloat16 matrix-core path), served (the "
                         "eight-dictionary "
                         "mix, workers only and with batched engines), served_batched (requests "
                         "for the batched workload's bfloat16 dictionary: engine vs workers), "
                         "paper_lasso (the paper's Pnoise Lasso experiment: normalised flops "
                         "and times of 4 rules x 3 strategies over 30 runs), paper_group (its "
                         "Group-Lasso group-size experiment), paper_illustration (its "
                         "introduction's 5000 x 50000 ISTA + SAFE run), large "
                         "(correlation roofline on 4096 x 40000 FP32), backtracking (the headline "
                         "workload with backtracking steps), sparsa (the headline workload with "
                         "SpaRSA's Barzilai-Borwein steps), dome (the headline workload with "
                         "the dynamic Dome test), cp (the headline workload with the "
                         "Chambolle-Pock update).  Profiling "
                         "helpers (run alone): 'screened' runs only the timed screened "
                         "solves; 'instrumented' only the instrumented single-signal pass "
                         "(no warmup); 'batched-instrumented' only one instrumented "
                         "batched solve; 'large-instrumented' only the large-dictionary leg")
    ap.add_argument("--serve-slots", type=int, default=8, help="worker slots of the serving leg")
    ap.add_argument("--serve-batch-slots", type=int, default=64,
                    help="resident signals of each batched engine in the serving mix's engine run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB device to device (a plain copy kernel of known "
                         "size, for scaling HBM counters)")
    args = ap.parse_args()
    legs = set(args.legs.split(","))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU layout is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1412_4080_amd import binding

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if legs == {"large-instrumented"}:
        print(json.dumps({"leg": "large-instrumented", "roofline_large_dictionary": large_leg(binding)}),
              flush=True)
        return
    D = datagen.gaussian_dictionary(N, K, datagen.DICT_SEED)
    D32 = datagen.to_storage(D, "f32")
    if legs == {"batched-instrumented"}:
        print(json.dumps({"leg": "batched-instrumented",
                          "roofline": batched_roofline(binding, batched_setup(binding, D))}),
              flush=True)
        return
    nsig = max(args.steps, args.warmup, INSTR_SIGNALS)
    ys_host = [datagen.to_storage(datagen.lasso_signal(D, j)[0], "f32") for j in range(nsig)]
    Dd, _ = _dev(D32, ys_host[0])
    ys = [torch.from_numpy(y.astype(np.float32)).cuda() for y in ys_host]
    L = binding.spectral_norm_sq(Dd, 300)   # per-dictionary constant, computed once
    torch.cuda.synchronize()

    if legs == {"instrumented"}:
        print(json.dumps({"leg": "instrumented",
                          "roofline": single_roofline(binding, Dd, ys, L)}), flush=True)
        return
    Ys = columns_of(ys)
    run_steps_concurrent(binding, Dd, Ys, args.warmup, "dst3", L)
    run_steps(binding, Dd, ys, args.warmup, "dst3", L)
    if legs == {"screened"}:
        run_steps_concurrent(binding, Dd, Ys, args.steps, "dst3", L)
        return
    # ---- timed region: screened solves, the five solves of a step concurrently ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = run_steps_concurrent(binding, Dd, Ys, args.steps, "dst3", L)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = n / dt

    # ---- plain (unscreened) solves on the same inputs, measured the same way ----
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_plain = run_steps_concurrent(binding, Dd, Ys, args.steps, "none", L)
    torch.cuda.synchronize()
    plain = n_plain / (time.perf_counter() - t1)

    # ---- one solve at a time: per-solve latency, and the sequential rates ----
    lat = []
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    n_seq = run_steps(binding, Dd, ys, args.steps, "dst3", L, lat)
    torch.cuda.synchronize()
    seq = n_seq / (time.perf_counter() - t2)
    t3 = time.perf_counter()
    n_seq_plain = run_steps(binding, Dd, ys, args.steps, "none", L)
    torch.cuda.synchronize()
    seq_plain = n_seq_plain / (time.perf_counter() - t3)

    # ---- instrumented pass: kernel execution spans of every correlation launch ----
    roof = single_roofline(binding, Dd, ys, L)

    out = {
        "metric": "Lasso solves/sec to gap 1e-6, screened vs plain; HBM GB/s; p50/p99 latency",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lasso_fista_dst3_gaussian_2000x10000_f32",
                   "N": N, "K": K, "lambda_ratios": list(RATIOS), "gap_tol": GAP_TOL,
                   "signals_per_step": 1, "solves_per_step": len(RATIOS),
                   "solves_in_flight": "the 5 of a step (lasso_solve, 5 columns)",
                   "snr_db": 20, "active_fraction": 0.02},
        "plain_solves_per_s": round(plain, 3),
        "screened_over_plain": round(value / plain, 4),
        "sequential": {"solves_per_s": round(seq, 3), "plain_solves_per_s": round(seq_plain, 3),
                       "screened_over_plain": round(seq / seq_plain, 4),
                       "note": "the same solves one at a time (latency is measured here)"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
        "roofline": roof,
    }
    if "batched" in legs:
        b = batched_leg(binding, D, max(1, args.steps // 2), 1)
        b["over_plain_single"] = round(b["solves_per_s"] / plain, 2)
        b["stream"] = batched_stream_leg(binding, D)
        b["stream"]["over_plain_single"] = round(b["stream"]["solves_per_s"] / plain, 2)
        out["batched"] = b
    if "batched_groups" in legs:
        out["batched_groups"] = batched_groups_leg(binding, D)
    if "seeds" in legs:
        out["per_lambda_30_signals"] = seeds_leg(binding, D, Dd, L)
    if "small" in legs:
        out["small_fp64"] = small_fp64_leg(binding)
    if "groups" in legs:
        out["groups"] = groups_leg(binding, D, Dd, L)
    if "paper_lasso" in legs:
        out["paper_lasso_pnoise"] = paper_lasso_leg(binding)
    if "paper_group" in legs:
        out["paper_group_sizes_pnoise"] = paper_group_leg(binding)
    if "paper_illustration" in legs:
        out["paper_illustration"] = paper_illustration_leg(binding)
    if "backtracking" in legs:
        bt = backtracking_leg(binding, Dd, ys, args.steps)
        it_c = []
        run_steps(binding, Dd, ys, 1, "dst3", L, iters=it_c)
        bt["constant_step_mean_iters"] = round(float(np.mean(it_c)), 1)
        bt["over_constant_step"] = round(bt["screened_solves_per_s"] / seq, 3)
        out["backtracking"] = bt
    if "dome" in legs:
        dm = dome_leg(binding, Dd, ys, args.steps, L)
        dm["over_dst3"] = round(dm["solves_per_s"] / seq, 3)
        out["dome"] = dm
    if "cp" in legs:
        cp = cp_leg(binding, Dd, ys, args.steps, L)
        cp["over_constant_step_fista"] = round(cp["screened_solves_per_s"] / seq, 3)
        out["cp"] = cp
    if "sparsa" in legs:
        sp = sparsa_leg(binding, Dd, ys, args.steps)
        sp["over_constant_step_fista"] = round(sp["memory0_screened_solves_per_s"] / seq, 3)
        out["sparsa"] = sp
    if "large" in legs:
        out["roofline_large_dictionary"] = large_leg(binding)
    if "served" in legs:
        out["served"] = served_leg(binding, slots=args.serve_slots)
        out["served"]["batched_engine"] = served_leg(binding, slots=args.serve_slots,
                                                     batch_slots=args.serve_batch_slots)
    if "served_batched" in legs:
        out["served_bf16_one_dictionary"] = served_batched_leg(binding, D)
    if not args.no_cpu:
        import oracle
        L64 = oracle.spectral_norm_sq(D32)
        out["cpu_baseline"] = cpu_baseline(D, D32, L64, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
