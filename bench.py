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


def batched_setup(binding, D):
    import torch
    Dbf = datagen.to_storage(D, "bf16")
    Dd = torch.from_numpy(np.ascontiguousarray(Dbf.T)).to(device="cuda", dtype=torch.bfloat16).T
    ys = np.stack([datagen.to_storage(datagen.lasso_signal(D, j)[0], "f32") for j in range(NB)])
    Y = torch.from_numpy(ys.astype(np.float32)).cuda().T
    ratios = datagen.lambda_ratios(NB, 0.1, 0.9, datagen.LAMBDA_SEED0)
    L = binding.spectral_norm_sq(Dd, 300)

    def one():
        _, infos = binding.solve(Dd, Y, ratios, step_L=L, gap_tol=GAP_TOL, max_iter=20000)
        if any(i["status"] != 0 for i in infos):
            raise RuntimeError("batched solve did not converge")
        return infos
    return one


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
    return {"bound": "mfma", "kernel": "k_b_zgemm", "achieved": round(achieved, 2),
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
        infos = one()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t1)
    dt = time.perf_counter() - t0
    iters = [i["iters"] for i in infos]
    return {
        "workload": "lasso_fista_dst3_gaussian_2000x10000_bf16_batch256",
        "signals": NB, "solves_per_s": round(NB * steps / dt, 2),
        "ms_per_batch": round(dt * 1e3 / steps, 3),
        "batch_latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                             "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
        "iterations": {"max": int(max(iters)), "mean": round(float(np.mean(iters)), 1)},
        "roofline": batched_roofline(binding, one),
    }


def single_roofline(binding, Dd, ys, steps, L):
    """Instrumented pass over the timed solves: HBM roofline of the correlation kernel."""
    binding.stats_reset()
    binding.stats_enable(True)
    run_steps(binding, Dd, ys, steps, "dst3", L)
    binding.stats_enable(False)
    st = binding.stats_read()[binding.STAT_CORR]
    avg_ms = st["ms"] / max(st["launches"], 1)
    ev_ms = st["ms_event"] / max(st["launches"], 1)
    bytes_per = st["bytes"] / max(st["launches"], 1)
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return {"bound": "hbm", "kernel": "k_corr_lasso",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_record(),
            "avg_launch_us": round(avg_ms * 1e3, 3),
            "event_avg_launch_us": round(ev_ms * 1e3, 3),
            "algorithmic_bytes_per_launch": round(bytes_per, 1),
            "launches": st["launches"]}


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
               seed=datagen.ARRIVAL_SEED):
    """Closed-loop saturation, then open-loop Poisson arrivals at 0.5x and 0.9x of it; the
    baseline is requests of the same mix solved one at a time without screening."""
    inputs = serve_inputs()
    rng = np.random.default_rng(seed)

    def draw(n):
        return [(int(rng.integers(len(inputs))), int(rng.integers(SERVE_POOL)),
                 float(rng.uniform(0.1, 0.9))) for _ in range(n)]

    def server(nslots):
        S = binding.Server(max_slots=nslots, hbm_budget_bytes=24 << 30, max_queue=1 << 14)
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

    S, ids = server(slots)
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


def flops_leg(binding, Dd, ys, L, nsig=3, ratios=RATIOS,
              workload="lasso_fista_dst3_gaussian_2000x10000_f32", rule="fista", group_ptr=None):
    """The experiments section's cost model, normalised by the unscreened run: per
    iteration (|I^c_t| + ||x_t||_0) N + 6 |I^c_t| + 5 N flops, plus K N for the screening
    set-up, from the per-iteration trace of each solve; wall time normalised the same way.
    Dynamic and static DST3 (DGST3 with group_ptr) against the unscreened run, with the
    given update rule (FISTA by default) on the given dictionary (the headline workload by
    default).  SpaRSA takes its own step; the other rules take L."""
    import torch

    def run(y, r, test, screening):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, _, tr = binding.solve_one(Dd, y, r, rule=rule, test=test, group_ptr=group_ptr,
                                           step_L=0.0 if rule == "sparsa" else L,
                                           gap_tol=GAP_TOL, max_iter=50000, trace=True,
                                           screened=False, screening=screening)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fl = sum((t["n_active"] + t["nnz"]) * N + 6 * t["n_active"] + 5 * N for t in tr)
        if test != "none":
            fl += K * N
        return fl, dt, info["iters"]

    # untimed warm-up of each mode: the first launch of a kernel instantiation in the
    # process is slower, and would otherwise be charged to the first ratio's first mode
    for test, scr in (("dst3", "dynamic"), ("dst3", "static"), ("none", "dynamic")):
        run(ys[0], ratios[0], test, scr)
    out = []
    for r in ratios:
        acc = {"dynamic": [0.0, 0.0], "static": [0.0, 0.0], "none": [0.0, 0.0]}
        for j in range(nsig):
            for mode, test, scr in (("dynamic", "dst3", "dynamic"), ("static", "dst3", "static"),
                                    ("none", "none", "dynamic")):
                fl, dt, _ = run(ys[j], r, test, scr)
                acc[mode][0] += fl
                acc[mode][1] += dt
        out.append({"lambda_ratio": r,
                    "flops_dynamic_over_plain": round(acc["dynamic"][0] / acc["none"][0], 4),
                    "flops_static_over_plain": round(acc["static"][0] / acc["none"][0], 4),
                    "time_dynamic_over_plain": round(acc["dynamic"][1] / acc["none"][1], 4),
                    "time_static_over_plain": round(acc["static"][1] / acc["none"][1], 4)})
    return {"workload": workload, "signals": nsig, "per_ratio": out}


# The Pnoise panel: the coherent dictionary of the experiments section (atoms e_1 plus small
# Gaussian perturbations) is ill-conditioned, so FISTA needs thousands of iterations; the
# panel takes lambda/lambda_* >= 0.3 and one signal to stay within the benchmark's budget.
PNOISE_RATIOS = (0.3, 0.5, 0.7, 0.9)


def pnoise_flops_leg(binding):
    """flops_leg on the 2000 x 10000 FP32 Pnoise dictionary (unit observation with 2%
    active atoms and 20 dB noise, as for the Gaussian workload)."""
    Dp = datagen.pnoise_dictionary(N, K, datagen.DICT_SEED)
    D32 = datagen.to_storage(Dp, "f32")
    y32 = datagen.to_storage(datagen.lasso_signal(Dp, 0)[0], "f32")
    Dd, yd = _dev(D32, y32)
    Lp = binding.spectral_norm_sq(Dd, 300)
    return flops_leg(binding, Dd, [yd], Lp, nsig=1, ratios=PNOISE_RATIOS,
                     workload="lasso_fista_dst3_pnoise_2000x10000_f32")


def algorithms_flops_leg(binding, Dd, ys, L):
    """The flops model for each update rule of Table 1 (ISTA, FISTA, SpaRSA, Chambolle-Pock)
    with dynamic and static DST3, each normalised by its own unscreened run, on the
    headline workload (one signal)."""
    return {rule: flops_leg(binding, Dd, ys, L, nsig=1, rule=rule,
                            workload=f"lasso_{rule}_dst3_gaussian_2000x10000_f32")
            for rule in ("ista", "fista", "sparsa", "cp")}


GROUP_SIZES = (5, 10, 50, 100)


def group_sizes_flops_leg(binding):
    """The Group-Lasso experiment: FISTA with dynamic and static DGST3 on the 2000 x 10000
    FP32 Pnoise dictionary split into contiguous groups of 5, 10, 50 and 100 atoms (w_g =
    sqrt(|g|)), one unit observation with 2% active groups and 20 dB noise per size."""
    Dp = datagen.pnoise_dictionary(N, K, datagen.DICT_SEED)
    D32 = datagen.to_storage(Dp, "f32")
    out = {}
    Dd = None
    for gs in GROUP_SIZES:
        gp = datagen.contiguous_groups(K, gs)
        y32 = datagen.to_storage(datagen.group_signal(Dp, gp, 0)[0], "f32")
        Dd, yd = _dev(D32, y32)
        Lp = binding.spectral_norm_sq(Dd, 300)
        out[str(gs)] = flops_leg(binding, Dd, [yd], Lp, nsig=1, ratios=PNOISE_RATIOS,
                                 group_ptr=gp,
                                 workload=f"group_lasso_fista_dgst3_pnoise_2000x10000_f32_size{gs}")
    return out


def kernel_source_sha(paths):
    """sha256 over the concatenated sources a kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_record():
    """HBM bytes per launch of the correlation kernel from the committed counter summary,
    or None when the kernel sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        sha = kernel_source_sha(rec["sources"])
    except (OSError, KeyError, ValueError):
        return None
    return rec["bytes_per_launch"] if sha == rec["sources_sha256"] else None


def cpu_baseline(D, D32, L, budget_s=20.0, max_signals=30):
    """FP64 oracle on the host cores: whole sweeps of consecutive signals until ~budget."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count()
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
    return {"value": n / dt, "unit": "solves/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{sig} signal(s) x {len(RATIOS)} lambda ratios of the same workload, "
                      f"FP64 NumPy, FISTA + DST3 to gap {GAP_TOL:g}, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--legs", default="single,batched,served,flops,large,backtracking,sparsa,dome,cp",
                    help="comma list of legs: single (headline), batched, served, flops, large "
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
    nsig = max(args.steps, args.warmup, 1)
    ys_host = [datagen.to_storage(datagen.lasso_signal(D, j)[0], "f32") for j in range(nsig)]
    Dd, _ = _dev(D32, ys_host[0])
    ys = [torch.from_numpy(y.astype(np.float32)).cuda() for y in ys_host]
    L = binding.spectral_norm_sq(Dd, 300)   # per-dictionary constant, computed once
    torch.cuda.synchronize()

    if legs == {"instrumented"}:
        print(json.dumps({"leg": "instrumented",
                          "roofline": single_roofline(binding, Dd, ys, args.steps, L)}), flush=True)
        return
    run_steps(binding, Dd, ys, args.warmup, "dst3", L)
    if legs == {"screened"}:
        run_steps(binding, Dd, ys, args.steps, "dst3", L)
        return
    # ---- timed region: screened solves ----
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = run_steps(binding, Dd, ys, args.steps, "dst3", L, lat)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = n / dt

    # ---- plain (unscreened) solves on the same inputs ----
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_plain = run_steps(binding, Dd, ys, args.steps, "none", L)
    torch.cuda.synchronize()
    plain = n_plain / (time.perf_counter() - t1)

    # ---- instrumented pass: kernel execution spans of every correlation launch ----
    roof = single_roofline(binding, Dd, ys, args.steps, L)

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
                   "snr_db": 20, "active_fraction": 0.02},
        "plain_solves_per_s": round(plain, 3),
        "screened_over_plain": round(value / plain, 4),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 3),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 3)},
        "roofline": roof,
    }
    if "batched" in legs:
        b = batched_leg(binding, D, max(1, args.steps // 2), 1)
        b["over_plain_single"] = round(b["solves_per_s"] / plain, 2)
        out["batched"] = b
    if "flops" in legs:
        out["flops_model"] = flops_leg(binding, Dd, ys, L, nsig=min(3, len(ys)))
        out["flops_model_pnoise"] = pnoise_flops_leg(binding)
        out["flops_model_algorithms"] = algorithms_flops_leg(binding, Dd, ys, L)
        out["flops_model_group_sizes_pnoise"] = group_sizes_flops_leg(binding)
    if "backtracking" in legs:
        bt = backtracking_leg(binding, Dd, ys, args.steps)
        it_c = []
        run_steps(binding, Dd, ys, 1, "dst3", L, iters=it_c)
        bt["constant_step_mean_iters"] = round(float(np.mean(it_c)), 1)
        bt["over_constant_step"] = round(bt["screened_solves_per_s"] / value, 3)
        out["backtracking"] = bt
    if "dome" in legs:
        dm = dome_leg(binding, Dd, ys, args.steps, L)
        dm["over_dst3"] = round(dm["solves_per_s"] / value, 3)
        out["dome"] = dm
    if "cp" in legs:
        cp = cp_leg(binding, Dd, ys, args.steps, L)
        cp["over_constant_step_fista"] = round(cp["screened_solves_per_s"] / value, 3)
        out["cp"] = cp
    if "sparsa" in legs:
        sp = sparsa_leg(binding, Dd, ys, args.steps)
        sp["over_constant_step_fista"] = round(sp["memory0_screened_solves_per_s"] / value, 3)
        out["sparsa"] = sp
    if "large" in legs:
        out["roofline_large_dictionary"] = large_leg(binding)
    if "served" in legs:
        out["served"] = served_leg(binding, slots=args.serve_slots)
    if not args.no_cpu:
        import oracle
        L64 = oracle.spectral_norm_sq(D32)
        out["cpu_baseline"] = cpu_baseline(D, D32, L64, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
