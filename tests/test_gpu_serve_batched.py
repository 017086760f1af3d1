"""Serving through the batched engine (ds_server_config.batch_slots > 0): requests for a
bfloat16 Lasso dictionary join the matrix-core engine's resident signals as slots free up.
Each result equals lasso_solve's batched result for the same y and lambda bit for bit, and
is the same whether the request ran alone or in a mix with other dictionaries, other
parameters and the single-signal workers."""
import time

import numpy as np
import pytest

from paper_1412_4080_amd import datagen
from tests._util import dev_matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def _dicts():
    """(D values (f64), stored dtype, group_ptr): two bfloat16 Lasso dictionaries and a
    bfloat16 grouped one (engines), an FP32 Lasso and an FP32 grouped one (single-signal
    workers)."""
    return [(datagen.gaussian_dictionary(512, 3000, 31), "bf16", None),
            (datagen.gaussian_dictionary(300, 1700, 32), "bf16", None),
            (datagen.gaussian_dictionary(256, 1000, 33), "f32", None),
            (datagen.gaussian_dictionary(300, 2000, 34), "f32", datagen.contiguous_groups(2000, 10)),
            (datagen.gaussian_dictionary(320, 2400, 37), "bf16", datagen.contiguous_groups(2400, 8))]


def _requests(dicts, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        d = (0, 1, 2, 0, 4, 1, 3, 4)[k % 8]   # three quarters for the engines
        D, _, gp = dicts[d]
        y = datagen.lasso_signal(D, 700 + k)[0] if gp is None else datagen.group_signal(D, gp, 700 + k)[0]
        out.append((d, datagen.to_storage(y, "f32").astype(np.float32), float(rng.uniform(0.1, 0.9))))
    return out


def _server(B, dicts, **kw):
    import torch
    S = B.Server(**kw)
    ids = [S.add_dict(dev_matrix(D, "f32"), group_ptr=gp, store=st) for D, st, gp in dicts]
    torch.cuda.synchronize()
    return S, ids


def _wait(S, pending, ids, timeout=180.0):
    """pending: {key: (rid, dict index)} -> {key: (x, info) or DsError}."""
    from paper_1412_4080_amd import binding
    out = {}
    t0 = time.time()
    while len(out) < len(pending):
        for k, (rid, d) in pending.items():
            if k in out:
                continue
            try:
                r = S.poll(rid, ids[d])
            except binding.DsError as e:
                r = e
            if r is not None:
                out[k] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.0005)
    return out


def _direct_batched(B, D, ys, ratios, L, group_ptr=None, **kw):
    """lasso_solve (glasso_solve) on the bfloat16 dictionary with every signal at once
    (batched path)."""
    import torch
    Dd = dev_matrix(D, "bf16")
    Y = torch.from_numpy(np.ascontiguousarray(np.stack(ys))).cuda().T
    X, infos = B.solve(Dd, Y, ratios, step_L=L, group_ptr=group_ptr, **kw)
    return X.cpu().numpy(), infos


def test_served_batched_equals_lasso_solve_alone_and_in_the_mix(B):
    dicts = _dicts()
    reqs = _requests(dicts, 64, 5)
    kw = dict(gap_tol=1e-6, max_iter=20000)
    # mix: four worker slots and 8-signal engines (more bfloat16 requests than slots, so
    # finished signals hand their slots on), everything submitted at once
    S, ids = _server(B, dicts, max_slots=4, batch_slots=8)
    pend = {k: (S.submit(ids[d], y, r, **kw), d) for k, (d, y, r) in enumerate(reqs)}
    mix = _wait(S, pend, ids)
    S.close()
    # alone: one request on the server at a time
    S, ids = _server(B, dicts, max_slots=1, batch_slots=8)
    alone = {}
    for k, (d, y, r) in enumerate(reqs):
        alone.update(_wait(S, {k: (S.submit(ids[d], y, r, **kw), d)}, ids))
    S.close()
    for k in range(len(reqs)):
        (xm, im), (xa, ia) = mix[k], alone[k]
        assert im["status"] == 0 and ia["status"] == 0, k
        assert np.array_equal(xm, xa), k
        assert im["iters"] == ia["iters"] and im["gap"] == ia["gap"], k
    # every bfloat16 request equals the batched lasso_solve (glasso_solve) of its
    # dictionary's signals
    for d in (0, 1, 4):
        ks = [k for k, (dd, _, _) in enumerate(reqs) if dd == d]
        assert len(ks) > 8
        L = mix[ks[0]][1]["L"]
        X, infos = _direct_batched(B, dicts[d][0], [reqs[k][1] for k in ks],
                                   [reqs[k][2] for k in ks], L, group_ptr=dicts[d][2], **kw)
        for j, k in enumerate(ks):
            assert np.array_equal(mix[k][0], X[:, j]), (d, k)
            assert mix[k][1]["iters"] == infos[j]["iters"]
            assert mix[k][1]["gap"] == infos[j]["gap"]


def test_served_batched_mixed_parameters(B):
    """Requests with different rules, tests and modes on one bfloat16 dictionary: the ones
    the engine supports (the Dome test among them) run in batches of equal parameters and
    equal lasso_solve's batched result with those parameters; the others (backtracking
    steps) run on the single-signal workers and equal ds_solve_one."""
    import torch
    D = datagen.gaussian_dictionary(400, 2500, 35)
    ys = [datagen.to_storage(datagen.lasso_signal(D, 800 + k)[0], "f32").astype(np.float32)
          for k in range(24)]
    variants = [dict(rule="fista", test="dst3"), dict(rule="ista", test="safe"),
                dict(rule="fista", test="none"), dict(rule="fista", test="dst3", screening="static"),
                dict(rule="fista", test="dome"), dict(rule="fista", test="dst3", step="backtracking")]
    S = B.Server(max_slots=3, batch_slots=4)
    did = S.add_dict(dev_matrix(D, "f32"), store="bf16")
    torch.cuda.synchronize()
    lam = [0.2 + 0.03 * k for k in range(len(ys))]
    pend = {k: (S.submit(did, ys[k], lam[k], gap_tol=1e-6, max_iter=20000,
                         **variants[k % len(variants)]), 0) for k in range(len(ys))}
    got = _wait(S, pend, [did])
    S.close()
    L = next(got[k][1]["L"] for k in range(len(ys)) if k % len(variants) == 0)
    Dd = dev_matrix(D, "bf16")
    for v, var in enumerate(variants):
        ks = [k for k in range(len(ys)) if k % len(variants) == v]
        for k in ks:
            assert got[k][1]["status"] == 0, (var, k)
        if var.get("step") == "backtracking":
            for k in ks:
                step_L = 0.0 if var.get("step") == "backtracking" else L
                x1, i1, _, _ = B.solve_one(Dd, torch.from_numpy(ys[k]).cuda(), lam[k],
                                           step_L=step_L, gap_tol=1e-6, max_iter=20000,
                                           trace=False, screened=False, **var)
                assert np.array_equal(got[k][0], x1.cpu().numpy()), (var, k)
        else:
            X, infos = _direct_batched(B, D, [ys[k] for k in ks], [lam[k] for k in ks], L,
                                       gap_tol=1e-6, max_iter=20000, **var)
            for j, k in enumerate(ks):
                assert np.array_equal(got[k][0], X[:, j]), (var, k)
                assert got[k][1]["iters"] == infos[j]["iters"]


def test_served_batched_failed_slot_and_bad_observation(B):
    """A request marked failed from the host (DS_SERVE_FAIL_REQUEST) and one whose y holds a
    NaN report DS_EDEVICE and DS_EINVAL; the engine's other requests are unchanged."""
    import os
    import torch
    D = datagen.gaussian_dictionary(300, 1500, 36)
    ys = [datagen.to_storage(datagen.lasso_signal(D, 900 + k)[0], "f32").astype(np.float32)
          for k in range(10)]

    def run(fail):
        if fail:
            os.environ["DS_SERVE_FAIL_REQUEST"] = "4"
        try:
            S = B.Server(max_slots=2, batch_slots=4)
        finally:
            os.environ.pop("DS_SERVE_FAIL_REQUEST", None)
        did = S.add_dict(dev_matrix(D, "f32"), store="bf16")
        torch.cuda.synchronize()
        yy = [y.copy() for y in ys]
        if fail:
            yy[6][17] = np.nan
        pend = {k: (S.submit(did, yy[k], 0.3 + 0.05 * k, gap_tol=1e-6, max_iter=20000), 0)
                for k in range(len(yy))}
        rids = [pend[k][0] for k in range(len(yy))]
        out = _wait(S, pend, [did])
        S.close()
        return rids, out

    rids, ref = run(False)
    rids_f, got = run(True)
    assert rids_f == rids and rids[3] == 4
    assert isinstance(got[3], B.DsError) and got[3].status == B.DS_EDEVICE
    assert "marked failed" in str(got[3])
    assert isinstance(got[6], B.DsError) and got[6].status == B.DS_EINVAL
    for k in (0, 1, 2, 4, 5, 7, 8, 9):
        assert np.array_equal(got[k][0], ref[k][0]) and got[k][1]["iters"] == ref[k][1]["iters"]


def test_engine_that_cannot_fit_the_budget_leaves_requests_to_the_workers(B):
    """With a budget below the batched engine's footprint (256 resident signals) but above a
    single solve's, requests for a bfloat16 dictionary run on the single-signal workers:
    their results equal ds_solve_one on the same stored dictionary."""
    import torch
    D = datagen.gaussian_dictionary(512, 3000, 38)
    ys = [datagen.to_storage(datagen.lasso_signal(D, 950 + k)[0], "f32").astype(np.float32)
          for k in range(4)]
    S = B.Server(max_slots=2, batch_slots=256, hbm_budget_bytes=32 << 20)
    did = S.add_dict(dev_matrix(D, "f32"), store="bf16")
    torch.cuda.synchronize()
    pend = {k: (S.submit(did, ys[k], 0.3 + 0.1 * k, gap_tol=1e-6, max_iter=20000), 0)
            for k in range(len(ys))}
    got = _wait(S, pend, [did])
    S.close()
    Dd = dev_matrix(D, "bf16")
    for k in range(len(ys)):
        assert got[k][1]["status"] == 0
        x1, i1, _, _ = B.solve_one(Dd, torch.from_numpy(ys[k]).cuda(), 0.3 + 0.1 * k,
                                   step_L=got[k][1]["L"], gap_tol=1e-6, max_iter=20000,
                                   trace=False, screened=False)
        assert np.array_equal(got[k][0], x1.cpu().numpy()), k
        assert got[k][1]["iters"] == i1["iters"]


def test_request_of_other_parameters_is_not_starved(B):
    """One engine, four slots: a request (ISTA + SAFE) queued behind the first of 80 FISTA +
    DST3 requests is overtaken at no more than 16 slot refills (at most 64 requests), so it
    starts before the last FISTA request does; every result equals the batched lasso_solve
    with its parameters."""
    import torch
    D = datagen.gaussian_dictionary(256, 1200, 39)
    ys = [datagen.to_storage(datagen.lasso_signal(D, 1100 + k)[0], "f32").astype(np.float32)
          for k in range(82)]
    lam = [0.3 + 0.005 * k for k in range(len(ys))]
    S = B.Server(max_slots=1, batch_slots=4)
    did = S.add_dict(dev_matrix(D, "f32"), store="bf16")
    torch.cuda.synchronize()
    kw = dict(gap_tol=1e-6, max_iter=20000)
    odd = dict(rule="ista", test="safe")
    t_sub, pend = {}, {}
    for k in range(len(ys)):
        var = odd if k == 1 else dict(rule="fista", test="dst3")
        t_sub[k] = time.perf_counter()
        pend[k] = (S.submit(did, ys[k], lam[k], **kw, **var), 0)
    got = _wait(S, pend, [did])
    S.close()
    start = {k: t_sub[k] + got[k][1]["queue_ms"] * 1e-3 for k in range(len(ys))}
    assert start[1] < max(start[k] for k in range(len(ys)) if k != 1)
    L = got[0][1]["L"]
    ks = [k for k in range(len(ys)) if k != 1]
    X, infos = _direct_batched(B, D, [ys[k] for k in ks], [lam[k] for k in ks], L, **kw)
    for j, k in enumerate(ks):
        assert got[k][1]["status"] == 0 and np.array_equal(got[k][0], X[:, j]), k
    X1, _ = _direct_batched(B, D, [ys[1], ys[1]], [lam[1], lam[1]], L, **kw, **odd)
    assert np.array_equal(got[1][0], X1[:, 0])
