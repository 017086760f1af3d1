"""The boundary's optional input and failure paths on the device, through the C-ABI:

* the initial point X_0 of Algorithm 3 (ds_params.x0) on the single-signal, multi-signal
  and served paths, against the oracle started from the same point;
* DS_NOT_CONVERGED when max_iter ends a solve above its tolerance (x and the gap still
  reported), single-signal and batched;
* serving: admission after a finished request under a budget of one request, and a slot
  marked failed from the host (DS_SERVE_FAIL_REQUEST) without touching the others.
"""
import ctypes as C
import os
import time

import numpy as np
import pytest

import oracle
from paper_1412_4080_amd import datagen
from tests._util import dev_matrix, dev_vector, instance, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def _lasso(N, K, seed, p=0.02):
    D = datagen.gaussian_dictionary(N, K, seed)
    y, _ = datagen.lasso_signal(D, seed, p=p)
    return D, y


# ------------------------------------------------------------ warm start
@pytest.mark.parametrize("rule,test", [("ista", "safe"), ("fista", "dst3"), ("cp", "dst3"),
                                       ("sparsa", "safe"), ("fista", "none")])
def test_warm_start_follows_the_oracle_fp64(B, rule, test):
    """From the same X_0 (an earlier iterate of the oracle), the device's FP64 trajectory
    equals the oracle's: iterate, objective and active-set sizes at every iteration."""
    c = datagen.lasso_small_fp64()
    D, y = c["D"], c["y"]
    L = oracle.spectral_norm_sq(D)
    start = oracle.solve_lasso(D, y, lam_ratio=0.5, rule="ista", test="none", L=L, max_iter=40,
                               gap_tol=0.0)
    x0 = start.x
    ref = oracle.solve_lasso(D, y, lam_ratio=0.5, rule=rule, test=test, L=L, max_iter=120,
                             gap_tol=0.0, record=True, x0=x0)
    Dd, yd = dev_matrix(D, "f64"), dev_vector(y, "f64")
    x, info, scr, tr = B.solve_one(Dd, yd, 0.5, rule=rule, test=test, step_L=L, gap_tol=0.0,
                                   max_iter=120, x0=dev_vector(x0, "f64"))
    x = x.cpu().numpy()
    assert info["iters"] == ref.iters == 120
    assert rel_err(x, ref.x) <= 1e-10
    assert info["primal"] == pytest.approx(ref.primal_p, rel=1e-12)
    assert [t["n_active"] for t in tr] == [h["n_active"] for h in ref.history]
    # the first gap is the certificate of X_0 itself, far below the cold start's
    cold = oracle.solve_lasso(D, y, lam_ratio=0.5, rule=rule, test=test, L=L, max_iter=1,
                              gap_tol=0.0)
    assert tr[0]["gap"] == pytest.approx(ref.history[0]["gap"], rel=1e-10)
    assert tr[0]["gap"] < cold.gap


def test_warm_start_continues_the_ista_trajectory_on_the_device(B):
    """ISTA depends on the previous iterate only: T iterations from x_T (unscreened) equal
    2T iterations from zero, on the device in FP64."""
    c = datagen.lasso_small_fp64()
    D, y = c["D"], c["y"]
    L = oracle.spectral_norm_sq(D)
    Dd, yd = dev_matrix(D, "f64"), dev_vector(y, "f64")
    x_a, _, _, _ = B.solve_one(Dd, yd, 0.5, rule="ista", test="none", step_L=L, gap_tol=0.0,
                               max_iter=80)
    x_b, _, _, _ = B.solve_one(Dd, yd, 0.5, rule="ista", test="none", step_L=L, gap_tol=0.0,
                               max_iter=40)
    x_c, _, _, _ = B.solve_one(Dd, yd, 0.5, rule="ista", test="none", step_L=L, gap_tol=0.0,
                               max_iter=40, x0=x_b)
    assert rel_err(x_c.cpu().numpy(), x_a.cpu().numpy()) <= 1e-12


@pytest.mark.parametrize("rule", ["ista", "fista"])
def test_warm_start_group_follows_the_oracle(B, rule):
    D = datagen.gaussian_dictionary(120, 600, 17)
    gp = datagen.contiguous_groups(600, 10)
    y, _ = datagen.group_signal(D, gp, 17)
    L = oracle.spectral_norm_sq(D)
    x0 = oracle.solve_group_lasso(D, y, gp, None, lam_ratio=0.4, rule="ista", test="none", L=L,
                                  max_iter=25, gap_tol=0.0).x
    ref = oracle.solve_group_lasso(D, y, gp, None, lam_ratio=0.4, rule=rule, test="dgst3", L=L,
                                   max_iter=80, gap_tol=0.0, record=True, x0=x0)
    Dd, yd = dev_matrix(D, "f64"), dev_vector(y, "f64")
    x, info, scr, tr = B.solve_one(Dd, yd, 0.4, group_ptr=gp, rule=rule, test="dgst3", step_L=L,
                                   gap_tol=0.0, max_iter=80, x0=dev_vector(x0, "f64"))
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-10
    assert [t["n_units"] for t in tr] == [h["n_active_groups"] for h in ref.history]


def test_warm_start_from_the_optimum_stops_at_once_fp32(B):
    """FP32, 2000 x 10000: started from a certified optimum, the first certificate already
    meets the tolerance."""
    D, y = _lasso(2000, 10000, 0)
    Di, yi = instance(D, y, "f32")
    L = oracle.spectral_norm_sq(Di)
    Dd, yd = dev_matrix(D, "f32"), dev_vector(yi, "f32")
    x, info, _, _ = B.solve_one(Dd, yd, 0.7, rule="fista", test="dst3", step_L=L, gap_tol=1e-7,
                                max_iter=20000)
    assert info["status"] == 0
    x2, info2, _, _ = B.solve_one(Dd, yd, 0.7, rule="fista", test="dst3", step_L=L,
                                  gap_tol=1e-6, max_iter=20000, x0=x)
    assert info2["status"] == 0 and info2["iters"] == 1
    assert info2["gap"] <= 1e-6 * float(yi @ yi)


def test_warm_start_columns_of_a_multi_signal_solve(B):
    """lasso_solve with B > 1 (FP32: single solves per column) reads column b of X_0 with
    X's leading dimension; each column equals its own single-signal warm solve."""
    import torch
    D = datagen.gaussian_dictionary(300, 1500, 4)
    Dd = dev_matrix(D, "f32")
    L = oracle.spectral_norm_sq(datagen.to_storage(D, "f32"))
    Y = np.stack([datagen.to_storage(datagen.lasso_signal(D, 40 + b)[0], "f32") for b in range(3)], 1)
    Yd = torch.from_numpy(np.ascontiguousarray(Y.T).astype(np.float32)).cuda().T
    X0 = torch.zeros(3, 1500, dtype=torch.float32, device="cuda").T
    for b in range(3):
        x, _, _, _ = B.solve_one(Dd, Yd[:, b].contiguous(), 0.5, rule="ista", test="safe",
                                 step_L=L, gap_tol=0.0, max_iter=15 + 5 * b)
        X0[:, b] = x
    X, infos = B.solve(Dd, Yd, [0.3, 0.5, 0.7], rule="fista", test="dst3", step_L=L,
                       gap_tol=1e-6, max_iter=20000, x0=X0)
    for b, r in enumerate((0.3, 0.5, 0.7)):
        x, info, _, _ = B.solve_one(Dd, Yd[:, b].contiguous(), r, rule="fista", test="dst3",
                                    step_L=L, gap_tol=1e-6, max_iter=20000,
                                    x0=X0[:, b].contiguous())
        assert torch.equal(X[:, b], x)
        assert infos[b]["iters"] == info["iters"]


def test_warm_start_is_refused_where_it_does_not_apply(B):
    import torch
    D, y = _lasso(200, 800, 5)
    Dd, yd = dev_matrix(D, "f32"), dev_vector(datagen.to_storage(y, "f32"), "f32")
    bad = torch.zeros(800, dtype=torch.float32, device="cuda")
    bad[17] = float("nan")
    with pytest.raises(B.DsError) as e:
        B.solve_one(Dd, yd, 0.5, x0=bad)
    assert e.value.status == B.DS_EINVAL
    # the batched bfloat16 path has no warm start
    Db = dev_matrix(D, "bf16")
    Y = yd.reshape(-1, 1).repeat(1, 4)
    Yc = torch.empty(4, 200, dtype=torch.float32, device="cuda").T
    Yc.copy_(Y)
    X0 = torch.zeros(4, 800, dtype=torch.float32, device="cuda").T
    with pytest.raises(B.DsError) as e:
        B.solve(Db, Yc, [0.5] * 4, x0=X0)
    assert e.value.status == B.DS_EINVAL


def test_served_warm_start_equals_the_direct_solve(B):
    import torch
    D = datagen.gaussian_dictionary(256, 1000, 21)
    Dd = dev_matrix(D, "f32")
    y = datagen.to_storage(datagen.lasso_signal(D, 3)[0], "f32").astype(np.float32)
    yd = torch.from_numpy(y).cuda()
    x0, _, _, _ = B.solve_one(Dd, yd, 0.4, rule="ista", test="safe", gap_tol=0.0, max_iter=10)
    S = B.Server(max_slots=2)
    did = S.add_dict(Dd)
    torch.cuda.synchronize()
    rid = S.submit(did, y, 0.4, gap_tol=1e-6, max_iter=20000, x0=x0.cpu().numpy())
    t0 = time.time()
    while (r := S.poll(rid, did)) is None:
        assert time.time() - t0 < 60
        time.sleep(0.001)
    xs, info = r
    S.close()
    # the direct solve with the server's cached step constant
    xd, infod, _, _ = B.solve_one(Dd, yd, 0.4, step_L=info["L"], gap_tol=1e-6, max_iter=20000,
                                  x0=x0)
    assert info["status"] == 0
    assert np.array_equal(xs, xd.cpu().numpy()) and info["iters"] == infod["iters"]


# ------------------------------------------------------------ DS_NOT_CONVERGED
def test_not_converged_reports_x_and_gap(B):
    import torch
    D, y = _lasso(500, 2500, 8)
    Di, yi = instance(D, y, "f32")
    Dd, yd = dev_matrix(D, "f32"), dev_vector(yi, "f32")
    prob = B.make_problem(Dd)
    prm = B.make_params(rule="fista", test="dst3", gap_tol=1e-9, max_iter=7)
    x = torch.full((2500,), float("nan"), dtype=torch.float32, device="cuda")
    info = B.Info()
    st = B._lib.ds_solve_one(C.byref(prob), C.c_void_p(yd.data_ptr()), 0.3, C.byref(prm),
                             C.c_void_p(x.data_ptr()), None, None, 0, C.byref(info),
                             B._stream_ptr(None))
    assert st == B.DS_NOT_CONVERGED and info.status == B.DS_NOT_CONVERGED
    assert info.iters == 7 and info.gap > 1e-9 * float(yi @ yi)
    xh = x.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(xh)) and np.any(xh != 0.0)
    # the returned x_t is the prox step from the certified point: no larger objective
    p = oracle.primal_objective(Di, yi, xh, info.lambda_, float(np.abs(xh).sum()))
    assert p <= info.primal * (1 + 1e-6)
    assert info.primal - info.dual == pytest.approx(info.gap, rel=1e-9, abs=1e-15)
    # the same through lasso_solve, and on the batched bfloat16 path
    X, infos = B.solve(Dd, yd, [0.3], gap_tol=1e-9, max_iter=7)
    assert infos[0]["status"] == B.DS_NOT_CONVERGED
    Db = dev_matrix(D, "bf16")
    Y = torch.empty(3, 500, dtype=torch.float32, device="cuda").T
    for b in range(3):
        Y[:, b] = yd
    X, infos = B.solve(Db, Y, [0.3, 0.5, 0.7], gap_tol=1e-9, max_iter=5)
    assert all(i["status"] == B.DS_NOT_CONVERGED and i["iters"] == 5 for i in infos)
    assert all(i["gap"] > 0.0 for i in infos)
    assert torch.isfinite(X).all()


# ------------------------------------------------------------ serving failure paths
def _wait(S, rid, did, timeout=60.0):
    t0 = time.time()
    while True:
        r = S.poll(rid, did)
        if r is not None:
            return r
        assert time.time() - t0 < timeout, "request was never admitted"
        time.sleep(0.001)


def test_admission_after_a_finished_request_under_a_one_request_budget(B):
    """max_slots = 8 and a budget between one and two requests' footprint: a request
    submitted after the previous one finished must be admitted (the idle worker that
    still holds the first request's memory has to give it back)."""
    import torch
    D = datagen.gaussian_dictionary(256, 1000, 21)
    Dd = dev_matrix(D, "f32")
    y = datagen.to_storage(datagen.lasso_signal(D, 9)[0], "f32").astype(np.float32)
    prm = B.make_params(gap_tol=1e-6, max_iter=20000)
    rid = C.c_uint64()
    budget = 1 << 16
    while True:  # smallest power of two holding one request: need <= budget < 2 need
        S = B.Server(max_slots=8, hbm_budget_bytes=budget)
        did = S.add_dict(Dd)
        torch.cuda.synchronize()
        st = B._lib.lasso_submit(S._h, did, y.ctypes.data_as(C.c_void_p), 0.5, C.byref(prm),
                                 C.byref(rid))
        if st == 0:
            break
        assert st == B.DS_ENOMEM
        S.close()
        budget *= 2
    first = _wait(S, rid.value, did)
    for k in range(6):
        r = _wait(S, S.submit(did, y, 0.5, gap_tol=1e-6, max_iter=20000), did)
        assert np.array_equal(r[0], first[0]), k
    S.close()


def test_a_slot_marked_failed_leaves_the_others_unchanged(B):
    import torch
    D = datagen.gaussian_dictionary(256, 1000, 21)
    Dd = dev_matrix(D, "f32")
    ys = [datagen.to_storage(datagen.lasso_signal(D, 60 + k)[0], "f32").astype(np.float32)
          for k in range(6)]

    def run(fail):
        if fail:
            os.environ["DS_SERVE_FAIL_REQUEST"] = "3"
        try:
            S = B.Server(max_slots=4)
        finally:
            os.environ.pop("DS_SERVE_FAIL_REQUEST", None)
        did = S.add_dict(Dd)
        torch.cuda.synchronize()
        rids = [S.submit(did, y, 0.4 + 0.05 * k, gap_tol=1e-6, max_iter=20000)
                for k, y in enumerate(ys)]
        out = {}
        for k, rid in enumerate(rids):
            try:
                out[k] = _wait(S, rid, did)
            except B.DsError as e:
                out[k] = e
        S.close()
        return rids, out

    rids, ref = run(False)
    rids_f, got = run(True)
    assert rids_f == rids and rids[2] == 3
    assert isinstance(got[2], B.DsError) and got[2].status == B.DS_EDEVICE
    assert "marked failed" in str(got[2])
    for k in (0, 1, 3, 4, 5):
        assert np.array_equal(got[k][0], ref[k][0]) and got[k][1]["iters"] == ref[k][1]["iters"]


# ------------------------------------------------------------ the experiments' stopping rule
@pytest.mark.parametrize("rule,test", [("ista", "safe"), ("fista", "dst3"), ("sparsa", "safe")])
def test_objective_change_stop_follows_the_oracle(B, rule, test):
    """obj_tol (the experiments section's relative objective change): FP64, the device stops
    at the oracle's iteration with the same iterate."""
    c = datagen.lasso_small_fp64()
    D, y = c["D"], c["y"]
    L = oracle.spectral_norm_sq(D)
    ref = oracle.solve_lasso(D, y, lam_ratio=0.5, rule=rule, test=test, L=L, max_iter=5000,
                             gap_tol=0.0, obj_tol=1e-7)
    assert ref.converged and ref.iters < 5000
    Dd, yd = dev_matrix(D, "f64"), dev_vector(y, "f64")
    x, info, _, tr = B.solve_one(Dd, yd, 0.5, rule=rule, test=test, step_L=L, gap_tol=0.0,
                                 max_iter=5000, obj_tol=1e-7)
    assert info["status"] == 0 and info["iters"] == ref.iters
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-10
