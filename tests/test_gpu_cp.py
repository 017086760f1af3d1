"""Chambolle-Pock (the Table 1 row with a carried dual iterate) on the single-signal path:
parity with the FP64 oracle (iterations, active sets per iteration, the returned certified
point, gap), a trajectory computed by hand, solves to the gap tolerance, groups, the served
path and the batched path's refusal."""
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


@pytest.mark.parametrize("test,gamma", [("none", 0.0), ("safe", 0.0), ("dst3", 0.0),
                                        ("dst3", 0.05)])
def test_fp64_fixed_iterations_follow_the_oracle(B, test, gamma):
    c = datagen.lasso_small_fp64()
    D, y = c["D"], c["y"]
    L = oracle.spectral_norm_sq(D)
    T = 300
    ref = oracle.solve_lasso(D, y, lam_ratio=0.5, rule="cp", test=test, L=L, max_iter=T,
                             gap_tol=0.0, record=True, cp_gamma=gamma)
    x, info, _, tr = B.solve_one(dev_matrix(D, "f64"), dev_vector(y, "f64"), 0.5, rule="cp",
                                 test=test, step_L=L, gap_tol=0.0, max_iter=T, cp_gamma=gamma)
    assert info["iters"] == ref.iters == T
    assert [t["n_active"] for t in tr] == [h["n_active"] for h in ref.history]
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-10
    assert abs(info["gap"] - ref.gap) <= 1e-10 * ref.primal_p
    assert info["primal"] == pytest.approx(ref.primal_p, rel=1e-12)


def test_fp64_groups_follow_the_oracle(B):
    c = datagen.lasso_small_fp64()
    gp = datagen.contiguous_groups(500, 10)
    y, _ = datagen.group_signal(c["D"], gp, 2)
    L = oracle.spectral_norm_sq(c["D"])
    T = 200
    ref = oracle.solve_group_lasso(c["D"], y, gp, lam_ratio=0.5, rule="cp", test="dgst3", L=L,
                                   max_iter=T, gap_tol=0.0, record=True)
    x, info, _, tr = B.solve_one(dev_matrix(c["D"], "f64"), dev_vector(y, "f64"), 0.5,
                                 group_ptr=gp, rule="cp", test="dst3", step_L=L, gap_tol=0.0,
                                 max_iter=T)
    assert info["iters"] == ref.iters == T
    assert [t["n_active"] for t in tr] == [h["n_active"] for h in ref.history]
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-10


def test_scalar_trajectory_computed_by_hand(B):
    """D = [1], y = 1, lambda = 1/2, tau = sigma = L = 1: after four iterations the certified
    point is u_3 = 1/2 with P(u_3) = 3/8 (the hand computation of the oracle's pin)."""
    import torch
    D = torch.ones(1, 1, dtype=torch.float64, device="cuda")
    y = torch.ones(1, dtype=torch.float64, device="cuda")
    x, info, _, _ = B.solve_one(D, y, 0.5, lambda_relative=False, rule="cp", test="none",
                                step_L=1.0, cp_tau=1.0, cp_sigma=1.0, gap_tol=0.0, max_iter=4)
    assert info["iters"] == 4
    assert float(x.cpu()[0]) == 0.5 and info["primal"] == 0.375


@pytest.mark.parametrize("ratio", [0.3, 0.7])
def test_fp32_to_gap_is_certified(B, ratio):
    D = datagen.gaussian_dictionary(800, 3000, 7)
    y, _ = datagen.lasso_signal(D, 7)
    Di, yi = instance(D, y, "f32")
    tol = 1e-6
    ref = oracle.solve_lasso(Di, yi, lam_ratio=ratio, rule="cp", test="dst3", max_iter=20000,
                             gap_tol=tol)
    x, info, scr, _ = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), ratio, rule="cp",
                                  test="dst3", gap_tol=tol, max_iter=20000, trace=False)
    yy = float(yi @ yi)
    assert info["status"] == 0 and ref.converged
    xs = x.cpu().numpy().astype(np.float64)
    star = oracle.solve_lasso(Di, yi, lam=ref.lam, rule="fista", test="none", max_iter=200000,
                              gap_tol=1e-13)
    p_x = oracle.primal_objective(Di, yi, xs, ref.lam, float(np.abs(xs).sum()))
    assert p_x - star.primal <= tol * yy * 1.01
    assert p_x == pytest.approx(info["primal"], rel=1e-5)   # the returned point is the certified one
    cert, _ = oracle.certified_inactive_lasso(Di, yi, ref.lam, star.x)
    assert np.all(cert[scr.cpu().numpy().astype(bool)])
    assert not star.x[scr.cpu().numpy().astype(bool)].any()
    assert abs(info["iters"] - ref.iters) <= max(5, ref.iters // 10)


def test_served_request_equals_the_direct_solve(B):
    import time
    import torch
    D = datagen.gaussian_dictionary(500, 2000, 13)
    y, _ = datagen.lasso_signal(D, 13)
    Di, yi = instance(D, y, "f32")
    Dd = dev_matrix(D, "f32")
    L = oracle.spectral_norm_sq(Di)
    x1, i1, _, _ = B.solve_one(Dd, dev_vector(yi, "f32"), 0.5, rule="cp", test="dst3", step_L=L,
                               gap_tol=1e-6, max_iter=20000, trace=False, screened=False)
    S = B.Server(max_slots=2)
    did = S.add_dict(Dd, store="f32")
    torch.cuda.synchronize()
    rid = S.submit(did, yi.astype(np.float32), 0.5, rule="cp", test="dst3", step_L=L,
                   gap_tol=1e-6, max_iter=20000)
    t0 = time.time()
    got = None
    while got is None:
        got = S.poll(rid, did)
        assert time.time() - t0 < 60
        time.sleep(0.001)
    S.close()
    x2, i2 = got
    assert i2["iters"] == i1["iters"]
    assert np.array_equal(np.asarray(x2), x1.cpu().numpy())


def test_batched_bf16_path_refuses_cp(B):
    import torch
    D = datagen.gaussian_dictionary(256, 1024, 15)
    y, _ = datagen.lasso_signal(D, 15)
    Y = torch.from_numpy(np.stack([y, y]).astype(np.float32)).cuda().T
    with pytest.raises(B.DsError) as e:
        B.solve(dev_matrix(D, "bf16"), Y, [0.5, 0.6], rule="cp")
    assert e.value.status == B.DS_EINVAL
