"""Backtracking step sizes (DS_STEP_BACKTRACK, the rule of Beck and Teboulle that Table 1
names for ISTA and FISTA) on the single-signal path: parity with the FP64 oracle's rule,
agreement with the constant-step path when nothing is rejected, the served path, and the
batched path's refusal."""
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


def _lasso_case(N, K, seed, p=0.02):
    D = datagen.gaussian_dictionary(N, K, seed)
    y, _ = datagen.lasso_signal(D, seed, p=p)
    return D, y


@pytest.mark.parametrize("rule,test", [("ista", "safe"), ("fista", "dst3"), ("fista", "none"),
                                       ("ista", "dst3")])
def test_fp64_fixed_iterations_follow_the_oracle(B, rule, test):
    """FP64, a fixed number of iterations from a small L_0: the accept / reject decisions,
    the final L and the iterate match the oracle's."""
    c = datagen.lasso_small_fp64()
    D, y = c["D"], c["y"]
    T = 300
    ref = oracle.solve_lasso(D, y, lam_ratio=0.5, rule=rule, test=test, L=0.05, eta=2.0,
                             max_iter=T, gap_tol=0.0, record=True, step="backtracking")
    assert sum(not h["accepted"] for h in ref.history) >= 3
    x, info, _, tr = B.solve_one(dev_matrix(D, "f64"), dev_vector(y, "f64"), 0.5, rule=rule,
                                 test=test, step_L=0.05, gap_tol=0.0, max_iter=T,
                                 step="backtracking", bt_eta=2.0)
    assert info["iters"] == ref.iters == T
    assert info["L"] == ref.L
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-10
    assert [t["n_active"] for t in tr] == [h["n_active"] for h in ref.history]


@pytest.mark.parametrize("rule", ["ista", "fista"])
@pytest.mark.parametrize("ratio", [0.3, 0.7])
def test_fp32_to_gap_matches_the_oracle(B, rule, ratio):
    """FP32, FISTA / ISTA + DST3 to gap 1e-6 from the default L_0 (largest squared atom
    norm): the certified objective and the solution agree with the oracle's run of the same
    rule, and L ends at the same power of eta (or one step away when a decision falls within
    rounding of the threshold)."""
    D, y = _lasso_case(800, 3000, 7)
    Di, yi = instance(D, y, "f32")
    tol = 1e-6
    ref = oracle.solve_lasso(Di, yi, lam_ratio=ratio, rule=rule, test="dst3", max_iter=20000,
                             gap_tol=tol, step="backtracking")
    x, info, _, _ = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), ratio, rule=rule,
                                test="dst3", gap_tol=tol, max_iter=20000, step="backtracking",
                                trace=False, screened=False)
    yy = float(yi @ yi)
    assert info["status"] == 0 and ref.converged
    # L_0 agrees to rounding (the device squares FP64 atom norms); then powers of eta
    assert any(info["L"] == pytest.approx(f * ref.L, rel=1e-12) for f in (1.0, 2.0, 0.5))
    assert abs(info["primal"] - ref.primal_p) <= 2 * tol * yy
    xs = x.cpu().numpy().astype(np.float64)
    star = oracle.solve_lasso(Di, yi, lam=ref.lam, rule="fista", test="none", max_iter=200000,
                              gap_tol=1e-13)
    # both are certified within tol ||y||^2; their distance to the optimum is bounded alike
    assert oracle.primal_objective(Di, yi, xs, ref.lam, float(np.abs(xs).sum())) - star.primal \
        <= tol * yy * 1.01
    assert abs(info["iters"] - ref.iters) <= max(3, ref.iters // 10)


@pytest.mark.parametrize("rule", ["ista", "fista"])
def test_group_fp32_to_gap_matches_the_oracle(B, rule):
    D = datagen.gaussian_dictionary(400, 1500, 11)
    gp = datagen.contiguous_groups(1500, 10)
    y, _ = datagen.group_signal(D, gp, 3)
    Di, yi = instance(D, y, "f32")
    tol = 1e-6
    ref = oracle.solve_group_lasso(Di, yi, gp, lam_ratio=0.5, rule=rule, test="dgst3",
                                   max_iter=20000, gap_tol=tol, step="backtracking")
    x, info, _, _ = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), 0.5, group_ptr=gp,
                                rule=rule, test="dst3", gap_tol=tol, max_iter=20000,
                                step="backtracking", trace=False, screened=False)
    yy = float(yi @ yi)
    assert info["status"] == 0 and ref.converged
    # L_0 agrees to rounding (the device squares FP64 atom norms); then powers of eta
    assert any(info["L"] == pytest.approx(f * ref.L, rel=1e-12) for f in (1.0, 2.0, 0.5))
    assert abs(info["primal"] - ref.primal_p) <= 2 * tol * yy
    assert abs(info["iters"] - ref.iters) <= max(3, ref.iters // 10)


def test_global_bound_start_equals_the_constant_step(B):
    """From L_0 = ||D||_2^2 no step is rejected: the iterates are those of the constant
    step, bit for bit (the check pass only adds work)."""
    D, y = _lasso_case(600, 2400, 9)
    Di, yi = instance(D, y, "f32")
    L = oracle.spectral_norm_sq(Di) * (1 + 1e-9)
    Dd, yd = dev_matrix(D, "f32"), dev_vector(yi, "f32")
    kw = dict(rule="fista", test="dst3", step_L=L, gap_tol=1e-6, max_iter=5000, trace=False,
              screened=False)
    xa, ia, _, _ = B.solve_one(Dd, yd, 0.4, **kw)
    xb, ib, _, _ = B.solve_one(Dd, yd, 0.4, step="backtracking", **kw)
    assert ia["iters"] == ib["iters"] and ib["L"] == ia["L"]
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())


def test_served_request_equals_the_direct_solve(B):
    import time
    import torch
    D, y = _lasso_case(500, 2000, 13)
    Di, yi = instance(D, y, "f32")
    Dd = dev_matrix(D, "f32")
    x1, i1, _, _ = B.solve_one(Dd, dev_vector(yi, "f32"), 0.5, rule="fista", test="dst3",
                               gap_tol=1e-6, max_iter=20000, step="backtracking", trace=False,
                               screened=False)
    S = B.Server(max_slots=2)
    did = S.add_dict(Dd, store="f32")
    torch.cuda.synchronize()
    rid = S.submit(did, yi.astype(np.float32), 0.5, rule="fista", test="dst3", gap_tol=1e-6,
                   max_iter=20000, step="backtracking")
    t0 = time.time()
    got = None
    while got is None:
        got = S.poll(rid, did)
        assert time.time() - t0 < 60
        time.sleep(0.001)
    S.close()
    x2, i2 = got
    assert i2["iters"] == i1["iters"] and i2["L"] == i1["L"]
    assert np.array_equal(np.asarray(x2), x1.cpu().numpy())


def test_batched_bf16_path_refuses_backtracking(B):
    import torch
    D, y = _lasso_case(256, 1024, 15)
    Dd = dev_matrix(D, "bf16")
    Y = torch.from_numpy(np.stack([y, y]).astype(np.float32)).cuda().T
    with pytest.raises(B.DsError) as e:
        B.solve(Dd, Y, [0.5, 0.6], step="backtracking")
    assert e.value.status == B.DS_EINVAL
