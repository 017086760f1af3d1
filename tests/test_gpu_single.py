"""Parity of the single-signal HIP path with the FP64 oracle, through the C-ABI."""
import numpy as np
import pytest

import oracle
from paper_1412_4080_amd import datagen
from tests._util import (GAP_DELTA_SINGLE, dev_matrix, dev_vector, gap_difference_near_stop,
                         group_margins_ref, instance, lasso_margins_ref, rel_err,
                         screened_sets_agree, stop_iteration_bracket)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def _lasso_case(N, K, seed, p=0.02):
    D = datagen.gaussian_dictionary(N, K, seed)
    y, _ = datagen.lasso_signal(D, seed, p=p)
    return D, y


def _fixed_iter_parity(B, D, y, dtype, ratio, rule, test, T, tol_x, tol_obj, group=None):
    """Run T iterations on both sides with the same L and compare everything."""
    Di, yi = instance(D, y, dtype)
    L = oracle.spectral_norm_sq(Di)
    if group is None:
        ref = oracle.solve_lasso(Di, yi, lam_ratio=ratio, rule=rule, test=test, L=L, max_iter=T,
                                 gap_tol=0.0, record=True)
    else:
        gp, w = group
        ref = oracle.solve_group_lasso(Di, yi, gp, w, lam_ratio=ratio, rule=rule,
                                       test={"safe": "gsafe", "dst3": "dgst3"}.get(test, test),
                                       L=L, max_iter=T, gap_tol=0.0, record=True)
    Dd, yd = dev_matrix(D, dtype), dev_vector(yi, dtype)
    x, info, scr, tr = B.solve_one(Dd, yd, ratio, group_ptr=None if group is None else group[0],
                                   weights=None if group is None else group[1], rule=rule,
                                   test=test, step_L=L, gap_tol=0.0, max_iter=T)
    x = x.cpu().numpy().astype(np.float64)
    scr = scr.cpu().numpy().astype(bool)
    assert info["iters"] == ref.iters == T
    assert info["lambda_max"] == pytest.approx(ref.lam_max, rel=1e-12)
    assert rel_err(x, ref.x) <= tol_x, rel_err(x, ref.x)
    assert abs(info["primal"] - ref.primal_p) <= tol_obj * max(abs(ref.primal_p), 1e-30)
    assert abs(info["gap"] - ref.gap) <= tol_obj * max(abs(ref.primal_p), 1e-30) + 1e-12
    # screened sets: identical except within the threshold band
    r_ref = min([h["r"] for h in ref.history[:-1]], default=np.inf)
    r_gpu = min([t["radius"] for t in tr[:-1]], default=np.inf)
    if group is None:
        m = lasso_margins_ref(Di, yi, ref.lam, test)
        assert screened_sets_agree(scr, ref.screened, m, r_ref, r_gpu, info["radius_slack"])
    else:
        gp, w = group
        m = group_margins_ref(Di, yi, ref.lam, {"safe": "gsafe", "dst3": "dgst3"}.get(test, test),
                              gp, w)
        unit = np.repeat(np.arange(gp.size - 1), np.diff(gp))
        assert screened_sets_agree(scr, ref.screened, m, r_ref, r_gpu, info["radius_slack"], unit)
    return ref, x, info, tr


# ------------------------------------------------------------ FP64 small workload
@pytest.mark.parametrize("test", ["safe", "dst3", "none", "dome"])
def test_small_fp64_500_iterations(B, test):
    c = datagen.lasso_small_fp64()
    ref, x, info, tr = _fixed_iter_parity(B, c["D"], c["y"], "f64", 0.5, "ista", test, 500,
                                          1e-10, 1e-12)
    assert [t["n_active"] for t in tr] == [h["n_active"] for h in ref.history]
    assert [t["nnz"] for t in tr] == [h["nnz"] for h in ref.history]


# ------------------------------------------------------------ FP32 trajectories
@pytest.mark.parametrize("rule,test", [("fista", "dst3"), ("ista", "safe"), ("fista", "none"),
                                       ("ista", "dst3"), ("fista", "dome")])
@pytest.mark.parametrize("ratio", [0.2, 0.6, 0.9])
def test_fp32_fixed_iteration_parity(B, rule, test, ratio):
    D, y = _lasso_case(500, 2500, 5)
    ref, x, info, tr = _fixed_iter_parity(B, D, y, "f32", ratio, rule, test, 60, 1e-5, 1e-6)
    # active-set trajectory: identical up to band effects of a few atoms
    na_gpu = np.array([t["n_active"] for t in tr])
    na_ref = np.array([h["n_active"] for h in ref.history])
    assert np.max(np.abs(na_gpu - na_ref)) <= 2


def test_fp32_full_size_trajectory(B):
    """2000 x 10000 dictionary, FISTA + DST3: the launch configuration of the benchmark."""
    D, y = _lasso_case(2000, 10000, 0)
    for ratio in (0.5, 0.8):
        ref, x, info, tr = _fixed_iter_parity(B, D, y, "f32", ratio, "fista", "dst3", 40, 1e-5,
                                              1e-6)
    assert tr[-1]["n_active"] < 10000  # screening took effect at 0.8 lambda_*


@pytest.mark.parametrize("test", ["dst3", "dome"])
@pytest.mark.parametrize("ratio", [0.1, 0.5, 0.9])
def test_fp32_solve_to_tolerance_is_certified(B, ratio, test):
    D, y = _lasso_case(400, 2000, 9)
    Di, yi = instance(D, y, "f32")
    L = oracle.spectral_norm_sq(Di)
    Dd, yd = dev_matrix(D, "f32"), dev_vector(yi, "f32")
    x, info, scr, tr = B.solve_one(Dd, yd, ratio, rule="fista", test=test, step_L=L,
                                   gap_tol=1e-6, max_iter=20000)
    assert info["status"] == 0 and info["gap"] <= 1e-6 * float(yi @ yi)
    x = x.cpu().numpy().astype(np.float64)
    scr = scr.cpu().numpy().astype(bool)
    star = oracle.solve_lasso(Di, yi, lam=info["lambda_"], rule="fista", test="none", L=L,
                              max_iter=200000, gap_tol=1e-13)
    p_gpu = oracle.primal_objective(Di, yi, x, info["lambda_"], float(np.abs(x).sum()))
    # the certificate bounds the objective error of the returned point
    assert p_gpu - star.primal <= info["gap"] + 1e-9
    # the GPU's own objective evaluation agrees with an FP64 evaluation of its iterate
    assert star.primal <= p_gpu
    # safety: every screened atom is certified inactive and zero at the optimum
    cert, gstar = oracle.certified_inactive_lasso(Di, yi, info["lambda_"], star.x)
    assert gstar < 1e-11
    assert np.all(cert[scr]), np.flatnonzero(scr & ~cert)[:10]
    assert not star.x[scr].any()
    # the device gap stays within GAP_DELTA_SINGLE tol of the oracle's near the stop, so the
    # stopping iteration lies in the bracket that bound implies
    tol_abs = 1e-6 * float(yi @ yi)
    ref = oracle.solve_lasso(Di, yi, lam=info["lambda_"], rule="fista", test=test, L=L,
                             max_iter=info["iters"], gap_tol=0.0, record=True)
    assert gap_difference_near_stop(tr, ref.history, tol_abs) <= GAP_DELTA_SINGLE * tol_abs
    t_lo, t_hi = stop_iteration_bracket(Di, yi, info["lambda_"], L, tol_abs, test=test)
    assert t_lo <= info["iters"] <= t_hi, (info["iters"], t_lo, t_hi)


# ------------------------------------------------------------ Dome test
def _correlated_case(N, K, seed, corr=0.8):
    """Unit atoms sharing a common direction (where the dome's cut removes most)."""
    rng = np.random.default_rng(seed)
    D = corr * rng.standard_normal((N, 1)) + rng.standard_normal((N, K))
    D /= np.linalg.norm(D, axis=0)
    y = D[:, :5] @ rng.standard_normal(5) + 0.1 * rng.standard_normal(N)
    return D, y / np.linalg.norm(y)


@pytest.mark.parametrize("ratio", [0.5, 0.8])
def test_dome_follows_the_oracle_and_screens_at_least_dst3(B, ratio):
    """FP64 on correlated atoms: the Dome run's active sets per iteration equal the
    oracle's, and are never larger than the DST3 run's (the dome lies inside DST3's ball)."""
    D, y = _correlated_case(300, 1500, 41)
    T = 150
    ref, x, info, tr = _fixed_iter_parity(B, D, y, "f64", ratio, "fista", "dome", T, 1e-10,
                                          1e-12)
    assert [t["n_active"] for t in tr] == [h["n_active"] for h in ref.history]
    L = oracle.spectral_norm_sq(D)
    _, _, _, tr3 = B.solve_one(dev_matrix(D, "f64"), dev_vector(y, "f64"), ratio, rule="fista",
                               test="dst3", step_L=L, gap_tol=0.0, max_iter=T)
    na_dome = np.array([t["n_active"] for t in tr])
    na_dst3 = np.array([t["n_active"] for t in tr3])
    assert np.all(na_dome <= na_dst3)


def test_dome_refused_for_groups(B):
    """The Dome test is stated for the Lasso: grouped problems are refused, single-signal
    and batched."""
    import torch
    D = datagen.gaussian_dictionary(256, 1000, 15)
    gp = datagen.contiguous_groups(1000, 10)
    y, _ = datagen.group_signal(D, gp, 3)
    with pytest.raises(B.DsError) as e:
        B.solve_one(dev_matrix(D, "f32"), dev_vector(y, "f32"), 0.5, group_ptr=gp, test="dome")
    assert e.value.status == B.DS_EINVAL
    Dd = dev_matrix(D, "bf16")
    Y = torch.from_numpy(np.stack([y, y]).astype(np.float32)).cuda().T
    with pytest.raises(B.DsError) as e:
        B.solve(Dd, Y, [0.5, 0.6], group_ptr=gp, test="dome")
    assert e.value.status == B.DS_EINVAL


# ------------------------------------------------------------ Group-Lasso
@pytest.mark.parametrize("rule,test", [("ista", "dst3"), ("ista", "safe"), ("fista", "dst3"),
                                       ("ista", "none")])
@pytest.mark.parametrize("ratio", [0.3, 0.7])
def test_group_fp32_fixed_iteration_parity(B, rule, test, ratio):
    D = datagen.gaussian_dictionary(500, 2500, 7)
    gp = datagen.contiguous_groups(2500, 10)
    y, _ = datagen.group_signal(D, gp, 3)
    w = np.sqrt(10.0) * np.ones(250)
    _fixed_iter_parity(B, D, y, "f32", ratio, rule, test, 60, 1e-5, 1e-6, group=(gp, w))


@pytest.mark.parametrize("ratio", [0.3, 0.7])
def test_group_full_size_workload(B, ratio):
    """The Group-Lasso configuration at full size: 2000 x 10000 FP32, 1000 contiguous groups
    of 10 (w_g = sqrt(10)), ISTA with the dynamic group sphere test.  A 30-iteration
    trajectory matches the oracle's; the solve to gap 1e-6 is checked by a certificate the
    oracle computes from the returned x alone (no full-size oracle solve): its duality gap,
    and every screened atom provably inactive."""
    D = datagen.gaussian_dictionary(2000, 10000, 0)
    gp = datagen.contiguous_groups(10000, 10)
    y, _ = datagen.group_signal(D, gp, 0)
    w = np.sqrt(10.0) * np.ones(1000)
    _fixed_iter_parity(B, D, y, "f32", ratio, "ista", "safe", 30, 1e-5, 1e-6, group=(gp, w))
    Di, yi = instance(D, y, "f32")
    L = oracle.spectral_norm_sq(Di)
    x, info, scr, _ = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), ratio,
                                  group_ptr=gp, rule="ista", test="safe", step_L=L,
                                  gap_tol=1e-6, max_iter=50000, trace=False)
    assert info["status"] == 0 and info["gap"] <= 1e-6 * float(yi @ yi)
    xs = x.cpu().numpy().astype(np.float64)
    amask, gmask, gap_x = oracle.certified_inactive_group(Di, yi, info["lambda_"], xs, gp)
    assert gap_x <= 2e-6 * float(yi @ yi)
    scr = scr.cpu().numpy().astype(bool)
    assert np.all(amask[scr]), np.flatnonzero(scr & ~amask)[:10]
    if ratio == 0.7:
        assert scr.sum() > 0


@pytest.mark.parametrize("ratio", [0.3, 0.7])
def test_group_solve_to_tolerance_is_certified(B, ratio):
    D = datagen.gaussian_dictionary(400, 2000, 8)
    gp = datagen.contiguous_groups(2000, 10)
    y, _ = datagen.group_signal(D, gp, 4)
    Di, yi = instance(D, y, "f32")
    L = oracle.spectral_norm_sq(Di)
    x, info, scr, tr = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), ratio,
                                   group_ptr=gp, rule="ista", test="dgst3", step_L=L,
                                   gap_tol=1e-6, max_iter=50000)
    assert info["status"] == 0
    scr = scr.cpu().numpy().astype(bool)
    star = oracle.solve_group_lasso(Di, yi, gp, None, lam=info["lambda_"], rule="fista",
                                    test="none", L=L, max_iter=200000, gap_tol=1e-13)
    amask, gmask, gstar = oracle.certified_inactive_group(Di, yi, info["lambda_"], star.x, gp)
    assert gstar < 1e-11
    assert np.all(amask[scr])


# ------------------------------------------------------------ group sizes and partitions
@pytest.mark.parametrize("sizes", [(5,), (50,), (64,), (100,), (128,), (3, 17, 64, 1, 9),
                                   (1, 128, 37, 100, 65, 2)])
def test_group_sizes_fixed_iteration_parity(B, sizes):
    """Group sizes of the paper's sweep (5, 10, 50, 100), the largest supported (128 atoms:
    two per lane), and groups of mixed sizes, with the default weights sqrt(|g|)."""
    sz = np.resize(np.array(sizes, dtype=np.int64), 2400 // int(np.mean(sizes)))
    gp = np.concatenate([[0], np.cumsum(sz)]).astype(np.int64)
    K = int(gp[-1])
    D = datagen.gaussian_dictionary(400, K, 21)
    y, _ = datagen.group_signal(D, gp, 5)
    w = np.sqrt(np.diff(gp).astype(np.float64))
    for rule, test in (("fista", "dst3"), ("ista", "safe")):
        _fixed_iter_parity(B, D, y, "f32", 0.5, rule, test, 50, 1e-5, 1e-6, group=(gp, w))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("sizes", [(5,), (3, 16, 9), (20, 32), (50, 7), (100,), (128, 1, 65)])
def test_group_spectral_norms_give_the_backtracking_start(B, dtype, sizes):
    """The backtracking rule starts from L_0 = max_g ||D_g||_2^2 and, stopped at the first
    iteration, returns it unchanged: the largest group spectral norm (Gram matrix,
    tridiagonal reduction, multisection) against the singular value decomposition.  One
    group is scaled up so that the maximum falls on a different group each time, and one
    repeats a column (a rank-deficient Gram matrix)."""
    sz = np.resize(np.array(sizes, dtype=np.int64), max(8, 1200 // int(np.mean(sizes))))
    gp = np.concatenate([[0], np.cumsum(sz)]).astype(np.int64)
    K, G = int(gp[-1]), sz.size
    D = datagen.gaussian_dictionary(300, K, 31)
    rng = np.random.default_rng(int(sum(sizes)))
    big = int(rng.integers(G))
    D[:, gp[big]:gp[big + 1]] *= 1.5
    rd = (big + 1) % G
    if sz[rd] > 1:
        D[:, gp[rd] + 1] = D[:, gp[rd]]
        D[:, gp[rd]:gp[rd + 1]] *= 1.7
    y, _ = datagen.group_signal(D, gp, 6)
    Di, yi = instance(D, y, dtype)
    ref = oracle.group_spectral_norms(Di, [np.arange(gp[g], gp[g + 1]) for g in range(G)])
    _, info, _, _ = B.solve_one(dev_matrix(D, dtype), dev_vector(yi, dtype), 0.5, group_ptr=gp,
                                rule="fista", test="dst3", gap_tol=0.0, max_iter=1,
                                step="backtracking", trace=False, screened=False)
    assert info["iters"] == 1
    assert info["L"] == pytest.approx(float(np.max(ref)) ** 2, rel=1e-12)


def test_non_contiguous_partition_through_a_column_permutation(B):
    """Any partition of the atoms is solved by permuting the columns of D so that each group
    is contiguous; the oracle solves the partition as given."""
    K = 1500
    rng = np.random.default_rng(77)
    perm = rng.permutation(K)
    sizes = np.resize(np.array([4, 11, 7, 20]), 200)
    sizes = sizes[np.cumsum(sizes) <= K]
    sizes = np.append(sizes, K - sizes.sum())
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    groups = [perm[bounds[g]:bounds[g + 1]] for g in range(sizes.size)]
    D = datagen.gaussian_dictionary(300, K, 23)
    Di = datagen.to_storage(D, "f32")
    rng2 = np.random.default_rng(78)
    x0 = np.zeros(K)
    for g in groups[::25]:
        x0[g] = rng2.standard_normal(g.size)
    y = Di @ x0 + 0.01 * rng2.standard_normal(300)
    yi = datagen.to_storage(y / np.linalg.norm(y), "f32")
    L = oracle.spectral_norm_sq(Di)
    T = 60
    ref = oracle.solve_group_lasso(Di, yi, groups, lam_ratio=0.5, rule="fista", test="dgst3",
                                   L=L, max_iter=T, gap_tol=0.0)
    order = np.concatenate(groups)                       # column order that makes groups contiguous
    Dp = dev_matrix(D[:, order], "f32")
    gp = bounds.astype(np.int64)
    x, info, _, _ = B.solve_one(Dp, dev_vector(yi, "f32"), 0.5, group_ptr=gp, rule="fista",
                                test="dst3", step_L=L, gap_tol=0.0, max_iter=T, trace=False,
                                screened=False)
    xp = np.zeros(K)
    xp[order] = x.cpu().numpy().astype(np.float64)
    assert info["iters"] == ref.iters == T
    assert rel_err(xp, ref.x) <= 1e-5
    assert abs(info["gap"] - ref.gap) <= 1e-6 * ref.primal_p + 1e-12


# ------------------------------------------------------------ edge cases
def test_trivial_regime_returns_zero(B):
    D, y = _lasso_case(200, 800, 2)
    Dd, yd = dev_matrix(D, "f32"), dev_vector(y, "f32")
    for ratio in (1.0, 1.5):
        x, info, scr, tr = B.solve_one(Dd, yd, ratio)
        assert info["iters"] == 0 and info["status"] == 0
        assert not x.cpu().numpy().any() and scr.cpu().numpy().all()


@pytest.mark.parametrize("N,K,ldd", [(37, 101, 37), (130, 333, 136), (1, 1, 1), (64, 5, 64),
                                     (257, 1031, 257)])
@pytest.mark.parametrize("dtype", ["f32", "f64", "bf16"])
def test_ragged_shapes(B, N, K, ldd, dtype):
    import torch
    D = datagen.gaussian_dictionary(N, K, 11)
    rng = np.random.default_rng(12)
    y = rng.standard_normal(N)
    y /= np.linalg.norm(y)
    Di, yi = instance(D, y, dtype)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    buf = torch.zeros(K, ldd, dtype=tdt)
    buf[:, :N] = torch.from_numpy(np.ascontiguousarray(Di.T))
    Dd = buf.to("cuda").T[:N, :]
    assert Dd.stride() == (1, ldd)
    L = oracle.spectral_norm_sq(Di)
    ref = oracle.solve_lasso(Di, yi, lam_ratio=0.4, rule="fista", test="dst3", L=L, max_iter=25,
                             gap_tol=0.0)
    x, info, scr, tr = B.solve_one(Dd, dev_vector(yi, dtype), 0.4, rule="fista", test="dst3",
                                   step_L=L, gap_tol=0.0, max_iter=25)
    tol = 1e-10 if dtype == "f64" else 1e-5
    if ref.iters == 0:
        assert info["iters"] == 0 and not x.cpu().numpy().any()
    else:
        assert rel_err(x.cpu().numpy(), ref.x) <= tol


def test_non_unit_and_zero_atoms(B):
    D = datagen.gaussian_dictionary(300, 1200, 13)
    rng = np.random.default_rng(14)
    D = np.asfortranarray(D * rng.uniform(0.5, 2.0, size=1200)[None, :])
    D[:, 17] = 0.0
    y, _ = datagen.lasso_signal(D, 15)
    ref, x, info, tr = _fixed_iter_parity(B, D, y, "f32", 0.5, "fista", "dst3", 80, 1e-5, 1e-6)
    assert x[17] == 0.0


def test_deterministic(B):
    D, y = _lasso_case(500, 2500, 16)
    Dd, yd = dev_matrix(D, "f32"), dev_vector(y, "f32")
    L = oracle.spectral_norm_sq(instance(D, y, "f32")[0])
    a = B.solve_one(Dd, yd, 0.3, step_L=L, gap_tol=1e-6)
    b = B.solve_one(Dd, yd, 0.3, step_L=L, gap_tol=1e-6)
    assert np.array_equal(a[0].cpu().numpy(), b[0].cpu().numpy())
    assert a[1]["iters"] == b[1]["iters"]


def test_lambda_max_and_spectral_norm(B):
    D, y = _lasso_case(700, 3000, 17)
    Di, yi = instance(D, y, "f32")
    Dd = dev_matrix(D, "f32")
    lm, arg = B.lambda_max(Dd, dev_vector(yi, "f32"))
    ref, iref = oracle.lambda_max_lasso(Di, yi)
    assert lm == pytest.approx(ref, rel=1e-13) and arg == iref
    L = B.spectral_norm_sq(Dd, 300)
    Lx = oracle.spectral_norm_sq(Di)
    assert Lx * (1 - 1e-12) <= L <= Lx * 1.02


def test_batched_call_matches_single(B):
    import torch
    D, _ = _lasso_case(300, 1500, 18)
    Ys = np.stack([datagen.lasso_signal(D, j)[0] for j in range(3)], axis=1)
    Dd = dev_matrix(D, "f32")
    Yd = torch.from_numpy(np.ascontiguousarray(Ys.T.astype(np.float32))).cuda().T
    L = oracle.spectral_norm_sq(instance(D, Ys[:, 0], "f32")[0])
    X, infos = B.solve(Dd, Yd, [0.3, 0.5, 0.7], step_L=L, gap_tol=1e-6)
    for j, r in enumerate([0.3, 0.5, 0.7]):
        x1, i1, _, _ = B.solve_one(Dd, Yd[:, j].contiguous(), r, step_L=L, gap_tol=1e-6)
        assert np.array_equal(X[:, j].cpu().numpy(), x1.cpu().numpy())
        assert infos[j]["iters"] == i1["iters"]


def test_instrumented_launch_records(B):
    """An instrumented solve records, per iteration, its correlation pass (active atoms,
    algorithmic bytes, device-clock time), the residual pass after it and the iteration as a
    whole, in launch order; the counters agree with the records."""
    D, y = _lasso_case(300, 1500, 41)
    Di, yi = instance(D, y, "f32")
    L = oracle.spectral_norm_sq(Di)
    B.stats_reset()
    B.stats_enable(True)
    try:
        _, info, _, tr = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), 0.5, step_L=L,
                                     gap_tol=1e-6, max_iter=2000)
    finally:
        B.stats_enable(False)
    recs = B.stats_launches()
    st = B.stats_read()
    T = info["iters"]
    corr = [r for r in recs if r["kernel"] == B.STAT_CORR]
    res = [r for r in recs if r["kernel"] == B.STAT_RESID]
    it = [r for r in recs if r["kernel"] == B.STAT_ITER]
    assert len(corr) == len(res) == len(it) == T == st[B.STAT_CORR]["launches"] == st[B.STAT_RESID]["launches"]
    assert [r["n_atoms"] for r in corr] == [t["n_active"] for t in tr]
    assert [r["n_atoms"] for r in res] == [r["n_atoms"] for r in corr] == [r["n_atoms"] for r in it]
    assert all(r["ms"] > 0 for r in corr + res + it)
    assert all(i["ms"] >= r["ms"] for i, r in zip(it, res))
    assert all(r["bytes"] >= 2 * 300 * 4 for r in res)
    assert sum(r["bytes"] for r in corr) == pytest.approx(st[B.STAT_CORR]["bytes"], rel=1e-12)
    B.stats_reset()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_concurrent_columns_match_single_solves(B, dtype):
    """lasso_solve with more columns than solve lanes (9 signals, lambdas out of order, one
    the low ones capped by max_iter): every column, its info and its screened mask equal the
    column's own single-signal solve bit for bit, DS_NOT_CONVERGED included."""
    import torch
    D, _ = _lasso_case(400, 2000, 23)
    Ys = np.stack([datagen.lasso_signal(D, j)[0] for j in range(9)], axis=1)
    Di = datagen.to_storage(D, dtype)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Dd = dev_matrix(D, dtype)
    Yd = torch.from_numpy(np.ascontiguousarray(datagen.to_storage(Ys, dtype).T)).to(
        device="cuda", dtype=tdt).T
    L = oracle.spectral_norm_sq(Di)
    ratios = [0.7, 0.2, 0.9, 0.4, 0.1, 0.6, 0.3, 0.8, 0.5]
    X, infos, mask = B.solve(Dd, Yd, ratios, step_L=L, gap_tol=1e-8, max_iter=150,
                             screened=True)
    assert any(i["status"] != 0 for i in infos)     # the lowest ratios stop at max_iter
    for j, r in enumerate(ratios):
        x1, i1, s1, _ = B.solve_one(Dd, Yd[:, j].contiguous(), r, step_L=L, gap_tol=1e-8,
                                    max_iter=150, trace=False)
        assert np.array_equal(X[:, j].cpu().numpy(), x1.cpu().numpy()), j
        assert np.array_equal(mask[:, j].cpu().numpy(), s1.cpu().numpy()), j
        assert infos[j]["iters"] == i1["iters"] and infos[j]["status"] == i1["status"]
        assert infos[j]["gap"] == i1["gap"]


def test_concurrent_columns_report_a_bad_column(B):
    """A non-finite observation in one column of a concurrent multi-signal call ends the call
    with DS_EINVAL and its message, and the next call on the same lanes runs normally."""
    import torch
    D, _ = _lasso_case(200, 900, 47)
    Ys = np.stack([datagen.lasso_signal(D, j)[0] for j in range(6)], axis=1).astype(np.float32)
    Ys[5, 3] = np.nan
    Dd = dev_matrix(D, "f32")
    L = oracle.spectral_norm_sq(datagen.to_storage(D, "f32"))
    Yd = torch.from_numpy(np.ascontiguousarray(Ys.T)).cuda().T
    with pytest.raises(B.DsError) as e:
        B.solve(Dd, Yd, [0.5] * 6, step_L=L, gap_tol=1e-6, max_iter=5000)
    assert e.value.status == B.DS_EINVAL and "NaN" in str(e.value)
    Ys[5, 3] = 0.0
    Yd = torch.from_numpy(np.ascontiguousarray(Ys.T)).cuda().T
    X, infos = B.solve(Dd, Yd, [0.5] * 6, step_L=L, gap_tol=1e-6, max_iter=5000)
    x1, i1, _, _ = B.solve_one(Dd, Yd[:, 3].contiguous(), 0.5, step_L=L, gap_tol=1e-6,
                               max_iter=5000, trace=False)
    assert all(i["status"] == 0 for i in infos)
    assert np.array_equal(X[:, 3].cpu().numpy(), x1.cpu().numpy())


def test_concurrent_group_columns_match_single_solves(B):
    """glasso_solve over 6 signals (groups of 10) runs the columns concurrently: each column
    equals its own single-signal Group-Lasso solve bit for bit."""
    import torch
    D = datagen.gaussian_dictionary(300, 1500, 29)
    gp = datagen.contiguous_groups(1500, 10)
    Ys = np.stack([datagen.group_signal(D, gp, j)[0] for j in range(6)], axis=1)
    Dd = dev_matrix(D, "f32")
    Yd = torch.from_numpy(np.ascontiguousarray(Ys.T.astype(np.float32))).cuda().T
    L = oracle.spectral_norm_sq(datagen.to_storage(D, "f32"))
    ratios = [0.5, 0.3, 0.8, 0.2, 0.6, 0.4]
    X, infos = B.solve(Dd, Yd, ratios, group_ptr=gp, rule="ista", test="dst3", step_L=L,
                       gap_tol=1e-6, max_iter=20000)
    for j, r in enumerate(ratios):
        x1, i1, _, _ = B.solve_one(Dd, Yd[:, j].contiguous(), r, group_ptr=gp, rule="ista",
                                   test="dst3", step_L=L, gap_tol=1e-6, max_iter=20000,
                                   trace=False)
        assert np.array_equal(X[:, j].cpu().numpy(), x1.cpu().numpy()), j
        assert infos[j]["iters"] == i1["iters"]


@pytest.mark.parametrize("rule,test", [("fista", "dst3"), ("ista", "safe"), ("fista", "dome")])
def test_static_screening_parity(B, rule, test):
    """Static mode (the test once, with the first dual point): same iterates, gap and
    screened set as the oracle's static run."""
    D, y = _lasso_case(500, 2500, 31)
    Di, yi = instance(D, y, "f32")
    L = oracle.spectral_norm_sq(Di)
    T = 40
    ref = oracle.solve_lasso(Di, yi, lam_ratio=0.6, rule=rule, test=test, L=L, max_iter=T,
                             gap_tol=0.0, record=True, screening="static")
    x, info, scr, tr = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), 0.6, rule=rule,
                                   test=test, step_L=L, gap_tol=0.0, max_iter=T,
                                   screening="static")
    x = x.cpu().numpy().astype(np.float64)
    scr = scr.cpu().numpy().astype(bool)
    assert info["iters"] == T
    assert rel_err(x, ref.x) <= 1e-5
    assert abs(info["gap"] - ref.gap) <= 1e-6 * ref.primal_p + 1e-12
    m = lasso_margins_ref(Di, yi, ref.lam, test)
    assert screened_sets_agree(scr, ref.screened, m, ref.history[0]["r"], tr[0]["radius"],
                               info["radius_slack"])
    # the active set never changes after the first iteration
    assert len({t["n_active"] for t in tr[1:]}) == 1
