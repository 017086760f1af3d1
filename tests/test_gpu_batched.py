"""Parity of the batched bfloat16 MFMA path (many signals, one dictionary) with the FP64
oracle, through the C-ABI.  The instance is the bfloat16-rounded dictionary with FP32
observations; the oracle solves exactly that instance in FP64."""
import numpy as np
import pytest

import oracle
from paper_1412_4080_amd import datagen
from tests._util import (GAP_DELTA_BATCHED, dev_matrix, lasso_margins_ref, rel_err,
                         stop_iteration_bracket)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def _batch(N, K, nsig, seed, ratios=None):
    D = datagen.gaussian_dictionary(N, K, seed)
    Dbf = datagen.to_storage(D, "bf16")
    ys = [datagen.to_storage(datagen.lasso_signal(D, seed * 100 + j)[0], "f32") for j in range(nsig)]
    if ratios is None:
        ratios = datagen.lambda_ratios(nsig, 0.1, 0.9, datagen.LAMBDA_SEED0 + seed)
    return D, Dbf, ys, np.asarray(ratios, dtype=np.float64)


def _dev_Y(ys):
    import torch
    Y = np.stack([np.asarray(y, dtype=np.float32) for y in ys])  # B x N row-major
    return torch.from_numpy(Y).cuda().T  # N x B column-major


def _check_mask(mask, ref, Dbf, y, ratio, test, info, hist):
    """Masks may differ only on atoms whose margin is within the rounding slack (plus the
    1e-6 band) of the oracle's final screening threshold."""
    if test == "none":
        assert not mask.any()
        return
    m = lasso_margins_ref(Dbf, y, ref.lam, test)
    diff = np.flatnonzero(mask != ref.screened)
    if diff.size == 0:
        return
    r_prev = min([h["r"] for h in hist[:-1]], default=np.inf)
    r_all = min([h["r"] for h in hist], default=np.inf)
    tol = 1e-6 + abs(info["radius"] - r_all) + info["radius_slack"]
    bad = diff[np.abs(m[diff] - r_prev) > tol]
    assert bad.size == 0, (bad[:5], m[bad[:5]], r_prev, tol)


@pytest.mark.parametrize("rule,test", [("fista", "dst3"), ("ista", "safe"), ("fista", "none"),
                                       ("ista", "dst3"), ("fista", "dome")])
def test_batched_fixed_iterations(B, rule, test):
    T = 30
    D, Dbf, ys, ratios = _batch(320, 1500, 12, 3)
    ratios = np.linspace(0.15, 0.85, 12)
    L = oracle.spectral_norm_sq(Dbf)
    X, infos, mask = B.solve(dev_matrix(D, "bf16"), _dev_Y(ys), ratios, rule=rule, test=test,
                             step_L=L, gap_tol=0.0, max_iter=T, screened=True)
    X = X.cpu().numpy().astype(np.float64)
    mask = mask.cpu().numpy().astype(bool)
    for j, (y, r) in enumerate(zip(ys, ratios)):
        ref = oracle.solve_lasso(Dbf, y, lam_ratio=r, rule=rule, test=test, L=L, max_iter=T,
                                 gap_tol=0.0, record=True)
        info = infos[j]
        assert info["status"] == 0 and info["iters"] == ref.iters == T
        assert info["lambda_max"] == pytest.approx(ref.lam_max, rel=1e-12)
        assert rel_err(X[:, j], ref.x) <= 1e-5, (j, rel_err(X[:, j], ref.x))
        assert abs(info["primal"] - ref.primal_p) <= 1e-6 * ref.primal_p, (j, info["primal"], ref.primal_p)
        assert abs(info["gap"] - ref.gap) <= 1e-6 * ref.primal_p, (j, info["gap"], ref.gap)
        _check_mask(mask[:, j], ref, Dbf, y, r, test, info, ref.history)
        # the screened atoms carry no weight
        assert not X[mask[:, j], j].any()


def test_batched_solve_to_tolerance_is_certified(B):
    D, Dbf, ys, ratios = _batch(400, 2000, 20, 5)
    L = oracle.spectral_norm_sq(Dbf)
    X, infos, mask = B.solve(dev_matrix(D, "bf16"), _dev_Y(ys), ratios, rule="fista",
                             test="dst3", step_L=L, gap_tol=1e-6, max_iter=20000, screened=True)
    X = X.cpu().numpy().astype(np.float64)
    mask = mask.cpu().numpy().astype(bool)
    for j, (y, r) in enumerate(zip(ys, ratios)):
        info = infos[j]
        yy = float(y @ y)
        assert info["status"] == 0 and info["gap"] <= 1e-6 * yy, (j, info)
        # the certificate holds against an independent high-accuracy optimum
        star = oracle.solve_lasso(Dbf, y, lam_ratio=r, rule="fista", test="none", L=L,
                                  max_iter=200000, gap_tol=1e-13)
        assert star.primal <= info["primal"] + 1e-12
        assert info["primal"] - star.primal <= info["gap"] + 1e-9
        # the returned x_t is no worse than the certified point
        res = Dbf @ X[:, j] - y
        px = 0.5 * float(res @ res) + info["lambda_"] * float(np.abs(X[:, j]).sum())
        assert px - star.primal <= info["gap"] + 1e-7
        # safety: every screened atom is certified inactive at the optimum
        cert, gstar = oracle.certified_inactive_lasso(Dbf, y, star.lam, star.x)
        assert gstar < 1e-11
        assert np.all(cert[mask[:, j]]), np.flatnonzero(mask[:, j] & ~cert)[:10]
        assert not star.x[mask[:, j]].any()
        assert not X[mask[:, j], j].any()
        # the MFMA run stops where the FP64 run's gap reaches tolerance (within the bracket
        # of its oscillating gap)
        t_lo, t_hi = stop_iteration_bracket(Dbf, y, info["lambda_"], L, 1e-6 * yy,
                                            delta=GAP_DELTA_BATCHED)
        assert t_lo <= info["iters"] <= t_hi, (j, info["iters"], t_lo, t_hi)


def test_batched_edge_cases(B):
    """Ragged N and K, trivial penalties (ratio >= 1), a zero observation and a signal
    solved next to them."""
    import torch
    N, K = 77, 203
    D = datagen.gaussian_dictionary(N, K, 11)
    Dbf = datagen.to_storage(D, "bf16")
    y1 = datagen.to_storage(datagen.lasso_signal(D, 11, p=0.05)[0], "f32")
    ys = [y1, y1, np.zeros(N), y1, y1]
    ratios = [1.0, 1.5, 0.5, 0.3, 0.6]
    L = oracle.spectral_norm_sq(Dbf)
    X, infos, mask = B.solve(dev_matrix(D, "bf16"), _dev_Y(ys), ratios, step_L=L, gap_tol=1e-6,
                             max_iter=20000, screened=True)
    X = X.cpu().numpy()
    mask = mask.cpu().numpy().astype(bool)
    for j in (0, 1, 2):
        assert infos[j]["status"] == 0 and infos[j]["iters"] == 0
        assert not X[:, j].any() and mask[:, j].all()
    for j in (3, 4):
        ref = oracle.solve_lasso(Dbf, ys[j], lam_ratio=ratios[j], rule="fista", test="dst3", L=L,
                                 max_iter=20000, gap_tol=1e-6)
        assert infos[j]["status"] == 0
        assert abs(infos[j]["primal"] - ref.primal_p) <= 2e-6 * float(ys[j] @ ys[j])
    # non-finite observation: rejected with DS_EINVAL
    bad = [y1.copy(), y1]
    bad[0][3] = np.nan
    with pytest.raises(B.DsError):
        B.solve(dev_matrix(D, "bf16"), _dev_Y(bad), [0.5, 0.5], step_L=L)
    torch.cuda.synchronize()


def test_batched_deterministic_and_independent_of_order(B):
    D, Dbf, ys, ratios = _batch(256, 1024, 10, 7)
    L = oracle.spectral_norm_sq(Dbf)
    Dd = dev_matrix(D, "bf16")
    X1, i1 = B.solve(Dd, _dev_Y(ys), ratios, step_L=L, gap_tol=1e-6)
    X2, i2 = B.solve(Dd, _dev_Y(ys), ratios, step_L=L, gap_tol=1e-6)
    assert np.array_equal(X1.cpu().numpy(), X2.cpu().numpy())
    assert [a["iters"] for a in i1] == [b["iters"] for b in i2]
    # the same signals in reverse order: each result is bit-identical
    X3, i3 = B.solve(Dd, _dev_Y(ys[::-1]), ratios[::-1], step_L=L, gap_tol=1e-6)
    assert np.array_equal(X1.cpu().numpy(), X3.cpu().numpy()[:, ::-1])
    assert [a["iters"] for a in i1] == [b["iters"] for b in i3[::-1]]


def test_batched_full_size_sampled(B):
    """The benchmarked configuration (2000 x 10000 bfloat16, 256 signals, lambda ratios
    uniform in [0.1, 0.9]); three signals checked against the oracle."""
    N, K, nsig = 2000, 10000, 256
    D = datagen.gaussian_dictionary(N, K, datagen.DICT_SEED)
    Dbf = datagen.to_storage(D, "bf16")
    ys = [datagen.to_storage(datagen.lasso_signal(D, j)[0], "f32") for j in range(nsig)]
    ratios = datagen.lambda_ratios(nsig, 0.1, 0.9, datagen.LAMBDA_SEED0)
    Dd = dev_matrix(D, "bf16")
    L = B.spectral_norm_sq(Dd, 300)
    X, infos, mask = B.solve(Dd, _dev_Y(ys), ratios, step_L=L, gap_tol=1e-6, max_iter=20000,
                             screened=True)
    assert all(i["status"] == 0 for i in infos)
    assert all(i["gap"] <= 1e-6 * float(y @ y) for i, y in zip(infos, ys))
    X = X.cpu().numpy().astype(np.float64)
    mask = mask.cpu().numpy().astype(bool)
    order = np.argsort(ratios)
    for j in (order[0], order[nsig // 2], order[-1]):
        y, r, info = ys[j], ratios[j], infos[j]
        ref = oracle.solve_lasso(Dbf, y, lam_ratio=r, rule="fista", test="dst3", L=L,
                                 max_iter=20000, gap_tol=1e-6)
        yy = float(y @ y)
        assert abs(info["primal"] - ref.primal_p) <= info["gap"] + ref.gap + 1e-9 * yy
        cert, _ = oracle.certified_inactive_lasso(Dbf, y, ref.lam, ref.x)
        assert np.all(cert[mask[:, j]])
        assert not X[mask[:, j], j].any()


def test_batched_static_screening(B):
    T = 30
    D, Dbf, ys, _ = _batch(320, 1500, 8, 4)
    ratios = np.linspace(0.3, 0.9, 8)
    L = oracle.spectral_norm_sq(Dbf)
    X, infos, mask = B.solve(dev_matrix(D, "bf16"), _dev_Y(ys), ratios, test="dst3", step_L=L,
                             gap_tol=0.0, max_iter=T, screened=True, screening="static")
    X = X.cpu().numpy().astype(np.float64)
    mask = mask.cpu().numpy().astype(bool)
    for j, (y, r) in enumerate(zip(ys, ratios)):
        ref = oracle.solve_lasso(Dbf, y, lam_ratio=r, test="dst3", L=L, max_iter=T, gap_tol=0.0,
                                 record=True, screening="static")
        assert rel_err(X[:, j], ref.x) <= 1e-5, (j, rel_err(X[:, j], ref.x))
        assert abs(infos[j]["gap"] - ref.gap) <= 1e-6 * ref.primal_p
        m = lasso_margins_ref(Dbf, y, ref.lam, "dst3")
        diff = np.flatnonzero(mask[:, j] != ref.screened)
        tol = 1e-6 + infos[j]["radius_slack"] + 1e-9
        assert np.all(np.abs(m[diff] - ref.history[0]["r"]) <= tol), (j, diff[:5])
        assert not X[mask[:, j], j].any()


@pytest.mark.parametrize("rule,test,N,K", [("fista", "dst3", 320, 1500), ("ista", "safe", 320, 1500),
                                           ("fista", "dst3", 40, 300)])
def test_refilled_slots_give_the_same_results(B, rule, test, N, K):
    """Continuous batching: with fewer resident slots than signals, finished signals hand
    their slot to waiting ones.  Each signal's arithmetic does not depend on its slot or on
    the other residents, so the results equal the all-resident solve bit for bit (also with
    N below 64, where the set-up products' row groups are shortest)."""
    D, Dbf, ys, ratios = _batch(N, K, 100, 9)
    Dd, Y = dev_matrix(D, "bf16"), _dev_Y(ys)
    L = oracle.spectral_norm_sq(Dbf)
    X0, i0, m0 = B.solve(Dd, Y, ratios, rule=rule, test=test, step_L=L, gap_tol=1e-6,
                         max_iter=20000, screened=True)
    X0, m0 = X0.cpu().numpy(), m0.cpu().numpy()
    assert all(i["status"] == 0 for i in i0)
    for slots in (64, 17, 1):
        X, infos, mask = B.solve(Dd, Y, ratios, rule=rule, test=test, step_L=L, gap_tol=1e-6,
                                 max_iter=20000, screened=True, batch_slots=slots)
        assert np.array_equal(X.cpu().numpy(), X0), slots
        assert np.array_equal(mask.cpu().numpy(), m0), slots
        assert [i["iters"] for i in infos] == [i["iters"] for i in i0], slots
        assert [i["gap"] for i in infos] == [i["gap"] for i in i0], slots
        assert [i["nnz"] for i in infos] == [i["nnz"] for i in i0], slots


def test_more_signals_than_slots_by_default(B):
    """600 signals: 512 resident (the default), the rest refilled; the results equal a solve
    with every signal resident, and a few are certified against the oracle."""
    D, Dbf, ys, ratios = _batch(200, 900, 600, 10)
    Dd, Y = dev_matrix(D, "bf16"), _dev_Y(ys)
    L = oracle.spectral_norm_sq(Dbf)
    X, infos = B.solve(Dd, Y, ratios, step_L=L, gap_tol=1e-6, max_iter=20000)
    Xa, ia = B.solve(Dd, Y, ratios, step_L=L, gap_tol=1e-6, max_iter=20000, batch_slots=600)
    assert np.array_equal(X.cpu().numpy(), Xa.cpu().numpy())
    assert [i["iters"] for i in infos] == [i["iters"] for i in ia]
    X = X.cpu().numpy().astype(np.float64)
    for j in (0, 300, 599):
        y = ys[j]
        assert infos[j]["status"] == 0 and infos[j]["gap"] <= 1e-6 * float(y @ y)
        star = oracle.solve_lasso(Dbf, y, lam=infos[j]["lambda_"], rule="fista", test="none",
                                  L=L, max_iter=200000, gap_tol=1e-13)
        p = oracle.primal_objective(Dbf, y, X[:, j], infos[j]["lambda_"], float(np.abs(X[:, j]).sum()))
        assert p - star.primal <= infos[j]["gap"] + 1e-9


def _correlated_case(N, K, seed, nsig, corr=0.8):
    """Unit atoms sharing a common direction (where the dome's cut removes most), rounded to
    bfloat16, and unit observations from five atoms each."""
    rng = np.random.default_rng(seed)
    D = corr * rng.standard_normal((N, 1)) + rng.standard_normal((N, K))
    D /= np.linalg.norm(D, axis=0)
    Dbf = datagen.to_storage(D, "bf16")
    ys = []
    for j in range(nsig):
        y = Dbf[:, rng.choice(K, 5, replace=False)] @ rng.standard_normal(5) + 0.1 * rng.standard_normal(N)
        ys.append(datagen.to_storage(y / np.linalg.norm(y), "f32"))
    return D, Dbf, ys


def test_batched_dome_is_certified_and_screens_at_least_dst3(B):
    """The dynamic Dome test on the batched path (correlated atoms): every signal reaches the
    tolerance with its screened atoms certified inactive at the FP64 optimum, and ends with
    no more active atoms than the same batch under DST3."""
    D, Dbf, ys = _correlated_case(300, 1500, 43, 12)
    ratios = np.linspace(0.3, 0.9, 12)
    L = oracle.spectral_norm_sq(Dbf)
    Dd, Y = dev_matrix(D, "bf16"), _dev_Y(ys)
    kw = dict(rule="fista", step_L=L, gap_tol=1e-6, max_iter=20000, screened=True)
    X, infos, mask = B.solve(Dd, Y, ratios, test="dome", **kw)
    _, infos3, mask3 = B.solve(Dd, Y, ratios, test="dst3", **kw)
    X = X.cpu().numpy().astype(np.float64)
    mask = mask.cpu().numpy().astype(bool)
    mask3 = mask3.cpu().numpy().astype(bool)
    assert mask.sum() >= mask3.sum() > 0
    for j, (y, r) in enumerate(zip(ys, ratios)):
        info = infos[j]
        yy = float(y @ y)
        assert info["status"] == 0 and info["gap"] <= 1e-6 * yy, (j, info)
        star = oracle.solve_lasso(Dbf, y, lam=info["lambda_"], rule="fista", test="none", L=L,
                                  max_iter=200000, gap_tol=1e-13)
        assert info["primal"] - star.primal <= info["gap"] + 1e-9
        cert, gstar = oracle.certified_inactive_lasso(Dbf, y, star.lam, star.x)
        assert gstar < 1e-11
        assert np.all(cert[mask[:, j]]), np.flatnonzero(mask[:, j] & ~cert)[:10]
        assert not X[mask[:, j], j].any()
