"""Seeded random sweep of the batched bfloat16 path (many signals sharing one dictionary):
random sizes (ragged, tiles partly filled), signal counts, update rules, screening tests
and modes, and per-signal lambda / lambda_*; for the Group-Lasso also random contiguous
partitions (1 to 128 atoms per group) and weights.  In each case a sample of the signals is
checked against the FP64 optimum of the stored instance: the returned objective, and
every screened atom provably inactive."""
import numpy as np
import pytest

import oracle
from paper_1412_4080_amd import datagen

pytestmark = pytest.mark.gpu

CASES = 16
SAMPLE = 6


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def draw(i):
    rng = np.random.default_rng(7000 + i)
    return dict(N=int(rng.integers(8, 600)), K=int(rng.integers(8, 3000)),
                nsig=int(rng.integers(2, 300)),
                rule=["ista", "fista"][int(rng.integers(2))],
                test=["none", "safe", "dst3"][int(rng.integers(3))],
                screening=["dynamic", "static"][int(rng.integers(2))],
                seed=int(rng.integers(1 << 30)))


@pytest.mark.parametrize("i", range(CASES))
def test_random_batch(B, i):
    import torch
    c = draw(i)
    N, K, nsig = c["N"], c["K"], c["nsig"]
    D = datagen.gaussian_dictionary(N, K, c["seed"])
    Dbf = datagen.to_storage(D, "bf16")
    rng = np.random.default_rng(c["seed"] + 1)
    Y = np.empty((nsig, N))
    for b in range(nsig):
        y = Dbf @ (rng.standard_normal(K) * (rng.random(K) < 0.03)) + 0.1 * rng.standard_normal(N)
        Y[b] = y / np.linalg.norm(y)
    Y = Y.astype(np.float32)
    ratios = rng.uniform(0.1, 0.9, nsig)
    print(f"case {i}: {c['rule']} {c['test']} {c['screening']} N={N} K={K} B={nsig}", flush=True)
    Dd = torch.from_numpy(np.ascontiguousarray(Dbf.T)).to(device="cuda", dtype=torch.bfloat16).T
    X, infos, mask = B.solve(Dd, torch.from_numpy(Y).cuda().T, ratios, rule=c["rule"],
                             test=c["test"], screening=c["screening"], gap_tol=1e-6,
                             max_iter=100000, screened=True)
    X = X.cpu().numpy().astype(np.float64)
    mask = mask.cpu().numpy().astype(bool)
    for b in rng.choice(nsig, size=min(SAMPLE, nsig), replace=False):
        yb = Y[b].astype(np.float64)
        info = infos[b]
        assert info["status"] == 0, (b, info)
        lam = info["lambda_"]
        star = oracle.solve_lasso(Dbf, yb, lam=lam, rule="fista", test="none", max_iter=500000,
                                  gap_tol=1e-12)
        assert star.converged
        xb = X[:, b]
        p_x = oracle.primal_objective(Dbf, yb, xb, lam, float(np.abs(xb).sum()))
        assert p_x - star.primal <= 1.01e-6 * float(yb @ yb) + 1e-12, b
        cert, _ = oracle.certified_inactive_lasso(Dbf, yb, lam, star.x)
        scr = mask[:, b]
        assert np.all(cert[scr]), (b, np.flatnonzero(scr & ~cert)[:10])
        assert not star.x[scr].any()
        assert not xb[scr].any()


GCASES = 10
GSAMPLE = 4


def gdraw(i):
    rng = np.random.default_rng(9100 + i)
    K = int(rng.integers(8, 2500))
    sizes, k = [], 0
    gmax = int(rng.choice([4, 16, 64, 128]))
    while k < K:
        m = min(K - k, int(rng.integers(1, gmax + 1)))
        sizes.append(m)
        k += m
    return dict(N=int(rng.integers(8, 500)), K=K, gp=np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64),
                nsig=int(rng.integers(2, 150)), rule=["ista", "fista"][int(rng.integers(2))],
                test=["none", "safe", "dst3"][int(rng.integers(3))],
                screening=["dynamic", "static"][int(rng.integers(2))],
                weights=bool(rng.integers(2)), seed=int(rng.integers(1 << 30)))


@pytest.mark.parametrize("i", range(GCASES))
def test_random_group_batch(B, i):
    import torch
    c = gdraw(i)
    N, K, nsig, gp = c["N"], c["K"], c["nsig"], c["gp"]
    G = gp.size - 1
    D = datagen.gaussian_dictionary(N, K, c["seed"])
    Dbf = datagen.to_storage(D, "bf16")
    rng = np.random.default_rng(c["seed"] + 1)
    w = np.sqrt(np.diff(gp).astype(np.float64)) * (rng.uniform(0.7, 1.4, G) if c["weights"] else 1.0)
    Y = np.empty((nsig, N))
    for b in range(nsig):
        act = np.repeat(rng.random(G) < 0.05, np.diff(gp))
        y = Dbf @ (rng.standard_normal(K) * act) + 0.1 * rng.standard_normal(N)
        Y[b] = y / np.linalg.norm(y)
    Y = Y.astype(np.float32)
    ratios = rng.uniform(0.1, 0.9, nsig)
    print(f"group case {i}: {c['rule']} {c['test']} {c['screening']} N={N} K={K} G={G} "
          f"B={nsig} weights={c['weights']}", flush=True)
    Dd = torch.from_numpy(np.ascontiguousarray(Dbf.T)).to(device="cuda", dtype=torch.bfloat16).T
    X, infos, mask = B.solve(Dd, torch.from_numpy(Y).cuda().T, ratios, group_ptr=gp, weights=w,
                             rule=c["rule"], test=c["test"], screening=c["screening"],
                             gap_tol=1e-6, max_iter=100000, screened=True)
    X = X.cpu().numpy().astype(np.float64)
    mask = mask.cpu().numpy().astype(bool)
    for b in rng.choice(nsig, size=min(GSAMPLE, nsig), replace=False):
        yb = Y[b].astype(np.float64)
        info = infos[b]
        assert info["status"] == 0, (b, info)
        lam = info["lambda_"]
        star = oracle.solve_group_lasso(Dbf, yb, gp, w, lam=lam, rule="fista", test="none",
                                        max_iter=500000, gap_tol=1e-12)
        assert star.converged
        xb = X[:, b]
        om = sum(w[g] * np.linalg.norm(xb[gp[g]:gp[g + 1]]) for g in range(G))
        p_x = oracle.primal_objective(Dbf, yb, xb, lam, om)
        assert p_x - star.primal <= 1.01e-6 * float(yb @ yb) + 1e-12, b
        amask, _, _ = oracle.certified_inactive_group(Dbf, yb, lam, star.x, gp, w)
        scr = mask[:, b]
        assert np.all(amask[scr]), (b, np.flatnonzero(scr & ~amask)[:10])
        assert not star.x[scr].any()
        assert not xb[scr].any()
