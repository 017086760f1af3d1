"""Seeded random sweep of the single-signal path: random sizes (ragged, down to N = K = 1),
padded leading dimensions, storage types, Lasso or random group partitions (sizes 1 to
128), every update rule, screening test and mode, and lambda / lambda_*.  Each solve to gap
1e-6 is checked against the FP64 optimum of the stored instance: its objective, and every
screened atom provably inactive there."""
import numpy as np
import pytest

import oracle
from paper_1412_4080_amd import datagen
from tests._util import dev_vector, instance

pytestmark = pytest.mark.gpu

CASES = 120


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def draw(i):
    """Case i: everything from one seeded generator."""
    rng = np.random.default_rng(9000 + i)
    N = int(rng.integers(1, 180))
    K = int(rng.integers(1, 700))
    group = bool(rng.integers(2)) and K >= 2
    gp = None
    if group:
        sizes = []
        while sum(sizes) < K:
            sizes.append(int(min(rng.integers(1, 129), K - sum(sizes))))
        gp = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return dict(
        N=N, K=K, ldd=N + int(rng.integers(0, 5)),
        dtype=["f64", "f32", "bf16"][int(rng.integers(3))],
        gp=gp,
        rule=["ista", "fista", "sparsa", "cp"][int(rng.integers(4))],
        test=(["none", "safe", "dst3"] if group else ["none", "safe", "dst3", "dome"])[
            int(rng.integers(3 if group else 4))],
        screening=["dynamic", "static"][int(rng.integers(2))],
        ratio=float(rng.uniform(0.05, 0.95)),
        seed=int(rng.integers(1 << 30)))


@pytest.mark.parametrize("i", range(CASES))
def test_random_case(B, i):
    import torch
    c = draw(i)
    N, K, gp = c["N"], c["K"], c["gp"]
    D = datagen.gaussian_dictionary(N, K, c["seed"])
    rng = np.random.default_rng(c["seed"] + 1)
    y = D @ (rng.standard_normal(K) * (rng.random(K) < 0.05)) + 0.1 * rng.standard_normal(N)
    if not np.any(y):
        y[0] = 1.0
    y /= np.linalg.norm(y)
    Di, yi = instance(D, y, c["dtype"])
    if gp is None:
        lam_max = oracle.lambda_max_lasso(Di, yi)[0]
    else:
        groups = [np.arange(gp[g], gp[g + 1]) for g in range(gp.size - 1)]
        lam_max = oracle.lambda_max_group(Di, yi, groups, np.sqrt(np.diff(gp).astype(float)))[0]
    lam = c["ratio"] * lam_max
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[c["dtype"]]
    buf = torch.zeros(K, c["ldd"], dtype=tdt)
    buf[:, :N] = torch.from_numpy(np.ascontiguousarray(Di.T))
    Dd = buf.to("cuda").T[:N, :]
    print(f"case {i}: {c['rule']} {c['test']} {c['screening']} {c['dtype']} N={N} K={K} "
          f"ldd={c['ldd']} groups={None if gp is None else gp.size - 1} ratio={c['ratio']:.3f}",
          flush=True)
    x, info, scr, _ = B.solve_one(Dd, dev_vector(yi, c["dtype"]), lam, lambda_relative=False,
                                  group_ptr=gp, rule=c["rule"], test=c["test"],
                                  screening=c["screening"], gap_tol=1e-6, max_iter=200000,
                                  trace=False)
    assert info["status"] == 0, info
    yy = float(yi @ yi)
    xs = x.cpu().numpy().astype(np.float64)
    scr = scr.cpu().numpy().astype(bool)
    if gp is None:
        star = oracle.solve_lasso(Di, yi, lam=lam, rule="fista", test="none", max_iter=500000,
                                  gap_tol=1e-12)
        cert, _ = oracle.certified_inactive_lasso(Di, yi, lam, star.x)
        p_x = oracle.primal_objective(Di, yi, xs, lam, float(np.abs(xs).sum()))
    else:
        star = oracle.solve_group_lasso(Di, yi, gp, lam=lam, rule="fista", test="none",
                                        max_iter=500000, gap_tol=1e-12)
        cert, _, _ = oracle.certified_inactive_group(Di, yi, lam, star.x, gp)
        w = np.sqrt(np.diff(gp).astype(float))
        om = float(sum(w[g] * np.linalg.norm(xs[gp[g]:gp[g + 1]]) for g in range(gp.size - 1)))
        p_x = oracle.primal_objective(Di, yi, xs, lam, om)
    assert star.converged
    assert p_x - star.primal <= 1.01e-6 * yy + 1e-12
    assert np.all(cert[scr]), np.flatnonzero(scr & ~cert)[:10]
    assert not star.x[scr].any()
    assert not xs[scr].any()
