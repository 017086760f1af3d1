"""SpaRSA (the Table 1 row: ISTA with the Barzilai-Borwein step and its acceptance test) on
the single-signal path: parity with the FP64 oracle's rule (iterations, screening trace,
final L and iterate), solves to the gap tolerance against the oracle, groups, the served
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


def _case(N, K, seed, p=0.05):
    D = datagen.gaussian_dictionary(N, K, seed)
    rng = np.random.default_rng(seed + 100)
    x0 = datagen.bernoulli_gaussian_code(K, p, rng)
    return D, datagen.observation(D, x0, rng, snr_db=20.0, normalize=True)


def _fp64_follows(B, D, y, ratio, test, memory, gp=None):
    T = 3000
    kw = dict(lam_ratio=ratio, rule="sparsa", L=0.05, max_iter=T, gap_tol=1e-12, record=True,
              bb_memory=memory)
    if gp is None:
        ref = oracle.solve_lasso(D, y, test=test, **kw)
    else:
        ref = oracle.solve_group_lasso(D, y, gp, test={"safe": "gsafe", "dst3": "dgst3"}.get(test, test),
                                       **kw)
    assert ref.converged and sum(not h["accepted"] for h in ref.history) >= 2
    x, info, _, tr = B.solve_one(dev_matrix(D, "f64"), dev_vector(y, "f64"), ratio, group_ptr=gp,
                                 rule="sparsa", test=test, step_L=0.05, gap_tol=1e-12,
                                 max_iter=T, bb_memory=memory)
    assert info["status"] == 0
    assert info["iters"] == ref.iters
    assert [t["n_active"] for t in tr] == [h["n_active"] for h in ref.history]
    # the last L is the Barzilai-Borwein quotient of a step close to the rounding level of
    # x (gap 1e-12), so rounding of the iterates shows in its leading digits only as ~1e-6
    assert info["L"] == pytest.approx(ref.L, rel=1e-4)
    assert rel_err(x.cpu().numpy(), ref.x) <= 1e-9
    return ref


@pytest.mark.parametrize("memory,test", [(0, "safe"), (0, "dst3"), (3, "dst3"), (5, "none")])
def test_fp64_small_workload_follows_the_oracle(B, memory, test):
    """FP64, from a small L_0 (the first steps are rejected) to gap 1e-12: the same number
    of iterations, the same active sets per iteration, the same final L and iterate."""
    c = datagen.lasso_small_fp64()
    _fp64_follows(B, c["D"], c["y"], 0.5, test, memory)


@pytest.mark.parametrize("test", ["none", "dst3"])
def test_fp64_nonmonotone_memory_follows_the_oracle(B, test):
    """A case where memory 4 accepts steps that raise the objective (the memory is used)."""
    D, y = _case(60, 200, 94)
    ref = _fp64_follows(B, D, y, 0.25, test, 4)
    pts = [h["primal_p"] for h, prev in zip(ref.history, [None] + ref.history[:-1])
           if prev is None or prev["accepted"]]
    assert np.max(np.diff(pts)) > 1e-9


@pytest.mark.parametrize("memory", [0, 4])
def test_fp64_groups_follow_the_oracle(B, memory):
    c = datagen.lasso_small_fp64()
    gp = datagen.contiguous_groups(500, 10)
    y, _ = datagen.group_signal(c["D"], gp, 2)
    _fp64_follows(B, c["D"], y, 0.5, "dst3", memory, gp=gp)


@pytest.mark.parametrize("memory", [0, 5])
@pytest.mark.parametrize("ratio", [0.3, 0.7])
def test_fp32_to_gap_matches_the_oracle(B, memory, ratio):
    """FP32 to gap 1e-6 from the default L_0: the certified objective agrees with the
    oracle's run of the same rule and the solution is certified against the optimum."""
    D = datagen.gaussian_dictionary(800, 3000, 7)
    y, _ = datagen.lasso_signal(D, 7)
    Di, yi = instance(D, y, "f32")
    tol = 1e-6
    ref = oracle.solve_lasso(Di, yi, lam_ratio=ratio, rule="sparsa", test="dst3", max_iter=20000,
                             gap_tol=tol, bb_memory=memory)
    x, info, _, _ = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), ratio, rule="sparsa",
                                test="dst3", gap_tol=tol, max_iter=20000, bb_memory=memory,
                                trace=False, screened=False)
    yy = float(yi @ yi)
    assert info["status"] == 0 and ref.converged
    assert abs(info["primal"] - ref.primal_p) <= 2 * tol * yy
    xs = x.cpu().numpy().astype(np.float64)
    star = oracle.solve_lasso(Di, yi, lam=ref.lam, rule="fista", test="none", max_iter=200000,
                              gap_tol=1e-13)
    assert oracle.primal_objective(Di, yi, xs, ref.lam, float(np.abs(xs).sum())) - star.primal \
        <= tol * yy * 1.01
    assert info["iters"] <= 2 * ref.iters + 10


@pytest.mark.parametrize("memory", [0, 4])
def test_group_fp32_to_gap_matches_the_oracle(B, memory):
    D = datagen.gaussian_dictionary(400, 1500, 11)
    gp = datagen.contiguous_groups(1500, 10)
    y, _ = datagen.group_signal(D, gp, 3)
    Di, yi = instance(D, y, "f32")
    tol = 1e-6
    ref = oracle.solve_group_lasso(Di, yi, gp, lam_ratio=0.5, rule="sparsa", test="dgst3",
                                   max_iter=20000, gap_tol=tol, bb_memory=memory)
    x, info, _, _ = B.solve_one(dev_matrix(D, "f32"), dev_vector(yi, "f32"), 0.5, group_ptr=gp,
                                rule="sparsa", test="dst3", gap_tol=tol, max_iter=20000,
                                bb_memory=memory, trace=False, screened=False)
    yy = float(yi @ yi)
    assert info["status"] == 0 and ref.converged
    assert abs(info["primal"] - ref.primal_p) <= 2 * tol * yy
    assert info["iters"] <= 2 * ref.iters + 10


def test_served_request_equals_the_direct_solve(B):
    import time
    import torch
    D = datagen.gaussian_dictionary(500, 2000, 13)
    y, _ = datagen.lasso_signal(D, 13)
    Di, yi = instance(D, y, "f32")
    Dd = dev_matrix(D, "f32")
    x1, i1, _, _ = B.solve_one(Dd, dev_vector(yi, "f32"), 0.5, rule="sparsa", test="dst3",
                               gap_tol=1e-6, max_iter=20000, bb_memory=3, trace=False,
                               screened=False)
    S = B.Server(max_slots=2)
    did = S.add_dict(Dd, store="f32")
    torch.cuda.synchronize()
    rid = S.submit(did, yi.astype(np.float32), 0.5, rule="sparsa", test="dst3", gap_tol=1e-6,
                   max_iter=20000, bb_memory=3)
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


def test_batched_bf16_path_refuses_sparsa(B):
    import torch
    D = datagen.gaussian_dictionary(256, 1024, 15)
    y, _ = datagen.lasso_signal(D, 15)
    Dd = dev_matrix(D, "bf16")
    Y = torch.from_numpy(np.stack([y, y]).astype(np.float32)).cuda().T
    with pytest.raises(B.DsError) as e:
        B.solve(Dd, Y, [0.5, 0.6], rule="sparsa")
    assert e.value.status == B.DS_EINVAL
