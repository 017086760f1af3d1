"""The benchmark's bookkeeping on the CPU: its flops model (the experiments section's
flops_N, flops_S, flops_D tables) equals the oracle's statement of it on recorded runs."""
import numpy as np

import bench
import oracle
from paper_1412_4080_amd import datagen


def test_bench_flops_model_equals_the_oracle():
    D = datagen.pnoise_dictionary(60, 300, 5)
    y = datagen.atom_like_observation(60, 3, "pnoise")
    for rule in ("ista", "fista"):
        for ratio in (0.3, 0.8):
            none = oracle.solve_lasso(D, y, lam_ratio=ratio, rule=rule, test="none", max_iter=200,
                                      gap_tol=0.0, obj_tol=1e-7, record=True)
            dyn = oracle.solve_lasso(D, y, lam_ratio=ratio, rule=rule, test="dst3", max_iter=200,
                                     gap_tol=0.0, obj_tol=1e-7, record=True)
            sta = oracle.solve_lasso(D, y, lam_ratio=ratio, rule=rule, test="dst3", max_iter=200,
                                     gap_tol=0.0, obj_tol=1e-7, record=True, screening="static")
            kept = sta.history[1]["n_active"] if len(sta.history) > 1 else 300
            assert bench.flops_none(none.history, 60, 300) == oracle.flops_none(none.history, 60, 300)
            assert bench.flops_dynamic(dyn.history, 60) == oracle.flops_dynamic(dyn.history, 60)
            assert bench.flops_static(sta.history, 60, 300, kept) == \
                oracle.flops_static(sta.history, 60, 300, kept)
    gp = datagen.contiguous_groups(300, 10)
    yg = datagen.group_signal(D, gp, 1, p=0.05)[0]
    r = oracle.solve_group_lasso(D, yg, gp, None, lam_ratio=0.5, rule="fista", test="dgst3",
                                 max_iter=200, gap_tol=0.0, obj_tol=1e-7, record=True)
    assert bench.flops_dynamic(r.history, 60, 30) == oracle.flops_dynamic(r.history, 60, 30)
    assert bench.flops_none(r.history, 60, 300, 30) == oracle.flops_none(r.history, 60, 300, 30)
    assert bench.flops_static(r.history, 60, 300, 120, 30) == \
        oracle.flops_static(r.history, 60, 300, 120, 30)


def test_quantiles_of_a_known_sample():
    q = bench._quantiles(np.arange(1, 102))
    assert q == {"median": 51.0, "p25": 26.0, "p75": 76.0}
