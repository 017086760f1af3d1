"""Shared helpers of the GPU tests: device placement and parity comparisons."""
import numpy as np

import oracle
from paper_1412_4080_amd import datagen


def dev_matrix(D: np.ndarray, dtype: str):
    """Column-major device tensor holding the stored values of D (f64 / f32 / bf16)."""
    import torch
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    src = datagen.to_storage(D, dtype)
    t = torch.from_numpy(np.ascontiguousarray(src.T)).to(device="cuda", dtype=tdt)
    return t.T


def dev_vector(y: np.ndarray, dtype: str):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(y)).to(device="cuda", dtype=tdt)


def instance(D, y, dtype):
    """The problem the stored values define, in float64 (what the oracle solves)."""
    return datagen.to_storage(D, dtype), datagen.to_storage(y, "f64" if dtype == "f64" else "f32")


def rel_err(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-30)
    return float(np.max(np.abs(np.asarray(a, dtype=np.float64) - b))) / scale


def lasso_margins_ref(D, y, lam, test):
    lam_max, i_star = oracle.lambda_max_lasso(D, y)
    if test == "dome":
        return oracle.dome_margins(D, y, lam, i_star)
    c, _ = oracle.lasso_center(D, y, lam, test, lam_max, i_star)
    return oracle.lasso_margins(D, c, test)


def group_margins_ref(D, y, lam, test, gp, w):
    groups = [np.arange(gp[k], gp[k + 1]) for k in range(gp.size - 1)]
    lam_max, g_star = oracle.lambda_max_group(D, y, groups, w)
    c, _ = oracle.group_center(D, y, lam, test, groups, w, lam_max, g_star)
    return oracle.group_margins(D, c, test, groups, w, oracle.group_spectral_norms(D, groups))


def screened_sets_agree(gpu_mask, ref_mask, margins_units, r_ref, r_gpu, slack, unit_of_atom=None,
                        band=1e-6):
    """GPU and oracle screened sets may differ only on units whose margin lies within the
    band of the screening threshold."""
    diff = np.flatnonzero(gpu_mask != ref_mask)
    if diff.size == 0:
        return True
    units = diff if unit_of_atom is None else np.unique(unit_of_atom[diff])
    tol = band + abs(r_gpu - r_ref) + slack
    return bool(np.all(np.abs(margins_units[units] - r_ref) <= tol))


# Bound on the difference between the device's gap certificate and the FP64 oracle's at the
# same iteration, near the stop (where either is below 10 tol), as a fraction of the
# tolerance.  The evaluation itself differs by ~1e-8 (FP32 theta, FP64 reductions); the
# rest is the drift of the FP32 iterates from the FP64 ones (a few 1e-7 relative), to which
# the gap is sensitive to first order through the dual point v = mu (D p - y).  Measured:
# at most 0.16 tol on the 2000 x 10000 solves and 0.26 tol on the 400 x 2000 solve at
# lambda / lambda_* = 0.1.  Single-signal path: 0.3, asserted along every traced solve that
# uses the bracket.  Batched path: 0.3 as well (FP32 matrix-core correlations; no
# per-iteration trace to check it against).
GAP_DELTA_SINGLE = 0.3
GAP_DELTA_BATCHED = 0.3


def stop_iteration_bracket(D, y, lam, L, tol_abs, rule="fista", test="dst3",
                           delta=GAP_DELTA_SINGLE, group_ptr=None):
    """The stopping iterations allowed by a device gap within delta * tol of the oracle's.

    The device stops at the first iteration T whose gap is <= tol.  If its gap differs from
    the oracle's by at most delta * tol, the oracle's gap at T is <= (1 + delta) tol, and at
    every earlier iteration it is > (1 - delta) tol.  So T lies between the oracle's first
    iteration with gap <= (1 + delta) tol and its first with gap <= (1 - delta) tol."""
    lo, hi = 1.0 + delta, 1.0 - delta
    if group_ptr is None:
        ref = oracle.solve_lasso(D, y, lam=lam, rule=rule, test=test, L=L, max_iter=50000,
                                 gap_tol=hi * tol_abs / float(y @ y), record=True)
    else:
        ref = oracle.solve_group_lasso(D, y, group_ptr, None, lam=lam, rule=rule, test=test, L=L,
                                       max_iter=50000, gap_tol=hi * tol_abs / float(y @ y),
                                       record=True)
    gaps = [h["gap"] for h in ref.history]
    t_lo = next(k + 1 for k, g in enumerate(gaps) if g <= lo * tol_abs)
    t_hi = next(k + 1 for k, g in enumerate(gaps) if g <= hi * tol_abs)
    return t_lo, t_hi


def gap_difference_near_stop(trace, history, tol_abs):
    """Largest |device gap - oracle gap| at equal iterations where either is below 10 tol."""
    g1 = np.array([t["gap"] for t in trace])
    g2 = np.array([h["gap"] for h in history])
    n = min(g1.size, g2.size)
    g1, g2 = g1[:n], g2[:n]
    near = np.minimum(g1, g2) <= 10.0 * tol_abs
    return float(np.max(np.abs(g1 - g2)[near])) if near.any() else 0.0
