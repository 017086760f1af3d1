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


def stop_iteration_bracket(D, y, lam, L, tol_abs, rule="fista", test="dst3", lo=1.3, hi=0.7):
    """First iterations at which the oracle's gap certificate falls below lo * tol and below
    hi * tol.  FISTA's gap oscillates near convergence, so a device run whose gap differs
    from the oracle's by a fraction of the tolerance can stop at a later dip; its stopping
    iteration must fall within this bracket."""
    ref = oracle.solve_lasso(D, y, lam=lam, rule=rule, test=test, L=L, max_iter=50000,
                             gap_tol=hi * tol_abs / float(y @ y), record=True)
    gaps = [h["gap"] for h in ref.history]
    t_lo = next(k + 1 for k, g in enumerate(gaps) if g <= lo * tol_abs)
    t_hi = next(k + 1 for k, g in enumerate(gaps) if g <= hi * tol_abs)
    return t_lo, t_hi
