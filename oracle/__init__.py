"""Plain FP64 CPU oracle for dynamically screened ISTA/FISTA (Lasso and Group-Lasso).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP implementation.

Everything here follows "Dynamic Screening: Accelerating First-Order Algorithms
for the Lasso and Group-Lasso" (Bonnefoy, Emiya, Ralaivola, Gribonval,
arXiv:1412.4080).  Each function cites the section, equation, lemma, table or
algorithm it restates.  Computation is in float64 throughout; inputs that were
stored in a lower precision are widened exactly, so the oracle solves the
problem defined by the stored values.
"""
from .dynscreen import (  # noqa: F401
    OracleResult,
    lambda_max_lasso,
    lambda_max_group,
    soft_threshold,
    group_soft_threshold,
    dual_scaling,
    primal_objective,
    dual_objective,
    lasso_center,
    group_center,
    lasso_margins,
    group_margins,
    dome_max,
    dome_setup,
    dome_margins,
    group_spectral_norms,
    spectral_norm_sq,
    solve_lasso,
    solve_group_lasso,
    certified_inactive_lasso,
    certified_inactive_group,
    flops_dynamic,
    flops_none,
    flops_static,
)
from .brute import brute_force_lasso  # noqa: F401
