"""Every update rule with every screening test, dynamic and static, on FP32 and bfloat16
storage (single-signal path): each solve reaches the gap tolerance, its returned point is
certified against the FP64 optimum of the stored instance, and every screened atom is
provably inactive there."""
import numpy as np
import pytest

import oracle
from paper_1412_4080_amd import datagen
from tests._util import dev_matrix, dev_vector, instance

pytestmark = pytest.mark.gpu

RULES = ["ista", "fista", "sparsa", "cp"]
TESTS = ["none", "safe", "dst3", "dome"]


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


@pytest.fixture(scope="module", params=["f32", "bf16"])
def case(request):
    dtype = request.param
    D = datagen.gaussian_dictionary(300, 1200, 51)
    y, _ = datagen.lasso_signal(D, 51, p=0.03)
    Di, yi = instance(D, y, dtype)
    lam = 0.8 * oracle.lambda_max_lasso(Di, yi)[0]   # static tests screen too at this ratio
    star = oracle.solve_lasso(Di, yi, lam=lam, rule="fista", test="none", max_iter=200000,
                              gap_tol=1e-14)
    cert, g = oracle.certified_inactive_lasso(Di, yi, lam, star.x)
    assert g < 1e-12
    return dict(dtype=dtype, D=D, Di=Di, yi=yi, lam=lam, star=star, cert=cert)


@pytest.mark.parametrize("screening", ["dynamic", "static"])
@pytest.mark.parametrize("test", TESTS)
@pytest.mark.parametrize("rule", RULES)
def test_rule_test_dtype_grid(B, case, rule, test, screening):
    Di, yi, lam = case["Di"], case["yi"], case["lam"]
    vdt = "f32"          # bfloat16 dictionaries take FP32 signals
    x, info, scr, _ = B.solve_one(dev_matrix(case["D"], case["dtype"]), dev_vector(yi, vdt),
                                  lam, lambda_relative=False, rule=rule, test=test,
                                  screening=screening, gap_tol=1e-6, max_iter=50000,
                                  trace=False)
    yy = float(yi @ yi)
    assert info["status"] == 0, info
    xs = x.cpu().numpy().astype(np.float64)
    p_x = oracle.primal_objective(Di, yi, xs, lam, float(np.abs(xs).sum()))
    assert p_x - case["star"].primal <= 1.01e-6 * yy
    scr = scr.cpu().numpy().astype(bool)
    assert np.all(case["cert"][scr]), np.flatnonzero(scr & ~case["cert"])[:10]
    assert not xs[scr].any()
    if test == "none":
        assert not scr.any()
    else:
        assert scr.sum() > 0.8 * scr.size   # both modes screen most atoms at 0.8 lambda_*
