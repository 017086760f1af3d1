"""ds_solve_one_noalloc (the allocation-free single-signal entry point) against ds_solve_one,
through the C-ABI: the same kernels on the library's fixed scratch array must give the same
results bit for bit, on consecutive calls that reuse the array (the second with a smaller
problem, so stale contents of the first are present), and problems that do not fit are
refused before any device work."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1412_4080_amd import datagen
from tests._util import dev_matrix, dev_vector, instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def _case(N, K, seed, dtype="f32", groups=None):
    D = datagen.gaussian_dictionary(N, K, seed)
    if groups is None:
        y, _ = datagen.lasso_signal(D, seed)
    else:
        y, _ = datagen.group_signal(D, groups, seed)
    Di, yi = instance(D, y, dtype)
    return dev_matrix(D, dtype), dev_vector(yi, dtype), oracle.spectral_norm_sq(Di)


def _same(B, Dd, yd, L, ratio, **kw):
    x_ref, i_ref, s_ref, _ = B.solve_one(Dd, yd, ratio, step_L=L, trace=False, **kw)
    x, info, scr = B.solve_one_noalloc(Dd, yd, ratio, step_L=L, **kw)
    assert info["status"] == i_ref["status"]
    assert info["iters"] == i_ref["iters"] and info["gap"] == i_ref["gap"]
    assert info["primal"] == i_ref["primal"] and info["n_active"] == i_ref["n_active"]
    assert np.array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
    assert np.array_equal(scr.cpu().numpy(), s_ref.cpu().numpy())
    return info


def test_noalloc_equals_solve_one_on_consecutive_calls(B):
    # a large call, then a smaller one on the same scratch array
    Dd, yd, L = _case(2000, 10000, 0)
    info = _same(B, Dd, yd, L, 0.5, rule="fista", test="dst3", gap_tol=1e-6, max_iter=20000)
    assert info["status"] == 0
    Dd2, yd2, L2 = _case(300, 1200, 3)
    _same(B, Dd2, yd2, L2, 0.3, rule="fista", test="dst3", gap_tol=1e-6, max_iter=20000)
    # and the large one again (the array now holds the small call's contents)
    _same(B, Dd, yd, L, 0.8, rule="ista", test="safe", gap_tol=1e-6, max_iter=20000)


def test_noalloc_groups_fp64_and_other_rules(B):
    gp = datagen.contiguous_groups(1500, 10)
    Dd, yd, L = _case(400, 1500, 5, groups=gp)
    _same(B, Dd, yd, L, 0.4, group_ptr=gp, rule="fista", test="dgst3", gap_tol=1e-6,
          max_iter=20000)
    Dd, yd, L = _case(100, 500, 7, dtype="f64")
    _same(B, Dd, yd, L, 0.5, rule="cp", test="dst3", gap_tol=1e-8, max_iter=20000)
    _same(B, Dd, yd, 0.0, 0.5, rule="sparsa", test="safe", gap_tol=1e-8, max_iter=20000)
    _same(B, Dd, yd, 0.0, 0.5, rule="fista", test="dst3", step="backtracking", gap_tol=1e-8,
          max_iter=20000)


def test_noalloc_refusals(B):
    import torch
    Dd, yd, L = _case(200, 800, 9)
    # a constant step needs the step constant
    with pytest.raises(B.DsError) as e:
        B.solve_one_noalloc(Dd, yd, 0.5, step_L=0.0)
    assert e.value.status == B.DS_EINVAL and "step_L" in str(e.value)
    # a problem whose workspace exceeds the array is refused on the host, before any launch
    # (the dictionary pointer is never read)
    prm = B.make_params(step_L=L)
    x = torch.empty(16, dtype=torch.float32, device="cuda")
    info = B.Info()
    for N, K, why in ((100_000, 200_000, "scratch"), (200, 4_000_000, "too large")):
        prob = B.Problem(B.DTYPES["f32"], N, K, N, C.c_void_p(Dd.data_ptr()), 0, None, None)
        st = B._lib.ds_solve_one_noalloc(C.byref(prob), C.c_void_p(yd.data_ptr()), 0.5,
                                         C.byref(prm), C.c_void_p(x.data_ptr()), None,
                                         C.byref(info), B._stream_ptr(None))
        assert st == B.DS_EINVAL and why in B.last_error()
    # the entry point still works afterwards
    _same(B, Dd, yd, L, 0.5, rule="fista", test="dst3", gap_tol=1e-6, max_iter=20000)
