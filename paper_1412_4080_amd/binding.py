"""ctypes binding of libdynscreen.so (C-ABI in include/dynscreen.h).

Argument marshalling only: every step of a solve runs in the library's HIP kernels.
PyTorch supplies device memory and the current stream; tensors are passed by pointer.
Importing this module raises ImportError when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
# DS_LIBRARY: another build of the same library (the sanitizer tests load one)
LIB_PATH = os.environ.get("DS_LIBRARY") or os.path.join(HERE, "libdynscreen.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1412_4080_amd.build` "
                      "(or __graft_entry__.build()) first")
_lib = C.CDLL(LIB_PATH)

# ------------------------------------------------------------------ enums / structs
DS_OK, DS_PENDING, DS_NOT_CONVERGED = 0, 1, 2
DS_EINVAL, DS_ENOMEM, DS_EDEVICE, DS_ENOTFOUND, DS_EBUSY = -1, -2, -3, -4, -5
DTYPES = {"f64": 0, "f32": 1, "bf16": 2}
RULES = {"ista": 0, "fista": 1, "sparsa": 2, "cp": 3}
TESTS = {"none": 0, "safe": 1, "dst3": 2, "gsafe": 1, "dgst3": 2, "dome": 3}
STATUS_NAMES = {0: "DS_OK", 1: "DS_PENDING", 2: "DS_NOT_CONVERGED", -1: "DS_EINVAL",
                -2: "DS_ENOMEM", -3: "DS_EDEVICE", -4: "DS_ENOTFOUND", -5: "DS_EBUSY"}
STEPS = {"constant": 0, "backtracking": 1}
STAT_CORR, STAT_RESID, STAT_SETUP, STAT_BATCH, STAT_BATCH_THETA, STAT_ITER, STAT_COUNT = 0, 1, 2, 3, 4, 5, 6


class Problem(C.Structure):
    _fields_ = [("dtype", C.c_int), ("N", C.c_int64), ("K", C.c_int64), ("ldd", C.c_int64),
                ("D", C.c_void_p), ("G", C.c_int64), ("group_ptr", C.POINTER(C.c_int64)),
                ("w", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("rule", C.c_int), ("test", C.c_int), ("lambda_mode", C.c_int),
                ("step_L", C.c_double), ("gap_tol", C.c_double), ("max_iter", C.c_int32),
                ("screening", C.c_int32), ("step_rule", C.c_int32), ("bt_eta", C.c_double),
                ("bb_memory", C.c_int32), ("bb_sigma", C.c_double), ("cp_tau", C.c_double),
                ("cp_sigma", C.c_double), ("cp_gamma", C.c_double), ("x0", C.c_void_p),
                ("obj_tol", C.c_double), ("batch_slots", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("n_active", C.c_int32),
                ("nnz", C.c_int32), ("lambda_", C.c_double), ("lambda_max", C.c_double),
                ("primal", C.c_double), ("dual", C.c_double), ("gap", C.c_double),
                ("radius", C.c_double), ("mu", C.c_double), ("L", C.c_double),
                ("radius_slack", C.c_double), ("queue_ms", C.c_double), ("run_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Trace(C.Structure):
    _fields_ = [("n_active", C.c_int32), ("n_units", C.c_int32), ("n_support", C.c_int32),
                ("nnz", C.c_int32), ("radius", C.c_double), ("gap", C.c_double)]


class ServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_slots", C.c_int32), ("hbm_budget_bytes", C.c_size_t),
                ("max_queue", C.c_int32), ("batch_slots", C.c_int32)]


class LaunchStat(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("n_atoms", C.c_int32), ("bytes", C.c_double),
                ("ms", C.c_double)]


class KernelStat(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double), ("ms_event", C.c_double)]


_P = C.POINTER
_sig = {
    "lasso_solve": (C.c_int, [_P(Problem), C.c_void_p, C.c_int64, C.c_int64, _P(C.c_double),
                              _P(Params), C.c_void_p, C.c_int64, _P(Info), C.c_void_p]),
    "glasso_solve": (C.c_int, [_P(Problem), C.c_void_p, C.c_int64, C.c_int64, _P(C.c_double),
                               _P(Params), C.c_void_p, C.c_int64, _P(Info), C.c_void_p]),
    "ds_solve_batch": (C.c_int, [_P(Problem), C.c_void_p, C.c_int64, C.c_int64, _P(C.c_double),
                                 _P(Params), C.c_void_p, C.c_int64, _P(Info), C.c_void_p,
                                 C.c_void_p]),
    "ds_solve_one": (C.c_int, [_P(Problem), C.c_void_p, C.c_double, _P(Params), C.c_void_p,
                               C.c_void_p, _P(Trace), C.c_int32, _P(Info), C.c_void_p]),
    "ds_solve_one_noalloc": (C.c_int, [_P(Problem), C.c_void_p, C.c_double, _P(Params),
                                       C.c_void_p, C.c_void_p, _P(Info), C.c_void_p]),
    "ds_lambda_max": (C.c_int, [_P(Problem), C.c_void_p, _P(C.c_double), _P(C.c_int64),
                                C.c_void_p]),
    "ds_spectral_norm_sq": (C.c_int, [_P(Problem), C.c_int32, _P(C.c_double), C.c_void_p]),
    "ds_server_create": (C.c_int, [_P(ServerConfig), _P(C.c_void_p)]),
    "ds_server_add_dict": (C.c_int, [C.c_void_p, _P(Problem), C.c_int, _P(C.c_int32)]),
    "ds_submit": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, _P(Params),
                            _P(C.c_uint64)]),
    "lasso_submit": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, _P(Params),
                               _P(C.c_uint64)]),
    "lasso_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, _P(Info)]),
    "ds_server_destroy": (C.c_int, [C.c_void_p]),
    "ds_stats_enable": (None, [C.c_int]),
    "ds_stats_reset": (None, []),
    "ds_stats_read": (C.c_int, [_P(KernelStat), C.c_int]),
    "ds_stats_launches": (C.c_int, [_P(LaunchStat), C.c_int]),
    "ds_batch_shape": (C.c_int, [_P(C.c_int), _P(C.c_int)]),
    "ds_last_error": (C.c_char_p, []),
    "ds_version": (C.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class DsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {last_error()}")


def last_error() -> str:
    return _lib.ds_last_error().decode()


def version() -> str:
    return _lib.ds_version().decode()


def _check(status: int, where: str) -> int:
    if status < 0:
        raise DsError(status, where)
    return status


# ------------------------------------------------------------------ tensor helpers
def _torch():
    import torch
    return torch


def _dtype_name(t) -> str:
    torch = _torch()
    return {torch.float64: "f64", torch.float32: "f32", torch.bfloat16: "bf16"}[t.dtype]


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class _Groups:
    ptr: object
    w: object
    G: int


def _groups(group_ptr, weights):
    if group_ptr is None:
        return _Groups(None, None, 0)
    import numpy as np
    gp = np.ascontiguousarray(np.asarray(group_ptr, dtype=np.int64))
    w = None if weights is None else np.ascontiguousarray(np.asarray(weights, dtype=np.float64))
    return _Groups(gp, w, gp.size - 1)


def make_problem(D, group_ptr=None, weights=None):
    """D: device tensor N x K in column-major layout (stride (1, ldd)), f64/f32/bf16."""
    if D.dim() != 2 or D.stride(0) != 1:
        raise ValueError("D must be an N x K column-major tensor (D.stride(0) == 1); "
                         "build it as torch.empty(K, N).T")
    N, K = D.shape
    ldd = D.stride(1) if K > 1 else N
    g = _groups(group_ptr, weights)
    p = Problem(DTYPES[_dtype_name(D)], N, K, ldd, C.c_void_p(D.data_ptr()), g.G,
                None if g.ptr is None else g.ptr.ctypes.data_as(_P(C.c_int64)),
                None if g.w is None else g.w.ctypes.data_as(_P(C.c_double)))
    p._keep = (D, g)  # keep host arrays alive with the struct
    return p


SCREENING = {"dynamic": 0, "static": 1}


def make_params(rule="fista", test="dst3", lambda_relative=True, step_L=0.0, gap_tol=1e-6,
                max_iter=10000, screening="dynamic", step="constant", bt_eta=0.0, bb_memory=0,
                bb_sigma=0.0, cp_tau=0.0, cp_sigma=0.0, cp_gamma=0.0, x0_ptr=None, obj_tol=0.0,
                batch_slots=0):
    return Params(RULES[rule], TESTS[test], 1 if lambda_relative else 0, float(step_L),
                  float(gap_tol), int(max_iter), SCREENING[screening], STEPS[step], float(bt_eta),
                  int(bb_memory), float(bb_sigma), float(cp_tau), float(cp_sigma),
                  float(cp_gamma), None if x0_ptr is None else C.c_void_p(x0_ptr),
                  float(obj_tol), int(batch_slots))


def solve(D, Y, lambdas, *, group_ptr=None, weights=None, rule="fista", test="dst3",
          lambda_relative=True, step_L=0.0, gap_tol=1e-6, max_iter=10000, stream=None, out=None,
          screened=False, screening="dynamic", step="constant", bt_eta=0.0, bb_memory=0,
          bb_sigma=0.0, cp_tau=0.0, cp_sigma=0.0, cp_gamma=0.0, x0=None, obj_tol=0.0,
          batch_slots=0):
    """Solve B Lasso (or Group-Lasso if group_ptr is given) problems sharing D.

    Y: device tensor (N,) or N x B column-major; lambdas: B floats (ratios to lambda_* when
    lambda_relative); x0: optional warm start laid out as X (device, K x B column-major
    with X's leading dimension, or (K,)).  Returns (X, infos) with X K x B column-major (or
    (K,) for 1-D Y);
    with screened=True returns (X, infos, mask), mask a K x B uint8 device tensor
    (1 = screened) from ds_solve_batch.
    """
    torch = _torch()
    one = Y.dim() == 1
    Y2 = Y.reshape(-1, 1) if one else Y
    if Y2.stride(0) != 1:
        raise ValueError("Y must be column-major")
    N, B = Y2.shape
    K = D.shape[1]
    vdt = torch.float64 if D.dtype == torch.float64 else torch.float32
    if Y2.dtype != vdt:
        raise ValueError(f"Y must be {vdt} for a {D.dtype} dictionary")
    ldy = Y2.stride(1) if B > 1 else N
    if out is None:
        X = torch.empty(B, K, dtype=vdt, device=Y.device).T
    else:
        X = out.reshape(-1, 1) if out.dim() == 1 else out
    ldx = X.stride(1) if B > 1 else K
    if x0 is not None:
        x0c = x0.reshape(-1, 1) if x0.dim() == 1 else x0
        if x0c.dtype != vdt or x0c.stride(0) != 1 or tuple(x0c.shape) != (K, B) or \
                (B > 1 and x0c.stride(1) != ldx):
            raise ValueError("x0 must have X's dtype, shape and layout")
    lam = (C.c_double * B)(*[float(v) for v in (lambdas if hasattr(lambdas, "__len__") else [lambdas])])
    infos = (Info * B)()
    prob = make_problem(D, group_ptr, weights)
    prm = make_params(rule, test, lambda_relative, step_L, gap_tol, max_iter, screening, step, bt_eta,
                      bb_memory, bb_sigma, cp_tau, cp_sigma, cp_gamma,
                      None if x0 is None else x0.data_ptr(), obj_tol, batch_slots)
    if screened:
        mask = torch.empty(B, K, dtype=torch.uint8, device=Y.device).T
        st = _lib.ds_solve_batch(C.byref(prob), C.c_void_p(Y2.data_ptr()), B, ldy, lam,
                                 C.byref(prm), C.c_void_p(X.data_ptr()), ldx, infos,
                                 C.c_void_p(mask.data_ptr()), _stream_ptr(stream))
        _check(st, "ds_solve_batch")
        infos = [i.as_dict() for i in infos]
        return (X[:, 0] if one else X), infos, (mask[:, 0] if one else mask)
    fn = _lib.glasso_solve if group_ptr is not None else _lib.lasso_solve
    st = fn(C.byref(prob), C.c_void_p(Y2.data_ptr()), B, ldy, lam, C.byref(prm),
            C.c_void_p(X.data_ptr()), ldx, infos, _stream_ptr(stream))
    _check(st, "glasso_solve" if group_ptr is not None else "lasso_solve")
    infos = [i.as_dict() for i in infos]
    return (X[:, 0] if one else X), infos


def solve_one(D, y, lam, *, group_ptr=None, weights=None, rule="fista", test="dst3",
              lambda_relative=True, step_L=0.0, gap_tol=1e-6, max_iter=10000, trace=True,
              screened=True, stream=None, screening="dynamic", step="constant", bt_eta=0.0,
              bb_memory=0, bb_sigma=0.0, cp_tau=0.0, cp_sigma=0.0, cp_gamma=0.0, x0=None, obj_tol=0.0):
    """Single-signal solve returning (x, info, screened_mask or None, trace list or None).
    x0: optional warm start, a contiguous 1-D device tensor of K values (x's dtype)."""
    torch = _torch()
    K = D.shape[1]
    vdt = torch.float64 if D.dtype == torch.float64 else torch.float32
    if y.dtype != vdt or y.dim() != 1 or not y.is_contiguous():
        raise ValueError(f"y must be a contiguous 1-D {vdt} tensor")
    if x0 is not None and (x0.dtype != vdt or x0.dim() != 1 or not x0.is_contiguous()
                           or x0.numel() != K):
        raise ValueError(f"x0 must be a contiguous 1-D {vdt} tensor of {K} values")
    x = torch.empty(K, dtype=vdt, device=y.device)
    scr = torch.empty(K, dtype=torch.uint8, device=y.device) if screened else None
    cap = int(max_iter) if trace else 0
    tr = (Trace * max(cap, 1))()
    info = Info()
    prob = make_problem(D, group_ptr, weights)
    prm = make_params(rule, test, lambda_relative, step_L, gap_tol, max_iter, screening, step, bt_eta,
                      bb_memory, bb_sigma, cp_tau, cp_sigma, cp_gamma,
                      None if x0 is None else x0.data_ptr(), obj_tol)
    st = _lib.ds_solve_one(C.byref(prob), C.c_void_p(y.data_ptr()), float(lam), C.byref(prm),
                           C.c_void_p(x.data_ptr()),
                           C.c_void_p(scr.data_ptr()) if scr is not None else None,
                           tr if trace else None, cap, C.byref(info), _stream_ptr(stream))
    _check(st, "ds_solve_one")
    inf = info.as_dict()
    trace_list = None
    if trace:
        n = min(inf["iters"], cap)
        trace_list = [dict(n_active=t.n_active, n_units=t.n_units, n_support=t.n_support,
                           nnz=t.nnz, radius=t.radius, gap=t.gap) for t in tr[:n]]
    return x, inf, scr, trace_list


def solve_one_noalloc(D, y, lam, *, group_ptr=None, weights=None, rule="fista", test="dst3",
                      lambda_relative=True, step_L=0.0, gap_tol=1e-6, max_iter=10000,
                      screened=True, stream=None, screening="dynamic", step="constant",
                      bt_eta=0.0, bb_memory=0, bb_sigma=0.0, cp_tau=0.0, cp_sigma=0.0,
                      cp_gamma=0.0, x0=None, out=None, screened_out=None, obj_tol=0.0):
    """ds_solve_one_noalloc: the single-signal solve on the library's fixed scratch array
    (no device allocation inside the call).  Returns (x, info, screened_mask or None); x and
    the mask are written into `out` / `screened_out` when given."""
    torch = _torch()
    K = D.shape[1]
    vdt = torch.float64 if D.dtype == torch.float64 else torch.float32
    if y.dtype != vdt or y.dim() != 1 or not y.is_contiguous():
        raise ValueError(f"y must be a contiguous 1-D {vdt} tensor")
    x = out if out is not None else torch.empty(K, dtype=vdt, device=y.device)
    scr = screened_out if screened_out is not None else (
        torch.empty(K, dtype=torch.uint8, device=y.device) if screened else None)
    info = Info()
    prob = make_problem(D, group_ptr, weights)
    prm = make_params(rule, test, lambda_relative, step_L, gap_tol, max_iter, screening, step, bt_eta,
                      bb_memory, bb_sigma, cp_tau, cp_sigma, cp_gamma,
                      None if x0 is None else x0.data_ptr(), obj_tol)
    st = _lib.ds_solve_one_noalloc(C.byref(prob), C.c_void_p(y.data_ptr()), float(lam),
                                   C.byref(prm), C.c_void_p(x.data_ptr()),
                                   C.c_void_p(scr.data_ptr()) if scr is not None else None,
                                   C.byref(info), _stream_ptr(stream))
    _check(st, "ds_solve_one_noalloc")
    return x, info.as_dict(), scr


def lambda_max(D, y, *, group_ptr=None, weights=None, stream=None):
    prob = make_problem(D, group_ptr, weights)
    out = C.c_double()
    arg = C.c_int64()
    _check(_lib.ds_lambda_max(C.byref(prob), C.c_void_p(y.data_ptr()), C.byref(out),
                              C.byref(arg), _stream_ptr(stream)), "ds_lambda_max")
    return out.value, arg.value


def spectral_norm_sq(D, iters=0, *, stream=None):
    prob = make_problem(D)
    out = C.c_double()
    _check(_lib.ds_spectral_norm_sq(C.byref(prob), int(iters), C.byref(out), _stream_ptr(stream)),
           "ds_spectral_norm_sq")
    return out.value


def batch_shape():
    """(index, atoms, signals) of the Z-GEMM block shape of the last batched solve."""
    a, b = C.c_int(0), C.c_int(0)
    k = _lib.ds_batch_shape(C.byref(a), C.byref(b))
    return k, a.value, b.value


def stats_enable(on=True):
    _lib.ds_stats_enable(1 if on else 0)


def stats_reset():
    _lib.ds_stats_reset()


def stats_read():
    arr = (KernelStat * STAT_COUNT)()
    n = _lib.ds_stats_read(arr, STAT_COUNT)
    return [dict(launches=a.launches, ms=a.ms, bytes=a.bytes, flops=a.flops, ms_event=a.ms_event)
            for a in arr[:n]]


def stats_launches(cap=1 << 20):
    """Per-launch records (kernel: STAT_CORR / STAT_RESID / STAT_ITER, n_atoms, bytes, ms) of
    the instrumented single-signal solves since the last reset."""
    arr = (LaunchStat * cap)()
    n = _lib.ds_stats_launches(arr, cap)
    return [dict(kernel=a.kernel, n_atoms=a.n_atoms, bytes=a.bytes, ms=a.ms) for a in arr[:n]]


# ------------------------------------------------------------------ serving
class Server:
    """Continuous-batching request loop (ds_server_* / lasso_submit / lasso_poll)."""

    def __init__(self, device=0, max_slots=64, hbm_budget_bytes=8 << 30, max_queue=4096,
                 batch_slots=0):
        """batch_slots > 0: bfloat16 Lasso dictionaries get a batched engine with this many
        resident signals, which runs the requests whose parameters it supports."""
        cfg = ServerConfig(device, max_slots, hbm_budget_bytes, max_queue, batch_slots)
        h = C.c_void_p()
        _check(_lib.ds_server_create(C.byref(cfg), C.byref(h)), "ds_server_create")
        self._h = h
        self._dicts = {}

    def add_dict(self, D, *, group_ptr=None, weights=None, store=None):
        prob = make_problem(D, group_ptr, weights)
        did = C.c_int32()
        store_code = DTYPES[store] if store is not None else prob.dtype
        _check(_lib.ds_server_add_dict(self._h, C.byref(prob), store_code, C.byref(did)),
               "ds_server_add_dict")
        self._dicts[did.value] = (D.shape[0], D.shape[1], prob.dtype, store_code)
        return did.value

    def submit(self, dict_id, y_host, lam, *, rule="fista", test="dst3", lambda_relative=True,
               step_L=0.0, gap_tol=1e-6, max_iter=10000, screening="dynamic", step="constant",
               bt_eta=0.0, bb_memory=0, bb_sigma=0.0, cp_tau=0.0, cp_sigma=0.0, cp_gamma=0.0,
               x0=None, obj_tol=0.0):
        """x0: optional warm start on the host (K values), copied at submit."""
        import numpy as np
        N, K, dt, store = self._dicts[dict_id]
        vt = np.float64 if store == 0 else np.float32
        y = np.ascontiguousarray(y_host, dtype=vt)
        assert y.size == N
        x0h = None if x0 is None else np.ascontiguousarray(x0, dtype=vt)
        assert x0h is None or x0h.size == K
        prm = make_params(rule, test, lambda_relative, step_L, gap_tol, max_iter, screening, step,
                          bt_eta, bb_memory, bb_sigma, cp_tau, cp_sigma, cp_gamma,
                          None if x0h is None else x0h.ctypes.data, obj_tol)
        rid = C.c_uint64()
        st = _lib.lasso_submit(self._h, int(dict_id), y.ctypes.data_as(C.c_void_p), float(lam),
                               C.byref(prm), C.byref(rid))
        _check(st, "lasso_submit")
        return rid.value

    def poll(self, rid, dict_id):
        import numpy as np
        N, K, dt, store = self._dicts[dict_id]
        x = np.empty(K, dtype=np.float64 if store == 0 else np.float32)
        info = Info()
        st = _lib.lasso_poll(self._h, C.c_uint64(rid), x.ctypes.data_as(C.c_void_p),
                             C.byref(info))
        if st == DS_PENDING:
            return None
        _check(st, "lasso_poll")
        return x, info.as_dict()

    def close(self):
        if self._h:
            _check(_lib.ds_server_destroy(self._h), "ds_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
