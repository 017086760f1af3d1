"""Serving (ds_server_* / lasso_submit / lasso_poll) on the device: every request's result
is the same solved alone and in a concurrent mix, admission respects the memory budget,
and the error paths report their codes."""
import time

import numpy as np
import pytest

import oracle
from paper_1412_4080_amd import datagen
from tests._util import dev_matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1412_4080_amd import binding
    return binding


def _dicts():
    """(name, D values (f64), stored dtype, group_ptr) of a small mixed set."""
    out = []
    D = datagen.gaussian_dictionary(256, 1000, 21)
    out.append(("lasso_f32", D, "f32", None))
    D = datagen.gaussian_dictionary(512, 3000, 22)
    out.append(("lasso_bf16", D, "bf16", None))
    D = datagen.gaussian_dictionary(300, 2000, 23)
    out.append(("group_f32", D, "f32", datagen.contiguous_groups(2000, 10)))
    return out


def _requests(dicts, n, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        d = int(rng.integers(len(dicts)))
        _, D, _, gp = dicts[d]
        if gp is None:
            y = datagen.lasso_signal(D, 500 + k)[0]
        else:
            y = datagen.group_signal(D, gp, 500 + k)[0]
        reqs.append((d, datagen.to_storage(y, "f32").astype(np.float32), float(rng.uniform(0.1, 0.9))))
    return reqs


def _server(B, dicts, **kw):
    import torch
    S = B.Server(**kw)
    ids = []
    for _, D, store, gp in dicts:
        Dd = dev_matrix(D, "f32")  # FP32 input; the server rounds to bfloat16 when asked
        ids.append(S.add_dict(Dd, group_ptr=gp, store=store))
    torch.cuda.synchronize()
    return S, ids


def _collect(S, ids, rid_of, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(rid_of):
        for k, (rid, d) in rid_of.items():
            if k in out:
                continue
            r = S.poll(rid, ids[d])
            if r is not None:
                out[k] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.0005)
    return out


def test_results_same_alone_and_in_the_mix(B):
    dicts = _dicts()
    reqs = _requests(dicts, 24, 1)
    # alone: one slot, one request on the device at a time
    S, ids = _server(B, dicts, max_slots=1)
    alone = {}
    for k, (d, y, r) in enumerate(reqs):
        rid = S.submit(ids[d], y, r, gap_tol=1e-6, max_iter=20000)
        alone.update(_collect(S, ids, {k: (rid, d)}))
    S.close()
    # mix: eight slots, everything submitted at once
    S, ids = _server(B, dicts, max_slots=8)
    rid_of = {k: (S.submit(ids[d], y, r, gap_tol=1e-6, max_iter=20000), d)
              for k, (d, y, r) in enumerate(reqs)}
    mix = _collect(S, ids, rid_of)
    S.close()
    for k in range(len(reqs)):
        xa, ia = alone[k]
        xm, im = mix[k]
        assert ia["status"] == 0 and im["status"] == 0
        assert np.array_equal(xa, xm), k
        assert ia["iters"] == im["iters"] and ia["gap"] == im["gap"]
    # the served solutions are certified against the oracle's optimum of the stored instance
    for k in (0, 1, 2, 3, 4, 5):
        d, y, r = reqs[k]
        _, D, store, gp = dicts[d]
        Di = datagen.to_storage(D, store)
        x, info = mix[k]
        yy = float(y.astype(np.float64) @ y.astype(np.float64))
        assert info["gap"] <= 1e-6 * yy
        if gp is None:
            star = oracle.solve_lasso(Di, y.astype(np.float64), lam=info["lambda_"], rule="fista",
                                      test="none", L=info["L"], max_iter=200000, gap_tol=1e-12)
        else:
            star = oracle.solve_group_lasso(Di, y.astype(np.float64), gp, None, lam=info["lambda_"],
                                            rule="fista", test="none", L=info["L"],
                                            max_iter=200000, gap_tol=1e-12)
        assert info["primal"] - star.primal <= info["gap"] + 1e-9
        # the primal value comes from theta rounded to FP32 (relative error ~2^-24)
        assert star.primal <= info["primal"] + 1e-7 * star.primal


def test_mixed_parameters_same_alone_and_in_the_mix(B):
    """Requests with different update rules, screening tests and modes and step rules share
    the workers: each result equals the one obtained with that request alone, bit for bit
    (no state of one request reaches another)."""
    dicts = _dicts()
    reqs = _requests(dicts, 32, 3)
    rng = np.random.default_rng(4)
    prm = []
    for d, _, _ in reqs:
        group = dicts[d][3] is not None
        rule = ["ista", "fista", "sparsa", "cp"][int(rng.integers(4))]
        kw = dict(rule=rule, test=(["none", "safe", "dst3"] if group else
                                   ["none", "safe", "dst3", "dome"])[int(rng.integers(3 if group else 4))],
                  screening=["dynamic", "static"][int(rng.integers(2))], gap_tol=1e-6,
                  max_iter=20000)
        if rule in ("ista", "fista") and rng.random() < 0.5:
            kw["step"] = "backtracking"
        if rule == "sparsa":
            kw["bb_memory"] = int(rng.integers(0, 6))
        prm.append(kw)
    S, ids = _server(B, dicts, max_slots=1)
    alone = {}
    for k, (d, y, r) in enumerate(reqs):
        rid = S.submit(ids[d], y, r, **prm[k])
        alone.update(_collect(S, ids, {k: (rid, d)}))
    S.close()
    S, ids = _server(B, dicts, max_slots=8)
    rid_of = {k: (S.submit(ids[d], y, r, **prm[k]), d) for k, (d, y, r) in enumerate(reqs)}
    mix = _collect(S, ids, rid_of)
    S.close()
    for k in range(len(reqs)):
        xa, ia = alone[k]
        xm, im = mix[k]
        assert ia["status"] == 0 and im["status"] == 0, (k, prm[k])
        assert np.array_equal(xa, xm), (k, prm[k])
        assert ia["iters"] == im["iters"] and ia["gap"] == im["gap"] and ia["L"] == im["L"]


def test_admission_under_a_tight_budget(B):
    """A budget that holds about two requests at a time: all finish, results unchanged."""
    dicts = _dicts()
    reqs = _requests(dicts, 12, 2)
    S, ids = _server(B, dicts, max_slots=8)
    rid_of = {k: (S.submit(ids[d], y, r, gap_tol=1e-6, max_iter=20000), d)
              for k, (d, y, r) in enumerate(reqs)}
    ref = _collect(S, ids, rid_of)
    S.close()
    S, ids = _server(B, dicts, max_slots=8, hbm_budget_bytes=12 << 20)
    rid_of = {k: (S.submit(ids[d], y, r, gap_tol=1e-6, max_iter=20000), d)
              for k, (d, y, r) in enumerate(reqs)}
    got = _collect(S, ids, rid_of)
    S.close()
    for k in range(len(reqs)):
        assert np.array_equal(ref[k][0], got[k][0])


def test_error_codes(B):
    import ctypes as C
    dicts = _dicts()[:1]
    S, ids = _server(B, dicts, max_slots=1, max_queue=1)
    y = datagen.to_storage(datagen.lasso_signal(dicts[0][1], 7)[0], "f32").astype(np.float32)
    prm = B.make_params()
    rid = C.c_uint64()
    st = B._lib.lasso_submit(S._h, 99, y.ctypes.data_as(C.c_void_p), 0.5, C.byref(prm), C.byref(rid))
    assert st == B.DS_ENOTFOUND
    info = B.Info()
    assert B._lib.lasso_poll(S._h, C.c_uint64(123456), None, C.byref(info)) == B.DS_ENOTFOUND
    S.close()
    # a request larger than the whole budget can never be admitted
    S, ids = _server(B, dicts, max_slots=1, hbm_budget_bytes=64 << 10)
    st = B._lib.lasso_submit(S._h, ids[0], y.ctypes.data_as(C.c_void_p), 0.5, C.byref(prm), C.byref(rid))
    assert st == B.DS_ENOMEM
    S.close()
    # a full queue: one worker busy on a slow solve, one request waiting, the next refused
    D = datagen.gaussian_dictionary(2000, 10000, 0)
    S, ids = _server(B, [("big", D, "f32", None)], max_slots=1, max_queue=1)
    yb = datagen.to_storage(datagen.lasso_signal(D, 0)[0], "f32").astype(np.float32)
    codes = []
    rids = []
    for _ in range(3):
        st = B._lib.lasso_submit(S._h, ids[0], yb.ctypes.data_as(C.c_void_p), 0.1, C.byref(prm),
                                 C.byref(rid))
        codes.append(st)
        if st == 0:
            rids.append(rid.value)
    assert B.DS_EBUSY in codes, codes
    _collect(S, ids, {k: (r, 0) for k, r in enumerate(rids)})
    S.close()


def test_dictionary_beyond_the_single_signal_kernels_refused(B):
    """The workers serve every dictionary with single-signal solves, so a dictionary with more
    atoms than the correlation pass covers (16384 blocks of 16) is refused when it is added,
    before its copy is made (the dictionary pointer is never read); the server goes on
    serving."""
    import ctypes as C
    dicts = _dicts()[:1]
    S, ids = _server(B, dicts, max_slots=1)
    p = B.Problem(B.DTYPES["f32"], 100, 262_145, 100, C.c_void_p(0x1000), 0, None, None)
    did = C.c_int32()
    st = B._lib.ds_server_add_dict(S._h, C.byref(p), B.DTYPES["bf16"], C.byref(did))
    assert st == B.DS_EINVAL and "at most 262144 atoms" in B.last_error()
    y = datagen.to_storage(datagen.lasso_signal(dicts[0][1], 3)[0], "f32").astype(np.float32)
    rid = S.submit(ids[0], y, 0.5)
    _collect(S, ids, {0: (rid, 0)})
    S.close()
