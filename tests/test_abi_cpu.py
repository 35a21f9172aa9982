"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, and rejects invalid arguments before touching a device."""
import ctypes

import pytest

import paper_2210_11362_amd as P
from paper_2210_11362_amd import _lib as C


def test_library_exports_header_symbols():
    L = P.lib()
    names = P.header_symbols()
    assert "tr_als_init" in names and "tr_als_sweep" in names and "tr_als_fit" in names
    for n in names:
        assert hasattr(L, n), n


def test_strerror_codes():
    L = P.lib()
    assert L.tr_als_strerror(0) == b"ok"
    assert L.tr_als_strerror(-4) == b"singular coefficient matrix"
    assert L.tr_als_strerror(-5) == b"non-finite value"
    assert L.tr_als_strerror(123) == b"unknown status"


@pytest.mark.parametrize("case", ["order1", "order9", "null_dims", "bad_dtype", "bad_variant", "rank0", "rank_big",
                                  "dim0", "null_core"])
def test_init_rejects_invalid_arguments(case):
    L = P.lib()
    N = {"order1": 1, "order9": 9}.get(case, 3)
    dims = (ctypes.c_int64 * 9)(*([4] * 9))
    ranks = (ctypes.c_int64 * 9)(*([2] * 9))
    if case == "rank0":
        ranks[1] = 0
    if case == "rank_big":
        ranks[1] = 33
    if case == "dim0":
        dims[2] = 0
    cores = (ctypes.c_void_p * 9)(*([0x1000] * 9))
    if case == "null_core":
        cores[2] = None
    h = ctypes.c_void_p(0xdead)
    rc = L.tr_als_init(ctypes.byref(h), N, None if case == "null_dims" else dims, ranks, ctypes.c_void_p(0x1000),
                       7 if case == "bad_dtype" else C.TR_F32, cores, 5 if case == "bad_variant" else C.TR_NE, None)
    assert rc == C.TR_EINVAL
    assert not h.value


def test_null_context_calls():
    L = P.lib()
    assert L.tr_als_destroy(None) == 0
    assert L.tr_als_sweep(None, 1, 1, 1) == C.TR_EINVAL
    d = ctypes.c_double()
    assert L.tr_als_fit(None, ctypes.byref(d)) == C.TR_EINVAL
    assert L.tr_als_last_error(None) == b"null context"


def _desc(**kw):
    d = C.JobDesc()
    d.N = kw.get("N", 3)
    for k in range(8):
        d.dims[k] = 8
        d.ranks[k] = 2
    d.variant = kw.get("variant", C.TR_NE)
    d.prec_mixed, d.nsweeps_mixed = kw.get("prec_mixed", C.TR_BF16), kw.get("nsweeps_mixed", 2)
    d.prec_fin, d.nsweeps_fin = C.TR_F32, 1
    d.refine = kw.get("refine", 1)
    d.eta = kw.get("eta", 0.01)
    d.x_dtype = kw.get("x_dtype", C.TR_F32)
    return d


def test_serving_rejects_invalid_arguments_before_the_device():
    L = P.lib()
    h = ctypes.c_void_p(0xdead)
    assert L.tr_srv_create(ctypes.byref(h), 1 << 20, 0, 0) == C.TR_EINVAL      # no slots
    assert L.tr_srv_create(ctypes.byref(h), 1 << 20, 65, 0) == C.TR_EINVAL     # too many slots
    assert L.tr_srv_create(ctypes.byref(h), 1 << 20, 4, 8) == C.TR_EINVAL      # unknown flag
    assert not h.value
    assert L.tr_srv_create(None, 1 << 20, 4, 0) == C.TR_EINVAL
    jid = ctypes.c_uint64()
    assert L.tr_srv_submit(None, ctypes.byref(_desc()), ctypes.byref(jid)) == C.TR_EINVAL
    info = C.JobInfo()
    assert L.tr_srv_poll(None, 1, ctypes.byref(info)) == C.TR_EINVAL
    assert L.tr_srv_wait(None, 1, ctypes.byref(info)) == C.TR_EINVAL
    assert L.tr_srv_drain(None) == C.TR_EINVAL
    assert L.tr_srv_destroy(None) == C.TR_OK
    assert L.tr_srv_job_error(None, 1) == b"null server"


@pytest.mark.parametrize("case", ["order1", "rank0", "dim0", "null_X"])
def test_gen_planted_rejects_invalid_arguments(case):
    L = P.lib()
    N = 1 if case == "order1" else 3
    dims = (ctypes.c_int64 * 3)(4, 0 if case == "dim0" else 5, 6)
    ranks = (ctypes.c_int64 * 3)(2, 0 if case == "rank0" else 2, 2)
    X = None if case == "null_X" else ctypes.c_void_p(0x1000)
    assert L.tr_gen_planted(N, dims, ranks, 1, 0.01, X, C.TR_F32, None, None, None) == C.TR_EINVAL
