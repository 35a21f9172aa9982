"""Host code of the library on a CPU stand-in of the HIP runtime.

The library's objects are linked against ``tests/hostrt/stand_in_hip.cpp``
(no GPU needed, kernels not executed), and the C ABI is driven with the shapes
of the GPU tests and with serving streams.  The stand-in checks every launch
(grid, block, dynamic LDS, pointer arguments inside live allocations, operand
extents of the modelled kernels), every copy and fill, graph captures (no
fill, allocation, free or synchronisation while one is open) and which host
threads call the runtime while a server is alive.
"""
import pytest

from tests.hostrt import replay as R
from tests.test_gpu_parity import INV_SHAPES, SHAPES
from tests.test_gpu_qr import LARGE_QR_SHAPES, QR_SHAPES
from tests.test_gpu_serving import LANE_JOBS, _mix_jobs

GB = 1 << 30
KW = dict(eta=0.01, prec_mixed="bf16", nsweeps_mixed=4, prec_fin="f32", nsweeps_fin=2)


@pytest.fixture(scope="module")
def host():
    h = R.Host(R.build_host_lib())
    h.L.fakehip_set_delay_us(0)
    return h


def _clean(h, what):
    v = h.violations()
    assert not v, f"{what}: {len(v)} problems, first: {v[:3]}"


@pytest.mark.parametrize("dims,ranks", SHAPES + INV_SHAPES, ids=[f"{d}-{r}" for d, r in SHAPES + INV_SHAPES])
def test_ne_contexts_stay_inside_their_buffers(host, dims, ranks):
    host.reset()
    codes = R.run_context(host, dims, ranks, precs=("f64", "f32", "bf16", "fp8"), xdt="f32")
    assert all(rc == 0 for _, rc in codes), codes
    _clean(host, f"NE {dims} {ranks}")
    if len(dims) >= 3:   # order 2: the ring is one Gram, realigned without a product
        assert host.L.fakehip_launches(b"gemm64_kernel") + host.L.fakehip_launches(b"gemm64_pair_kernel") > 0


@pytest.mark.parametrize("variant", ["qr", "qrne"])
@pytest.mark.parametrize("dims,ranks", QR_SHAPES, ids=[f"{d}-{r}" for d, r in QR_SHAPES])
def test_qr_contexts_stay_inside_their_buffers(host, dims, ranks, variant):
    host.reset()
    codes = R.run_context(host, dims, ranks, variant=variant, precs=("f64", "bf16"), xdt="f64")
    assert all(rc == 0 for _, rc in codes), codes
    _clean(host, f"{variant} {dims} {ranks}")


@pytest.mark.parametrize("variant", ["qr", "qrne"])
@pytest.mark.parametrize("dims,ranks", LARGE_QR_SHAPES, ids=[f"{d}-{r}" for d, r in LARGE_QR_SHAPES])
def test_qr_large_bond_products_host_side(host, dims, ranks, variant):
    """R_n R_{n+1} > 128: every rocBLAS operand inside its buffer, none issued
    on a stream under capture, the slice products of a middle mode in bounds."""
    host.reset()
    codes = R.run_context(host, dims, ranks, variant=variant, precs=("f64", "f32", "bf16"), xdt="f32")
    assert all(rc == 0 for _, rc in codes), codes
    _clean(host, f"{variant} {dims} {ranks}")
    calls = {k: host.L.fakehip_launches(k.encode()) for k in ("rocblas_dsyrk", "rocblas_dtrsm", "rocblas_dgemm",
                                                              "rocblas_dgemm_strided_batched")}
    assert calls["rocblas_dgemm"] + calls["rocblas_dgemm_strided_batched"] > 0, calls
    if variant == "qr":
        assert calls["rocblas_dgemm_strided_batched"] > 0 and calls["rocblas_dtrsm"] > 0, calls
    assert calls["rocblas_dsyrk"] == 0, calls   # rocBLAS's SYRK is slow at these shapes


def test_ring_intermediates_exceed_one_gram_when_ranks_alternate(host):
    """The ring's intermediates are R_{m+1}^2 x R_j^2: with alternating ranks
    they exceed max_k (R_k R_{k+1})^2, the size the ring workspaces once had
    (the launches of this shape then wrote 360 bytes past a 288-byte buffer).
    The workspaces are now sized over the ring (previous test: in bounds)."""
    dims, ranks = (6, 7, 5, 8, 6), (2, 3, 2, 2, 3)
    host.reset()
    R.run_context(host, dims, ranks, precs=("f64",), xdt="f64", sweeps=1)
    one_gram = max((ranks[k] * ranks[(k + 1) % 5]) ** 2 for k in range(5))
    ring = [m * n for m, n, realign, _ in host.gemm_log() if not realign]
    assert max(ring) == 81 and one_gram == 36
    _clean(host, "ring")


def test_serving_alone_and_in_mix_host_side(host):
    host.reset()
    host.L.fakehip_set_delay_us(200)
    jobs = _mix_jobs()
    s = R.Server(host, 4 * GB, 1)
    for j in jobs:
        rc, jid = s.submit(j["dims"], j["ranks"], seed=j["seed"], **KW)
        assert rc == 0
        assert s.wait(jid).state == 2, s.error(jid)
    assert s.close() == 1                      # only the executor thread called the runtime
    host.L.fakehip_set_delay_us(10000)         # jobs in flight overlap the 2 ms arrivals
    s = R.Server(host, 4 * GB, 6)
    for k, j in enumerate(jobs):
        assert s.submit(j["dims"], j["ranks"], seed=j["seed"], t_arrival=0.002 * k, **KW)[0] == 0
    s.drain()
    st = s.stats()
    assert st["done"] == len(jobs) and st["failed"] == 0 and st["max_running"] >= 2
    assert s.close() == 1
    host.L.fakehip_set_delay_us(0)
    _clean(host, "serving mix")


def test_admission_under_a_tight_budget_host_side(host):
    host.reset()
    host.L.fakehip_set_delay_us(500)
    dims, ranks = (40, 40, 40, 40), (5, 5, 5, 5)
    s = R.Server(host, 4 * GB, 1)
    rc, jid = s.submit(dims, ranks, seed=1, **KW)
    F = s.wait(jid).footprint
    s.close()
    s = R.Server(host, int(2.5 * F), 8)
    ids = [s.submit(dims, ranks, seed=10 + k, **KW)[1] for k in range(6)]
    assert s.submit((60, 60, 60, 60), ranks, seed=2, **KW)[0] != 0      # can never fit
    s.drain()
    st = s.stats()
    assert st["done"] == 6 and st["max_running"] == 2 and st["peak_in_use"] <= st["arena_bytes"]
    adm = [s.poll(j).t_admit for j in ids]
    assert adm == sorted(adm)
    assert s.close() == 1
    host.L.fakehip_set_delay_us(0)
    _clean(host, "admission")


def test_batch_lane_waiting_for_memory_launches_no_empty_batch(host):
    """Small jobs that do not fit while the other lane runs leave the idle lane
    unlaunched (an empty batch would be a zero-size grid)."""
    host.reset()
    host.L.fakehip_set_delay_us(3000)
    s = R.Server(host, 3 << 20, 2, batch=True)
    ids = [s.submit(d, r, seed=k, **KW)[1] for k, (d, r) in enumerate(LANE_JOBS * 4)]
    s.drain()
    assert all(s.poll(j).state == 2 and s.poll(j).batched for j in ids)
    assert s.close() == 1
    host.L.fakehip_set_delay_us(0)
    _clean(host, "lanes")
    assert host.L.fakehip_launches(b"tiny_als_kernel") > 1


def test_serving_stream_host_side(host):
    """300 Poisson arrivals, orders 3-5, modes 16-128, ranks 2-12, lanes on."""
    host.reset()
    host.L.fakehip_set_delay_us(300)
    s = R.Server(host, 64 * GB, 8, batch=True)
    res = [s.submit(j["dims"], j["ranks"], seed=j["seed"], t_arrival=j["t_arrival"], prec_mixed="bf16",
                    nsweeps_mixed=8, prec_fin="f32", nsweeps_fin=2) for j in R.serving_stream(300)]
    s.drain()
    st = s.stats()
    ok = sum(1 for rc, _ in res if rc == 0)
    assert st["done"] == ok and st["failed"] == 0 and ok >= 280
    assert s.close() == 1
    host.L.fakehip_set_delay_us(0)
    _clean(host, "stream")
    assert host.L.fakehip_live_allocations() == 0


def test_generator_without_allocation_host_side(host):
    """tr_gen_planted_noalloc: no allocation, free or synchronisation; the
    kernels' operands lie inside the library's scratch array; an oversized job
    is refused before anything is enqueued."""
    import ctypes
    import numpy as np
    C = host.C
    L = host.L
    L.fakehip_calls.restype = ctypes.c_long
    L.fakehip_calls.argtypes = [ctypes.c_char_p]
    f = L.tr_gen_planted_noalloc
    f.restype = ctypes.c_int
    f.argtypes = C._SIGS["tr_gen_planted_noalloc"][1]
    for dims, ranks in (((40, 36, 30), (5, 6, 4)), ((13, 9, 11), (3, 4, 2))):
        N = len(dims)
        X = host.alloc(int(np.prod(dims)) * 4)
        init = [host.alloc(R.core_elems(dims, ranks, k) * 8) for k in range(N)]
        host.reset()
        rc = f(N, (ctypes.c_int64 * N)(*dims), (ctypes.c_int64 * N)(*ranks), 7, 0.01, ctypes.c_void_p(X), C.TR_F32,
               None, (ctypes.c_void_p * N)(*init), None)
        assert rc == 0
        assert L.fakehip_launches(None) > 0
        for what in (b"alloc", b"host alloc", b"free", b"sync"):
            assert L.fakehip_calls(what) == 0, what
        _clean(host, f"generator {dims}")
        for p in init + [X]:
            host.free(p)
    dims, ranks = (128, 128, 128, 128), (24, 24, 24, 24)      # tables far beyond the scratch array
    host.reset()
    rc = f(4, (ctypes.c_int64 * 4)(*dims), (ctypes.c_int64 * 4)(*ranks), 7, 0.01, ctypes.c_void_p(0x1000),
           C.TR_F32, None, None, None)
    assert rc == C.TR_ENOMEM and L.fakehip_launches(None) == 0


@pytest.mark.parametrize("variant", ["ne", "qr", "qrne"])
def test_in_loop_error_and_inner_product_host_side(host, variant):
    """tr_als_run (sweeps + the in-loop error kernels) and tr_inner / tr_norm:
    every launch in bounds, the workspace of tr_inner released."""
    import ctypes
    import numpy as np
    L, C = host.L, host.C
    dims, ranks, rb = (17, 20, 13, 11), (2, 3, 4, 3), (3, 2, 2, 4)
    N = 4
    X = host.alloc(int(np.prod(dims)) * 8)
    ca = [host.alloc(R.core_elems(dims, ranks, k) * 8) for k in range(N)]
    cb = [host.alloc(R.core_elems(dims, rb, k) * 8) for k in range(N)]
    host.reset()
    ctx = ctypes.c_void_p()
    d, r, s = (ctypes.c_int64 * N)(*dims), (ctypes.c_int64 * N)(*ranks), (ctypes.c_int64 * N)(*rb)
    assert L.tr_als_init(ctypes.byref(ctx), N, d, r, ctypes.c_void_p(X), C.TR_F64, (ctypes.c_void_p * N)(*ca),
                         C.VARIANT[variant], None) == 0
    k, f = ctypes.c_int(), ctypes.c_double()
    # stand-in data are zeros: the estimate repeats, so tol 0 stops after the second sweep
    assert L.tr_als_run(ctx, 3, C.TR_F64, 1, 0.0, ctypes.byref(k), ctypes.byref(f)) == 0 and k.value == 2
    assert L.fakehip_launches(b"cheap_fit_kernel") == 2
    L.tr_als_destroy(ctx)
    v = ctypes.c_double()
    live = L.fakehip_live_allocations()
    assert L.tr_inner(N, d, r, (ctypes.c_void_p * N)(*ca), s, (ctypes.c_void_p * N)(*cb), ctypes.byref(v), None) == 0
    assert L.tr_norm(N, d, s, (ctypes.c_void_p * N)(*cb), ctypes.byref(v), None) == 0
    assert L.fakehip_live_allocations() == live
    _clean(host, f"run / inner {variant}")
    for p in ca + cb + [X]:
        host.free(p)
