"""The allocation-free generator entry point (tr_gen_planted_noalloc), through
the C ABI, against the allocating one (tr_gen_planted): the same X, true
cores and initial cores bit for bit, on two calls in a row (the second with a
smaller job, so the shared scratch array still holds the first call's data),
and an oversized job refused with TR_ENOMEM without touching its outputs."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _buffers(dims, ranks, dtype):
    import torch
    N = len(dims)
    X = torch.full((int(np.prod(dims)),), -7.0, dtype=dtype, device="cuda")
    cores = lambda: [torch.full((ranks[k] * dims[k] * ranks[(k + 1) % N],), -7.0, dtype=torch.float64,
                                device="cuda") for k in range(N)]
    return X, cores(), cores()


def _call(fn, dims, ranks, seed, eta, X, true, init):
    import torch
    from paper_2210_11362_amd import _lib as C
    N = len(dims)
    ptrs = lambda cs: (ctypes.c_void_p * N)(*[c.data_ptr() for c in cs])
    xdt = C.TR_F32 if X.dtype == torch.float32 else C.TR_F64
    stream = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    return getattr(C.lib(), fn)(N, (ctypes.c_int64 * N)(*dims), (ctypes.c_int64 * N)(*ranks),
                                ctypes.c_uint64(seed), float(eta), ctypes.c_void_p(X.data_ptr()), xdt,
                                ptrs(true), ptrs(init), stream)


def test_noalloc_generator_matches_allocating_one():
    import torch
    cases = [((48, 40, 36, 30), (6, 5, 6, 4), torch.float32, 91),
             ((13, 9, 11), (3, 4, 2), torch.float64, 92)]
    for dims, ranks, dt, seed in cases:
        say(f"[noalloc] dims={dims} ranks={ranks} {dt}")
        Xa, ta, ia = _buffers(dims, ranks, dt)
        Xb, tb, ib = _buffers(dims, ranks, dt)
        assert _call("tr_gen_planted", dims, ranks, seed, 0.02, Xa, ta, ia) == 0
        assert _call("tr_gen_planted_noalloc", dims, ranks, seed, 0.02, Xb, tb, ib) == 0
        torch.cuda.synchronize()
        assert torch.equal(Xa, Xb)
        for a, b in zip(ta + ia, tb + ib):
            assert torch.equal(a, b)
        assert float(Xb.abs().max()) > 0
    from paper_2210_11362_amd import _lib as C
    dims, ranks = (128, 128, 128, 128), (24, 24, 24, 24)        # workspace far beyond the scratch array
    X = torch.full((128 ** 4,), 3.0, dtype=torch.float32, device="cuda")
    N = 4
    rc = C.lib().tr_gen_planted_noalloc(N, (ctypes.c_int64 * N)(*dims), (ctypes.c_int64 * N)(*ranks),
                                        ctypes.c_uint64(1), 0.01, ctypes.c_void_p(X.data_ptr()), C.TR_F32,
                                        None, None, None)
    torch.cuda.synchronize()
    assert rc == C.TR_ENOMEM
    assert bool((X == 3.0).all())
    del X
