"""Thin object wrapper over the C ABI, using torch tensors for device memory."""
from __future__ import annotations

import ctypes

from . import _lib as C


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


class TRContext:
    """One decomposition job.  ``X`` is a CUDA tensor (float32/float64) whose
    memory holds the tensor with the first index fastest (a contiguous tensor of
    shape (I_N, ..., I_1), or a flat one); ``cores`` are CUDA float64 tensors
    holding core n (R_n x I_n x R_{n+1}) with element (a, i, b) at a + R_n*(i + I_n*b).
    The cores are overwritten in place by every ``sweep``."""

    def __init__(self, X, dims, ranks, cores, variant: str = "ne", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("TRContext needs a GPU")
        L = C.lib()
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(r) for r in ranks)
        self.N = len(self.dims)
        if not X.is_cuda or not X.is_contiguous():
            raise ValueError("X must be a contiguous CUDA tensor")
        xdt = {torch.float64: C.TR_F64, torch.float32: C.TR_F32}.get(X.dtype)
        if xdt is None:
            raise ValueError("X must be float32 or float64")
        for c in cores:
            if not c.is_cuda or c.dtype != torch.float64 or not c.is_contiguous():
                raise ValueError("cores must be contiguous CUDA float64 tensors")
        self.X = X
        self.cores = list(cores)
        self._stream = stream
        d = (ctypes.c_int64 * self.N)(*self.dims)
        r = (ctypes.c_int64 * self.N)(*self.ranks)
        cp = (ctypes.c_void_p * self.N)(*[c.data_ptr() for c in self.cores])
        h = ctypes.c_void_p()
        rc = L.tr_als_init(ctypes.byref(h), self.N, d, r, ctypes.c_void_p(X.data_ptr()), xdt, cp,
                           C.VARIANT[variant], _stream_handle(stream))
        C.check(rc, None, "tr_als_init")
        self._h = h

    # -- C-ABI calls ---------------------------------------------------------
    def sweep(self, nsweeps: int = 1, prec: str = "f32", refine: int = 1):
        return C.check(C.lib().tr_als_sweep(self._h, int(nsweeps), C.PREC[prec], int(refine)), self._h, "tr_als_sweep")

    def set_solve(self, solve: str = "factor", rcond: float = 0.0):
        """``factor`` (default) or ``pinv`` (rank-deficient-safe, ``tr_als_set_solve``)."""
        C.check(C.lib().tr_als_set_solve(self._h, C.SOLVE[solve], float(rcond)), self._h, "tr_als_set_solve")

    def run(self, max_sweeps: int, prec: str = "f64", refine: int = 1, tol: float = 0.0):
        """Sweeps until the in-loop error estimate changes by at most ``tol``
        (``tr_als_run``): returns (sweeps run, last estimate)."""
        k, f = ctypes.c_int(), ctypes.c_double()
        C.check(C.lib().tr_als_run(self._h, int(max_sweeps), C.PREC[prec], int(refine), float(tol), ctypes.byref(k),
                                   ctypes.byref(f)), self._h, "tr_als_run")
        return k.value, f.value

    def fit(self) -> float:
        v = ctypes.c_double()
        C.check(C.lib().tr_als_fit(self._h, ctypes.byref(v)), self._h, "tr_als_fit")
        return v.value

    def update_mode(self, n: int, prec: str = "f32", refine: int = 1):
        return C.check(C.lib().tr_als_update_mode(self._h, int(n), C.PREC[prec], int(refine)), self._h,
                       "tr_als_update_mode")

    def store_cores(self):
        return C.check(C.lib().tr_als_store_cores(self._h), self._h, "tr_als_store_cores")

    def _rr(self, n):
        return self.ranks[n - 1] * self.ranks[n % self.N]

    def mttsp(self, n: int, prec: str = "f32"):
        """M_n as an (I_n, R_nR_{n+1}) float64 CUDA tensor."""
        import torch
        out = torch.empty((self._rr(n), self.dims[n - 1]), dtype=torch.float64, device=self.X.device)
        C.check(C.lib().tr_als_mttsp(self._h, int(n), C.PREC[prec], ctypes.c_void_p(out.data_ptr())), self._h,
                "tr_als_mttsp")
        return out.t()

    def coef(self, n: int):
        import torch
        rr = self._rr(n)
        out = torch.empty((rr, rr), dtype=torch.float64, device=self.X.device)
        C.check(C.lib().tr_als_coef(self._h, int(n), ctypes.c_void_p(out.data_ptr())), self._h, "tr_als_coef")
        return out.t()

    def gram(self, k: int):
        import torch
        rr = self._rr(k)
        out = torch.empty((rr, rr), dtype=torch.float64, device=self.X.device)
        C.check(C.lib().tr_als_gram(self._h, int(k), ctypes.c_void_p(out.data_ptr())), self._h, "tr_als_gram")
        return out.t()

    def regime(self, n: int) -> int:
        """X-contraction kernel of mode n: 1 two-stage GEMM, 2 fused single pass."""
        r = C.lib().tr_als_mode_regime(self._h, int(n))
        if r < 0:
            C.check(r, self._h, "tr_als_mode_regime")
        return r

    def xnorm2(self) -> float:
        v = ctypes.c_double()
        C.check(C.lib().tr_als_xnorm2(self._h, ctypes.byref(v)), self._h, "tr_als_xnorm2")
        return v.value

    def profile_enable(self, on: bool = True):
        C.check(C.lib().tr_als_profile_enable(self._h, 1 if on else 0), self._h, "tr_als_profile_enable")

    def profile_read(self):
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        C.check(C.lib().tr_als_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b)), self._h,
                "tr_als_profile_read")
        return ms.value, n.value, b.value

    def graphs(self):
        """(number of captured sweep graphs, why the last capture was abandoned)."""
        buf = ctypes.create_string_buffer(256)
        r = C.lib().tr_als_debug_graphs(self._h, buf, len(buf))
        if r < 0:
            C.check(r, self._h, "tr_als_debug_graphs")
        return r, buf.value.decode()

    def shadow(self, prec: str, transposed: bool = False):
        """(raw shadow bytes as a flat CUDA uint8 tensor, scale, split K) of
        the BF16 or FP8 copy of X the contraction reads."""
        import torch
        numel = 1
        for d in self.dims:
            numel *= d
        out = torch.empty(numel * (2 if prec == "bf16" else 1), dtype=torch.uint8, device=self.X.device)
        sc, k = ctypes.c_float(), ctypes.c_int64()
        C.check(C.lib().tr_als_debug_shadow(self._h, C.PREC[prec], 1 if transposed else 0,
                                            ctypes.c_void_p(out.data_ptr()), ctypes.byref(sc), ctypes.byref(k)),
                self._h, "tr_als_debug_shadow")
        return out, sc.value, k.value

    def close(self):
        if getattr(self, "_h", None):
            C.lib().tr_als_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def gen_planted(dims, ranks, seed: int, eta: float, dtype=None, want_true: bool = False, want_init: bool = True,
                stream=None):
    """Planted TR tensor generated on the device (``tr_gen_planted``): returns
    (X flat CUDA tensor, true cores or None, initial cores or None); cores are
    flat CUDA float64 tensors in the core layout."""
    import torch
    dtype = dtype or torch.float32
    xdt = {torch.float64: C.TR_F64, torch.float32: C.TR_F32}[dtype]
    dims = tuple(int(d) for d in dims)
    ranks = tuple(int(r) for r in ranks)
    N = len(dims)
    numel = 1
    for d in dims:
        numel *= d
    X = torch.empty(numel, dtype=dtype, device="cuda")

    def cores():
        return [torch.empty(ranks[k] * dims[k] * ranks[(k + 1) % N], dtype=torch.float64, device="cuda")
                for k in range(N)]

    true = cores() if want_true else None
    init = cores() if want_init else None
    ptrs = lambda cs: (ctypes.c_void_p * N)(*[c.data_ptr() for c in cs]) if cs is not None else None
    rc = C.lib().tr_gen_planted(N, (ctypes.c_int64 * N)(*dims), (ctypes.c_int64 * N)(*ranks),
                                ctypes.c_uint64(int(seed) & (2**64 - 1)), float(eta), ctypes.c_void_p(X.data_ptr()),
                                xdt, ptrs(true), ptrs(init), _stream_handle(stream))
    C.check(rc, None, "tr_gen_planted")
    return X, true, init


class TRServer:
    """Request loop over the serving C ABI (``tr_srv_*``): jobs are submitted
    with an arrival time, admitted by HBM footprint into the server's arena and
    run concurrently on its slots."""

    def __init__(self, hbm_budget_bytes: int = 0, slots: int = 8, batch: bool = False):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("TRServer needs a GPU")
        h = ctypes.c_void_p()
        rc = C.lib().tr_srv_create(ctypes.byref(h), ctypes.c_size_t(int(hbm_budget_bytes)), int(slots),
                                   C.TR_SRV_BATCH if batch else 0)
        C.check(rc, None, "tr_srv_create")
        self._h = h
        self._keep = {}

    def submit(self, dims, ranks, seed: int = 0, eta: float = 0.01, prec_mixed: str = "bf16",
               nsweeps_mixed: int = 8, prec_fin: str = "f32", nsweeps_fin: int = 2, refine: int = 1,
               variant: str = "ne", t_arrival: float = 0.0, X=None, init_cores=None, x_dtype: str = "f32") -> int:
        import torch
        d = C.JobDesc()
        N = len(dims)
        d.N = N
        for k in range(N):
            d.dims[k] = int(dims[k])
            d.ranks[k] = int(ranks[k])
        d.variant = C.VARIANT[variant]
        d.prec_mixed, d.nsweeps_mixed = C.PREC[prec_mixed], int(nsweeps_mixed)
        d.prec_fin, d.nsweeps_fin = C.PREC[prec_fin], int(nsweeps_fin)
        d.refine = int(refine)
        d.seed = int(seed) & (2**64 - 1)
        d.eta = float(eta)
        keep = []
        if X is not None:
            if not X.is_cuda or not X.is_contiguous():
                raise ValueError("X must be a contiguous CUDA tensor")
            d.X = ctypes.c_void_p(X.data_ptr())
            d.x_dtype = {torch.float64: C.TR_F64, torch.float32: C.TR_F32}[X.dtype]
            keep.append(X)
        else:
            d.x_dtype = C.PREC[x_dtype]
        if init_cores is not None:
            arr = (ctypes.c_void_p * N)(*[c.data_ptr() for c in init_cores])
            d.init_cores = ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p))
            keep += [arr, *init_cores]
        d.t_arrival = float(t_arrival)
        jid = ctypes.c_uint64()
        C.check(C.lib().tr_srv_submit(self._h, ctypes.byref(d), ctypes.byref(jid)), None, "tr_srv_submit")
        if keep:
            self._keep[jid.value] = keep
        return jid.value

    @staticmethod
    def _info(i):
        return {"state": i.state, "status": i.status, "rel_err": i.rel_err, "t_arrival": i.t_arrival,
                "t_admit": i.t_admit, "t_done": i.t_done, "footprint": i.footprint, "slot": i.slot,
                "batched": bool(i.batched)}

    def poll(self, jid: int) -> dict:
        i = C.JobInfo()
        C.check(C.lib().tr_srv_poll(self._h, ctypes.c_uint64(jid), ctypes.byref(i)), None, "tr_srv_poll")
        return self._info(i)

    def wait(self, jid: int) -> dict:
        i = C.JobInfo()
        C.check(C.lib().tr_srv_wait(self._h, ctypes.c_uint64(jid), ctypes.byref(i)), None, "tr_srv_wait")
        self._keep.pop(jid, None)
        return self._info(i)

    def error(self, jid: int) -> str:
        return C.lib().tr_srv_job_error(self._h, ctypes.c_uint64(jid)).decode()

    def result(self, jid: int, dims, ranks):
        """Final cores of a finished job as Fortran-ordered numpy arrays."""
        import numpy as np
        N = len(dims)
        outs = [np.zeros(int(ranks[k]) * int(dims[k]) * int(ranks[(k + 1) % N]), dtype=np.float64)
                for k in range(N)]
        arr = (ctypes.c_void_p * N)(*[o.ctypes.data for o in outs])
        C.check(C.lib().tr_srv_result(self._h, ctypes.c_uint64(jid), arr), None, "tr_srv_result")
        return [np.asfortranarray(o.reshape((int(ranks[k]), int(dims[k]), int(ranks[(k + 1) % N])), order="F"))
                for k, o in enumerate(outs)]

    def drain(self):
        C.check(C.lib().tr_srv_drain(self._h), None, "tr_srv_drain")
        self._keep.clear()

    def stats(self) -> dict:
        s = C.SrvStats()
        C.check(C.lib().tr_srv_stats_read(self._h, ctypes.byref(s)), None, "tr_srv_stats_read")
        return {k: getattr(s, k) for k, _ in C.SrvStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            C.lib().tr_srv_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _core_ptrs(cores):
    return (ctypes.c_void_p * len(cores))(*[c.data_ptr() for c in cores])


def tr_inner(dims, ranks_a, cores_a, ranks_b, cores_b, stream=None) -> float:
    """<A, B> of two tensors in TR format (``tr_inner``); cores are flat CUDA
    float64 tensors in the core layout."""
    N = len(dims)
    v = ctypes.c_double()
    C.check(C.lib().tr_inner(N, (ctypes.c_int64 * N)(*dims), (ctypes.c_int64 * N)(*ranks_a), _core_ptrs(cores_a),
                             (ctypes.c_int64 * N)(*ranks_b), _core_ptrs(cores_b), ctypes.byref(v),
                             _stream_handle(stream)), None, "tr_inner")
    return v.value


def tr_norm(dims, ranks, cores, stream=None) -> float:
    """||A||_F of a tensor in TR format (``tr_norm``)."""
    N = len(dims)
    v = ctypes.c_double()
    C.check(C.lib().tr_norm(N, (ctypes.c_int64 * N)(*dims), (ctypes.c_int64 * N)(*ranks), _core_ptrs(cores),
                            ctypes.byref(v), _stream_handle(stream)), None, "tr_norm")
    return v.value
