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
