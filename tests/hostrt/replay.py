"""Host-side replay of the library on the CPU stand-in of the HIP runtime.

``build_host_lib`` links the library's hipcc objects against
``stand_in_hip.cpp``; the functions below drive the C ABI the way the GPU
tests and the serving stream do (same shapes, same calls, buffers from the
stand-in's allocator), so every launch, copy, capture and thread of the host
code is checked without a GPU.  Kernels do not run, so no numbers are checked
here: the GPU tests do that.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2210_11362_amd", "csrc")
OBJ = os.path.join(ROOT, "_build")
OUT = os.path.join(ROOT, "_build", "host")
CLANG = "/opt/rocm/llvm/bin/clang++"


def _stale(objdir: str) -> bool:
    srcs = [f for f in os.listdir(CSRC) if f.endswith(".hip")]
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hdrs.append(os.path.join(ROOT, "include", "tr_als.h"))
    newest_hdr = max(os.path.getmtime(h) for h in hdrs)
    for f in srcs:
        o = os.path.join(objdir, f[:-4] + ".o")
        if not os.path.exists(o):
            return True
        if os.path.getmtime(o) < max(os.path.getmtime(os.path.join(CSRC, f)), newest_hdr):
            return True
    return False


def build_host_lib() -> str:
    """Library objects (rebuilt by the package build when stale) + stand-in runtime."""
    if _stale(OBJ):
        from paper_2210_11362_amd.build import build
        build()
    os.makedirs(OUT, exist_ok=True)
    so = os.path.join(OUT, "libtrals_host.so")
    stub = os.path.join(OUT, "stand_in_hip.o")
    src = os.path.join(HERE, "stand_in_hip.cpp")
    subprocess.run([CLANG, "-std=c++17", "-O1", "-g", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-w", "-c", src, "-o", stub], check=True)
    objs = sorted(os.path.join(OBJ, f) for f in os.listdir(OBJ) if f.endswith(".o"))
    subprocess.run(["g++", "-shared", "-o", so + ".tmp", *objs, stub, "-lpthread"], check=True)
    os.replace(so + ".tmp", so)
    return so


class Host:
    """The host library with the C-ABI signatures of the package's loader."""

    def __init__(self, path: str):
        from paper_2210_11362_amd import _lib as C
        self.C = C
        L = ctypes.CDLL(path)
        for name, (res, args) in C._SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        L.fakehip_violation.restype = ctypes.c_char_p
        L.fakehip_launches.restype = ctypes.c_long
        L.fakehip_launches.argtypes = [ctypes.c_char_p]
        L.fakehip_device_alloc.restype = ctypes.c_void_p
        L.fakehip_device_alloc.argtypes = [ctypes.c_size_t]
        L.fakehip_device_free.argtypes = [ctypes.c_void_p]
        L.fakehip_gemm_log.argtypes = [ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]
        self.L = L

    def violations(self):
        return [self.L.fakehip_violation(k).decode() for k in range(self.L.fakehip_violation_count())]

    def reset(self):
        self.L.fakehip_reset()

    def alloc(self, nbytes: int) -> int:
        p = self.L.fakehip_device_alloc(max(int(nbytes), 1))
        assert p, "stand-in allocation failed"
        return p

    def free(self, p):
        self.L.fakehip_device_free(p)

    def gemm_log(self):
        n = self.L.fakehip_gemm_log(None, 0)
        buf = (ctypes.c_longlong * (4 * max(n, 1)))()
        self.L.fakehip_gemm_log(buf, n)
        return [tuple(buf[4 * k:4 * k + 4]) for k in range(n)]


def core_elems(dims, ranks, k):
    N = len(dims)
    return ranks[k] * dims[k] * ranks[(k + 1) % N]


def run_context(h: Host, dims, ranks, variant="ne", precs=("f64",), xdt="f64", sweeps=2, steps=True):
    """One context through the calls the parity tests make: init, sweeps in
    each precision, the per-step entry points, the fit, destroy.  Returns the
    status codes of the calls."""
    C = h.C
    N = len(dims)
    numel = int(np.prod(dims))
    es = 8 if xdt == "f64" else 4
    X = h.alloc(numel * es)
    cores = [h.alloc(core_elems(dims, ranks, k) * 8) for k in range(N)]
    d = (ctypes.c_int64 * N)(*dims)
    r = (ctypes.c_int64 * N)(*ranks)
    cp = (ctypes.c_void_p * N)(*cores)
    ctx = ctypes.c_void_p()
    codes = []
    rc = h.L.tr_als_init(ctypes.byref(ctx), N, d, r, ctypes.c_void_p(X), C.PREC[xdt], cp, C.VARIANT[variant], None)
    codes.append(("init", rc))
    if rc == 0:
        for p in precs:
            codes.append((f"sweep {p}", h.L.tr_als_sweep(ctx, sweeps, C.PREC[p], 1)))
        if steps:
            rr = max(ranks[k] * ranks[(k + 1) % N] for k in range(N))
            out = h.alloc(max(dims) * rr * 8 + rr * rr * 8)
            for n in range(1, N + 1):
                for p in precs:
                    codes.append((f"mttsp {n} {p}", h.L.tr_als_mttsp(ctx, n, C.PREC[p], ctypes.c_void_p(out))))
                codes.append((f"coef {n}", h.L.tr_als_coef(ctx, n, ctypes.c_void_p(out))))
                codes.append((f"gram {n}", h.L.tr_als_gram(ctx, n, ctypes.c_void_p(out))))
                codes.append((f"update {n}", h.L.tr_als_update_mode(ctx, n, C.PREC[precs[0]], 1)))
            h.free(out)
        f = ctypes.c_double()
        codes.append(("fit", h.L.tr_als_fit(ctx, ctypes.byref(f))))
        h.L.tr_als_destroy(ctx)
    for p in cores + [X]:
        h.free(p)
    return codes


def job_desc(C, dims, ranks, seed=0, prec_mixed="bf16", nsweeps_mixed=4, prec_fin="f32", nsweeps_fin=2,
             t_arrival=0.0, eta=0.01, x_dtype="f32", variant="ne", X=None, init=None):
    d = C.JobDesc()
    d.N = len(dims)
    for k in range(d.N):
        d.dims[k] = int(dims[k])
        d.ranks[k] = int(ranks[k])
    d.variant = C.VARIANT[variant]
    d.prec_mixed, d.nsweeps_mixed = C.PREC[prec_mixed], int(nsweeps_mixed)
    d.prec_fin, d.nsweeps_fin = C.PREC[prec_fin], int(nsweeps_fin)
    d.refine = 1
    d.seed = int(seed)
    d.eta = float(eta)
    d.x_dtype = C.PREC[x_dtype]
    d.t_arrival = float(t_arrival)
    if X is not None:
        d.X = ctypes.c_void_p(X)
    keep = None
    if init is not None:
        keep = (ctypes.c_void_p * d.N)(*init)
        d.init_cores = ctypes.cast(keep, ctypes.POINTER(ctypes.c_void_p))
    return d, keep


class Server:
    """A server on the stand-in.  Between creation and destruction only the
    executor thread may call into the runtime: ``threads`` is the number of
    distinct threads that did."""

    def __init__(self, h: Host, budget: int, slots: int, batch: bool = False):
        self.h = h
        self.s = ctypes.c_void_p()
        rc = h.L.tr_srv_create(ctypes.byref(self.s), ctypes.c_size_t(budget), slots, h.C.TR_SRV_BATCH if batch else 0)
        assert rc == 0, rc
        h.L.fakehip_window_begin()
        self.keep = []
        self.threads = None

    def submit(self, dims, ranks, **kw):
        d, keep = job_desc(self.h.C, dims, ranks, **kw)
        self.keep.append(keep)
        jid = ctypes.c_uint64()
        rc = self.h.L.tr_srv_submit(self.s, ctypes.byref(d), ctypes.byref(jid))
        return rc, jid.value

    def wait(self, jid):
        info = self.h.C.JobInfo()
        assert self.h.L.tr_srv_wait(self.s, ctypes.c_uint64(jid), ctypes.byref(info)) == 0
        return info

    def poll(self, jid):
        info = self.h.C.JobInfo()
        assert self.h.L.tr_srv_poll(self.s, ctypes.c_uint64(jid), ctypes.byref(info)) == 0
        return info

    def result(self, jid, dims, ranks):
        N = len(dims)
        outs = [np.zeros(core_elems(dims, ranks, k)) for k in range(N)]
        arr = (ctypes.c_void_p * N)(*[o.ctypes.data for o in outs])
        assert self.h.L.tr_srv_result(self.s, ctypes.c_uint64(jid), arr) == 0
        return outs

    def drain(self):
        assert self.h.L.tr_srv_drain(self.s) == 0

    def stats(self):
        st = self.h.C.SrvStats()
        assert self.h.L.tr_srv_stats_read(self.s, ctypes.byref(st)) == 0
        return {k: getattr(st, k) for k, _ in self.h.C.SrvStats._fields_}

    def error(self, jid):
        return self.h.L.tr_srv_job_error(self.s, ctypes.c_uint64(jid)).decode()

    def close(self):
        if self.s:
            self.threads = self.h.L.fakehip_window_end()
            self.h.L.tr_srv_destroy(self.s)
            self.s = None
        return self.threads


def serving_stream(njobs: int, seed: int = 7, rate: float = 200.0, orders=(3, 4, 5), dmin=16, dmax=128, rmin=2,
                   rmax=12):
    """Poisson arrivals; order, mode sizes and one rank per job drawn uniformly."""
    g = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for k in range(njobs):
        t += g.exponential(1.0 / rate)
        N = int(g.choice(orders))
        dims = tuple(int(v) for v in g.integers(dmin, dmax + 1, size=N))
        R = int(g.integers(rmin, rmax + 1))
        jobs.append(dict(dims=dims, ranks=(R,) * N, seed=1000 + k, t_arrival=t))
    return jobs
