"""Seeded synthetic workloads for tensor-ring (TR) decomposition.

Layout rule (the paper's single index rule, Sec. 2, linear index definition):
the first index is fastest.  A tensor of dims (I_1..I_N) is a Fortran-ordered
numpy array; a TR-core G_n of size R_n x I_n x R_{n+1} is a Fortran-ordered
array, so element (a, i, b) sits at flat offset a + R_n*(i + I_n*b).

Every random draw comes from ``numpy.random.SeedSequence([seed, cfg, purpose])``
with purpose 0 = true cores, 1 = noise, 2 = initial cores, 3 = field
parameters.  Nothing here runs an ALS step.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

PURPOSE_TRUE = 0
PURPOSE_NOISE = 1
PURPOSE_INIT = 2
PURPOSE_FIELD = 3

__all__ = [
    "PURPOSE_TRUE", "PURPOSE_NOISE", "PURPOSE_INIT", "PURPOSE_FIELD",
    "rng_for", "gaussian_cores", "conditioned_cores", "planted_tensor",
    "add_noise", "sinusoid_field", "Workload", "make_workload", "CONFIGS",
    "serving_stream", "to_flat",
]


def rng_for(seed: int, cfg: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(cfg), int(purpose)]))


def _ring(ranks):
    ranks = [int(r) for r in ranks]
    return ranks + [ranks[0]]


def gaussian_cores(dims, ranks, g: np.random.Generator):
    """i.i.d. N(0,1) cores of sizes R_n x I_n x R_{n+1} (Sec. 4 generator)."""
    rr = _ring(ranks)
    out = []
    for n, I in enumerate(dims):
        flat = g.standard_normal(rr[n] * int(I) * rr[n + 1])
        out.append(np.asfortranarray(flat.reshape((rr[n], int(I), rr[n + 1]), order="F")))
    return out


def conditioned_cores(dims, ranks, g: np.random.Generator, cond: float = 1e4):
    """Cores whose mode-2 unfolding G_(2) = U diag(s) V^T has a fixed condition
    number: U, V from QR of Gaussian matrices (signs fixed by diag(R) > 0) and s
    log-spaced on [1/cond, 1] over min(I, R_n R_{n+1}) values.
    Stand-in for the ill-conditioned cores of the stability experiments (Sec. 4.2)."""
    rr = _ring(ranks)
    out = []
    for n, I in enumerate(dims):
        I = int(I)
        C = rr[n] * rr[n + 1]
        k = min(I, C)
        U, ru = np.linalg.qr(g.standard_normal((I, k)))
        U = U * np.sign(np.diag(ru))
        V, rv = np.linalg.qr(g.standard_normal((C, k)))
        V = V * np.sign(np.diag(rv))
        s = np.logspace(0.0, -math.log10(cond), k)
        G2 = (U * s) @ V.T  # I x (R_n R_{n+1}), column a + R_n*b
        core = G2.reshape((I, rr[n], rr[n + 1]), order="F").transpose(1, 0, 2)
        out.append(np.asfortranarray(core))
    return out


def _half_chain(cores):
    """Merge consecutive cores into one 3-way array (R_first, prod I, R_last),
    first merged index fastest."""
    z = cores[0]
    for c in cores[1:]:
        ra, J, rb = z.shape
        _, I, rc = c.shape
        # z2[a, j, i, c] = sum_b z[a, j, b] c[b, i, c]
        z2 = np.tensordot(z, c, axes=([2], [0]))  # (ra, J, I, rc) in C-index order
        z = np.asfortranarray(z2.reshape((ra, J * I, rc), order="F"))
    return z


def planted_tensor(cores) -> np.ndarray:
    """Full tensor of a TR: X(i_1..i_N) = trace(G_1(i_1) ... G_N(i_N)) (Sec. 1).
    Built as trace(Left(p) Right(q)) with p over the first half of the modes and
    q over the rest, so the largest temporary is the result itself."""
    N = len(cores)
    dims = [c.shape[1] for c in cores]
    if N == 1:
        c = cores[0]
        return np.asfortranarray(np.einsum("aia->i", c))
    # split to balance prod of dims
    best, split = None, 1
    for m in range(1, N):
        p = math.prod(dims[:m])
        q = math.prod(dims[m:])
        v = max(p, q)
        if best is None or v < best:
            best, split = v, m
    L = _half_chain(cores[:split])   # (R_1, P, R_m)
    Rt = _half_chain(cores[split:])  # (R_m, Q, R_1)
    r1, P, rm = L.shape
    _, Q, _ = Rt.shape
    A = L.transpose(1, 0, 2).reshape((P, r1 * rm), order="F")    # A[p, a + r1*c] = L[a,p,c]
    B = Rt.transpose(2, 0, 1).reshape((r1 * rm, Q), order="F")   # B[a + r1*c, q] = Rt[c,q,a]
    X = A @ B
    return np.asfortranarray(X.reshape(tuple(dims), order="F"))


def add_noise(X_true: np.ndarray, eta: float, g: np.random.Generator) -> np.ndarray:
    """X = X_true + eta * (||X_true|| / ||N||) * N with N i.i.d. N(0,1) (Sec. 4)."""
    if eta == 0.0:
        return X_true
    Nz = g.standard_normal(X_true.size).reshape(X_true.shape, order="F")
    scale = eta * np.linalg.norm(X_true.ravel(order="K")) / np.linalg.norm(Nz.ravel(order="K"))
    return np.asfortranarray(X_true + scale * Nz)


def sinusoid_field(dims, g: np.random.Generator, nterms: int = 50, fmin=1.0, fmax=8.0):
    """Smooth low-rank field: sum_k (1/k) prod_d sin(2 pi f_kd (i_d)/I_d + phi_kd),
    f ~ U[fmin, fmax], phi ~ U[0, 2 pi).  Stand-in for the image/video tensors."""
    dims = [int(d) for d in dims]
    f = g.uniform(fmin, fmax, size=(nterms, len(dims)))
    ph = g.uniform(0.0, 2.0 * math.pi, size=(nterms, len(dims)))
    facs = []
    for d, I in enumerate(dims):
        i = np.arange(I, dtype=np.float64)
        facs.append(np.sin(2.0 * math.pi * f[:, d][None, :] * i[:, None] / I + ph[:, d][None, :]))  # I x K
    w = 1.0 / np.arange(1, nterms + 1, dtype=np.float64)
    # X_(1) = (F_1 diag(w)) KR^T with KR the row-wise products over modes 2..N
    # (rows ordered with i_2 fastest).
    kr = facs[1] if len(dims) > 1 else np.ones((1, nterms))
    for d in range(2, len(dims)):
        kr = (kr[:, None, :] * facs[d][None, :, :]).reshape(kr.shape[0] * dims[d], nterms, order="F")
    X = (facs[0] * w[None, :]) @ kr.T
    return np.asfortranarray(X.reshape(tuple(dims), order="F"))


def to_flat(a: np.ndarray) -> np.ndarray:
    """Column-major flat view (first index fastest)."""
    return np.ascontiguousarray(a.ravel(order="F"))


@dataclass
class Workload:
    name: str
    dims: tuple
    ranks: tuple            # fit ranks R_1..R_N
    X: np.ndarray           # stored values (Fortran order) in the storage dtype
    init_cores: list        # float64 Fortran cores
    sweeps: int
    dtype: str              # storage type of X: "f64" or "f32"
    eta: float
    true_cores: list = field(default_factory=list)
    note: str = ""

    @property
    def numel(self):
        return int(np.prod(self.dims))


# The five workloads: dims, true ranks / generator, noise, storage, fit ranks, sweeps.
CONFIGS = {
    1: dict(name="cfg1-20^4-R3-f64", dims=(20, 20, 20, 20), ranks=(3, 3, 3, 3), gen="gauss",
            eta=1e-3, dtype="f64", sweeps=10),
    2: dict(name="cfg2-100^4-R10-f32", dims=(100, 100, 100, 100), ranks=(10, 10, 10, 10), gen="gauss",
            eta=1e-2, dtype="f32", sweeps=20),
    3: dict(name="cfg3-40^5-R(6,8,10,8,6)-cond1e4-f32", dims=(40,) * 5, ranks=(6, 8, 10, 8, 6), gen="cond",
            eta=1e-2, dtype="f32", sweeps=20),
    4: dict(name="cfg4-512x512x256-R20-sinusoid-f32", dims=(512, 512, 256), ranks=(20, 20, 20), gen="sin",
            eta=2e-2, dtype="f32", sweeps=30),
}


def make_workload(cfg: int, seed: int = 0, dims=None, ranks=None, eta=None, dtype=None,
                  keep_true=False) -> Workload:
    """Build one workload from its recipe.  ``dims``/``ranks``/``eta``/``dtype``
    override the recipe (used for reduced-size parity cases with the same
    generator and value distribution)."""
    spec = dict(CONFIGS[cfg])
    dims = tuple(int(d) for d in (dims if dims is not None else spec["dims"]))
    ranks = tuple(int(r) for r in (ranks if ranks is not None else spec["ranks"]))
    eta = float(spec["eta"] if eta is None else eta)
    dtype = dtype or spec["dtype"]
    if len(ranks) != len(dims):
        raise ValueError("one rank per mode")
    true_cores = []
    if spec["gen"] == "gauss":
        true_cores = gaussian_cores(dims, ranks, rng_for(seed, cfg, PURPOSE_TRUE))
        Xt = planted_tensor(true_cores)
    elif spec["gen"] == "cond":
        true_cores = conditioned_cores(dims, ranks, rng_for(seed, cfg, PURPOSE_TRUE))
        Xt = planted_tensor(true_cores)
    elif spec["gen"] == "sin":
        Xt = sinusoid_field(dims, rng_for(seed, cfg, PURPOSE_FIELD))
    else:
        raise ValueError(spec["gen"])
    X = add_noise(Xt, eta, rng_for(seed, cfg, PURPOSE_NOISE))
    del Xt
    npdt = np.float64 if dtype == "f64" else np.float32
    X = np.asfortranarray(X.astype(npdt))
    init = gaussian_cores(dims, ranks, rng_for(seed, cfg, PURPOSE_INIT))
    return Workload(name=spec["name"], dims=dims, ranks=ranks, X=X, init_cores=init,
                    sweeps=int(spec["sweeps"]), dtype=dtype, eta=eta,
                    true_cores=true_cores if keep_true else [])


def serving_stream(njobs: int = 2000, rate_per_s: float = 200.0, seed: int = 0,
                   orders=(3, 4, 5), dim_range=(16, 128), rank_range=(2, 12)):
    """Job descriptors of the serving stream: Poisson arrivals (exponential
    inter-arrival times), order uniform in ``orders``, every mode size uniform in
    ``dim_range``, one TR rank per job uniform in ``rank_range``."""
    g = rng_for(seed, 5, PURPOSE_FIELD)
    t = np.cumsum(g.exponential(1.0 / rate_per_s, size=njobs))
    jobs = []
    for k in range(njobs):
        N = int(g.choice(orders))
        dims = tuple(int(v) for v in g.integers(dim_range[0], dim_range[1] + 1, size=N))
        R = int(g.integers(rank_range[0], rank_range[1] + 1))
        jobs.append(dict(id=k, t_arrive=float(t[k]), dims=dims, ranks=(R,) * N,
                         seed=int(g.integers(0, 2**62))))
    return jobs
