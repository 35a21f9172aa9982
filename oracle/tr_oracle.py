"""Plain FP64 CPU oracle for tensor-ring ALS (arXiv 2210.11362).

TEST INFRASTRUCTURE ONLY -- see the package docstring.  No product code may
import or call this module.

Conventions (paper, Sec. 2 "Preliminaries"): indices are 0-based here, tensors
are Fortran-ordered numpy arrays so the first index is fastest, exactly as the
linear index definition of Sec. 2.  A TR-core G_n has shape (R_n, I_n, R_{n+1})
with R_{N+1} = R_1 (Sec. 1).  Modes ``n`` are 1-based in every public function
to match the paper's notation.

Parity status of each function (pins live in tests/test_oracle_pins.py):
  tr_entry, tr_full_bruteforce ... pinned: they ARE the trace definition (Sec. 1),
                                   cross-checked against an exact integer case
  unfold_mode, fold_mode,
  unfold_classical, unfold_n ..... pinned entry by entry against the index maps
                                   of their definitions (Sec. 2)
  subchain*, tr_full ............. pinned by brute-force trace evaluation
  regular_objective .............. pinned by the brute-force residual norm, the
                                   same for every mode, = rel_error * ||X||
  ttm, multi_ttm ................. pinned by Prop. 2.1 (Kronecker form) and loops
  subchain_product ............... pinned by Prop. 2.2 and by slice products
  gram_tensor, general_contract,
  coef_matrix_paper .............. pinned by Prop. 3.1 against explicit A^T A
  mttsp .......................... pinned by brute-force sums on tiny tensors
  als_update / tr_als ............ pinned by: lstsq on brute-force-built systems,
                                   fixed point at the true cores, planted
                                   noiseless recovery, monotone objective,
                                   N=2 Eckart-Young, R=1 rank-1 closed form
  tr_als_qr_literal (Alg. 3) ..... pinned by agreement with tr_als from the same
                                   start on well-conditioned data
  tr_als_ne_literal (Alg. 2) ..... same
  tr_als_qrne_literal (Alg. 4) ... same, and its R-core Grams against the
                                   cores' Grams (Q_j has orthonormal columns)
  tr_inner ....................... pinned by brute-force <A,B> (corrected reading
                                   of the by-product proposition, Sec. 3.4)
  cheap_fit_terms ................ pinned by the explicit error (Sec. 4 identities)
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.linalg as sla

__all__ = [
    "ring_ranks", "tr_entry", "tr_full_bruteforce", "unfold_classical", "unfold_mode",
    "fold_mode", "unfold_n", "core_unfold2", "core_fold2", "subchain_product", "subchain",
    "subchain_slices_bruteforce", "subchain_unfold2", "tr_full", "mttsp", "gram_tensor",
    "general_contract", "coef_matrix_paper", "coef_matrix_explicit", "solve_ls",
    "als_update", "tr_als", "rel_error", "mode2_qr", "ttm", "multi_ttm",
    "tr_als_qr_literal", "tr_als_ne_literal", "tr_als_qrne_literal", "tr_inner", "cheap_fit_terms",
    "regular_objective",
]


# ----------------------------------------------------------------------------
# Sec. 1: the TR format
# ----------------------------------------------------------------------------
def ring_ranks(cores):
    """[R_1, ..., R_N, R_{N+1}=R_1] read from the core shapes."""
    r = [c.shape[0] for c in cores]
    return r + [r[0]]


def tr_entry(cores, idx):
    """X(i_1..i_N) = Trace(G_1(i_1) G_2(i_2) ... G_N(i_N)) (Sec. 1).  ``idx`` is
    0-based.  Works on float or object (exact integer/Fraction) cores."""
    prod = None
    for G, i in zip(cores, idx):
        S = G[:, i, :]
        prod = S if prod is None else prod.dot(S)
    return sum(prod[a, a] for a in range(prod.shape[0]))


def tr_full_bruteforce(cores):
    """Full tensor by evaluating the trace formula entry by entry (tiny only)."""
    dims = [c.shape[1] for c in cores]
    X = np.zeros(dims, dtype=np.float64, order="F")
    for idx in itertools.product(*[range(d) for d in dims]):
        X[idx] = tr_entry(cores, idx)
    return X


# ----------------------------------------------------------------------------
# Sec. 2: unfoldings
# ----------------------------------------------------------------------------
def unfold_classical(X, n):
    """X_(n): I_n x prod_{j!=n} I_j, columns (i_1..i_{n-1}, i_{n+1}..i_N) with the
    first fastest (Definition "Classical Mode-n Unfolding")."""
    N = X.ndim
    order = [n - 1] + [j for j in range(N) if j != n - 1]
    return np.asfortranarray(np.transpose(X, order).reshape((X.shape[n - 1], -1), order="F"))


def _cyclic_order(N, n):
    """Axes (n, n+1, ..., N, 1, ..., n-1), 0-based."""
    return [(n - 1 + k) % N for k in range(N)]


def unfold_mode(X, n):
    """X_[n]: I_n x prod_{j!=n} I_j, columns (i_{n+1}..i_N, i_1..i_{n-1}) with
    i_{n+1} fastest (Definition "Mode-n Unfolding")."""
    return np.asfortranarray(np.transpose(X, _cyclic_order(X.ndim, n)).reshape((X.shape[n - 1], -1), order="F"))


def fold_mode(Xn, n, dims):
    """Inverse of unfold_mode."""
    N = len(dims)
    order = _cyclic_order(N, n)
    T = Xn.reshape([dims[k] for k in order], order="F")
    inv = np.argsort(order)
    return np.asfortranarray(np.transpose(T, inv))


def unfold_n(X, n):
    """X_<n>: rows (i_1..i_n), columns (i_{n+1}..i_N), first fastest
    (Definition "n-Unfolding")."""
    rows = int(np.prod(X.shape[:n]))
    return X.reshape((rows, -1), order="F")


def core_unfold2(G):
    """Classical mode-2 unfolding of a core: G_(2)[i, a + R_n*b] = G[a, i, b]."""
    Rn, I, Rn1 = G.shape
    return np.asfortranarray(np.transpose(G, (1, 0, 2)).reshape((I, Rn * Rn1), order="F"))


def core_fold2(Z, Rn, Rn1):
    """Inverse of core_unfold2."""
    I = Z.shape[0]
    return np.asfortranarray(np.transpose(Z.reshape((I, Rn, Rn1), order="F"), (1, 0, 2)))


# ----------------------------------------------------------------------------
# Sec. 2: subchain product and subchain tensor
# ----------------------------------------------------------------------------
def subchain_product(A, B):
    """Mode-2 subchain product (Definition "Subchain Product"): for A (I1 x J1 x K)
    and B (K x J2 x I2), C(:, j1 + J1*j2, :) = A(:, j1, :) B(:, j2, :)."""
    I1, J1, K = A.shape
    K2, J2, I2 = B.shape
    if K != K2:
        raise ValueError("subchain product: bond mismatch")
    # T[a, j1, j2, c] = sum_k A[a, j1, k] B[k, j2, c]
    T = np.tensordot(A, B, axes=([2], [0]))
    return np.asfortranarray(T.reshape((I1, J1 * J2, I2), order="F"))


def _chain_order(N, n):
    """Core order of the subchain for mode n: n+1, ..., N, 1, ..., n-1 (1-based)."""
    return [((n - 1 + k) % N) + 1 for k in range(1, N)]


def subchain(cores, n):
    """G^{!=n} = G_{n+1} [x]_2 ... [x]_2 G_N [x]_2 G_1 [x]_2 ... [x]_2 G_{n-1}
    (Definition "subchain tensor" and its subchain-product form, Sec. 2).
    Shape R_{n+1} x prod_{j!=n} I_j x R_n."""
    N = len(cores)
    order = _chain_order(N, n)
    Z = cores[order[0] - 1]
    for k in order[1:]:
        Z = subchain_product(Z, cores[k - 1])
    return Z


def subchain_slices_bruteforce(cores, n):
    """G^{!=n}(j) = prod_{j=n+1}^{N} G_j(i_j) prod_{j=1}^{n-1} G_j(i_j), one slice at
    a time, j running over (i_{n+1}..i_N, i_1..i_{n-1}) with i_{n+1} fastest."""
    N = len(cores)
    order = _chain_order(N, n)
    dims = [cores[k - 1].shape[1] for k in order]
    rr = ring_ranks(cores)
    J = int(np.prod(dims))
    out = np.zeros((rr[n % N], J, rr[n - 1]), order="F")
    for j in range(J):
        rem, idx = j, []
        for d in dims:
            idx.append(rem % d)
            rem //= d
        P = np.eye(rr[order[0] - 1])
        for k, i in zip(order, idx):
            P = P @ cores[k - 1][:, i, :]
        out[:, j, :] = P
    return out


def subchain_unfold2(cores, n):
    """G^{!=n}_[2]: J_n x R_n R_{n+1} with A[j, a + R_n*b] = G^{!=n}[b, j, a]
    (mode-2 unfolding of the 3rd-order subchain, columns (a, b) with a fastest,
    the same column order as G_n(2); Sec. 2, the LS form of the subproblem)."""
    Z = subchain(cores, n)
    Rb, J, Ra = Z.shape
    return np.asfortranarray(np.transpose(Z, (1, 2, 0)).reshape((J, Ra * Rb), order="F"))


def tr_full(cores):
    """Full tensor via X_[1] = G_1(2) (G^{!=1}_[2])^T (the LS form of the
    subproblem in Sec. 2)."""
    dims = [c.shape[1] for c in cores]
    if len(cores) == 1:
        return np.asfortranarray(np.einsum("aia->i", cores[0]))
    X1 = core_unfold2(cores[0]) @ subchain_unfold2(cores, 1).T
    return fold_mode(X1, 1, dims)


# ----------------------------------------------------------------------------
# Sec. 3.1: MTTSP, Gram tensors, general contracted product, coefficient matrix
# ----------------------------------------------------------------------------
def mttsp(X, cores, n):
    """M_n = X_[n] G^{!=n}_[2] (Alg. 2, the MTTSP step)."""
    return unfold_mode(X, n) @ subchain_unfold2(cores, n)


def gram_tensor(G, Z=None):
    """P = sum_i G(i)^T o Z(i)^T, P(p, q, r, s) = sum_i G[q, i, p] Z[s, i, r]
    (Alg. 2, Gram tensor step; Z = G for the ALS Gram)."""
    if Z is None:
        Z = G
    return np.einsum("qip,sir->pqrs", G, Z, optimize=True)


def general_contract(A, B):
    """(A x_{2,4}^{1,3} B)(i1, i2, r1, r2) = sum_{j,k} A(i1, j, r1, k) B(j, i2, k, r2)
    (Remark after Prop. 3.1)."""
    return np.einsum("ijrk,jlks->ilrs", A, B, optimize=True)


def _unfold2_4way(T):
    """T_<2> of a 4th-order tensor: rows (i1, i2), columns (i3, i4), first fastest."""
    a, b, c, d = T.shape
    return T.reshape((a * b, c * d), order="F")


def coef_matrix_paper(cores, n, grams=None):
    """S_n<2> with S_n = P_{n-1} x P_{n-2} x ... x P_1 x P_N x ... x P_{n+1}
    (general contracted products), the structured coefficient matrix of Prop. 3.1
    as used in Alg. 2."""
    N = len(cores)
    if grams is None:
        grams = [gram_tensor(G) for G in cores]
    seq = [((n - 2 - k) % N) + 1 for k in range(N - 1)]  # n-1, n-2, ..., 1, N, ..., n+1
    S = grams[seq[0] - 1]
    for k in seq[1:]:
        S = general_contract(S, grams[k - 1])
    return _unfold2_4way(S)


def coef_matrix_explicit(cores, n):
    """(G^{!=n}_[2])^T G^{!=n}_[2] from the exploded subchain."""
    A = subchain_unfold2(cores, n)
    return A.T @ A


# ----------------------------------------------------------------------------
# Alg. 1: regular TR-ALS
# ----------------------------------------------------------------------------
def solve_ls(A, B, mode="qr"):
    """argmin_Z ||A Z - B||_F.
    qr    : Householder QR of A (LAPACK), Z = R^{-1} Q^T B;
    ne    : Cholesky of A^T A on the normal equations;
    lstsq : SVD-based minimum-norm solution."""
    if mode == "qr":
        Q, R = np.linalg.qr(A, mode="reduced")
        d = np.abs(np.diag(R))
        if d.size and d.min() <= A.shape[0] * np.finfo(float).eps * d.max():
            return np.linalg.lstsq(A, B, rcond=None)[0]
        return sla.solve_triangular(R, Q.T @ B, lower=False)
    if mode == "ne":
        c = sla.cho_factor(A.T @ A, lower=True)
        return sla.cho_solve(c, A.T @ B)
    if mode == "lstsq":
        return np.linalg.lstsq(A, B, rcond=None)[0]
    raise ValueError(mode)


def regular_objective(X, cores, n):
    """||X_[n] - G_n(2) (G^{!=n}_[2])^T||_F = ||X - TR(G)||_F."""
    A = subchain_unfold2(cores, n)
    return float(np.linalg.norm(unfold_mode(X, n) - core_unfold2(cores[n - 1]) @ A.T))


def als_update(X, cores, n, solve="qr", objective=False):
    """One mode update of Alg. 1: build G^{!=n}_[2] explicitly, solve
    min ||G^{!=n}_[2] G_n(2)^T - X_[n]^T||_F, write the core back.
    Returns (new core, objective or None).  ``cores`` is not modified."""
    rr = ring_ranks(cores)
    A = subchain_unfold2(cores, n)
    B = unfold_mode(X, n).T
    Zt = solve_ls(A, B, solve)              # (R_n R_{n+1}) x I_n
    Gn = core_fold2(np.asfortranarray(Zt.T), rr[n - 1], rr[n])
    obj = None
    if objective:
        obj = float(np.linalg.norm(A @ Zt - B))
    return Gn, obj


def tr_als(X, cores0, sweeps, solve="qr", record_objective=False, callback=None):
    """Regular TR-ALS (Alg. 1): Gauss-Seidel over n = 1..N, a fixed number of
    sweeps (Sec. 4 termination).  Returns (cores, objectives) where
    objectives[s*N + n-1] is the explicit objective after that update."""
    X = np.asarray(X, dtype=np.float64)
    cores = [np.asfortranarray(np.array(c, dtype=np.float64)) for c in cores0]
    N = len(cores)
    objs = []
    for s in range(sweeps):
        for n in range(1, N + 1):
            cores[n - 1], o = als_update(X, cores, n, solve, record_objective)
            if record_objective:
                objs.append(o)
        if callback is not None:
            callback(s, cores)
    return cores, objs


def rel_error(X, cores):
    """||X - TR(G)||_F / ||X||_F with an explicit reconstruction (Sec. 4)."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.linalg.norm(X - tr_full(cores)) / np.linalg.norm(X))


# ----------------------------------------------------------------------------
# Sec. 3.2: mode-2 QR of a core, TTM, Multi-TTM, Alg. 3 (TR-ALS-QR)
# ----------------------------------------------------------------------------
def mode2_qr(G):
    """Mode-2 QR of a 3rd-order core (Definition "Mode-n QR Factorization"):
    G = R x_2 Q with G_(2) = Q R_(2).  Q is I x min(I, R_n R_{n+1}) with
    orthonormal columns; R has shape (R_n, min(I, R_n R_{n+1}), R_{n+1}) and its
    mode-2 unfolding is upper triangular (square) or upper trapezoidal."""
    Rn, I, Rn1 = G.shape
    Q, R2 = np.linalg.qr(core_unfold2(G), mode="reduced")
    return np.asfortranarray(Q), core_fold2(np.asfortranarray(R2), Rn, Rn1)


def ttm(X, U, n):
    """(X x_n U)(.., j, ..) = sum_{i_n} X(.., i_n, ..) U(j, i_n) (Definition TTM)."""
    T = np.tensordot(U, X, axes=([1], [n - 1]))     # new axis first
    order = list(range(1, n)) + [0] + list(range(n, X.ndim))
    return np.asfortranarray(np.transpose(T, order))


def multi_ttm(X, Us, skip=None):
    """X x_1 U_1 ... x_N U_N, skipping mode ``skip`` (Multi-TTM, Sec. 2)."""
    Y = X
    for k, U in enumerate(Us, start=1):
        if k == skip or U is None:
            continue
        Y = ttm(Y, U, k)
    return Y


def tr_als_qr_literal(X, cores0, sweeps):
    """TR-ALS-QR (Alg. 3) written out: core QRs, V_n = subchain of the R-cores,
    QR of V_n[2] = Q_0 R_[2] (the unfolding whose columns match G_n(2)),
    Y = X x_{j!=n} Q_j^T, W_n = Y_[n] Q_0, solve G_n(2) R_[2]^T = W_n,
    re-factor the updated core."""
    X = np.asarray(X, dtype=np.float64)
    cores = [np.asfortranarray(np.array(c, dtype=np.float64)) for c in cores0]
    N = len(cores)
    rr = ring_ranks(cores)
    qrs = [mode2_qr(G) for G in cores]
    for _ in range(sweeps):
        for n in range(1, N + 1):
            Rcores = [q[1] for q in qrs]
            V2 = subchain_unfold2(Rcores, n)                 # V_n[2]
            Q0, R = np.linalg.qr(V2, mode="reduced")
            Y = multi_ttm(X, [q[0].T for q in qrs], skip=n)
            W = unfold_mode(Y, n) @ Q0
            Gt = sla.solve_triangular(R, W.T, lower=False)   # R G^T = W^T
            cores[n - 1] = core_fold2(np.asfortranarray(Gt.T), rr[n - 1], rr[n])
            qrs[n - 1] = mode2_qr(cores[n - 1])
    return cores


def tr_als_ne_literal(X, cores0, sweeps):
    """TR-ALS-NE (Alg. 2) written out: Gram tensors P_j, S_n by general
    contractions, explicit subchain, MTTSP, Cholesky solve of
    G_n(2) S_n<2> = M_n, Gram refresh."""
    X = np.asarray(X, dtype=np.float64)
    cores = [np.asfortranarray(np.array(c, dtype=np.float64)) for c in cores0]
    N = len(cores)
    rr = ring_ranks(cores)
    grams = [gram_tensor(G) for G in cores]
    for _ in range(sweeps):
        for n in range(1, N + 1):
            S = coef_matrix_paper(cores, n, grams)
            M = mttsp(X, cores, n)
            c = sla.cho_factor(S, lower=True)
            Gt = sla.cho_solve(c, M.T)                       # S G^T = M^T (S symmetric)
            cores[n - 1] = core_fold2(np.asfortranarray(Gt.T), rr[n - 1], rr[n])
            grams[n - 1] = gram_tensor(cores[n - 1])
    return cores


def tr_als_qrne_literal(X, cores0, sweeps):
    """TR-ALS-QRNE (Alg. 4, Sec. 3.3) written out: mode-2 QRs of the cores,
    Gram tensors of the R-cores, and per mode: S_n from the R-core Grams (Prop.
    3.1 applied to the R-cores), V_n = subchain of the R-cores,
    Y = X x_{j!=n} Q_j^T, M_n = Y_[n] V_n[2], Cholesky solve of
    G_n(2) S_n<2> = M_n, re-factor the updated core and refresh its R-core
    Gram."""
    X = np.asarray(X, dtype=np.float64)
    cores = [np.asfortranarray(np.array(c, dtype=np.float64)) for c in cores0]
    N = len(cores)
    rr = ring_ranks(cores)
    qrs = [mode2_qr(G) for G in cores]
    grams = [gram_tensor(q[1]) for q in qrs]
    for _ in range(sweeps):
        for n in range(1, N + 1):
            Rcores = [q[1] for q in qrs]
            S = coef_matrix_paper(Rcores, n, grams)
            V2 = subchain_unfold2(Rcores, n)                 # V_n[2]
            Y = multi_ttm(X, [q[0].T for q in qrs], skip=n)
            M = unfold_mode(Y, n) @ V2
            c = sla.cho_factor(S, lower=True)
            Gt = sla.cho_solve(c, M.T)                       # S G^T = M^T
            cores[n - 1] = core_fold2(np.asfortranarray(Gt.T), rr[n - 1], rr[n])
            qrs[n - 1] = mode2_qr(cores[n - 1])
            grams[n - 1] = gram_tensor(qrs[n - 1][1])
    return cores


# ----------------------------------------------------------------------------
# Sec. 3.4 by-product (corrected reading) and Sec. 4 cheap-error identities
# ----------------------------------------------------------------------------
def tr_inner(coresA, coresB):
    """<A, B> for two TRs of the same dims.  With P_n = sum_i G_n(i)^T o Z_n(i)^T
    and T = P_N x P_{N-1} x ... x P_1, T(x, y, x', y') collects
    (G_1..G_N)^T(x, y) (Z_1..Z_N)^T(x', y') summed over all indices, so
    <A, B> = sum_{x, x'} T(x, x, x', x') (the pair-space trace; the printed
    statement takes Trace(T_<2>), which is a different quantity)."""
    N = len(coresA)
    Ps = [gram_tensor(G, Z) for G, Z in zip(coresA, coresB)]
    T = Ps[N - 1]
    for k in range(N - 2, -1, -1):
        T = general_contract(T, Ps[k])
    return float(np.einsum("xxyy->", T))


def cheap_fit_terms(X, cores):
    """The Sec. 4 identities for the last mode N: <X, Xhat> = <M_N, G_N(2)> and
    ||Xhat||^2 = <S_N<2>, (P_N^T)<2>> with P_N^T = permute(P_N, [2,1,4,3]).
    Returns (<X,Xhat>, ||Xhat||^2) computed that way."""
    N = len(cores)
    M = mttsp(X, cores, N)
    GN = core_unfold2(cores[N - 1])
    ip = float(np.sum(M * GN))
    S = coef_matrix_paper(cores, N)
    PT = np.transpose(gram_tensor(cores[N - 1]), (1, 0, 3, 2))
    nrm2 = float(np.sum(S * _unfold2_4way(PT)))
    return ip, nrm2
