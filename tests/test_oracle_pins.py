"""Pins of the CPU oracle against facts fixed outside it: hand-worked examples,
brute-force definitions, the paper's propositions on random operands, closed
forms and textbook reductions.  CPU only."""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def rand_cores(dims, ranks, seed):
    g = np.random.default_rng(seed)
    return W.gaussian_cores(dims, ranks, g)


# ---------------------------------------------------------------------------
# The trace definition (Sec. 1) on hand-worked examples
# ---------------------------------------------------------------------------
def test_trace_hand_example_n2():
    # G_1 (1 x 2 x 2): slices [1 2], [3 4];  G_2 (2 x 3 x 1): [1;0], [0;1], [1;-1]
    G1 = np.zeros((1, 2, 2), order="F")
    G1[0, 0, :] = [1, 2]
    G1[0, 1, :] = [3, 4]
    G2 = np.zeros((2, 3, 1), order="F")
    G2[:, 0, 0] = [1, 0]
    G2[:, 1, 0] = [0, 1]
    G2[:, 2, 0] = [1, -1]
    expect = np.array([[1.0, 2.0, -1.0], [3.0, 4.0, -1.0]])   # worked by hand
    np.testing.assert_array_equal(O.tr_full_bruteforce([G1, G2]), expect)
    np.testing.assert_array_equal(O.tr_full([G1, G2]), expect)


def test_trace_hand_example_ring3():
    # A=[[1,1],[0,1]], B=diag(2,1), C_0=I, C_1=[[0,1],[1,0]]:
    # trace(ABC_0) = trace([[2,1],[0,1]]) = 3, trace(ABC_1) = trace([[1,2],[1,0]]) = 1
    G1 = np.array([[1.0, 1.0], [0.0, 1.0]]).reshape(2, 1, 2)
    G2 = np.array([[2.0, 0.0], [0.0, 1.0]]).reshape(2, 1, 2)
    G3 = np.zeros((2, 2, 2))
    G3[:, 0, :] = np.eye(2)
    G3[:, 1, :] = [[0, 1], [1, 0]]
    cores = [np.asfortranarray(c) for c in (G1, G2, G3)]
    X = O.tr_full(cores)
    assert X.shape == (1, 1, 2)
    assert X[0, 0, 0] == pytest.approx(3.0, abs=1e-15)
    assert X[0, 0, 1] == pytest.approx(1.0, abs=1e-15)


def test_trace_exact_integer_cores():
    """Integer cores: the float reconstruction is exact (all partial sums are small
    integers), so it must equal the exact-integer trace bit for bit."""
    g = np.random.default_rng(7)
    dims, ranks = (3, 2, 4, 2), (2, 3, 1, 2)
    rr = list(ranks) + [ranks[0]]
    cores_i = [g.integers(-3, 4, size=(rr[n], dims[n], rr[n + 1])).astype(object) for n in range(4)]
    cores_f = [np.asfortranarray(c.astype(np.float64)) for c in cores_i]
    Xf = O.tr_full(cores_f)
    for idx in itertools.product(*[range(d) for d in dims]):
        assert Xf[idx] == float(O.tr_entry(cores_i, idx))


def test_generator_planted_tensor_matches_trace():
    cores = rand_cores((3, 4, 2, 3), (2, 3, 2, 4), 1)
    np.testing.assert_allclose(W.planted_tensor(cores), O.tr_full_bruteforce(cores), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# Unfoldings and the subchain (Sec. 2)
# ---------------------------------------------------------------------------
DIMS, RANKS = (3, 4, 2, 3), (2, 3, 2, 4)


def _col_mode(idx, dims, n):
    """Column of X_[n] by the definition: indices i_{n+1}..i_N, i_1..i_{n-1},
    first fastest."""
    N = len(dims)
    order = [(n - 1 + k) % N for k in range(1, N)]
    col, stride = 0, 1
    for k in order:
        col += idx[k] * stride
        stride *= dims[k]
    return col


def test_unfold_mode_by_definition():
    g = np.random.default_rng(2)
    X = np.asfortranarray(g.standard_normal(DIMS))
    for n in range(1, 5):
        Xn = O.unfold_mode(X, n)
        for idx in itertools.product(*[range(d) for d in DIMS]):
            assert Xn[idx[n - 1], _col_mode(idx, DIMS, n)] == X[idx]
        np.testing.assert_array_equal(O.fold_mode(Xn, n, DIMS), X)


def _col_classical(idx, dims, n):
    """Column of X_(n) by the definition: indices i_1..i_{n-1}, i_{n+1}..i_N,
    first fastest."""
    col, stride = 0, 1
    for k in range(len(dims)):
        if k == n - 1:
            continue
        col += idx[k] * stride
        stride *= dims[k]
    return col


def test_unfold_classical_by_definition():
    """Classical mode-n unfolding (Sec. 2, its definition) entry by entry."""
    g = np.random.default_rng(21)
    X = np.asfortranarray(g.standard_normal(DIMS))
    for n in range(1, 5):
        Xc = O.unfold_classical(X, n)
        assert Xc.shape == (DIMS[n - 1], int(np.prod(DIMS)) // DIMS[n - 1])
        for idx in itertools.product(*[range(d) for d in DIMS]):
            assert Xc[idx[n - 1], _col_classical(idx, DIMS, n)] == X[idx]
    # mode 1 and mode N: the classical and the cyclic unfoldings coincide
    np.testing.assert_array_equal(O.unfold_classical(X, 1), O.unfold_mode(X, 1))
    # for n = N the cyclic order (i_1..i_{N-1}) is also the classical one
    np.testing.assert_array_equal(O.unfold_classical(X, 4), O.unfold_mode(X, 4))


def test_unfold_n_by_definition():
    """n-unfolding (Sec. 2, its definition): rows (i_1..i_n), columns
    (i_{n+1}..i_N), first index fastest on both sides."""
    g = np.random.default_rng(22)
    X = np.asfortranarray(g.standard_normal(DIMS))
    for n in range(1, 4):
        Xu = O.unfold_n(X, n)
        assert Xu.shape == (int(np.prod(DIMS[:n])), int(np.prod(DIMS[n:])))
        for idx in itertools.product(*[range(d) for d in DIMS]):
            row = sum(idx[k] * int(np.prod(DIMS[:k])) for k in range(n))
            col = sum(idx[k] * int(np.prod(DIMS[n:k])) for k in range(n, 4))
            assert Xu[row, col] == X[idx]


def test_reconstruction_every_mode():
    cores = rand_cores(DIMS, RANKS, 3)
    Xb = O.tr_full_bruteforce(cores)
    for n in range(1, 5):
        Xn = O.core_unfold2(cores[n - 1]) @ O.subchain_unfold2(cores, n).T
        np.testing.assert_allclose(O.fold_mode(Xn, n, DIMS), Xb, rtol=1e-13, atol=1e-12)


def test_subchain_vs_slice_products():
    cores = rand_cores(DIMS, RANKS, 4)
    for n in range(1, 5):
        np.testing.assert_allclose(O.subchain(cores, n), O.subchain_slices_bruteforce(cores, n),
                                   rtol=1e-13, atol=1e-13)


def test_core_unfold_layout():
    g = np.random.default_rng(5)
    G = np.asfortranarray(g.standard_normal((2, 5, 3)))
    Z = O.core_unfold2(G)
    for a, i, b in itertools.product(range(2), range(5), range(3)):
        assert Z[i, a + 2 * b] == G[a, i, b]
    # flat memory layout: element (a, i, b) at a + R_n (i + I_n b)
    flat = G.ravel(order="F")
    assert flat[1 + 2 * (3 + 5 * 2)] == G[1, 3, 2]


# ---------------------------------------------------------------------------
# TTM and Prop. 2.1, Prop. 2.2
# ---------------------------------------------------------------------------
def test_ttm_by_loops():
    g = np.random.default_rng(6)
    X = np.asfortranarray(g.standard_normal((3, 4, 2)))
    U = g.standard_normal((5, 4))
    Y = O.ttm(X, U, 2)
    for i, j, k in itertools.product(range(3), range(5), range(2)):
        assert Y[i, j, k] == pytest.approx(sum(X[i, m, k] * U[j, m] for m in range(4)), abs=1e-13)


def test_prop_2_1_multi_ttm_unfolding():
    g = np.random.default_rng(8)
    dims = (3, 4, 2, 3)
    X = np.asfortranarray(g.standard_normal(dims))
    Us = [g.standard_normal((d + 1, d)) for d in dims]
    Y = O.multi_ttm(X, Us)
    for n in range(1, 5):
        # U_{n-1} (x) ... (x) U_1 (x) U_N (x) ... (x) U_{n+1}
        seq = [((n - 2 - k) % 4) for k in range(3)]
        K = Us[seq[0]]
        for s in seq[1:]:
            K = np.kron(K, Us[s])
        rhs = Us[n - 1] @ O.unfold_mode(X, n) @ K.T
        np.testing.assert_allclose(O.unfold_mode(Y, n), rhs, rtol=1e-12, atol=1e-12)


def test_prop_2_2_subchain_kron():
    g = np.random.default_rng(9)
    A = np.asfortranarray(g.standard_normal((2, 3, 4)))
    B = np.asfortranarray(g.standard_normal((4, 5, 3)))
    Am = g.standard_normal((6, 3))
    Bm = g.standard_normal((2, 5))
    lhs = O.subchain_product(O.ttm(A, Am, 2), O.ttm(B, Bm, 2))
    rhs = O.ttm(O.subchain_product(A, B), np.kron(Bm, Am), 2)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Prop. 3.1 and the structured coefficient matrix
# ---------------------------------------------------------------------------
def test_prop_3_1_general_operands():
    g = np.random.default_rng(10)
    I1, J, K1, R, L1 = 2, 3, 4, 5, 3
    I2, K2, L2 = 3, 2, 2
    A = np.asfortranarray(g.standard_normal((I1, J, K1)))
    B = np.asfortranarray(g.standard_normal((K1, R, L1)))
    C = np.asfortranarray(g.standard_normal((I2, J, K2)))
    D = np.asfortranarray(g.standard_normal((K2, R, L2)))
    lhs = O.unfold_mode(O.subchain_product(A, B), 2).T @ O.unfold_mode(O.subchain_product(C, D), 2)
    PB = sum(np.multiply.outer(B[:, r, :].T, D[:, r, :].T) for r in range(R))
    PA = sum(np.multiply.outer(A[:, j, :].T, C[:, j, :].T) for j in range(J))
    T = O.general_contract(PB, PA)
    rhs = T.reshape((T.shape[0] * T.shape[1], -1), order="F")
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N,dims,ranks", [(3, (3, 4, 5), (2, 3, 2)), (4, DIMS, RANKS), (5, (2, 3, 2, 2, 3), (2, 1, 3, 2, 2))])
def test_coef_matrix_structured_equals_explicit(N, dims, ranks):
    cores = rand_cores(dims, ranks, 11)
    for n in range(1, N + 1):
        S1 = O.coef_matrix_paper(cores, n)
        S2 = O.coef_matrix_explicit(cores, n)
        np.testing.assert_allclose(S1, S2, rtol=1e-13, atol=1e-13 * np.abs(S2).max())


def test_mttsp_bruteforce():
    cores = rand_cores(DIMS, RANKS, 12)
    g = np.random.default_rng(13)
    X = np.asfortranarray(g.standard_normal(DIMS))
    rr = list(RANKS) + [RANKS[0]]
    for n in range(1, 5):
        sl = O.subchain_slices_bruteforce(cores, n)   # (R_{n+1}, J, R_n)
        M = np.zeros((DIMS[n - 1], rr[n - 1] * rr[n]))
        for idx in itertools.product(*[range(d) for d in DIMS]):
            j = _col_mode(idx, DIMS, n)
            for a in range(rr[n - 1]):
                for b in range(rr[n]):
                    M[idx[n - 1], a + rr[n - 1] * b] += X[idx] * sl[b, j, a]
        np.testing.assert_allclose(O.mttsp(X, cores, n), M, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Regular ALS (Alg. 1)
# ---------------------------------------------------------------------------
def _explicit_system(X, cores, n):
    """Design matrix and right-hand sides of the subproblem, built by loops."""
    dims = X.shape
    rr = O.ring_ranks(cores)
    sl = O.subchain_slices_bruteforce(cores, n)
    J = sl.shape[1]
    A = np.zeros((J, rr[n - 1] * rr[n]))
    for j in range(J):
        for a in range(rr[n - 1]):
            for b in range(rr[n]):
                A[j, a + rr[n - 1] * b] = sl[b, j, a]
    Bm = np.zeros((J, dims[n - 1]))
    for idx in itertools.product(*[range(d) for d in dims]):
        Bm[_col_mode(idx, dims, n), idx[n - 1]] = X[idx]
    return A, Bm


@pytest.mark.parametrize("mode", ["qr", "ne", "lstsq"])
def test_single_update_vs_lstsq(mode):
    cores = rand_cores(DIMS, RANKS, 14)
    g = np.random.default_rng(15)
    X = np.asfortranarray(g.standard_normal(DIMS))
    rr = O.ring_ranks(cores)
    for n in range(1, 5):
        A, Bm = _explicit_system(X, cores, n)
        Zt = np.linalg.lstsq(A, Bm, rcond=None)[0]
        Gn, _ = O.als_update(X, cores, n, solve=mode)
        for a, i, b in itertools.product(range(rr[n - 1]), range(DIMS[n - 1]), range(rr[n])):
            assert Gn[a, i, b] == pytest.approx(Zt[a + rr[n - 1] * b, i], rel=1e-9, abs=1e-10)


def test_fixed_point_at_true_cores():
    dims, ranks = (6, 7, 5, 6), (2, 3, 2, 3)
    cores = rand_cores(dims, ranks, 16)
    X = O.tr_full(cores)
    out, _ = O.tr_als(X, cores, 1)
    for a, b in zip(out, cores):
        assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(b)
    assert O.rel_error(X, out) <= 1e-13


def test_planted_noiseless_recovery():
    dims, ranks = (8, 9, 10, 7), (2, 3, 2, 3)
    true = rand_cores(dims, ranks, 17)
    X = O.tr_full(true)
    init = rand_cores(dims, ranks, 18)
    cores, _ = O.tr_als(X, init, 300)
    e = O.rel_error(X, cores)
    if e > 1e-12:   # ALS may swamp from a random start; near the truth it must converge
        pert = [c + 1e-2 * np.random.default_rng(19).standard_normal(c.shape) for c in true]
        cores, _ = O.tr_als(X, pert, 50)
        e = O.rel_error(X, cores)
    assert e <= 1e-12


def test_monotone_objective():
    dims, ranks = (6, 5, 7, 4), (2, 3, 3, 2)
    g = np.random.default_rng(20)
    X = np.asfortranarray(g.standard_normal(dims))
    init = rand_cores(dims, ranks, 21)
    _, objs = O.tr_als(X, init, 6, record_objective=True)
    for a, b in zip(objs, objs[1:]):
        assert b <= a * (1 + 1e-12)
    # the recorded objective is the explicit ||X - TR||
    cores, objs = O.tr_als(X, init, 1, record_objective=True)
    assert objs[-1] == pytest.approx(O.rel_error(X, cores) * np.linalg.norm(X), rel=1e-12)


def test_order2_reaches_eckart_young():
    """N = 2: X(i,j) = trace(G_1(i) G_2(j)) is a rank-R_1R_2 factorization, so ALS
    converges to the truncated-SVD error."""
    g = np.random.default_rng(22)
    I1, I2, R1, R2 = 12, 15, 2, 3
    U, _ = np.linalg.qr(g.standard_normal((I1, I1)))
    V, _ = np.linalg.qr(g.standard_normal((I2, I2)))
    s = np.array([10, 9, 8, 7, 6, 5, 0.5, 0.4, 0.3, 0.2, 0.1, 0.05])
    X = np.asfortranarray((U * s) @ V[:, :I1].T)
    init = rand_cores((I1, I2), (R1, R2), 23)
    cores, _ = O.tr_als(X, init, 200)
    k = R1 * R2
    ey = math.sqrt(np.sum(s[k:] ** 2)) / math.sqrt(np.sum(s ** 2))
    assert O.rel_error(X, cores) == pytest.approx(ey, rel=1e-10)


def test_rank1_closed_form_update():
    """R_n = 1: TR is rank-1 CP, and the update of mode n has the closed form
    g_n(i) = <X(.., i, ..), o_{j!=n} g_j> / prod_{j!=n} ||g_j||^2."""
    dims = (4, 5, 3, 6)
    g = np.random.default_rng(24)
    X = np.asfortranarray(g.standard_normal(dims))
    cores = rand_cores(dims, (1, 1, 1, 1), 25)
    vecs = [c[0, :, 0].copy() for c in cores]
    for n in range(1, 5):
        Gn, _ = O.als_update(X, cores, n)
        others = [vecs[j] for j in range(4) if j != n - 1]
        letters = "abcd"
        sub = letters[:4]
        ops = ",".join(letters[j] for j in range(4) if j != n - 1)
        num = np.einsum(f"{sub},{ops}->{letters[n - 1]}", X, *others)
        den = np.prod([v @ v for v in others])
        np.testing.assert_allclose(Gn[0, :, 0], num / den, rtol=1e-13, atol=1e-13)
        cores[n - 1] = Gn
        vecs[n - 1] = Gn[0, :, 0].copy()


def test_noisy_fit_near_noise_floor():
    """From the true cores, noisy exact-rank data converges to an error close to
    eta*sqrt(1 - d/numel), d = sum I_n R_n R_{n+1} - sum R_n^2 (loose, +-10%)."""
    dims, ranks = (10, 11, 9, 12), (2, 3, 2, 3)
    true = rand_cores(dims, ranks, 26)
    Xt = O.tr_full(true)
    eta = 1e-2
    X = W.add_noise(Xt, eta, np.random.default_rng(27))
    cores, _ = O.tr_als(X, true, 30)
    rr = list(ranks) + [ranks[0]]
    d = sum(dims[n] * rr[n] * rr[n + 1] for n in range(4)) - sum(r * r for r in ranks)
    numel = np.prod(dims)
    expect = eta * math.sqrt(1 - d / numel)
    assert O.rel_error(X, cores) == pytest.approx(expect, rel=0.1)


# ---------------------------------------------------------------------------
# Equivalence of Alg. 1, Alg. 2 and Alg. 3 from the same start
# ---------------------------------------------------------------------------
def test_variants_equivalent():
    dims, ranks = (7, 8, 6, 9), (2, 3, 2, 2)
    true = rand_cores(dims, ranks, 28)
    X = W.add_noise(O.tr_full(true), 1e-2, np.random.default_rng(29))
    init = rand_cores(dims, ranks, 30)
    ref, _ = O.tr_als(X, init, 10, solve="qr")
    for other in (O.tr_als(X, init, 10, solve="ne")[0], O.tr_als(X, init, 10, solve="lstsq")[0],
                  O.tr_als_qr_literal(X, init, 10), O.tr_als_ne_literal(X, init, 10),
                  O.tr_als_qrne_literal(X, init, 10)):
        for a, b in zip(other, ref):
            assert np.linalg.norm(a - b) <= 1e-10 * np.linalg.norm(b)


def test_qr_literal_case_short_core():
    """Mode-2 QR with I_j < R_j R_{j+1} (square Q, trapezoidal R) still gives the
    regular-ALS update."""
    dims, ranks = (3, 8, 9, 7), (2, 2, 3, 2)   # core 1 is 2 x 3 x 2: I=3 < 4
    true = rand_cores(dims, ranks, 31)
    X = W.add_noise(O.tr_full(true), 1e-2, np.random.default_rng(32))
    init = rand_cores(dims, ranks, 33)
    ref, _ = O.tr_als(X, init, 3)
    for out in (O.tr_als_qr_literal(X, init, 3), O.tr_als_qrne_literal(X, init, 3)):
        for a, b in zip(out, ref):
            assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)


def test_r_core_grams_equal_core_grams():
    """Alg. 4 forms its Grams from the R-cores: G(2) = Q R(2) with orthonormal
    Q, so the R-core Gram equals the core's Gram (also when I < R_n R_{n+1})."""
    for dims, ranks, seed in (((9, 3), (2, 3), 40), ((12, 5, 7), (3, 2, 2), 41)):
        for G in rand_cores(dims, ranks, seed):
            _, Rc = O.mode2_qr(G)
            assert np.allclose(O.gram_tensor(Rc), O.gram_tensor(G), rtol=0, atol=1e-12 * np.abs(G).max() ** 2)


# ---------------------------------------------------------------------------
# Sec. 3.4 by-product (corrected) and Sec. 4 error identities
# ---------------------------------------------------------------------------
def test_tr_inner_product_and_printed_form():
    dims = (3, 2, 4)
    A = rand_cores(dims, (2, 3, 2), 34)
    B = rand_cores(dims, (3, 1, 2), 35)
    XA, XB = O.tr_full_bruteforce(A), O.tr_full_bruteforce(B)
    truth = float(np.sum(XA * XB))
    assert O.tr_inner(A, B) == pytest.approx(truth, rel=1e-13)
    assert O.tr_inner(A, A) == pytest.approx(float(np.sum(XA * XA)), rel=1e-13)
    # the printed Trace(T_<2>) is another number (reading recorded with the oracle)
    Ps = [O.gram_tensor(G, Z) for G, Z in zip(A, B)]
    T = O.general_contract(O.general_contract(Ps[2], Ps[1]), Ps[0])
    printed = float(np.trace(T.reshape((T.shape[0] * T.shape[1], -1), order="F")))
    assert abs(printed - truth) > 1e-6 * abs(truth)


def test_regular_objective_is_the_residual_norm():
    """The LS objective of any mode equals ||X - TR(G)||_F with TR(G) built by the
    brute-force trace (Sec. 1), so it is the same number for every n and equals
    rel_error * ||X||_F."""
    dims, ranks = (3, 4, 2, 3), (2, 3, 2, 2)
    g = np.random.default_rng(38)
    X = np.asfortranarray(g.standard_normal(dims))
    cores = rand_cores(dims, ranks, 39)
    truth = float(np.sqrt(np.sum((X - O.tr_full_bruteforce(cores)) ** 2)))
    for n in range(1, 5):
        assert O.regular_objective(X, cores, n) == pytest.approx(truth, rel=1e-13)
    assert O.rel_error(X, cores) * float(np.linalg.norm(X)) == pytest.approx(truth, rel=1e-13)
    # at the true cores of a noiseless planted tensor the objective vanishes
    Xp = O.tr_full_bruteforce(cores)
    assert O.regular_objective(Xp, cores, 2) <= 1e-12 * float(np.linalg.norm(Xp))


def test_cheap_fit_identities():
    dims, ranks = (5, 4, 6, 3), (2, 3, 2, 2)
    g = np.random.default_rng(36)
    X = np.asfortranarray(g.standard_normal(dims))
    cores = rand_cores(dims, ranks, 37)
    Xh = O.tr_full(cores)
    ip, nrm2 = O.cheap_fit_terms(X, cores)
    assert ip == pytest.approx(float(np.sum(X * Xh)), rel=1e-12)
    assert nrm2 == pytest.approx(float(np.sum(Xh * Xh)), rel=1e-12)


# ---------------------------------------------------------------------------
# Narrow formats of the X shadows: encoders written from the format
# definitions, pinned by values the definitions fix.
# ---------------------------------------------------------------------------
def test_bf16_encoder_fixed_values():
    from oracle.lowp_formats import bf16_bits, bf16_value
    cases = {1.0: 0x3F80, -2.0: 0xC000, 0.0: 0x0000, 1.0 + 2.0 ** -8: 0x3F80,     # tie, even stays
             1.0 + 3 * 2.0 ** -8: 0x3F82,                                         # tie, odd rounds up
             1.0 + 2.0 ** -8 + 2.0 ** -20: 0x3F81,                                # above the tie
             float(np.finfo(np.float32).max): 0x7F80}                             # rounds to infinity
    for x, want in cases.items():
        assert int(bf16_bits(np.float32(x))) == want, (x, hex(int(bf16_bits(np.float32(x)))))
    assert int(bf16_bits(np.float32(-0.0))) == 0x8000
    allb = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    vals = bf16_value(allb).astype(np.float32)
    ok = ~np.isnan(vals)
    assert np.array_equal(bf16_bits(vals[ok]), allb[ok])                 # exact values round-trip


def test_fp8_e4m3_encoder_fixed_values():
    from oracle.lowp_formats import fp8_e4m3_bits, fp8_e4m3_value
    cases = {1.0: 0x38, 448.0: 0x7E, -448.0: 0xFE, 2.0 ** -6: 0x08, 2.0 ** -9: 0x01, 2.0 ** -10: 0x00,
             3 * 2.0 ** -10: 0x02, 7.5 * 2.0 ** -9: 0x08, 1.0 + 1 / 16: 0x38, 1.0 + 3 / 16: 0x3A,
             1.0 + 15 / 16: 0x40, 0.0: 0x00, 240.0: 0x77, 0.875 * 2.0 ** -6: 0x07}
    for x, want in cases.items():
        got = int(fp8_e4m3_bits(np.float32(x)))
        assert got == want, (x, hex(got), hex(want))
    assert int(fp8_e4m3_bits(np.float32(-0.0))) == 0x80
    codes = np.array([b for b in range(256) if (b & 0x7F) != 0x7F], dtype=np.uint8)
    vals = fp8_e4m3_value(codes)
    assert np.nanmax(np.abs(fp8_e4m3_value(np.arange(256, dtype=np.uint8)))) == 448.0
    back = fp8_e4m3_bits(vals.astype(np.float32))
    assert np.array_equal(back[vals != 0], codes[vals != 0])
    assert int(fp8_e4m3_bits(np.float32(464.0))) == 0x7E      # tie between 448 and 480: the even fraction
    with pytest.raises(ValueError):
        fp8_e4m3_bits(np.float32(465.0))                      # nearer to 480, which E4M3 cannot hold
    # nearest: a value between two codes goes to the closer one
    g = np.random.default_rng(3)
    x = (g.standard_normal(20000) * 30).astype(np.float32)
    q = fp8_e4m3_value(fp8_e4m3_bits(x))
    fin = np.sort(np.unique(np.abs(vals)))
    for xv, qv in zip(x[:2000], q[:2000]):
        d = np.abs(fin - abs(float(xv)))
        assert abs(abs(qv) - abs(float(xv))) <= d.min() + 1e-12


def test_lstsq_minimum_norm_on_a_duplicated_column():
    """With A = [A1, A1[:, 0]] (one column repeated) the least-squares fit is the
    full-rank fit of A1; the minimum-norm coefficients split the repeated
    column's weight equally between its two copies.  Pins the oracle's
    rank-deficient solve (lstsq) and the fallback of its default (qr) mode."""
    g = np.random.default_rng(60)
    A1 = g.standard_normal((40, 5))
    B = g.standard_normal((40, 3))
    A = np.hstack([A1, A1[:, :1]])
    Z1 = O.solve_ls(A1, B, "qr")
    want = np.vstack([Z1[:1] / 2, Z1[1:], Z1[:1] / 2])
    for mode in ("lstsq", "qr"):
        assert np.allclose(O.solve_ls(A, B, mode), want, rtol=0, atol=1e-12)
