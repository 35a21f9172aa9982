"""Plant plausible mistakes in the oracle (on the CPU, via monkeypatch) and check
that the pins catch each one: evidence that the pins constrain the oracle."""
import numpy as np
import pytest

import oracle as O
import oracle.tr_oracle as T
import tests.test_oracle_pins as P

PINS = [
    P.test_reconstruction_every_mode,
    P.test_subchain_vs_slice_products,
    P.test_coef_matrix_structured_equals_explicit.__wrapped__ if hasattr(P.test_coef_matrix_structured_equals_explicit, "__wrapped__") else None,
    P.test_mttsp_bruteforce,
    P.test_fixed_point_at_true_cores,
    P.test_unfold_mode_by_definition,
    P.test_prop_2_1_multi_ttm_unfolding,
    P.test_cheap_fit_identities,
    P.test_variants_equivalent,
    P.test_tr_inner_product_and_printed_form,
    P.test_unfold_classical_by_definition,
    P.test_unfold_n_by_definition,
    P.test_regular_objective_is_the_residual_norm,
]


def _run_pins():
    failed = 0
    for f in PINS:
        if f is None:
            continue
        try:
            f()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            failed += 1
    for N, dims, ranks in [(4, P.DIMS, P.RANKS)]:
        try:
            P.test_coef_matrix_structured_equals_explicit(N, dims, ranks)
        except (AssertionError, ValueError, IndexError):
            failed += 1
    try:
        P.test_single_update_vs_lstsq("qr")
    except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
        failed += 1
    return failed


def _reversed_chain(N, n):
    return list(reversed([((n - 1 + k) % N) + 1 for k in range(1, N)]))


def _core_unfold2_swapped(G):
    Rn, I, Rn1 = G.shape
    return np.asfortranarray(G.transpose(1, 2, 0).reshape((I, Rn * Rn1), order="F"))


def _subchain_unfold2_swapped(cores, n):
    Z = T.subchain(cores, n)
    Rb, J, Ra = Z.shape
    return np.asfortranarray(np.transpose(Z, (1, 0, 2)).reshape((J, Ra * Rb), order="F"))


def _unfold_mode_classical(X, n):
    return T.unfold_classical(X, n)


def _gram_transposed(G, Z=None):
    if Z is None:
        Z = G
    return np.einsum("piq,ris->pqrs", G, Z, optimize=True)


def _contract_wrong(A, B):
    return np.einsum("ijrk,kljs->ilrs", A, B, optimize=True)


def _unfold_classical_cyclic(X, n):
    return T.unfold_mode(X, n)


def _unfold_n_c_order(X, n):
    rows = int(np.prod(X.shape[:n]))
    return np.ascontiguousarray(X).reshape((rows, -1), order="C")


def _objective_wrong_core(X, cores, n):
    N = len(cores)
    A = T.subchain_unfold2(cores, n)
    G = cores[n % N] if cores[n % N].shape == cores[n - 1].shape else 2.0 * cores[n - 1]
    return float(np.linalg.norm(T.unfold_mode(X, n) - T.core_unfold2(G) @ A.T))


MUTATIONS = [
    ("unfold_classical", _unfold_classical_cyclic),
    ("unfold_n", _unfold_n_c_order),
    ("regular_objective", _objective_wrong_core),
    ("_chain_order", _reversed_chain),
    ("core_unfold2", _core_unfold2_swapped),
    ("subchain_unfold2", _subchain_unfold2_swapped),
    ("unfold_mode", _unfold_mode_classical),
    ("gram_tensor", _gram_transposed),
    ("general_contract", _contract_wrong),
]


def test_pins_pass_unmutated():
    assert _run_pins() == 0


@pytest.mark.parametrize("name,fn", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(T, name, fn)
    if hasattr(O, name):
        monkeypatch.setattr(O, name, fn)
    assert _run_pins() >= 1
