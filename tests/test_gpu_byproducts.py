"""By-products of the ALS intermediates on the GPU, against the oracle:

* the in-loop error estimate of Sec. 4 (``tr_als_run``) equals the explicit
  relative error of the same cores (FP64 path, every variant), and the
  tolerance-based termination stops at the sweep the oracle's own error
  trajectory says it should;
* the inner product and norm of tensors in TR format (Sec. 3.4, corrected
  reading) equal the oracle's pair-space trace and the norm of the
  explicitly reconstructed tensor.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cores_from_dev, cores_to_dev, say, to_dev_flat

pytestmark = pytest.mark.gpu


def _data(dims, ranks, seed, eta=0.05):
    g = np.random.default_rng(seed)
    true = W.gaussian_cores(dims, ranks, g)
    X = np.asfortranarray(W.add_noise(W.planted_tensor(true), eta, g))
    init = W.gaussian_cores(dims, ranks, g)
    return X, init


@pytest.mark.parametrize("variant", ["ne", "qr", "qrne"])
@pytest.mark.parametrize("dims,ranks", [((17, 20, 13, 11), (2, 3, 4, 3)), ((30, 28, 26), (4, 5, 6)),
                                        ((7, 8, 6, 9, 5), (2, 3, 2, 2, 3))])
def test_in_loop_error_equals_explicit_error(dims, ranks, variant):
    from paper_2210_11362_amd import TRContext
    X, init = _data(dims, ranks, 51)
    dev = cores_to_dev(init)
    ctx = TRContext(to_dev_flat(X), dims, ranks, dev, variant=variant)
    for s in range(3):
        k, f_cheap = ctx.run(1, "f64", refine=1)
        assert k == 1
        f_exp = ctx.fit()
        cores = cores_from_dev(dev, dims, ranks)
        ip, nrm2 = O.cheap_fit_terms(X, cores)
        xx = float(np.sum(X * X))
        f_or = np.sqrt(max(0.0, xx - 2 * ip + nrm2) / xx)
        say(f"[{variant} {dims}] sweep {s + 1}: in-loop {f_cheap:.15e} explicit {f_exp:.15e} oracle {f_or:.15e}")
        assert abs(f_cheap - f_exp) <= 1e-10
        assert abs(f_cheap - f_or) <= 1e-10
        assert abs(f_exp - O.rel_error(X, cores)) <= 1e-12
    ctx.close()


def test_run_stops_where_the_error_trajectory_says():
    from paper_2210_11362_amd import TRContext
    dims, ranks = (20, 18, 16, 14), (3, 3, 3, 3)
    X, init = _data(dims, ranks, 52, eta=0.02)
    fits = []
    O.tr_als(X, init, 25, callback=lambda s, cs: fits.append(O.rel_error(X, cs)))
    d = np.abs(np.diff(fits))                 # d[j] = |f_{j+2} - f_{j+1}| (errors after sweeps j+1, j+2)
    # the first change clearly below every earlier one; a tolerance between them
    j = next(j for j in range(4, len(d)) if d[j] < 0.8 * d[:j].min())
    tol = float(np.sqrt(d[j] * d[:j].min()))
    expect = j + 2                              # the run stops after the sweep whose change is d[j]
    assert np.all(d[:j] > tol) and d[j] < tol
    ctx = TRContext(to_dev_flat(X), dims, ranks, cores_to_dev(init))
    k, f = ctx.run(40, "f64", refine=1, tol=tol)
    say(f"[run tol={tol:.3e}] stopped after {k} sweeps (oracle trajectory: {expect}); error {f:.12e}")
    assert k == expect
    assert abs(f - fits[k - 1]) <= 1e-10
    ctx.close()
    ctx = TRContext(to_dev_flat(X), dims, ranks, cores_to_dev(init))
    k2, f2 = ctx.run(3, "f64", refine=1, tol=0.0)     # early sweeps change the error: all three run
    assert k2 == 3 and abs(f2 - fits[2]) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("dims,ra,rb", [((9, 7), (2, 3), (3, 2)),
                                        ((12, 10, 8), (2, 3, 4), (3, 3, 2)),
                                        ((6, 5, 7, 4, 5), (2, 3, 2, 2, 3), (1, 2, 3, 2, 2)),
                                        ((40, 36, 30), (10, 12, 8), (6, 7, 9))])
def test_tr_inner_and_norm(dims, ra, rb):
    from paper_2210_11362_amd import tr_inner, tr_norm
    g = np.random.default_rng(53)
    A = W.gaussian_cores(dims, ra, g)
    B = W.gaussian_cores(dims, rb, g)
    da, db = cores_to_dev(A), cores_to_dev(B)
    v = tr_inner(dims, ra, da, rb, db)
    ref = O.tr_inner(A, B)
    explicit = float(np.sum(O.tr_full(A) * O.tr_full(B)))
    say(f"[inner {dims}] gpu {v:.15e} oracle {ref:.15e} explicit {explicit:.15e}")
    scale = np.linalg.norm(O.tr_full(A)) * np.linalg.norm(O.tr_full(B))
    assert abs(v - ref) <= 1e-12 * scale
    assert abs(v - explicit) <= 1e-12 * scale
    nA = tr_norm(dims, ra, da)
    assert abs(nA - np.linalg.norm(O.tr_full(A))) <= 1e-12 * nA
    # symmetric in its arguments
    assert abs(tr_inner(dims, rb, db, ra, da) - v) <= 1e-12 * scale
