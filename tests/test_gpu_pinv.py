"""The rank-deficient-safe solve (tr_als_set_solve TR_SOLVE_PINV) against the
oracle's minimum-norm regular ALS (lstsq solves).

Rank deficiency is planted exactly: the last core's two right slices are
equal, so G^{!=1}_[2] has two equal columns for every pair (a=0, b), (a=1, b);
the minimum-norm update of mode 1 then makes core 1's two left slices equal,
which repeats the deficiency at mode N every sweep.  Every variant follows
the oracle's trajectory within 1e-8 per sweep (the pseudo-inverse of S_n
works on squared singular values; the oracle uses the SVD of G^{!=n}_[2]).
On full-rank problems the pseudo-inverse solve equals the default one.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cores_from_dev, cores_to_dev, rel, say, to_dev_flat

pytestmark = pytest.mark.gpu


def _deficient(dims, ranks, seed):
    g = np.random.default_rng(seed)
    true = W.gaussian_cores(dims, ranks, g)
    X = np.asfortranarray(W.add_noise(W.planted_tensor(true), 0.05, g))
    init = [np.array(c) for c in W.gaussian_cores(dims, ranks, g)]
    init[-1][:, :, 1] = init[-1][:, :, 0]
    return X, [np.asfortranarray(c) for c in init]


@pytest.mark.parametrize("variant", ["ne", "qrne", "qr"])
@pytest.mark.parametrize("dims,ranks", [((12, 10, 9, 8), (2, 3, 2, 3)), ((15, 13, 11), (3, 2, 4)),
                                        ((7, 8, 6, 9, 5), (2, 3, 2, 2, 3))])
def test_pinv_follows_minimum_norm_als(dims, ranks, variant):
    from paper_2210_11362_amd import TRContext
    X, init = _deficient(dims, ranks, 61)
    A = O.subchain_unfold2(init, 1)
    s = np.linalg.svd(A, compute_uv=False)
    say(f"[pinv {variant}] dims={dims} ranks={ranks}: sigma_min/sigma_max of G^(!=1) = {s[-1] / s[0]:.1e}")
    assert s[-1] / s[0] < 1e-13                                   # the planted deficiency
    dev = cores_to_dev(init)
    ctx = TRContext(to_dev_flat(X), dims, ranks, dev, variant=variant)
    ctx.set_solve("pinv")
    ref = [np.array(c) for c in init]
    for sweep in range(3):
        ref, _ = O.tr_als(X, ref, 1, solve="lstsq")
        ctx.sweep(1, "f64", refine=1)
        got = cores_from_dev(dev, dims, ranks)
        errs = [rel(a, b) for a, b in zip(got, ref)]
        say(f"   sweep {sweep + 1}: max core rel err {max(errs):.2e}")
        assert max(errs) <= 1e-8
    assert abs(ctx.fit() - O.rel_error(X, ref)) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("dims,ranks", [((37, 29, 23), (3, 4, 2)), ((17, 20, 13, 11), (2, 3, 4, 3))])
def test_pinv_equals_default_solve_on_full_rank(dims, ranks):
    from paper_2210_11362_amd import TRContext
    g = np.random.default_rng(62)
    true = W.gaussian_cores(dims, ranks, g)
    X = np.asfortranarray(W.add_noise(W.planted_tensor(true), 0.05, g))
    init = W.gaussian_cores(dims, ranks, g)
    ref, _ = O.tr_als(X, init, 2)
    dev = cores_to_dev(init)
    ctx = TRContext(to_dev_flat(X), dims, ranks, dev)
    ctx.set_solve("pinv")
    ctx.sweep(2, "f64", refine=1)
    errs = [rel(a, b) for a, b in zip(cores_from_dev(dev, dims, ranks), ref)]
    say(f"[pinv full rank] {dims}: max core rel err {max(errs):.2e}")
    assert max(errs) <= 1e-10
    ctx.close()
