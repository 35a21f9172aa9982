"""The QR-based updates on the GPU -- TR-ALS-QR (Alg. 3) and TR-ALS-QRNE
(Alg. 4) -- against the oracle's regular ALS from the same initial cores (the
variants are mathematically equivalent), and against the oracle's literal
Alg. 3 / Alg. 4 on conditioned cores."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cores_from_dev, cores_to_dev, rel, say, to_dev_flat

pytestmark = pytest.mark.gpu

QR_SHAPES = [
    ((30, 40), (3, 4)),
    ((17, 20, 13, 11), (2, 3, 4, 3)),
    ((3, 8, 9, 7), (2, 2, 3, 2)),          # core 1: I = 3 < R_1 R_2 = 4 (square Q, trapezoidal R)
    ((6, 7, 5, 8, 6), (2, 3, 2, 2, 3)),
    ((40, 36, 30), (5, 6, 4)),
    ((100, 12, 10), (3, 4, 2)),            # core QR with 65..128 rows per column
    ((150, 20, 12), (2, 3, 2)),            # 129..256 rows
    ((300, 8, 6), (2, 2, 3)),              # more than 256 rows: the global-memory factorization
    ((11, 13, 9), (3, 3, 3)),              # odd V_n[2] height: the LDS-staged Gram
    ((60, 60, 60), (7, 7, 7)),             # odd height, four 16-column blocks
    ((110, 110, 110), (10, 10, 10)),       # even height, seven blocks: the register-fragment Gram
    ((24, 26, 22), (8, 14, 8)),            # n = 112: tall products with all seven k blocks (none trimmed)
]


def _ctx(X, cores, dims, ranks, variant):
    from paper_2210_11362_amd import TRContext
    dev = cores_to_dev(cores)
    return TRContext(X, dims, ranks, dev, variant=variant), dev


def _data(dims, ranks, seed, dtype=np.float64):
    g = np.random.default_rng(seed)
    true = W.gaussian_cores(dims, ranks, g)
    X = W.add_noise(W.planted_tensor(true), 0.05, g)
    init = W.gaussian_cores(dims, ranks, g)
    return np.asfortranarray(X.astype(dtype)), init


# R_n R_{n+1} > 128: the Cholesky-QR factor blocked, the large FP64 products
# (Gram of V_n[2], the triangular passes, Y_[n] Q_0 or Y_[n] V_n[2], the
# substitution with R_[2]) on rocBLAS
LARGE_QR_SHAPES = [
    ((24, 22, 20), (20, 20, 20)),          # n = 400, every core factor square (I_k < 400)
    ((40, 36, 30), (12, 11, 13)),          # n = 132, 143, 156; the middle mode sums slice products
    ((30, 28, 26, 12), (12, 12, 11, 2)),   # order 4: n = 144, 132 beside n = 22, 24
    ((150, 150, 20), (12, 12, 2)),         # core 1 unfolding 150 x 144: Cholesky-QR of a tall core
    ((150, 30, 28), (20, 20, 20)),         # core 1 unfolding 150 x 400: register-Householder panels of
                                           # 64, 64 and 22 columns with block Gram-Schmidt between them
]


@pytest.mark.parametrize("variant", ["qr", "qrne"])
@pytest.mark.parametrize("dims,ranks", LARGE_QR_SHAPES, ids=[str(s[1]) for s in LARGE_QR_SHAPES])
def test_qr_variants_large_bond_products_f64(dims, ranks, variant):
    say(f"[{variant} f64, large n] dims={dims} ranks={ranks}")
    X, init = _data(dims, ranks, 17)
    ctx, dev = _ctx(to_dev_flat(X), init, dims, ranks, variant)
    ref = [np.array(c) for c in init]
    for s in range(2):
        ref, _ = O.tr_als(X, ref, 1)
        ctx.sweep(1, "f64")
        got = cores_from_dev(dev, dims, ranks)
        errs = [rel(a, b) for a, b in zip(got, ref)]
        say(f"   sweep {s + 1}: max core rel err {max(errs):.2e}")
        assert max(errs) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("variant", ["qr", "qrne"])
@pytest.mark.parametrize("dims,ranks", QR_SHAPES, ids=[str(s[0]) for s in QR_SHAPES])
def test_qr_variant_per_sweep_f64(dims, ranks, variant):
    say(f"[{variant} f64] dims={dims} ranks={ranks}")
    X, init = _data(dims, ranks, 11)
    ctx, dev = _ctx(to_dev_flat(X), init, dims, ranks, variant)
    ref = [np.array(c) for c in init]
    for s in range(3):
        ref, _ = O.tr_als(X, ref, 1)
        ctx.sweep(1, "f64")
        got = cores_from_dev(dev, dims, ranks)
        errs = [rel(a, b) for a, b in zip(got, ref)]
        say(f"   sweep {s + 1}: max core rel err {max(errs):.2e}")
        assert max(errs) <= 1e-10
    ctx.close()


@pytest.mark.parametrize("variant", ["qr", "qrne"])
def test_qr_matches_literal_alg_on_conditioned_cores(variant):
    """Config 3's recipe (cores with condition number 1e4, ranks (6,8,10,8,6) scaled
    to (2,3,4,3,2)) at 9^5: GPU QR / QRNE sweeps track the oracle's literal
    Alg. 3 / Alg. 4."""
    w = W.make_workload(3, dims=(9, 9, 9, 9, 9), ranks=(2, 3, 4, 3, 2))
    X = w.X.astype(np.float64)
    ctx, dev = _ctx(to_dev_flat(w.X), w.init_cores, w.dims, w.ranks, variant)
    ctx.sweep(2, "f64")
    got = cores_from_dev(dev, w.dims, w.ranks)
    lit = O.tr_als_qr_literal if variant == "qr" else O.tr_als_qrne_literal
    ref = lit(X, w.init_cores, 2)
    errs = [rel(a, b) for a, b in zip(got, ref)]
    say(f"   core rel errs {[f'{e:.1e}' for e in errs]}")
    assert max(errs) <= 1e-8
    ctx.close()


@pytest.mark.parametrize("variant", ["qr", "qrne"])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_qr_variant_fit_mixed(prec, variant):
    w = W.make_workload(2, dims=(18, 20, 16, 14), ranks=(4, 4, 4, 4))
    ctx, dev = _ctx(to_dev_flat(w.X), w.init_cores, w.dims, w.ranks, variant)
    ctx.sweep(6, prec)
    ctx.sweep(2, "f32")
    f_gpu = ctx.fit()
    ref, _ = O.tr_als(w.X.astype(np.float64), w.init_cores, 8)
    f_ref = O.rel_error(w.X.astype(np.float64), ref)
    say(f"   [{variant} {prec}] fit gpu {f_gpu:.6e} oracle {f_ref:.6e}")
    assert abs(f_gpu - f_ref) <= 1e-3
    ctx.close()


@pytest.mark.parametrize("variant", ["qr", "qrne"])
def test_qr_and_ne_agree(variant):
    dims, ranks = (20, 18, 16, 14), (3, 4, 3, 4)
    X, init = _data(dims, ranks, 12)
    a, da = _ctx(to_dev_flat(X), init, dims, ranks, "ne")
    b, db = _ctx(to_dev_flat(X), init, dims, ranks, variant)
    a.sweep(4, "f64")
    b.sweep(4, "f64")
    for x, y in zip(cores_from_dev(da, dims, ranks), cores_from_dev(db, dims, ranks)):
        assert rel(x, y) <= 1e-9
    a.close()
    b.close()


@pytest.mark.parametrize("variant", ["qr", "qrne"])
def test_sweep_mode_pairs_match_single_mode_updates(variant):
    """Within a sweep, modes p and p+1 (p even) share the Multi-TTM part over
    the other modes; a single-mode update forms its Y from X.  Both are the Y
    of Alg. 3 / Alg. 4 (the same products in another order), so one sweep and
    N single-mode updates from the same cores agree to rounding.  Order 5:
    two pairs and one mode on its own."""
    dims, ranks = (14, 12, 10, 9, 8), (2, 3, 2, 3, 2)
    say(f"[{variant} f64, pairs vs single] dims={dims} ranks={ranks}")
    X, init = _data(dims, ranks, 23)
    Xd = to_dev_flat(X)
    a, da = _ctx(Xd, init, dims, ranks, variant)
    b, db = _ctx(Xd, init, dims, ranks, variant)
    a.sweep(1, "f64")
    for n in range(1, len(dims) + 1):
        b.update_mode(n, "f64")
    b.store_cores()
    ga = cores_from_dev(da, dims, ranks)
    gb = cores_from_dev(db, dims, ranks)
    errs = [rel(x, y) for x, y in zip(ga, gb)]
    say(f"   max core rel diff {max(errs):.2e}")
    assert max(errs) <= 1e-11
    ref, _ = O.tr_als(X, [np.array(c) for c in init], 1)
    assert max(rel(x, y) for x, y in zip(ga, ref)) <= 1e-10
    a.close()
    b.close()
