"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances:
  FP64 contraction: per-sweep core relative error <= 1e-10 (stated target).
  FP32 contraction: per-sweep core relative error <= 1e-5 (stated target);
                    M_n relative Frobenius error <= 1e-5.
  BF16 / FP8:       M_n relative Frobenius error <= 2e-2 / 1.5e-1 (unit roundoff
                    2^-8 / 2^-4 of both operands, errors averaging over the sum);
                    final fit within 1e-3 of the oracle after FP32 finishing sweeps.
Gram and coefficient matrices are FP64 end to end: <= 1e-12 relative.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.gpu_util import cores_from_dev, cores_to_dev, rel, say, to_dev_flat

pytestmark = pytest.mark.gpu

SHAPES = [
    # (dims, ranks): ragged sizes spanning several K tiles, every mode position
    ((50, 70), (3, 4)),
    ((37, 29, 23), (3, 4, 2)),
    ((17, 20, 13, 11), (2, 3, 4, 3)),
    ((6, 7, 5, 8, 6), (2, 3, 2, 2, 3)),
    ((150, 40, 30), (12, 11, 13)),        # row tiles (I > 128) and column tiles (R_nR_{n+1} > 128)
    ((64, 64, 64), (4, 4, 4)),
]


def _ctx(X, cores, dims, ranks, variant="ne"):
    from paper_2210_11362_amd import TRContext
    dev = cores_to_dev(cores)
    return TRContext(X, dims, ranks, dev, variant=variant), dev


def _data(dims, ranks, seed, dtype=np.float64):
    g = np.random.default_rng(seed)
    true = W.gaussian_cores(dims, ranks, g)
    X = W.add_noise(W.planted_tensor(true), 0.05, g)
    init = W.gaussian_cores(dims, ranks, g)
    return np.asfortranarray(X.astype(dtype)), init


@pytest.mark.parametrize("dims,ranks", SHAPES, ids=[str(s[0]) for s in SHAPES])
def test_gram_and_coef(dims, ranks):
    say(f"[gram/coef] dims={dims} ranks={ranks}")
    X, init = _data(dims, ranks, 1)
    ctx, _ = _ctx(to_dev_flat(X), init, dims, ranks)
    N = len(dims)
    for k in range(1, N + 1):
        Z = O.core_unfold2(init[k - 1])
        E = ctx.gram(k).cpu().numpy()
        assert rel(E, Z.T @ Z) <= 1e-12
    for n in range(1, N + 1):
        S = ctx.coef(n).cpu().numpy()
        assert rel(S, O.coef_matrix_explicit(init, n)) <= 1e-12, n
    ctx.close()


@pytest.fixture
def force_regime(request, monkeypatch):
    """Pin the MTTSP kernel: 1 = two-stage GEMM wherever a group exists,
    2 = single pass (the slab kernel for order 3 with R_n R_{n+1} > 128, else
    the fused kernel), 2f = the fused kernel, 0 = the cost rule."""
    monkeypatch.setenv("TR_ALS_FORCE_REGIME", str(request.param)[0])
    if request.param == "2f":   # the fused kernel also where the slab kernel would run (order 3, R_n R_{n+1} > 128)
        monkeypatch.setenv("TR_ALS_NO_SLAB", "1")
    return request.param


@pytest.mark.parametrize("force_regime", [0, 1, 2, "2f"], indirect=True)
@pytest.mark.parametrize("prec,xdt,tol", [("f64", np.float64, 1e-12), ("f32", np.float32, 1e-5),
                                          ("bf16", np.float32, 2e-2), ("fp8", np.float32, 8e-2)])
@pytest.mark.parametrize("dims,ranks", SHAPES, ids=[str(s[0]) for s in SHAPES])
def test_mttsp(dims, ranks, prec, xdt, tol, force_regime):
    say(f"[mttsp] dims={dims} ranks={ranks} prec={prec} regime={force_regime}")
    X, init = _data(dims, ranks, 2, xdt)
    ctx, _ = _ctx(to_dev_flat(X), init, dims, ranks)
    Xd = X.astype(np.float64)
    for n in range(1, len(dims) + 1):
        M = ctx.mttsp(n, prec).cpu().numpy()
        Mo = O.mttsp(Xd, init, n)
        e = rel(M, Mo)
        say(f"   mode {n}: rel err {e:.3e}")
        assert e <= tol, (n, e)
    ctx.close()


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5), ("bf16", 2e-2)])
def test_slab_kernel_vector_path(prec, tol, monkeypatch):
    """Order 3 with R_n R_{n+1} > 128 and every mode size a multiple of 8: the
    slab kernel, whose BF16 form loads 8 elements at a time (rows i contiguous
    for mode 1, k contiguous for modes 2 and 3) and fetches a chunk ahead."""
    monkeypatch.setenv("TR_ALS_FORCE_REGIME", "2")
    dims, ranks = (48, 40, 32), (12, 11, 13)
    X, init = _data(dims, ranks, 8, np.float32)
    ctx, _ = _ctx(to_dev_flat(X), init, dims, ranks)
    assert all(ctx.regime(n) == 3 for n in range(1, 4))
    Xd = X.astype(np.float64)
    for n in range(1, 4):
        M = ctx.mttsp(n, prec).cpu().numpy()
        e = rel(M, O.mttsp(Xd, init, n))
        say(f"   [slab {prec}] mode {n}: rel err {e:.3e}")
        assert e <= tol, (n, e)
    ctx.close()


# ranks whose products R_nR_{n+1} give coefficient matrices of 1 to 8 blocks of
# 16 (n = 12..128, ragged and full last blocks) for the in-register inverse
INV_SHAPES = [
    ((20, 24, 30), (4, 8, 16)),    # n = 32, 128, 64
    ((26, 22, 18), (3, 11, 5)),    # n = 33, 55, 15
    ((30, 26, 22), (8, 9, 4)),     # n = 72, 36, 32
    ((30, 28, 26), (9, 9, 10)),    # n = 81, 90, 90
    ((24, 40, 28), (2, 6, 10)),    # n = 12, 60, 20
]


@pytest.mark.parametrize("dims,ranks", INV_SHAPES, ids=[str(s[1]) for s in INV_SHAPES])
def test_update_f64_every_inverse_block_count(dims, ranks):
    say(f"[update f64, inverse sizes] dims={dims} ranks={ranks}")
    X, init = _data(dims, ranks, 5)
    ctx, dev = _ctx(to_dev_flat(X), init, dims, ranks)
    ref, _ = O.tr_als(X, init, 2)
    ctx.sweep(2, "f64", refine=1)
    got = cores_from_dev(dev, dims, ranks)
    for a, b in zip(got, ref):
        assert rel(a, b) <= 1e-10
    ctx.close()


# coefficient matrices larger than the one-workgroup inverse (R_n R_{n+1} > 128):
# inverted by blocks through Schur complements (one and three levels)
BLOCKED_SHAPES = [((30, 28, 26), (12, 11, 13)),   # n = 132, 143, 156
                  ((24, 22, 20), (20, 20, 20))]   # n = 400, the rank-20 field workload's size


@pytest.mark.parametrize("dims,ranks", BLOCKED_SHAPES, ids=[str(s[1]) for s in BLOCKED_SHAPES])
def test_update_f64_blocked_inverse(dims, ranks):
    say(f"[update f64, blocked inverse] dims={dims} ranks={ranks}")
    X, init = _data(dims, ranks, 6)
    ctx, dev = _ctx(to_dev_flat(X), init, dims, ranks)
    ref = [np.array(c) for c in init]
    for s in range(2):
        ref, _ = O.tr_als(X, ref, 1)
        ctx.sweep(1, "f64", refine=1)
        got = cores_from_dev(dev, dims, ranks)
        errs = [rel(a, b) for a, b in zip(got, ref)]
        say(f"   sweep {s + 1}: max core rel err {max(errs):.2e}")
        assert max(errs) <= 1e-9
    ctx.close()


@pytest.mark.parametrize("dims,ranks", SHAPES[:4], ids=[str(s[0]) for s in SHAPES[:4]])
def test_update_f64_matches_regular_als(dims, ranks):
    say(f"[update f64] dims={dims} ranks={ranks}")
    X, init = _data(dims, ranks, 3)
    ctx, dev = _ctx(to_dev_flat(X), init, dims, ranks)
    ref, _ = O.tr_als(X, init, 2)
    ctx.sweep(2, "f64", refine=1)
    got = cores_from_dev(dev, dims, ranks)
    for a, b in zip(got, ref):
        assert rel(a, b) <= 1e-10
    ctx.close()


def test_cfg1_fp64_per_sweep():
    """Config 1 at full size: 20^4, ranks 3, FP64 path, 10 sweeps; every sweep's
    cores within 1e-10 of the oracle's."""
    w = W.make_workload(1)
    say(f"[cfg1] {w.name}")
    X = w.X
    ctx, dev = _ctx(to_dev_flat(X), w.init_cores, w.dims, w.ranks)
    ref = [np.array(c) for c in w.init_cores]
    for s in range(w.sweeps):
        ref, _ = O.tr_als(X, ref, 1)
        ctx.sweep(1, "f64", refine=1)
        got = cores_from_dev(dev, w.dims, w.ranks)
        errs = [rel(a, b) for a, b in zip(got, ref)]
        say(f"   sweep {s + 1}: max core rel err {max(errs):.2e}")
        assert max(errs) <= 1e-10
    f_gpu = ctx.fit()
    f_ref = O.rel_error(X, ref)
    assert abs(f_gpu - f_ref) <= 1e-12 * max(1.0, f_ref) + 1e-13
    ctx.close()


def test_cfg2_reduced_fp32_per_sweep():
    """Config 2's recipe (Gaussian TR, R=10, 1% noise, FP32 storage) at 24^4:
    FP32 path, every sweep's cores within 1e-5 of the oracle's."""
    w = W.make_workload(2, dims=(24, 24, 24, 24))
    say(f"[cfg2 reduced] {w.dims}")
    X = w.X
    ctx, dev = _ctx(to_dev_flat(X), w.init_cores, w.dims, w.ranks)
    ref = [np.array(c) for c in w.init_cores]
    Xd = X.astype(np.float64)
    for s in range(4):
        ref, _ = O.tr_als(Xd, ref, 1)
        ctx.sweep(1, "f32", refine=1)
        got = cores_from_dev(dev, w.dims, w.ranks)
        errs = [rel(a, b) for a, b in zip(got, ref)]
        say(f"   sweep {s + 1}: max core rel err {max(errs):.2e}")
        assert max(errs) <= 1e-5
    ctx.close()


def test_cfg2_fullsize_first_sweep_fp32():
    """Config 2 at full size (100^4, R=10, FP32): the first sweep's cores from the
    same initial cores within 1e-5 of the oracle's (oracle ~10 s per mode)."""
    w = W.make_workload(2)
    say(f"[cfg2 full] {w.name}")
    X = w.X
    ctx, dev = _ctx(to_dev_flat(X), w.init_cores, w.dims, w.ranks)
    ctx.sweep(1, "f32", refine=1)
    got = cores_from_dev(dev, w.dims, w.ranks)
    ref, _ = O.tr_als(X.astype(np.float64), w.init_cores, 1)
    errs = [rel(a, b) for a, b in zip(got, ref)]
    say(f"   core rel errs {[f'{e:.2e}' for e in errs]}")
    assert max(errs) <= 1e-5
    ctx.close()


@pytest.mark.parametrize("dims,ranks", SHAPES[1:4], ids=[str(s[0]) for s in SHAPES[1:4]])
def test_fit_matches_oracle(dims, ranks):
    say(f"[fit] dims={dims}")
    X, init = _data(dims, ranks, 4)
    ctx, _ = _ctx(to_dev_flat(X), init, dims, ranks)
    assert ctx.xnorm2() == pytest.approx(float(np.sum(X * X)), rel=1e-12)
    assert ctx.fit() == pytest.approx(O.rel_error(X, init), rel=1e-11)
    ctx.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_mixed_schedule_final_fit(prec):
    """Mixed sweeps then FP32 finishing sweeps end within 1e-3 of the oracle's fit."""
    w = W.make_workload(2, dims=(28, 28, 28, 28), ranks=(6, 6, 6, 6))
    say(f"[mixed {prec}] {w.dims}")
    ctx, dev = _ctx(to_dev_flat(w.X), w.init_cores, w.dims, w.ranks)
    ctx.sweep(8, prec, refine=1)
    ctx.sweep(2, "f32", refine=1)
    f_gpu = ctx.fit()
    ref, _ = O.tr_als(w.X.astype(np.float64), w.init_cores, 10)
    f_ref = O.rel_error(w.X.astype(np.float64), ref)
    say(f"   fit gpu {f_gpu:.6e} oracle {f_ref:.6e}")
    assert abs(f_gpu - f_ref) <= 1e-3
    ctx.close()


def test_graph_replays_match_eager(monkeypatch):
    """Sweeps replayed from the captured graph equal eager sweeps bit for bit,
    replay after replay, with host synchronisation in between."""
    w = W.make_workload(2, dims=(20, 22, 18, 16), ranks=(4, 5, 3, 4))
    monkeypatch.setenv("TR_ALS_NO_GRAPH", "1")
    eager, de = _ctx(to_dev_flat(w.X), w.init_cores, w.dims, w.ranks)
    monkeypatch.delenv("TR_ALS_NO_GRAPH")
    graph, dg = _ctx(to_dev_flat(w.X), w.init_cores, w.dims, w.ranks)
    for prec in ("f32", "bf16", "fp8", "f32"):
        for rep in range(3):
            eager.sweep(1, prec, refine=1)
            graph.sweep(1, prec, refine=1)
            a = cores_from_dev(de, w.dims, w.ranks)
            b = cores_from_dev(dg, w.dims, w.ranks)
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (prec, rep)
    assert eager.graphs()[0] == 0
    n, note = graph.graphs()
    assert n == 3 and note == "", (n, note)   # f32, bf16 and fp8 sweeps were captured, not run eagerly
    eager.close()
    graph.close()


def test_singular_and_nonfinite_paths():
    import torch
    from paper_2210_11362_amd import TRError
    dims, ranks = (9, 8, 7), (2, 2, 2)
    X, init = _data(dims, ranks, 5)
    # X = 0: mode 1 gives G_1 = 0, so S_2 (built from G_1's Gram) is singular
    ctx, dev = _ctx(torch.zeros(int(np.prod(dims)), dtype=torch.float64, device="cuda"), init, dims, ranks)
    with pytest.raises(TRError) as ei:
        ctx.sweep(1, "f64")
    assert ei.value.code == -4
    got = cores_from_dev(dev, dims, ranks)
    assert np.all(got[0] == 0) and rel(got[1], init[1]) == 0.0   # last good update kept
    ctx.close()
    Xn = X.copy()
    Xn[3, 2, 1] = np.nan
    ctx, dev = _ctx(to_dev_flat(Xn), init, dims, ranks)
    with pytest.raises(TRError) as ei:
        ctx.sweep(1, "f64")
    assert ei.value.code == -5
    got = cores_from_dev(dev, dims, ranks)
    assert all(rel(a, b) == 0.0 for a, b in zip(got, init))
    # the context stays usable
    ctx.close()
