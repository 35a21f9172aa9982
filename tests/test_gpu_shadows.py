"""The BF16 and FP8 shadows of X, byte for byte, against encoders written from
the format definitions (``oracle/lowp_formats.py``): BF16 rounds each FP32
entry to nearest even; FP8 is OCP E4M3 of float32(x) * s with one scale per
tensor s = 448 / max|x|, nearest even.  Both layouts: X's own and the
transposed copy the slowest-modes contractions read."""
import numpy as np
import pytest

import workloads as W
from oracle.lowp_formats import bf16_bits, fp8_e4m3_bits, fp8_shadow_scale
from tests.gpu_util import cores_to_dev, say, to_dev_flat

pytestmark = pytest.mark.gpu

SHAPES = [((40, 36, 32, 30), (6, 6, 6, 6)),     # two-stage modes: a transposed shadow exists
          ((37, 29, 23), (3, 4, 2)),
          ((100, 100, 100, 100), (10, 10, 10, 10))]


@pytest.mark.parametrize("dims,ranks", SHAPES, ids=[str(s[0]) for s in SHAPES])
def test_shadow_bytes_match_format_definitions(dims, ranks):
    from paper_2210_11362_amd import TRContext
    g = np.random.default_rng(21)
    numel = int(np.prod(dims))
    X = np.asfortranarray((g.standard_normal(dims) * np.exp(g.uniform(-6, 3, dims))).astype(np.float32))
    init = W.gaussian_cores(dims, ranks, g)
    ctx = TRContext(to_dev_flat(X), dims, ranks, cores_to_dev(init))
    x = W.to_flat(X)
    b, sc, _ = ctx.shadow("bf16")
    got = b.cpu().numpy().view(np.uint16)
    want = bf16_bits(x)
    say(f"[shadows] dims={dims}: bf16 mismatches {int(np.sum(got != want))}")
    assert np.array_equal(got, want)
    f, sc, _ = ctx.shadow("fp8")
    s_ref = fp8_shadow_scale(x)
    say(f"   fp8 scale {sc!r} (format definition {s_ref!r})")
    assert np.float32(sc) == s_ref
    want8 = fp8_e4m3_bits(x * np.float32(sc))
    got8 = f.cpu().numpy()
    bad = np.nonzero(got8 != want8)[0]
    say(f"   fp8 mismatches {bad.size}" + (f", first at {bad[0]}: x*s={x[bad[0]] * sc!r} "
                                            f"got {got8[bad[0]]:#x} want {want8[bad[0]]:#x}" if bad.size else ""))
    assert bad.size == 0
    assert np.sum((want8 & 0x78) == 0) > 0 or numel < 10 ** 5      # subnormal codes are exercised
    # the transposed copies, where the context keeps them
    try:
        bt, _, K = ctx.shadow("bf16", transposed=True)
    except Exception:
        K = 0
    if K:
        Mr = numel // K
        xt = x.reshape((K, Mr)).T.ravel()     # out[k + K r] = X[r + M k]
        assert np.array_equal(bt.cpu().numpy().view(np.uint16), bf16_bits(xt))
        ft, sct, K2 = ctx.shadow("fp8", transposed=True)
        assert K2 == K and sct == sc
        assert np.array_equal(ft.cpu().numpy(), fp8_e4m3_bits(xt * np.float32(sc)))
        say(f"   transposed shadows (K = {K}) match")
    ctx.close()
