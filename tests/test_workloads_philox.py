"""Pins of the counter-based input generator used by the serving jobs
(``workloads/philox.py``): the published Philox4x32-10 known-answer vectors,
the Box-Muller pairing, the moments of the normals, and the planted-job recipe
(noise-free part = the TR of the true cores; relative noise level = eta)."""
import math
import os

import numpy as np
import pytest

import workloads as W
from workloads import philox as PH

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        line = line.split("#")[0].split()
        if line:
            v = [int(x, 16) for x in line]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = PH.philox4x32_10(np.array([ctr], dtype=np.uint64), key)[0]
        assert [int(x) for x in got] == out


def test_normals_pairing_and_offsets():
    seed = 0x123456789ABCDEF
    z = PH.philox_normals(seed, 7, 1000)
    # any window of the stream is the same numbers
    assert np.array_equal(PH.philox_normals(seed, 7, 10, start=500), z[500:510])
    # a Box-Muller pair shares its radius: z0^2 + z1^2 = -2 ln u of the pair's word
    ctr = np.array([[3, 0, 7, 0]], dtype=np.uint64)
    w = PH.philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))[0]
    u = ((((int(w[1]) << 32) | int(w[0])) >> 11) + 0.5) * 2.0 ** -53
    assert z[6] ** 2 + z[7] ** 2 == pytest.approx(-2.0 * math.log(u), rel=1e-13)
    # different streams and keys give different numbers
    assert not np.allclose(PH.philox_normals(seed, 8, 1000), z)
    assert not np.allclose(PH.philox_normals(seed + 1, 7, 1000), z)


def test_normals_moments():
    z = PH.philox_normals(2024, 0, 400_000)
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 0.05
    # fraction within one standard deviation (0.6827)
    assert abs(np.mean(np.abs(z) < 1.0) - 0.682689) < 0.005


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_planted_job_recipe(dtype):
    dims, ranks, seed = (9, 7, 8, 5), (2, 3, 2, 3), 99
    X0, true, init = PH.planted_job(dims, ranks, seed, 0.0, dtype)
    xt = W.planted_tensor(true)
    assert np.array_equal(X0, xt.astype(dtype))
    for k, c in enumerate(true):
        assert c.shape == (ranks[k], dims[k], ranks[(k + 1) % 4])
        assert np.array_equal(W.to_flat(c), PH.philox_normals(seed, PH.SID_TRUE + k, c.size))
        assert np.array_equal(W.to_flat(init[k]), PH.philox_normals(seed, PH.SID_INIT + k, c.size))
    eta = 0.05
    X, _, _ = PH.planted_job(dims, ranks, seed, eta, dtype)
    rel = np.linalg.norm((X.astype(np.float64) - xt).ravel()) / np.linalg.norm(xt.ravel())
    assert rel == pytest.approx(eta, rel=1e-4 if dtype == np.float32 else 1e-12)
