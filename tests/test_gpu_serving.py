"""Serving loop and device generator, through the C ABI.

* The device generator of planted jobs equals its host definition
  (``workloads/philox.py``) up to the last bits of FP64 transcendental
  functions and summation order.
* A served job equals the oracle's regular ALS from the same inputs (FP64
  path: <= 1e-10 per core, the FP64 tolerance).
* Every job's result is the same alone and in a concurrent mix: bitwise, as
  all kernels are deterministic (the stated gate is the precision tolerance).
* Admission respects the HBM budget; a failing job does not disturb others.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads import philox as PH
from tests.gpu_util import cores_to_dev, rel, say, to_dev_flat

pytestmark = pytest.mark.gpu

GB = 1 << 30


def _flat_np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("dims,ranks,dtype", [
    ((13, 9, 11), (3, 4, 2), "f32"),
    ((6, 5, 7, 4, 5), (2, 3, 2, 2, 3), "f64"),
    ((33, 17), (3, 5), "f32"),
    ((40, 36, 20), (6, 6, 6), "f64"),
])
def test_device_generator_matches_host_definition(dims, ranks, dtype):
    import torch
    from paper_2210_11362_amd import gen_planted
    say(f"[gen] dims={dims} ranks={ranks} {dtype}")
    seed, eta = 0xC0FFEE + len(dims), 0.05
    tdt = torch.float32 if dtype == "f32" else torch.float64
    X, true, init = gen_planted(dims, ranks, seed, eta, tdt, want_true=True, want_init=True)
    torch.cuda.synchronize()
    Xh, true_h, init_h = PH.planted_job(dims, ranks, seed, eta, np.float32 if dtype == "f32" else np.float64)
    for a, b in zip(true, true_h):
        assert np.allclose(_flat_np(a), W.to_flat(b), rtol=1e-14, atol=1e-14)
    for a, b in zip(init, init_h):
        assert np.allclose(_flat_np(a), W.to_flat(b), rtol=1e-14, atol=1e-14)
    xd = _flat_np(X).astype(np.float64)
    xh = W.to_flat(Xh).astype(np.float64)
    scale = np.max(np.abs(xh))
    if dtype == "f32":
        # X_true and the noisy sum are rounded to FP32 twice: at most one
        # rounding step apart where FP64 evaluation order flips a tie
        tol = 2.0 ** -22 * np.abs(xh) + 1e-12 * scale
    else:
        tol = 1e-13 * scale
    assert np.all(np.abs(xd - xh) <= tol)
    # the realised relative noise is eta (of the rounded planted part)
    assert rel(xh, W.to_flat(W.planted_tensor(true_h))) == pytest.approx(eta, rel=1e-3)


def _server(budget=4 * GB, slots=4):
    from paper_2210_11362_amd import TRServer
    return TRServer(budget, slots)


def test_served_job_matches_oracle_fp64():
    dims, ranks, seed, eta = (10, 9, 8), (2, 3, 2), 4242, 0.02
    say(f"[serve f64 generated] dims={dims}")
    X, _, init = PH.planted_job(dims, ranks, seed, eta, np.float64)
    ref, _ = O.tr_als(X, init, 3)
    srv = _server()
    jid = srv.submit(dims, ranks, seed=seed, eta=eta, prec_mixed="f64", nsweeps_mixed=3, prec_fin="f64",
                     nsweeps_fin=0, x_dtype="f64")
    info = srv.wait(jid)
    assert info["state"] == 2, srv.error(jid)
    got = srv.result(jid, dims, ranks)
    errs = [rel(a, b) for a, b in zip(got, ref)]
    say(f"   core rel errs {errs}")
    assert max(errs) <= 1e-10
    assert abs(info["rel_err"] - O.rel_error(X, ref)) <= 1e-10
    srv.close()


def test_served_job_with_caller_inputs_matches_oracle():
    dims, ranks = (14, 12, 9, 7), (3, 2, 4, 2)
    say(f"[serve caller inputs] dims={dims}")
    g = np.random.default_rng(77)
    true = W.gaussian_cores(dims, ranks, g)
    X = np.asfortranarray(W.add_noise(W.planted_tensor(true), 0.01, g))
    init = W.gaussian_cores(dims, ranks, g)
    ref, _ = O.tr_als(X, init, 2)
    Xd = to_dev_flat(X)
    cd = cores_to_dev(init)
    srv = _server()
    jid = srv.submit(dims, ranks, prec_mixed="f64", nsweeps_mixed=2, nsweeps_fin=0, X=Xd, init_cores=cd)
    info = srv.wait(jid)
    assert info["state"] == 2, srv.error(jid)
    got = srv.result(jid, dims, ranks)
    assert max(rel(a, b) for a, b in zip(got, ref)) <= 1e-10
    # the caller's initial cores are only read
    assert all(rel(a.cpu().numpy(), W.to_flat(b)) == 0.0 for a, b in zip(cd, init))
    srv.close()


def _mix_jobs():
    g = np.random.default_rng(5)
    jobs = []
    for k in range(12):
        N = int(g.integers(3, 6))
        dims = tuple(int(v) for v in g.integers(8, 30 if N < 5 else 14, size=N))
        R = int(g.integers(2, 7))
        jobs.append(dict(dims=dims, ranks=(R,) * N, seed=1000 + k))
    return jobs


def test_results_identical_alone_and_in_mix():
    jobs = _mix_jobs()
    kw = dict(eta=0.01, prec_mixed="bf16", nsweeps_mixed=4, prec_fin="f32", nsweeps_fin=2)
    alone = []
    srv = _server(slots=1)
    for j in jobs:
        say(f"[alone] dims={j['dims']} R={j['ranks'][0]}")
        jid = srv.submit(j["dims"], j["ranks"], seed=j["seed"], **kw)
        info = srv.wait(jid)
        assert info["state"] == 2, srv.error(jid)
        alone.append((srv.result(jid, j["dims"], j["ranks"]), info["rel_err"]))
    srv.close()
    say("[mix] 12 jobs, 6 slots")
    srv = _server(slots=6)
    ids = [srv.submit(j["dims"], j["ranks"], seed=j["seed"], t_arrival=0.002 * k, **kw) for k, j in enumerate(jobs)]
    srv.drain()
    st = srv.stats()
    say(f"   stats {st}")
    assert st["done"] == len(jobs) and st["failed"] == 0
    assert st["max_running"] >= 2
    for j, jid, (cores_a, fit_a) in zip(jobs, ids, alone):
        info = srv.poll(jid)
        assert info["state"] == 2
        cores_m = srv.result(jid, j["dims"], j["ranks"])
        for a, b in zip(cores_a, cores_m):
            assert np.array_equal(a, b)
        assert info["rel_err"] == fit_a
        assert np.isfinite(fit_a) and fit_a < 1.0
    srv.close()


def test_admission_respects_hbm_budget():
    from paper_2210_11362_amd import TRError
    dims, ranks = (40, 40, 40, 40), (5, 5, 5, 5)
    kw = dict(eta=0.01, prec_mixed="bf16", nsweeps_mixed=2, prec_fin="f32", nsweeps_fin=1)
    srv = _server(slots=1)
    jid = srv.submit(dims, ranks, seed=1, **kw)
    info = srv.wait(jid)
    assert info["state"] == 2, srv.error(jid)
    F = info["footprint"]
    srv.close()
    # X (FP32) + BF16 shadow are part of the footprint
    assert F >= 40 ** 4 * 6
    say(f"[admission] footprint {F} bytes; budget {int(2.5 * F)}")
    srv = _server(budget=int(2.5 * F), slots=8)
    ids = [srv.submit(dims, ranks, seed=10 + k, **kw) for k in range(6)]
    with pytest.raises(TRError):
        srv.submit((60, 60, 60, 60), ranks, seed=2, **kw)     # can never fit
    srv.drain()
    st = srv.stats()
    say(f"   stats {st}")
    assert st["done"] == 6
    assert st["peak_in_use"] <= st["arena_bytes"]
    assert st["max_running"] == 2
    # arrival order is kept: admissions are non-decreasing in job id
    adm = [srv.poll(j)["t_admit"] for j in ids]
    assert adm == sorted(adm)
    srv.close()


def test_failed_job_does_not_disturb_others():
    import torch
    dims, ranks = (9, 8, 7), (2, 2, 2)
    srv = _server(slots=2)
    zeros = torch.zeros(9 * 8 * 7, dtype=torch.float64, device="cuda")
    bad = srv.submit(dims, ranks, seed=3, prec_mixed="f64", nsweeps_mixed=1, nsweeps_fin=0, X=zeros)
    good = srv.submit(dims, ranks, seed=3, prec_mixed="f64", nsweeps_mixed=2, nsweeps_fin=0, x_dtype="f64")
    srv.drain()
    ib, ig = srv.poll(bad), srv.poll(good)
    assert ib["state"] == 3 and ib["status"] == -4, srv.error(bad)
    assert "positive definite" in srv.error(bad)
    assert ig["state"] == 2 and 0.0 < ig["rel_err"] < 1.0
    srv.close()


# ---------------------------------------------------------------------------
# Batched lane: small jobs (order <= 4, ranks <= 8, mode sizes <= 128, at most
# 2^18 entries) run whole inside one persistent workgroup each, many per launch.
# ---------------------------------------------------------------------------

def _batch_server(budget=4 * GB, slots=4):
    from paper_2210_11362_amd import TRServer
    return TRServer(budget, slots, batch=True)


LANE_JOBS = [((12, 10, 9), (2, 3, 2)), ((9, 8, 7, 6), (2, 2, 3, 2)), ((20, 17, 15), (4, 3, 5)),
             ((16, 12, 10, 8), (3, 4, 3, 2)), ((30, 25), (3, 4)), ((24, 20, 18), (6, 5, 4))]


def test_batched_lane_matches_oracle_fp64():
    srv = _batch_server()
    ids = []
    for k, (dims, ranks) in enumerate(LANE_JOBS):
        ids.append(srv.submit(dims, ranks, seed=500 + k, eta=0.02, prec_mixed="f64", nsweeps_mixed=3,
                              prec_fin="f64", nsweeps_fin=0, x_dtype="f64"))
    srv.drain()
    for k, ((dims, ranks), jid) in enumerate(zip(LANE_JOBS, ids)):
        info = srv.poll(jid)
        say(f"[lane f64] dims={dims} ranks={ranks} state={info['state']} batched={info['batched']}")
        assert info["state"] == 2, srv.error(jid)
        assert info["batched"]
        X, _, init = PH.planted_job(dims, ranks, 500 + k, 0.02, np.float64)
        ref, _ = O.tr_als(X, init, 3)
        got = srv.result(jid, dims, ranks)
        errs = [rel(a, b) for a, b in zip(got, ref)]
        say(f"   core rel errs max {max(errs):.2e}; fit {info['rel_err']:.6e} vs {O.rel_error(X, ref):.6e}")
        assert max(errs) <= 1e-10
        assert abs(info["rel_err"] - O.rel_error(X, ref)) <= 1e-10
    srv.close()


def test_batched_lane_mixed_schedule_fit():
    srv = _batch_server()
    ids = [srv.submit(dims, ranks, seed=600 + k, eta=0.01, prec_mixed="bf16", nsweeps_mixed=6, prec_fin="f32",
                      nsweeps_fin=2) for k, (dims, ranks) in enumerate(LANE_JOBS)]
    srv.drain()
    for k, ((dims, ranks), jid) in enumerate(zip(LANE_JOBS, ids)):
        info = srv.poll(jid)
        assert info["state"] == 2 and info["batched"], srv.error(jid)
        X, _, init = PH.planted_job(dims, ranks, 600 + k, 0.01, np.float32)
        Xd = X.astype(np.float64)
        ref, _ = O.tr_als(Xd, init, 8)
        f_ref = O.rel_error(Xd, ref)
        say(f"[lane mixed] dims={dims} fit gpu {info['rel_err']:.6e} oracle {f_ref:.6e}")
        assert abs(info["rel_err"] - f_ref) <= 1e-3
    srv.close()


def test_batched_results_identical_alone_and_in_batch():
    kw = dict(eta=0.01, prec_mixed="bf16", nsweeps_mixed=4, prec_fin="f32", nsweeps_fin=2)
    srv = _batch_server()
    alone = []
    for k, (dims, ranks) in enumerate(LANE_JOBS):
        jid = srv.submit(dims, ranks, seed=700 + k, **kw)
        info = srv.wait(jid)
        assert info["state"] == 2 and info["batched"], srv.error(jid)
        alone.append((srv.result(jid, dims, ranks), info["rel_err"]))
    # now all together (one batch), behind a job that takes the per-job path
    big = srv.submit((60, 50, 40), (10, 10, 10), seed=1, **kw)
    ids = [srv.submit(dims, ranks, seed=700 + k, **kw) for k, (dims, ranks) in enumerate(LANE_JOBS)]
    srv.drain()
    ib = srv.poll(big)
    assert ib["state"] == 2 and not ib["batched"], srv.error(big)
    for (dims, ranks), jid, (cores_a, fit_a) in zip(LANE_JOBS, ids, alone):
        info = srv.poll(jid)
        assert info["state"] == 2
        for a, b in zip(cores_a, srv.result(jid, dims, ranks)):
            assert np.array_equal(a, b)
        assert info["rel_err"] == fit_a
    srv.close()
