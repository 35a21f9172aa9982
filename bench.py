"""Benchmark of the TR-ALS sweep on one MI355X.

Workload: order-4 tensor 100x100x100x100 (FP32 storage) built as a TR of
Gaussian cores with ranks 10 plus 1% relative Gaussian noise, fit ranks 10,
normal-equation variant.  A step is one ALS sweep (N = 4 mode updates: X
stream, Gram ring, FP64 Cholesky solve with one refinement step, Gram refresh)
with the X contraction in BF16 (the mixed-precision path).  Also reported:
the plain FP32 sweep, the 20-sweep schedules (18 BF16 + 2 FP32 finishing vs
20 FP32) and their final fits, the roofline of the X-stream kernel measured
with HIP events on the library's stream, and the CPU oracle timed on a bounded
sample.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
XBYTES = {"f32": 4, "f64": 8, "bf16": 2, "fp8": 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="bf16", choices=["f32", "bf16", "fp8", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-schedules", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-qr", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the legs on the other workloads (20^4 FP64, 40^5 conditioned, 512x512x256 field)")
    ap.add_argument("--configs", default="1,3,4",
                    help="which of the other workloads to run (comma list of 1, 3, 4)")
    ap.add_argument("--serving-full", action="store_true",
                    help="serving leg on the full stream distribution: orders 3-5, modes 16-128, ranks 2-12, "
                         "batch lanes on")
    ap.add_argument("--serving-jobs", type=int, default=400)
    ap.add_argument("--serving-only", action="store_true",
                    help="only run the serving stream and print its JSON (the bench runs it in a child process)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (the X stream of one GPU "
              "is the unit; see the sharding notes shipped with the package)", file=sys.stderr)
        sys.exit(2)

    if args.serving_only:
        print(json.dumps(serving_leg(args.serving_jobs, args.serving_full)))
        return
    import torch
    if args.copy_probe:
        n = 1 << 28                      # 2^28 float32 = 1 GiB read + 1 GiB written per copy
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "copies": 3}))
        return
    import workloads as W
    from paper_2210_11362_amd import TRContext

    def to_dev_flat(a):
        return torch.from_numpy(W.to_flat(np.asarray(a))).cuda()

    def cores_to_dev(cs):
        return [to_dev_flat(np.asarray(c, dtype=np.float64)) for c in cs]

    cfg = 2
    w = W.make_workload(cfg, seed=0)
    dims, ranks, N = w.dims, w.ranks, len(w.dims)
    X = to_dev_flat(w.X)
    init = w.init_cores

    def fresh(variant="ne"):
        dev = cores_to_dev(init)
        return TRContext(X, dims, ranks, dev, variant=variant), dev

    # ---- timed steps: K sweeps in the chosen precision --------------------
    # Throughput: the K sweeps issued as one tr_als_sweep call, the way a
    # decomposition job runs them (every sweep executed in full; the library
    # synchronises once at the end to read its status word).
    ctx, dev = fresh()
    ctx.sweep(args.warmup, args.prec, refine=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.sweep(args.steps, args.prec, refine=1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    ms_per_step = 1000.0 * wall / args.steps
    # Latency: K single-sweep calls, each ending with the status synchronisation.
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for e0, e1 in evs:
        e0.record()
        ctx.sweep(1, args.prec, refine=1)
        e1.record()
    torch.cuda.synchronize()
    per = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    p50 = per[len(per) // 2]
    p99 = per[min(len(per) - 1, int(round(0.99 * (len(per) - 1))))]

    # ---- roofline of the X-stream kernel (HIP events on the library stream) --
    regimes = sorted({ctx.regime(n) for n in range(1, N + 1)})
    kname = {1: "xgemm_kernel (two-stage X contraction, stage 1)", 2: "xstream_kernel (fused X contraction)",
             3: "xslab_kernel (slab X contraction, order 3)"}
    ctx.profile_enable(True)
    ctx.sweep(3, args.prec, refine=1)
    kms, nl, bpl = ctx.profile_read()
    ctx.profile_enable(False)
    avg_kernel_s = (kms / max(nl, 1)) / 1000.0
    algo_bytes = float(w.numel) * XBYTES[args.prec]
    achieved_gbs = algo_bytes / avg_kernel_s / 1e9
    flops_launch = 2.0 * w.numel * ranks[0] * ranks[1]
    achieved_tf = flops_launch / avg_kernel_s / 1e12
    bound = "hbm"
    if args.prec == "f32" and flops_launch / algo_bytes > MFMA_PEAK_TFLOPS["f32"] * 1e12 / (HBM_PEAK_GBS * 1e9):
        bound = "mfma"
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic() if args.prec == "bf16" else None}
    else:
        roof = {"bound": "mfma", "achieved": round(achieved_tf, 2), "peak": MFMA_PEAK_TFLOPS["f32"],
                "unit": "TFLOP/s", "frac": round(achieved_tf / MFMA_PEAK_TFLOPS["f32"], 4), "traffic": None}
    roof.update({"kernel": " + ".join(kname[r] for r in regimes), "avg_kernel_us": round(avg_kernel_s * 1e6, 2),
                 "launches": nl, "algo_bytes_per_launch": algo_bytes, "flops_per_launch": flops_launch,
                 "achieved_tflops": round(achieved_tf, 2)})
    ctx.close()

    extra = {}
    # ---- plain FP32 sweep and the two 20-sweep schedules at equal fit --------
    if not args.no_schedules:
        ctx, dev = fresh()
        ctx.sweep(1, "f32", refine=1)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ctx.sweep(5, "f32", refine=1)
        tb = time.perf_counter()
        extra["plain_f32_ms_per_sweep"] = round(1000 * (tb - ta) / 5, 4)
        extra["plain_f32_roofline"] = kernel_roofline(ctx, "f32", w.numel, ranks[0] * ranks[1])
        for p in ("f64", "fp8"):
            ctx.sweep(1, p, refine=1)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            ctx.sweep(3, p, refine=1)
            tb = time.perf_counter()
            extra[f"{p}_path_ms_per_sweep"] = round(1000 * (tb - ta) / 3, 4)
        ctx.close()
        sched = {}
        for name, plan in (("mixed", [(args.prec, w.sweeps - 2), ("f32", 2)]), ("plain", [("f32", w.sweeps)])):
            ctx, dev = fresh()
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for p, k in plan:
                ctx.sweep(k, p, refine=1)
            tb = time.perf_counter()
            sched[name] = {"sweeps": sum(k for _, k in plan), "plan": [f"{k}x{p}" for p, k in plan],
                           "seconds": round(tb - ta, 5), "fit": ctx.fit()}
            ctx.close()
        sched["fit_delta"] = abs(sched["mixed"]["fit"] - sched["plain"]["fit"])
        sched["speedup_mixed_vs_plain"] = round(sched["plain"]["seconds"] / sched["mixed"]["seconds"], 3)
        extra["schedules_20_sweeps"] = sched

    # ---- the QR-based variants (Alg. 3 and Alg. 4) on the same workload -----
    if not args.no_qr:
        for variant in ("qr", "qrne"):
            try:
                qr = {}
                for p in ("f32", args.prec):
                    ctx, dev = fresh(variant)
                    ctx.sweep(1, p, refine=1)
                    torch.cuda.synchronize()
                    ta = time.perf_counter()
                    ctx.sweep(3, p, refine=1)
                    tb = time.perf_counter()
                    qr[f"{p}_ms_per_sweep"] = round(1000 * (tb - ta) / 3, 4)
                    qr[f"{p}_fit_after_4_sweeps"] = ctx.fit()
                    ctx.close()
                extra[f"{variant}_variant"] = qr
            except Exception as e:   # reported, never fatal to the bench line
                extra[f"{variant}_variant"] = {"error": str(e)[:200]}

    # ---- the other workloads ------------------------------------------------
    if not args.no_configs:
        extra["other_workloads"] = config_legs({int(v) for v in args.configs.split(",") if v.strip()})

    # ---- serving: a Poisson stream of small jobs through the request loop ---
    if not args.no_serving and args.serving_jobs > 0:
        extra["serving"] = serving_child(args.serving_jobs, args.serving_full)

    # ---- CPU oracle on a bounded sample ------------------------------------
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        try:
            nthreads = len(os.sched_getaffinity(0))
        except Exception:
            nthreads = os.cpu_count() or 1
        Xd = w.X.astype(np.float64)
        ta = time.perf_counter()
        O.als_update(Xd, init, 1)
        tb = time.perf_counter()
        t_mode = tb - ta
        cpu = {"value": round(1.0 / (N * t_mode), 6), "unit": "sweeps/s", "cores": nthreads, "kind": "oracle",
               "sample": "one regular-ALS mode update (mode 1, explicit subchain + Householder QR) of the full "
                         f"100^4 tensor in FP64 numpy/LAPACK, {t_mode:.2f} s, scaled x{N} to one sweep",
               "cpu_model": cpu_model(), "blas": blas_name()}

    out = {
        "metric": "TR-ALS sweep time, % roofline, mixed vs plain at equal fit; p50/p99 latency",
        "value": round(args.steps / wall, 4),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "timing": "value/ms_per_step: the K sweeps as one tr_als_sweep call (one status sync); "
                  "sweep_ms_p50/p99: K single-sweep calls, each with its status sync",
        "sweep_ms_p50": round(p50, 4),
        "sweep_ms_p99": round(p99, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "order-4 100x100x100x100 FP32 tensor, Gaussian TR ranks 10 + 1% noise, "
                               "fit ranks 10, NE variant, one sweep per step",
                   "dims": list(dims), "ranks": list(ranks), "variant": "ne", "refine_steps": 1},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def blas_name():
    try:
        cfg = np.show_config(mode="dicts")["Build Dependencies"]["blas"]
        return f"{cfg.get('name')} {cfg.get('version', '')}".strip()
    except Exception:
        return None


def kernel_roofline(ctx, prec, numel, C, sweeps=2):
    """Average duration (HIP events on the library stream) of the X-contraction
    launches of `sweeps` sweeps in `prec`, with achieved GB/s and TFLOP/s against
    the HBM and the precision's MFMA peak (algorithmic bytes = numel x bytes as
    read; flops = 2 numel R_n R_{n+1})."""
    ctx.profile_enable(True)
    ctx.sweep(sweeps, prec, refine=1)
    kms, nl, bpl = ctx.profile_read()
    ctx.profile_enable(False)
    t = (kms / max(nl, 1)) / 1000.0
    gbs = numel * XBYTES[prec] / t / 1e9
    tfl = 2.0 * numel * C / t / 1e12
    hbm_time = numel * XBYTES[prec] / (HBM_PEAK_GBS * 1e9)
    mfma_time = 2.0 * numel * C / (MFMA_PEAK_TFLOPS[prec] * 1e12)
    bound = "hbm" if hbm_time >= mfma_time else "mfma"
    return {"bound": bound, "avg_kernel_us": round(t * 1e6, 2), "launches": nl, "achieved_gbs": round(gbs, 1),
            "achieved_tflops": round(tfl, 2),
            "frac": round((hbm_time if bound == "hbm" else mfma_time) / t, 4),
            "peak": HBM_PEAK_GBS if bound == "hbm" else MFMA_PEAK_TFLOPS[prec],
            "unit": "GB/s" if bound == "hbm" else "TFLOP/s"}


def config_legs(which=(1, 3, 4)):
    """Sweep times (and rooflines of the X contraction) on the other workloads:
    20^4 ranks 3 FP64 (all variants, FP64 path); the conditioned order-5 40^5
    ranks (6,8,10,8,6) (NE / QR / QRNE, BF16 and FP8 mixed schedules of 18 + 2
    FP32 finishing sweeps, final fits beside the all-FP32 schedule); the
    512x512x256 sinusoid field at ranks 20 (FP32 vs 28 BF16 or 28 FP8 + 2
    FP32).  Every leg is reported, never fatal."""
    import torch
    import workloads as W
    from paper_2210_11362_amd import TRContext

    def dev_flat(a):
        return torch.from_numpy(W.to_flat(np.asarray(a))).cuda()

    def timed(ctx, k, p):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ctx.sweep(k, p, refine=1)
        torch.cuda.synchronize()
        return time.perf_counter() - ta

    def leg(fn):
        try:
            return fn()
        except Exception as e:
            return {"error": str(e)[:240]}

    out = {}
    if 1 in which:
        out["cfg1_20x4_R3_f64"] = leg(lambda: cfg1_leg(W, TRContext, dev_flat, timed))
    if 3 in which:
        out["cfg3_40x5_cond1e4"] = leg(lambda: cfg3_leg(W, TRContext, dev_flat, timed, leg))
    if 4 in which:
        out["cfg4_512x512x256_R20"] = leg(lambda: cfg4_leg(W, TRContext, dev_flat, timed))
    return out


def cfg1_leg(W, TRContext, dev_flat, timed):
    w1 = W.make_workload(1)
    X1 = dev_flat(w1.X)

    def cfg1():
        r = {"workload": "20^4 FP64, Gaussian TR ranks 3 + 0.1% noise, fit ranks 3, FP64 path, 10 sweeps"}
        for v in ("ne", "qr", "qrne"):
            ctx = TRContext(X1, w1.dims, w1.ranks, [dev_flat(c) for c in w1.init_cores], variant=v)
            ctx.sweep(1, "f64")
            dt = timed(ctx, 10, "f64")
            r[v] = {"ms_per_sweep": round(1000 * dt / 10, 4), "sweeps_per_s": round(10 / dt, 1), "fit": ctx.fit()}
            ctx.close()
        return r
    return cfg1()


def cfg3_leg(W, TRContext, dev_flat, timed, leg):
    w3 = W.make_workload(3)
    X3 = dev_flat(w3.X)

    def cfg3():
        r = {"workload": "40^5 FP32, TR cores of condition 1e4, ranks (6,8,10,8,6), 1% noise; 20 sweeps"}
        ctx = TRContext(X3, w3.dims, w3.ranks, [dev_flat(c) for c in w3.init_cores])
        dt = timed(ctx, 20, "f32")
        r["plain_f32"] = {"ms_per_sweep": round(1000 * dt / 20, 4), "fit": ctx.fit()}
        ctx.close()
        for v in ("ne", "qr", "qrne"):
            for p in ("bf16", "fp8"):
                def one():
                    ctx = TRContext(X3, w3.dims, w3.ranks, [dev_flat(c) for c in w3.init_cores], variant=v)
                    try:
                        dt = timed(ctx, 18, p)
                        dt2 = timed(ctx, 2, "f32")
                        res = {"ms_per_mixed_sweep": round(1000 * dt / 18, 4), "seconds_20": round(dt + dt2, 4),
                               "fit": ctx.fit()}
                        res["fit_delta_vs_plain"] = abs(res["fit"] - r["plain_f32"]["fit"])
                        if v == "ne":
                            res["roofline"] = kernel_roofline(ctx, p, w3.numel, max(
                                w3.ranks[k] * w3.ranks[(k + 1) % 5] for k in range(5)), sweeps=1)
                        return res
                    finally:
                        ctx.close()
                r[f"{v}_{p}"] = leg(one)
        def pinv_fp8():
            ctx = TRContext(X3, w3.dims, w3.ranks, [dev_flat(c) for c in w3.init_cores])
            try:
                ctx.set_solve("pinv")
                dt = timed(ctx, 18, "fp8")
                timed(ctx, 2, "f32")
                f = ctx.fit()
                return {"ms_per_mixed_sweep": round(1000 * dt / 18, 4), "fit": f,
                        "fit_delta_vs_plain": abs(f - r["plain_f32"]["fit"])}
            finally:
                ctx.close()
        r["ne_fp8_pinv_solve"] = leg(pinv_fp8)
        return r
    return cfg3()


def cfg4_leg(W, TRContext, dev_flat, timed):
    w4 = W.make_workload(4)
    X4 = dev_flat(w4.X)

    def cfg4():
        r = {"workload": "512x512x256 FP32 sinusoid field (50 terms) + 2% noise, fit ranks 20, 30 sweeps, NE"}
        for name, plan in (("mixed", [("bf16", 28), ("f32", 2)]), ("mixed_fp8", [("fp8", 28), ("f32", 2)]),
                           ("plain", [("f32", 30)])):
            ctx = TRContext(X4, w4.dims, w4.ranks, [dev_flat(c) for c in w4.init_cores])
            tot = 0.0
            per = {}
            for p, k in plan:
                dt = timed(ctx, k, p)
                tot += dt
                per[p] = round(1000 * dt / k, 4)
            r[name] = {"plan": [f"{k}x{p}" for p, k in plan], "seconds": round(tot, 4), "ms_per_sweep": per,
                       "fit": ctx.fit()}
            r[name]["roofline_" + plan[0][0]] = kernel_roofline(ctx, plan[0][0], w4.numel, 400, sweeps=1)
            ctx.close()
        r["fit_delta"] = abs(r["mixed"]["fit"] - r["plain"]["fit"])
        r["speedup_mixed_vs_plain"] = round(r["plain"]["seconds"] / r["mixed"]["seconds"], 3)
        r["fit_delta_fp8"] = abs(r["mixed_fp8"]["fit"] - r["plain"]["fit"])
        return r
    return cfg4()


def xgemm_source_sha():
    """sha256 of the X-contraction kernel source and of the code that picks its
    launch configuration (xg_config: tiles, split-K count, grid)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2210_11362_amd", "csrc")
    kern = open(os.path.join(csrc, "k_xgemm.hip"), "rb").read()
    host = open(os.path.join(csrc, "tr_als.hip"), "rb").read()
    a = host.index(b"XgArgs xg_config(")
    b = host.index(b"\n}\n", a)
    return hashlib.sha256(kern + host[a:b]).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the BF16 X-contraction kernel on this workload,
    from the committed FETCH_SIZE / WRITE_SIZE counter summary (copy-calibrated);
    None when the kernel or its launch configuration changed since the counters
    were taken."""
    prof = os.path.join(ROOT, "profiles", "xgemm_bf16_100x4_R10_hbm_counters.md")
    try:
        fields = dict(l.split(":", 1) for l in open(prof) if l.startswith(("traffic_bytes_per_launch:",
                                                                            "kernel_source_sha256:")))
        if fields["kernel_source_sha256"].strip() != xgemm_source_sha():
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def serving_child(njobs: int, full: bool = False):
    """The serving stream in a child process (its own device context): a failure
    there is reported in the bench line instead of ending the bench."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--serving-only", "--serving-jobs", str(njobs)]
    if full:
        cmd.append("--serving-full")
    try:
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=900)
    except subprocess.TimeoutExpired:
        return {"error": "serving stream timed out after 900 s"}
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    if p.returncode != 0 or not lines:
        return {"error": f"serving stream exited with status {p.returncode}", "stderr_tail": p.stderr[-400:]}
    return json.loads(lines[-1])


def serving_leg(njobs: int, full: bool = False):
    """Latency and throughput of the request loop on a Poisson stream (200 jobs/s)
    of planted-TR jobs (8 BF16 + 2 FP32 sweeps each), generated on the device.
    Default: orders 3-4, mode sizes 16-48, ranks 2-8, 8 slots, 16 GiB arena.
    full: the whole distribution -- orders 3-5, mode sizes 16-128, ranks 2-12 --
    with batch lanes on, 8 slots, 240 GiB arena."""
    import numpy as np
    import workloads as W
    from paper_2210_11362_amd import TRServer
    if full:
        jobs = W.serving_stream(njobs)
        srv = TRServer(240 << 30, 8, batch=True)
        desc = f"{njobs} jobs, Poisson 200/s, order 3-5, dims 16-128, ranks 2-12, 8xbf16+2xf32 sweeps, lanes on"
    else:
        jobs = W.serving_stream(njobs, orders=(3, 4), dim_range=(16, 48), rank_range=(2, 8))
        srv = TRServer(16 << 30, 8)
        desc = f"{njobs} jobs, Poisson 200/s, order 3-4, dims 16-48, ranks 2-8, 8xbf16+2xf32 sweeps"
    t_submit0 = time.perf_counter()
    from paper_2210_11362_amd import TRError
    ids, refused = [], 0
    for j in jobs:
        try:
            ids.append(srv.submit(j["dims"], j["ranks"], seed=j["seed"], eta=0.01, prec_mixed="bf16",
                                  nsweeps_mixed=8, prec_fin="f32", nsweeps_fin=2, t_arrival=0.05 + j["t_arrive"]))
        except TRError:
            refused += 1          # footprint larger than the whole arena
    # wait for the stream to finish, with a progress line every ~10 s
    t_last = time.perf_counter()
    while True:
        st = srv.stats()
        if st["done"] + st["failed"] >= len(ids):
            break
        time.sleep(0.05)
        if time.perf_counter() - t_last > 10.0:
            t_last = time.perf_counter()
            print(f"serving: {st['done']} done, {st['failed']} failed of {len(ids)}", file=sys.stderr, flush=True)
    srv.drain()
    infos = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.close()
    ok = [i for i in infos if i["state"] == 2]
    lat = np.array([i["t_done"] - i["t_arrival"] for i in ok])
    span = max(i["t_done"] for i in infos) - min(i["t_arrival"] for i in infos)
    offered = njobs / max(1e-9, max(i["t_arrival"] for i in infos) - min(i["t_arrival"] for i in infos))
    return {"stream": desc,
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "jobs_per_s": round(len(ok) / span, 2), "offered_jobs_per_s": round(offered, 2),
            "failed": int(len(infos) - len(ok)), "refused_at_submit": refused,
            "batched": int(sum(bool(i["batched"]) for i in infos)),
            "wall_s": round(time.perf_counter() - t_submit0, 2),
            "slots": st["slots"], "max_running": st["max_running"], "peak_hbm_bytes": st["peak_in_use"]}


if __name__ == "__main__":
    main()
