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
        print(json.dumps(serving_leg(args.serving_jobs)))
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
    kname = {1: "xgemm_kernel (two-stage X contraction, stage 1)", 2: "xstream_kernel (fused X contraction)"}
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

    # ---- the QR-stabilised variant (Alg. 3) on the same workload ------------
    if not args.no_qr:
        try:
            qr = {}
            for p in ("f32", args.prec):
                ctx, dev = fresh("qr")
                ctx.sweep(1, p, refine=1)
                torch.cuda.synchronize()
                ta = time.perf_counter()
                ctx.sweep(3, p, refine=1)
                tb = time.perf_counter()
                qr[f"{p}_ms_per_sweep"] = round(1000 * (tb - ta) / 3, 4)
                qr[f"{p}_fit_after_4_sweeps"] = ctx.fit()
                ctx.close()
            extra["qr_variant"] = qr
        except Exception as e:   # reported, never fatal to the bench line
            extra["qr_variant"] = {"error": str(e)[:200]}

    # ---- serving: a Poisson stream of small jobs through the request loop ---
    if not args.no_serving and args.serving_jobs > 0:
        extra["serving"] = serving_child(args.serving_jobs)

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
                         f"100^4 tensor in FP64 numpy/LAPACK, {t_mode:.2f} s, scaled x{N} to one sweep"}

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


def serving_child(njobs: int):
    """The serving stream in a child process (its own device context): a failure
    there is reported in the bench line instead of ending the bench."""
    import subprocess
    try:
        p = subprocess.run([sys.executable, os.path.abspath(__file__), "--serving-only", "--serving-jobs", str(njobs)],
                           stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    except subprocess.TimeoutExpired:
        return {"error": "serving stream timed out after 300 s"}
    lines = [l for l in p.stdout.splitlines() if l.startswith("{")]
    if p.returncode != 0 or not lines:
        return {"error": f"serving stream exited with status {p.returncode}", "stderr_tail": p.stderr[-400:]}
    return json.loads(lines[-1])


def serving_leg(njobs: int):
    """Latency and throughput of the request loop on a Poisson stream (200 jobs/s)
    of planted-TR jobs of order 3-4, mode sizes 16-48, ranks 2-8 (8 BF16 + 2 FP32
    sweeps each), generated on the device; 8 slots, 16 GiB arena."""
    import numpy as np
    import workloads as W
    from paper_2210_11362_amd import TRServer
    jobs = W.serving_stream(njobs, orders=(3, 4), dim_range=(16, 48), rank_range=(2, 8))
    srv = TRServer(16 << 30, 8)
    ids = [srv.submit(j["dims"], j["ranks"], seed=j["seed"], eta=0.01, prec_mixed="bf16", nsweeps_mixed=8,
                      prec_fin="f32", nsweeps_fin=2, t_arrival=0.05 + j["t_arrive"]) for j in jobs]
    srv.drain()
    infos = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.close()
    lat = np.array([i["t_done"] - i["t_arrival"] for i in infos])
    span = max(i["t_done"] for i in infos) - min(i["t_arrival"] for i in infos)
    return {"stream": f"{njobs} jobs, Poisson 200/s, order 3-4, dims 16-48, ranks 2-8, 8xbf16+2xf32 sweeps",
            "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
            "jobs_per_s": round(njobs / span, 2), "failed": int(sum(i["state"] != 2 for i in infos)),
            "slots": st["slots"], "max_running": st["max_running"], "peak_hbm_bytes": st["peak_in_use"]}


if __name__ == "__main__":
    main()
