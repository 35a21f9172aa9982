"""Build the gfx950 shared library ``libtrals.so`` from ``csrc/*.hip`` with hipcc.

Usage: ``python -m paper_2210_11362_amd.build`` (also called by the repo's
``__graft_entry__.build()``).  Always recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtrals.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", "-Wno-unused-value",
    "-I", os.path.join(ROOT, "include"),
]


# rocBLAS: the plain FP64 products of the QR-based variants at R_n R_{n+1} > 128
LINK = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocblas"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    return p.returncode, out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    jobs = []
    for f in srcs:
        obj = os.path.join(BUILD, f[:-4] + ".o")
        jobs.append((f, [HIPCC, *FLAGS, "-c", os.path.join(CSRC, f), "-o", obj], obj))
    nproc = min(len(jobs), max(1, min(16, os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(nproc) as ex:
        res = list(ex.map(lambda j: (j[0], *_run(j[1])), jobs))
    bad = [(f, out) for f, rc, out in res if rc != 0]
    for f, rc, out in res:
        if verbose or rc != 0:
            if out.strip():
                print(f"--- {f}\n{out}", file=sys.stderr)
    if bad:
        raise RuntimeError("hipcc failed for: " + ", ".join(f for f, _ in bad))
    tmp = LIB + ".tmp"
    rc, out = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-o", tmp, *[j[2] for j in jobs], *LINK])
    if rc != 0:
        print(out, file=sys.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
