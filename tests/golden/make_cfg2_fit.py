"""Writes ``cfg2_fit_20_sweeps.json``: the oracle's relative error after each
of the 20 regular-ALS sweeps (Alg. 1, FP64, Householder-QR solves) on the
order-4 100^4 workload (Gaussian TR cores of ranks 10, 1% noise, FP32 storage,
seed 0) from its seeded Gaussian initial cores.  Calls only ``oracle/`` and the
seeded input generators; takes several minutes on the CPU.

    python tests/golden/make_cfg2_fit.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    w = W.make_workload(2, seed=0)
    X = w.X.astype(np.float64)
    fits = []
    t0 = time.time()

    def cb(s, cores):
        fits.append(O.rel_error(X, cores))
        print(f"sweep {s + 1}: rel error {fits[-1]:.12e} ({time.time() - t0:.0f} s)", flush=True)

    O.tr_als(X, w.init_cores, w.sweeps, callback=cb)
    out = {"workload": w.name, "dims": list(w.dims), "ranks": list(w.ranks), "eta": w.eta, "seed": 0,
           "sweeps": w.sweeps, "solve": "qr", "rel_error_after_sweep": fits}
    with open(os.path.join(HERE, "cfg2_fit_20_sweeps.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
