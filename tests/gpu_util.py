"""Helpers shared by the GPU tests: move seeded inputs to the device and pull
cores back.  Holds no ALS arithmetic."""
import sys

import numpy as np

import workloads as W


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev_flat(a, dtype=None):
    import torch
    flat = W.to_flat(np.asarray(a))
    if dtype is not None:
        flat = flat.astype(dtype)
    return torch.from_numpy(flat).cuda()


def cores_to_dev(cores):
    return [to_dev_flat(c, np.float64) for c in cores]


def cores_from_dev(dev, dims, ranks):
    rr = list(ranks) + [ranks[0]]
    out = []
    for n, t in enumerate(dev):
        h = t.detach().cpu().numpy()
        out.append(np.asfortranarray(h.reshape((rr[n], dims[n], rr[n + 1]), order="F")))
    return out


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
