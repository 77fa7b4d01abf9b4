"""Shared helpers of the GPU tests (device placement of seeded workloads)."""

import numpy as np


def to_dev(arrs):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda") for a in arrs]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(1e-300, np.linalg.norm(np.asarray(b))))


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
