"""Helpers for the GPU parity tests (device transfer, case banners)."""

import sys

import numpy as np


def banner(msg):
    """Print what the next GPU step is before it runs (flushed)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_fro(a, b):
    d = np.linalg.norm(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    return d / max(np.linalg.norm(np.asarray(b, dtype=np.float64)), 1e-300)
