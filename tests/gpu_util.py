"""Helpers for the GPU parity tests (device transfer, norms, logging)."""
import sys

import numpy as np


def log(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def spectral_norm_estimate(apply, shape, iters=40, seed=0):
    """Largest eigenvalue of an SPD operator by power iteration (a lower
    bound that is within a few percent after 40 steps on these operators)."""
    x = np.random.default_rng(seed).standard_normal(shape)
    lam = 0.0
    for _ in range(iters):
        y = apply(x)
        lam = np.linalg.norm(y) / np.linalg.norm(x)
        x = y / np.linalg.norm(y)
    return lam
