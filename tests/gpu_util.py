"""Helpers shared by the GPU parity tests."""

import numpy as np
import torch


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda").contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def maxrel(a, b):
    """max |a - b| / max |b| (normwise infinity relative error)."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def l2rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(*what):
    """Name the case before a GPU step (flushed, so a fault still shows it)."""
    print("GPU case:", *what, flush=True)
