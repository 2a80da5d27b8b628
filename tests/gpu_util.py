"""Helpers shared by the GPU tests (device tensors, library handles)."""
import sys

import numpy as np


def announce(*parts):
    """Print the case about to run on the GPU (flushed, so a crash names it)."""
    print("[gpu-case]", *parts, file=sys.stderr, flush=True)


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a).ravel())
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def to_host(t):
    return t.detach().to("cpu").to(dtype=t.dtype).numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
