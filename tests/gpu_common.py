"""Helpers shared by the GPU parity tests (imported by tests only)."""

import sys

import numpy as np
import pytest


def torch_gpu():
    """(torch, device) or skip when this machine has no GPU.  When a GPU is
    present the native library must load -- a missing build is an error."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU on this machine")
    import paper_2511_18207_amd as ph
    ph.lib()  # raises if libprohd.so is missing
    return torch, torch.device("cuda:0")


def to_dev(torch, X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()


def banner(msg):
    """Name the case on stdout before any GPU work (flushed)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)
