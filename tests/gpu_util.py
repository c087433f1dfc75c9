"""Shared helpers of the GPU parity tests (seeded inputs, tolerances)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2609_16863_amd import _abi
    _abi.load()   # raises loudly when the library is missing


def announce(*what):
    """Name the case before a GPU step (flushed, so a crash still names it)."""
    print("[gpu-case]", *what, file=sys.stderr, flush=True)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
