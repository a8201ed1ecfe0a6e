"""Helpers shared by the GPU tests (device checks and host<->device conversions)."""
import sys

import numpy as np


def device():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    return torch.device("cuda:0")


def to_dev(a: np.ndarray, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device())


def to_host(t) -> np.ndarray:
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def note(*args):
    """Print (and flush) what names the case before a GPU step."""
    print(*args, file=sys.stderr, flush=True)


def max_err(a: np.ndarray, b: np.ndarray) -> float:
    """Element-wise error: max |a - b| over max |b| (every entry is held to the same scale)."""
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))
