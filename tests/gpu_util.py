"""Helpers for the GPU parity tests (HIP library vs the FP64 CPU oracle)."""
from __future__ import annotations

import numpy as np
import torch

DEV = torch.device("cuda", 0)


def dev(a, dtype=torch.float64) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_max(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.abs(b).max()
    return float(np.abs(a - b).max() / (nb if nb > 0 else 1.0))


def say(*args):
    print("[case]", *args, flush=True)
