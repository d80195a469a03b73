"""Helpers shared by the GPU tests (not collected by pytest)."""
import sys

import numpy as np
import torch


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel(got: np.ndarray, want: np.ndarray) -> float:
    """Relative error in the 2-norm (Frobenius norm for matrices and link fields)."""
    return float(np.linalg.norm((got - want).ravel()) / np.linalg.norm(want.ravel()))


def rel_max(got: np.ndarray, want: np.ndarray) -> float:
    return float(np.abs(got - want).max() / np.abs(want).max())
