"""Helpers for the GPU tests: host <-> device column-major transfers."""
import numpy as np
import torch


def to_dev(a: np.ndarray) -> torch.Tensor:
    """numpy matrix -> column-major CUDA tensor with the same values."""
    a = np.asarray(a)
    if a.ndim == 1:
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return torch.from_numpy(np.ascontiguousarray(a.T)).cuda().t()


def to_host(t: torch.Tensor) -> np.ndarray:
    """column-major CUDA tensor -> Fortran-ordered numpy array."""
    if t.dim() == 1:
        return t.cpu().numpy()
    return np.asfortranarray(t.t().cpu().numpy().T)


def announce(msg: str):
    print("[gpu-case] " + msg, flush=True)
