"""Helpers shared by the GPU tests: host arrays <-> device tensors."""
import numpy as np
import torch


def to_dev(a: np.ndarray, device) -> torch.Tensor:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32).copy()).to(device)


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def first_mismatch(got: np.ndarray, want: np.ndarray):
    bad = np.nonzero(np.any(got != want, axis=1))[0]
    return (len(bad), int(bad[0]) if len(bad) else -1)
