"""Helpers shared by the GPU parity tests."""
import numpy as np
import torch

from paper_2603_14926_amd import mpx


def to_gpu(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_np(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bits_equal(a: np.ndarray, b: np.ndarray) -> bool:
    """Bitwise equality (distinguishes -0.0 from 0.0, compares NaN payloads)."""
    a = np.ascontiguousarray(a); b = np.ascontiguousarray(b)
    if a.shape != b.shape or a.dtype != b.dtype:
        return False
    iv = np.int64 if a.dtype == np.float64 else np.int32
    return bool(np.array_equal(a.view(iv), b.view(iv)))


def first_mismatch(a, b):
    iv = np.int64 if a.dtype == np.float64 else np.int32
    d = np.argwhere(a.view(iv) != b.view(iv))
    return None if d.size == 0 else tuple(d[0])


PREC_K = [("dd", 2, np.float64), ("td", 3, np.float64), ("qd", 4, np.float64), ("ff", 2, np.float32)]
