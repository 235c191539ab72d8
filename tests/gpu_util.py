"""Helpers shared by the GPU tests: host <-> device copies of uint32 keys."""
import numpy as np


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32).copy()).cuda()


def to_np(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def require_gpu():
    import torch
    from paper_1312_0138_amd import _lib
    assert torch.cuda.is_available(), "the gpu tests need a HIP device"
    _lib.lib()  # raises when libbitsort.so is missing: no fallback
