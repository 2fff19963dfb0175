"""Equality of bit patterns, for the checks that claim identical bits rather than equal
values: -0 and +0 differ here, and so do NaNs with different payloads."""
import numpy as np
import torch

_INT = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def same_bits(a, b) -> bool:
    if isinstance(a, torch.Tensor) or isinstance(b, torch.Tensor):
        if not (isinstance(a, torch.Tensor) and isinstance(b, torch.Tensor)):
            return False
        a, b = a.detach().cpu(), b.detach().cpu()
        a, b = a.numpy(), b.numpy()
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    if a.shape != b.shape or a.dtype != b.dtype:
        return False
    if a.dtype.kind == "f":
        it = _INT[a.dtype.itemsize]
        return bool(np.array_equal(a.view(it), b.view(it)))
    return bool(np.array_equal(a, b))
