"""Helpers shared by the GPU tests (device transfers only)."""
import numpy as np


def dev(a, dtype=None):
    import torch
    a = np.ascontiguousarray(a)
    if dtype is None:
        dtype = torch.int32 if a.dtype.kind in "iu" else torch.float64
    return torch.as_tensor(a, dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_max(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def elem_err(got, ref):
    """Largest element-wise difference relative to the largest reference entry
    (max_i |got_i - ref_i| / max_i |ref_i|)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))
