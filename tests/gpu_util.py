"""Helpers for GPU parity tests (device buffers through torch, comparisons)."""
import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def empty(shape, dtype):
    """An output buffer on the device, pre-filled with NaN (floating point) or -1
    (integers) so that an entry the library leaves unwritten fails the comparison."""
    import torch
    t = {np.float64: torch.float64, np.float32: torch.float32, np.int32: torch.int32}[dtype]
    return torch.full(shape, float("nan") if t.is_floating_point else -1, dtype=t, device="cuda")


def rel_l2(x, ref):
    """||x - ref||_2 / ||ref||_2 over the whole array (Frobenius for matrices)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def max_cell_rel(x, ref):
    """Largest per-cell relative L2 error (cells along axis 0)."""
    x = np.asarray(x, dtype=np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(ref), -1)
    num = np.linalg.norm(x - ref, axis=1)
    den = np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    return float((num / den).max())
