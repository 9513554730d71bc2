"""Helpers shared by the GPU tests (comparison metrics only; no method
arithmetic)."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, want):
    scale = max(float(np.abs(want).max()), 1e-300)
    return float(np.abs(np.asarray(got) - np.asarray(want)).max()) / scale


def mps_vector(tensors):
    """Dense state vector of an MPS given as [Dl][d][Dr] arrays (small L)."""
    v = tensors[0]
    for a in tensors[1:]:
        v = np.tensordot(v, a, axes=([v.ndim - 1], [0]))
    return v.reshape(-1)


def mps_overlap(A, B):
    """<A|B> by transfer matrices (comparison metric for any L)."""
    E = np.ones((1, 1))
    for a, b in zip(A, B):
        t = np.tensordot(E, b, axes=([1], [0]))            # [a', s, b]
        E = np.tensordot(a, t, axes=([0, 1], [0, 1]))       # [b', b]
    return float(E[0, 0])
