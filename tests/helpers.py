"""Shared test helpers (no arithmetic of the method)."""
import numpy as np


def to_dev(a, device="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)


def to_host(t):
    return t.detach().cpu().numpy()


def vec_err(a, b):
    """Largest per-vector error of a against b: both are split along their last axis
    into vectors (one spinor field, one shifted solution, one moment vector), and
    each vector's max_i |a_i - b_i| is divided by that vector's max_i |b_i|. A few
    wrong entries in one vector therefore fail the bar, which a norm taken over
    everything would let through."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    a = a.reshape(-1, a.shape[-1])
    b = b.reshape(-1, b.shape[-1])
    den = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return float((np.abs(a - b).max(axis=1) / den).max())


def case(msg):
    print(f"[case] {msg}", flush=True)
