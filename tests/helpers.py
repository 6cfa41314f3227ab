"""Shared test helpers (no arithmetic of the method)."""
import numpy as np


def to_dev(a, device="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)


def to_host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def case(msg):
    print(f"[case] {msg}", flush=True)
