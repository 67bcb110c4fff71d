"""Helpers shared by the GPU parity tests (device transfer, error norms)."""
import numpy as np


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, ref, floor=0.0):
    """Per-macro normwise relative error max_m |got_m - ref_m| / max(|ref_m|, floor_m)."""
    M = ref.shape[0]
    g = got.reshape(M, -1)
    r = ref.reshape(M, -1)
    num = np.linalg.norm(g - r, axis=1)
    den = np.maximum(np.linalg.norm(r, axis=1), floor)
    return float(np.max(num / den))


def banner(msg):
    print(f"[gpu] {msg}", flush=True)
