"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np


def to_dev(v):
    import torch
    return torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
