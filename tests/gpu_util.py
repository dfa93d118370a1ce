"""Helpers shared by the GPU parity tests (marshalling between numpy and torch)."""
import numpy as np
import torch

DEV = "cuda:0"


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def t32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=DEV)


def np64(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def rel_err(a, b, scale):
    """max |a - b| / max(scale): scale is |K| |u| style magnitude per entry."""
    return float(np.abs(a - b).max() / max(np.abs(scale).max(), 1e-300))
