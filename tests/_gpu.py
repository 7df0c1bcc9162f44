"""Shared helpers of the GPU tests: seeded inputs moved to the device, error metrics."""
import math

import numpy as np
import torch

DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    return t.detach().cpu().numpy()


def scaled_err(I, I_ref, f):
    """max |I - I_ref| / max(I_ref, sum f^2) (intensity error scale; speckle nulls
    are measured against the incoherent level sum f^2)."""
    inc = float(np.sum(np.asarray(f, dtype=np.float64) ** 2))
    return float(np.max(np.abs(np.asarray(I) - np.asarray(I_ref)) / np.maximum(np.asarray(I_ref), inc)))


def grad_err(g, g_ref):
    """max_j |g_j - g_ref_j| / RMS_j |g_ref_j|."""
    g = np.asarray(g, dtype=np.float64).reshape(-1, 3)
    g_ref = np.asarray(g_ref, dtype=np.float64).reshape(-1, 3)
    rms = math.sqrt(np.mean(np.sum(g_ref * g_ref, axis=1)))
    return float(np.max(np.linalg.norm(g - g_ref, axis=1)) / rms)


def bitwise_equal(a, b):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))
