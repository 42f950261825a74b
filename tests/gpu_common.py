"""Helpers shared by the GPU test modules (marshalling and comparisons only)."""
import numpy as np
import pytest
import torch


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def rel_err(gpu, ref):
    """Relative error per element; both-inf (same sign) and both-NaN count as 0,
    any other mismatch of finiteness as inf."""
    g = np.asarray(gpu, np.float64)
    r = np.asarray(ref, np.float64)
    out = np.zeros(g.shape)
    both_nan = np.isnan(g) & np.isnan(r)
    both_inf = np.isinf(g) & np.isinf(r) & (np.sign(g) == np.sign(r))
    fin = np.isfinite(g) & np.isfinite(r)
    out[fin] = np.abs(g[fin] - r[fin]) / np.maximum(np.abs(r[fin]), 1e-300)
    bad = ~(fin | both_nan | both_inf)
    out[bad] = np.inf
    return out


def grad_err(g_gpu, g_ref):
    """max_j |g_gpu - g_ref| / max_j |g_ref|"""
    g_gpu = np.asarray(g_gpu, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    return float(np.max(np.abs(g_gpu - g_ref)) / max(np.max(np.abs(g_ref)), 1e-300))


def say(*a):
    print(*a, flush=True)
