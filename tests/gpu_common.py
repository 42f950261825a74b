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


def slot_errors(g_gpu, g_ref, x, floor=1e-3):
    """Gradient comparison per parameter slot, in log space.

    The calibration moves phi = ln x, so the gradient that matters for slot j
    is x_j * dL/dx_j.  With a = x * g_gpu and b = x * g_ref:
      abs_j = |a_j - b_j| / max_k |b_k|     (every slot, one common scale)
      rel_j = |a_j - b_j| / |b_j|           (slots with |b_j| >= floor * max |b|)
    Slots with x_j = 0 (unused, or a parameter switched off) have a = b = 0.
    Returns (abs, rel, big) as arrays over the slots; rel is NaN where the
    slot is below the floor."""
    g_gpu = np.asarray(g_gpu, np.float64)
    g_ref = np.asarray(g_ref, np.float64)
    x = np.abs(np.asarray(x, np.float64))
    assert g_gpu.shape == g_ref.shape == x.shape, (g_gpu.shape, g_ref.shape, x.shape)
    assert np.all(np.isfinite(g_gpu)) and np.all(np.isfinite(g_ref))
    a, b = x * g_gpu, x * g_ref
    scale = float(np.max(np.abs(b))) if b.size else 0.0
    if scale == 0.0:
        return np.abs(a), np.full(a.shape, np.nan), np.zeros(a.shape, bool)
    d = np.abs(a - b)
    big = np.abs(b) >= floor * scale
    rel = np.full(a.shape, np.nan)
    rel[big] = d[big] / np.abs(b[big])
    return d / scale, rel, big


def check_grad(g_gpu, g_ref, x, what, tol=1e-4, floor=1e-3, names=None):
    """Assert per-slot gradient parity (see slot_errors) and print each slot's
    log-space gradient, its error against the common scale and, above the
    floor, its own relative error."""
    ab, rel, big = slot_errors(g_gpu, g_ref, x, floor)
    b = np.abs(np.asarray(x, np.float64)) * np.asarray(g_ref, np.float64)
    say(f"{what}: max abs {ab.max():.2e}, max rel over {int(big.sum())} slots "
        f"{(np.nanmax(rel) if big.any() else 0.0):.2e}")
    for j in range(len(ab)):
        nm = names[j] if names is not None else str(j)
        say(f"   {j:2d} {nm:>14s}  x*g_ref {b[j]: .6e}  abs {ab[j]:.2e}  rel "
            + (f"{rel[j]:.2e}" if big[j] else "   (below floor)"))
    assert ab.max() <= tol, (what, "abs", ab)
    if big.any():
        assert np.nanmax(rel) <= tol, (what, "rel", rel)
    return ab, rel


def say(*a):
    print(*a, flush=True)
