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


# float32 Jacobian rows carry a few ulp of rounding each; 8 ulp of a slot's
# absolute sum bounds what that rounding can leave in the slot's sum
F32_TERM_BOUND = 2.0 ** -21
# slots whose sum cancels by more than this (absolute sum over |sum|) are
# ill-conditioned for float32 terms: 200 x 8 ulp ~ 1e-4
MAX_COND_F32 = 200.0


def check_grad(g_gpu, g_ref, x, what, tol=1e-4, floor=1e-3, names=None, absum=None):
    """Assert per-slot gradient parity (see slot_errors) and print each slot's
    log-space gradient, its error against the common scale and, above the
    floor, its own relative error.

    absum (optional, per slot): the sum over descriptors of |x_j w_i dT_i/dx_j|
    from the oracle, for a gradient formed from float32 Jacobian rows.  A
    slot whose sum cancels by more than MAX_COND_F32 (absum / |x_j g_j|) is
    then held to F32_TERM_BOUND * absum instead of tol * |x_j g_j|: float32
    rounding of the terms alone can exceed the relative bound there (the
    float64-exact calls are checked without absum)."""
    ab, rel, big = slot_errors(g_gpu, g_ref, x, floor)
    xa = np.abs(np.asarray(x, np.float64))
    b = xa * np.asarray(g_ref, np.float64)
    d = np.abs(xa * np.asarray(g_gpu, np.float64) - b)
    cond = np.full(b.shape, np.nan) if absum is None else np.asarray(absum) / np.maximum(np.abs(b), 1e-300)
    ill = np.zeros(b.shape, bool) if absum is None else big & (cond > MAX_COND_F32)
    strict = big & ~ill
    say(f"{what}: max abs {ab.max():.2e}, max rel over {int(strict.sum())} slots "
        f"{(np.nanmax(rel[strict]) if strict.any() else 0.0):.2e}"
        + (f", {int(ill.sum())} ill-conditioned slots within {np.max(d[ill] / np.asarray(absum)[ill]):.2e} "
           f"of their absolute sums" if ill.any() else ""))
    for j in range(len(ab)):
        nm = names[j] if names is not None else str(j)
        tail = (f"{rel[j]:.2e}" if big[j] else "   (below floor)")
        if absum is not None:
            tail += f"  cond {cond[j]:.1e}" + ("  (ill-conditioned)" if ill[j] else "")
        say(f"   {j:2d} {nm:>14s}  x*g_ref {b[j]: .6e}  abs {ab[j]:.2e}  rel " + tail)
    assert ab.max() <= tol, (what, "abs", ab)
    if strict.any():
        assert np.nanmax(rel[strict]) <= tol, (what, "rel", rel)
    if ill.any():
        assert np.all(d[ill] <= F32_TERM_BOUND * np.asarray(absum)[ill]), (what, "ill-conditioned", d, absum)
    return ab, rel


def loss_grad_absum(orc, p, d, m):
    """Per slot, sum over descriptors of |x_j w_i dT_i/dx_j| / count (the
    loss gradient's terms in log space, from the oracle; w_i = sign(T_i -
    m_i) / m_i over finite T and measured m > 0)."""
    T, _ = orc.predict(p, d)
    m = np.asarray(m, np.float64)
    f = np.isfinite(T) & np.isfinite(m) & (m > 0)
    J = orc.jacobian(p, d)[f]
    w = np.abs(np.sign(T[f] - m[f])) / m[f]
    return (w[:, None] * np.abs(J)).sum(0) * np.abs(np.asarray(p.theta)) / max(int(f.sum()), 1)


def say(*a):
    print(*a, flush=True)
