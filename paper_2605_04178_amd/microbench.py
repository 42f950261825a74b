"""Recalibration of the wavefront-centric model on the GPU it runs on.

Two halves, following the paper's workflow (Section IV-D, Table "parameters",
Section V-A):

* ``measure()`` drives the microbenchmarks of libwmbench.so (include/
  wm_microbench.h): read bandwidth against working-set size, dependent-load
  latency against working-set size, throughput per data type, empty-kernel
  launch / workgroup-dispatch / barrier costs, two-stream interference and
  host-device copies.  ``derive_params()`` turns those raw measurements into
  a parameter set (first-principles values, no fitting to kernel times).
* ``validation_cases()`` times the validation kernels (copy, triad, FMA
  chains of varying intensity, reduction, stencil, two transposes, LDS-tiled
  FP32 GEMMs with 8/16/32 tiles, a matrix-core BF16 GEMM) and describes each
  by the model's descriptor fields (flops and bytes from the algorithm,
  VGPRs and LDS as compiled, grid as launched).  ``score()`` computes the
  mean absolute relative error of a parameter set and of the naive roofline
  against those times; calibration on a training split then uses
  ``wavemodel.calibrate``.

The derivation functions are host arithmetic on measured numbers and run
without a GPU (they are unit-tested on synthetic curves).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os
import threading
from typing import Dict, List, Optional

import numpy as np

from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwmbench.so")
MIB = 1 << 20

PEAK_KINDS = ("fp64", "fp32", "bf16", "fp8", "int8")
VAL = dict(copy=0, triad=1, fma=2, stencil=3, transpose_naive=4, transpose_lds=5, reduce=6,
           gemm8=7, gemm16=8, gemm32=9, gemm_mfma=10, bias=11, gemm_mfma_bias=12)

# MI355X (gfx950) structure: 256 CUs of 4 SIMDs, 64-wide waves, 512 VGPRs and
# 8 wave slots per SIMD, 160 KB LDS per CU, 256 MB Infinity Cache, 2.4 GHz.
MI355X_STRUCT = dict(n_levels=4, n_cu=256, n_simd=4, wave=64, vgpr_simd=512, vgpr_gran=8,
                     waves_simd=8, lds_cu=160 * 1024, lds_gran=512, bytes_inflight_wave=16384,
                     mwp=0, cwp=0, combine=0, f_clk=2.4e9, w_lo_mib=205.0, c_llc_mib=256.0)
# datasheet figures for the naive roofline (dense, no sparsity)
MI355X_DATASHEET = dict(hbm=8.0e12, fp64=78.6e12, fp32=157.3e12, bf16=2.5e15, fp8=5.0e15,
                        int8=5.0e15)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2605_04178_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
        L.wmb_last_hip_error.restype = i32
        L.wmb_read_bw.argtypes = [vp, i64, i32, i32, i32, vp, i32, vp, dp]
        L.wmb_read_bw.restype = i32
        L.wmb_chase.argtypes = [vp, i64, i64, i64, vp, vp, vp, dp]
        L.wmb_chase.restype = i32
        L.wmb_clock.argtypes = [i32, i32, vp, vp, vp, dp]
        L.wmb_clock.restype = i32
        L.wmb_sync.argtypes = [i32, vp, vp, dp]
        L.wmb_sync.restype = i32
        L.wmb_peak.argtypes = [i32, i32, i32, vp, i32, vp, dp, dp]
        L.wmb_peak.restype = i32
        L.wmb_empty.argtypes = [i32, i32, i32, vp, i32, vp, dp]
        L.wmb_empty.restype = i32
        L.wmb_val_attr.argtypes = [i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
        L.wmb_val_attr.restype = i32
        L.wmb_val_bytes.argtypes = [i32, i64, i32]
        L.wmb_val_bytes.restype = i64
        L.wmb_val_run.argtypes = [i32, vp, i64, vp, i64, vp, i64, i64, i32, i32, vp, dp,
                                  C.POINTER(i64)]
        L.wmb_val_run.restype = i32
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc} (hip error {lib().wmb_last_hip_error()})")


def _stream(torch, s=None):
    s = s if s is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------------------
# measurement (needs a GPU)
# ---------------------------------------------------------------------------
def clock_hz(blocks: int = 1, spins: int = 1 << 20) -> float:
    """Shader clock (Hz) measured by wmb_clock on cuda:0: blocks = 1 for a
    lightly loaded part, several per CU for the clock under load."""
    import torch
    L = lib()
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    ticks = torch.zeros(2, dtype=torch.int64, device="cuda")
    hz = C.c_double()
    _check(L.wmb_clock(int(blocks), int(spins), C.c_void_p(sink.data_ptr()), C.c_void_p(ticks.data_ptr()),
                       _stream(torch), C.byref(hz)), "wmb_clock")
    return hz.value


def chase_chain(n_nodes: int, stride_words: int, seed: int) -> np.ndarray:
    """A random single cycle over n_nodes nodes spaced stride_words uint32
    apart: entry node*stride holds the index of the next node's entry."""
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(n_nodes)
    order = order[np.concatenate([np.flatnonzero(order == 0), np.flatnonzero(order != 0)])]
    nxt = np.zeros(n_nodes * stride_words, np.uint32)
    src = order * stride_words
    dst = np.roll(order, -1) * stride_words
    nxt[src] = dst.astype(np.uint32)
    assert int(nxt.max()) < nxt.shape[0]
    return nxt


def fusion_times(sizes, launches: int = 10, log=print) -> list:
    """(n, T_gemm, T_bias, T_fused) for the BF16 matrix-core GEMM, the bias
    kernel and the GEMM with the bias fused into its epilogue."""
    import torch
    L = lib()
    st = _stream(torch)
    sec, grid = C.c_double(), C.c_int64()
    res = []
    for n in sizes:
        nb = [[int(L.wmb_val_bytes(k, n, w)) for w in range(3)] for k in (VAL["gemm_mfma"], VAL["bias"],
                                                                           VAL["gemm_mfma_bias"])]
        A = torch.rand(n * n, device="cuda").to(torch.bfloat16)
        Bb = torch.zeros(nb[2][1] // 2, dtype=torch.bfloat16, device="cuda")
        Bb[: n * n] = torch.rand(n * n, device="cuda").to(torch.bfloat16)
        Bb[n * n:].view(torch.float32).copy_(torch.rand(n, device="cuda"))
        Cm = torch.empty(n * n, dtype=torch.float32, device="cuda")
        bias = Bb[n * n:].view(torch.float32)
        t = []
        for k, (a, b) in ((VAL["gemm_mfma"], (A, Bb)), (VAL["bias"], (bias, None)), (VAL["gemm_mfma_bias"], (A, Bb))):
            kb = nb[[VAL["gemm_mfma"], VAL["bias"], VAL["gemm_mfma_bias"]].index(k)]
            _check(L.wmb_val_run(k, C.c_void_p(a.data_ptr()), kb[0], C.c_void_p(b.data_ptr()) if b is not None else None,
                                 kb[1], C.c_void_p(Cm.data_ptr()), kb[2], n, 0, launches, st, C.byref(sec),
                                 C.byref(grid)), "wmb_val_run fusion")
            t.append(sec.value)
        res.append((n, t[0], t[1], t[2]))
        log(f"fusion n={n}: GEMM {t[0] * 1e6:.1f} us + bias {t[1] * 1e6:.1f} us unfused, fused {t[2] * 1e6:.1f} us")
        del A, Bb, Cm
    return res


def measure(quick: bool = False, log=print) -> dict:
    """Run every microbenchmark on cuda:0; raw results as plain numbers."""
    import torch
    L = lib()
    dev = torch.device("cuda:0")
    st = _stream(torch)
    out: Dict[str, object] = {}
    props = torch.cuda.get_device_properties(dev)
    out["device"] = {"name": props.name, "cus": props.multi_processor_count,
                     "gcn_arch": getattr(props, "gcnArchName", "")}
    sinkf = torch.zeros(256, dtype=torch.float32, device=dev)
    sinki = torch.zeros(4, dtype=torch.int32, device=dev)
    sec = C.c_double()
    cus = props.multi_processor_count
    out["clock_hz"] = {"one_wave": clock_hz(1), "loaded": clock_hz(cus * 32)}
    log(f"shader clock {out['clock_hz']['one_wave'] / 1e9:.3f} GHz (one wave), "
        f"{out['clock_hz']['loaded'] / 1e9:.3f} GHz (32 waves per CU)")

    # --- read bandwidth against working set ---
    # every block reads the whole buffer up to 4 MiB (per-CU L1, per-XCD L2),
    # then grid-stride partitions (L2 share per XCD, Infinity Cache, HBM)
    top = 28 if quick else 33                      # up to 256 MiB / 8 GiB
    big = torch.ones((1 << top) // 4, dtype=torch.float32, device=dev)
    bw = []
    blocks = cus * 8
    sizes = [1 << lg for lg in range(13, top + 1)]
    # extra points through the Infinity Cache transition and just above it
    sizes += [m * MIB for m in (160, 192, 208, 216, 224, 232, 240, 248, 320, 384, 768) if m * MIB <= (1 << top)]
    for W in sorted(sizes):
        shared = 1 if W <= (4 << 20) else 0
        per_pass = W * (blocks if shared else 1)
        passes = int(min(65536, max(1, (16 << 30) // per_pass)))
        _check(L.wmb_read_bw(C.c_void_p(big.data_ptr()), W, passes, blocks, shared,
                             C.c_void_p(sinkf.data_ptr()), 5, st, C.byref(sec)), "wmb_read_bw")
        rate = per_pass * passes / sec.value
        bw.append((W, rate, shared))
        log(f"read bw W={W >> 10} KiB shared={shared}: {rate / 1e12:.2f} TB/s ({sec.value * 1e6:.0f} us)")
    out["read_bw"] = bw
    del big

    # --- dependent-load latency against working set ---
    # Up to 256 MiB: a warm pass of 2^18 steps, then the same 2^18 lines
    # (32 MiB, beyond an XCD's 4 MiB L2 from 32 MiB up, within the 256 MiB
    # Infinity Cache) timed again: the level that holds the visited lines.
    # From 512 MiB: the Infinity Cache is emptied of the chain by streaming a
    # 1 GiB buffer, then a cold pass of 2^16 steps, each a line not cached
    # anywhere: HBM (with the translation misses of a 0.5-2 GiB footprint).
    lat = []
    top_l = 28 if quick else 31
    ticks = torch.zeros(1, dtype=torch.int64, device=dev)
    sinku = torch.zeros(1, dtype=torch.int32, device=dev)
    evict = torch.ones((1 << 30) // 4, dtype=torch.float32, device=dev) if top_l >= 29 else None
    for lg in range(13, top_l + 1):
        W = 1 << lg
        stride = 32                                  # 128 B between nodes
        n_nodes = W // 128
        nxt = torch.from_numpy(chase_chain(n_nodes, stride, lg).view(np.int32)).to(dev)
        cold = W >= (512 << 20)
        steps = (1 << 16) if cold else (1 << 18)
        if cold:
            _check(L.wmb_read_bw(C.c_void_p(evict.data_ptr()), 1 << 30, 1, cus * 8, 0,
                                 C.c_void_p(sinkf.data_ptr()), 1, st, C.byref(sec)), "wmb_read_bw")
        ns = C.c_double()
        _check(L.wmb_chase(C.c_void_p(nxt.data_ptr()), nxt.numel(), steps, 0 if cold else steps,
                           C.c_void_p(sinku.data_ptr()), C.c_void_p(ticks.data_ptr()), st, C.byref(ns)),
               "wmb_chase")
        lat.append((W, ns.value))
        log(f"latency W={W >> 10} KiB ({'cold' if cold else 'warm'}): {ns.value:.1f} ns")
        del nxt
    del evict
    out["latency_ns"] = lat

    # --- throughput per data type ---
    flops = C.c_double()
    peaks = {}
    for kind, name in enumerate(PEAK_KINDS):
        iters = 2048 if kind != 1 else 8192
        _check(L.wmb_peak(kind, iters, cus * 8, C.c_void_p(sinkf.data_ptr()), 5, st, C.byref(sec),
                          C.byref(flops)), "wmb_peak")
        peaks[name] = flops.value / sec.value
        log(f"peak {name}: {peaks[name] / 1e12:.1f} TF/s")
    out["peak"] = peaks

    # --- launch, dispatch, barriers ---
    def empty(blocks, block, barriers, launches=20):
        _check(L.wmb_empty(blocks, block, barriers, C.c_void_p(sinki.data_ptr()), launches, st,
                           C.byref(sec)), "wmb_empty")
        return sec.value
    out["empty_1"] = empty(1, 64, 0)
    out["empty_blocks"] = [(g, empty(g, 64, 0)) for g in (1, 1024, 16384, 131072, 1 << 20)]
    res_blocks = cus * 8                              # one round of 256-thread blocks
    out["barriers"] = [(k, empty(res_blocks, 256, k)) for k in (0, 1024, 4096, 16384)]
    out["barrier_blocks"] = res_blocks
    log(f"empty kernel {out['empty_1'] * 1e6:.2f} us")

    # --- host synchronisation (tau_sync) ---
    per = C.c_double()
    syncs = []
    for _ in range(5):
        _check(L.wmb_sync(200, C.c_void_p(sinki.data_ptr()), st, C.byref(per)), "wmb_sync")
        syncs.append(per.value)
    out["sync_s"] = syncs
    log(f"host synchronisation {float(np.median(syncs)) * 1e6:.2f} us")

    # --- fusion: GEMM, bias and the fused GEMM + bias (tau_fusion) ---
    out["fusion"] = fusion_times([2048, 4096] if quick else [2048, 4096, 8192], log=log)

    # --- two concurrent streams (interference) ---
    buf = torch.ones((64 << 20) // 4, dtype=torch.float32, device=dev)
    sink2 = torch.zeros(256, dtype=torch.float32, device=dev)

    def rd(stream_obj, res, key):
        s2 = C.c_double()
        _check(L.wmb_read_bw(C.c_void_p(buf.data_ptr()), 64 << 20, 1, 64, 0,
                             C.c_void_p(sink2.data_ptr()), 20, _stream(torch, stream_obj),
                             C.byref(s2)), "wmb_read_bw")
        res[key] = s2.value
    solo = {}
    rd(None, solo, "a")
    s_a, s_b = torch.cuda.Stream(), torch.cuda.Stream()
    both = {}
    ta = threading.Thread(target=rd, args=(s_a, both, "a"))
    tb = threading.Thread(target=rd, args=(s_b, both, "b"))
    ta.start(); tb.start(); ta.join(); tb.join()
    out["interference"] = {"solo": solo["a"], "concurrent": [both["a"], both["b"]]}
    del buf

    # --- host <-> device copies (pinned) ---
    cp = {"h2d": [], "d2h": []}
    for lg in range(12, 31, 2):
        n = 1 << lg
        h = torch.empty(n, dtype=torch.uint8, pin_memory=True)
        d = torch.empty(n, dtype=torch.uint8, device=dev)
        for key, fn in (("h2d", lambda: d.copy_(h, non_blocking=True)),
                        ("d2h", lambda: h.copy_(d, non_blocking=True))):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 10
            ts = []
            for _ in range(reps):
                e0.record(); fn(); e1.record(); e1.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            cp[key].append((n, float(np.median(ts))))
        del h, d
    out["copies"] = cp
    log("measurements done")
    return out


# ---------------------------------------------------------------------------
# derivation (host arithmetic; no GPU)
# ---------------------------------------------------------------------------
def _window(pairs, lo, hi):
    return [v for (w, v) in pairs if lo <= w <= hi]


def plateau(pairs, lo, hi, stat="median"):
    """Median (or max) of the measured values whose size lies in [lo, hi]."""
    v = _window(pairs, lo, hi)
    if not v:
        raise ValueError(f"no measurement between {lo} and {hi}")
    return float(np.median(v) if stat == "median" else np.max(v))


def linear_fit(xs, ys):
    """Least-squares y = a + b x; returns (a, b)."""
    x = np.asarray(xs, np.float64)
    y = np.asarray(ys, np.float64)
    A = np.vstack([np.ones_like(x), x]).T
    (a, b), *_ = np.linalg.lstsq(A, y, rcond=None)
    return float(a), float(b)


def llc_hit_from_bw(bw, bw_llc, bw_hbm):
    """Fraction of bytes served by the LLC that makes the two-level
    harmonic mix 1/bw = h/bw_llc + (1 - h)/bw_hbm (Eq. (10) with two levels
    served) reproduce a measured bandwidth; clipped to [0, 1]."""
    h = (1.0 / bw - 1.0 / bw_hbm) / (1.0 / bw_llc - 1.0 / bw_hbm)
    return float(min(1.0, max(0.0, h)))


def fit_llc_exponents(points, w_lo_mib, c_mib):
    """Exponents of Table "hlcc-piecewise" from (W MiB, h) points: alpha from
    the transition W_lo < W <= C, h = ((C - W)/(C - W_lo))^alpha; beta from
    the streaming side W > C, h = (C/W)^beta.  Least squares in log h through
    the origin; None where no usable point lies in the regime."""
    def fit(xs, ys):
        xs, ys = np.asarray(xs), np.asarray(ys)
        ok = (ys > 1e-6) & (ys < 1.0) & (xs > 0.0) & (xs < 1.0)
        if not ok.any():
            return None
        lx, ly = np.log(xs[ok]), np.log(ys[ok])
        return float(np.dot(lx, ly) / np.dot(lx, lx))
    tr = [(((c_mib - w) / (c_mib - w_lo_mib)), h) for w, h in points if w_lo_mib < w <= c_mib]
    st = [((c_mib / w), h) for w, h in points if w > c_mib]
    alpha = fit([t[0] for t in tr], [t[1] for t in tr]) if tr else None
    beta = fit([t[0] for t in st], [t[1] for t in st]) if st else None
    return alpha, beta


def fit_streaming(points, bw_llc, c_mib):
    """HBM bandwidth and the streaming exponent beta from (W bytes, bandwidth)
    points with W above the LLC capacity C: the measured bandwidth is the
    harmonic mix 1/bw = h/bw_llc + (1 - h)/bw_hbm with h = (C/W)^beta (Table
    "hlcc-piecewise").  For each beta on a grid (refined twice) 1/bw_hbm is
    the least-squares solution of the linear problem; the pair with the
    smallest squared error in 1/bw wins."""
    W = np.array([w / MIB for w, _ in points if w / MIB > c_mib], np.float64)
    y = np.array([1.0 / b for w, b in points if w / MIB > c_mib], np.float64)
    if W.size < 2:
        raise ValueError("need two bandwidth points above the LLC capacity")

    def solve(beta):
        h = (c_mib / W) ** beta
        rhs = y - h / bw_llc
        g = 1.0 - h
        inv = float(np.dot(rhs, g) / np.dot(g, g))
        err = float(np.sum((h / bw_llc + g * inv - y) ** 2))
        return err, inv
    lo, hi = 0.05, 6.0
    best = None
    for _ in range(3):
        grid = np.linspace(lo, hi, 241)
        errs = [solve(b)[0] for b in grid]
        k = int(np.argmin(errs))
        best = grid[k]
        step = grid[1] - grid[0]
        lo, hi = max(0.01, best - 2 * step), best + 2 * step
    # final refinement by golden-section search on [lo, hi]
    g = (math.sqrt(5) - 1) / 2
    a, b = lo, hi
    for _ in range(80):
        c1, c2 = b - g * (b - a), a + g * (b - a)
        if solve(c1)[0] < solve(c2)[0]:
            b = c2
        else:
            a = c1
    beta = 0.5 * (a + b)
    return 1.0 / solve(beta)[1], float(beta)


def derive_params(meas: dict, struct: Optional[dict] = None) -> "synth.ParamSet":
    """Parameter set from raw microbenchmark results (see measure())."""
    s = dict(MI355X_STRUCT)
    s.update(struct or {})
    s["n_cu"] = int(meas.get("device", {}).get("cus", s["n_cu"]))
    bw = [(r[0], r[1]) for r in meas["read_bw"]]
    lat = [(w, v) for w, v in meas["latency_ns"]]
    KB, MB = 1 << 10, 1 << 20
    cus = s["n_cu"]
    # bandwidth plateaus: whole buffer per block within L1 (32 KB per CU) and
    # within L2 (4 MB per XCD); partitions within the Infinity Cache (below
    # W_lo and above the 8 x 4 MB of L2); HBM (>= 2 GiB)
    bw_l1 = plateau(bw, 1, 16 * KB, "max")
    bw_l2 = plateau(bw, 256 * KB, 2 * MB)
    bw_llc = plateau(bw, 64 * MB, int(s["w_lo_mib"] * MB * 0.75))
    # HBM and beta jointly from the streaming side (W > C); alpha from the
    # transition W_lo < W <= C with that HBM bandwidth
    bw_hbm, beta = fit_streaming([(w, v) for w, v in bw], bw_llc, s["c_llc_mib"])
    f = s["f_clk"]
    lat_l1 = plateau(lat, 1, 16 * KB) * 1e-9 * f
    lat_l2 = plateau(lat, 256 * KB, 2 * MB) * 1e-9 * f
    lat_llc = plateau(lat, 32 * MB, 128 * MB) * 1e-9 * f
    lat_hbm = plateau(lat, 1 << 30, 1 << 40) * 1e-9 * f
    pts = [(w / MB, llc_hit_from_bw(v, bw_llc, bw_hbm)) for w, v in bw if w >= 64 * MB]
    alpha, _ = fit_llc_exponents(pts, s["w_lo_mib"], s["c_llc_mib"])
    pk = meas["peak"]
    # launch: empty single-workgroup kernel; dispatch: slope over workgroups;
    # barrier: slope over barriers per workgroup in one round
    t_launch = float(meas["empty_1"])
    g, t = zip(*meas["empty_blocks"])
    _, tau_wg = linear_fit(g, t)
    k, tb = zip(*meas["barriers"])
    _, tau_bar = linear_fit(k, tb)
    inter = meas.get("interference")
    tau_interf = max(0.0, float(np.mean(inter["concurrent"])) - inter["solo"]) if inter else 0.0
    th = [0.0] * 24
    th[0:4] = [bw_l1, bw_l2, bw_llc, bw_hbm]
    th[4:8] = [lat_l1, lat_l2, lat_llc, lat_hbm]
    th[8:13] = [pk["fp64"], pk["fp32"], pk["bf16"], pk["fp8"], pk["int8"]]
    th[13] = t_launch
    th[14] = max(tau_wg, 0.0)
    th[15] = max(tau_bar, 0.0)
    th[16] = tau_interf
    th[17] = 0.0        # one GPU: no multi-device measurement
    # the fused kernel's time over the plain GEMM's (the epilogue's own flops
    # and bytes are below 0.05 % of the GEMM's, so the model's two
    # descriptors differ by a negligible amount): median over sizes
    fus = meas.get("fusion", [])
    th[18] = float(np.median([max(0.0, tf - tg) for _, tg, _, tf in fus])) if fus else 0.0
    th[19] = max(0.0, float(np.median(meas["sync_s"]))) if meas.get("sync_s") else 0.0
    th[20] = alpha if alpha else 1.0
    th[21] = beta if beta else 1.0
    th[22] = 0.0        # Eq. (16) blend off (not identifiable with an LLC)
    th[23] = bw_hbm * 1.2
    p = synth.ParamSet(**{k2: s[k2] for k2 in ("n_levels", "n_cu", "n_simd", "wave", "vgpr_simd",
                                              "vgpr_gran", "waves_simd", "lds_cu", "lds_gran",
                                              "bytes_inflight_wave", "mwp", "cwp", "combine",
                                              "f_clk", "w_lo_mib", "c_llc_mib")}, theta=th)
    return p


def copy_model(meas: dict):
    """(bandwidth B/s, fixed cost s) per direction from the copy sweep,
    Eq. (15): T = S / B + tau."""
    out = {}
    for key in ("h2d", "d2h"):
        n, t = zip(*meas["copies"][key])
        a, b = linear_fit(n, t)
        out[key] = (1.0 / b, max(a, 0.0))
    return out


# ---------------------------------------------------------------------------
# validation kernels
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Case:
    name: str
    kind: str
    n: int
    iters: int
    F: float
    B: float
    r1: float
    r2: float
    K: float
    W: float
    dtype: int
    seconds: float = float("nan")
    grid: int = 0
    vgpr: int = 0
    lds: int = 0
    block: int = 256
    fused: int = 0      # 1: a fused kernel (the model adds tau_fusion)


def case_list(quick: bool = False) -> List[Case]:
    """Validation cases with flops and bytes from the algorithms (see
    wm_microbench.h for the kernels).  Readings: B counts every byte the
    kernel requests from the memory system (loads and stores); r1 / r2 are
    the fractions served by L1 / L2 when the data layout makes them
    certain; W is the footprint in bytes."""
    cs: List[Case] = []
    sizes1 = [1 << 14, 1 << 18, 1 << 22, 1 << 26] if quick else [1 << 12, 1 << 14, 1 << 18, 1 << 20, 1 << 22, 1 << 24, 1 << 26, 1 << 28]
    for n in sizes1:
        cs.append(Case(f"copy_{n}", "copy", n, 0, 0.0, 8.0 * n, 0, 0, 1, 8.0 * n, 1))
        cs.append(Case(f"triad_{n}", "triad", n, 0, 2.0 * n, 12.0 * n, 0, 0, 1, 12.0 * n, 1))
        cs.append(Case(f"reduce_{n}", "reduce", n, 0, 1.0 * n, 4.0 * n, 0, 0, 1, 4.0 * n, 1))
    for it in ([1, 64, 1024] if quick else [1, 4, 16, 64, 256, 1024]):
        n = 1 << 24
        cs.append(Case(f"fma{it}_{n}", "fma", n, it, 2.0 * it * n, 8.0 * n, 0, 0, 1, 8.0 * n, 1))
    for m in ([2048, 8192] if quick else [1024, 4096, 8192, 16384]):
        el = float(m) * m
        # 5 loads + 1 store per point; of the loads, the centre row's three
        # share lines (L1), the north / south rows are one L2 reuse of two
        cs.append(Case(f"stencil_{m}", "stencil", m, 0, 5.0 * el, 24.0 * el, 0.6, 0.5, 1, 8.0 * el, 1))
        cs.append(Case(f"transpose_naive_{m}", "transpose_naive", m, 0, 0.0, 8.0 * el, 0, 0, 1, 8.0 * el, 1))
        cs.append(Case(f"transpose_lds_{m}", "transpose_lds", m, 0, 0.0, 8.0 * el, 0, 0, 1, 8.0 * el, 1))
    for m in ([1024, 2048] if quick else [512, 1024, 2048, 4096]):
        for t, kind in ((8, "gemm8"), (16, "gemm16"), (32, "gemm32")):
            loaded = 8.0 * m ** 3 / t
            unique = 12.0 * m * m
            cs.append(Case(f"{kind}_{m}", kind, m, 0, 2.0 * m ** 3, loaded + 4.0 * m * m, 0.0,
                           max(0.0, 1.0 - unique / loaded), m / t, unique, 1))
    for m in ([1024, 4096] if quick else [1024, 2048, 4096, 8192]):
        loaded = m ** 3 / 8.0          # each wave streams 32 rows of A and of B^T
        unique = 8.0 * m * m
        cs.append(Case(f"gemm_mfma_{m}", "gemm_mfma", m, 0, 2.0 * m ** 3, loaded + 4.0 * m * m, 0.5,
                       max(0.0, 1.0 - unique / (loaded / 2.0)), m / 16, unique, 2))
        # the fusion pair: the bias kernel alone (read C and the bias, write
        # C) and the GEMM with the bias added in its epilogue
        cs.append(Case(f"bias_{m}", "bias", m, 0, 1.0 * m * m, 8.0 * m * m + 4.0 * m, 0, 0, 1,
                       8.0 * m * m, 1))
        cs.append(Case(f"gemm_mfma_bias_{m}", "gemm_mfma_bias", m, 0, 2.0 * m ** 3 + m * m,
                       loaded + 4.0 * m * m + 4.0 * m, 0.5, max(0.0, 1.0 - unique / (loaded / 2.0)), m / 16,
                       unique, 2, fused=1))
    return cs


def run_cases(cases: List[Case], launches: int = 100, log=print, warmup: int = 10) -> List[Case]:
    """Time every case: `warmup` untimed launches, then the median of
    `launches` event-timed ones (the paper's protocol, Section V: 10 warm-ups,
    100 timed runs, median).  Each case issues warmup + 1 + launches
    dispatches of its kernel (wmb_val_run itself runs one untimed launch
    before its timed ones)."""
    import torch
    L = lib()
    dev = torch.device("cuda:0")
    st = _stream(torch)
    sec = C.c_double()
    grid = C.c_int64()
    vg, ld, bl = C.c_int32(), C.c_int32(), C.c_int32()
    bufs = {}

    def buf(tag, nbytes, dtype=torch.float32):
        key = (tag, nbytes, dtype)
        if key not in bufs:
            for k in [k for k in bufs if k[0] == tag]:
                del bufs[k]
            esz = torch.tensor([], dtype=dtype).element_size()
            bufs[key] = torch.rand(max(nbytes // esz, 1), device=dev).to(dtype)
        return bufs[key]

    for c in cases:
        kind = VAL[c.kind]
        log(f"case {c.name}")
        _check(L.wmb_val_attr(kind, C.byref(vg), C.byref(ld), C.byref(bl)), "wmb_val_attr")
        c.vgpr, c.lds, c.block = vg.value, ld.value, bl.value
        nbytes = [int(L.wmb_val_bytes(kind, c.n, w)) for w in range(3)]
        if nbytes[0] < 0:
            raise ValueError(c.name)
        dt = torch.bfloat16 if c.kind in ("gemm_mfma", "gemm_mfma_bias") else torch.float32
        a = buf("a", nbytes[0], dt)
        b = buf("b", nbytes[1], dt) if nbytes[1] > 0 else None
        cc = buf("c", nbytes[2])
        args = (kind, C.c_void_p(a.data_ptr()), nbytes[0],
                C.c_void_p(b.data_ptr()) if b is not None else None, nbytes[1],
                C.c_void_p(cc.data_ptr()), nbytes[2], c.n, c.iters)
        if warmup > 1:
            _check(L.wmb_val_run(*args, warmup - 1, st, C.byref(sec), C.byref(grid)), "wmb_val_run " + c.name)
        _check(L.wmb_val_run(*args, launches, st, C.byref(sec), C.byref(grid)), "wmb_val_run " + c.name)
        c.seconds, c.grid = sec.value, grid.value
        if c.kind == "reduce":     # grid-stride loop: iterations per workgroup
            c.K = float(math.ceil(c.n / 4 / (c.grid * 256)))
        log(f"{c.name}: {c.seconds * 1e6:.1f} us grid {c.grid} vgpr {c.vgpr} lds {c.lds}")
    return cases


def descriptors_of(cases: List[Case]) -> "synth.Descriptors":
    f32 = np.float32
    n = len(cases)
    g = np.array([c.block for c in cases], np.int64)
    gp = synth.pack_gpack(g, np.array([c.dtype for c in cases]), np.ones(n, np.int64),
                          np.ones(n, np.int64), np.array([c.fused for c in cases], np.int64),
                          np.zeros(n, np.int64))
    return synth.Descriptors(
        F=np.array([c.F for c in cases], f32), B=np.array([c.B for c in cases], f32),
        r1=np.array([c.r1 for c in cases], f32), r2=np.array([c.r2 for c in cases], f32),
        r3=np.zeros(n, f32), K=np.array([c.K for c in cases], f32), u=np.ones(n, f32),
        W=np.array([c.W for c in cases], f32), vgpr=np.array([max(c.vgpr, 1) for c in cases], np.int32),
        lds=np.array([c.lds for c in cases], np.int32), gpack=gp.astype(np.int32),
        grid=np.array([max(c.grid, 1) for c in cases], np.int32))


def roofline_naive(cases: List[Case], sheet: dict = MI355X_DATASHEET) -> np.ndarray:
    """max(F / P_dtype, B / B_HBM) with datasheet peaks (Section V-A)."""
    peaks = [sheet["fp64"], sheet["fp32"], sheet["bf16"], sheet["fp8"], sheet["int8"]]
    return np.array([max(c.F / peaks[c.dtype], c.B / sheet["hbm"]) for c in cases])


def mae(pred, meas) -> float:
    """Mean absolute relative error |pred - meas| / meas over finite pairs."""
    p = np.asarray(pred, np.float64)
    m = np.asarray(meas, np.float64)
    ok = np.isfinite(p) & np.isfinite(m) & (m > 0)
    return float(np.mean(np.abs(p[ok] - m[ok]) / m[ok])) if ok.any() else float("nan")


def split(cases: List[Case], holdout_every: int = 3):
    """Deterministic train / holdout split: every `holdout_every`-th case of
    each kernel family (in size order) is held out."""
    train, hold = [], []
    seen: Dict[str, int] = {}
    for c in cases:
        fam = c.kind
        k = seen.get(fam, 0)
        seen[fam] = k + 1
        (hold if k % holdout_every == holdout_every - 1 else train).append(c)
    return train, hold
