"""Seeded synthetic inputs for the CDNA wavefront-centric execution-time model.

This module draws random numbers and packs them into arrays; it performs none
of the model's arithmetic (no occupancy, traffic split, stage times or tile
derivation). Both the FP64 oracle and the HIP path consume what it returns.

The paper evaluates its model on measured kernels (microbenchmarks, Rodinia,
SPEChpc; Section V) that are not available here, so these sweeps stand in for
them. Value ranges follow the paper where it prints them: cache levels and
latencies (Table "parameters"), 304 CUs / 64 KB LDS / 32 waves per CU
(Table "arch-params"), utilisation 0.4-0.7 (Table "model-summary"),
tau_interf = 50 us and tau_sync = 3 us (Table "parameters"), barrier and
coherence cost 100-200 ns (Table "model-summary").

Everything is NumPy PCG64 seeded; the same seed always gives the same bytes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

# ---------------------------------------------------------------------------
# parameter-vector slot names (Section IV-B symbols); 24 slots
# ---------------------------------------------------------------------------
THETA_NAMES = [
    "BW_L1", "BW_L2", "BW_LLC", "BW_HBM",          # 0-3   bytes/s
    "Lat_L1", "Lat_L2", "Lat_LLC", "Lat_HBM",      # 4-7   cycles
    "P_fp64", "P_fp32", "P_bf16", "P_fp8", "P_int8",  # 8-12 flop/s
    "T_launch",                                    # 13    s
    "tau_wg",                                      # 14    s per workgroup
    "tau_bar",                                     # 15    s per WG round x step
    "tau_interf",                                  # 16    s per extra concurrent kernel
    "tau_gpu",                                     # 17    s per extra device
    "tau_fusion",                                  # 18    s if fused
    "tau_sync",                                    # 19    s per host sync
    "alpha", "beta",                               # 20-21 LLC hit-rate exponents
    "w0", "B_peak",                                # 22-23 working-set blend
]
N_THETA = 24
MIB = float(1 << 20)

# Slots the calibration tests fit (bit j = slot j).  Three-level sets leave
# the LLC slots (BW_LLC, Lat_LLC, alpha, beta) unused.  With an LLC, w0 (the
# Eq. (16) blend scale) is held: the cache serves every working set below
# W_lo, so the blend is seen only through its tail exp(-W/w0) beyond W_lo,
# where its amplitude (B_peak) and scale (w0) are nearly collinear (the
# Fisher identifiability pin in the oracle tests measures both).
FIT_MASK_L4 = 0xFFFFFF & ~(1 << 22)
FIT_MASK_L3 = 0xFFFFFF & ~((1 << 2) | (1 << 6) | (1 << 20) | (1 << 21))


def fit_mask(n_levels: int) -> int:
    return FIT_MASK_L4 if n_levels == 4 else FIT_MASK_L3

# gpack bit layout of the int32 descriptor field: WG threads, dtype, counts
GPACK_G_BITS = 11
GPACK_DTYPE_SHIFT = 11
GPACK_NCONC_SHIFT = 14
GPACK_NDEV_SHIFT = 17
GPACK_FUSED_SHIFT = 20
GPACK_NSYNC_SHIFT = 21

# tile-candidate code layout: mt | nt<<2 | kd<<4 | (waves-1)<<6
TILE_MN = (32, 64, 128, 256)
TILE_KD = (16, 32, 64)
N_TILES = 4 * 4 * 3 * 8


@dataclasses.dataclass
class ParamSet:
    """Structural integers plus the 24-slot parameter vector theta."""
    n_levels: int = 4
    n_cu: int = 304
    n_simd: int = 4
    wave: int = 64
    vgpr_simd: int = 512
    vgpr_gran: int = 8
    waves_simd: int = 8
    lds_cu: int = 65536
    lds_gran: int = 512
    bytes_inflight_wave: int = 16384
    mwp: int = 0
    cwp: int = 0
    combine: int = 0            # 0 = max of stages, 1 = occupancy-overlap step
    f_clk: float = 2.1e9
    w_lo_mib: float = 205.0
    c_llc_mib: float = 256.0
    theta: List[float] = dataclasses.field(default_factory=lambda: [0.0] * N_THETA)

    def copy(self, **kw) -> "ParamSet":
        d = dataclasses.asdict(self)
        d["theta"] = list(self.theta)
        d.update(kw)
        return ParamSet(**d)


@dataclasses.dataclass
class Descriptors:
    """Structure-of-arrays kernel descriptors: 8 float32 + 4 int32 arrays."""
    F: np.ndarray
    B: np.ndarray
    r1: np.ndarray
    r2: np.ndarray
    r3: np.ndarray
    K: np.ndarray
    u: np.ndarray
    W: np.ndarray
    vgpr: np.ndarray
    lds: np.ndarray
    gpack: np.ndarray
    grid: np.ndarray

    FLOAT_FIELDS = ("F", "B", "r1", "r2", "r3", "K", "u", "W")
    INT_FIELDS = ("vgpr", "lds", "gpack", "grid")

    @property
    def n(self) -> int:
        return int(self.F.shape[0])

    def fields(self):
        return [getattr(self, f) for f in self.FLOAT_FIELDS + self.INT_FIELDS]

    def slice(self, a: int, b: int) -> "Descriptors":
        return Descriptors(*[x[a:b] for x in self.fields()])

    def take(self, idx) -> "Descriptors":
        return Descriptors(*[np.ascontiguousarray(x[idx]) for x in self.fields()])

    @staticmethod
    def concat(parts) -> "Descriptors":
        names = Descriptors.FLOAT_FIELDS + Descriptors.INT_FIELDS
        return Descriptors(*[np.concatenate([getattr(p, f) for p in parts]) for f in names])


def pack_gpack(g, dtype, n_conc=1, n_dev=1, fused=0, n_sync=0):
    """Bit-pack the small integer descriptor fields (layout above)."""
    g = np.asarray(g, dtype=np.int64)
    v = (g | (np.asarray(dtype, np.int64) << GPACK_DTYPE_SHIFT)
         | ((np.asarray(n_conc, np.int64) - 1) << GPACK_NCONC_SHIFT)
         | ((np.asarray(n_dev, np.int64) - 1) << GPACK_NDEV_SHIFT)
         | (np.asarray(fused, np.int64) << GPACK_FUSED_SHIFT)
         | (np.asarray(n_sync, np.int64) << GPACK_NSYNC_SHIFT))
    return v.astype(np.int32)


def _logu(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


# ---------------------------------------------------------------------------
# parameter sets
# ---------------------------------------------------------------------------
def param_set(seed: int = 0, n_levels: int = 4, combine: int = 0) -> ParamSet:
    """One CDNA-style parameter set with seeded synthetic values.

    Bandwidths: 4 x log-U[2, 80] TB/s sorted fast-to-slow (L1 .. HBM);
    latencies: 4 x U[50, 800] cycles sorted ascending; both redrawn until
    neighbouring levels differ by at least 1.5x in bandwidth and 50 cycles in
    latency (a level indistinguishable from the next one leaves the LLC
    hit-rate exponents unidentifiable); five dtype peaks; overhead constants
    in the ranges quoted in the module docstring.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    th = [0.0] * N_THETA
    while True:
        bw = np.sort(_logu(rng, 2e12, 80e12, 4))[::-1]
        if np.all(bw[:-1] / bw[1:] >= 1.5):
            break
    while True:
        lat = np.sort(rng.uniform(50.0, 800.0, 4))
        if np.all(np.diff(lat) >= 50.0):
            break
    th[0:4] = [float(x) for x in bw]
    th[4:8] = [float(x) for x in lat]
    th[8] = float(_logu(rng, 30e12, 160e12))
    th[9] = float(_logu(rng, 60e12, 320e12))
    th[10] = float(_logu(rng, 500e12, 2600e12))
    th[11] = float(_logu(rng, 1000e12, 5200e12))
    th[12] = float(_logu(rng, 1000e12, 5200e12))
    th[13] = float(rng.uniform(2e-6, 12e-6))
    th[14] = float(_logu(rng, 1e-9, 20e-9))
    th[15] = float(_logu(rng, 50e-9, 200e-9))
    th[16] = float(_logu(rng, 10e-6, 100e-6))
    th[17] = float(_logu(rng, 10e-6, 100e-6))
    th[18] = float(_logu(rng, 1e-6, 10e-6))
    th[19] = float(_logu(rng, 1e-6, 10e-6))
    th[20] = float(rng.uniform(0.5, 3.0))
    th[21] = float(rng.uniform(0.5, 2.0))
    th[22] = float(_logu(rng, 16 * MIB, 512 * MIB))
    th[23] = float(th[3] * rng.uniform(1.1, 1.6))
    return ParamSet(n_levels=n_levels, combine=combine, theta=th)


def mi300a_like() -> ParamSet:
    """Values the paper prints for MI300A (Tables "arch-params" and
    "parameters"): 304 CUs, Infinity Cache 17.2 TB/s, HBM 5.3 TB/s,
    latencies 5/50/150/400 cycles, FP8 1307 TF, FP64 61.3 TF, 64 KB LDS,
    32 waves per CU, tau_interf 50 us, tau_sync 3 us, coherence 100-200 ns.
    L1/L2 bandwidths, the FP32/BF16/INT8 peaks, T_launch and the remaining
    overheads are not printed; the values below for them are placeholders
    (FP32 and BF16 scaled from FP64/FP8 by MFMA width)."""
    th = [0.0] * N_THETA
    th[0:4] = [64e12, 34e12, 17.2e12, 5.3e12]
    th[4:8] = [5.0, 50.0, 150.0, 400.0]
    th[8:13] = [61.3e12, 122.6e12, 653.5e12, 1307e12, 1307e12]
    th[13] = 5e-6
    th[14] = 5e-9
    th[15] = 150e-9
    th[16] = 50e-6
    th[17] = 50e-6
    th[18] = 2e-6
    th[19] = 3e-6
    th[20] = 1.0
    th[21] = 1.0
    th[22] = 64 * MIB
    th[23] = 5.3e12 * 1.3
    return ParamSet(n_levels=4, n_cu=304, theta=th)


def multi_arch_sets(base_seed: int = 0, n_sets: int = 6, seed0: int = 110) -> List[ParamSet]:
    """Six architecture variants of the seed-0 base set: 3 or 4 levels,
    104-304 CUs, bandwidth and peak scales log-U[0.5, 2]."""
    base = param_set(base_seed)
    out = []
    for i in range(n_sets):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        L = int(rng.integers(3, 5))
        ncu = int(rng.integers(104, 305))
        sbw = float(_logu(rng, 0.5, 2.0))
        spk = float(_logu(rng, 0.5, 2.0))
        th = list(base.theta)
        for j in (0, 1, 2, 3, 23):
            th[j] *= sbw
        for j in range(8, 13):
            th[j] *= spk
        out.append(base.copy(n_levels=L, n_cu=ncu, theta=th))
    return out


def multi_arch_sizes(n_sets: int = 6, seed0: int = 110, lo: int = 1 << 18, hi: int = 1 << 22):
    out = []
    for i in range(n_sets):
        rng = np.random.Generator(np.random.PCG64(10_000 + seed0 + i))
        out.append(int(round(float(_logu(rng, lo, hi)))))
    return out


def perturb_theta(p: ParamSet, seed: int, factor: float = 1.5, mask=None) -> ParamSet:
    """theta0 = theta* x exp(U(-ln f, ln f)) on the slots in `mask`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.uniform(-math.log(factor), math.log(factor), N_THETA)
    th = list(p.theta)
    for j in range(N_THETA):
        if mask is None or (mask >> j) & 1:
            th[j] = th[j] * math.exp(z[j])
    return p.copy(theta=th)


# ---------------------------------------------------------------------------
# descriptors
# ---------------------------------------------------------------------------
def descriptors(n: int, seed: int = 100) -> Descriptors:
    """Kernel-descriptor sweep: flops log-U[1e6, 1e13], bytes log-U[1e4, 1e11],
    per-level reuse U(0,1), VGPRs/thread U-int[16, 512], LDS/WG U-int[0, 64 KiB],
    WG size in {64..1024}, grid round(log-U[1, 2^20]); dtype U{0..4};
    K round(log-U[1, 4096]); u U[0.4, 0.7]; W = 0 with p = 1/2 else
    log-U[1 MiB, 4 GiB]; n_conc, n_dev = 1 with p = 1/2 else U{2..8};
    fused ~ Bernoulli(1/4); n_sync = 0 with p = 1/2 else U{1..15}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f32 = np.float32
    F = _logu(rng, 1e6, 1e13, n).astype(f32)
    B = _logu(rng, 1e4, 1e11, n).astype(f32)
    r1 = rng.random(n, dtype=np.float32)
    r2 = rng.random(n, dtype=np.float32)
    r3 = rng.random(n, dtype=np.float32)
    K = np.round(_logu(rng, 1.0, 4096.0, n)).astype(f32)
    u = rng.uniform(0.4, 0.7, n).astype(f32)
    wsel = rng.random(n) < 0.5
    W = np.where(wsel, 0.0, _logu(rng, MIB, 4096.0 * MIB, n)).astype(f32)
    vgpr = rng.integers(16, 513, n, dtype=np.int32)
    lds = rng.integers(0, 65537, n, dtype=np.int32)
    g = np.array([64, 128, 256, 512, 1024], np.int32)[rng.integers(0, 5, n)]
    grid = np.round(_logu(rng, 1.0, float(1 << 20), n)).astype(np.int32)
    dtype = rng.integers(0, 5, n)
    nconc = np.where(rng.random(n) < 0.5, 1, rng.integers(2, 9, n))
    ndev = np.where(rng.random(n) < 0.5, 1, rng.integers(2, 9, n))
    fused = (rng.random(n) < 0.25).astype(np.int64)
    nsync = np.where(rng.random(n) < 0.5, 0, rng.integers(1, 16, n))
    gpack = pack_gpack(g, dtype, nconc, ndev, fused, nsync)
    return Descriptors(F, B, r1, r2, r3, K, u, W, vgpr, lds, gpack, grid)


def streaming_descriptors(n: int, seed: int = 500, w_lo_mib: float = 205.0,
                          c_llc_mib: float = 256.0) -> Descriptors:
    """Memory-streaming descriptors that sweep the working-set regimes, the
    synthetic counterpart of the paper's bandwidth and working-set
    microbenchmarks (Section IV-D): bytes log-U[1e8, 1e11], flops per byte
    log-U[1e-3, 1e-1], L1 / L2 hit rates U[0, 0.2], grids round(log-U[2^12,
    2^20]) of workgroups with U-int[16, 128] VGPRs and U-int[0, 16 KiB] LDS,
    K round(log-U[1, 64]); the other fields as in descriptors().  Working
    sets: 30 % W = 0 with an explicit LLC hit rate r3 ~ U(0, 1), 20 % inside
    the Infinity-Cache transition zone U[W_lo + 0.5, C - 0.5] MiB (Table
    "hlcc-piecewise"), 50 % log-U[8 MiB, 2 GiB] (below, across and above the
    cache, where Eq. (16) blends the HBM bandwidth)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = descriptors(n, seed + 1)
    f32 = np.float32
    d.B = _logu(rng, 1e8, 1e11, n).astype(f32)
    d.F = (d.B.astype(np.float64) * _logu(rng, 1e-3, 1e-1, n)).astype(f32)
    d.r1 = rng.uniform(0.0, 0.2, n).astype(f32)
    d.r2 = rng.uniform(0.0, 0.2, n).astype(f32)
    d.r3 = rng.random(n, dtype=f32)
    sel = rng.random(n)
    W = np.where(sel < 0.3, 0.0,
                 np.where(sel < 0.5, rng.uniform(w_lo_mib + 0.5, c_llc_mib - 0.5, n) * MIB,
                          _logu(rng, 8.0 * MIB, 2048.0 * MIB, n)))
    d.W = W.astype(f32)
    d.grid = np.round(_logu(rng, float(1 << 12), float(1 << 20), n)).astype(np.int32)
    d.vgpr = rng.integers(16, 129, n, dtype=np.int32)
    d.lds = rng.integers(0, 16385, n, dtype=np.int32)
    d.K = np.round(_logu(rng, 1.0, 64.0, n)).astype(f32)
    return d


def calibration_descriptors(n: int, seed: int = 103, stream_frac: float = 0.5) -> Descriptors:
    """The calibration sweep: descriptors(n - n_s, seed) followed by
    n_s = round(stream_frac * n) streaming_descriptors(n_s, seed + 400), so
    that the working-set slots (alpha, beta, w0, B_peak) are excited for a
    real share of the measurements, as the paper's calibration draws each
    parameter from a microbenchmark that isolates it."""
    ns = int(round(stream_frac * n))
    return Descriptors.concat([descriptors(n - ns, seed), streaming_descriptors(ns, seed + 400)])


def lognormal_noise(n: int, seed: int = 2, sigma: float = 0.02) -> np.ndarray:
    """Multiplicative measurement noise exp(sigma * z), z ~ N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(sigma * rng.standard_normal(n))


# ---------------------------------------------------------------------------
# GEMM-like shapes and ragged candidate tile lists
# ---------------------------------------------------------------------------
def tile_code(mt_code, nt_code, kd_code, wpw):
    return (np.asarray(mt_code) | (np.asarray(nt_code) << 2) | (np.asarray(kd_code) << 4)
            | ((np.asarray(wpw) - 1) << 6)).astype(np.uint32)


def all_tile_codes() -> np.ndarray:
    codes = [int(tile_code(a, b, c, w)) for a in range(4) for b in range(4)
             for c in range(3) for w in range(1, 9)]
    return np.array(codes, dtype=np.uint32)


@dataclasses.dataclass
class Shapes:
    M: np.ndarray
    N: np.ndarray
    K: np.ndarray
    dtype: np.ndarray
    cand_off: np.ndarray   # int32 [n+1], CSR offsets into cand_code
    cand_code: np.ndarray  # uint32 packed tile codes

    @property
    def n(self) -> int:
        return int(self.M.shape[0])


def shapes(n: int, seed: int = 102, cmin: int = 8, cmax: int = 96,
           lo: float = 128.0, hi: float = 16384.0) -> Shapes:
    """GEMM shapes with M, N, K round(log-U[128, 16384]) and dtype in
    {fp64, fp32, bf16, fp8}; each gets U-int[8, 96] distinct candidate tiles
    drawn without replacement from the 384 tiles, in shuffled order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = np.round(_logu(rng, lo, hi, n)).astype(np.int32)
    N = np.round(_logu(rng, lo, hi, n)).astype(np.int32)
    K = np.round(_logu(rng, lo, hi, n)).astype(np.int32)
    dt = rng.integers(0, 4, n).astype(np.int32)
    cnt = rng.integers(cmin, cmax + 1, n)
    tiles = all_tile_codes()
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    codes = np.empty(int(off[-1]), np.uint32)
    for i in range(n):
        codes[off[i]:off[i + 1]] = tiles[rng.permutation(N_TILES)[:cnt[i]]]
    return Shapes(M, N, K, dt, off.astype(np.int32), codes)


# ---------------------------------------------------------------------------
# workload segments: applications as lists of (kernel, executions) segments
# ---------------------------------------------------------------------------
SEG_CLASSES = ("memory", "compute", "balanced", "stencil")


@dataclasses.dataclass
class SegParams:
    """Per-class kernel-time scales, host<->device bandwidths (B/s) and the
    fixed cost per transfer episode (s).  Defaults: scales 1, 45 GB/s each
    way and 2 us per transfer (the defaults printed in Table "parameters")."""
    kappa: List[float] = dataclasses.field(default_factory=lambda: [1.0, 1.0, 1.0, 1.0])
    bw_h2d: float = 45e9
    bw_d2h: float = 45e9
    tau_memcpy: float = 2e-6


@dataclasses.dataclass
class Segments:
    app_off: np.ndarray   # int32 [n_apps + 1], CSR offsets into the segment rows
    n_exec: np.ndarray    # float32
    n_kern: np.ndarray    # int32 >= 1
    cls: np.ndarray       # int32 0..3
    h2d: np.ndarray       # float32 bytes per execution
    d2h: np.ndarray

    @property
    def n_apps(self) -> int:
        return int(self.app_off.shape[0] - 1)


def seg_params(seed: int = 7) -> SegParams:
    rng = np.random.Generator(np.random.PCG64(seed))
    return SegParams(kappa=[float(x) for x in rng.uniform(0.7, 1.5, 4)],
                     bw_h2d=float(_logu(rng, 20e9, 64e9)), bw_d2h=float(_logu(rng, 20e9, 64e9)),
                     tau_memcpy=float(_logu(rng, 1e-6, 10e-6)))


def segments(n_apps: int, seed: int = 120, smin: int = 1, smax: int = 12):
    """Applications with U-int[1, 12] segments each (multi-segment benchmarks
    of a few dominant kernels); per segment n_exec round(log-U[1, 1e4]),
    1-4 kernels per execution, class U{0..3}, host-to-device and
    device-to-host bytes 0 with p = 1/2 else log-U[1 KB, 1 GB].  Returns the
    segment table and a matching descriptor sweep (one kernel per segment,
    drawn as in descriptors() but with VGPRs/thread U-int[16, 128] so that
    every kernel fits on a CU)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cnt = rng.integers(smin, smax + 1, n_apps)
    off = np.zeros(n_apps + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    n = int(off[-1])
    n_exec = np.round(_logu(rng, 1.0, 1e4, n)).astype(np.float32)
    n_kern = rng.integers(1, 5, n).astype(np.int32)
    cls = rng.integers(0, 4, n).astype(np.int32)
    h2d = np.where(rng.random(n) < 0.5, 0.0, _logu(rng, 1e3, 1e9, n)).astype(np.float32)
    d2h = np.where(rng.random(n) < 0.5, 0.0, _logu(rng, 1e3, 1e9, n)).astype(np.float32)
    sg = Segments(off.astype(np.int32), n_exec, n_kern, cls, h2d, d2h)
    d = descriptors(n, seed + 1)
    # kernels of a running application launch: VGPRs/thread U-int[16, 128]
    d.vgpr = rng.integers(16, 129, n, dtype=np.int32)
    return sg, d


# ---------------------------------------------------------------------------
# kernel chains for fusion planning; grouped measurements for multipliers
# ---------------------------------------------------------------------------
def chains(n_chains: int, seed: int = 160, lmin: int = 2, lmax: int = 16):
    """Chains of U-int[lmin, lmax] kernels executed in order (the operator
    sequences a fusion pass looks at).  Returns (offsets int32 [n_chains + 1],
    descriptors, edge float32 [n]): each row's descriptor is drawn as in
    descriptors() with VGPRs U-int[16, 128]; edge[i] = bytes row i hands to
    row i + 1, U(0.05, 0.45) x min(B_i, B_i+1) (0 on a chain's last row)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cnt = rng.integers(lmin, lmax + 1, n_chains)
    off = np.zeros(n_chains + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    n = int(off[-1])
    d = descriptors(n, seed + 1)
    d.vgpr = rng.integers(16, 129, n, dtype=np.int32)
    nxtB = np.concatenate([d.B[1:], np.zeros(1, np.float32)]).astype(np.float64)
    edge = rng.uniform(0.05, 0.45, n) * np.minimum(d.B.astype(np.float64), nxtB)
    last = np.zeros(n, bool)
    last[off[1:] - 1] = True
    edge[last] = 0.0
    return off.astype(np.int32), d, edge.astype(np.float32)


def grouped_measurements(n_groups: int, seed: int = 170, gmin: int = 1, gmax: int = 40,
                         sigma: float = 0.05, holdout: float = 1.0 / 3.0):
    """Cases grouped for per-case multipliers: U-int[gmin, gmax] rows per
    group; each group's true factor log-U[0.5, 2]; returns (offsets int32
    [n_groups + 1], factor [n_groups], noise [n] (exp(sigma z)), train uint8 [n]
    with each row held out with probability `holdout`), plus descriptors for
    the rows.  Measured times are factor x T x noise for the caller's T."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cnt = rng.integers(gmin, gmax + 1, n_groups)
    off = np.zeros(n_groups + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    n = int(off[-1])
    factor = np.exp(rng.uniform(np.log(0.5), np.log(2.0), n_groups))
    noise = np.exp(sigma * rng.standard_normal(n))
    train = (rng.random(n) >= holdout).astype(np.uint8)
    d = descriptors(n, seed + 1)
    d.vgpr = rng.integers(16, 129, n, dtype=np.int32)
    return off.astype(np.int32), factor, noise, train, d


# ---------------------------------------------------------------------------
# Blackwell stage-centric family: parameter sets and tile-kernel descriptors
# ---------------------------------------------------------------------------
BW_THETA_NAMES = ("BW_TMEM_read", "BW_TMEM_write", "L_mma", "R_TC_fp64", "R_TC_tf32", "R_TC_fp16",
                  "R_TC_fp8", "R_TC_fp4", "S_2SM", "L_TMA", "B_TMA", "L_mbar", "L_commit", "BW_link",
                  "eta_DE", "R_decomp", "L_decomp_setup", "eps_exposed", "B_gmem", "L_store_setup",
                  "L_tmem_mgmt", "O_misc", "T_launch", "BW_dsmem")


@dataclasses.dataclass
class BwParamSet:
    """Structure plus the 24-slot Blackwell parameter vector (rates per SM,
    latencies in cycles, times in seconds)."""
    n_sm: int = 148
    max_cta: int = 1
    tmem_bytes: int = 256 * 1024
    f_clk: float = 1.965e9
    theta: List[float] = dataclasses.field(default_factory=lambda: [0.0] * N_THETA)

    def copy(self, **kw) -> "BwParamSet":
        d = dataclasses.asdict(self)
        d["theta"] = list(self.theta)
        d.update(kw)
        return BwParamSet(**d)


def b200_like() -> BwParamSet:
    """Values the paper prints for B200 (Table "parameters" and Section IV-A):
    TMEM 16 / 8 TB/s, L_TMA 420 cycles, tcgen05.mma latency 11-14 cycles
    (12), tensor throughput 44.8 (FP64) to 7702 (FP4) TFLOP/s over 148 SMs,
    L_mbar and L_commit 40-50 cycles (45), alpha 0.85-0.95 (exposed 0.1),
    2-SM speedup 1.30.  TF32/FP16/FP8 throughput, the TMA, link, store and
    DSMEM rates and the remaining latencies are not printed: placeholders."""
    sm = 148.0
    th = [0.0] * N_THETA
    th[0], th[1], th[2] = 16e12, 8e12, 12.0
    th[3:8] = [44.8e12 / sm, 1100e12 / sm, 2250e12 / sm, 4500e12 / sm, 7702e12 / sm]
    th[8], th[9], th[10] = 1.30, 420.0, 64e9
    th[11], th[12] = 45.0, 45.0
    th[13], th[14], th[15], th[16] = 64e9, 0.9, 256e9, 200.0
    th[17] = 0.1
    th[18], th[19] = 48e9, 500.0
    th[20], th[21], th[22], th[23] = 2000.0, 5e-9, 4e-6, 128e9
    return BwParamSet(theta=th)


def bw_param_set(seed: int = 0) -> BwParamSet:
    """Seeded synthetic Blackwell-style set around the b200_like values:
    each positive slot scaled by exp(U(+-ln 1.6)); the exposed fraction
    U[0.05, 0.3], the 2-SM speedup U[1.1, 1.6], eta_DE U[0.6, 0.95]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    base = b200_like()
    th = [float(t * np.exp(rng.uniform(-np.log(1.6), np.log(1.6)))) for t in base.theta]
    th[8] = float(rng.uniform(1.1, 1.6))
    th[14] = float(rng.uniform(0.6, 0.95))
    th[17] = float(rng.uniform(0.05, 0.3))
    return base.copy(theta=th, max_cta=int(rng.integers(1, 3)))


@dataclasses.dataclass
class BwDescriptors:
    bM: np.ndarray
    bN: np.ndarray
    bK: np.ndarray
    G: np.ndarray
    flags: np.ndarray
    Kt: np.ndarray
    CR: np.ndarray
    ob: np.ndarray

    @property
    def n(self) -> int:
        return int(self.bM.shape[0])

    def slice(self, a: int, b: int) -> "BwDescriptors":
        return BwDescriptors(*[getattr(self, f.name)[a:b] for f in dataclasses.fields(self)])


def pack_bw_flags(dtype, pair, stratB, PA, PB, nbar, comp):
    """Blackwell descriptor flags: [0,3) dtype, [3] 2-SM pair, [4] TMEM
    strategy B, [5,9) P_A - 1, [9,13) P_B - 1, [13,16) barriers, [16] compressed."""
    return (np.asarray(dtype) | (np.asarray(pair) << 3) | (np.asarray(stratB) << 4)
            | ((np.asarray(PA) - 1) << 5) | ((np.asarray(PB) - 1) << 9) | (np.asarray(nbar) << 13)
            | (np.asarray(comp) << 16)).astype(np.int32)


def bw_descriptors(n: int, seed: int = 200) -> BwDescriptors:
    """Tile-kernel sweep: bM, bN in {64, 128, 256}, bK in {16, 32, 64, 128},
    Kt round(log-U[1, 1024]), CTAs round(log-U[1, 2^16]), dtype U{0..4},
    2-SM pair and TMEM strategy B Bernoulli(1/2), P_A and P_B in {1, 2, 4}
    (1 with p = 1/2), barriers U{1, 2}, compressed Bernoulli(1/4) with
    CR U[1, 4], output element bytes in {2, 4}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tiles = np.array([64, 128, 256])
    bM = tiles[rng.integers(0, 3, n)].astype(np.int32)
    bN = tiles[rng.integers(0, 3, n)].astype(np.int32)
    bK = np.array([16, 32, 64, 128])[rng.integers(0, 4, n)].astype(np.int32)
    Kt = np.round(_logu(rng, 1.0, 1024.0, n)).astype(np.float32)
    G = np.round(_logu(rng, 1.0, 65536.0, n)).astype(np.int32)
    dt = rng.integers(0, 5, n)
    pair = (rng.random(n) < 0.5).astype(np.int64)
    sb = (rng.random(n) < 0.5).astype(np.int64)
    pp = np.array([1, 2, 4])
    PA = np.where(rng.random(n) < 0.5, 1, pp[rng.integers(0, 3, n)])
    PB = np.where(rng.random(n) < 0.5, 1, pp[rng.integers(0, 3, n)])
    nbar = rng.integers(1, 3, n)
    comp = (rng.random(n) < 0.25).astype(np.int64)
    CR = np.where(comp == 1, rng.uniform(1.0, 4.0, n), 1.0).astype(np.float32)
    ob = np.array([2.0, 4.0], np.float32)[rng.integers(0, 2, n)]
    return BwDescriptors(bM, bN, bK, G, pack_bw_flags(dt, pair, sb, PA, PB, nbar, comp), Kt, CR, ob)


def bw_tmem_tiles(n: int, seed: int = 600) -> BwDescriptors:
    """Compute-heavy Blackwell tiles that bring the TMEM and tensor-core
    terms of Eq. (2)/(3) forward: FP16/BF16, FP8 or FP4, bM in {128, 256},
    bN in {64, 128, 256}, bK in {16, 128}, TMEM strategy B and 2-SM pairs
    Bernoulli(1/2), multicast P_A, P_B in {2, 4} (less I/O per CTA), one or
    two barriers, no compression; K-steps, CTAs and output bytes as in
    bw_descriptors()."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = bw_descriptors(n, seed + 1)
    d.bM = np.array([128, 256])[rng.integers(0, 2, n)].astype(np.int32)
    d.bN = np.array([64, 128, 256])[rng.integers(0, 3, n)].astype(np.int32)
    d.bK = np.array([16, 128])[rng.integers(0, 2, n)].astype(np.int32)
    dt = rng.integers(2, 5, n)
    pair = (rng.random(n) < 0.5).astype(np.int64)
    sb = (rng.random(n) < 0.5).astype(np.int64)
    PA = np.array([2, 4])[rng.integers(0, 2, n)]
    PB = np.array([2, 4])[rng.integers(0, 2, n)]
    nbar = rng.integers(1, 3, n)
    d.flags = pack_bw_flags(dt, pair, sb, PA, PB, nbar, np.zeros(n, np.int64))
    d.CR = np.ones(n, np.float32)
    return d


def bw_calibration_descriptors(n: int, seed: int = 226, tmem_frac: float = 0.25) -> BwDescriptors:
    """The Blackwell calibration sweep: bw_descriptors(n - n_t, seed)
    followed by n_t = round(tmem_frac * n) bw_tmem_tiles(n_t, seed + 400)."""
    nt = int(round(tmem_frac * n))
    a, b = bw_descriptors(n - nt, seed), bw_tmem_tiles(nt, seed + 400)
    return BwDescriptors(*[np.concatenate([getattr(a, f.name), getattr(b, f.name)])
                           for f in dataclasses.fields(BwDescriptors)])


# Blackwell slots the calibration tests fit.  Held: eta_DE (Eq. (5) sees only
# the product BW_link eta_DE), the exposed fraction eps (it multiplies every
# I/O term, so it trades exactly against a common scale of the I/O rates and
# latencies), O_misc (a per-step constant in both regimes, it trades exactly
# against L_mma on compute-bound and eps L_TMA on I/O-bound steps) and the
# TMEM read rate (apart from the accumulator, which it shares with the write
# rate, it only sees the strategy-B A-tile read, at most ~2 % of a step).
BW_FIT_MASK = 0xFFFFFF & ~((1 << 0) | (1 << 14) | (1 << 17) | (1 << 21))

