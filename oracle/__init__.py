"""ctypes front-end of the FP64 CPU oracle (oracle/wm_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark use it; the product package never imports it.
It accepts the plain data containers of the seeded input generators
(parameter sets, descriptor arrays, shapes) and returns NumPy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
N_THETA = 24


class OrcParams(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "n_levels", "n_cu", "n_simd", "wave", "vgpr_simd", "vgpr_gran", "waves_simd",
        "lds_cu", "lds_gran", "bytes_inflight_wave", "mwp", "cwp", "combine", "pad_")] + [
        ("f_clk", C.c_double), ("w_lo_mib", C.c_double), ("c_llc_mib", C.c_double),
        ("theta", C.c_double * N_THETA)]


class OrcDesc(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "F", "B", "r1", "r2", "r3", "K", "u", "W", "vgpr", "lds", "gpack", "grid")] + [
        ("n", C.c_int64)]


class OrcTrace(C.Structure):
    _fields_ = [("valid", C.c_int32), ("stage", C.c_int32), ("eta_saturated", C.c_int32),
                ("pad_", C.c_int32)] + [(n, C.c_int64) for n in ("k", "o", "n_wf", "n_r", "n_eff")] + [
        ("h", C.c_double * 3), ("s", C.c_double * 4)] + [(n, C.c_double) for n in (
            "S", "Lam", "bw_hbm_eff", "blend_e", "T_c", "T_b", "T_lat", "T_m", "eta", "T_ov", "T")]


class OrcTile(C.Structure):
    _fields_ = [("valid", C.c_int32), ("pad_", C.c_int32)] + [
        (n, C.c_int64) for n in ("G", "Ks", "g", "v", "s")] + [
        (n, C.c_double) for n in ("F", "B", "U", "r2")]


class OrcCalibOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("order", C.c_int32)] + [
        (n, C.c_double) for n in ("lr", "lr_final", "beta1", "beta2", "eps")] + [
        ("free_mask", C.c_uint32), ("pad2_", C.c_uint32),
        ("lo", C.c_double * N_THETA), ("hi", C.c_double * N_THETA)]


_lib = None


def lib():
    """The oracle library: oracle/liboracle.so, or the variant build named by
    the WM_ORACLE_LIB environment variable (the sanitizer run of the pins)."""
    global _lib
    if _lib is None:
        path = os.environ.get("WM_ORACLE_LIB") or LIB_PATH
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = load(path)
    return _lib


def load(path):
    """Open an oracle library built from these sources (the default one, or a
    variant that the tests build, e.g. with sanitizers or a planted mistake)
    and declare its entry points."""
    L = C.CDLL(path)
    P, D = C.POINTER(OrcParams), C.POINTER(OrcDesc)
    vp = C.c_void_p
    L.orc_occupancy.argtypes = [P, C.c_int64, C.c_int64, C.c_int64, C.POINTER(C.c_int64)]
    L.orc_occupancy.restype = C.c_int64
    L.orc_h_llc.argtypes = [P, C.c_double]
    L.orc_h_llc.restype = C.c_double
    L.orc_bw_hbm_eff.argtypes = [P, C.c_double]
    L.orc_bw_hbm_eff.restype = C.c_double
    L.orc_eval.argtypes = [P] + [C.c_double] * 8 + [C.c_int64] * 4 + [C.POINTER(OrcTrace), vp]
    L.orc_eval.restype = None
    L.orc_predict.argtypes = [P, D, vp, vp]
    L.orc_trace.argtypes = [P, D, vp]
    L.orc_jacobian.argtypes = [P, D, vp]
    L.orc_roofline.argtypes = [P, D, vp]
    L.orc_weighted_grad.argtypes = [P, D, vp, C.c_int, vp]
    L.orc_calibrate.argtypes = [P, D, vp, C.POINTER(OrcCalibOpts), P, vp]
    L.orc_calibrate.restype = C.c_int
    L.orc_isotonic_inc.argtypes = [vp, C.c_int]
    L.orc_tile_derive.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_uint32,
                                  C.c_int64, C.POINTER(OrcTile)]
    L.orc_tile_cost.argtypes = [P, C.c_int64, C.c_int64, C.c_int64, C.c_int64, C.c_uint32]
    L.orc_tile_cost.restype = C.c_double
    L.orc_tile_costs.argtypes = [P, C.c_int64] + [vp] * 7
    L.orc_select_tile.argtypes = [P, C.c_int64] + [vp] * 9
    return L


# ----------------------------------------------------------------------------
def params(p) -> OrcParams:
    """Marshal a parameter set (any object with the generator's attributes)."""
    o = OrcParams()
    for f in ("n_levels", "n_cu", "n_simd", "wave", "vgpr_simd", "vgpr_gran", "waves_simd",
              "lds_cu", "lds_gran", "bytes_inflight_wave", "mwp", "cwp", "combine"):
        setattr(o, f, int(getattr(p, f)))
    o.f_clk = float(p.f_clk)
    o.w_lo_mib = float(p.w_lo_mib)
    o.c_llc_mib = float(p.c_llc_mib)
    for j in range(N_THETA):
        o.theta[j] = float(p.theta[j])
    return o


def theta_of(o: OrcParams) -> np.ndarray:
    return np.array([o.theta[j] for j in range(N_THETA)])


_FLOATS = ("F", "B", "r1", "r2", "r3", "K", "u", "W")
_INTS = ("vgpr", "lds", "gpack", "grid")


def _desc(d):
    keep = []
    o = OrcDesc()
    for f in _FLOATS:
        a = np.ascontiguousarray(getattr(d, f), dtype=np.float32)
        keep.append(a)
        setattr(o, f, a.ctypes.data)
    for f in _INTS:
        a = np.ascontiguousarray(getattr(d, f), dtype=np.int32)
        keep.append(a)
        setattr(o, f, a.ctypes.data)
    o.n = int(keep[0].shape[0])
    return o, keep


def predict(p, d):
    """FP64 predicted time T [s] and occupancy (WGs/CU; -1 invalid, 0 infeasible)."""
    o, keep = _desc(d)
    T = np.empty(o.n, np.float64)
    occ = np.empty(o.n, np.int32)
    lib().orc_predict(C.byref(params(p)), C.byref(o), T.ctypes.data, occ.ctypes.data)
    return T, occ


def trace(p, d):
    """Per-descriptor intermediates as a dict of arrays."""
    o, keep = _desc(d)
    buf = (OrcTrace * max(o.n, 1))()
    lib().orc_trace(C.byref(params(p)), C.byref(o), C.addressof(buf))
    arr = np.ctypeslib.as_array(buf)[: o.n]
    return {name: np.array(arr[name]) for name in arr.dtype.names if not name.startswith("pad")}


def eval_one(p, F, B, r1, r2, r3, K, u, W, v, s, gpack, G, with_grad=False, L=None):
    tr = OrcTrace()
    J = np.zeros(N_THETA) if with_grad else None
    (L or lib()).orc_eval(C.byref(params(p)), float(F), float(B), float(r1), float(r2), float(r3),
                   float(K), float(u), float(W), int(v), int(s), int(gpack), int(G), C.byref(tr),
                   J.ctypes.data if with_grad else None)
    return (tr, J) if with_grad else tr


def occupancy(p, v, s, g):
    k = C.c_int64()
    o = lib().orc_occupancy(C.byref(params(p)), int(v), int(s), int(g), C.byref(k))
    return int(o), int(k.value)


def h_llc(p, W):
    return lib().orc_h_llc(C.byref(params(p)), float(W))


def bw_hbm_eff(p, W):
    return lib().orc_bw_hbm_eff(C.byref(params(p)), float(W))


def jacobian(p, d):
    o, keep = _desc(d)
    J = np.empty((o.n, N_THETA), np.float64)
    lib().orc_jacobian(C.byref(params(p)), C.byref(o), J.ctypes.data)
    return J


def roofline(p, d):
    o, keep = _desc(d)
    T = np.empty(o.n, np.float64)
    lib().orc_roofline(C.byref(params(p)), C.byref(o), T.ctypes.data)
    return T


def vjp(p, d, dL_dT):
    o, keep = _desc(d)
    w = np.ascontiguousarray(dL_dT, dtype=np.float32)
    out = np.zeros(26)
    lib().orc_weighted_grad(C.byref(params(p)), C.byref(o), w.ctypes.data, 0, out.ctypes.data)
    return out[2:]


def loss_grad(p, d, measured):
    """(mean relative error, count, dL/dtheta[24]) in FP64."""
    o, keep = _desc(d)
    m = np.ascontiguousarray(measured, dtype=np.float32)
    out = np.zeros(26)
    lib().orc_weighted_grad(C.byref(params(p)), C.byref(o), m.ctypes.data, 1, out.ctypes.data)
    return float(out[0]), int(out[1]), out[2:].copy()


def calibrate(p0, d, measured, steps=500, lr=0.02, lr_final=0.0, beta1=0.9, beta2=0.999,
              eps=1e-8, free_mask=0xFFFFFF, lo=None, hi=None, order=0):
    """Adam on log(theta); lo / hi per-slot boxes (0 = none), order bit 0:
    slots 0-3 non-increasing, bit 1: slots 4-7 non-decreasing."""
    o, keep = _desc(d)
    m = np.ascontiguousarray(measured, dtype=np.float32)
    opts = OrcCalibOpts(steps=steps, order=order, lr=lr, lr_final=lr_final, beta1=beta1, beta2=beta2,
                        eps=eps, free_mask=free_mask)
    for j in range(N_THETA):
        opts.lo[j] = 0.0 if lo is None else float(lo[j])
        opts.hi[j] = 0.0 if hi is None else float(hi[j])
    pout = OrcParams()
    hist = np.zeros(max(steps, 1))
    rc = lib().orc_calibrate(C.byref(params(p0)), C.byref(o), m.ctypes.data, C.byref(opts),
                             C.byref(pout), hist.ctypes.data)
    return rc, theta_of(pout), hist[:steps]


def isotonic_inc(y):
    """The oracle's least-squares non-decreasing fit of y (pool adjacent
    violators)."""
    a = np.array(y, dtype=np.float64)
    lib().orc_isotonic_inc(a.ctypes.data, len(a))
    return a


def tile_derive(M, N, K, t, code, wave=64):
    o = OrcTile()
    lib().orc_tile_derive(int(M), int(N), int(K), int(t), int(code), int(wave), C.byref(o))
    return o


def tile_cost(p, M, N, K, t, code):
    return lib().orc_tile_cost(C.byref(params(p)), int(M), int(N), int(K), int(t), int(code))


def _shape_arrays(sh):
    a = [np.ascontiguousarray(x, dtype=np.int32) for x in (sh.M, sh.N, sh.K, sh.dtype, sh.cand_off)]
    a.append(np.ascontiguousarray(sh.cand_code, dtype=np.uint32))
    return a


def tile_costs(p, sh):
    a = _shape_arrays(sh)
    cost = np.empty(a[-1].shape[0], np.float64)
    lib().orc_tile_costs(C.byref(params(p)), sh.n, *[x.ctypes.data for x in a], cost.ctypes.data)
    return cost


def select_tile(p, sh):
    a = _shape_arrays(sh)
    n = sh.n
    best = np.empty(n, np.int32)
    cost = np.empty(n, np.float64)
    nt = np.empty(n, np.uint8)
    lib().orc_select_tile(C.byref(params(p)), n, *[x.ctypes.data for x in a], best.ctypes.data,
                          cost.ctypes.data, nt.ctypes.data)
    return best, cost, nt


# ----------------------------------------------------------------------------
# workload segments
# ----------------------------------------------------------------------------
class OrcSegs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("app_off", "n_exec", "n_kern", "cls", "h2d", "d2h")] + [
        ("n_apps", C.c_int64)]


class OrcSegp(C.Structure):
    _fields_ = [("kappa", C.c_double * 4), ("bw_h2d", C.c_double), ("bw_d2h", C.c_double),
                ("tau_memcpy", C.c_double)]


N_SEGP = 7


def _segs(sg):
    keep = [np.ascontiguousarray(sg.app_off, np.int32), np.ascontiguousarray(sg.n_exec, np.float32),
            np.ascontiguousarray(sg.n_kern, np.int32), np.ascontiguousarray(sg.cls, np.int32),
            np.ascontiguousarray(sg.h2d, np.float32), np.ascontiguousarray(sg.d2h, np.float32)]
    o = OrcSegs(*[k.ctypes.data for k in keep], int(keep[0].shape[0] - 1))
    return o, keep


def segp(q) -> OrcSegp:
    o = OrcSegp()
    for c in range(4):
        o.kappa[c] = float(q.kappa[c])
    o.bw_h2d, o.bw_d2h, o.tau_memcpy = float(q.bw_h2d), float(q.bw_d2h), float(q.tau_memcpy)
    return o


def _seg_lib():
    L = lib()
    if not hasattr(L, "_seg_ready"):
        P, D = C.POINTER(OrcParams), C.POINTER(OrcDesc)
        L.orc_predict_apps.argtypes = [P, C.POINTER(OrcSegp), D, C.POINTER(OrcSegs), C.c_void_p, C.c_void_p]
        L.orc_apps_loss_grad.argtypes = [P, C.POINTER(OrcSegp), D, C.POINTER(OrcSegs), C.c_void_p, C.c_void_p]
        L.orc_segment.argtypes = [P, C.POINTER(OrcSegp), D, C.POINTER(OrcSegs), C.c_int64, C.c_void_p, C.c_void_p]
        L.orc_segment.restype = C.c_double
        L._seg_ready = True
    return L


def predict_apps(p, q, d, sg):
    """(T_app float64 [n_apps], T_seg float64 [n_segments])."""
    o, keep = _desc(d)
    so, skeep = _segs(sg)
    Ta = np.empty(so.n_apps, np.float64)
    Ts = np.empty(o.n, np.float64)
    _seg_lib().orc_predict_apps(C.byref(params(p)), C.byref(segp(q)), C.byref(o), C.byref(so),
                                Ta.ctypes.data, Ts.ctypes.data)
    return Ta, Ts


def apps_loss_grad(p, q, d, sg, measured):
    """(loss, count, dL/dtheta[24], dL/dsegparam[7])."""
    o, keep = _desc(d)
    so, skeep = _segs(sg)
    m = np.ascontiguousarray(measured, np.float64)
    out = np.zeros(2 + N_THETA + N_SEGP)
    _seg_lib().orc_apps_loss_grad(C.byref(params(p)), C.byref(segp(q)), C.byref(o), C.byref(so),
                                  m.ctypes.data, out.ctypes.data)
    return float(out[0]), int(out[1]), out[2:2 + N_THETA].copy(), out[2 + N_THETA:].copy()


# ----------------------------------------------------------------------------
# calibration multipliers and fusion planning
# ----------------------------------------------------------------------------
class OrcFDesc(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("F", "B", "r1", "r2", "r3", "K", "u", "W")] + [
        (n, C.c_int64) for n in ("v", "s", "gpack", "G")]


def _plan_lib():
    L = lib()
    if not hasattr(L, "_plan_ready"):
        P, D = C.POINTER(OrcParams), C.POINTER(OrcDesc)
        vp = C.c_void_p
        L.orc_fit_multipliers.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp, vp]
        L.orc_fuse.argtypes = [P, D, vp, C.c_int64, C.c_int64, C.POINTER(OrcFDesc)]
        L.orc_fuse.restype = C.c_int
        L.orc_fused_cost.argtypes = [P, D, vp, C.c_int64, C.c_int64]
        L.orc_fused_cost.restype = C.c_double
        L.orc_plan_fusion.argtypes = [P, D, vp, vp, C.c_int64, C.c_int32, vp, vp, vp]
        L._plan_ready = True
    return L


def fit_multipliers(T, m, off, train):
    """(mult [n_groups], T_scaled [n], (train loss sum, train count, holdout
    loss sum, holdout count))."""
    T = np.ascontiguousarray(T, np.float64)
    m = np.ascontiguousarray(m, np.float64)
    off = np.ascontiguousarray(off, np.int32)
    tr = np.ascontiguousarray(train, np.uint8)
    ng = off.shape[0] - 1
    mult = np.empty(max(ng, 1), np.float64)
    Ts = np.empty(max(T.shape[0], 1), np.float64)
    st = np.zeros(4)
    _plan_lib().orc_fit_multipliers(T.ctypes.data, m.ctypes.data, off.ctypes.data, ng, tr.ctypes.data,
                                    mult.ctypes.data, Ts.ctypes.data, st.ctypes.data)
    return mult[:ng], Ts[:T.shape[0]], tuple(st)


def fuse(p, d, edge, a, length):
    """(ok, dict of the fused descriptor's fields)."""
    o, keep = _desc(d)
    e = np.ascontiguousarray(edge, np.float32)
    f = OrcFDesc()
    ok = _plan_lib().orc_fuse(C.byref(params(p)), C.byref(o), e.ctypes.data, int(a), int(length), C.byref(f))
    return bool(ok), {n: getattr(f, n) for n, _ in OrcFDesc._fields_}


def fused_cost(p, d, edge, a, length):
    o, keep = _desc(d)
    e = np.ascontiguousarray(edge, np.float32)
    return _plan_lib().orc_fused_cost(C.byref(params(p)), C.byref(o), e.ctypes.data, int(a), int(length))


def plan_fusion(p, d, edge, off, R):
    """(total [n_chains], unfused [n_chains], start uint8 [n])."""
    o, keep = _desc(d)
    e = np.ascontiguousarray(edge, np.float32)
    off = np.ascontiguousarray(off, np.int32)
    nc = off.shape[0] - 1
    tot = np.empty(max(nc, 1))
    unf = np.empty(max(nc, 1))
    st = np.zeros(max(o.n, 1), np.uint8)
    _plan_lib().orc_plan_fusion(C.byref(params(p)), C.byref(o), e.ctypes.data, off.ctypes.data, nc, int(R),
                                tot.ctypes.data, unf.ctypes.data, st.ctypes.data)
    return tot[:nc], unf[:nc], st[:o.n]


# ----------------------------------------------------------------------------
# Blackwell stage-centric family (bw_oracle.c)
# ----------------------------------------------------------------------------
BW_NTHETA = 24


class BwParams(C.Structure):
    _fields_ = [("n_sm", C.c_int32), ("max_cta", C.c_int32), ("tmem_bytes", C.c_int64),
                ("f_clk", C.c_double), ("theta", C.c_double * BW_NTHETA)]


class BwDesc(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("bM", "bN", "bK", "G", "flags", "Kt", "CR", "ob")] + [
        ("n", C.c_int64)]


class BwTrace(C.Structure):
    _fields_ = [("valid", C.c_int32), ("compute_bound", C.c_int32), ("c", C.c_int32), ("pad_", C.c_int32),
                ("n_r", C.c_int64)] + [(n, C.c_double) for n in (
                    "MA", "MB", "D_acc", "T_tmem", "T_mgmt", "T_compute", "T_tma", "T_decomp", "T_dsm",
                    "T_sync", "T_io", "T_step", "T_store", "T")]


def _bw_lib():
    L = lib()
    if not hasattr(L, "_bw_ready"):
        P, D = C.POINTER(BwParams), C.POINTER(BwDesc)
        vp = C.c_void_p
        L.bw_eval.argtypes = [P] + [C.c_int64] * 5 + [C.c_double] * 3 + [C.POINTER(BwTrace), vp]
        L.bw_predict.argtypes = [P, D, vp, vp]
        L.bw_trace.argtypes = [P, D, vp]
        L.bw_jacobian.argtypes = [P, D, vp]
        L.bw_weighted_grad.argtypes = [P, D, vp, C.c_int, vp]
        L.bw_calibrate.argtypes = [P, D, vp, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                   C.c_double, C.c_uint32, P, vp]
        L.bw_calibrate.restype = C.c_int
        L._bw_ready = True
    return L


def bw_params(p) -> BwParams:
    o = BwParams()
    o.n_sm, o.max_cta, o.tmem_bytes, o.f_clk = int(p.n_sm), int(p.max_cta), int(p.tmem_bytes), float(p.f_clk)
    for j in range(BW_NTHETA):
        o.theta[j] = float(p.theta[j])
    return o


_BW_INT = ("bM", "bN", "bK", "G", "flags")
_BW_FLT = ("Kt", "CR", "ob")


def _bw_desc(d):
    keep = []
    o = BwDesc()
    for f in _BW_INT:
        a = np.ascontiguousarray(getattr(d, f), np.int32)
        keep.append(a)
        setattr(o, f, a.ctypes.data)
    for f in _BW_FLT:
        a = np.ascontiguousarray(getattr(d, f), np.float32)
        keep.append(a)
        setattr(o, f, a.ctypes.data)
    o.n = int(keep[0].shape[0])
    return o, keep


def bw_eval_one(p, bM, bN, bK, G, flags, Kt, CR, ob, with_grad=False):
    tr = BwTrace()
    J = np.zeros(BW_NTHETA) if with_grad else None
    _bw_lib().bw_eval(C.byref(bw_params(p)), int(bM), int(bN), int(bK), int(G), int(flags), float(Kt),
                      float(CR), float(ob), C.byref(tr), J.ctypes.data if with_grad else None)
    return (tr, J) if with_grad else tr


def bw_predict(p, d):
    o, keep = _bw_desc(d)
    T = np.empty(max(o.n, 1))
    c = np.empty(max(o.n, 1), np.int32)
    _bw_lib().bw_predict(C.byref(bw_params(p)), C.byref(o), T.ctypes.data, c.ctypes.data)
    return T[:o.n], c[:o.n]


def bw_trace(p, d):
    o, keep = _bw_desc(d)
    buf = (BwTrace * max(o.n, 1))()
    _bw_lib().bw_trace(C.byref(bw_params(p)), C.byref(o), C.addressof(buf))
    arr = np.ctypeslib.as_array(buf)[: o.n]
    return {name: np.array(arr[name]) for name in arr.dtype.names if not name.startswith("pad")}


def bw_jacobian(p, d):
    o, keep = _bw_desc(d)
    J = np.empty((max(o.n, 1), BW_NTHETA))
    _bw_lib().bw_jacobian(C.byref(bw_params(p)), C.byref(o), J.ctypes.data)
    return J[:o.n]


def bw_vjp(p, d, w):
    o, keep = _bw_desc(d)
    wv = np.ascontiguousarray(w, np.float32)
    out = np.zeros(26)
    _bw_lib().bw_weighted_grad(C.byref(bw_params(p)), C.byref(o), wv.ctypes.data, 0, out.ctypes.data)
    return out[2:]


def bw_loss_grad(p, d, measured):
    o, keep = _bw_desc(d)
    m = np.ascontiguousarray(measured, np.float32)
    out = np.zeros(26)
    _bw_lib().bw_weighted_grad(C.byref(bw_params(p)), C.byref(o), m.ctypes.data, 1, out.ctypes.data)
    return float(out[0]), int(out[1]), out[2:].copy()


def bw_calibrate(p0, d, measured, steps=500, lr=0.05, lr_final=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 free_mask=0xFFFFFF):
    o, keep = _bw_desc(d)
    m = np.ascontiguousarray(measured, np.float32)
    pout = BwParams()
    hist = np.zeros(steps)
    rc = _bw_lib().bw_calibrate(C.byref(bw_params(p0)), C.byref(o), m.ctypes.data, int(steps), lr, lr_final,
                                beta1, beta2, eps, int(free_mask), C.byref(pout), hist.ctypes.data)
    return rc, np.array([pout.theta[j] for j in range(BW_NTHETA)]), hist


def apps_vjp(p, q, d, sg, w_app):
    """(sum_a w_a dT_a/dtheta [24], sum_a w_a dT_a/dsegparam [7])."""
    L = _seg_lib()
    if not hasattr(L, "_vjp_ready"):
        L.orc_apps_vjp.argtypes = [C.POINTER(OrcParams), C.POINTER(OrcSegp), C.POINTER(OrcDesc),
                                   C.POINTER(OrcSegs), C.c_void_p, C.c_void_p]
        L._vjp_ready = True
    o, keep = _desc(d)
    so, skeep = _segs(sg)
    w = np.ascontiguousarray(w_app, np.float64)
    out = np.zeros(N_THETA + N_SEGP)
    L.orc_apps_vjp(C.byref(params(p)), C.byref(segp(q)), C.byref(o), C.byref(so), w.ctypes.data,
                   out.ctypes.data)
    return out[:N_THETA].copy(), out[N_THETA:].copy()


def set_threads(n: int = 0) -> int:
    """Set the OpenMP thread count (n > 0); returns the count in effect."""
    L = lib()
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = C.c_int
    return int(L.orc_set_threads(int(n)))
