"""Python binding of libwavemodel.so (include/wavemodel.h).

Argument marshalling only: every step of the model runs in the HIP kernels of
the library.  PyTorch supplies device memory and the current stream.  The
library must be built (``python -m paper_2605_04178_amd.build``); without it
every call raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwavemodel.so")
N_THETA = 24

WM_OK, WM_EINVAL, WM_EWORKSPACE, WM_EHIP, WM_EDIVERGED, WM_ETOOLARGE = 0, -1, -2, -3, -4, -5
NOALLOC_MAX_N = 1 << 26
(OP_PREDICT, OP_ROOFLINE, OP_VJP, OP_LOSS_GRAD, OP_SELECT_TILE, OP_CALIBRATE, OP_CALIBRATE_BATCHED,
 OP_PREDICT_APPS, OP_APPS_LOSS_GRAD, OP_FIT_MULTIPLIERS) = range(10)
N_SEGPARAMS = 7

EXPORTED = ("wm_strerror", "wm_last_hip_error", "wm_validate_params", "wm_workspace_bytes",
            "wm_predict", "wm_roofline", "wm_predict_vjp", "wm_loss_grad", "wm_select_tile",
            "wm_calibrate", "wm_calibrate_batched", "wm_get_launch", "wm_set_launch",
            "wm_autotune_predict", "wm_autotune_grad", "wm_autotune_select_tile",
            "wm_autotune_batched", "wm_apps_workspace_bytes", "wm_predict_apps", "wm_apps_loss_grad",
            "wm_autotune_apps", "wm_fit_multipliers", "wm_plan_workspace_bytes", "wm_plan_fusion",
            "wm_bw_validate_params", "wm_bw_workspace_bytes", "wm_bw_predict", "wm_bw_predict_vjp",
            "wm_bw_loss_grad", "wm_bw_calibrate", "wm_predict_apps_vjp", "wm_loss_grad_noalloc",
            "wm_noalloc_scratch_bytes", "wm_predict_vjp_exact", "wm_loss_grad_exact", "wm_tile_costs",
            "wm_calibrate_resume")
BW_OP_GRAD, BW_OP_CALIBRATE = 0, 1


class WmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = f"{what}: {lib().wm_strerror(status).decode()} ({status})"
        if status == WM_EHIP:
            msg += f", hip error {lib().wm_last_hip_error()}"
        super().__init__(msg)


class WmParams(C.Structure):
    _fields_ = [(n, C.c_int32) for n in (
        "n_levels", "n_cu", "n_simd", "wave", "vgpr_simd", "vgpr_gran", "waves_simd", "lds_cu",
        "lds_gran", "bytes_inflight_wave", "mwp", "cwp", "combine", "reserved")] + [
        ("f_clk", C.c_double), ("w_lo_mib", C.c_double), ("c_llc_mib", C.c_double),
        ("theta", C.c_double * N_THETA)]


class WmDesc(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "F", "B", "r1", "r2", "r3", "K", "u", "W", "vgpr", "lds", "gpack", "grid")] + [("n", C.c_int64)]


class WmShapes(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("M", "N", "K", "dtype")] + [("n", C.c_int64)]


class WmLaunch(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("block", "per_thread", "grid_mult", "chunk")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


class WmSegs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("app_off", "n_exec", "n_kern", "cls", "h2d", "d2h")] + [
        ("n_apps", C.c_int64)]


class WmSegParams(C.Structure):
    _fields_ = [("kappa", C.c_double * 4), ("bw_h2d", C.c_double), ("bw_d2h", C.c_double),
                ("tau_memcpy", C.c_double)]


class WmBwParams(C.Structure):
    _fields_ = [("n_sm", C.c_int32), ("max_cta", C.c_int32), ("tmem_bytes", C.c_int64),
                ("f_clk", C.c_double), ("theta", C.c_double * N_THETA)]


class WmBwDesc(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("bM", "bN", "bK", "G", "flags", "Kt", "CR", "ob")] + [
        ("n", C.c_int64)]


class WmCalibState(C.Structure):
    _fields_ = [(n, C.c_double * N_THETA) for n in ("theta", "theta_ok", "phi", "m", "v")] + [
        ("step", C.c_int32), ("diverged", C.c_int32)]


class WmCalibOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("order", C.c_int32)] + [
        (n, C.c_double) for n in ("lr", "lr_final", "beta1", "beta2", "eps")] + [
        ("free_mask", C.c_uint32), ("reserved2", C.c_uint32),
        ("lo", C.c_double * N_THETA), ("hi", C.c_double * N_THETA)]


# order bits of a calibration: bandwidths L1 >= L2 >= LLC >= HBM (slots 0-3),
# latencies L1 <= L2 <= LLC <= HBM (slots 4-7)
ORDER_BW, ORDER_LAT = 1, 2


_lib = None


def lib():
    """Load libwavemodel.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2605_04178_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        P, D = C.POINTER(WmParams), C.POINTER(WmDesc)
        L.wm_strerror.argtypes = [i32]
        L.wm_strerror.restype = C.c_char_p
        L.wm_last_hip_error.argtypes = []
        L.wm_last_hip_error.restype = i32
        L.wm_validate_params.argtypes = [P]
        L.wm_validate_params.restype = i32
        L.wm_workspace_bytes.argtypes = [i32, i64, i32, i32]
        L.wm_workspace_bytes.restype = sz
        L.wm_predict.argtypes = [D, P, vp, vp, vp]
        L.wm_predict.restype = i32
        L.wm_roofline.argtypes = [D, P, vp, vp]
        L.wm_roofline.restype = i32
        L.wm_predict_vjp.argtypes = [D, P, vp, vp, vp, sz, vp]
        L.wm_predict_vjp.restype = i32
        L.wm_loss_grad.argtypes = [D, vp, P, vp, vp, sz, vp]
        L.wm_loss_grad.restype = i32
        L.wm_predict_vjp_exact.argtypes = [D, P, vp, vp, vp, sz, vp]
        L.wm_predict_vjp_exact.restype = i32
        L.wm_loss_grad_exact.argtypes = [D, vp, P, vp, vp, sz, vp]
        L.wm_loss_grad_exact.restype = i32
        L.wm_loss_grad_noalloc.argtypes = [D, vp, P, vp, vp]
        L.wm_loss_grad_noalloc.restype = i32
        L.wm_noalloc_scratch_bytes.argtypes = []
        L.wm_noalloc_scratch_bytes.restype = sz
        L.wm_select_tile.argtypes = [C.POINTER(WmShapes), vp, vp, i64, P, vp, vp, vp, vp]
        L.wm_tile_costs.argtypes = [C.POINTER(WmShapes), vp, vp, i64, P, vp, vp]
        L.wm_tile_costs.restype = i32
        L.wm_select_tile.restype = i32
        L.wm_calibrate.argtypes = [D, vp, P, C.POINTER(WmCalibOpts), P, vp, vp, sz, vp]
        L.wm_calibrate.restype = i32
        L.wm_calibrate_resume.argtypes = [D, vp, P, C.POINTER(WmCalibOpts), C.POINTER(WmCalibState), i32,
                                          C.POINTER(WmCalibState), P, vp, vp, sz, vp]
        L.wm_calibrate_resume.restype = i32
        L.wm_calibrate_batched.argtypes = [i32, D, vp, P, C.POINTER(WmCalibOpts), P, vp, vp, sz, vp]
        L.wm_calibrate_batched.restype = i32
        LP = C.POINTER(WmLaunch)
        dp = C.POINTER(C.c_double)
        L.wm_get_launch.argtypes = [i32, i64, LP]
        L.wm_get_launch.restype = i32
        L.wm_set_launch.argtypes = [i32, i64, LP]
        L.wm_set_launch.restype = i32
        L.wm_autotune_predict.argtypes = [D, P, vp, vp, vp, LP, dp]
        L.wm_autotune_predict.restype = i32
        L.wm_autotune_grad.argtypes = [i32, D, vp, P, vp, vp, sz, vp, LP, dp]
        L.wm_autotune_grad.restype = i32
        L.wm_autotune_select_tile.argtypes = [C.POINTER(WmShapes), vp, vp, i64, P, vp, vp, vp, vp, LP, dp]
        L.wm_autotune_select_tile.restype = i32
        L.wm_autotune_batched.argtypes = [i32, D, vp, P, C.POINTER(WmCalibOpts), vp, sz, vp, LP, dp]
        L.wm_autotune_batched.restype = i32
        SG, SP = C.POINTER(WmSegs), C.POINTER(WmSegParams)
        L.wm_apps_workspace_bytes.argtypes = [i64, i64]
        L.wm_apps_workspace_bytes.restype = sz
        L.wm_predict_apps.argtypes = [D, SG, P, SP, vp, vp, vp]
        L.wm_predict_apps.restype = i32
        L.wm_apps_loss_grad.argtypes = [D, SG, vp, P, SP, vp, vp, sz, vp]
        L.wm_apps_loss_grad.restype = i32
        L.wm_predict_apps_vjp.argtypes = [D, SG, vp, P, SP, vp, vp, sz, vp]
        L.wm_predict_apps_vjp.restype = i32
        L.wm_autotune_apps.argtypes = [i32, D, SG, vp, P, SP, vp, vp, vp, sz, vp, LP, dp]
        L.wm_autotune_apps.restype = i32
        L.wm_fit_multipliers.argtypes = [vp, vp, vp, i64, i64, vp, vp, vp, vp, vp, sz, vp]
        L.wm_fit_multipliers.restype = i32
        L.wm_plan_workspace_bytes.argtypes = [i64, i32]
        L.wm_plan_workspace_bytes.restype = sz
        L.wm_plan_fusion.argtypes = [D, vp, vp, i64, i32, P, vp, vp, vp, vp, sz, vp]
        L.wm_plan_fusion.restype = i32
        BP, BD = C.POINTER(WmBwParams), C.POINTER(WmBwDesc)
        L.wm_bw_validate_params.argtypes = [BP]
        L.wm_bw_validate_params.restype = i32
        L.wm_bw_workspace_bytes.argtypes = [i32, i64, i32]
        L.wm_bw_workspace_bytes.restype = sz
        L.wm_bw_predict.argtypes = [BD, BP, vp, vp, vp]
        L.wm_bw_predict.restype = i32
        L.wm_bw_predict_vjp.argtypes = [BD, BP, vp, vp, vp, sz, vp]
        L.wm_bw_predict_vjp.restype = i32
        L.wm_bw_loss_grad.argtypes = [BD, vp, BP, vp, vp, sz, vp]
        L.wm_bw_loss_grad.restype = i32
        L.wm_bw_calibrate.argtypes = [BD, vp, BP, C.POINTER(WmCalibOpts), BP, vp, vp, sz, vp]
        L.wm_bw_calibrate.restype = i32
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != WM_OK:
        raise WmError(rc, what)


# ---------------------------------------------------------------------------
# marshalling
# ---------------------------------------------------------------------------
_PFIELDS = ("n_levels", "n_cu", "n_simd", "wave", "vgpr_simd", "vgpr_gran", "waves_simd", "lds_cu",
            "lds_gran", "bytes_inflight_wave", "mwp", "cwp", "combine")


def params_struct(p, theta: Optional[Sequence[float]] = None) -> WmParams:
    """Marshal any object with the parameter-set attributes (structural ints,
    f_clk, w_lo_mib, c_llc_mib, theta[24])."""
    o = WmParams()
    for f in _PFIELDS:
        setattr(o, f, int(getattr(p, f)))
    o.f_clk = float(p.f_clk)
    o.w_lo_mib = float(p.w_lo_mib)
    o.c_llc_mib = float(p.c_llc_mib)
    th = p.theta if theta is None else theta
    for j in range(N_THETA):
        o.theta[j] = float(th[j])
    return o


def theta_of(o: WmParams) -> np.ndarray:
    return np.array([o.theta[j] for j in range(N_THETA)])


def validate_params(p) -> bool:
    return lib().wm_validate_params(C.byref(params_struct(p))) == WM_OK


def workspace_bytes(op: int, n: int, n_sets: int = 1, steps: int = 0) -> int:
    return int(lib().wm_workspace_bytes(op, n, n_sets, steps))


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _workspace(nbytes: int, device) -> Optional[torch.Tensor]:
    if nbytes == 0:
        return None
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


class DeviceDescriptors:
    """The 12 structure-of-arrays descriptor fields as device tensors."""
    FLOATS = ("F", "B", "r1", "r2", "r3", "K", "u", "W")
    INTS = ("vgpr", "lds", "gpack", "grid")

    def __init__(self, tensors: dict):
        n = None
        for f in self.FLOATS + self.INTS:
            t = tensors[f]
            want = torch.float32 if f in self.FLOATS else torch.int32
            if t.dtype != want or not t.is_contiguous() or t.dim() != 1:
                raise ValueError(f"descriptor field {f} must be a contiguous 1-D {want} tensor")
            if n is None:
                n = t.shape[0]
            if t.shape[0] != n:
                raise ValueError("descriptor fields differ in length")
            setattr(self, f, t)
        self.n = int(n)
        self.device = tensors["F"].device

    @classmethod
    def from_host(cls, d, device="cuda") -> "DeviceDescriptors":
        out = {}
        for f in cls.FLOATS + cls.INTS:
            a = np.ascontiguousarray(getattr(d, f))
            out[f] = torch.from_numpy(a).to(device)
        return cls(out)

    def slice(self, a: int, b: int) -> "DeviceDescriptors":
        return DeviceDescriptors({f: getattr(self, f)[a:b] for f in self.FLOATS + self.INTS})

    def struct(self) -> WmDesc:
        o = WmDesc()
        for f in self.FLOATS + self.INTS:
            setattr(o, f, getattr(self, f).data_ptr())
        o.n = self.n
        return o


class DeviceSegments:
    """Segment rows (parallel to a DeviceDescriptors) and application offsets
    as device tensors."""
    FIELDS = (("app_off", torch.int32), ("n_exec", torch.float32), ("n_kern", torch.int32),
              ("cls", torch.int32), ("h2d", torch.float32), ("d2h", torch.float32))

    def __init__(self, tensors: dict):
        for f, dt in self.FIELDS:
            t = tensors[f]
            if t.dtype != dt or not t.is_contiguous() or t.dim() != 1:
                raise ValueError(f"segment field {f} must be a contiguous 1-D {dt} tensor")
            setattr(self, f, t)
        self.n = int(self.n_exec.shape[0])
        for f, _ in self.FIELDS[1:]:
            if getattr(self, f).shape[0] != self.n:
                raise ValueError("segment fields differ in length")
        self.n_apps = int(self.app_off.shape[0]) - 1
        if self.n_apps < 0:
            raise ValueError("app_off needs n_apps + 1 entries")
        self.device = self.n_exec.device

    @classmethod
    def from_host(cls, sg, device="cuda") -> "DeviceSegments":
        out = {}
        for f, dt in cls.FIELDS:
            npdt = np.int32 if dt == torch.int32 else np.float32
            out[f] = torch.from_numpy(np.ascontiguousarray(getattr(sg, f), dtype=npdt)).to(device)
        return cls(out)

    def struct(self) -> WmSegs:
        o = WmSegs()
        for f, _ in self.FIELDS:
            setattr(o, f, getattr(self, f).data_ptr())
        o.n_apps = self.n_apps
        return o


def segparams_struct(q) -> WmSegParams:
    """Marshal segment parameters (kappa[4], bw_h2d, bw_d2h, tau_memcpy)."""
    o = WmSegParams()
    for c in range(4):
        o.kappa[c] = float(q.kappa[c])
    o.bw_h2d, o.bw_d2h, o.tau_memcpy = float(q.bw_h2d), float(q.bw_d2h), float(q.tau_memcpy)
    return o


class DeviceShapes:
    def __init__(self, M, N, K, dtype, cand_off, cand_code):
        self.M, self.N, self.K, self.dtype = M, N, K, dtype
        self.cand_off, self.cand_code = cand_off, cand_code
        self.n = int(M.shape[0])
        self.device = M.device

    @classmethod
    def from_host(cls, sh, device="cuda") -> "DeviceShapes":
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
        return cls(t(sh.M, np.int32), t(sh.N, np.int32), t(sh.K, np.int32), t(sh.dtype, np.int32),
                   t(sh.cand_off, np.int32), t(sh.cand_code.view(np.int32), np.int32))


# ---------------------------------------------------------------------------
# calls
# ---------------------------------------------------------------------------
def predict(desc: DeviceDescriptors, params, out_T=None, out_occ=None, want_occ=True, stream=None):
    """Predicted time T (float32 seconds) and occupancy (int32, or None)."""
    T = out_T if out_T is not None else torch.empty(desc.n, dtype=torch.float32, device=desc.device)
    occ = out_occ
    if occ is None and want_occ:
        occ = torch.empty(desc.n, dtype=torch.int32, device=desc.device)
    ds = desc.struct()
    ps = params_struct(params)
    _check(lib().wm_predict(C.byref(ds), C.byref(ps), _ptr(T), _ptr(occ), _stream(stream)), "wm_predict")
    return T, occ


def roofline(desc: DeviceDescriptors, params, stream=None):
    T = torch.empty(desc.n, dtype=torch.float32, device=desc.device)
    _check(lib().wm_roofline(C.byref(desc.struct()), C.byref(params_struct(params)), _ptr(T),
                             _stream(stream)), "wm_roofline")
    return T


def vjp(desc: DeviceDescriptors, params, dL_dT: torch.Tensor, ws=None, theta=None, stream=None,
        exact=False):
    """dL/dtheta (float64 [24], device) for an upstream gradient dL/dT;
    exact=True calls wm_predict_vjp_exact (float64 throughout the sweep)."""
    out = torch.empty(N_THETA, dtype=torch.float64, device=desc.device)
    if ws is None:
        ws = _workspace(workspace_bytes(OP_VJP, desc.n), desc.device)
    nb = 0 if ws is None else ws.numel()
    fn = lib().wm_predict_vjp_exact if exact else lib().wm_predict_vjp
    rc = fn(C.byref(desc.struct()), C.byref(params_struct(params, theta)),
            _ptr(dL_dT.contiguous()), _ptr(out), _ptr(ws), nb, _stream(stream))
    _check(rc, "wm_predict_vjp_exact" if exact else "wm_predict_vjp")
    return out


def loss_grad(desc: DeviceDescriptors, measured: torch.Tensor, params, ws=None, theta=None,
              out=None, stream=None, exact=False):
    """[loss, count, grad[24]] float64 on the device (mean relative error);
    exact=True calls wm_loss_grad_exact (float64 throughout the sweep)."""
    if out is None:
        out = torch.empty(26, dtype=torch.float64, device=desc.device)
    if ws is None:
        ws = _workspace(workspace_bytes(OP_LOSS_GRAD, desc.n), desc.device)
    nb = 0 if ws is None else ws.numel()
    fn = lib().wm_loss_grad_exact if exact else lib().wm_loss_grad
    rc = fn(C.byref(desc.struct()), _ptr(measured), C.byref(params_struct(params, theta)),
            _ptr(out), _ptr(ws), nb, _stream(stream))
    _check(rc, "wm_loss_grad_exact" if exact else "wm_loss_grad")
    return out


def loss_grad_noalloc(desc: DeviceDescriptors, measured: torch.Tensor, params, out, stream=None):
    """wm_loss_grad_noalloc: the same [loss, count, grad[24]] as loss_grad,
    written into the caller's float64 tensor `out` [26], with the library's
    fixed per-GPU scratch as workspace (nothing is allocated)."""
    rc = lib().wm_loss_grad_noalloc(C.byref(desc.struct()), _ptr(measured), C.byref(params_struct(params)),
                                    _ptr(out), _stream(stream))
    _check(rc, "wm_loss_grad_noalloc")
    return out


def select_tile(shapes: DeviceShapes, params, out=None, stream=None):
    """(best local index int32, best float64 cost, near-tie uint8) per shape."""
    dev = shapes.device
    if out is None:
        out = (torch.empty(shapes.n, dtype=torch.int32, device=dev),
               torch.empty(shapes.n, dtype=torch.float64, device=dev),
               torch.empty(shapes.n, dtype=torch.uint8, device=dev))
    best, cost, tie = out
    s = WmShapes(shapes.M.data_ptr(), shapes.N.data_ptr(), shapes.K.data_ptr(),
                 shapes.dtype.data_ptr(), shapes.n)
    rc = lib().wm_select_tile(C.byref(s), _ptr(shapes.cand_off), _ptr(shapes.cand_code),
                              int(shapes.cand_code.numel()), C.byref(params_struct(params)),
                              _ptr(best), _ptr(cost), _ptr(tie), _stream(stream))
    _check(rc, "wm_select_tile")
    return best, cost, tie


def tile_costs(shapes: DeviceShapes, params, out=None, stream=None):
    """Every candidate's float32 cost (float32 [n_cand], +inf if infeasible)."""
    nc = int(shapes.cand_code.numel())
    if out is None:
        out = torch.empty(nc, dtype=torch.float32, device=shapes.device)
    s = WmShapes(shapes.M.data_ptr(), shapes.N.data_ptr(), shapes.K.data_ptr(),
                 shapes.dtype.data_ptr(), shapes.n)
    rc = lib().wm_tile_costs(C.byref(s), _ptr(shapes.cand_off), _ptr(shapes.cand_code), nc,
                             C.byref(params_struct(params)), _ptr(out), _stream(stream))
    _check(rc, "wm_tile_costs")
    return out


def apps_workspace_bytes(n: int, n_apps: int) -> int:
    return int(lib().wm_apps_workspace_bytes(n, n_apps))


def _check_rows(desc: DeviceDescriptors, segs: DeviceSegments):
    if desc.n != segs.n:
        raise ValueError(f"{desc.n} descriptor rows but {segs.n} segment rows")


def predict_apps(desc: DeviceDescriptors, segs: DeviceSegments, params, segp, want_seg=False,
                 out=None, stream=None):
    """Application times (float32 [n_apps]) and, if want_seg, segment times."""
    _check_rows(desc, segs)
    T_app = out if out is not None else torch.empty(segs.n_apps, dtype=torch.float32, device=desc.device)
    T_seg = torch.empty(segs.n, dtype=torch.float32, device=desc.device) if want_seg else None
    rc = lib().wm_predict_apps(C.byref(desc.struct()), C.byref(segs.struct()),
                               C.byref(params_struct(params)), C.byref(segparams_struct(segp)),
                               _ptr(T_app), _ptr(T_seg), _stream(stream))
    _check(rc, "wm_predict_apps")
    return T_app, T_seg


def apps_loss_grad(desc: DeviceDescriptors, segs: DeviceSegments, measured: torch.Tensor, params,
                   segp, ws=None, out=None, stream=None):
    """[loss, count, grad theta[24], grad (kappa[4], bw_h2d, bw_d2h, tau_memcpy)]
    float64 on the device (application mean relative error)."""
    _check_rows(desc, segs)
    if out is None:
        out = torch.empty(2 + N_THETA + N_SEGPARAMS, dtype=torch.float64, device=desc.device)
    if ws is None:
        ws = _workspace(apps_workspace_bytes(desc.n, segs.n_apps), desc.device)
    nb = 0 if ws is None else ws.numel()
    rc = lib().wm_apps_loss_grad(C.byref(desc.struct()), C.byref(segs.struct()), _ptr(measured),
                                 C.byref(params_struct(params)), C.byref(segparams_struct(segp)),
                                 _ptr(out), _ptr(ws), nb, _stream(stream))
    _check(rc, "wm_apps_loss_grad")
    return out


def fit_multipliers(T: torch.Tensor, measured: torch.Tensor, group_off: torch.Tensor,
                    train: torch.Tensor, ws=None, stream=None):
    """Per-group weighted-median multipliers on the training rows.  Returns
    (mult float64 [n_groups], T_scaled float32 [n], stats float64 [4]: training
    error sum, training rows, held-out error sum, held-out rows) on the device."""
    dev = T.device
    n = int(T.numel())
    ng = int(group_off.numel()) - 1
    if measured.numel() != n or train.numel() != n or ng < 0:
        raise ValueError("T, measured and train must have one entry per row; group_off n_groups + 1")
    mult = torch.empty(max(ng, 1), dtype=torch.float64, device=dev)
    Ts = torch.empty(max(n, 1), dtype=torch.float32, device=dev)
    stats = torch.empty(4, dtype=torch.float64, device=dev)
    if ws is None:
        ws = _workspace(workspace_bytes(OP_FIT_MULTIPLIERS, n), dev)
    rc = lib().wm_fit_multipliers(_ptr(T), _ptr(measured), _ptr(group_off), ng, n, _ptr(train), _ptr(mult),
                                  _ptr(Ts), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "wm_fit_multipliers")
    return mult[:ng], Ts[:n], stats


def plan_workspace_bytes(n: int, R: int) -> int:
    return int(lib().wm_plan_workspace_bytes(n, R))


def plan_redone(ws: torch.Tensor) -> int:
    """Diagnostic: the number of chains the last plan_fusion call with this
    workspace redid in float64 (the uint32 that starts the workspace's last
    256 bytes)."""
    return int(ws[-256:-252].cpu().numpy().view(np.uint32)[0])


def plan_fusion(desc: DeviceDescriptors, edge: torch.Tensor, chain_off: torch.Tensor, params, R: int = 8,
                ws=None, stream=None):
    """Optimal fusion plans: (total float64 [n_chains], unfused float64
    [n_chains], start uint8 [n]) on the device."""
    dev = desc.device
    nc = int(chain_off.numel()) - 1
    if edge.numel() != desc.n:
        raise ValueError("edge needs one entry per descriptor row")
    total = torch.empty(max(nc, 1), dtype=torch.float64, device=dev)
    unf = torch.empty(max(nc, 1), dtype=torch.float64, device=dev)
    start = torch.empty(max(desc.n, 1), dtype=torch.uint8, device=dev)
    if ws is None:
        ws = _workspace(plan_workspace_bytes(desc.n, R), dev)
    rc = lib().wm_plan_fusion(C.byref(desc.struct()), _ptr(edge), _ptr(chain_off), nc, int(R),
                              C.byref(params_struct(params)), _ptr(total), _ptr(unf), _ptr(start), _ptr(ws),
                              0 if ws is None else ws.numel(), _stream(stream))
    _check(rc, "wm_plan_fusion")
    return total[:nc], unf[:nc], start[:desc.n]


# ---------------------------------------------------------------------------
# Blackwell stage-centric family
# ---------------------------------------------------------------------------
def bw_params_struct(p, theta: Optional[Sequence[float]] = None) -> WmBwParams:
    """Marshal a Blackwell parameter set (n_sm, max_cta, tmem_bytes, f_clk, theta)."""
    o = WmBwParams()
    o.n_sm, o.max_cta, o.tmem_bytes, o.f_clk = int(p.n_sm), int(p.max_cta), int(p.tmem_bytes), float(p.f_clk)
    th = p.theta if theta is None else theta
    for j in range(N_THETA):
        o.theta[j] = float(th[j])
    return o


def bw_validate_params(p) -> bool:
    return lib().wm_bw_validate_params(C.byref(bw_params_struct(p))) == WM_OK


class DeviceBwDescriptors:
    """Blackwell tile-kernel descriptors: 5 int32 + 3 float32 device arrays."""
    INTS = ("bM", "bN", "bK", "G", "flags")
    FLOATS = ("Kt", "CR", "ob")

    def __init__(self, tensors: dict):
        n = None
        for f in self.INTS + self.FLOATS:
            t = tensors[f]
            want = torch.int32 if f in self.INTS else torch.float32
            if t.dtype != want or not t.is_contiguous() or t.dim() != 1:
                raise ValueError(f"descriptor field {f} must be a contiguous 1-D {want} tensor")
            n = t.shape[0] if n is None else n
            if t.shape[0] != n:
                raise ValueError("descriptor fields differ in length")
            setattr(self, f, t)
        self.n = int(n)
        self.device = tensors["bM"].device

    @classmethod
    def from_host(cls, d, device="cuda") -> "DeviceBwDescriptors":
        return cls({f: torch.from_numpy(np.ascontiguousarray(getattr(d, f))).to(device)
                    for f in cls.INTS + cls.FLOATS})

    def struct(self) -> WmBwDesc:
        o = WmBwDesc()
        for f in self.INTS + self.FLOATS:
            setattr(o, f, getattr(self, f).data_ptr())
        o.n = self.n
        return o


def bw_workspace_bytes(op: int, n: int, steps: int = 0) -> int:
    return int(lib().wm_bw_workspace_bytes(op, n, steps))


def bw_predict(desc: DeviceBwDescriptors, params, out_T=None, want_cta=True, stream=None):
    T = out_T if out_T is not None else torch.empty(desc.n, dtype=torch.float32, device=desc.device)
    cta = torch.empty(desc.n, dtype=torch.int32, device=desc.device) if want_cta else None
    _check(lib().wm_bw_predict(C.byref(desc.struct()), C.byref(bw_params_struct(params)), _ptr(T), _ptr(cta),
                               _stream(stream)), "wm_bw_predict")
    return T, cta


def bw_vjp(desc: DeviceBwDescriptors, params, dL_dT: torch.Tensor, ws=None, stream=None):
    out = torch.empty(N_THETA, dtype=torch.float64, device=desc.device)
    if ws is None:
        ws = _workspace(bw_workspace_bytes(BW_OP_GRAD, desc.n), desc.device)
    _check(lib().wm_bw_predict_vjp(C.byref(desc.struct()), C.byref(bw_params_struct(params)),
                                   _ptr(dL_dT.contiguous()), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)),
           "wm_bw_predict_vjp")
    return out


def bw_loss_grad(desc: DeviceBwDescriptors, measured: torch.Tensor, params, ws=None, out=None, stream=None):
    if out is None:
        out = torch.empty(26, dtype=torch.float64, device=desc.device)
    if ws is None:
        ws = _workspace(bw_workspace_bytes(BW_OP_GRAD, desc.n), desc.device)
    _check(lib().wm_bw_loss_grad(C.byref(desc.struct()), _ptr(measured), C.byref(bw_params_struct(params)),
                                 _ptr(out), _ptr(ws), ws.numel(), _stream(stream)), "wm_bw_loss_grad")
    return out


def bw_calibrate(desc: DeviceBwDescriptors, measured: torch.Tensor, p0, steps=500, lr=0.05, lr_final=1e-3,
                 beta1=0.9, beta2=0.999, eps=1e-8, free_mask=0xFFFFFF, ws=None, stream=None, lo=None, hi=None):
    """Device Adam on log(theta) for the Blackwell model.  Returns (status,
    theta float64 [24], loss history)."""
    opts = calib_opts(steps, lr, lr_final, beta1, beta2, eps, free_mask, lo=lo, hi=hi)
    if ws is None:
        ws = _workspace(bw_workspace_bytes(BW_OP_CALIBRATE, desc.n, steps), desc.device)
    pout = WmBwParams()
    hist = np.zeros(steps)
    rc = lib().wm_bw_calibrate(C.byref(desc.struct()), _ptr(measured), C.byref(bw_params_struct(p0)),
                               C.byref(opts), C.byref(pout), hist.ctypes.data, _ptr(ws), ws.numel(),
                               _stream(stream))
    if rc not in (WM_OK, WM_EDIVERGED):
        raise WmError(rc, "wm_bw_calibrate")
    return rc, np.array([pout.theta[j] for j in range(N_THETA)]), hist


def apps_vjp(desc: DeviceDescriptors, segs: DeviceSegments, dL_dTapp: torch.Tensor, params, segp,
             ws=None, stream=None, theta=None):
    """dL/d(theta[24], kappa[4], bw_h2d, bw_d2h, tau_memcpy) float64 [31] on the
    device for an upstream gradient of the application times."""
    _check_rows(desc, segs)
    out = torch.empty(N_THETA + N_SEGPARAMS, dtype=torch.float64, device=desc.device)
    if ws is None:
        ws = _workspace(apps_workspace_bytes(desc.n, segs.n_apps), desc.device)
    rc = lib().wm_predict_apps_vjp(C.byref(desc.struct()), C.byref(segs.struct()), _ptr(dL_dTapp.contiguous()),
                                   C.byref(params_struct(params, theta)), C.byref(segparams_struct(segp)),
                                   _ptr(out), _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream))
    _check(rc, "wm_predict_apps_vjp")
    return out


class _SegVec:
    """Segment parameters from a 7-vector (kappa[4], bw_h2d, bw_d2h, tau)."""

    def __init__(self, v):
        self.kappa = [float(x) for x in v[:4]]
        self.bw_h2d, self.bw_d2h, self.tau_memcpy = float(v[4]), float(v[5]), float(v[6])


class WMPredictApps(torch.autograd.Function):
    """T_app = WMPredictApps.apply(desc, segs, theta, segvec, params): theta
    float64 [24] and segvec float64 [7] (kappa[4], bw_h2d, bw_d2h,
    tau_memcpy); T_app float32 [n_apps].  backward returns the gradients of
    both from the application adjoint (wm_predict_apps_vjp)."""

    @staticmethod
    def forward(ctx, desc, segs, theta, segvec, params):
        th = theta.detach().to("cpu", torch.float64).numpy()
        sv = _SegVec(segvec.detach().to("cpu", torch.float64).numpy())
        ctx.desc, ctx.segs, ctx.params, ctx.th, ctx.sv = desc, segs, params, th, sv
        ctx.dev_t, ctx.dev_s = theta.device, segvec.device
        T = torch.empty(segs.n_apps, dtype=torch.float32, device=desc.device)
        rc = lib().wm_predict_apps(C.byref(desc.struct()), C.byref(segs.struct()),
                                   C.byref(params_struct(params, th)), C.byref(segparams_struct(sv)),
                                   _ptr(T), None, _stream())
        _check(rc, "wm_predict_apps")
        return T

    @staticmethod
    def backward(ctx, dL_dT):
        g = apps_vjp(ctx.desc, ctx.segs, dL_dT.to(torch.float32).contiguous(), ctx.params, ctx.sv, theta=ctx.th)
        return None, None, g[:N_THETA].to(ctx.dev_t), g[N_THETA:].to(ctx.dev_s), None


def calib_opts(steps=500, lr=0.05, lr_final=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
               free_mask=0xFFFFFF, lo=None, hi=None, order=0) -> WmCalibOpts:
    """Calibration options; lo / hi: per-slot boxes (24 values, 0 = none),
    order: ORDER_BW | ORDER_LAT level orderings."""
    o = WmCalibOpts(steps=steps, order=order, lr=lr, lr_final=lr_final, beta1=beta1, beta2=beta2, eps=eps,
                    free_mask=free_mask)
    for j in range(N_THETA):
        o.lo[j] = 0.0 if lo is None else float(lo[j])
        o.hi[j] = 0.0 if hi is None else float(hi[j])
    return o


def calibrate(desc: DeviceDescriptors, measured: torch.Tensor, p0, steps=500, lr=0.05,
              lr_final=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, free_mask=0xFFFFFF, ws=None,
              stream=None, raise_on_diverged=False, lo=None, hi=None, order=0):
    """Device Adam on log(theta), optionally projected onto per-slot boxes
    and level orderings.  Returns (status, theta float64 [24], loss history)."""
    opts = calib_opts(steps, lr, lr_final, beta1, beta2, eps, free_mask, lo=lo, hi=hi, order=order)
    if ws is None:
        ws = _workspace(workspace_bytes(OP_CALIBRATE, desc.n, 1, steps), desc.device)
    pout = WmParams()
    hist = np.zeros(steps)
    rc = lib().wm_calibrate(C.byref(desc.struct()), _ptr(measured), C.byref(params_struct(p0)),
                            C.byref(opts), C.byref(pout), hist.ctypes.data, _ptr(ws), ws.numel(),
                            _stream(stream))
    if rc not in (WM_OK, WM_EDIVERGED) or (raise_on_diverged and rc != WM_OK):
        raise WmError(rc, "wm_calibrate")
    return rc, theta_of(pout), hist


def calibrate_resume(desc: DeviceDescriptors, measured: torch.Tensor, p0, steps, run_steps, state=None,
                     lr=0.05, lr_final=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, free_mask=0xFFFFFF, ws=None,
                     stream=None, lo=None, hi=None, order=0):
    """Run `run_steps` steps of a `steps`-step calibration from `state` (a
    WmCalibState; None = fresh start from p0).  Returns (status, theta, loss
    history of these steps, state after them)."""
    opts = calib_opts(steps, lr, lr_final, beta1, beta2, eps, free_mask, lo=lo, hi=hi, order=order)
    if ws is None:
        ws = _workspace(workspace_bytes(OP_CALIBRATE, desc.n, 1, steps), desc.device)
    pout = WmParams()
    hist = np.zeros(run_steps)
    out = WmCalibState()
    rc = lib().wm_calibrate_resume(C.byref(desc.struct()), _ptr(measured), C.byref(params_struct(p0)),
                                   C.byref(opts), None if state is None else C.byref(state), int(run_steps),
                                   C.byref(out), C.byref(pout), hist.ctypes.data, _ptr(ws), ws.numel(),
                                   _stream(stream))
    if rc not in (WM_OK, WM_EDIVERGED):
        raise WmError(rc, "wm_calibrate_resume")
    return rc, theta_of(pout), hist, out


def save_calib_state(path, state: WmCalibState):
    """Write a calibration state to an .npz file (exact doubles, no pickling)."""
    np.savez(path, **{f: np.array(getattr(state, f)) for f in ("theta", "theta_ok", "phi", "m", "v")},
             step=np.int32(state.step), diverged=np.int32(state.diverged))


def load_calib_state(path) -> WmCalibState:
    z = np.load(path, allow_pickle=False)
    st = WmCalibState()
    for f in ("theta", "theta_ok", "phi", "m", "v"):
        getattr(st, f)[:] = [float(x) for x in z[f]]
    st.step, st.diverged = int(z["step"]), int(z["diverged"])
    return st


def calibrate_batched(descs: List[DeviceDescriptors], measured: List[torch.Tensor], p0s, opts_list,
                      ws=None, stream=None):
    """Several calibration problems in one persistent sweep per step.
    Returns (status, thetas [n_sets, 24], loss history [n_sets, steps])."""
    k = len(descs)
    steps = int(opts_list[0].steps)
    D = (WmDesc * k)(*[d.struct() for d in descs])
    M = (C.c_void_p * k)(*[m.data_ptr() for m in measured])
    P0 = (WmParams * k)(*[params_struct(p) for p in p0s])
    O = (WmCalibOpts * k)(*opts_list)
    POUT = (WmParams * k)()
    n_total = sum(d.n for d in descs)
    if ws is None:
        ws = _workspace(workspace_bytes(OP_CALIBRATE_BATCHED, n_total, k, steps), descs[0].device)
    hist = np.zeros((k, steps))
    rc = lib().wm_calibrate_batched(k, D, M, P0, O, POUT, hist.ctypes.data, _ptr(ws), ws.numel(),
                                    _stream(stream))
    if rc not in (WM_OK, WM_EDIVERGED):
        raise WmError(rc, "wm_calibrate_batched")
    return rc, np.stack([theta_of(POUT[i]) for i in range(k)]), hist


# ---------------------------------------------------------------------------
# launch configurations and autotuning
# ---------------------------------------------------------------------------
def get_launch(op: int, n: int) -> dict:
    c = WmLaunch()
    _check(lib().wm_get_launch(op, n, C.byref(c)), "wm_get_launch")
    return c.as_dict()


def set_launch(op: int, n: int, block=256, per_thread=1, grid_mult=1, chunk=0):
    c = WmLaunch(block, per_thread, grid_mult, chunk)
    _check(lib().wm_set_launch(op, n, C.byref(c)), "wm_set_launch")


def _tuned(rc, what, best, us):
    _check(rc, what)
    return {**best.as_dict(), "us": us.value}


def autotune_predict(desc: DeviceDescriptors, params, stream=None) -> dict:
    T = torch.empty(desc.n, dtype=torch.float32, device=desc.device)
    occ = torch.empty(desc.n, dtype=torch.int32, device=desc.device)
    best, us = WmLaunch(), C.c_double()
    rc = lib().wm_autotune_predict(C.byref(desc.struct()), C.byref(params_struct(params)), _ptr(T),
                                   _ptr(occ), _stream(stream), C.byref(best), C.byref(us))
    return _tuned(rc, "wm_autotune_predict", best, us)


def autotune_grad(op: int, desc: DeviceDescriptors, w: torch.Tensor, params, stream=None) -> dict:
    out = torch.empty(26, dtype=torch.float64, device=desc.device)
    ws = _workspace(workspace_bytes(op, desc.n), desc.device)
    best, us = WmLaunch(), C.c_double()
    rc = lib().wm_autotune_grad(op, C.byref(desc.struct()), _ptr(w), C.byref(params_struct(params)),
                                _ptr(out), _ptr(ws), ws.numel(), _stream(stream), C.byref(best),
                                C.byref(us))
    return _tuned(rc, "wm_autotune_grad", best, us)


def autotune_select_tile(shapes: DeviceShapes, params, stream=None) -> dict:
    dev = shapes.device
    best_i = torch.empty(shapes.n, dtype=torch.int32, device=dev)
    cost = torch.empty(shapes.n, dtype=torch.float64, device=dev)
    tie = torch.empty(shapes.n, dtype=torch.uint8, device=dev)
    s = WmShapes(shapes.M.data_ptr(), shapes.N.data_ptr(), shapes.K.data_ptr(),
                 shapes.dtype.data_ptr(), shapes.n)
    best, us = WmLaunch(), C.c_double()
    rc = lib().wm_autotune_select_tile(C.byref(s), _ptr(shapes.cand_off), _ptr(shapes.cand_code),
                                       int(shapes.cand_code.numel()), C.byref(params_struct(params)),
                                       _ptr(best_i), _ptr(cost), _ptr(tie), _stream(stream),
                                       C.byref(best), C.byref(us))
    return _tuned(rc, "wm_autotune_select_tile", best, us)


def autotune_apps(op: int, desc: DeviceDescriptors, segs: DeviceSegments, measured, params, segp,
                  stream=None) -> dict:
    """Tune the application sweep of predict_apps (op OP_PREDICT_APPS) or
    apps_loss_grad (OP_APPS_LOSS_GRAD, needs measured)."""
    _check_rows(desc, segs)
    best, us = WmLaunch(), C.c_double()
    dev = desc.device
    T = ws = out = None
    if op == OP_PREDICT_APPS:
        T = torch.empty(max(segs.n_apps, 1), dtype=torch.float32, device=dev)
    else:
        out = torch.empty(2 + N_THETA + N_SEGPARAMS, dtype=torch.float64, device=dev)
        ws = _workspace(apps_workspace_bytes(desc.n, segs.n_apps), dev)
    rc = lib().wm_autotune_apps(op, C.byref(desc.struct()), C.byref(segs.struct()), _ptr(measured),
                                C.byref(params_struct(params)), C.byref(segparams_struct(segp)),
                                _ptr(T), _ptr(out), _ptr(ws), 0 if ws is None else ws.numel(),
                                _stream(stream), C.byref(best), C.byref(us))
    return _tuned(rc, "wm_autotune_apps", best, us)


def autotune_batched(descs, measured, p0s, opts_list, stream=None) -> dict:
    k = len(descs)
    steps = int(opts_list[0].steps)
    D = (WmDesc * k)(*[d.struct() for d in descs])
    M = (C.c_void_p * k)(*[m.data_ptr() for m in measured])
    P0 = (WmParams * k)(*[params_struct(p) for p in p0s])
    O = (WmCalibOpts * k)(*opts_list)
    n_total = sum(d.n for d in descs)
    ws = _workspace(workspace_bytes(OP_CALIBRATE_BATCHED, n_total, k, steps), descs[0].device)
    best, us = WmLaunch(), C.c_double()
    rc = lib().wm_autotune_batched(k, D, M, P0, O, _ptr(ws), ws.numel(), _stream(stream),
                                   C.byref(best), C.byref(us))
    return _tuned(rc, "wm_autotune_batched", best, us)


# ---------------------------------------------------------------------------
# autograd: T = model(descriptors; theta), dL/dtheta by the adjoint kernel
# ---------------------------------------------------------------------------
class WMPredict(torch.autograd.Function):
    """T = WMPredict.apply(desc, theta, params): theta is a float64 [24] tensor
    (CPU or device); T is float32 [n] on the descriptors' device.  backward
    returns dL/dtheta as float64 on theta's device, computed by the adjoint
    kernel with FP64 reductions."""

    @staticmethod
    def forward(ctx, desc: DeviceDescriptors, theta: torch.Tensor, params):
        th = theta.detach().to("cpu", torch.float64).numpy()
        ctx.desc, ctx.params, ctx.theta_np, ctx.theta_dev = desc, params, th, theta.device
        T = torch.empty(desc.n, dtype=torch.float32, device=desc.device)
        ds = desc.struct()
        ps = params_struct(params, th)
        _check(lib().wm_predict(C.byref(ds), C.byref(ps), _ptr(T), None, _stream()), "wm_predict")
        return T

    @staticmethod
    def backward(ctx, dL_dT):
        g = vjp(ctx.desc, ctx.params, dL_dT.to(torch.float32).contiguous(), theta=ctx.theta_np)
        return None, g.to(ctx.theta_dev), None
