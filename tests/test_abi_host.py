"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and validates arguments before any HIP call (these calls
return before touching a device, so they run without a GPU)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2605_04178_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wavemodel.h")


@pytest.fixture(scope="module")
def wmb():
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_calls():
    names = _declared()
    for n in ("wm_predict", "wm_roofline", "wm_predict_vjp", "wm_loss_grad", "wm_select_tile",
              "wm_calibrate", "wm_calibrate_batched", "wm_workspace_bytes", "wm_strerror",
              "wm_last_hip_error", "wm_validate_params", "wm_predict_apps", "wm_apps_loss_grad",
              "wm_apps_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol(wmb):
    lib = wmb.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", wmb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(wm_\w+)", out))
    assert set(_declared()) <= exported
    assert set(wmb.EXPORTED) <= exported


def test_library_is_gfx950_only(wmb):
    out = subprocess.run(["/opt/rocm/llvm/bin/clang-offload-bundler", "--list", "--type=o",
                          "--input=" + wmb.LIB_PATH], capture_output=True, text=True)
    if out.returncode == 0 and out.stdout.strip():
        targets = [t for t in out.stdout.split() if "amdgcn" in t]
        assert targets and all("gfx950" in t for t in targets)


def test_struct_sizes_match_header(wmb):
    # 14 int32 + 3 double + 24 double
    assert C.sizeof(wmb.WmParams) == 14 * 4 + 3 * 8 + 24 * 8
    assert C.sizeof(wmb.WmDesc) == 12 * 8 + 8
    assert C.sizeof(wmb.WmCalibOpts) == 4 + 4 + 5 * 8 + 4 + 4 + 2 * 24 * 8


def test_strerror(wmb):
    L = wmb.lib()
    assert L.wm_strerror(0) == b"ok"
    for s in (-1, -2, -3, -4, 7):
        assert isinstance(L.wm_strerror(s), bytes) and L.wm_strerror(s)


def _bad_params():
    base = synth.param_set(0)
    bad = [dict(n_levels=2), dict(n_cu=0), dict(wave=48), dict(vgpr_gran=3), dict(lds_gran=0),
           dict(waves_simd=0), dict(combine=2), dict(f_clk=0.0), dict(w_lo_mib=300.0),
           dict(w_lo_mib=205.1), dict(mwp=-1), dict(bytes_inflight_wave=0), dict(lds_cu=-1)]
    out = [base.copy(**kw) for kw in bad]
    for j, v in ((0, 0.0), (3, -1.0), (8, 0.0), (12, float("inf")), (13, -1e-6), (20, 0.0),
                 (23, 0.0), (5, float("nan")), (4, -1.0)):
        th = list(base.theta)
        th[j] = v
        out.append(base.copy(theta=th))
    return out


def test_validate_params(wmb):
    assert wmb.validate_params(synth.param_set(0))
    assert wmb.validate_params(synth.param_set(0, n_levels=3))
    assert wmb.validate_params(synth.mi300a_like())
    for p in synth.multi_arch_sets():
        assert wmb.validate_params(p)
    for p in _bad_params():
        assert not wmb.validate_params(p), p
    # alpha/beta/LLC slots are unused with three levels
    th = list(synth.param_set(0).theta)
    th[2], th[6], th[20], th[21] = 0.0, 0.0, 0.0, 0.0
    assert wmb.validate_params(synth.param_set(0, n_levels=3).copy(theta=th))
    # w0 <= 0 switches the blend off and is allowed
    th = list(synth.param_set(0).theta)
    th[22] = 0.0
    assert wmb.validate_params(synth.param_set(0).copy(theta=th))


def test_workspace_bytes(wmb):
    assert wmb.workspace_bytes(wmb.OP_PREDICT, 1 << 20) == 0
    assert wmb.workspace_bytes(wmb.OP_SELECT_TILE, 1 << 20) == 0
    a = wmb.workspace_bytes(wmb.OP_LOSS_GRAD, 1 << 20)
    assert a > 0 and a % 256 == 0
    assert wmb.workspace_bytes(wmb.OP_VJP, 0) > 0
    assert wmb.workspace_bytes(wmb.OP_CALIBRATE, 1 << 20, 1, 0) == 0
    assert wmb.workspace_bytes(wmb.OP_CALIBRATE, 1 << 20, 1, 500) > a
    assert wmb.workspace_bytes(wmb.OP_CALIBRATE_BATCHED, 1 << 20, 17, 10) == 0
    assert wmb.workspace_bytes(wmb.OP_CALIBRATE_BATCHED, 1 << 20, 6, 10) > 0
    assert wmb.workspace_bytes(wmb.OP_LOSS_GRAD, -1) == 0


def _fake_desc(wmb, n):
    d = wmb.WmDesc()
    for i, f in enumerate(wmb.DeviceDescriptors.FLOATS + wmb.DeviceDescriptors.INTS):
        setattr(d, f, 0x1000 * (i + 1))
    d.n = n
    return d


def test_argument_errors_before_any_hip_call(wmb):
    """Every call below is rejected by host validation; none reaches HIP."""
    L = wmb.lib()
    p = wmb.params_struct(synth.param_set(0))
    bad = wmb.params_struct(synth.param_set(0).copy(n_levels=5))
    d = _fake_desc(wmb, 16)
    neg = _fake_desc(wmb, -1)
    T = C.c_void_p(0x2000)
    assert L.wm_predict(None, C.byref(p), T, None, None) == wmb.WM_EINVAL
    assert L.wm_predict(C.byref(d), None, T, None, None) == wmb.WM_EINVAL
    assert L.wm_predict(C.byref(d), C.byref(bad), T, None, None) == wmb.WM_EINVAL
    assert L.wm_predict(C.byref(neg), C.byref(p), T, None, None) == wmb.WM_EINVAL
    assert L.wm_predict(C.byref(d), C.byref(p), None, None, None) == wmb.WM_EINVAL
    d0 = _fake_desc(wmb, 0)
    assert L.wm_predict(C.byref(d0), C.byref(p), None, None, None) == wmb.WM_OK
    dnull = _fake_desc(wmb, 16)
    dnull.gpack = None
    assert L.wm_predict(C.byref(dnull), C.byref(p), T, None, None) == wmb.WM_EINVAL
    assert L.wm_roofline(C.byref(d), C.byref(bad), T, None) == wmb.WM_EINVAL
    # gradient calls: missing workspace / too small / misaligned
    out = C.c_void_p(0x3000)
    w = C.c_void_p(0x4000)
    assert L.wm_loss_grad(C.byref(d), w, C.byref(p), out, None, 0, None) == wmb.WM_EWORKSPACE
    assert L.wm_loss_grad(C.byref(d), w, C.byref(p), out, C.c_void_p(0x10000), 8, None) == wmb.WM_EWORKSPACE
    need = wmb.workspace_bytes(wmb.OP_LOSS_GRAD, 16)
    assert L.wm_loss_grad(C.byref(d), w, C.byref(p), out, C.c_void_p(0x10008), need, None) == wmb.WM_EWORKSPACE
    assert L.wm_loss_grad(C.byref(d), None, C.byref(p), out, C.c_void_p(0x10000), need, None) == wmb.WM_EINVAL
    assert L.wm_predict_vjp(C.byref(d), C.byref(p), w, None, C.c_void_p(0x10000), need, None) == wmb.WM_EINVAL
    assert L.wm_loss_grad_exact(C.byref(d), w, C.byref(p), out, C.c_void_p(0x10000), 8, None) == wmb.WM_EWORKSPACE
    assert L.wm_loss_grad_exact(C.byref(d), None, C.byref(p), out, C.c_void_p(0x10000), need, None) == wmb.WM_EINVAL
    assert L.wm_predict_vjp_exact(C.byref(d), C.byref(p), w, None, C.c_void_p(0x10000), need, None) == wmb.WM_EINVAL
    # tile selection
    sh = wmb.WmShapes(0x100, 0x200, 0x300, 0x400, 4)
    assert L.wm_select_tile(C.byref(sh), None, None, 0, C.byref(p), out, out, out, None) == wmb.WM_EINVAL
    assert L.wm_select_tile(C.byref(sh), C.c_void_p(0x500), None, 10, C.byref(p), out, out, out, None) == wmb.WM_EINVAL
    sh0 = wmb.WmShapes(None, None, None, None, 0)
    assert L.wm_select_tile(C.byref(sh0), None, None, 0, C.byref(p), None, None, None, None) == wmb.WM_OK
    shn = wmb.WmShapes(0x100, 0x200, 0x300, 0x400, -2)
    assert L.wm_select_tile(C.byref(shn), C.c_void_p(0x500), None, 0, C.byref(p), out, out, out, None) == wmb.WM_EINVAL
    # calibration options
    pout = wmb.WmParams()
    for kw in (dict(steps=0), dict(lr=0.0), dict(lr=float("nan")), dict(beta1=1.0), dict(eps=0.0),
               dict(free_mask=1 << 24), dict(lr_final=-1.0)):
        o = wmb.calib_opts(**{**dict(steps=5), **kw})
        rc = L.wm_calibrate(C.byref(d), w, C.byref(p), C.byref(o), C.byref(pout), None,
                            C.c_void_p(0x10000), 1 << 30, None)
        assert rc == wmb.WM_EINVAL, kw
    o = wmb.calib_opts(steps=5)
    assert L.wm_calibrate(C.byref(d), w, C.byref(p), C.byref(o), C.byref(pout), None, None, 0,
                          None) == wmb.WM_EWORKSPACE
    # constraints: valid boxes and orderings pass validation (then the
    # missing workspace is reported); each malformed one is rejected
    th0 = np.array(synth.param_set(0).theta)
    lo_ok, hi_ok = np.where(th0 > 0, th0 / 2, 0.0), np.where(th0 > 0, th0 * 2, 0.0)
    ok = dict(steps=5, lo=lo_ok, hi=hi_ok, order=3, free_mask=synth.FIT_MASK_L4)
    o = wmb.calib_opts(**ok)
    assert L.wm_calibrate(C.byref(d), w, C.byref(p), C.byref(o), C.byref(pout), None, None, 0,
                          None) == wmb.WM_EWORKSPACE

    def with_(j, lo=None, hi=None):
        a, b = lo_ok.copy(), hi_ok.copy()
        if lo is not None:
            a[j] = lo
        if hi is not None:
            b[j] = hi
        return dict(ok, lo=a, hi=b)
    bad = [with_(3, lo=hi_ok[3] * 1.5),                  # lo > hi
           with_(13, lo=-1.0), with_(13, hi=float("nan")), with_(14, hi=float("inf")),
           dict(ok, order=4),                            # unknown ordering bit
           dict(ok, free_mask=synth.FIT_MASK_L4 & ~(1 << 2)),           # ordered group not all free
           dict(ok, order=2, free_mask=synth.FIT_MASK_L4 & ~(1 << 7)),
           with_(1, hi=hi_ok[0] * 1.5),                  # bandwidth boxes not non-increasing
           with_(5, lo=lo_ok[6] * 1.5)]                  # latency boxes not non-decreasing
    for kw in bad:
        o = wmb.calib_opts(**kw)
        rc = L.wm_calibrate(C.byref(d), w, C.byref(p), C.byref(o), C.byref(pout), None,
                            C.c_void_p(0x10000), 1 << 30, None)
        assert rc == wmb.WM_EINVAL, kw
    # a free slot must be positive (log-space update)
    th = list(synth.param_set(0).theta)
    th[13] = 0.0
    pz = wmb.params_struct(synth.param_set(0).copy(theta=th))
    assert L.wm_calibrate(C.byref(d), w, C.byref(pz), C.byref(o), C.byref(pout), None,
                          C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    # batched: set count, mismatched steps
    D = (wmb.WmDesc * 2)(d, d)
    M = (C.c_void_p * 2)(0x4000, 0x5000)
    P0 = (wmb.WmParams * 2)(p, p)
    O = (wmb.WmCalibOpts * 2)(wmb.calib_opts(steps=5), wmb.calib_opts(steps=6))
    PO = (wmb.WmParams * 2)()
    assert L.wm_calibrate_batched(2, D, M, P0, O, PO, None, C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    assert L.wm_calibrate_batched(0, D, M, P0, O, PO, None, C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    assert L.wm_calibrate_batched(17, D, M, P0, O, PO, None, C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    # measurements may be NULL only for an empty set
    o = wmb.calib_opts(steps=5)
    assert L.wm_calibrate(C.byref(d), None, C.byref(p), C.byref(o), C.byref(pout), None,
                          C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    O2 = (wmb.WmCalibOpts * 2)(o, o)
    M0 = (C.c_void_p * 2)(0x4000, None)
    assert L.wm_calibrate_batched(2, D, M0, P0, O2, PO, None, C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    assert L.wm_last_hip_error() == 0


def _fake_segs(wmb, n_apps):
    s = wmb.WmSegs()
    for i, f in enumerate(("app_off", "n_exec", "n_kern", "cls", "h2d", "d2h")):
        setattr(s, f, 0x20000 * (i + 1))
    s.n_apps = n_apps
    return s


def test_segment_calls_validate_before_any_hip_call(wmb):
    L = wmb.lib()
    p = wmb.params_struct(synth.param_set(0))
    q = wmb.segparams_struct(synth.SegParams())
    d = _fake_desc(wmb, 16)
    sg = _fake_segs(wmb, 4)
    T = C.c_void_p(0x2000)
    out = C.c_void_p(0x3000)
    m = C.c_void_p(0x4000)
    assert C.sizeof(wmb.WmSegs) == 6 * 8 + 8 and C.sizeof(wmb.WmSegParams) == 7 * 8
    assert L.wm_predict_apps(C.byref(d), None, C.byref(p), C.byref(q), T, None, None) == wmb.WM_EINVAL
    assert L.wm_predict_apps(C.byref(d), C.byref(sg), C.byref(p), None, T, None, None) == wmb.WM_EINVAL
    assert L.wm_predict_apps(C.byref(d), C.byref(sg), C.byref(p), C.byref(q), None, None, None) == wmb.WM_EINVAL
    for kw in (dict(kappa=[1, 1, -1, 1]), dict(kappa=[1, float("nan"), 1, 1]), dict(bw_h2d=0.0),
               dict(bw_d2h=-5.0), dict(tau_memcpy=-1e-6), dict(bw_h2d=float("inf"))):
        bad = wmb.segparams_struct(synth.SegParams(**kw))
        assert L.wm_predict_apps(C.byref(d), C.byref(sg), C.byref(p), C.byref(bad), T, None, None) == wmb.WM_EINVAL, kw
    # rows without applications, a missing row field, negative count
    assert L.wm_predict_apps(C.byref(d), C.byref(_fake_segs(wmb, 0)), C.byref(p), C.byref(q), T, None,
                             None) == wmb.WM_EINVAL
    s2 = _fake_segs(wmb, 4)
    s2.cls = None
    assert L.wm_predict_apps(C.byref(d), C.byref(s2), C.byref(p), C.byref(q), T, None, None) == wmb.WM_EINVAL
    assert L.wm_predict_apps(C.byref(d), C.byref(_fake_segs(wmb, -1)), C.byref(p), C.byref(q), T, None,
                             None) == wmb.WM_EINVAL
    # nothing to do
    d0 = _fake_desc(wmb, 0)
    assert L.wm_predict_apps(C.byref(d0), C.byref(_fake_segs(wmb, 0)), C.byref(p), C.byref(q), None, None,
                             None) == wmb.WM_OK
    # loss gradient: workspace and measured
    need = wmb.apps_workspace_bytes(16, 4)
    assert need > 0 and need % 256 == 0
    assert wmb.apps_workspace_bytes(16, 1 << 20) > need and wmb.apps_workspace_bytes(-1, 4) == 0
    assert L.wm_apps_loss_grad(C.byref(d), C.byref(sg), m, C.byref(p), C.byref(q), out, None, 0,
                               None) == wmb.WM_EWORKSPACE
    assert L.wm_apps_loss_grad(C.byref(d), C.byref(sg), m, C.byref(p), C.byref(q), out,
                               C.c_void_p(0x10000), need - 256, None) == wmb.WM_EWORKSPACE
    assert L.wm_apps_loss_grad(C.byref(d), C.byref(sg), None, C.byref(p), C.byref(q), out,
                               C.c_void_p(0x10000), need, None) == wmb.WM_EINVAL
    assert L.wm_apps_loss_grad(C.byref(d), C.byref(sg), m, C.byref(p), C.byref(q), None,
                               C.c_void_p(0x10000), need, None) == wmb.WM_EINVAL
    assert L.wm_last_hip_error() == 0


def test_planning_calls_validate_before_any_hip_call(wmb):
    L = wmb.lib()
    p = wmb.params_struct(synth.param_set(0))
    d = _fake_desc(wmb, 16)
    x = C.c_void_p(0x7000)
    ws = C.c_void_p(0x10000)
    need = wmb.workspace_bytes(wmb.OP_FIT_MULTIPLIERS, 16)
    assert need > 0 and need % 256 == 0 and wmb.workspace_bytes(wmb.OP_FIT_MULTIPLIERS, 1 << 30) == need
    assert L.wm_fit_multipliers(x, x, x, 2, -1, x, x, x, x, ws, need, None) == wmb.WM_EINVAL
    assert L.wm_fit_multipliers(x, x, x, -1, 16, x, x, x, x, ws, need, None) == wmb.WM_EINVAL
    assert L.wm_fit_multipliers(None, x, x, 2, 16, x, x, x, x, ws, need, None) == wmb.WM_EINVAL
    assert L.wm_fit_multipliers(x, x, None, 2, 16, x, x, x, x, ws, need, None) == wmb.WM_EINVAL
    assert L.wm_fit_multipliers(x, x, x, 2, 16, x, x, x, None, ws, need, None) == wmb.WM_EINVAL
    assert L.wm_fit_multipliers(x, x, x, 2, 16, x, x, x, x, ws, need - 1, None) == wmb.WM_EWORKSPACE
    assert wmb.plan_workspace_bytes(16, 0) == 0 and wmb.plan_workspace_bytes(16, 33) == 0
    pw = wmb.plan_workspace_bytes(16, 8)
    assert pw > 0 and wmb.plan_workspace_bytes(1 << 20, 8) > pw
    for R in (0, 33):
        assert L.wm_plan_fusion(C.byref(d), x, x, 2, R, C.byref(p), x, x, x, ws, 1 << 30, None) == wmb.WM_EINVAL
    assert L.wm_plan_fusion(C.byref(d), x, x, 0, 8, C.byref(p), None, None, None, None, 0, None) == wmb.WM_OK
    assert L.wm_plan_fusion(C.byref(d), None, x, 2, 8, C.byref(p), x, x, x, ws, 1 << 30, None) == wmb.WM_EINVAL
    assert L.wm_plan_fusion(C.byref(d), x, x, 2, 8, C.byref(p), x, x, x, ws, pw - 1, None) == wmb.WM_EWORKSPACE
    assert L.wm_last_hip_error() == 0


def test_blackwell_calls_validate_before_any_hip_call(wmb):
    L = wmb.lib()
    assert C.sizeof(wmb.WmBwParams) == 4 + 4 + 8 + 8 + 24 * 8 and C.sizeof(wmb.WmBwDesc) == 8 * 8 + 8
    p = synth.b200_like()
    assert wmb.bw_validate_params(p)
    for s in range(5):
        assert wmb.bw_validate_params(synth.bw_param_set(s))
    for kw in (dict(n_sm=0), dict(max_cta=0), dict(tmem_bytes=0), dict(f_clk=0.0)):
        assert not wmb.bw_validate_params(p.copy(**kw)), kw
    for j, v in ((0, 0.0), (5, -1.0), (8, 0.0), (14, 0.0), (17, -0.1), (22, -1e-6), (9, float("nan"))):
        th = list(p.theta)
        th[j] = v
        assert not wmb.bw_validate_params(p.copy(theta=th)), (j, v)
    ps = wmb.bw_params_struct(p)
    d = wmb.WmBwDesc()
    for i, f in enumerate(wmb.DeviceBwDescriptors.INTS + wmb.DeviceBwDescriptors.FLOATS):
        setattr(d, f, 0x1000 * (i + 1))
    d.n = 16
    x = C.c_void_p(0x9000)
    assert L.wm_bw_predict(C.byref(d), C.byref(ps), None, None, None) == wmb.WM_EINVAL
    d0 = wmb.WmBwDesc()
    assert L.wm_bw_predict(C.byref(d0), C.byref(ps), None, None, None) == wmb.WM_OK
    need = wmb.bw_workspace_bytes(wmb.BW_OP_GRAD, 16)
    assert need > 0 and wmb.bw_workspace_bytes(wmb.BW_OP_CALIBRATE, 16, 0) == 0
    assert wmb.bw_workspace_bytes(wmb.BW_OP_CALIBRATE, 16, 10) > need
    assert L.wm_bw_loss_grad(C.byref(d), x, C.byref(ps), x, None, 0, None) == wmb.WM_EWORKSPACE
    assert L.wm_bw_loss_grad(C.byref(d), None, C.byref(ps), x, C.c_void_p(0x10000), need, None) == wmb.WM_EINVAL
    o = wmb.calib_opts(steps=5, free_mask=1 << 17)
    th = list(p.theta)
    th[17] = 0.0
    assert L.wm_bw_calibrate(C.byref(d), x, C.byref(wmb.bw_params_struct(p.copy(theta=th))), C.byref(o),
                             C.byref(wmb.WmBwParams()), None, C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    # measurements may be NULL only when there are no descriptors
    o = wmb.calib_opts(steps=5, free_mask=1 << 0)
    assert L.wm_bw_calibrate(C.byref(d), None, C.byref(ps), C.byref(o), C.byref(wmb.WmBwParams()), None,
                             C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    # boxes apply to the Blackwell slots too; the level orderings name CDNA slots
    lo = np.array([t / 2 if t > 0 else 0.0 for t in p.theta])
    o = wmb.calib_opts(steps=5, free_mask=0xF, lo=lo)
    assert L.wm_bw_calibrate(C.byref(d), x, C.byref(ps), C.byref(o), C.byref(wmb.WmBwParams()), None,
                             None, 0, None) == wmb.WM_EWORKSPACE
    o = wmb.calib_opts(steps=5, free_mask=0xFF, order=wmb.ORDER_BW)
    assert L.wm_bw_calibrate(C.byref(d), x, C.byref(ps), C.byref(o), C.byref(wmb.WmBwParams()), None,
                             C.c_void_p(0x10000), 1 << 30, None) == wmb.WM_EINVAL
    assert L.wm_last_hip_error() == 0


def test_product_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2605_04178_amd import wavemodel
    monkeypatch.setattr(wavemodel, "_lib", None)
    monkeypatch.setattr(wavemodel, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        wavemodel.lib()


def test_product_package_does_not_reference_oracle():
    pkg = os.path.join(ROOT, "paper_2605_04178_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"(import|from)\s+oracle|liboracle|wm_oracle", src), f


def test_set_launch_rejects_invalid_configs_without_a_gpu(wmb):
    L = wmb.lib()
    bad = [(wmb.OP_PREDICT, (96, 4, 1, 0)), (wmb.OP_PREDICT, (256, 3, 1, 0)),
           (wmb.OP_LOSS_GRAD, (256, 1, 0, 0)), (wmb.OP_LOSS_GRAD, (256, 1, 9, 0)),
           (wmb.OP_SELECT_TILE, (1024, 1, 1, 0)), (wmb.OP_CALIBRATE_BATCHED, (128, 1, 1, 16384)),
           (wmb.OP_CALIBRATE_BATCHED, (256, 1, 1, 3000)), (wmb.OP_CALIBRATE_BATCHED, (256, 1, 1, 128)), (wmb.OP_CALIBRATE_BATCHED, (256, 1, 1, 1 << 17)),
           (wmb.OP_ROOFLINE, (256, 1, 1, 0)), (99, (256, 1, 1, 0))]
    for op, cfg in bad:
        c = wmb.WmLaunch(*cfg)
        assert L.wm_set_launch(op, 1000, C.byref(c)) == wmb.WM_EINVAL, (op, cfg)
    assert L.wm_set_launch(wmb.OP_PREDICT, -1, C.byref(wmb.WmLaunch(256, 4, 1, 0))) == wmb.WM_EINVAL
    assert L.wm_set_launch(wmb.OP_PREDICT, 10, None) == wmb.WM_EINVAL
    assert L.wm_get_launch(wmb.OP_PREDICT, 10, None) == wmb.WM_EINVAL
    assert L.wm_get_launch(99, 10, C.byref(wmb.WmLaunch())) == wmb.WM_EINVAL
    # tuners validate their arguments first
    p = wmb.params_struct(synth.param_set(0))
    assert L.wm_autotune_predict(None, C.byref(p), None, None, None, None, None) == wmb.WM_EINVAL
    assert L.wm_autotune_grad(wmb.OP_PREDICT, None, None, C.byref(p), None, None, 0, None, None,
                              None) == wmb.WM_EINVAL


def test_noalloc_loss_grad_rejects_bad_arguments_and_sizes_before_any_hip_call(wmb):
    """wm_loss_grad_noalloc checks every argument and the size limit on the
    host; none of these calls reaches HIP (there is no GPU here)."""
    L = wmb.lib()
    p = wmb.params_struct(synth.param_set(0))
    out, w = C.c_void_p(0x20000), C.c_void_p(0x30000)
    d = _fake_desc(wmb, wmb.NOALLOC_MAX_N + 1)
    assert L.wm_loss_grad_noalloc(C.byref(d), w, C.byref(p), out, None) == wmb.WM_ETOOLARGE
    d.n = 1 << 40
    assert L.wm_loss_grad_noalloc(C.byref(d), w, C.byref(p), out, None) == wmb.WM_ETOOLARGE
    d.n = -1
    assert L.wm_loss_grad_noalloc(C.byref(d), w, C.byref(p), out, None) == wmb.WM_EINVAL
    d.n = 16
    assert L.wm_loss_grad_noalloc(C.byref(d), None, C.byref(p), out, None) == wmb.WM_EINVAL
    assert L.wm_loss_grad_noalloc(C.byref(d), w, C.byref(p), None, None) == wmb.WM_EINVAL
    assert L.wm_loss_grad_noalloc(None, w, C.byref(p), out, None) == wmb.WM_EINVAL
    bad = wmb.params_struct(synth.param_set(0).copy(n_levels=5))
    assert L.wm_loss_grad_noalloc(C.byref(d), w, C.byref(bad), out, None) == wmb.WM_EINVAL
    # the fixed scratch covers the workspace of the largest accepted input
    assert L.wm_noalloc_scratch_bytes() >= wmb.workspace_bytes(wmb.OP_LOSS_GRAD, wmb.NOALLOC_MAX_N)
    assert L.wm_noalloc_scratch_bytes() < 16 << 20
    assert L.wm_strerror(wmb.WM_ETOOLARGE).decode() == "input larger than the fixed scratch allows"


def test_calibrate_resume_rejects_bad_states_before_any_hip_call(wmb):
    L = wmb.lib()
    p = wmb.params_struct(synth.param_set(0))
    d = _fake_desc(wmb, 64)
    w = C.c_void_p(0x30000)
    o = wmb.calib_opts(steps=100, free_mask=synth.FIT_MASK_L4)
    pout = wmb.WmParams()
    st = wmb.WmCalibState()
    for j in range(24):
        st.theta[j] = synth.param_set(0).theta[j]
        st.theta_ok[j] = st.theta[j]
    ws = C.c_void_p(0x10000)
    call = lambda state, run: L.wm_calibrate_resume(C.byref(d), w, C.byref(p), C.byref(o), state, run, None,
                                                    C.byref(pout), None, ws, 1 << 40, None)
    assert call(None, 0) == wmb.WM_EINVAL              # no steps
    assert call(None, 101) == wmb.WM_EINVAL            # past the schedule
    st.step = 90
    assert call(C.byref(st), 11) == wmb.WM_EINVAL      # 90 + 11 > 100
    st.step = -1
    assert call(C.byref(st), 1) == wmb.WM_EINVAL
    st.step = 10
    st.diverged = 1
    assert call(C.byref(st), 1) == wmb.WM_EINVAL       # a diverged state
    st.diverged = 0
    st.theta[0] = float("nan")
    assert call(C.byref(st), 1) == wmb.WM_EINVAL       # parameters that are not a valid set
    st.theta[0] = synth.param_set(0).theta[0]
    st.theta[13] = 0.0
    assert call(C.byref(st), 1) == wmb.WM_EINVAL       # a fitted slot must stay positive
    # a valid state with a workspace that is too small stops at the workspace check
    st.theta[13] = synth.param_set(0).theta[13]
    assert L.wm_calibrate_resume(C.byref(d), w, C.byref(p), C.byref(o), C.byref(st), 5, None, C.byref(pout),
                                 None, ws, 8, None) == wmb.WM_EWORKSPACE
