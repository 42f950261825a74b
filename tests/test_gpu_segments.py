"""Parity of the workload-segment calls (wm_predict_apps, wm_apps_loss_grad)
with the FP64 oracle: application and segment times element by element,
the application-level loss, count and gradient, the float64 sign pass near
T = m, ragged and degenerate application lists, and every launch
configuration."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import check_grad, need_gpu, rel_err, say

pytestmark = pytest.mark.gpu
TTOL = 1e-5
GTOL = 1e-4


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def _dev(wmb, sg, d):
    return wmb.DeviceDescriptors.from_host(d), wmb.DeviceSegments.from_host(sg)


def _check_times(wmb, orc, p, q, sg, d, tag):
    dd, ds = _dev(wmb, sg, d)
    Ta, Ts = wmb.predict_apps(dd, ds, p, q, want_seg=True)
    torch.cuda.synchronize()
    Ra, Rs = orc.predict_apps(p, q, d, sg)
    ea = rel_err(Ta.cpu().numpy(), Ra)
    es = rel_err(Ts.cpu().numpy(), Rs)
    say(tag, "apps", sg.n_apps, "rows", d.F.shape[0], "max rel", ea.max() if ea.size else 0.0,
        es.max() if es.size else 0.0)
    assert ea.size == 0 or ea.max() <= TTOL
    assert es.size == 0 or es.max() <= TTOL
    return Ta, Ra


@pytest.mark.parametrize("L,combine", [(4, 0), (3, 0), (4, 1)])
def test_predict_apps_parity(wmb, orc, L, combine):
    p = synth.param_set(3, n_levels=L, combine=combine)
    q = synth.seg_params(11)
    sg, d = synth.segments(30001, 140)
    _check_times(wmb, orc, p, q, sg, d, f"L{L} c{combine}")


def test_predict_apps_ragged_and_degenerate(wmb, orc):
    p = synth.param_set(0)
    q = synth.seg_params(12)
    sg, d = synth.segments(700, 141)
    n = d.F.shape[0]
    # application lengths: empty ones, one row, one application over several
    # LDS pieces (3000 rows), and a tail that is not a multiple of the block
    lens = [0, 1, 0, 0, 3000, 5, 0, 1] + [2] * 37
    rest = n - sum(lens)
    assert rest > 0
    lens += [rest] + [0, 0, 0]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    sg2 = dataclasses.replace(sg, app_off=off)
    # invalid rows and an infeasible kernel inside long applications
    sg2.cls[4 + 10] = 7
    sg2.n_kern[4 + 2000] = 0
    d.vgpr[off[9]] = 4096
    d.gpack[off[9]] = int(synth.pack_gpack(1024, 1, 1, 1, 0, 0))
    Ta, Ra = _check_times(wmb, orc, p, q, sg2, d, "ragged")
    Ta = Ta.cpu().numpy()
    assert Ta[0] == 0.0 and Ta[2] == 0.0 and Ta[-1] == 0.0
    assert np.isnan(Ta[4]) and np.isinf(Ta[9])
    # one application holding every row; only empty applications
    one = dataclasses.replace(sg, app_off=np.array([0, n], np.int32))
    _check_times(wmb, orc, p, q, one, d, "single")
    d0 = synth.descriptors(0, 1)
    s0 = synth.Segments(np.zeros(4, np.int32), *[np.zeros(0, t) for t in
                        (np.float32, np.int32, np.int32, np.float32, np.float32)])
    Ta, _ = _check_times(wmb, orc, p, q, s0, d0, "empty")
    assert np.array_equal(Ta.cpu().numpy(), np.zeros(3, np.float32))


def _grad_check(wmb, orc, p, q, sg, d, m, tag):
    dd, ds = _dev(wmb, sg, d)
    mt = torch.from_numpy(m.astype(np.float32)).cuda()
    out = wmb.apps_loss_grad(dd, ds, mt, p, q).cpu().numpy()
    loss, cnt, gth, gsp = orc.apps_loss_grad(p, q, d, sg, m.astype(np.float32).astype(np.float64))
    say(tag, "count", int(out[1]), cnt, "loss", out[0], loss)
    assert int(out[1]) == cnt
    assert abs(out[0] - loss) <= 1e-5 * loss
    _check_both(out[2:26], out[26:], gth, gsp, p, q, tag)
    return out


def _seg_x(q):
    return np.array(list(q.kappa) + [q.bw_h2d, q.bw_d2h, q.tau_memcpy])


def _check_both(g_th, g_sp, gth, gsp, p, q, tag):
    """theta and the segment parameters share one log-space scale (both are
    fitted together), then each group is also checked slot by slot."""
    names = list(synth.THETA_NAMES) + ["kappa0", "kappa1", "kappa2", "kappa3", "bw_h2d", "bw_d2h", "tau_memcpy"]
    check_grad(np.concatenate([g_th, g_sp]), np.concatenate([gth, gsp]),
               np.concatenate([np.asarray(p.theta), _seg_x(q)]), tag, GTOL, names=names)


@pytest.mark.parametrize("L,combine", [(4, 0), (3, 0), (4, 1)])
def test_apps_loss_grad_parity(wmb, orc, L, combine):
    p_true = synth.param_set(4, n_levels=L, combine=combine)
    q_true = synth.seg_params(13)
    sg, d = synth.segments(20000, 142)
    Ta, _ = orc.predict_apps(p_true, q_true, d, sg)
    m = Ta * synth.lognormal_noise(sg.n_apps, 143, 0.05)
    p0 = synth.perturb_theta(p_true, 144, factor=1.3)
    q0 = synth.seg_params(14)
    _grad_check(wmb, orc, p0, q0, sg, d, m, f"L{L} c{combine}")


def test_apps_loss_grad_sign_pass_near_optimum(wmb, orc):
    """At the true parameters with noise-free measurements for half the
    applications, |T/m - 1| is of the order of float32 rounding: the sign
    is taken from the float64 pass."""
    p = synth.param_set(5)
    q = synth.seg_params(15)
    sg, d = synth.segments(20000, 145)
    Ta, _ = orc.predict_apps(p, q, d, sg)
    noise = synth.lognormal_noise(sg.n_apps, 146, 0.03)
    noise[::2] = 1.0
    _grad_check(wmb, orc, p, q, sg, d, Ta * noise, "near optimum")


def test_apps_loss_grad_bad_measurements_and_empty(wmb, orc):
    p = synth.param_set(6)
    q = synth.seg_params(16)
    sg, d = synth.segments(3000, 147)
    Ta, _ = orc.predict_apps(p, q, d, sg)
    m = Ta * 1.07
    m[:6] = [0.0, -1.0, np.nan, np.inf, m[4], m[5]]
    out = _grad_check(wmb, orc, p, q, sg, d, m, "bad measurements")
    assert int(out[1]) == sg.n_apps - 4
    # no applications at all: zeros
    d0 = synth.descriptors(0, 1)
    s0 = synth.Segments(np.zeros(1, np.int32), *[np.zeros(0, t) for t in
                        (np.float32, np.int32, np.int32, np.float32, np.float32)])
    dd, ds = _dev(wmb, s0, d0)
    out = wmb.apps_loss_grad(dd, ds, torch.zeros(0, dtype=torch.float32, device="cuda"), p, q)
    assert np.array_equal(out.cpu().numpy(), np.zeros(33))


def test_apps_every_config(wmb, orc):
    p = synth.param_set(7)
    q = synth.seg_params(17)
    sg, d = synth.segments(50001, 148)
    Ta, _ = orc.predict_apps(p, q, d, sg)
    mt = torch.from_numpy((Ta * synth.lognormal_noise(sg.n_apps, 149, 0.05)).astype(np.float32)).cuda()
    dd, ds = _dev(wmb, sg, d)
    refT = wmb.predict_apps(dd, ds, p, q)[0].clone()
    refG = wmb.apps_loss_grad(dd, ds, mt, p, q).cpu().numpy()
    for block in (64, 128, 256, 512):
        for gm in (1, 2, 4):
            wmb.set_launch(wmb.OP_PREDICT_APPS, sg.n_apps, block, 1, gm)
            wmb.set_launch(wmb.OP_APPS_LOSS_GRAD, sg.n_apps, block, 1, gm)
            T = wmb.predict_apps(dd, ds, p, q)[0]
            assert torch.equal(torch.nan_to_num(T, nan=-1.0), torch.nan_to_num(refT, nan=-1.0)), (block, gm)
            g = wmb.apps_loss_grad(dd, ds, mt, p, q).cpu().numpy()
            assert g[1] == refG[1]
            # other launch shapes split the rows differently over lanes, which
            # keep float32 partial sums before the float64 reductions
            assert np.max(np.abs(g - refG) / np.maximum(np.abs(refG), 1e-300)) <= 1e-6, (block, gm)
    for op, m in ((wmb.OP_PREDICT_APPS, None), (wmb.OP_APPS_LOSS_GRAD, mt)):
        best = wmb.autotune_apps(op, dd, ds, m, p, q)
        say("tuned", op, best)
        assert best["block"] in (64, 128, 256, 512) and 1 <= best["grid_mult"] <= 4
        assert wmb.get_launch(op, sg.n_apps)["block"] == best["block"]
    T = wmb.predict_apps(dd, ds, p, q)[0]
    assert torch.equal(torch.nan_to_num(T, nan=-1.0), torch.nan_to_num(refT, nan=-1.0))
    g = wmb.apps_loss_grad(dd, ds, mt, p, q).cpu().numpy()
    assert np.max(np.abs(g - refG) / np.maximum(np.abs(refG), 1e-300)) <= 1e-6
    wmb.set_launch(wmb.OP_PREDICT_APPS, sg.n_apps, 256, 1, 1)
    wmb.set_launch(wmb.OP_APPS_LOSS_GRAD, sg.n_apps, 256, 1, 1)


def test_apps_full_size(wmb, orc):
    """2^20 applications (about 6.8 million rows), checked in full."""
    p = synth.param_set(0)
    q = synth.seg_params(7)
    sg, d = synth.segments(1 << 20, 150)
    Ta, Ra = _check_times(wmb, orc, p, q, sg, d, "full size")
    m = Ra * synth.lognormal_noise(sg.n_apps, 151, 0.05)
    p0 = synth.perturb_theta(p, 152, factor=1.2)
    _grad_check(wmb, orc, p0, q, sg, d, m, "full size")


def test_apps_vjp_and_autograd(wmb, orc):
    p = synth.param_set(8)
    q = synth.seg_params(18)
    sg, d = synth.segments(40000, 153)
    dd, ds = _dev(wmb, sg, d)
    w = np.random.default_rng(9).standard_normal(sg.n_apps).astype(np.float32)
    g = wmb.apps_vjp(dd, ds, torch.from_numpy(w).cuda(), p, q).cpu().numpy()
    gth, gsp = orc.apps_vjp(p, q, d, sg, w.astype(np.float64))
    _check_both(g[:24], g[24:], gth, gsp, p, q, "apps vjp")
    # through autograd: L = sum(w * T_app) over finite applications
    theta = torch.tensor(p.theta, dtype=torch.float64, requires_grad=True)
    sv = torch.tensor(list(q.kappa) + [q.bw_h2d, q.bw_d2h, q.tau_memcpy], dtype=torch.float64,
                      requires_grad=True)
    T = wmb.WMPredictApps.apply(dd, ds, theta, sv, p)
    wt = torch.from_numpy(w).cuda()
    fin = torch.isfinite(T)
    (wt[fin] * T[fin]).double().sum().backward()
    _check_both(theta.grad.numpy(), sv.grad.numpy(), gth, gsp, p, q, "apps autograd")
    # no applications: zeros
    d0 = synth.descriptors(0, 1)
    s0 = synth.Segments(np.zeros(1, np.int32), *[np.zeros(0, t) for t in
                        (np.float32, np.int32, np.int32, np.float32, np.float32)])
    z = wmb.apps_vjp(*_dev(wmb, s0, d0), torch.zeros(0, device="cuda"), p, q)
    assert np.array_equal(z.cpu().numpy(), np.zeros(31))
