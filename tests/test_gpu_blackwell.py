"""Parity of the Blackwell stage-centric family on the GPU with the FP64
oracle: forward times (float32, 1e-5) and CTA residency (exact), the
adjoint and loss gradient (1e-4), descriptors near the compute / I-O switch
and near T = m (float64 pass), ragged sizes, and calibration recovery."""
import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import check_grad, need_gpu, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bw_forward_parity(wmb, orc, seed):
    p = synth.bw_param_set(seed)
    d = synth.bw_descriptors(200003, 210 + seed)
    say("bw forward", seed)
    T, cta = wmb.bw_predict(wmb.DeviceBwDescriptors.from_host(d), p)
    To, co = orc.bw_predict(p, d)
    assert np.array_equal(cta.cpu().numpy(), co)
    e = rel_err(T.cpu().numpy(), To)
    say("  max rel err", e.max())
    assert e.max() <= 1e-5


def test_bw_forward_edge_cases(wmb, orc):
    p = synth.b200_like().copy(max_cta=2)
    d = synth.bw_descriptors(64, 219)
    F = synth.pack_bw_flags
    d.bM[0], d.bN[0], d.flags[0] = 256, 256, F(0, 0, 0, 1, 1, 1, 0)     # FP64 accumulators overflow TMEM
    d.bM[1] = 0                                                         # invalid tile
    d.flags[2] = int(d.flags[2]) | (1 << 20)                            # reserved bit
    d.Kt[3] = 0.5
    d.CR[4] = 0.5
    d.ob[5] = 0.0
    d.flags[6] = F(5, 0, 0, 1, 1, 1, 0)
    d.G[7] = 296                                                        # exactly two rounds of 148 x 1
    for n in (1, 3, 63, 64):
        T, cta = wmb.bw_predict(wmb.DeviceBwDescriptors.from_host(d.slice(0, n)), p)
        To, co = orc.bw_predict(p, d.slice(0, n))
        assert np.array_equal(cta.cpu().numpy(), co)
        assert rel_err(T.cpu().numpy(), To).max() <= 1e-5
    T, cta = wmb.bw_predict(wmb.DeviceBwDescriptors.from_host(d), p)
    T, cta = T.cpu().numpy(), cta.cpu().numpy()
    assert np.isinf(T[0]) and cta[0] == 0
    assert all(np.isnan(T[i]) and cta[i] == -1 for i in range(1, 7))


def test_bw_tile_extents_at_the_int32_limit(wmb, orc):
    """Tile extents up to 2^31 - 1: accumulators that cannot fit in TMEM are
    infeasible (+inf, 0 CTAs) on both sides, for FP64 and narrower types,
    including products of the extents beyond 2^63; the largest tiles that
    still fit stay finite and match."""
    p = synth.b200_like().copy(max_cta=2)
    d = synth.bw_descriptors(12, 232)
    big = 2 ** 31 - 1
    F = synth.pack_bw_flags
    rows = [(big, big, 0), (big, big, 2), (big, 1, 2), (1, big, 0), (65536, 65536, 2), (1 << 20, 1 << 20, 3),
            (2 ** 30, 1, 2), (256, 256, 2), (256, 256, 0), (256, 128, 0), (1, 65536, 2), (1, 32768, 0)]
    for i, (bm, bn, dt) in enumerate(rows):
        d.bM[i], d.bN[i] = bm, bn
        d.flags[i] = F(dt, 0, 0, 1, 1, 1, 0)
        d.bK[i] = 16
    T, cta = wmb.bw_predict(wmb.DeviceBwDescriptors.from_host(d), p)
    To, co = orc.bw_predict(p, d)
    cta, T = cta.cpu().numpy(), T.cpu().numpy()
    say("int32-limit tiles: CTAs", cta, "oracle", co)
    assert np.array_equal(cta, co)
    fits = np.array([0, 0, 0, 0, 0, 0, 0, 1, 0, 1, 1, 1], bool)   # 256 x 256 x 8 B = 2 x TMEM does not
    assert np.all(cta[~fits] == 0) and np.all(np.isinf(T[~fits]))
    assert np.all(cta[fits] >= 1) and np.all(np.isfinite(T[fits]))
    assert rel_err(T, To).max() <= 1e-5


@pytest.mark.parametrize("seed", [3, 4])
def test_bw_vjp_and_loss_grad_parity(wmb, orc, seed):
    p = synth.bw_param_set(seed)
    d = synth.bw_descriptors(1 << 17, 220 + seed)
    dd = wmb.DeviceBwDescriptors.from_host(d)
    w = np.random.default_rng(seed).standard_normal(d.n).astype(np.float32)
    g = wmb.bw_vjp(dd, p, torch.from_numpy(w).cuda()).cpu().numpy()
    go = orc.bw_vjp(p, d, w)
    check_grad(g, go, p.theta, f"bw vjp seed {seed}", 1e-4, names=synth.BW_THETA_NAMES)
    To, _ = orc.bw_predict(p, d)
    p0 = synth.bw_param_set(seed + 10)
    m = (To * synth.lognormal_noise(d.n, seed, 0.05)).astype(np.float32)
    out = wmb.bw_loss_grad(dd, torch.from_numpy(m).cuda(), p0).cpu().numpy()
    loss, cnt, gl = orc.bw_loss_grad(p0, d, m)
    say("bw loss", out[0], loss, "count", out[1], cnt)
    assert int(out[1]) == cnt and abs(out[0] - loss) <= 1e-5 * loss
    check_grad(out[2:], gl, p0.theta, f"bw loss gradient seed {seed}", 1e-4, names=synth.BW_THETA_NAMES)


def test_bw_loss_grad_near_optimum_and_switch(wmb, orc):
    """Noise-free measurements put |T/m - 1| at float32 rounding for every
    descriptor; an exposed fraction tuned so that many descriptors sit at the
    compute / I-O switch exercises the other float64 decision."""
    p = synth.bw_param_set(5)
    d = synth.bw_descriptors(1 << 16, 225)
    dd = wmb.DeviceBwDescriptors.from_host(d)
    To, _ = orc.bw_predict(p, d)
    m = To.astype(np.float32)
    out = wmb.bw_loss_grad(dd, torch.from_numpy(m).cuda(), p).cpu().numpy()
    loss, cnt, gl = orc.bw_loss_grad(p, d, m)
    assert int(out[1]) == cnt and abs(out[0] - loss) <= 1e-5 * max(loss, 1e-12) + 1e-9
    check_grad(out[2:], gl, p.theta, "bw loss gradient with m = T", 1e-4, names=synth.BW_THETA_NAMES)
    # put descriptors at the switch: scale eps so that T_io equals T_compute for one tile shape
    tr = orc.bw_trace(p, d)
    fin = np.isfinite(tr["T"])
    i = int(np.flatnonzero(fin & (tr["T_io"] > tr["T_sync"] * 1.5))[0])
    raw = tr["T_tma"][i] + tr["T_decomp"][i] + tr["T_dsm"][i]
    th = list(p.theta)
    th[17] = float((tr["T_compute"][i] - tr["T_sync"][i]) / raw)
    p2 = p.copy(theta=th)
    same = np.flatnonzero((d.bM == d.bM[i]) & (d.bN == d.bN[i]) & (d.bK == d.bK[i]) & (d.flags == d.flags[i])
                          & (d.CR == d.CR[i]))
    say("descriptors at the switch", len(same))
    w = np.ones(d.n, np.float32)
    g = wmb.bw_vjp(dd, p2, torch.from_numpy(w).cuda()).cpu().numpy()
    check_grad(g, orc.bw_vjp(p2, d, w), p2.theta, "bw vjp at the switch", 1e-4, names=synth.BW_THETA_NAMES)


def test_bw_calibration_recovers_parameters(wmb, orc):
    """2^18 measurements over the Blackwell calibration sweep, sigma = 0.02,
    500 Adam steps from a +-30 % start: all 20 fitted slots (every slot but
    the four the oracle tests show unidentifiable: eta_DE, the exposed
    fraction, O_misc and the TMEM read rate) within 3 %."""
    p_true = synth.bw_param_set(7)
    d = synth.bw_calibration_descriptors(1 << 18, 226)
    To, _ = orc.bw_predict(p_true, d)
    m = (To * synth.lognormal_noise(d.n, 227, 0.02)).astype(np.float32)
    mask = synth.BW_FIT_MASK
    free = [j for j in range(24) if mask >> j & 1]
    assert len(free) == 20
    rng = np.random.default_rng(3)
    th0 = list(p_true.theta)
    for j in free:
        th0[j] *= float(np.exp(rng.uniform(-np.log(1.3), np.log(1.3))))
    p0 = p_true.copy(theta=th0)
    rc, th, hist = wmb.bw_calibrate(wmb.DeviceBwDescriptors.from_host(d), torch.from_numpy(m).cuda(), p0,
                                    steps=500, lr=0.05, lr_final=1e-3, free_mask=mask)
    err = {synth.BW_THETA_NAMES[j]: abs(th[j] / p_true.theta[j] - 1) for j in free}
    say("bw calibration", rc, "loss", hist[0], "->", hist[-1], "recovery error per fitted slot:",
        " ".join(f"{k}={v * 100:.2f}%" for k, v in err.items()))
    assert rc == 0 and hist[-1] < hist[0] and max(err.values()) < 0.03
    assert all(th[j] == p0.theta[j] for j in range(24) if j not in free)
    # the oracle's calibration from the same start, on a sample, follows the same path
    sub = d.slice(0, 1 << 14)
    rc_o, th_o, hist_o = orc.bw_calibrate(p0, sub, m[: 1 << 14], steps=50, lr=0.05, lr_final=1e-3, free_mask=mask)
    rc_g, th_g, hist_g = wmb.bw_calibrate(wmb.DeviceBwDescriptors.from_host(sub),
                                          torch.from_numpy(m[: 1 << 14]).cuda(), p0, steps=50, lr=0.05,
                                          lr_final=1e-3, free_mask=mask)
    assert np.allclose(hist_g, hist_o, rtol=1e-5)
    assert np.allclose(th_g, th_o, rtol=1e-4)
