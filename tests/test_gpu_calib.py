"""Device calibration (wm_calibrate, wm_calibrate_batched): Adam on log(theta)
in captured HIP graphs.  Recovery of the ground-truth parameters, gradient
parity with the FP64 oracle along the trajectory, divergence handling, and
batched-vs-plain agreement."""
import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import check_grad, loss_grad_absum, need_gpu, say

pytestmark = pytest.mark.gpu

# every used slot; with an LLC all but w0 (its identifiability pin is in the
# oracle tests)
MASK_L4 = synth.FIT_MASK_L4
MASK_L3 = synth.FIT_MASK_L3
# Runs that split the same descriptors differently over lanes (batched against
# per-set sweeps, other work-item sizes) agree to the float32 rounding of the
# lanes' partial sums (~1e-7 relative in the loss), not to the float64 order.
PARTITION_RTOL = 1e-6


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def _problem(orc, n, L=4, sigma=0.02, seed_d=103, seed_p=1, mask=MASK_L4, combine=0):
    """Config 3: measured times from the seed-1 set over the calibration sweep
    (half config-1 draws, half memory-streaming descriptors)."""
    ps = synth.param_set(seed_p, n_levels=L, combine=combine)
    d = synth.calibration_descriptors(n, seed_d)
    T, _ = orc.predict(ps, d)
    m = (T * synth.lognormal_noise(n, 2, sigma)).astype(np.float32)
    p0 = synth.perturb_theta(ps, 3, mask=mask)
    return ps, d, m, p0


def _rec_err(th, ps, mask, tag=None):
    idx = [j for j in range(24) if mask >> j & 1]
    e = np.abs(np.asarray(th)[idx] / np.array(ps.theta)[idx] - 1)
    if tag is not None:
        say(tag, "recovery error per fitted slot:",
            " ".join(f"{synth.THETA_NAMES[j]}={x * 100:.2f}%" for j, x in zip(idx, e)))
    return float(np.max(e))


@pytest.mark.parametrize("L,combine", [(4, 0), (3, 0), (4, 1), (3, 1)])
def test_calibration_recovers_within_3pct(wmb, orc, L, combine):
    """2^20 measured times with lognormal noise sigma = 0.02, 500 Adam steps,
    under both combine modes (Eq. (1)/(14) max of the stages and the Eq. (9)/
    (12) occupancy overlap); every fitted slot within 3 %."""
    n = 1 << 20
    mask = synth.fit_mask(L)
    ps, d, m, p0 = _problem(orc, n, L=L, mask=mask, combine=combine)
    dd = wmb.DeviceDescriptors.from_host(d)
    say("calibrate L", L, "combine", combine)
    rc, th, hist = wmb.calibrate(dd, torch.from_numpy(m).cuda(), p0, steps=500, free_mask=mask)
    assert rc == wmb.WM_OK
    err = _rec_err(th, ps, mask, f"L{L} combine {combine}")
    say("max recovery error", err)
    assert err <= 0.03
    loss0 = orc.loss_grad(p0, d, m)[0]
    assert abs(hist[0] - loss0) <= 1e-5 * loss0
    assert hist[-1] < hist[0]
    # fixed slots did not move
    for j in range(24):
        if not (mask >> j & 1):
            assert th[j] == p0.theta[j]


def test_calibration_noiseless_recovery(wmb, orc):
    n = 1 << 16
    ps, d, m, p0 = _problem(orc, n, sigma=0.0)
    dd = wmb.DeviceDescriptors.from_host(d)
    rc, th, hist = wmb.calibrate(dd, torch.from_numpy(m).cuda(), p0, steps=500, free_mask=MASK_L4)
    assert rc == wmb.WM_OK
    assert _rec_err(th, ps, MASK_L4) <= 1e-3


def test_gradients_along_the_trajectory(wmb, orc):
    """GPU loss gradient vs the oracle's FP64 gradient at theta0 and at three
    points of the GPU's own Adam trajectory, slot by slot: the default call
    (float32 Jacobian rows; a slot that cancels by more than 200x is held to
    8 ulp of its absolute sum) and the float64-exact call (1e-4 relative for
    every slot at 1e-3 of the largest or more, at every point)."""
    n = 1 << 18
    ps, d, m, p0 = _problem(orc, n)
    dd = wmb.DeviceDescriptors.from_host(d)
    mt = torch.from_numpy(m).cuda()
    pts = [p0]
    for steps in (40, 150, 400):
        rc, th, _ = wmb.calibrate(dd, mt, p0, steps=steps, free_mask=MASK_L4)
        pts.append(p0.copy(theta=list(th)))
    for k, p in enumerate(pts):
        out = wmb.loss_grad(dd, mt, p).cpu().numpy()
        loss, cnt, g = orc.loss_grad(p, d, m)
        assert int(out[1]) == cnt
        assert abs(out[0] - loss) <= 1e-5 * loss
        check_grad(out[2:], g, p.theta, f"trajectory point {k}", 1e-4, names=synth.THETA_NAMES,
                   absum=loss_grad_absum(orc, p, d, m))
        ex = wmb.loss_grad(dd, mt, p, exact=True).cpu().numpy()
        assert int(ex[1]) == cnt and abs(ex[0] - loss) <= 1e-12 * loss
        check_grad(ex[2:], g, p.theta, f"trajectory point {k}, exact call", 1e-4, names=synth.THETA_NAMES)


def test_calibration_matches_oracle_adam_loss_history(wmb, orc):
    """Short run: the device Adam follows the oracle's Adam (same loss history
    to 1e-6 relative over 20 steps)."""
    n = 1 << 16
    ps, d, m, p0 = _problem(orc, n, sigma=0.05)
    dd = wmb.DeviceDescriptors.from_host(d)
    rc, th, hist = wmb.calibrate(dd, torch.from_numpy(m).cuda(), p0, steps=20, free_mask=MASK_L4)
    rco, tho, histo = orc.calibrate(p0, d, m, steps=20, lr=0.05, lr_final=1e-3, free_mask=MASK_L4)
    assert rc == 0 and rco == 0
    assert np.allclose(hist, histo, rtol=1e-6, atol=0)
    assert np.allclose(th, tho, rtol=1e-6, atol=0)


def test_constrained_calibration_matches_oracle(wmb, orc):
    """Boxes and level orderings: from a start that violates both orderings,
    with one box binding (BW_L2 capped below its true value) and the others
    around the truth, the device's projected Adam follows the oracle's (loss
    history and theta to 1e-6 relative over 30 steps) and every slot ends
    feasible; a resumed run in two pieces ends on the same theta."""
    n = 1 << 16
    ps, d, m, p0 = _problem(orc, n, sigma=0.05)
    th = np.array(p0.theta)
    th[0], th[1] = 0.6 * ps.theta[0], 1.7 * ps.theta[0]
    th[6], th[7] = 1.8 * ps.theta[7], 0.7 * ps.theta[7]
    p0 = ps.copy(theta=list(th))
    tt = np.array(ps.theta)
    lo = np.where(tt > 0, tt / 3, 0.0) * np.array([(MASK_L4 >> j) & 1 for j in range(24)])
    hi = np.where(tt > 0, tt * 3, 0.0) * np.array([(MASK_L4 >> j) & 1 for j in range(24)])
    hi[1] = 0.8 * tt[1]
    # boxes ordered like the levels (bandwidths non-increasing, latencies
    # non-decreasing), as the orderings require
    lo[0:4], hi[0:4] = np.minimum.accumulate(lo[0:4]), np.minimum.accumulate(hi[0:4])
    lo[4:8], hi[4:8] = np.maximum.accumulate(lo[4:8]), np.maximum.accumulate(hi[4:8])
    kw = dict(steps=30, lr=0.05, lr_final=1e-3, free_mask=MASK_L4, lo=lo, hi=hi, order=3)
    dd = wmb.DeviceDescriptors.from_host(d)
    mt = torch.from_numpy(m).cuda()
    rc, thg, hist = wmb.calibrate(dd, mt, p0, **kw)
    rco, tho, histo = orc.calibrate(p0, d, m, **kw)
    assert rc == 0 and rco == 0
    assert np.allclose(hist, histo, rtol=1e-6, atol=0)
    assert np.allclose(thg, tho, rtol=1e-6, atol=0)
    assert thg[0] >= thg[1] >= thg[2] >= thg[3] and thg[4] <= thg[5] <= thg[6] <= thg[7]
    f = [j for j in range(24) if MASK_L4 >> j & 1]
    assert np.all(thg[f] >= lo[f] * (1 - 1e-12)) and np.all(thg[f] <= hi[f] * (1 + 1e-12))
    assert thg[1] == pytest.approx(hi[1], rel=1e-12)
    _, _, _, st = wmb.calibrate_resume(dd, mt, p0, 30, 11, **{k: v for k, v in kw.items() if k != "steps"})
    _, th2, _, _ = wmb.calibrate_resume(dd, mt, p0, 30, 19, state=st,
                                        **{k: v for k, v in kw.items() if k != "steps"})
    assert np.array_equal(th2, thg)


def test_calibration_divergence_returns_last_finite_theta(wmb, orc):
    n = 1 << 14
    ps, d, m, p0 = _problem(orc, n)
    dd = wmb.DeviceDescriptors.from_host(d)
    rc, th, hist = wmb.calibrate(dd, torch.from_numpy(m).cuda(), p0, steps=5, lr=1e300,
                                 lr_final=0.0, free_mask=MASK_L4)
    assert rc == wmb.WM_EDIVERGED
    assert np.array_equal(th, np.array(p0.theta))
    assert np.isfinite(hist[0]) and np.all(np.isnan(hist[1:]))
    rco, tho, histo = orc.calibrate(p0, d, m, steps=5, lr=1e300, lr_final=0.0, free_mask=MASK_L4)
    assert rco == 1 and np.array_equal(tho, np.array(p0.theta))


def test_calibration_step_counts_around_graph_chunk(wmb, orc):
    """Step counts that are not a multiple of the captured chunk replay a
    remainder graph; the loss history must continue seamlessly."""
    n = 1 << 14
    ps, d, m, p0 = _problem(orc, n)
    dd = wmb.DeviceDescriptors.from_host(d)
    mt = torch.from_numpy(m).cuda()
    _, th_a, h_a = wmb.calibrate(dd, mt, p0, steps=73, free_mask=MASK_L4)
    _, th_b, h_b = wmb.calibrate(dd, mt, p0, steps=73, free_mask=MASK_L4)
    assert np.array_equal(th_a, th_b) and np.array_equal(h_a, h_b)
    _, th_c, h_c = wmb.calibrate(dd, mt, p0, steps=1, free_mask=MASK_L4)
    assert h_c[0] == h_a[0]


def _batched_problem(orc, wmb, scale_down):
    sets = synth.multi_arch_sets()
    sizes = [max(4096, s // scale_down) for s in synth.multi_arch_sizes()]
    descs, hdesc, meas, p0s, masks = [], [], [], [], []
    for k, (pk, nk) in enumerate(zip(sets, sizes)):
        dk = synth.calibration_descriptors(nk, 120 + k)
        Tk, _ = orc.predict(pk, dk)
        mk = (Tk * synth.lognormal_noise(nk, 130 + k, 0.02)).astype(np.float32)
        mask = synth.fit_mask(pk.n_levels)
        hdesc.append(dk)
        descs.append(wmb.DeviceDescriptors.from_host(dk))
        meas.append(torch.from_numpy(mk).cuda())
        p0s.append(synth.perturb_theta(pk, 140 + k, mask=mask))
        masks.append(mask)
    return sets, sizes, descs, hdesc, meas, p0s, masks


def test_batched_matches_plain_per_set(wmb, orc):
    sets, sizes, descs, hdesc, meas, p0s, masks = _batched_problem(orc, wmb, 16)
    steps = 60
    opts = [wmb.calib_opts(steps=steps, free_mask=mk) for mk in masks]
    rc, thb, histb = wmb.calibrate_batched(descs, meas, p0s, opts)
    assert rc == wmb.WM_OK
    for k in range(len(sets)):
        rck, thk, histk = wmb.calibrate(descs[k], meas[k], p0s[k], steps=steps, free_mask=masks[k])
        say("set", k, "n", sizes[k], "L", sets[k].n_levels)
        # the two runs split the descriptors differently over lanes, and each
        # lane sums its descriptors in float32 before the float64 reductions:
        # they agree to float32 rounding of those partial sums
        assert np.allclose(histb[k], histk, rtol=PARTITION_RTOL, atol=0), k
        assert np.allclose(thb[k], thk, rtol=PARTITION_RTOL, atol=0), k
        # first-step loss equals the oracle's at theta0
        l0 = orc.loss_grad(p0s[k], hdesc[k], meas[k].cpu().numpy())[0]
        assert abs(histb[k][0] - l0) <= 1e-5 * l0


def test_batched_recovery_within_3pct(wmb, orc):
    sets, sizes, descs, hdesc, meas, p0s, masks = _batched_problem(orc, wmb, 1)
    say("batched sizes", sizes)
    opts = [wmb.calib_opts(steps=500, free_mask=mk) for mk in masks]
    rc, thb, histb = wmb.calibrate_batched(descs, meas, p0s, opts)
    assert rc == wmb.WM_OK
    for k, pk in enumerate(sets):
        e = _rec_err(thb[k], pk, masks[k], f"set {k} (L{pk.n_levels}, n {sizes[k]})")
        assert e <= 0.03


def test_batched_sixteen_ragged_sets_match_per_set(wmb, orc):
    """The 16-set maximum with ragged sizes: an empty set, sets shorter than
    one wave, sizes on both sides of 64, 256 and the 2048-descriptor default
    item; work items of 256 and of 2048 descriptors.  Every set's loss
    history and theta equal its own plain calibration (FP64 sums in another
    order only)."""
    sizes = [0, 1, 63, 64, 65, 255, 256, 257, 1000, 2047, 2048, 2049, 4097, 700, 3, 9000]
    base = synth.multi_arch_sets()
    descs, meas, p0s, opts, masks = [], [], [], [], []
    for k, nk in enumerate(sizes):
        pk = base[k % len(base)]
        mask = synth.fit_mask(pk.n_levels)
        if nk == 0:
            dd = wmb.DeviceDescriptors.from_host(synth.descriptors(64, 300)).slice(0, 0)
            mt = torch.ones(1, dtype=torch.float32, device="cuda")
        else:
            dk = synth.descriptors(nk, 300 + k)
            Tk, _ = orc.predict(pk, dk)
            dd = wmb.DeviceDescriptors.from_host(dk)
            mt = torch.from_numpy((Tk * synth.lognormal_noise(nk, 330 + k, 0.02)).astype(np.float32)).cuda()
        descs.append(dd)
        meas.append(mt)
        p0s.append(synth.perturb_theta(pk, 360 + k, mask=mask))
        opts.append(wmb.calib_opts(steps=20, free_mask=mask))
        masks.append(mask)
    ntot = sum(sizes)
    default = wmb.get_launch(wmb.OP_CALIBRATE_BATCHED, ntot)
    ref = [wmb.calibrate(descs[k], meas[k], p0s[k], steps=20, free_mask=masks[k]) for k in range(len(sizes))]
    try:
        for chunk in (256, 2048):
            wmb.set_launch(wmb.OP_CALIBRATE_BATCHED, ntot, 256, 1, 1, chunk)
            say("16 ragged sets, chunk", chunk)
            rc, thb, histb = wmb.calibrate_batched(descs, meas, p0s, opts)
            assert rc == wmb.WM_OK
            for k, (rck, thk, histk) in enumerate(ref):
                assert np.allclose(histb[k], histk, rtol=PARTITION_RTOL, atol=0), (chunk, k, sizes[k])
                assert np.allclose(thb[k], thk, rtol=PARTITION_RTOL, atol=0), (chunk, k, sizes[k])
        # the empty set: zero loss, theta unchanged (up to exp(log theta))
        assert np.all(histb[0] == 0.0)
        assert np.allclose(thb[0], np.asarray(p0s[0].theta), rtol=1e-12, atol=0)
    finally:
        wmb.set_launch(wmb.OP_CALIBRATE_BATCHED, ntot, default["block"], default["per_thread"],
                       default["grid_mult"], default["chunk"])


def test_calibration_resumes_bit_identically_from_a_checkpoint(wmb, orc, tmp_path):
    """A 120-step calibration run as 45 steps, a checkpoint written to disk
    and read back, then 75 more steps (and as 30 + 30 + 60 with the state
    carried in memory) gives the parameters and loss history of one call,
    bit for bit."""
    n = 1 << 16
    ps, d, m, p0 = _problem(orc, n)
    dd = wmb.DeviceDescriptors.from_host(d)
    mt = torch.from_numpy(m).cuda()
    rc, th, hist = wmb.calibrate(dd, mt, p0, steps=120, free_mask=MASK_L4)
    assert rc == wmb.WM_OK
    rc1, th1, h1, st1 = wmb.calibrate_resume(dd, mt, p0, 120, 45, free_mask=MASK_L4)
    assert rc1 == wmb.WM_OK and st1.step == 45 and st1.diverged == 0
    path = tmp_path / "calib_checkpoint.npz"
    wmb.save_calib_state(path, st1)
    st = wmb.load_calib_state(path)
    assert st.step == 45 and list(st.m) == list(st1.m) and list(st.theta) == list(st1.theta)
    rc2, th2, h2, st2 = wmb.calibrate_resume(dd, mt, p0, 120, 75, state=st, free_mask=MASK_L4)
    assert rc2 == wmb.WM_OK and st2.step == 120
    assert np.array_equal(th2, th)
    assert np.array_equal(np.concatenate([h1, h2]), hist)
    pieces, state = [], None
    for k in (30, 30, 60):
        _, thk, hk, state = wmb.calibrate_resume(dd, mt, p0, 120, k, state=state, free_mask=MASK_L4)
        pieces.append(hk)
    assert np.array_equal(thk, th) and np.array_equal(np.concatenate(pieces), hist)
    say("resume: 45 + 75 and 30 + 30 + 60 steps equal one 120-step call bit for bit")
