"""Maximum sizes.  (1) Arrays past 4 GiB: 257 copies of a 2^22-descriptor set
(1.08e9 descriptors; every float array holds 4.3 GB, so element byte offsets
pass 2^31 and 2^32) through the forward sweep and the loss gradient.  Each
output depends on its own descriptor only, so sampled outputs must equal the
oracle on the base set, and the loss and gradient (means over descriptors)
must equal the base set's.  (2) Tile selection with 2.11e9 candidates, just
under the int32 offset limit.  (3) Application totals over 1.09e9 segment
rows.  (4) The Blackwell forward over 1.08e9 descriptors."""
import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import check_grad, need_gpu, rel_err, say

pytestmark = pytest.mark.gpu
N0 = 1 << 22
REPS = 257
TOL = 1e-5
GTOL = 1e-4


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def test_forward_and_loss_grad_past_4_gib(wmb, orc):
    n = REPS * N0
    free, _ = torch.cuda.mem_get_info()
    need = n * (48 + 4 + 4 + 4) + (4 << 30)
    if free < need:
        pytest.skip(f"needs {need / 2 ** 30:.0f} GiB of device memory, {free / 2 ** 30:.0f} free")
    p_true = synth.param_set(1)
    p0 = synth.perturb_theta(p_true, 3)
    d = synth.descriptors(N0, 104)
    m0 = (orc.predict(p_true, d)[0] * synth.lognormal_noise(N0, 5, 0.02)).astype(np.float32)
    say("large: base set and measurements ready; replicating to", n)
    base = wmb.DeviceDescriptors.from_host(d)
    fields = wmb.DeviceDescriptors.FLOATS + wmb.DeviceDescriptors.INTS
    big = wmb.DeviceDescriptors({f: getattr(base, f).repeat(REPS) for f in fields})
    assert big.n == n and big.F.numel() * 4 > (1 << 32)

    # forward: sampled outputs, including the elements at byte offsets 2^31 and 2^32
    T, occ = wmb.predict(big, p0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    edges = np.array([(1 << 29) - 1, 1 << 29, (1 << 30) - 1, 1 << 30, (1 << 30) + 1, n - 2, n - 1])
    idx = np.unique(np.concatenate([rng.choice(n, 1 << 14, replace=False), edges]))
    it = torch.from_numpy(idx).cuda()
    Ts = T[it].cpu().numpy()
    occs = occ[it].cpu().numpy()
    del T, occ
    To, occo = orc.predict(p0, d.take(idx % N0))
    assert np.array_equal(occs, occo)
    assert rel_err(Ts, To).max() <= TOL
    say("large: forward sampled outputs match")

    # loss and gradient: the same mean as the base set
    mt = torch.from_numpy(m0).cuda()
    out_big = wmb.loss_grad(big, mt.repeat(REPS), p0).cpu().numpy()
    out_base = wmb.loss_grad(base, mt, p0).cpu().numpy()
    del big
    torch.cuda.empty_cache()
    assert int(out_big[1]) == REPS * int(out_base[1])
    # the replicated sweep gives each lane ~2700 descriptors, the base sweep a
    # few: they agree to the float32 rounding of the lanes' partial sums
    assert abs(out_big[0] - out_base[0]) <= 1e-6 * out_base[0]
    check_grad(out_big[2:], out_base[2:], p0.theta, "large: replicated set against the base set", 1e-6,
               names=synth.THETA_NAMES)
    loss, cnt, g = orc.loss_grad(p0, d, m0)
    assert int(out_base[1]) == cnt
    assert abs(out_big[0] - loss) <= 1e-5 * loss
    check_grad(out_big[2:], g, p0.theta, "large: loss gradient against the oracle", GTOL,
               names=synth.THETA_NAMES)
    say("large: loss gradient over", n, "descriptors matches the base set and the oracle")


def test_select_tile_near_the_int32_candidate_limit(wmb, orc):
    """2^25 shapes of 63 candidates each: 2.11e9 candidates, just under the
    int32 offset limit (8.5 GB of codes), as 512 copies of a 2^16-shape set;
    sampled shapes against the oracle on the base set, the tail included."""
    n0, per, reps = 1 << 16, 63, 512
    n = n0 * reps
    free, _ = torch.cuda.mem_get_info()
    need = n * per * 4 + n * 40 + (4 << 30)
    if free < need:
        pytest.skip(f"needs {need / 2 ** 30:.0f} GiB of device memory, {free / 2 ** 30:.0f} free")
    sh = synth.shapes(n0, 105, cmin=per, cmax=per)
    assert np.all(np.diff(sh.cand_off) == per)
    p = synth.param_set(0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()
    big = wmb.DeviceShapes(t(sh.M).repeat(reps), t(sh.N).repeat(reps), t(sh.K).repeat(reps),
                           t(sh.dtype).repeat(reps),
                           torch.arange(n + 1, dtype=torch.int64, device="cuda").mul_(per).to(torch.int32),
                           t(sh.cand_code.view(np.int32)).repeat(reps))
    assert int(big.cand_off[-1].item()) == n * per < 2 ** 31
    say("large: select_tile over", n, "shapes,", n * per, "candidates")
    best, cost, tie = wmb.select_tile(big, p)
    torch.cuda.synchronize()
    rng = np.random.default_rng(13)
    idx = np.unique(np.concatenate([rng.choice(n, 1 << 13, replace=False), [n // 2, n - 2, n - 1]]))
    it = torch.from_numpy(idx).cuda()
    b, c, tt = (x[it].cpu().numpy() for x in (best, cost, tie))
    del big, best, cost, tie
    torch.cuda.empty_cache()
    bo, co, to = orc.select_tile(p, sh)
    j = idx % n0
    assert np.array_equal(tt, to[j])
    clean = to[j] == 0
    assert np.array_equal(b[clean], bo[j][clean])
    fin = np.isfinite(co[j])
    assert np.array_equal(np.isfinite(c), fin)
    assert np.all(np.abs(c[fin] - co[j][fin]) <= 1e-12 * co[j][fin])
    say("large: sampled tile choices match")


def test_application_totals_past_2p30_rows(wmb, orc):
    """640 copies of 2^18 applications: 1.09e9 segment rows (74 GB of rows
    and descriptors, row indices past 2^30); sampled application totals
    against the oracle on the base set."""
    na0, reps = 1 << 18, 640
    sg, d = synth.segments(na0, 150)
    rows0 = int(sg.app_off[-1])
    n_rows, n_apps = rows0 * reps, na0 * reps
    free, _ = torch.cuda.mem_get_info()
    need = n_rows * (48 + 20) + n_apps * 8 + (4 << 30)
    if free < need or n_rows >= 2 ** 31:
        pytest.skip(f"needs {need / 2 ** 30:.0f} GiB of device memory, {free / 2 ** 30:.0f} free")
    p, q = synth.param_set(0), synth.seg_params(7)
    base = wmb.DeviceDescriptors.from_host(d)
    fields = wmb.DeviceDescriptors.FLOATS + wmb.DeviceDescriptors.INTS
    big = wmb.DeviceDescriptors({f: getattr(base, f).repeat(reps) for f in fields})
    del base
    s0 = wmb.DeviceSegments.from_host(sg)
    off0 = s0.app_off[:-1].to(torch.int64)
    shift = (torch.arange(reps, dtype=torch.int64, device="cuda") * rows0).repeat_interleave(na0)
    off = torch.cat([off0.repeat(reps) + shift, torch.tensor([n_rows], dtype=torch.int64, device="cuda")])
    segs = wmb.DeviceSegments({"app_off": off.to(torch.int32), **{f: getattr(s0, f).repeat(reps)
                                                                  for f, _ in wmb.DeviceSegments.FIELDS[1:]}})
    assert segs.n == n_rows > 2 ** 30 and segs.n_apps == n_apps
    say("large: application totals over", n_apps, "applications,", n_rows, "rows")
    Ta, _ = wmb.predict_apps(big, segs, p, q)
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    idx = np.unique(np.concatenate([rng.choice(n_apps, 1 << 14, replace=False), [n_apps - 1]]))
    Ts = Ta[torch.from_numpy(idx).cuda()].cpu().numpy()
    del big, segs, Ta, off, shift
    torch.cuda.empty_cache()
    Ra, _ = orc.predict_apps(p, q, d, sg)
    assert rel_err(Ts, Ra[idx % na0]).max() <= TOL
    say("large: sampled application totals match")


def test_blackwell_forward_past_4_gib(wmb, orc):
    """The Blackwell forward over 1.08e9 descriptors (257 copies of 2^22;
    4.3 GB per array); sampled times and CTA residencies against the oracle
    on the base set."""
    n0, reps = 1 << 22, 257
    n = n0 * reps
    free, _ = torch.cuda.mem_get_info()
    need = n * (32 + 8) + (4 << 30)
    if free < need:
        pytest.skip(f"needs {need / 2 ** 30:.0f} GiB of device memory, {free / 2 ** 30:.0f} free")
    p = synth.bw_param_set(1)
    d = synth.bw_descriptors(n0, 230)
    base = wmb.DeviceBwDescriptors.from_host(d)
    big = wmb.DeviceBwDescriptors({f: getattr(base, f).repeat(reps)
                                   for f in wmb.DeviceBwDescriptors.INTS + wmb.DeviceBwDescriptors.FLOATS})
    del base
    say("large: Blackwell forward over", n, "descriptors")
    T, cta = wmb.bw_predict(big, p)
    torch.cuda.synchronize()
    rng = np.random.default_rng(19)
    idx = np.unique(np.concatenate([rng.choice(n, 1 << 14, replace=False), [(1 << 30) - 1, 1 << 30, n - 1]]))
    it = torch.from_numpy(idx).cuda()
    Ts, cs = T[it].cpu().numpy(), cta[it].cpu().numpy()
    del big, T, cta
    torch.cuda.empty_cache()
    To, co = orc.bw_predict(p, d)
    j = idx % n0
    assert np.array_equal(cs, co[j])
    assert rel_err(Ts, To[j]).max() <= TOL
    say("large: sampled Blackwell outputs match")
