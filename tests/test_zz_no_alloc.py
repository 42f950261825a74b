"""wm_loss_grad_noalloc (the loss + gradient call with the library's fixed
per-GPU scratch instead of a caller workspace) against wm_loss_grad on the
same inputs: two calls in a row, the second on a smaller input, then an
empty one; results must be bit-identical to the workspace call (same
kernels, same launch configuration) and the first call's gradient within the
per-slot bound of the FP64 oracle."""
import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import check_grad, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def _case(orc, n, seed_d, seed_m):
    ps = synth.param_set(1)
    d = synth.descriptors(n, seed_d)
    T, _ = orc.predict(ps, d)
    m = (T * synth.lognormal_noise(n, seed_m, 0.02)).astype(np.float32)
    return ps, synth.perturb_theta(ps, 3), d, m


def test_noalloc_matches_workspace_call_twice_then_smaller(wmb, orc):
    assert wmb.lib().wm_noalloc_scratch_bytes() >= wmb.workspace_bytes(wmb.OP_LOSS_GRAD, wmb.NOALLOC_MAX_N)
    out = torch.full((26,), float("nan"), dtype=torch.float64, device="cuda")
    for k, (n, sd, sm) in enumerate(((300001, 400, 401), (70001, 402, 403))):
        ps, p0, d, m = _case(orc, n, sd, sm)
        say("no-alloc call", k, "n", n)
        dd = wmb.DeviceDescriptors.from_host(d)
        mt = torch.from_numpy(m).cuda()
        wmb.loss_grad_noalloc(dd, mt, p0, out)
        ref = wmb.loss_grad(dd, mt, p0)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (k, out.cpu().numpy(), ref.cpu().numpy())
        if k == 0:
            loss, cnt, g = orc.loss_grad(p0, d, m)
            o = out.cpu().numpy()
            assert int(o[1]) == cnt and abs(o[0] - loss) <= 1e-5 * loss
            check_grad(o[2:], g, p0.theta, "no-alloc loss gradient", 1e-4, names=synth.THETA_NAMES)
    # an empty input after the larger ones: zeros, as wm_loss_grad gives
    d0 = wmb.DeviceDescriptors.from_host(synth.descriptors(0, 1))
    wmb.loss_grad_noalloc(d0, torch.ones(1, device="cuda"), synth.param_set(1), out)
    assert torch.count_nonzero(out).item() == 0


def test_noalloc_on_a_side_stream_and_size_limit(wmb, orc):
    ps, p0, d, m = _case(orc, 4099, 404, 405)
    dd = wmb.DeviceDescriptors.from_host(d)
    mt = torch.from_numpy(m).cuda()
    ref = wmb.loss_grad(dd, mt, p0)
    s = torch.cuda.Stream()
    out = torch.empty(26, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        wmb.loss_grad_noalloc(dd, mt, p0, out, stream=s)
    s.synchronize()
    assert torch.equal(out, ref)
    # n above the maximum is rejected before any work is queued (the arrays'
    # pointers are real, non-null; only the count is too large)
    big = dd.slice(0, dd.n)
    big.n = wmb.NOALLOC_MAX_N + 1
    with pytest.raises(wmb.WmError) as ei:
        wmb.loss_grad_noalloc(big, mt, p0, out)
    assert ei.value.status == wmb.WM_ETOOLARGE
