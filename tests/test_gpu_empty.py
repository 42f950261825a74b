"""Empty inputs at every entry point: n == 0 returns WM_OK without touching
the (possibly NULL) arrays; the gradient calls still write their zero
outputs, and calibration over no descriptors leaves theta where it was."""
import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def test_empty_descriptor_calls(wmb):
    p = synth.param_set(0)
    d0 = wmb.DeviceDescriptors.from_host(synth.descriptors(0, 1))
    assert d0.n == 0
    none = torch.empty(0, dtype=torch.float32, device="cuda")
    out = torch.full((26,), 7.0, dtype=torch.float64, device="cuda")
    wmb.loss_grad(d0, none, p, out=out)
    assert torch.count_nonzero(out).item() == 0
    T, occ = wmb.predict(d0, p)
    assert T.numel() == 0 and occ.numel() == 0
    rc, th, hist = wmb.calibrate(d0, none, p, steps=5, free_mask=synth.FIT_MASK_L4)
    assert rc == wmb.WM_OK and np.all(hist == 0.0)
    assert np.allclose(th, np.asarray(p.theta), rtol=1e-12, atol=0)


def test_empty_shape_list(wmb):
    p = synth.param_set(0)
    z = torch.empty(0, dtype=torch.int32, device="cuda")
    sh = wmb.DeviceShapes(z, z, z, z, torch.zeros(1, dtype=torch.int32, device="cuda"), z)
    best, cost, tie = wmb.select_tile(sh, p)
    assert best.numel() == 0 and cost.numel() == 0 and tie.numel() == 0


def test_empty_blackwell_calls(wmb):
    p = synth.b200_like()
    d0 = wmb.DeviceBwDescriptors.from_host(synth.bw_descriptors(64, 219).slice(0, 0))
    assert d0.n == 0
    none = torch.empty(0, dtype=torch.float32, device="cuda")
    T, cta = wmb.bw_predict(d0, p)
    assert T.numel() == 0
    out = wmb.bw_loss_grad(d0, none, p)
    assert torch.count_nonzero(out).item() == 0
    mask = sum(1 << j for j, v in enumerate(p.theta) if v > 0)
    rc, th, hist = wmb.bw_calibrate(d0, none, p, steps=5, free_mask=mask)
    assert rc == wmb.WM_OK and np.all(hist == 0.0)
    assert np.allclose(th, np.asarray(p.theta), rtol=1e-12, atol=0)
