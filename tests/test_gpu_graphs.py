"""The entry points a caller may capture (predict, the loss gradient, the
vector-Jacobian product, the application calls and the Blackwell forward and
loss gradient) recorded in one HIP graph and replayed, with eager work and
synchronisations between replays: every replay must reproduce the eager
results bit for bit (none of these calls records a memset or a sync, and
their reductions run in a fixed order)."""
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


def _bits(x):
    return x.view(torch.int64) if x.element_size() == 8 else x.view(torch.int32) if x.element_size() == 4 else x


def test_entry_points_replayed_from_a_graph(wmb):
    p, q, pb = synth.param_set(0), synth.seg_params(7), synth.bw_param_set(1)
    n = 100_000
    dd = wmb.DeviceDescriptors.from_host(synth.descriptors(n, 400))
    T0, _ = wmb.predict(dd, p)
    meas = (T0 * 1.03).contiguous()
    w = torch.randn(n, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    sg, d2 = synth.segments(4096, 401)
    da, ds = wmb.DeviceDescriptors.from_host(d2), wmb.DeviceSegments.from_host(sg)
    Ta0, _ = wmb.predict_apps(da, ds, p, q)
    ma = (Ta0 * 0.97).contiguous()
    db = wmb.DeviceBwDescriptors.from_host(synth.bw_descriptors(n, 402))
    Tb0, _ = wmb.bw_predict(db, pb)
    mb = (Tb0 * 1.02).contiguous()

    ws_l = wmb._workspace(wmb.workspace_bytes(wmb.OP_LOSS_GRAD, n), "cuda")
    ws_v = wmb._workspace(wmb.workspace_bytes(wmb.OP_VJP, n), "cuda")
    ws_a = wmb._workspace(wmb.apps_workspace_bytes(da.n, ds.n_apps), "cuda")
    ws_b = wmb._workspace(wmb.bw_workspace_bytes(wmb.BW_OP_GRAD, n), "cuda")
    outT = torch.empty(n, dtype=torch.float32, device="cuda")
    outO = torch.empty(n, dtype=torch.int32, device="cuda")
    out_l = torch.empty(26, dtype=torch.float64, device="cuda")
    out_ta = torch.empty(ds.n_apps, dtype=torch.float32, device="cuda")
    out_a = torch.empty(2 + wmb.N_THETA + wmb.N_SEGPARAMS, dtype=torch.float64, device="cuda")
    out_bT = torch.empty(n, dtype=torch.float32, device="cuda")
    out_b = torch.empty(26, dtype=torch.float64, device="cuda")

    def run():
        wmb.predict(dd, p, out_T=outT, out_occ=outO)
        wmb.loss_grad(dd, meas, p, ws=ws_l, out=out_l)
        gv = wmb.vjp(dd, p, w, ws=ws_v)
        wmb.predict_apps(da, ds, p, q, out=out_ta)
        wmb.apps_loss_grad(da, ds, ma, p, q, ws=ws_a, out=out_a)
        wmb.bw_predict(db, pb, out_T=out_bT, want_cta=False)
        wmb.bw_loss_grad(db, mb, pb, ws=ws_b, out=out_b)
        return gv

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gv = run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    eager = [x.clone() for x in (outT, outO, out_l, gv, out_ta, out_a, out_bT, out_b)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gv_g = run()
    outs = (outT, outO, out_l, gv_g, out_ta, out_a, out_bT, out_b)
    for r in range(4):
        for x in outs:
            x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(outs, eager)):
            assert torch.equal(_bits(a), _bits(b)), (r, k)
        _ = torch.randn(1000, device="cuda").sum().item()   # eager work between replays
