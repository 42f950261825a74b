"""Launch configurations and the autotuner: every candidate configuration of
every op gives the same results (forward and tile selection bit for bit;
gradient sums to 1e-12 relative where every lane sees one descriptor, so only
the FP64 addition order changes, and to the float32 rounding of the lanes'
partial sums, 1e-6, where lanes sum several), the tuners install a valid
configuration, and the JSON-lines cache round-trips."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def _restore(wmb, op, n):
    d = {wmb.OP_PREDICT: (256, 4, 1, 0), wmb.OP_CALIBRATE_BATCHED: (256, 1, 1, 2048)}.get(op, (256, 1, 1, 0))
    wmb.set_launch(op, n, *d)


def test_predict_every_config_bitwise_identical(wmb):
    n = 300007
    p = synth.param_set(0)
    dd = wmb.DeviceDescriptors.from_host(synth.descriptors(n, 40))
    ref_T, ref_o = [x.clone() for x in wmb.predict(dd, p)]
    for block in (64, 128, 256, 512):
        for vec in (1, 2, 4, 8):
            wmb.set_launch(wmb.OP_PREDICT, n, block, vec)
            assert wmb.get_launch(wmb.OP_PREDICT, n)["per_thread"] == vec
            T, o = wmb.predict(dd, p)
            torch.cuda.synchronize()
            assert torch.equal(torch.nan_to_num(T, nan=-1.0), torch.nan_to_num(ref_T, nan=-1.0)), (block, vec)
            assert torch.equal(o, ref_o)
    _restore(wmb, wmb.OP_PREDICT, n)


@pytest.mark.parametrize("op", ["vjp", "loss"])
def test_gradient_every_config_matches_default(wmb, orc, op):
    n = 250001
    ps = synth.param_set(1)
    d = synth.descriptors(n, 41)
    dd = wmb.DeviceDescriptors.from_host(d)
    if op == "loss":
        T, _ = orc.predict(ps, d)
        w = torch.from_numpy((T * synth.lognormal_noise(n, 2, 0.02)).astype(np.float32)).cuda()
        code = wmb.OP_LOSS_GRAD
        run = lambda: wmb.loss_grad(dd, w, ps)
    else:
        w = torch.from_numpy(np.random.default_rng(1).standard_normal(n).astype(np.float32)).cuda()
        code = wmb.OP_VJP
        run = lambda: wmb.vjp(dd, ps, w)
    ref = run().cpu().numpy()
    for block in (64, 128, 256, 512):
        for gm in (1, 2, 4):
            wmb.set_launch(code, n, block, 1, gm)
            g = run().cpu().numpy()
            scale = np.abs(ref).max()
            assert np.max(np.abs(g - ref)) <= 1e-12 * scale, (block, gm)
            if op == "loss":
                assert g[1] == ref[1]
    _restore(wmb, code, n)


def test_select_tile_every_config_identical(wmb):
    p = synth.param_set(0)
    sh = synth.shapes(30000, 42)
    dsh = wmb.DeviceShapes.from_host(sh)
    ref = [x.clone() for x in wmb.select_tile(dsh, p)]
    for block in (64, 128, 256, 512):
        for gm in (1, 2, 4):
            wmb.set_launch(wmb.OP_SELECT_TILE, sh.n, block, 1, gm)
            out = wmb.select_tile(dsh, p)
            for a, b in zip(out, ref):
                assert torch.equal(a, b), (block, gm)
    _restore(wmb, wmb.OP_SELECT_TILE, sh.n)


def test_batched_chunks_match(wmb, orc):
    sets = synth.multi_arch_sets()[:3]
    sizes = [20000, 70001, 45000]
    descs, meas, p0s, opts = [], [], [], []
    for k, (pk, nk) in enumerate(zip(sets, sizes)):
        dk = synth.descriptors(nk, 150 + k)
        Tk, _ = orc.predict(pk, dk)
        descs.append(wmb.DeviceDescriptors.from_host(dk))
        meas.append(torch.from_numpy((Tk * synth.lognormal_noise(nk, 160 + k, 0.02)).astype(np.float32)).cuda())
        mask = synth.fit_mask(pk.n_levels)
        p0s.append(synth.perturb_theta(pk, 170 + k, mask=mask))
        opts.append(wmb.calib_opts(steps=25, free_mask=mask))
    ntot = sum(sizes)
    _, th_ref, h_ref = wmb.calibrate_batched(descs, meas, p0s, opts)
    for chunk in (256, 4096, 65536):
        for gm in (1, 2):
            wmb.set_launch(wmb.OP_CALIBRATE_BATCHED, ntot, 256, 1, gm, chunk)
            _, th, h = wmb.calibrate_batched(descs, meas, p0s, opts)
            # other work items split the descriptors differently over lanes,
            # which sum in float32 before the float64 reductions
            assert np.allclose(h, h_ref, rtol=1e-6, atol=0), (chunk, gm)
            assert np.allclose(th, th_ref, rtol=1e-6, atol=0), (chunk, gm)
    _restore(wmb, wmb.OP_CALIBRATE_BATCHED, ntot)
    best = wmb.autotune_batched(descs, meas, p0s, opts)
    say("batched tuned", best)
    assert best["block"] == 256 and best["chunk"] in [1 << k for k in range(8, 17)]
    _restore(wmb, wmb.OP_CALIBRATE_BATCHED, ntot)


def test_autotuners_install_valid_configs_and_cache_roundtrip(wmb, orc, tmp_path):
    cache = tmp_path / "tune.jsonl"
    os.environ["WAVEMODEL_TUNE_CACHE"] = str(cache)
    try:
        n = 1 << 20
        p = synth.param_set(0)
        d = synth.descriptors(n, 43)
        dd = wmb.DeviceDescriptors.from_host(d)
        bp = wmb.autotune_predict(dd, p)
        say("predict tuned", bp)
        assert bp["block"] in (64, 128, 256, 512) and bp["per_thread"] in (1, 2, 4, 8)
        assert wmb.get_launch(wmb.OP_PREDICT, n)["per_thread"] == bp["per_thread"]
        # results with the tuned configuration still match the oracle
        T, occ = wmb.predict(dd, p)
        To, occo = orc.predict(p, d)
        assert np.array_equal(occ.cpu().numpy(), occo)
        Tg = T.cpu().numpy().astype(np.float64)
        f = np.isfinite(To)
        assert np.max(np.abs(Tg[f] - To[f]) / To[f]) <= 1e-5
        w = torch.from_numpy(np.random.default_rng(2).standard_normal(n).astype(np.float32)).cuda()
        bg = wmb.autotune_grad(wmb.OP_VJP, dd, w, p)
        say("vjp tuned", bg)
        sh = synth.shapes(20000, 44)
        bs = wmb.autotune_select_tile(wmb.DeviceShapes.from_host(sh), p)
        say("select tuned", bs)
        lines = [json.loads(l) for l in open(cache)]
        assert {l["op"] for l in lines} == {wmb.OP_PREDICT, wmb.OP_VJP, wmb.OP_SELECT_TILE}
        # a fresh process reads the cache back
        code = ("import sys; sys.path.insert(0, %r); from paper_2605_04178_amd import wavemodel as w; "
                "import json; print(json.dumps([w.get_launch(w.OP_PREDICT, %d), w.get_launch(w.OP_VJP, %d), "
                "w.get_launch(w.OP_SELECT_TILE, %d)]))" % (ROOT, n, n, sh.n))
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240,
                             env=dict(os.environ))
        assert out.returncode == 0, out.stderr[-2000:]
        got = json.loads(out.stdout.strip().splitlines()[-1])
        assert got[0]["block"] == bp["block"] and got[0]["per_thread"] == bp["per_thread"]
        assert got[1]["block"] == bg["block"] and got[1]["grid_mult"] == bg["grid_mult"]
        assert got[2]["block"] == bs["block"] and got[2]["grid_mult"] == bs["grid_mult"]
    finally:
        del os.environ["WAVEMODEL_TUNE_CACHE"]
        _restore(wmb, wmb.OP_PREDICT, 1 << 20)
        _restore(wmb, wmb.OP_VJP, 1 << 20)
        _restore(wmb, wmb.OP_SELECT_TILE, 20000)
