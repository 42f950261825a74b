"""The validation kernels compute what their flop and byte counts assume
(outputs checked against NumPy on small and ragged sizes), and each
microbenchmark runs and reports a finite positive figure."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mb():
    need_gpu()
    from paper_2605_04178_amd import microbench
    microbench.lib()
    return microbench


def _run(mb, kind, a, b, c, n, iters=0):
    L = mb.lib()
    sec, grid = C.c_double(), C.c_int64()
    say("val kernel", kind, n)
    rc = L.wmb_val_run(mb.VAL[kind], C.c_void_p(a.data_ptr()), a.numel() * a.element_size(),
                       C.c_void_p(b.data_ptr()) if b is not None else None,
                       0 if b is None else b.numel() * b.element_size(),
                       C.c_void_p(c.data_ptr()), c.numel() * c.element_size(), n, iters, 2,
                       C.c_void_p(torch.cuda.current_stream().cuda_stream), C.byref(sec), C.byref(grid))
    assert rc == 0, (kind, rc, L.wmb_last_hip_error())
    torch.cuda.synchronize()
    assert sec.value > 0
    return grid.value


def test_elementwise_kernels(mb):
    rng = np.random.default_rng(0)
    n = 4 * 1000
    a = torch.from_numpy(rng.random(n, dtype=np.float32)).cuda()
    b = torch.from_numpy(rng.random(n, dtype=np.float32)).cuda()
    c = torch.zeros(n, device="cuda")
    _run(mb, "copy", a, None, c, n)
    assert torch.equal(c, a)
    _run(mb, "triad", a, b, c, n)
    assert torch.allclose(c, a + 1.5 * b, rtol=1e-6, atol=0)
    _run(mb, "fma", a, None, c, n, iters=10)
    x = a.cpu().numpy().astype(np.float64)
    for _ in range(10):
        x = x * np.float32(0.9999) + np.float32(1e-4)
    assert np.allclose(c.cpu().numpy(), x, rtol=1e-5)
    part = torch.zeros(4096, device="cuda")
    g = _run(mb, "reduce", a, None, part, n)
    assert abs(part[:g].double().sum().item() - a.double().sum().item()) < 1e-3


@pytest.mark.parametrize("m", [64, 100])
def test_stencil_and_transposes(mb, m):
    rng = np.random.default_rng(1)
    x = rng.random((m, m), dtype=np.float32)
    a = torch.from_numpy(x).cuda().reshape(-1)
    c = torch.zeros(m * m, device="cuda")
    _run(mb, "stencil", a, None, c, m)
    got = c.cpu().numpy().reshape(m, m)
    ref = np.float32(0.2) * ((((x[1:-1, 1:-1] + x[1:-1, :-2]) + x[1:-1, 2:]) + x[:-2, 1:-1]) + x[2:, 1:-1])
    assert np.allclose(got[1:-1, 1:-1], ref, rtol=1e-6, atol=0)
    for kind in ("transpose_naive", "transpose_lds"):
        c.zero_()
        _run(mb, kind, a, None, c, m)
        assert np.array_equal(c.cpu().numpy().reshape(m, m), x.T), kind


@pytest.mark.parametrize("kind", ["gemm8", "gemm16", "gemm32"])
def test_tiled_gemms(mb, kind):
    m = 100
    rng = np.random.default_rng(2)
    A = rng.standard_normal((m, m)).astype(np.float32)
    B = rng.standard_normal((m, m)).astype(np.float32)
    c = torch.zeros(m * m, device="cuda")
    _run(mb, kind, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), c, m)
    ref = A.astype(np.float64) @ B.astype(np.float64)
    assert np.allclose(c.cpu().numpy().reshape(m, m), ref, rtol=1e-4, atol=1e-4)


@pytest.mark.parametrize("m", [64, 192])
def test_matrix_core_gemm(mb, m):
    rng = np.random.default_rng(3)
    A = torch.from_numpy(rng.standard_normal((m, m)).astype(np.float32)).to(torch.bfloat16)
    Bt = torch.from_numpy(rng.standard_normal((m, m)).astype(np.float32)).to(torch.bfloat16)
    c = torch.zeros(m * m, device="cuda")
    _run(mb, "gemm_mfma", A.cuda().contiguous(), Bt.cuda().contiguous(), c, m)
    ref = A.double().numpy() @ Bt.double().numpy().T
    assert np.allclose(c.cpu().numpy().reshape(m, m), ref, rtol=1e-3, atol=1e-3)


@pytest.mark.parametrize("m", [128, 256])
def test_bias_and_fused_gemm_bias(mb, m):
    """The fusion pair: the bias kernel adds bias[col] to every row; the fused
    GEMM equals the plain GEMM plus the bias."""
    rng = np.random.default_rng(m + 1)
    A = torch.from_numpy(rng.standard_normal((m, m)).astype(np.float32)).to(torch.bfloat16)
    Bt = torch.from_numpy(rng.standard_normal((m, m)).astype(np.float32)).to(torch.bfloat16)
    bias = rng.standard_normal(m).astype(np.float32)
    bbuf = torch.zeros(m * m + 2 * m, dtype=torch.bfloat16)
    bbuf[: m * m] = Bt.reshape(-1)
    bbuf[m * m:].view(torch.float32).copy_(torch.from_numpy(bias))
    c = torch.zeros(m * m, dtype=torch.float32, device="cuda")
    _run(mb, "gemm_mfma_bias", A.cuda().contiguous().reshape(-1), bbuf.cuda(), c, m)
    ref = A.double().numpy() @ Bt.double().numpy().T + bias[None, :]
    assert np.allclose(c.cpu().numpy().reshape(m, m), ref, rtol=1e-3, atol=1e-3)
    x = rng.standard_normal((m, m)).astype(np.float32)
    cb = torch.from_numpy(x.reshape(-1)).cuda()
    # wmb_val_run runs the kernel once untimed and `launches` times timed
    L = mb.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    sec, g = C.c_double(), C.c_int64()
    bd = torch.from_numpy(bias).cuda()
    assert L.wmb_val_run(mb.VAL["bias"], C.c_void_p(bd.data_ptr()), m * 4, None, 0, C.c_void_p(cb.data_ptr()),
                         m * m * 4, m, 0, 2, st, C.byref(sec), C.byref(g)) == 0
    assert np.allclose(cb.cpu().numpy().reshape(m, m), x + 3 * bias[None, :], rtol=1e-5, atol=1e-5)


def test_host_sync_cost(mb):
    L = mb.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    si = torch.zeros(4, dtype=torch.int32, device="cuda")
    per = C.c_double()
    assert L.wmb_sync(50, C.c_void_p(si.data_ptr()), st, C.byref(per)) == 0
    say("host sync us", per.value * 1e6)
    assert -1e-4 < per.value < 1e-3


def test_microbenchmarks_run(mb):
    L = mb.lib()
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    sec, fl = C.c_double(), C.c_double()
    buf = torch.ones(1 << 20, device="cuda")
    sink = torch.zeros(256, device="cuda")
    for shared in (0, 1):
        assert L.wmb_read_bw(C.c_void_p(buf.data_ptr()), 4 << 20, 2, 64, shared, C.c_void_p(sink.data_ptr()),
                             3, st, C.byref(sec)) == 0
        assert 0 < sec.value < 1
    nxt = torch.from_numpy(mb.chase_chain(1024, 32, 0).view(np.int32)).cuda()
    ticks = torch.zeros(1, dtype=torch.int64, device="cuda")
    su = torch.zeros(1, dtype=torch.int32, device="cuda")
    for warm in (4096, 0):
        assert L.wmb_chase(C.c_void_p(nxt.data_ptr()), nxt.numel(), 4096, warm, C.c_void_p(su.data_ptr()),
                           C.c_void_p(ticks.data_ptr()), st, C.byref(sec)) == 0
        say("chase ns/step, warm steps", warm, sec.value)
        assert 1 < sec.value < 1e4
        # after 4096 steps round a 1024-node cycle the chase is back at node 0
        assert int(su.item()) == 0
    for kind in range(5):
        assert L.wmb_peak(kind, 16, 64, C.c_void_p(sink.data_ptr()), 2, st, C.byref(sec), C.byref(fl)) == 0
        say("peak", kind, fl.value / sec.value / 1e12, "TF/s (small grid)")
        assert sec.value > 0 and fl.value > 0
    si = torch.zeros(4, dtype=torch.int32, device="cuda")
    assert L.wmb_empty(128, 256, 16, C.c_void_p(si.data_ptr()), 3, st, C.byref(sec)) == 0
    assert 0 < sec.value < 1e-2


def test_shader_clock(mb):
    """The shader-cycle counter against the constant-rate wall clock: a
    plausible clock for this part, lightly loaded and under load."""
    f1 = mb.clock_hz(1, 1 << 18)
    props = torch.cuda.get_device_properties(0)
    f2 = mb.clock_hz(props.multi_processor_count * 32, 1 << 18)
    say("shader clock GHz: one wave", f1 / 1e9, "loaded", f2 / 1e9)
    assert 0.5e9 < f1 < 5e9 and 0.5e9 < f2 < 5e9


def test_shipped_mi355x_parameters_predict_held_out_kernels(mb):
    """The shipped parameter file is valid and, on the held-out validation
    kernels re-timed on this GPU, the calibrated model's MAE is at most 0.6 of
    the naive roofline's and within 0.06 of the MAE recorded with the file."""
    import json
    import os
    from paper_2605_04178_amd import recalibrate as rc, wavemodel as wm
    path = os.path.join(os.path.dirname(mb.__file__), "params", "mi355x.json")
    rec = json.load(open(path))
    p = rc.load_params(path)
    assert wm.validate_params(p)
    names = {c["name"] for c in rec["cases"] if c["split"] == "hold"}
    cases = [c for c in mb.case_list() if c.name in names]
    assert len(cases) >= 10
    mb.run_cases(cases, launches=3, log=lambda *a: None)
    meas = np.array([c.seconds for c in cases])
    T, _ = rc.predict(wm, p, cases)
    e_model, e_roof = mb.mae(T, meas), mb.mae(mb.roofline_naive(cases), meas)
    say("held-out MAE calibrated", e_model, "roofline", e_roof, "recorded", rec["mae"]["calibrated_holdout"])
    # re-timing the kernels moves the MAE by well under 0.01 between runs on
    # one machine, but the recorded figure comes from another MI355X: across
    # machines the held-out MAE has read 0.186 to 0.223 (clocks and memory
    # timings differ by several per cent per kernel).  0.06 over the recorded
    # figure, and a bound relative to the roofline measured on this machine,
    # still fail a real regression.
    assert e_model <= 0.6 * e_roof and e_model <= rec["mae"]["calibrated_holdout"] + 0.06
