"""Parity of the HIP forward sweep (wm_predict, wm_roofline) with the FP64
oracle: occupancy bit-exact, predicted time within 1e-5 relative."""
import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import need_gpu, rel_err, say

pytestmark = pytest.mark.gpu
TOL = 1e-5
MIB = 1 << 20


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def _parity(wmb, orc, p, d, tag):
    say("predict parity", tag, "n =", d.n)
    dd = wmb.DeviceDescriptors.from_host(d)
    T, occ = wmb.predict(dd, p)
    torch.cuda.synchronize()
    To, occo = orc.predict(p, d)
    occ = occ.cpu().numpy()
    T = T.cpu().numpy()
    assert np.array_equal(occ, occo), tag
    err = rel_err(T, To)
    assert err.max() <= TOL, (tag, float(err.max()), int(err.argmax()))
    return T, occ, err


@pytest.mark.parametrize("L,combine", [(4, 0), (3, 0), (4, 1), (3, 1)])
def test_predict_parity_small_config(wmb, orc, L, combine):
    p = synth.param_set(0, n_levels=L, combine=combine)
    d = synth.descriptors(4096, 100)
    T, occ, err = _parity(wmb, orc, p, d, f"L{L} c{combine}")
    assert (occ == 0).mean() > 0.15 and (occ > 0).mean() > 0.5


@pytest.mark.parametrize("n", [1, 3, 5, 1023, 1025, 4097, 100003])
def test_predict_ragged_sizes(wmb, orc, n):
    p = synth.param_set(0)
    d = synth.descriptors(n, 200 + n)
    _parity(wmb, orc, p, d, f"ragged {n}")


def test_predict_misaligned_takes_scalar_path_with_same_results(wmb):
    p = synth.param_set(0)
    d = synth.descriptors(10001, 31)
    dd = wmb.DeviceDescriptors.from_host(d)
    T_full, occ_full = wmb.predict(dd, p)
    sub = dd.slice(1, dd.n)          # every array now 4 bytes off 16-byte alignment
    T_sub, occ_sub = wmb.predict(sub, p)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(T_sub, nan=-1.0), torch.nan_to_num(T_full[1:], nan=-1.0))
    assert torch.equal(occ_sub, occ_full[1:])


def test_predict_without_occupancy_output(wmb):
    p = synth.param_set(0)
    d = synth.descriptors(5000, 32)
    dd = wmb.DeviceDescriptors.from_host(d)
    T1, _ = wmb.predict(dd, p)
    T2, occ = wmb.predict(dd, p, want_occ=False)
    torch.cuda.synchronize()
    assert occ is None
    assert torch.equal(torch.nan_to_num(T1, nan=-1.0), torch.nan_to_num(T2, nan=-1.0))


def test_predict_is_deterministic(wmb):
    p = synth.param_set(0)
    dd = wmb.DeviceDescriptors.from_host(synth.descriptors(50000, 33))
    a, _ = wmb.predict(dd, p)
    b, _ = wmb.predict(dd, p)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(a, nan=-1.0), torch.nan_to_num(b, nan=-1.0))


def test_predict_empty(wmb):
    p = synth.param_set(0)
    dd = wmb.DeviceDescriptors.from_host(synth.descriptors(0, 1))
    T, occ = wmb.predict(dd, p)
    torch.cuda.synchronize()
    assert T.numel() == 0 and occ.numel() == 0


def test_predict_invalid_and_infeasible(wmb, orc):
    p = synth.param_set(0)
    d = synth.descriptors(64, 34)
    # plant invalid fields and infeasible launches
    d.F[0] = -1.0
    d.B[1] = np.inf
    d.u[2] = 0.0
    d.r2[3] = 1.5
    d.vgpr[4] = 0
    d.lds[5] = -3
    d.grid[6] = 0
    d.gpack[7] = int(synth.pack_gpack(2000, 1))
    d.gpack[8] = int(synth.pack_gpack(64, 6))
    d.gpack[9] = d.gpack[10] | (1 << 27)
    d.W[11] = np.nan
    d.K[12] = -1.0
    d.vgpr[20], d.gpack[20] = 512, int(synth.pack_gpack(1024, 1))   # 16 waves, 4 fit
    d.lds[21] = 65537                                               # more LDS than a CU has
    d.vgpr[22] = 513                                                # more VGPRs than a SIMD has
    T, occ, err = _parity(wmb, orc, p, d, "invalid/infeasible")
    for i in (0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 12):
        assert occ[i] == -1 and np.isnan(T[i]), i
    for i in (20, 21, 22):
        assert occ[i] == 0 and np.isinf(T[i]) and T[i] > 0, i


def test_predict_working_set_regimes(wmb, orc):
    """h_LLC(W) in every regime, including W right below C = 256 MiB where the
    transition branch nearly vanishes, and the Eq. (16) blend."""
    p = synth.param_set(0)
    d = synth.descriptors(20000, 35)
    rng = np.random.default_rng(0)
    W = np.concatenate([rng.uniform(1, 204.99, 4000), rng.uniform(205, 256, 8000),
                        256 - rng.integers(0, 2000, 4000) * 2.0 ** -16,
                        rng.uniform(256.001, 4096, 4000)]) * MIB
    d.W = W.astype(np.float32)
    _parity(wmb, orc, p, d, "W regimes")


def test_predict_overlap_combine_with_wave_caps(wmb, orc):
    p = synth.param_set(0, combine=1).copy(mwp=6, cwp=9)
    _parity(wmb, orc, p, synth.descriptors(30000, 36), "eta mwp/cwp")


def test_predict_mi300a_like_and_multi_arch(wmb, orc):
    d = synth.descriptors(20000, 37)
    _parity(wmb, orc, synth.mi300a_like(), d, "mi300a-like")
    for k, p in enumerate(synth.multi_arch_sets()):
        _parity(wmb, orc, p, d, f"arch{k}")


def test_roofline_parity(wmb, orc):
    p = synth.param_set(0)
    d = synth.descriptors(20000, 38)
    d.F[0] = -5.0
    dd = wmb.DeviceDescriptors.from_host(d)
    R = wmb.roofline(dd, p).cpu().numpy()
    Ro = orc.roofline(p, d)
    assert rel_err(R, Ro).max() <= 1e-6


def test_predict_full_size_sampled(wmb, orc):
    """2^24 descriptors in the launch configuration the benchmark times;
    2^16 sampled outputs recomputed by the oracle one by one."""
    n = 1 << 24
    p = synth.param_set(0)
    say("generating", n)
    d = synth.descriptors(n, 101)
    dd = wmb.DeviceDescriptors.from_host(d)
    T, occ = wmb.predict(dd, p)
    torch.cuda.synchronize()
    T = T.cpu().numpy()
    occ = occ.cpu().numpy()
    idx = np.sort(np.random.default_rng(7).choice(n, 1 << 16, replace=False))
    idx = np.concatenate([idx, np.arange(n - 5, n)])
    sub = d.take(idx)
    To, occo = orc.predict(p, sub)
    assert np.array_equal(occ[idx], occo)
    assert rel_err(T[idx], To).max() <= TOL
    # the autotuned launch configuration (what the benchmark times) gives the
    # same bytes
    best = wmb.autotune_predict(dd, p)
    say("tuned", best)
    T2, occ2 = wmb.predict(dd, p)
    torch.cuda.synchronize()
    assert np.array_equal(occ2.cpu().numpy(), occ)
    assert np.array_equal(np.nan_to_num(T2.cpu().numpy(), nan=-1.0), np.nan_to_num(T, nan=-1.0))
    wmb.set_launch(wmb.OP_PREDICT, n, 256, 4)
    # properties over every output
    assert np.all((occ >= -1) & (occ <= p.n_simd * p.waves_simd))
    assert np.all(np.isinf(T[occ == 0])) and np.all(np.isfinite(T[occ > 0]))
    assert np.all(T[occ > 0] >= p.theta[13] * (1 - 1e-6))


def test_predict_hand_worked_latency_and_overhead_rows(wmb):
    """The rows of tests/golden/latency_stage.txt and overhead_terms.txt
    (values worked by hand) through the forward sweep: occupancy exact, T
    within the float32 bound of the hand-worked value."""
    from test_oracle_latency_overhead import U, _params, _rows
    p = _params()
    lat, ovh = _rows("latency_stage.txt"), _rows("overhead_terms.txt")
    n1, n2 = len(lat), len(ovh)
    f = lambda v: np.array(v, np.float32)
    d = synth.Descriptors(
        F=np.zeros(n1 + n2, np.float32),
        B=f([float(r[5]) for r in lat] + [0.0] * n2),
        r1=f([float(r[6]) for r in lat] + [0.0] * n2),
        r2=f([float(r[7]) for r in lat] + [0.0] * n2),
        r3=np.zeros(n1 + n2, np.float32),
        K=f([0.0] * n1 + [float(r[2]) for r in ovh]),
        u=np.ones(n1 + n2, np.float32), W=np.zeros(n1 + n2, np.float32),
        vgpr=np.array([int(r[2]) for r in lat] + [128] * n2, np.int32),
        lds=np.array([int(r[3]) for r in lat] + [0] * n2, np.int32),
        gpack=np.concatenate([synth.pack_gpack(np.array([int(r[1]) for r in lat]), 1),
                              synth.pack_gpack(256, 1, np.array([int(r[3]) for r in ovh]),
                                               np.array([int(r[4]) for r in ovh]),
                                               np.array([int(r[5]) for r in ovh]),
                                               np.array([int(r[6]) for r in ovh]))]),
        grid=np.array([int(r[4]) for r in lat] + [int(r[1]) for r in ovh], np.int32))
    T, occ = wmb.predict(wmb.DeviceDescriptors.from_host(d), p)
    want_T = np.array([float(r[14]) * U for r in lat] + [float(r[14]) * U for r in ovh])
    want_o = np.array([int(r[9]) for r in lat] + [4] * n2, np.int32)
    assert np.array_equal(occ.cpu().numpy(), want_o)
    err = rel_err(T.cpu().numpy(), want_T)
    say("hand-worked rows on the GPU: max rel err", err.max())
    assert err.max() <= TOL
