"""Parity of per-group calibration multipliers (wm_fit_multipliers) and
fusion planning (wm_plan_fusion) with the FP64 oracle.  The optimal
objective values are unique and compared to rounding; where the oracle and
the GPU pick different multipliers or plans, the objective of the GPU's
choice must equal the optimum (a tie)."""
import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def _obj(mu, T, m):
    ok = np.isfinite(T) & (T > 0) & np.isfinite(m) & (m > 0)
    return float(np.sum(np.abs(mu * T[ok] - m[ok]) / m[ok]))


def _check_mult(wmb, orc, T, m, off, train, tag):
    T = np.asarray(T, np.float32)
    m = np.asarray(m, np.float32)
    say("multipliers", tag, "groups", len(off) - 1, "rows", T.shape[0])
    dT = torch.from_numpy(T).cuda()
    dm = torch.from_numpy(m).cuda()
    mult, Ts, st = wmb.fit_multipliers(dT, dm, torch.from_numpy(np.asarray(off, np.int32)).cuda(),
                                       torch.from_numpy(np.asarray(train, np.uint8)).cuda())
    mult, Ts, st = mult.cpu().numpy(), Ts.cpu().numpy(), st.cpu().numpy()
    om, oTs, ost = orc.fit_multipliers(T.astype(np.float64), m.astype(np.float64), off, train)
    diff = np.flatnonzero(mult != om)
    for g in diff:
        a, b = off[g], off[g + 1]
        sel = np.asarray(train[a:b], bool)
        Tg, mg = T[a:b][sel].astype(np.float64), m[a:b][sel].astype(np.float64)
        o1, o2 = _obj(mult[g], Tg, mg), _obj(om[g], Tg, mg)
        assert abs(o1 - o2) <= 1e-12 * max(o2, 1e-300), (g, mult[g], om[g], o1, o2)
    say("  groups differing (ties):", len(diff))
    assert len(diff) <= max(2, len(om) // 1000)
    same = np.repeat(mult == om, np.diff(off))
    assert np.array_equal(np.nan_to_num(Ts[same], nan=-1), np.nan_to_num(oTs[same].astype(np.float32), nan=-1))
    assert st[1] == ost[1] and st[3] == ost[3]
    for j in (0, 2):
        assert abs(st[j] - ost[j]) <= 1e-9 * max(ost[j], 1e-300)
    return mult


def test_multipliers_parity(wmb, orc):
    p = synth.param_set(0)
    off, fac, noise, train, d = synth.grouped_measurements(3000, 171)
    T, _ = orc.predict(p, d)
    g = np.repeat(np.arange(3000), np.diff(off))
    _check_mult(wmb, orc, T, T * fac[g] * noise, off, train, "noisy")


def test_multipliers_edge_cases(wmb, orc):
    rng = np.random.default_rng(5)
    # empty groups, a group with no training rows, invalid rows, exact ties,
    # one group of 3000 rows
    sizes = [0, 1, 5, 0, 7, 3000, 2, 0]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(off[-1])
    T = rng.uniform(1e-5, 1e-2, n)
    m = T * rng.uniform(0.5, 2.0, n)
    train = (rng.random(n) < 0.7).astype(np.uint8)
    train[off[4]:off[5]] = 0
    T[off[2]] = np.nan
    T[off[2] + 1] = np.inf
    m[off[2] + 2] = 0.0
    m[off[6]:off[7]] = 2.0 * T[off[6]:off[7]]       # equal ratios: a tie
    mult = _check_mult(wmb, orc, T, m, off, train, "edges")
    assert mult[0] == 1.0 and mult[3] == 1.0 and mult[4] == 1.0
    # no groups at all
    z = torch.zeros(0, device="cuda")
    _, _, st = wmb.fit_multipliers(z, z, torch.zeros(1, dtype=torch.int32, device="cuda"),
                                   torch.zeros(0, dtype=torch.uint8, device="cuda"))
    assert np.array_equal(st.cpu().numpy(), np.zeros(4))


def _check_plan(wmb, orc, p, off, d, e, R, tag):
    say("fusion", tag, "chains", len(off) - 1, "rows", off[-1], "R", R)
    dd = wmb.DeviceDescriptors.from_host(d)
    tot, unf, st = wmb.plan_fusion(dd, torch.from_numpy(e).cuda(), torch.from_numpy(off).cuda(), p, R)
    tot, unf, st = tot.cpu().numpy(), unf.cpu().numpy(), st.cpu().numpy()
    otot, ounf, ost = orc.plan_fusion(p, d, e, off, R)
    fin = np.isfinite(otot)
    assert np.array_equal(np.isfinite(tot), fin) and np.array_equal(np.isfinite(unf), np.isfinite(ounf))
    assert np.all(np.abs(tot[fin] - otot[fin]) <= 1e-12 * otot[fin])
    f2 = np.isfinite(ounf)
    assert np.all(np.abs(unf[f2] - ounf[f2]) <= 1e-12 * ounf[f2])
    diff = [c for c in range(len(off) - 1) if not np.array_equal(st[off[c]:off[c + 1]], ost[off[c]:off[c + 1]])]
    for c in diff:
        a, b = off[c], off[c + 1]
        starts = list(np.flatnonzero(st[a:b])) + [b - a]
        assert starts[0] == 0
        cost = sum(orc.fused_cost(p, d, e, a + starts[k], starts[k + 1] - starts[k]) for k in range(len(starts) - 1))
        assert all(1 <= starts[k + 1] - starts[k] <= R for k in range(len(starts) - 1))
        assert abs(cost - otot[c]) <= 1e-12 * otot[c], (c, cost, otot[c])
    say("  chains with a different (tied) plan:", len(diff), "fused share", 1 - st.mean())
    assert len(diff) <= max(2, (len(off) - 1) // 1000)
    return tot, unf, st


@pytest.mark.parametrize("R", [1, 4, 8, 32])
def test_fusion_plan_parity(wmb, orc, R):
    p = synth.param_set(2)
    off, d, e = synth.chains(3000, 162)
    tot, unf, st = _check_plan(wmb, orc, p, off, d, e, R, f"R={R}")
    if R == 1:
        assert np.array_equal(tot, unf) and st.all()


def test_fusion_edge_cases(wmb, orc):
    p = synth.param_set(3, n_levels=3, combine=1)
    off, d, e = synth.chains(400, 163, lmin=1, lmax=40)
    d.u[off[5] + 0] = 1.5        # an invalid row: its chain is infinite
    # empty chains inside the list
    off2 = np.concatenate([off[:10], off[9:10], off[10:]]).astype(np.int32)
    _check_plan(wmb, orc, p, off2, d, e, 8, "edges")


def test_planning_full_size(wmb, orc):
    p = synth.param_set(0)
    off, d, e = synth.chains(1 << 16, 164)
    _check_plan(wmb, orc, p, off, d, e, 8, "2^16 chains")
    off, fac, noise, train, d2 = synth.grouped_measurements(1 << 16, 172)
    T, _ = orc.predict(p, d2)
    g = np.repeat(np.arange(1 << 16), np.diff(off))
    _check_mult(wmb, orc, T, T * fac[g] * noise, off, train, "2^16 groups")
