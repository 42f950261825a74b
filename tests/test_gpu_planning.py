"""Parity of per-group calibration multipliers (wm_fit_multipliers) and
fusion planning (wm_plan_fusion) with the FP64 oracle.  The optimal
objective values are unique and compared to rounding; where the oracle and
the GPU pick different multipliers or plans, the objective of the GPU's
choice must equal the optimum (a tie).

Fusion-plan costs are evaluated in float32 on the GPU, so plan totals
follow the oracle to the model's 1e-5 relative tolerance; chains with a
decision closer than the float32 error could settle are redone in float64,
so the plans themselves (the start flags) match the oracle's except at its
own ties, and the totals of those chains match to 1e-12."""
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


def test_multipliers_group_size_limits(wmb, orc):
    # sizes at the limits of each form: pairs of groups of at most 32 rows
    # (wave halves), one group of 33-64 rows per wave, the candidate scan
    # above 64 rows, pairs mixing them, an empty group, and an odd group
    # count (the last wave's upper half has no group); exact ratio ties and
    # invalid rows inside the sorted groups
    rng = np.random.default_rng(11)
    sizes = [32, 32, 33, 1, 64, 0, 65, 64, 31, 32, 17, 64, 64, 2, 40, 40, 129]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    n = int(off[-1])
    T = rng.uniform(1e-5, 1e-2, n)
    m = T * rng.choice([0.5, 0.8, 1.0, 1.25, 2.0], n)        # many equal ratios
    m[off[10]:off[11]] = T[off[10]:off[11]] * rng.uniform(0.5, 2.0, sizes[10])
    train = (rng.random(n) < 0.75).astype(np.uint8)
    T[off[4] + 3] = np.nan
    m[off[7] + 63] = 0.0
    T[off[0] + 31] = np.inf
    _check_mult(wmb, orc, T, m, off, train, "size limits")


# plan totals and all-singles sums: float32 run costs (the model's prediction
# tolerance), summed in float64
PLAN_RTOL = 1e-5


def _check_plan(wmb, orc, p, off, d, e, R, tag):
    say("fusion", tag, "chains", len(off) - 1, "rows", off[-1], "R", R)
    dd = wmb.DeviceDescriptors.from_host(d)
    tot, unf, st = wmb.plan_fusion(dd, torch.from_numpy(e).cuda(), torch.from_numpy(off).cuda(), p, R)
    tot, unf, st = tot.cpu().numpy(), unf.cpu().numpy(), st.cpu().numpy()
    otot, ounf, ost = orc.plan_fusion(p, d, e, off, R)
    fin = np.isfinite(otot)
    assert np.array_equal(np.isfinite(tot), fin) and np.array_equal(np.isfinite(unf), np.isfinite(ounf))
    assert np.all(np.abs(tot[fin] - otot[fin]) <= PLAN_RTOL * otot[fin])
    f2 = np.isfinite(ounf)
    assert np.all(np.abs(unf[f2] - ounf[f2]) <= PLAN_RTOL * ounf[f2])
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


@pytest.mark.parametrize("R", [1, 3, 4, 6, 8, 32])
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


def _near_tie_chains(n, seed):
    """Chains of three kernels A, B, A' with A' a copy of A whose bytes differ
    by up to 3e-5 relative and with equal edges A->B and B->A': where fusing
    A with B pays, the plans AB|A' and A|BA' cost nearly the same."""
    off, d, e = synth.chains(n, seed, lmin=3, lmax=3)
    rng = np.random.default_rng(seed)
    a = off[:-1].astype(np.int64)
    for arr in d.fields():
        arr[a + 2] = arr[a]
    d.B[a + 2] = (d.B[a].astype(np.float64) * (1.0 + rng.uniform(-3e-5, 3e-5, n))).astype(np.float32)
    e[a + 1] = e[a]
    return off, d, e


def test_fusion_near_ties_follow_float64(wmb, orc):
    # decisions within float32's reach but settled in float64: the plan must
    # be the oracle's, and the chain's total its float64 value
    p = synth.param_set(2)
    n = 2000
    off, d, e = _near_tie_chains(n, 901)
    T, _ = orc.predict(p, d)
    a = off[:-1].astype(np.int64)
    margin = np.full(n, np.nan)
    for c in range(n):
        s = int(a[c])
        f1 = orc.fused_cost(p, d, e, s, 2)
        if f1 < T[s] + T[s + 1]:
            v1, v2 = f1 + T[s + 2], T[s] + orc.fused_cost(p, d, e, s + 1, 2)
            margin[c] = abs(v1 - v2) / v2
    near = np.flatnonzero((margin > 1e-10) & (margin < 2e-5))
    # well within the window (float32 moves a margin by a few per cent of
    # 1e-5 at most): redone in float64
    inside = near[margin[near] < 0.9e-5]
    say("near-tie chains", len(near), "below 1e-7:", int(np.sum(margin[near] < 1e-7)),
        "inside the window:", len(inside))
    assert len(near) >= 100 and len(inside) >= 50
    tot, unf, st = _check_plan(wmb, orc, p, off, d, e, 2, "near ties")
    # every one of them went through the float64 redo
    ws = wmb._workspace(wmb.plan_workspace_bytes(d.n, 2), "cuda")
    wmb.plan_fusion(wmb.DeviceDescriptors.from_host(d), torch.from_numpy(e).cuda(),
                    torch.from_numpy(off).cuda(), p, 2, ws=ws)
    redone = wmb.plan_redone(ws)
    say("  chains redone in float64:", redone)
    assert redone >= len(inside)
    otot, _, ost = orc.plan_fusion(p, d, e, off, 2)
    for c in near:   # inside the window by the float64 redo, beyond it in float32
        assert np.array_equal(st[a[c]:a[c] + 3], ost[a[c]:a[c] + 3]), (c, margin[c])
    assert np.all(np.abs(tot[inside] - otot[inside]) <= 1e-12 * otot[inside])


def test_fusion_float32_cost_error_bounds_the_window(wmb, orc):
    # A plan decision compares two sums of run costs, each off by at most the
    # float32 model's relative error e, so it can only flip when the
    # runner-up is within 2e; decisions within 1e-5 are redone in float64.
    # Measure e on the run costs themselves (the workspace starts with the
    # n x R float64 cost array; chains redone in float64 hold float64 costs)
    # and require 1e-5 >= 4 x 2e.
    p = synth.param_set(0)
    off, d, e = synth.chains(4000, 168)
    R = 8
    ws = wmb._workspace(wmb.plan_workspace_bytes(d.n, R), "cuda")
    wmb.plan_fusion(wmb.DeviceDescriptors.from_host(d), torch.from_numpy(e).cuda(),
                    torch.from_numpy(off).cuda(), p, R, ws=ws)
    cost = ws[:8 * d.n * R].cpu().numpy().view(np.float64).reshape(d.n, R)
    err = []
    for c in range(0, 4000, 8):
        a, b = int(off[c]), int(off[c + 1])
        for j in range(b - a):
            for ln in range(1, min(R, j + 1) + 1):
                t = orc.fused_cost(p, d, e, a + j - ln + 1, ln)
                if np.isfinite(t) and t > 0:
                    err.append(abs(cost[a + j, ln - 1] - t) / t)
    err = np.array(err)
    say("fused-run costs checked", len(err), "max float32 relative error", err.max())
    assert len(err) > 5000
    assert 4 * 2 * err.max() <= 1e-5


def test_fusion_uncertain_runs_are_redone(wmb, orc):
    # Pairs whose fused run float32 cannot carry: (a) working sets summing to
    # just above the LLC capacity (2^28 B = 256 MiB): float64 sees W > C and
    # the streaming regime of Table "hlcc-piecewise", while float32 rounds
    # 2^28 + 16 down to 2^28, the transition regime with a hit rate of 0;
    # (b) flops that add up past the float32 range.  Both kinds must be
    # redone in float64, totals to 1e-12.  Plans: the oracle's for (a); for
    # (b) the run times dwarf every overhead, so fusing costs the unfused sum
    # to the last bit (float64 ties), and a plan that differs must cost the
    # optimum.
    p = synth.param_set(0)
    assert p.n_levels == 4 and p.c_llc_mib == 256.0
    n = 400
    off, d, e = synth.chains(n, 169, lmin=2, lmax=2)
    a = off[:-1].astype(np.int64)
    llc, big = a[: n // 2], a[n // 2:]
    d.W[llc] = np.float32(2 ** 27)
    d.W[llc + 1] = np.float32(2 ** 27 + 16)
    e[llc] = 0.0
    d.F[big] = np.float32(3e38)
    d.F[big + 1] = np.float32(3e38)
    ws = wmb._workspace(wmb.plan_workspace_bytes(d.n, 2), "cuda")
    tot, unf, st = wmb.plan_fusion(wmb.DeviceDescriptors.from_host(d), torch.from_numpy(e).cuda(),
                                   torch.from_numpy(off).cuda(), p, 2, ws=ws)
    tot, st = tot.cpu().numpy(), st.cpu().numpy()
    otot, _, ost = orc.plan_fusion(p, d, e, off, 2)
    redone = wmb.plan_redone(ws)
    say("uncertain-run chains", n, "redone", redone, "fused", int(n * 2 - st.sum()))
    assert redone >= n
    assert np.all(np.isfinite(otot)) and np.all(np.abs(tot - otot) <= 1e-12 * otot)
    nl = 2 * (n // 2)
    assert np.array_equal(st[:nl], ost[:nl])
    for c in range(n // 2, n):
        s0 = int(a[c])
        if np.array_equal(st[s0:s0 + 2], ost[s0:s0 + 2]):
            continue
        cost = (orc.fused_cost(p, d, e, s0, 2) if st[s0 + 1] == 0 else
                orc.fused_cost(p, d, e, s0, 1) + orc.fused_cost(p, d, e, s0 + 1, 1))
        assert abs(cost - otot[c]) <= 1e-12 * otot[c], (c, cost, otot[c])


def test_fusion_offsets_not_non_decreasing(wmb, orc):
    # chain 2 starts inside chain 0: its rows were costed as chain 0's, so it
    # reports NaN; chain 0 is planned as usual and chain 1 is empty
    p = synth.param_set(2)
    _, d, e = synth.chains(4, 166, lmin=5, lmax=5)
    off = np.array([0, 10, 5, 20], np.int32)
    dd = wmb.DeviceDescriptors.from_host(d)
    tot, unf, st = wmb.plan_fusion(dd, torch.from_numpy(e).cuda(), torch.from_numpy(off).cuda(), p, 8)
    tot, unf = tot.cpu().numpy(), unf.cpu().numpy()
    otot, ounf, _ = orc.plan_fusion(p, d, e, np.array([0, 10], np.int32), 8)
    assert abs(tot[0] - otot[0]) <= PLAN_RTOL * otot[0] and abs(unf[0] - ounf[0]) <= PLAN_RTOL * ounf[0]
    assert tot[1] == 0.0 and unf[1] == 0.0
    assert np.isnan(tot[2]) and np.isnan(unf[2])
    # no rows at all: every chain is empty
    dz = wmb.DeviceDescriptors.from_host(d.slice(0, 0))
    tot, unf, _ = wmb.plan_fusion(dz, torch.zeros(0, device="cuda"),
                                  torch.zeros(3, dtype=torch.int32, device="cuda"), p, 8)
    assert np.array_equal(tot.cpu().numpy(), np.zeros(2)) and np.array_equal(unf.cpu().numpy(), np.zeros(2))


def test_planning_full_size(wmb, orc):
    p = synth.param_set(0)
    off, d, e = synth.chains(1 << 16, 164)
    _check_plan(wmb, orc, p, off, d, e, 8, "2^16 chains")
    off, fac, noise, train, d2 = synth.grouped_measurements(1 << 16, 172)
    T, _ = orc.predict(p, d2)
    g = np.repeat(np.arange(1 << 16), np.diff(off))
    _check_mult(wmb, orc, T, T * fac[g] * noise, off, train, "2^16 groups")
