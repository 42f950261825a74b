"""Pins of the oracle's per-group calibration multipliers and kernel-fusion
planner: closed forms, brute force over every candidate multiplier and every
segmentation of small chains, invariances and degenerate cases.  CPU only."""
import itertools

import numpy as np
import pytest

from paper_2605_04178_amd import synth


def _obj(mu, T, m):
    return float(np.sum(np.abs(mu * T - m) / m))


# ---------------------------------------------------------------- multipliers
def test_single_row_and_equal_ratios(orc):
    mult, Ts, st = orc.fit_multipliers([2.0], [3.0], [0, 1], [1])
    assert mult[0] == 1.5 and Ts[0] == 3.0 and st == (0.0, 1.0, 0.0, 0.0)
    T = np.array([1.0, 2.0, 4.0, 8.0])
    mult, Ts, st = orc.fit_multipliers(T, 1.25 * T, [0, 4], [1, 1, 1, 1])
    assert mult[0] == 1.25 and st[0] == 0.0


def test_weighted_median_minimises_training_error_brute_force(orc):
    rng = np.random.default_rng(0)
    for trial in range(300):
        k = int(rng.integers(1, 9))
        T = rng.uniform(0.1, 10.0, k)
        m = T * np.exp(rng.normal(0, 0.5, k))
        if trial % 5 == 0:                      # exact ties in the ratios
            m[: k // 2] = 2.0 * T[: k // 2]
        mult, _, _ = orc.fit_multipliers(T, m, [0, k], np.ones(k, np.uint8))
        mu = mult[0]
        cands = m / T
        best = min(_obj(c, T, m) for c in cands)
        assert _obj(mu, T, m) <= best * (1 + 1e-12) + 1e-15
        # the smallest minimiser among the candidates
        minimisers = [c for c in cands if _obj(c, T, m) <= best * (1 + 1e-12) + 1e-15]
        assert mu == min(minimisers)
        # and no point between candidates does better
        for z in rng.uniform(cands.min() * 0.5, cands.max() * 1.5, 20):
            assert _obj(mu, T, m) <= _obj(z, T, m) * (1 + 1e-12) + 1e-15


def test_scaling_holdout_and_empty_groups(orc):
    rng = np.random.default_rng(1)
    T = rng.uniform(1, 5, 12)
    m = T * rng.uniform(0.5, 2.0, 12)
    off = [0, 5, 5, 12]
    train = np.array([1, 1, 0, 1, 1, 0, 0, 0, 0, 0, 0, 0], np.uint8)
    mult, Ts, st = orc.fit_multipliers(T, m, off, train)
    mult2, _, _ = orc.fit_multipliers(3.0 * T, m, off, train)
    assert abs(mult2[0] - mult[0] / 3.0) <= 1e-14 * mult2[0] and mult2[1] == 1.0
    # group 1 has no rows, group 2 no training rows: multiplier 1
    assert mult[1] == 1.0 and mult[2] == 1.0
    assert np.array_equal(Ts[5:], T[5:])
    assert st[1] == 4 and st[3] == 8
    hold = np.sum(np.abs(Ts[train == 0] - m[train == 0]) / m[train == 0])
    assert abs(st[2] - hold) <= 1e-12 * hold


def test_invalid_rows_are_skipped(orc):
    T = np.array([1.0, np.nan, np.inf, 2.0, 0.0, 1.0])
    m = np.array([2.0, 1.0, 1.0, 4.0, 1.0, -1.0])
    mult, Ts, st = orc.fit_multipliers(T, m, [0, 6], np.ones(6, np.uint8))
    assert mult[0] == 2.0 and st[1] == 2


def test_planted_factors_recovered_without_noise(orc):
    p = synth.param_set(0)
    off, fac, noise, train, d = synth.grouped_measurements(60, sigma=0.0)
    T, _ = orc.predict(p, d)
    g = np.repeat(np.arange(60), np.diff(off))
    mult, _, st = orc.fit_multipliers(T, T * fac[g], off, train)
    has = np.array([np.any(train[off[i]:off[i + 1]].astype(bool) & np.isfinite(T[off[i]:off[i + 1]]))
                    for i in range(60)])
    assert has.sum() > 40
    assert np.allclose(mult[has], fac[has], rtol=1e-13)
    assert st[0] < 1e-12 * st[1]
    # held-out rows of groups with training data are predicted exactly too
    m = T * fac[g]
    _, Ts, _ = orc.fit_multipliers(T, m, off, train)
    sel = has[g] & (train == 0) & np.isfinite(T)
    assert sel.sum() > 100 and np.allclose(Ts[sel], m[sel], rtol=1e-12)


# ---------------------------------------------------------------- fusion
def _two(F=(1e9, 2e9), B=(1e8, 3e8), r1=(0.2, 0.4), K=(3, 5), u=(0.5, 0.8), W=(0.0, 0.0),
         dt=(1, 1), g=(256, 128), v=(32, 64), s=(0, 4096), G=(100, 50), ns=(1, 2)):
    gp = synth.pack_gpack(np.array(g), np.array(dt), np.ones(2, np.int64), np.ones(2, np.int64),
                          np.zeros(2, np.int64), np.array(ns))
    f32 = np.float32
    return synth.Descriptors(F=np.array(F, f32), B=np.array(B, f32), r1=np.array(r1, f32),
                             r2=np.zeros(2, f32), r3=np.array([0.5, 0.25], f32), K=np.array(K, f32),
                             u=np.array(u, f32), W=np.array(W, f32), vgpr=np.array(v, np.int32),
                             lds=np.array(s, np.int32), gpack=gp.astype(np.int32), grid=np.array(G, np.int32))


def test_fuse_single_row_is_the_row(orc):
    p = synth.param_set(0)
    off, d, e = synth.chains(20)
    T, _ = orc.predict(p, d)
    for i in range(0, off[-1], 7):
        ok, f = orc.fuse(p, d, e, i, 1)
        assert ok and f["F"] == float(d.F[i]) and f["gpack"] == int(d.gpack[i])
        c = orc.fused_cost(p, d, e, i, 1)
        assert (c == T[i]) or (np.isnan(c) and np.isnan(T[i]))


def test_fuse_combination_rule_by_hand(orc):
    p = synth.param_set(0)
    d = _two()
    e = np.array([5e7, 0.0], np.float32)
    ok, f = orc.fuse(p, d, e, 0, 2)
    assert ok
    assert f["F"] == 3e9 and f["B"] == 4e8 - 1e8
    assert abs(f["r1"] - (0.2 * 1e8 + 0.4 * 3e8) / 4e8) < 1e-7
    assert abs(f["r3"] - (0.5 * 1e8 + 0.25 * 3e8) / 4e8) < 1e-9
    assert f["K"] == 8 and f["W"] == 0.0
    assert f["v"] == 64 and f["s"] == 4096 and f["G"] == 100
    # compute time is preserved: F / (u P) = sum F_k / (u_k P)
    assert abs(f["u"] - 3e9 / (1e9 / 0.5 + 2e9 / float(np.float32(0.8)))) < 1e-12
    gp = int(synth.pack_gpack(256, 1, 1, 1, 1, 3))
    assert f["gpack"] == gp
    # mixed dtypes: the larger-flop row's dtype; u capped at 1
    d2 = _two(dt=(0, 2), F=(1e9, 4e9))
    ok, f2 = orc.fuse(p, d2, e, 0, 2)
    P = p.theta
    u0, u1 = float(np.float32(0.5)), float(np.float32(0.8))
    want = min(1.0, 5e9 / (P[10] * (1e9 / (u0 * P[8]) + 4e9 / (u1 * P[10]))))
    assert (f2["gpack"] >> 11) & 7 == 2 and abs(f2["u"] - want) < 1e-12
    # intermediate bytes larger than the traffic: clipped at zero
    ok, f3 = orc.fuse(p, d, np.array([1e9, 0], np.float32), 0, 2)
    assert f3["B"] == 0.0
    # invalid edge or row
    assert not orc.fuse(p, d, np.array([-1.0, 0], np.float32), 0, 2)[0]
    d.u[1] = 0.0
    assert not orc.fuse(p, d, e, 0, 2)[0]


def _all_plans(n, R):
    for cuts in itertools.product([0, 1], repeat=n - 1):
        runs, start = [], 0
        for i, c in enumerate(cuts):
            if c:
                runs.append((start, i + 1 - start))
                start = i + 1
        runs.append((start, n - start))
        if all(L <= R for _, L in runs):
            yield runs


@pytest.mark.parametrize("R", [1, 2, 3, 8])
def test_plan_is_optimal_by_brute_force(orc, R):
    p = synth.param_set(1)
    off, d, e = synth.chains(40, seed=161, lmin=1, lmax=9)
    tot, unf, st = orc.plan_fusion(p, d, e, off, R)
    for c in range(40):
        a, b = off[c], off[c + 1]
        n = b - a
        costs = {}
        def cost(s, L):
            if (s, L) not in costs:
                t = orc.fused_cost(p, d, e, a + s, L)
                costs[(s, L)] = np.inf if np.isnan(t) else t
            return costs[(s, L)]
        best = min(sum(cost(s, L) for s, L in runs) for runs in _all_plans(n, R))
        assert (tot[c] == best) or abs(tot[c] - best) <= 1e-12 * best
        single = sum(cost(s, 1) for s in range(n))
        assert unf[c] == single or abs(unf[c] - single) <= 1e-12 * single
        # the reported plan is valid and costs the total
        starts = list(np.flatnonzero(st[a:b])) + [n]
        assert starts[0] == 0
        runs = [(starts[k], starts[k + 1] - starts[k]) for k in range(len(starts) - 1)]
        assert all(1 <= L <= R for _, L in runs)
        got = sum(cost(s, L) for s, L in runs)
        assert got == tot[c] or abs(got - tot[c]) <= 1e-12 * tot[c]
        if R == 1:
            assert tot[c] == unf[c] and st[a:b].all()


def test_launch_bound_pair_fuses_exactly_when_cheaper(orc):
    base = synth.param_set(0)
    th = list(base.theta)
    for j in range(14, 20):
        th[j] = 0.0
    th[13] = 5e-6
    d = _two(F=(0.0, 0.0), B=(64.0, 64.0), K=(1, 1), G=(1, 1), ns=(0, 0))
    e = np.zeros(2, np.float32)
    for tau_f, fused in ((1e-6, True), (9e-6, False)):
        th[18] = tau_f
        p = base.copy(theta=th)
        tot, unf, st = orc.plan_fusion(p, d, e, [0, 2], 2)
        assert list(st) == ([1, 0] if fused else [1, 1])
        singles = orc.fused_cost(p, d, e, 0, 1) + orc.fused_cost(p, d, e, 1, 1)
        assert unf[0] == singles
        assert tot[0] == (orc.fused_cost(p, d, e, 0, 2) if fused else singles)


def test_invalid_row_makes_the_chain_infinite(orc):
    p = synth.param_set(0)
    off, d, e = synth.chains(5, lmin=3, lmax=3)
    d.u[4] = 2.0
    tot, unf, st = orc.plan_fusion(p, d, e, off, 4)
    assert np.isinf(tot[1]) and np.isfinite(tot[0]) and np.isinf(unf[1])
