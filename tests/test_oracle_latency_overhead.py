"""Pins of the oracle's latency stage and overhead sum against hand-worked
fixtures (tests/golden/latency_stage.txt, tests/golden/overhead_terms.txt).

Eq. (10) (N_loads times the hit-weighted latency bracket), serialised over
Eq. (14)'s workgroup rounds, and the overhead of Eq. (1) / Eq. (13) /
Eq. (14) with the interference, multi-GPU and fusion terms of Section IV-B
and the per-sync term of Section IV-E.  Every value in the fixtures is an
exact binary fraction, so the oracle must reproduce them bit for bit.

The second half plants plausible mistakes in copies of the oracle's source
(whole-grid rounds ceil(G/o), rounds without the ceiling, loads counted per
thread instead of per wave, a barrier term without the rounds, one
interference term too many) and checks that the fixtures reject each one.
"""
import os

import numpy as np
import pytest

from paper_2605_04178_amd import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
U = 2.0 ** -30          # time unit of the fixtures: one cycle at f_clk = 2^30 Hz


def _params():
    th = [0.0] * 24
    th[0], th[1], th[2], th[3] = 2.0 ** 50, 2.0 ** 49, 2.0 ** 48, 2.0 ** 48
    th[4], th[5], th[6], th[7] = 4.0, 8.0, 12.0, 16.0
    for j in range(8, 13):
        th[j] = 2.0 ** 50
    th[13], th[14], th[15] = 2.0 ** -20, 2.0 ** -30, 2.0 ** -26
    th[16], th[17], th[18], th[19] = 2.0 ** -16, 2.0 ** -15, 2.0 ** -18, 2.0 ** -19
    th[20], th[21], th[22], th[23] = 1.0, 1.0, 0.0, 2.0 ** 48
    return synth.ParamSet(n_levels=3, n_cu=4, n_simd=4, wave=64, vgpr_simd=512, vgpr_gran=8,
                          waves_simd=8, lds_cu=65536, lds_gran=512, bytes_inflight_wave=1024,
                          combine=0, f_clk=2.0 ** 30, theta=th)


def _rows(name):
    out = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                out.append(line)
    return out


def _latency_mismatches(orc, L=None):
    """Rows of latency_stage.txt whose oracle evaluation differs from the
    hand-worked values (empty when the oracle agrees bit for bit)."""
    p = _params()
    bad = []
    rows = _rows("latency_stage.txt")
    assert len(rows) == 9
    for r in rows:
        name = r[0]
        g, v, s, G = (int(x) for x in r[1:5])
        B, r1, r2 = float(r[5]), float(r[6]), float(r[7])
        k, o, n_r = (int(x) for x in r[8:11])
        n_loads, lam, t_lat, t = (float(x) for x in r[11:15])
        assert np.float32(B) == B
        gp = int(synth.pack_gpack(g, 1))
        tr = orc.eval_one(p, 0.0, B, r1, r2, 0.0, 0.0, 1.0, 0.0, v, s, gp, G, L=L)
        got = (tr.k, tr.o, tr.n_r, tr.Lam, tr.T_lat, tr.T)
        want = (k, o, n_r, lam, t_lat * U, t * U)
        if got != want:
            bad.append((name, got, want))
        # the stage that decides T is the latency stage
        if not (tr.T_lat > tr.T_b and tr.T_c == 0.0):
            bad.append((name, "latency stage not dominant", tr.T_lat, tr.T_b))
        # N_loads as a continuous count: T_lat / (n_r Lam / f)
        if tr.T_lat != n_r * n_loads * lam * U:
            bad.append((name, "N_loads", tr.T_lat / (n_r * lam * U), n_loads))
    return bad


def _overhead_mismatches(orc, L=None):
    p = _params()
    bad = []
    rows = _rows("overhead_terms.txt")
    assert len(rows) == 10
    for r in rows:
        name = r[0]
        G = int(r[1])
        K = float(r[2])
        n_conc, n_dev, fused, n_sync = (int(x) for x in r[3:7])
        coef = [float(x) for x in r[7:14]]
        t = float(r[14])
        gp = int(synth.pack_gpack(256, 1, n_conc, n_dev, fused, n_sync))
        tr, J = orc.eval_one(p, 0.0, 0.0, 0.0, 0.0, 0.0, K, 1.0, 0.0, 128, 0, gp, G, with_grad=True, L=L)
        if (tr.T_c, tr.T_b, tr.T_lat) != (0.0, 0.0, 0.0):
            bad.append((name, "stage times not zero"))
        if tr.T_ov != t * U or tr.T != t * U:
            bad.append((name, "T", tr.T_ov / U, tr.T / U, t))
        # the coefficients are the derivative of T with respect to slots 13..19
        if list(J[13:20]) != coef:
            bad.append((name, "dT/dtheta[13:20]", list(J[13:20]), coef))
        # and the sum of coefficient x parameter is T
        if sum(c * x for c, x in zip(coef, p.theta[13:20])) != t * U:
            bad.append((name, "fixture arithmetic"))
    return bad


def test_latency_stage_matches_hand_worked_rows(orc):
    assert _latency_mismatches(orc) == []


def test_overhead_sum_matches_hand_worked_rows(orc):
    assert _overhead_mismatches(orc) == []


def test_batched_predict_equals_the_rows(orc):
    """The same rows through orc_predict (the array entry point)."""
    p = _params()
    rows = _rows("latency_stage.txt")
    n = len(rows)
    d = synth.Descriptors(
        F=np.zeros(n, np.float32), B=np.array([float(r[5]) for r in rows], np.float32),
        r1=np.array([float(r[6]) for r in rows], np.float32), r2=np.array([float(r[7]) for r in rows], np.float32),
        r3=np.zeros(n, np.float32), K=np.zeros(n, np.float32), u=np.ones(n, np.float32),
        W=np.zeros(n, np.float32), vgpr=np.array([int(r[2]) for r in rows], np.int32),
        lds=np.array([int(r[3]) for r in rows], np.int32),
        gpack=synth.pack_gpack(np.array([int(r[1]) for r in rows]), 1),
        grid=np.array([int(r[4]) for r in rows], np.int32))
    T, occ = orc.predict(p, d)
    assert np.array_equal(T, np.array([float(r[14]) * U for r in rows]))
    assert np.array_equal(occ, np.array([int(r[9]) for r in rows], np.int32))


# ---------------------------------------------------------------------------
# planted mistakes: each must be caught
# ---------------------------------------------------------------------------
MUTANTS = {
    "rounds over the whole grid, ceil(G/o)":
        [("wm_oracle.c", "int64_t n_r = ceil_div(G, (int64_t)p->n_cu * o);",
          "int64_t n_r = ceil_div(G, o);")],
    "rounds without the ceiling":
        [("wm_oracle.c", "int64_t n_r = ceil_div(G, (int64_t)p->n_cu * o);",
          "int64_t n_r = G / ((int64_t)p->n_cu * o);")],
    "loads counted per thread":
        [("wm_oracle.c", "double n_loads = B / ((double)G * (double)k * (double)p->bytes_inflight_wave);",
          "double n_loads = B / ((double)G * (double)g * (double)p->bytes_inflight_wave);")],
    "barrier term without the rounds":
        [("wm_oracle.c", "+ th[S_TAU_BAR] * (double)n_r * K", "+ th[S_TAU_BAR] * K")],
    "barrier derivative without the rounds":
        [("wm_oracle.c", "dT[S_TAU_BAR] = (double)n_r * K;", "dT[S_TAU_BAR] = K;")],
    "one interference term per kernel, not per extra kernel":
        [("wm_oracle.c", "+ (double)(n_conc - 1) * th[S_TAU_INTERF]", "+ (double)n_conc * th[S_TAU_INTERF]")],
    "dispatch cost per round instead of per workgroup":
        [("wm_oracle.c", "+ th[S_TAU_WG] * (double)G", "+ th[S_TAU_WG] * (double)n_r")],
}


@pytest.mark.parametrize("what", list(MUTANTS))
def test_planted_mistake_is_caught(orc, tmp_path, what):
    from oracle import build as orc_build
    so = orc_build.build_variant(str(tmp_path / "liboracle_mutant.so"), replace=MUTANTS[what])
    L = orc.load(so)
    bad = _latency_mismatches(orc, L) + _overhead_mismatches(orc, L)
    assert bad, f"the fixtures did not catch: {what}"
