"""Pins of the oracle's workload-segment evaluation (Sections IV-E, IV-F and
V-B): an application is a list of segments, each a kernel descriptor run
n_exec times with n_kern launches per execution, a class scale on the kernel
time and optional host-device transfers (Eq. (15)).

The checks use the paper's printed defaults (tests/golden/memcpy_eq15.txt),
reduction to the single-kernel model, exact linearity and additivity, the
invalid / infeasible / empty cases, and central finite differences of the
application-level loss.  CPU only.
"""
import dataclasses
import os

import numpy as np
import pytest

from paper_2605_04178_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _sub(sg, d, idx):
    """Segments idx (in that order) as one application each."""
    idx = np.asarray(idx)
    s2 = synth.Segments(np.arange(len(idx) + 1, dtype=np.int32), sg.n_exec[idx].copy(),
                        sg.n_kern[idx].copy(), sg.cls[idx].copy(), sg.h2d[idx].copy(),
                        sg.d2h[idx].copy())
    d2 = synth.Descriptors(*[getattr(d, f.name)[idx].copy() for f in dataclasses.fields(d)])
    return s2, d2


def _plain(n):
    return synth.Segments(np.arange(n + 1, dtype=np.int32), np.ones(n, np.float32),
                          np.ones(n, np.int32), np.zeros(n, np.int32), np.zeros(n, np.float32),
                          np.zeros(n, np.float32))


@pytest.fixture(scope="module")
def case():
    p = synth.param_set(0)
    q = synth.seg_params(7)
    sg, d = synth.segments(400, 120)
    return p, q, sg, d


def test_single_plain_segment_is_the_kernel_model(orc, case):
    p, q, _, _ = case
    d = synth.descriptors(3000, 5)
    Tk, _ = orc.predict(p, d)
    q1 = synth.SegParams()
    Ta, Ts = orc.predict_apps(p, q1, d, _plain(d.F.shape[0]))
    same = np.isfinite(Tk)
    assert same.mean() > 0.5
    assert np.array_equal(Ta[same], Tk[same]) and np.array_equal(Ts[same], Tk[same])
    assert np.array_equal(np.isnan(Ta), np.isnan(Tk)) and np.array_equal(np.isinf(Ta), np.isinf(Tk))


def test_memcpy_term_matches_eq15_defaults(orc, case):
    p, _, sg, d = case
    q = synth.SegParams()          # 45 GB/s each way, 2 us per episode
    rows = [[float(x) for x in l.split()] for l in open(os.path.join(GOLD, "memcpy_eq15.txt"))
            if l.split("#")[0].strip()]
    s1, d1 = _sub(sg, d, [0])
    s1.h2d[:] = 0
    s1.d2h[:] = 0
    s1.n_exec[:] = 3
    base, _ = orc.predict_apps(p, q, d1, s1)
    for S, bw, tau, want in rows:
        assert bw == q.bw_h2d and tau == q.tau_memcpy
        for field in ("h2d", "d2h"):
            s2 = dataclasses.replace(s1, **{field: np.array([S], np.float32)})
            T, _ = orc.predict_apps(p, q, d1, s2)
            got = (T[0] - base[0]) / 3.0
            assert abs(got - want) <= 1e-9 * want + 1e-12 * base[0], (field, S, got, want)
        # both directions: two episodes
        s3 = dataclasses.replace(s1, h2d=np.array([S], np.float32), d2h=np.array([S], np.float32))
        T, _ = orc.predict_apps(p, q, d1, s3)
        assert abs((T[0] - base[0]) / 3.0 - 2 * want) <= 2e-9 * want + 1e-12 * base[0]


def test_extra_launches_cost_t_launch_each(orc, case):
    p, q, sg, d = case
    s1, d1 = _sub(sg, d, np.arange(50))
    s1.n_kern[:] = 1
    T1, _ = orc.predict_apps(p, q, d1, s1)
    for nk in (2, 4, 9):
        s2 = dataclasses.replace(s1, n_kern=np.full(50, nk, np.int32))
        T2, _ = orc.predict_apps(p, q, d1, s2)
        want = s1.n_exec.astype(np.float64) * (nk - 1) * p.theta[13]
        assert np.allclose(T2 - T1, want, rtol=1e-9, atol=1e-12 * T1.max())


def test_class_scale_multiplies_the_kernel_time_only(orc, case):
    p, q, sg, d = case
    s1, d1 = _sub(sg, d, np.arange(80))
    q0 = synth.SegParams(kappa=[1.0] * 4, bw_h2d=q.bw_h2d, bw_d2h=q.bw_d2h, tau_memcpy=q.tau_memcpy)
    T0, _ = orc.predict_apps(p, q0, d1, s1)
    Tk, _ = orc.predict(p, d1)
    ne = s1.n_exec.astype(np.float64)
    for c in range(4):
        kap = [1.0] * 4
        kap[c] = 2.5
        qc = dataclasses.replace(q0, kappa=kap)
        Tc, _ = orc.predict_apps(p, qc, d1, s1)
        want = np.where(s1.cls == c, 1.5 * ne * Tk, 0.0)
        assert np.allclose(Tc - T0, want, rtol=1e-9, atol=1e-12 * T0.max())


def test_linear_in_executions_and_zero_executions(orc, case):
    p, q, sg, d = case
    s1, d1 = _sub(sg, d, np.arange(60))
    s1.n_exec[:] = 1
    T1, _ = orc.predict_apps(p, q, d1, s1)
    for k in (0, 7, 1000):
        s2 = dataclasses.replace(s1, n_exec=np.full(60, k, np.float32))
        T2, _ = orc.predict_apps(p, q, d1, s2)
        assert np.allclose(T2, k * T1, rtol=1e-12, atol=0)
    assert np.all(T1 > 0)


def test_applications_add_and_ignore_segment_order(orc, case):
    p, q, sg, d = case
    Ta, Ts = orc.predict_apps(p, q, d, sg)
    # every application total equals the sum of its segments taken one per application
    s1, d1 = _sub(sg, d, np.arange(sg.app_off[-1]))
    T1, _ = orc.predict_apps(p, q, d1, s1)
    sums = np.array([T1[sg.app_off[a]:sg.app_off[a + 1]].sum() for a in range(sg.n_apps)])
    assert np.allclose(Ta, sums, rtol=1e-13, atol=0)
    assert np.array_equal(Ts, T1)
    # reverse the segments inside each application
    perm = np.concatenate([np.arange(sg.app_off[a + 1] - 1, sg.app_off[a] - 1, -1)
                           for a in range(sg.n_apps)])
    sr, dr = _sub(sg, d, perm)
    sr = dataclasses.replace(sr, app_off=sg.app_off.copy())
    Tr, _ = orc.predict_apps(p, q, dr, sr)
    assert np.allclose(Tr, Ta, rtol=1e-13, atol=0)
    # merge applications pairwise: totals add
    off2 = sg.app_off[::2].copy()
    if off2[-1] != sg.app_off[-1]:
        off2 = np.append(off2, sg.app_off[-1])
    Tm, _ = orc.predict_apps(p, q, d, dataclasses.replace(sg, app_off=off2.astype(np.int32)))
    pair = np.array([Ta[2 * k:2 * k + 2].sum() for k in range(len(off2) - 1)])
    assert np.allclose(Tm, pair, rtol=1e-13, atol=0)


def test_invalid_infeasible_and_empty(orc, case):
    p, q, sg, d = case
    s1, d1 = _sub(sg, d, np.arange(8))
    s1 = dataclasses.replace(s1, app_off=np.array([0, 2, 2, 4, 6, 8], np.int32))
    s1.cls[0] = 4          # app 0: bad class
    s1.n_kern[2] = 0       # app 2: no kernel
    s1.h2d[5] = np.nan     # app 3: bad transfer size
    d1.vgpr[6] = 4096      # app 4: a kernel that cannot be resident
    d1.gpack[6] = int(synth.pack_gpack(1024, 1, 1, 1, 0, 0))
    Ta, Ts = orc.predict_apps(p, q, d1, s1)
    assert np.isnan(Ta[0]) and Ta[1] == 0.0 and np.isnan(Ta[2]) and np.isnan(Ta[3])
    assert np.isinf(Ta[4]) and Ta[4] > 0
    assert np.isnan(Ts[0]) and np.isinf(Ts[6])
    for bad in (dict(n_exec=np.float32(-1)), dict(d2h=np.float32(-5)), dict(cls=np.int32(-1))):
        s2 = dataclasses.replace(s1, **{k: getattr(s1, k).copy() for k in bad})
        for k, v in bad.items():
            getattr(s2, k)[7] = v
        T2, _ = orc.predict_apps(p, q, d1, s2)
        assert np.isnan(T2[4])


def _finite_sign_stable(orc, p, q, d, sg, m, rel):
    Ta, _ = orc.predict_apps(p, q, d, sg)
    return np.isfinite(Ta) & (np.abs(Ta / m - 1) > rel)


def test_app_loss_gradient_matches_central_differences(orc):
    p = synth.param_set(2)
    q = synth.seg_params(9)
    sg, d = synth.segments(300, 130)
    Ta, _ = orc.predict_apps(p, q, d, sg)
    m = Ta * synth.lognormal_noise(sg.n_apps, 131, 0.1)
    loss, cnt, gth, gsp = orc.apps_loss_grad(p, q, d, sg, m)
    ok = np.isfinite(Ta)
    assert cnt == ok.sum()
    assert abs(loss - np.mean(np.abs(Ta[ok] - m[ok]) / m[ok])) <= 1e-13 * loss

    def L(th=None, qq=None):
        pp = p if th is None else p.copy(theta=list(th))
        return orc.apps_loss_grad(pp, qq or q, d, sg, m)[0]

    h = 1e-6
    th0 = np.array(p.theta)
    used = [j for j in range(24) if abs(gth[j]) * th0[j] > 1e-9 * loss]
    assert len(used) >= 12
    for j in used:
        tp, tm = th0.copy(), th0.copy()
        tp[j] *= 1 + h
        tm[j] *= 1 - h
        fd = (L(tp) - L(tm)) / (2 * h * th0[j])
        assert abs(fd - gth[j]) <= 2e-4 * abs(gth[j]) + 1e-6 * loss / th0[j], (j, fd, gth[j])
    names = ("kappa0", "kappa1", "kappa2", "kappa3", "bw_h2d", "bw_d2h", "tau_memcpy")
    vals = list(q.kappa) + [q.bw_h2d, q.bw_d2h, q.tau_memcpy]
    for j, nm in enumerate(names):
        def qq(v):
            x = list(vals)
            x[j] = v
            return synth.SegParams(kappa=x[:4], bw_h2d=x[4], bw_d2h=x[5], tau_memcpy=x[6])
        fd = (L(qq=qq(vals[j] * (1 + h))) - L(qq=qq(vals[j] * (1 - h)))) / (2 * h * vals[j])
        assert abs(gsp[j]) > 0, nm
        assert abs(fd - gsp[j]) <= 2e-4 * abs(gsp[j]), (nm, fd, gsp[j])


def test_app_loss_skips_nonfinite_and_bad_measurements(orc, case):
    p, q, sg, d = case
    Ta, _ = orc.predict_apps(p, q, d, sg)
    m = Ta * 1.1
    m[:5] = [0.0, -1.0, np.nan, np.inf, m[4]]
    loss, cnt, _, _ = orc.apps_loss_grad(p, q, d, sg, m)
    assert cnt == sg.n_apps - 4
    assert abs(loss - 0.1 / 1.1) <= 1e-12


def test_app_vjp_matches_finite_differences(orc):
    p = synth.param_set(3)
    q = synth.seg_params(10)
    sg, d = synth.segments(200, 132)
    Ta, _ = orc.predict_apps(p, q, d, sg)
    w = np.random.default_rng(4).standard_normal(sg.n_apps)
    gth, gsp = orc.apps_vjp(p, q, d, sg, w)
    ok = np.isfinite(Ta)

    def F(pp=None, qq=None):
        T, _ = orc.predict_apps(pp or p, qq or q, d, sg)
        return float(np.sum(w[ok] * T[ok]))
    h = 1e-6
    th0 = np.array(p.theta)
    tr = orc.trace(p, d)
    for j in range(24):
        if gth[j] == 0.0:
            continue
        tp, tm = th0.copy(), th0.copy()
        tp[j] *= 1 + h
        tm[j] *= 1 - h
        fd = (F(pp=p.copy(theta=list(tp))) - F(pp=p.copy(theta=list(tm)))) / (2 * h * th0[j])
        scale = np.sum(np.abs(w[ok] * Ta[ok])) / th0[j]
        assert abs(fd - gth[j]) <= 1e-4 * abs(gth[j]) + 1e-7 * scale, (j, fd, gth[j])
    vals = list(q.kappa) + [q.bw_h2d, q.bw_d2h, q.tau_memcpy]
    for j in range(7):
        def qq(v):
            x = list(vals)
            x[j] = v
            return synth.SegParams(kappa=x[:4], bw_h2d=x[4], bw_d2h=x[5], tau_memcpy=x[6])
        # T is linear in kappa and tau (large steps are exact), smooth in 1/B
        hs = 1e-4 if j in (4, 5) else 1e-2
        fd = (F(qq=qq(vals[j] * (1 + hs))) - F(qq=qq(vals[j] * (1 - hs)))) / (2 * hs * vals[j])
        assert abs(fd - gsp[j]) <= 1e-6 * abs(gsp[j]) + 1e-12, (j, fd, gsp[j])
