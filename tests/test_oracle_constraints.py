"""Pins of the oracle's calibration constraints (boxes on fitted slots and
the level orderings of the cache bandwidths and latencies): the isotonic fit
against scikit-learn's and against the min-max formula written out here,
and constrained calibrations against what projected Adam must give."""
import itertools

import numpy as np
import pytest
from sklearn.isotonic import IsotonicRegression

from paper_2605_04178_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def minmax_isotonic(y):
    """Non-decreasing least-squares fit: element i is the max over a <= i of
    the min over b >= i of the mean of y[a..b]."""
    n = len(y)
    return np.array([max(min(np.mean(y[a:b + 1]) for b in range(i, n)) for a in range(i + 1))
                     for i in range(n)])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_isotonic_matches_sklearn_and_minmax(orc, n):
    rng = np.random.default_rng(n)
    for _ in range(50):
        y = rng.standard_normal(n) * rng.choice([1e-3, 1.0, 30.0])
        a = orc.isotonic_inc(y)
        ref = IsotonicRegression().fit_transform(np.arange(n), y)
        assert np.allclose(a, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(y).max()))
        assert np.allclose(a, minmax_isotonic(y), rtol=0, atol=1e-12 * max(1.0, np.abs(y).max()))
        assert np.all(np.diff(a) >= -1e-15)
        assert np.sum(a) == pytest.approx(np.sum(y), abs=1e-12 * max(1.0, np.abs(y).sum()))


def test_isotonic_keeps_ordered_input_and_pools_ties(orc):
    assert np.array_equal(orc.isotonic_inc([1.0, 2.0, 2.0, 5.0]), [1.0, 2.0, 2.0, 5.0])
    assert np.array_equal(orc.isotonic_inc([3.0, 1.0]), [2.0, 2.0])
    assert np.array_equal(orc.isotonic_inc([4.0, 3.0, 2.0, 1.0]), [2.5, 2.5, 2.5, 2.5])
    assert np.array_equal(orc.isotonic_inc([1.0, 3.0, 2.0, 4.0]), [1.0, 2.5, 2.5, 4.0])


MASK = synth.FIT_MASK_L4


def _problem(orc, n=1 << 13, sigma=0.02):
    ps = synth.param_set(1, n_levels=4)
    d = synth.calibration_descriptors(n, 103)
    T, _ = orc.predict(ps, d)
    m = (T * synth.lognormal_noise(n, 2, sigma)).astype(np.float32)
    return ps, d, m


def test_inactive_boxes_give_the_unconstrained_trajectory(orc):
    ps, d, m = _problem(orc)
    p0 = synth.perturb_theta(ps, 3, mask=MASK)
    th0 = np.array(p0.theta)
    lo = np.where(th0 > 0, th0 / 1e6, 0.0)
    hi = np.where(th0 > 0, th0 * 1e6, 0.0)
    r1 = orc.calibrate(p0, d, m, steps=60, lr=0.05, lr_final=1e-3, free_mask=MASK)
    r2 = orc.calibrate(p0, d, m, steps=60, lr=0.05, lr_final=1e-3, free_mask=MASK, lo=lo, hi=hi)
    assert r1[0] == r2[0] == 0
    assert np.array_equal(r1[1], r2[1]) and np.array_equal(r1[2], r2[2])


def test_binding_box_pins_the_slot_and_the_gradient_points_out(orc):
    """The true BW_L2 lies above the box: projected Adam ends on the box's
    upper face, where the loss still decreases outward (dL/dtheta < 0)."""
    ps, d, m = _problem(orc)
    p0 = synth.perturb_theta(ps, 3, mask=MASK)
    hi = np.zeros(24)
    hi[1] = 0.8 * ps.theta[1]
    lo = np.zeros(24)
    rc, th, hist = orc.calibrate(p0, d, m, steps=400, lr=0.05, lr_final=1e-3, free_mask=MASK, lo=lo, hi=hi)
    assert rc == 0
    assert th[1] == pytest.approx(hi[1], rel=1e-12)
    _, _, g = orc.loss_grad(ps.copy(theta=list(th)), d, m)
    assert g[1] < 0


def test_violated_order_ends_ordered_and_every_step_is_feasible(orc):
    ps, d, m = _problem(orc)
    th = np.array(synth.perturb_theta(ps, 3, mask=MASK).theta)
    # start with L2 faster than L1 and the LLC slower (in latency) than HBM
    th[0], th[1] = 0.5 * ps.theta[0], 2.0 * ps.theta[0]
    th[6], th[7] = 2.0 * ps.theta[7], 0.5 * ps.theta[7]
    p0 = ps.copy(theta=list(th))
    lo = np.zeros(24)
    hi = np.zeros(24)
    for steps in (1, 7, 120):
        rc, t, _ = orc.calibrate(p0, d, m, steps=steps, lr=0.05, lr_final=1e-3, free_mask=MASK, order=3)
        assert rc == 0
        assert t[0] >= t[1] >= t[2] >= t[3], steps
        assert t[4] <= t[5] <= t[6] <= t[7], steps
    # the orderings alone do not bind at the true theta: the fit moves toward it
    assert abs(np.log(t[1] / ps.theta[1])) < abs(np.log(th[1] / ps.theta[1]))


def test_projection_is_order_then_box_on_log_theta(orc):
    """One step with lr small enough that Adam barely moves: the result is
    the box-clamped isotonic fit of log theta of the start."""
    ps, d, m = _problem(orc, n=1 << 10)
    th = np.array(ps.theta)
    th[0:4] = [1.0e13, 3.0e13, 2.0e12, 4.0e12]      # two violations
    th[4:8] = [90.0, 60.0, 800.0, 500.0]
    lo = np.zeros(24)
    hi = np.zeros(24)
    lo[0:4] = [1.0e13, 1.0e13, 1.0e12, 1.0e12]      # ordered like the group
    hi[4:8] = [70.0, 80.0, 900.0, 900.0]
    rc, t, _ = orc.calibrate(ps.copy(theta=list(th)), d, m, steps=1, lr=1e-12, lr_final=0.0,
                             free_mask=MASK, lo=lo, hi=hi, order=3)
    assert rc == 0
    bw = -minmax_isotonic(-np.log(th[0:4]))
    bw = np.maximum(bw, np.log(lo[0:4]))
    lat = np.minimum(minmax_isotonic(np.log(th[4:8])), np.log(hi[4:8]))
    assert np.allclose(np.log(t[0:4]), bw, rtol=0, atol=1e-9)
    assert np.allclose(np.log(t[4:8]), lat, rtol=0, atol=1e-9)


# Plausible mistakes in the constraint code, each planted in an oracle build
# of its own; the pins above (run against that build in a child process)
# must fail for every one.
MUTANTS = {
    "bandwidths ordered the wrong way":
        [("wm_oracle.c", "for (int k = 0; k < 4; ++k) y[k] = -phi[k];", "for (int k = 0; k < 4; ++k) y[k] = phi[k];"),
         ("wm_oracle.c", "for (int k = 0; k < 4; ++k) phi[k] = -y[k];", "for (int k = 0; k < 4; ++k) phi[k] = y[k];")],
    "boxes before the orderings":
        [("wm_oracle.c", "    if (o->order & 2) orc_isotonic_inc(phi + 4, 4);\n    for (int j = 0; j < N_THETA; ++j) {\n"
                         "        if (!(o->free_mask >> j & 1u)) continue;\n"
                         "        if (o->lo[j] > 0.0 && phi[j] < log(o->lo[j])) phi[j] = log(o->lo[j]);\n"
                         "        if (o->hi[j] > 0.0 && phi[j] > log(o->hi[j])) phi[j] = log(o->hi[j]);\n    }",
          "    for (int j = 0; j < N_THETA; ++j) {\n"
          "        if (!(o->free_mask >> j & 1u)) continue;\n"
          "        if (o->lo[j] > 0.0 && phi[j] < log(o->lo[j])) phi[j] = log(o->lo[j]);\n"
          "        if (o->hi[j] > 0.0 && phi[j] > log(o->hi[j])) phi[j] = log(o->hi[j]);\n    }\n"
          "    if (o->order & 2) orc_isotonic_inc(phi + 4, 4);")],
    "a violating pair merged only once":
        [("wm_oracle.c", "while (nb > 1 && mean[nb - 2] > mean[nb - 1]) {", "if (nb > 1 && mean[nb - 2] > mean[nb - 1]) {")],
    "upper bound applied as a lower one":
        [("wm_oracle.c", "if (o->hi[j] > 0.0 && phi[j] > log(o->hi[j])) phi[j] = log(o->hi[j]);",
          "if (o->hi[j] > 0.0 && phi[j] < log(o->hi[j])) phi[j] = log(o->hi[j]);")],
}


def _pins_in_child(tmp_path, replace):
    import os
    import subprocess
    import sys
    from oracle import build as orc_build
    so = orc_build.build_variant(str(tmp_path / "liboracle_variant.so"), replace=replace)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, WM_ORACLE_LIB=so)
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           os.path.join(root, "tests", "test_oracle_constraints.py"), "-k",
                           "not planted and not unmodified"],
                          cwd=root, env=env, capture_output=True, text=True, timeout=300)


def test_pins_pass_on_an_unmodified_build_in_a_child(tmp_path):
    r = _pins_in_child(tmp_path, ())
    assert r.returncode == 0, r.stdout[-1500:]


@pytest.mark.parametrize("what", list(MUTANTS))
def test_planted_constraint_mistake_is_caught(tmp_path, what):
    r = _pins_in_child(tmp_path, MUTANTS[what])
    assert r.returncode != 0, f"the pins did not catch: {what}\n{r.stdout[-1500:]}"
