"""Host-side logic of the recalibration path: the pointer-chase chain, the
parameter derivation from microbenchmark curves (on synthetic curves with
planted values), the validation-case descriptors and split, and argument
checks of libwmbench.so that return before any HIP call."""
import ctypes as C
import math

import numpy as np
import pytest

from paper_2605_04178_amd import microbench as mb
from paper_2605_04178_amd import synth

KB, MB = 1 << 10, 1 << 20


@pytest.mark.parametrize("n_nodes,stride", [(1, 32), (2, 1), (64, 32), (4096, 32), (1 << 15, 4)])
def test_chase_chain_is_one_cycle_over_every_node(n_nodes, stride):
    nxt = mb.chase_chain(n_nodes, stride, 7)
    assert nxt.shape[0] == n_nodes * stride
    seen, i = set(), 0
    for _ in range(n_nodes):
        assert i % stride == 0 and i not in seen
        seen.add(i)
        i = int(nxt[i])
    assert i == 0 and len(seen) == n_nodes
    # every entry, used or not, is an index inside the array
    assert int(nxt.max()) < nxt.shape[0]


def test_linear_fit_and_plateau():
    a, b = mb.linear_fit([1, 2, 3, 4], [3.0, 5.0, 7.0, 9.0])
    assert abs(a - 1.0) < 1e-12 and abs(b - 2.0) < 1e-12
    pairs = [(1, 5.0), (2, 7.0), (4, 6.0), (8, 100.0)]
    assert mb.plateau(pairs, 1, 4) == 6.0 and mb.plateau(pairs, 1, 8, "max") == 100.0
    with pytest.raises(ValueError):
        mb.plateau(pairs, 16, 32)


def test_llc_hit_inverts_the_two_level_mix():
    bw_llc, bw_hbm = 17.2e12, 5.3e12
    for h in (0.0, 0.1, 0.5, 0.93, 1.0):
        bw = 1.0 / (h / bw_llc + (1 - h) / bw_hbm)
        assert abs(mb.llc_hit_from_bw(bw, bw_llc, bw_hbm) - h) < 1e-12
    assert mb.llc_hit_from_bw(1e9, bw_llc, bw_hbm) == 0.0
    assert mb.llc_hit_from_bw(1e15, bw_llc, bw_hbm) == 1.0


def test_streaming_fit_recovers_hbm_and_beta():
    bw_llc, bw_hbm, beta, c = 14e12, 5e12, 1.1, 256.0
    pts = []
    for lg in range(27, 34):
        W = float(1 << lg)
        h = min(1.0, (c / (W / MB)) ** beta)
        pts.append((W, 1.0 / (h / bw_llc + (1 - h) / bw_hbm)))
    hb, b = mb.fit_streaming(pts, bw_llc, c)
    assert abs(hb - bw_hbm) < 1e-6 * bw_hbm and abs(b - beta) < 1e-6
    with pytest.raises(ValueError):
        mb.fit_streaming(pts[:2], bw_llc, c)


def test_llc_exponents_recovered_from_table_regimes():
    w_lo, c = 205.0, 256.0
    alpha, beta = 1.7, 0.8
    pts = []
    for w in np.linspace(64, 2048, 200):
        if w <= w_lo:
            h = 1.0
        elif w <= c:
            h = ((c - w) / (c - w_lo)) ** alpha
        else:
            h = (c / w) ** beta
        pts.append((float(w), float(h)))
    a, b = mb.fit_llc_exponents(pts, w_lo, c)
    assert abs(a - alpha) < 1e-9 and abs(b - beta) < 1e-9
    assert mb.fit_llc_exponents([(100.0, 1.0)], w_lo, c) == (None, None)


def _synthetic_measurements():
    """Curves with planted plateaus, latencies, peaks, launch / dispatch /
    barrier costs and an LLC hit curve with alpha = 1.5, beta = 1.1."""
    bw_l1, bw_l2, bw_llc, bw_hbm = 90e12, 30e12, 14e12, 5e12
    w_lo, c = 205.0, 256.0
    bw = []
    sizes = [1 << lg for lg in range(13, 34)] + [m * MB for m in (208, 216, 224, 232, 240, 248, 320, 384)]
    for W in sorted(sizes):
        if W <= 16 * KB:
            v = bw_l1
        elif W <= 4 * MB:
            v = bw_l2 if W >= 256 * KB else 0.5 * (bw_l1 + bw_l2)
        elif W < 64 * MB:
            v = 0.5 * (bw_l2 + bw_llc)
        else:
            wm = W / MB
            h = 1.0 if wm <= w_lo else (((c - wm) / (c - w_lo)) ** 1.5 if wm <= c else (c / wm) ** 1.1)
            v = 1.0 / (h / bw_llc + (1 - h) / bw_hbm)
        bw.append((W, v, 1 if W <= 4 * MB else 0))
    lat = []
    for lg in range(13, 32):
        W = 1 << lg
        ns = 40.0 if W <= 16 * KB else (200.0 if W <= 2 * MB else (400.0 if W <= 128 * MB else 900.0))
        lat.append((W, ns))
    return {
        "device": {"cus": 256},
        "read_bw": bw, "latency_ns": lat,
        "peak": {"fp64": 70e12, "fp32": 80e12, "bf16": 2.2e15, "fp8": 4.4e15, "int8": 4.3e15},
        "empty_1": 4e-6,
        "empty_blocks": [(g, 4e-6 + 2e-9 * g) for g in (1, 1024, 16384, 131072, 1 << 20)],
        "barriers": [(k, 5e-6 + 3e-8 * k) for k in (0, 1024, 4096, 16384)],
        "barrier_blocks": 2048,
        "interference": {"solo": 20e-6, "concurrent": [31e-6, 29e-6]},
        "sync_s": [7e-6, 6e-6, 9e-6],
        "fusion": [(2048, 100e-6, 30e-6, 101e-6), (4096, 700e-6, 110e-6, 703e-6), (8192, 5e-3, 4e-4, 4.99e-3)],
        "copies": {"h2d": [(n, 2e-6 + n / 50e9) for n in (1 << 12, 1 << 20, 1 << 28)],
                   "d2h": [(n, 3e-6 + n / 40e9) for n in (1 << 12, 1 << 20, 1 << 28)]},
    }


def test_derive_params_recovers_planted_values(wmb_lib):
    m = _synthetic_measurements()
    p = mb.derive_params(m)
    th = p.theta
    assert th[0:2] == [90e12, 30e12]
    assert abs(th[2] - 14e12) < 1e-9 * 14e12 and abs(th[3] - 5e12) < 1e-6 * 5e12
    f = p.f_clk
    for j, ns in zip(range(4, 8), (40.0, 200.0, 400.0, 900.0)):
        assert abs(th[j] - ns * 1e-9 * f) < 1e-9 * th[j]
    assert th[8:13] == [70e12, 80e12, 2.2e15, 4.4e15, 4.3e15]
    assert abs(th[13] - 4e-6) < 1e-18 and abs(th[14] - 2e-9) < 1e-15 and abs(th[15] - 3e-8) < 1e-14
    assert abs(th[16] - 10e-6) < 1e-12
    # tau_fusion: median of the fused-over-plain GEMM excess, floored at 0;
    # tau_sync: median per-sync cost
    assert abs(th[18] - 1e-6) < 1e-15 and abs(th[19] - 7e-6) < 1e-15
    assert abs(th[20] - 1.5) < 1e-6 and abs(th[21] - 1.1) < 1e-6
    assert p.n_cu == 256 and p.n_levels == 4
    # the derived set is one the library accepts
    assert wmb_lib.validate_params(p)
    cm = mb.copy_model(m)
    assert abs(cm["h2d"][0] - 50e9) < 1e-3 * 50e9 and abs(cm["h2d"][1] - 2e-6) < 1e-9
    assert abs(cm["d2h"][0] - 40e9) < 1e-3 * 40e9 and abs(cm["d2h"][1] - 3e-6) < 1e-9


@pytest.fixture(scope="module")
def wmb_lib():
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def test_cases_descriptors_split_and_roofline(wmb_lib):
    cs = mb.case_list()
    names = [c.name for c in cs]
    assert len(set(names)) == len(names)
    d = mb.descriptors_of(cs)
    assert np.all(d.F >= 0) and np.all(d.B > 0) and np.all((d.r1 >= 0) & (d.r1 <= 1))
    assert np.all((d.r2 >= 0) & (d.r2 <= 1)) and np.all(d.u == 1)
    # GEMM reuse: loaded bytes 8 n^3 / T, unique 12 n^2
    g = [c for c in cs if c.kind == "gemm16" and c.n == 1024][0]
    assert g.B == 8.0 * 1024 ** 3 / 16 + 4.0 * 1024 ** 2
    assert abs(g.r2 - (1 - 12.0 * 1024 ** 2 / (8.0 * 1024 ** 3 / 16))) < 1e-15
    tr, ho = mb.split(cs)
    assert len(tr) + len(ho) == len(cs) and len(ho) >= len(cs) // 4
    assert {c.kind for c in ho} == {c.kind for c in cs}
    assert mb.split(cs) == (tr, ho)
    rf = mb.roofline_naive(cs)
    c0 = [c for c in cs if c.kind == "copy"][0]
    assert rf[cs.index(c0)] == c0.B / 8e12
    assert mb.mae([1.0, 3.0], [2.0, 2.0]) == 0.5
    assert mb.mae([1.0, np.nan], [2.0, 2.0]) == 0.5


def test_wmbench_argument_checks_without_a_gpu():
    L = mb.lib()
    d = C.c_double()
    assert L.wmb_read_bw(None, 1024, 1, 1, 0, C.c_void_p(0x100), 1, None, C.byref(d)) == -1
    assert L.wmb_read_bw(C.c_void_p(0x1000), 1000, 1, 1, 0, C.c_void_p(0x100), 1, None, C.byref(d)) == -1
    assert L.wmb_read_bw(C.c_void_p(0x1008), 1024, 1, 1, 0, C.c_void_p(0x100), 1, None, C.byref(d)) == -1
    assert L.wmb_chase(C.c_void_p(0x1000), 1000, 10, 0, C.c_void_p(0x100), C.c_void_p(0x200), None, C.byref(d)) == -1
    assert L.wmb_chase(C.c_void_p(0x1000), 1024, 10, -1, C.c_void_p(0x100), C.c_void_p(0x200), None, C.byref(d)) == -1
    assert L.wmb_peak(7, 10, 1, C.c_void_p(0x100), 1, None, C.byref(d), C.byref(d)) == -1
    assert L.wmb_empty(1, 100, 0, C.c_void_p(0x100), 1, None, C.byref(d)) == -1
    assert L.wmb_clock(0, 10, C.c_void_p(0x100), C.c_void_p(0x200), None, C.byref(d)) == -1
    assert L.wmb_clock(1, 0, C.c_void_p(0x100), C.c_void_p(0x200), None, C.byref(d)) == -1
    assert L.wmb_clock(1, 10, None, C.c_void_p(0x200), None, C.byref(d)) == -1
    assert L.wmb_sync(0, C.c_void_p(0x100), None, C.byref(d)) == -1
    assert L.wmb_val_bytes(mb.VAL["bias"], 100, 0) == -1                       # n % 64
    assert L.wmb_val_bytes(mb.VAL["bias"], 128, 0) == 128 * 4
    assert L.wmb_val_bytes(mb.VAL["bias"], 128, 2) == 128 * 128 * 4
    assert L.wmb_val_bytes(mb.VAL["gemm_mfma_bias"], 128, 1) == 128 * 128 * 2 + 128 * 4
    assert L.wmb_val_bytes(99, 1024, 0) == -1
    assert L.wmb_val_bytes(mb.VAL["copy"], 1023, 0) == -1
    assert L.wmb_val_bytes(mb.VAL["gemm_mfma"], 100, 0) == -1
    assert L.wmb_val_bytes(mb.VAL["gemm_mfma"], 128, 0) == 128 * 128 * 2
    assert L.wmb_val_bytes(mb.VAL["triad"], 1024, 1) == 4096
    assert L.wmb_val_bytes(mb.VAL["copy"], 1024, 1) == 0
    g = C.c_int64()
    # buffers smaller than the kernel needs are refused
    assert L.wmb_val_run(mb.VAL["copy"], C.c_void_p(0x1000), 4095, None, 0, C.c_void_p(0x2000), 4096,
                         1024, 0, 1, None, C.byref(d), C.byref(g)) == -1
    assert L.wmb_val_run(mb.VAL["triad"], C.c_void_p(0x1000), 4096, None, 0, C.c_void_p(0x2000), 4096,
                         1024, 0, 1, None, C.byref(d), C.byref(g)) == -1
    assert L.wmb_last_hip_error() == 0


def test_wmbench_exports_every_declared_symbol():
    import os
    import re
    import subprocess
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                       "wm_microbench.h")
    src = re.sub(r"/\*.*?\*/", "", open(hdr).read(), flags=re.S)
    declared = set(re.findall(r"\b(wmb_[a-z_]+)\s*\(", src))
    assert {"wmb_read_bw", "wmb_chase", "wmb_peak", "wmb_empty", "wmb_val_run", "wmb_clock",
            "wmb_sync"} <= declared
    out = subprocess.run(["nm", "-D", "--defined-only", mb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    assert declared <= set(re.findall(r"\s[TW]\s+(wmb_\w+)", out))


def test_tile_choice_scores_predicted_against_measured_best():
    from paper_2605_04178_amd import recalibrate as rc
    mk = lambda kind, n, s, pc, pm: dict(name=f"{kind}_{n}", kind=kind, n=n, seconds=s, pred_calibrated=pc,
                                         pred_microbench=pm, pred_multiplied=pc, pred_roofline=pm)
    cases = [mk("gemm8", 512, 3.0, 3.0, 1.0), mk("gemm16", 512, 2.0, 2.5, 2.0), mk("gemm32", 512, 2.2, 1.0, 3.0),
             mk("gemm8", 1024, 9.0, 9.0, 9.0), mk("copy", 1024, 1.0, 1.0, 1.0)]
    rows = rc.tile_choice(cases)
    assert len(rows) == 1 and rows[0]["n"] == 512          # one tile at 1024: nothing to choose
    r = rows[0]
    assert r["measured_best"] == "gemm16"
    assert r["calibrated_pick"] == "gemm32" and abs(r["calibrated_slowdown"] - 0.1) < 1e-12
    assert r["microbench_pick"] == "gemm8" and abs(r["microbench_slowdown"] - 0.5) < 1e-12


def test_shipped_calibrated_parameters_are_physical():
    """The shipped MI355X set keeps the cache levels in physical order
    (bandwidths L1 >= L2 >= LLC >= HBM, latencies L1 <= ... <= HBM) and every
    calibrated slot inside its box around the microbenchmark value."""
    import json
    import os
    from paper_2605_04178_amd import recalibrate as rc
    rec = json.load(open(os.path.join(os.path.dirname(mb.__file__), "params", "mi355x.json")))
    th = np.array(rec["theta_calibrated"])
    assert th[0] >= th[1] >= th[2] >= th[3]
    assert th[4] <= th[5] <= th[6] <= th[7]
    lo, hi, _ = rc.calibration_bounds(rec["theta_microbench"])
    mask = rec["calibration"]["free_mask"]
    for j in range(24):
        if (mask >> j) & 1 and lo[j] > 0:
            assert lo[j] * (1 - 1e-9) <= th[j] <= hi[j] * (1 + 1e-9), (j, th[j], lo[j], hi[j])


def test_calibration_bounds_are_ordered_like_the_levels():
    th = [36e12, 33e12, 6.7e12, 6.9e12, 60.0, 171.0, 495.0, 494.0] + [1.0] * 16
    lo, hi, order = rc_bounds(th)
    assert order == 3
    assert np.all(np.diff(lo[0:4]) <= 0) and np.all(np.diff(hi[0:4]) <= 0)
    assert np.all(np.diff(lo[4:8]) >= 0) and np.all(np.diff(hi[4:8]) >= 0)


def rc_bounds(th):
    from paper_2605_04178_amd import recalibrate as rc
    return rc.calibration_bounds(th)
