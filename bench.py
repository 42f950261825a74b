"""Throughput of the CDNA wavefront-model hot path on one MI355X.

One step = one forward sweep (wm_predict) over 2^24 synthetic descriptors in
HBM (FP32 structure-of-arrays, one parameter set).  `value` is forward
evaluations per second over the timed steps.  The same JSON line also carries
the forward+adjoint sweep (wm_loss_grad) over the same descriptors, the tile
selection sweep (2^16 shapes, ragged 8-96 candidates), device calibration
(2^20 descriptors, Adam steps in HIP graphs) and the multi-set batched
calibration, each timed with HIP events on the stream the kernels run on,
plus the roofline of the forward kernel and the FP64 CPU oracle's rate on a
bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "model evals/sec (fwd; fwd+adjoint) and % HBM peak at ≤1e-5 rel err vs FP64"
HBM_PEAK_GBS = 8000.0
FWD_BYTES = 56      # 8 f32 + 4 i32 read, T f32 + occ i32 written
ADJ_BYTES = 52      # 8 f32 + 4 i32 + measured f32 read
SEG_ROW_BYTES = 68  # descriptor (48) + segment row (n_exec, n_kern, cls, h2d, d2h: 20)
APP_BYTES = 8       # offset int32 + T_app (or measured) f32 per application


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed(fn, steps, warmup):
    """(wall ms per step, event ms per step) over `steps` calls after warm-up."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return wall, e0.elapsed_time(e1) / steps


def kernel_name(kind, cfg):
    """Demangled name of the kernel instance a launch configuration selects."""
    if kind == "predict":
        return f"void wm::k_predict<{cfg['per_thread']}, {cfg['block']}>"
    if kind == "loss_grad":
        return f"void wm::k_grad<1, false, {cfg['block']}, false>"
    if kind == "predict_apps":
        return f"void wm::k_apps<{cfg['block']}, 0>"
    if kind == "apps_loss_grad":
        return f"void wm::k_apps_grad<{cfg['block']}, 1>"
    return kind


KERNEL_FILES = (("wm::k_apps", "wm_segments.hip"), ("wm::k_zero_words", "wm_segments.hip"),
                ("wm::k_fuse_costs", "wm_planning.hip"), ("wm::k_plan", "wm_planning.hip"),
                ("wm::k_redo_", "wm_planning.hip"),
                ("wm::k_fit_mult", "wm_planning.hip"), ("wm::k_bw", "wm_blackwell.hip"),
                ("wm::k_select_tile", "wm_tile.hip"), ("wm::k_tile_costs", "wm_tile.hip"),
                ("wm::k_", "wm_kernels.hip"))


def kernel_file(kernel: str) -> str:
    """The source file that defines a kernel of this library."""
    for key, f in KERNEL_FILES:
        if key in kernel:
            return f
    return ""


def kernel_sources(kernel: str) -> bytes:
    """The bytes that determine a kernel's code: its defining file and every
    device header, in name order (the fingerprint tying a counter summary to
    the kernel instances it measured)."""
    csrc = os.path.join(ROOT, "paper_2605_04178_amd", "csrc")
    names = sorted(f for f in os.listdir(csrc) if f.endswith(".hpp"))
    kf = kernel_file(kernel)
    names = ([kf] if kf else []) + names
    return b"".join(open(os.path.join(csrc, f), "rb").read() for f in names)


def counted_traffic(kernel_prefix):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (profiles/traffic.json), or None when the kernel's sources changed
    since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for name, v in rec["kernels"].items():
        if name.startswith(kernel_prefix):
            if hashlib.sha256(kernel_sources(name)).hexdigest()[:16] != v.get("source_sha256_16"):
                return None
            return v["read_bytes"] + v["write_bytes"]
    return None


def profile_summary(kt_dir, fetch_dir, write_dir, sq_dir=None):
    """Summarise the three rocprofv3 runs of `bench.py --profile` (kernel
    trace with --stats, --pmc FETCH_SIZE, --pmc WRITE_SIZE): writes
    profiles/traffic.json (per kernel instance: HBM bytes read and written
    per launch, average duration, source fingerprint) and prints the
    markdown tables of durations and traffic.  Counter KiB are scaled by what
    the same counter reads for the reference copy (1 GiB read, 1 GiB
    written per launch)."""
    import csv
    import glob
    import hashlib

    def one(d, pat):
        f = sorted(glob.glob(os.path.join(d, "**", pat), recursive=True))
        if not f:
            sys.exit(f"no {pat} under {d}")
        return f[0]

    def counter(d, name):
        per = {}
        for r in csv.DictReader(open(one(d, "*counter_collection.csv"))):
            if r["Counter_Name"] == name:
                per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in per.items()}

    stats = list(csv.DictReader(open(one(kt_dir, "*kernel_stats.csv"))))
    fetch, write = counter(fetch_dir, "FETCH_SIZE"), counter(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    if not copy or copy[0] not in write:
        sys.exit("the reference copy kernel is missing from the counter runs")
    gib = float(1 << 30)
    sf, sw = gib / (fetch[copy[0]] * 1024.0), gib / (write[copy[0]] * 1024.0)
    rec = {"scale_fetch": sf, "scale_write": sw, "kernels": {}}
    rows = []
    for r in stats:
        k = r["Name"]
        avg_ns = float(r["AverageNs"])
        rows.append((k, int(r["Calls"]), avg_ns / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3))
        if k.startswith("void wm::") or k.startswith("wm::"):
            if k in fetch and k in write:
                rec["kernels"][k] = {
                    "read_bytes": fetch[k] * 1024.0 * sf, "write_bytes": write[k] * 1024.0 * sw,
                    "avg_ns": avg_ns,
                    "source_sha256_16": hashlib.sha256(kernel_sources(k)).hexdigest()[:16]}
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(rec, f, indent=1)
    short = lambda k: k.split("(")[0]
    print("| kernel instance | calls | average us | min us | max us |")
    print("|---|---|---|---|---|")
    for k, c, a, lo, hi in sorted(rows, key=lambda x: -x[2]):
        print(f"| `{short(k)}` | {c} | {a:.1f} | {lo:.1f} | {hi:.1f} |")
    print()
    print(f"Counter scale (reference copy): FETCH_SIZE x {sf:.4f}, WRITE_SIZE x {sw:.4f}")
    print()
    print("| kernel instance | read MB / launch | written MB / launch | average us | GB/s counted |")
    print("|---|---|---|---|---|")
    for k, v in sorted(rec["kernels"].items(), key=lambda x: -x[1]["avg_ns"]):
        tot = v["read_bytes"] + v["write_bytes"]
        print(f"| `{short(k)}` | {v['read_bytes'] / 1e6:.1f} | {v['write_bytes'] / 1e6:.1f} | "
              f"{v['avg_ns'] / 1e3:.1f} | {tot / v['avg_ns']:.0f} |")
    # per-unit figures of the streamed kernels of the profile run: (unit,
    # units per launch, algorithmic bytes per unit)
    rows_apps = 6817250   # 2^20 applications, seed 150
    units = (("void wm::k_predict<", "descriptor", 1 << 24, FWD_BYTES),
             ("void wm::k_grad<1, false,", "descriptor", 1 << 24, 52),
             ("void wm::k_apps<", "row", rows_apps, 68 + 8 * (1 << 20) / rows_apps),
             ("void wm::k_apps_grad<", "row", rows_apps, 68 + 8 * (1 << 20) / rows_apps),
             ("void wm::k_bw_predict<", "descriptor", 1 << 24, 40),
             ("void wm::k_bw_grad<1, false,", "descriptor", 1 << 24, 36))
    print()
    for k, v in sorted(rec["kernels"].items()):
        for pre, unit, cnt, bpu in units:
            if k.startswith(pre):
                tot = v["read_bytes"] + v["write_bytes"]
                gbs = bpu * cnt / v["avg_ns"]
                print(f"* `{short(k)}`: {tot / cnt:.2f} B/{unit} counted vs {bpu:.2f} algorithmic; "
                      f"average {v['avg_ns'] / 1e3:.1f} us -> {gbs:.0f} GB/s algorithmic = "
                      f"{100 * gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s")
    if sq_dir:
        # GRBM_GUI_ACTIVE sums the eight XCDs; VALU issue per CU-cycle =
        # SQ_INSTS_VALU / (256 CUs x GUI cycles per XCD)
        names = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS",
                 "GRBM_GUI_ACTIVE")
        c = {n: counter(sq_dir, n) for n in names}
        print()
        print("| kernel instance | waves | VALU wave-instr | SALU | VMEM reads | LDS | GUI cycles / XCD "
              "| VALU per CU-cycle |")
        print("|---|---|---|---|---|---|---|---|")
        for k in sorted(c["SQ_INSTS_VALU"], key=lambda x: -c["SQ_INSTS_VALU"][x]):
            if not (k.startswith("void wm::") or k.startswith("wm::")):
                continue
            g = c["GRBM_GUI_ACTIVE"].get(k, 0.0) / 8.0
            v = c["SQ_INSTS_VALU"][k]
            print(f"| `{short(k)}` | {c['SQ_WAVES'].get(k, 0):.0f} | {v:.4g} | {c['SQ_INSTS_SALU'].get(k, 0):.3g} "
                  f"| {c['SQ_INSTS_VMEM_RD'].get(k, 0):.3g} | {c['SQ_INSTS_LDS'].get(k, 0):.3g} | {g:.4g} "
                  f"| {v / (256.0 * g) if g else 0:.2f} |")


def _rate(fn, units, seconds):
    fn()                                  # warm-up (thread pool, page faults)
    reps, t0 = 0, time.perf_counter()
    while True:
        fn()
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds and reps >= 3:
            return reps * units / el, reps, el


def cpu_baseline(p, d, synth, seconds=10.0):
    """The FP64 oracle on the host cores: forward rate on a bounded sample of
    the workload (all cores: the reported baseline), plus shorter context
    figures: the same on one core, loss + gradient, tile candidates."""
    import oracle
    n = min(d.n, 1 << 22)
    sub = d.slice(0, n)
    threads = oracle.set_threads(0)
    rate, reps, el = _rate(lambda: oracle.predict(p, sub), n, seconds)
    out = {"value": rate, "unit": "evals/s", "cores": threads, "kind": "oracle",
           "sample": f"FP64 oracle predict on the first {n} descriptors of the 2^24 workload, "
                     f"{reps} repetitions, {el:.1f} s"}
    n1 = 1 << 18
    oracle.set_threads(1)
    r1, _, _ = _rate(lambda: oracle.predict(p, d.slice(0, n1)), n1, 3.0)
    oracle.set_threads(threads)
    ps = synth.param_set(1)
    m = np.ones(n1, np.float32) * 1e-3
    rg, _, _ = _rate(lambda: oracle.loss_grad(ps, d.slice(0, n1), m), n1, 3.0)
    sh = synth.shapes(1 << 12, 102)
    nc = int(sh.cand_code.shape[0])
    rt, _, _ = _rate(lambda: oracle.select_tile(p, sh), nc, 3.0)
    out["context"] = {"predict_1_core_evals_per_s": r1, "loss_grad_evals_per_s": rg,
                      "select_tile_candidates_per_s": rt,
                      "samples": f"2^18 descriptors (1 core; loss + gradient on {threads} cores), "
                                 f"2^12 shapes / {nc} candidates on {threads} cores, about 3 s each"}
    return out


def profile_run(wm, synth, dd, p, n, dev):
    """Autotune as the benchmark does, then run each hot kernel a few times in
    its tuned configuration, then the reference copy."""
    import torch
    T = torch.empty(n, dtype=torch.float32, device=dev)
    occ = torch.empty(n, dtype=torch.int32, device=dev)
    log("profile: tuned", wm.autotune_predict(dd, p))
    for _ in range(5):
        wm.predict(dd, p, out_T=T, out_occ=occ)
    torch.cuda.synchronize()
    log("profile: predict x5 done")
    meas = (T.clamp(min=1e-6, max=1.0) * 1.01).contiguous()
    ws = wm._workspace(wm.workspace_bytes(wm.OP_LOSS_GRAD, n), dev)
    log("profile: tuned", wm.autotune_grad(wm.OP_LOSS_GRAD, dd, meas, p))
    for _ in range(3):
        wm.loss_grad(dd, meas, p, ws=ws)
    torch.cuda.synchronize()
    log("profile: loss_grad x3 done")
    sh = synth.shapes(1 << 16, 102)
    dsh = wm.DeviceShapes.from_host(sh, dev)
    log("profile: tuned", wm.autotune_select_tile(dsh, p))
    for _ in range(3):
        wm.select_tile(dsh, p)
    torch.cuda.synchronize()
    log("profile: select_tile x3 done")
    del T, occ, meas, ws
    na = 1 << 20
    q = synth.seg_params(7)
    sg, d = synth.segments(na, 150)
    dd2 = wm.DeviceDescriptors.from_host(d, dev)
    ds = wm.DeviceSegments.from_host(sg, dev)
    log("profile: tuned", wm.autotune_apps(wm.OP_PREDICT_APPS, dd2, ds, None, p, q))
    for _ in range(3):
        Ta, _ = wm.predict_apps(dd2, ds, p, q)
    meas = (Ta * 1.05).contiguous()
    log("profile: tuned", wm.autotune_apps(wm.OP_APPS_LOSS_GRAD, dd2, ds, meas, p, q))
    for _ in range(3):
        wm.apps_loss_grad(dd2, ds, meas, p, q)
    torch.cuda.synchronize()
    log("profile: predict_apps x3, apps_loss_grad x3 done")
    del dd2, ds, Ta, meas
    off, d3, e = synth.chains(1 << 16, 164)
    dd3 = wm.DeviceDescriptors.from_host(d3, dev)
    de, doff = torch.from_numpy(e).to(dev), torch.from_numpy(off).to(dev)
    for _ in range(3):
        wm.plan_fusion(dd3, de, doff, p, 8)
    goff, fac, noise, train, d4 = synth.grouped_measurements(1 << 16, 172)
    T4, _ = wm.predict(wm.DeviceDescriptors.from_host(d4, dev), p, want_occ=False)
    m4 = (T4 * 1.1).contiguous()
    for _ in range(3):
        wm.fit_multipliers(T4, m4, torch.from_numpy(goff).to(dev), torch.from_numpy(train).to(dev))
    torch.cuda.synchronize()
    log("profile: plan_fusion x3, fit_multipliers x3 done")
    del dd3, de, doff, T4, m4
    pb = synth.bw_param_set(0)
    db = wm.DeviceBwDescriptors.from_host(synth.bw_descriptors(n, 230), dev)
    for _ in range(5):
        Tb, _ = wm.bw_predict(db, pb)
    mb_ = (Tb * 1.02).contiguous()
    for _ in range(3):
        wm.bw_loss_grad(db, mb_, synth.bw_param_set(1))
    torch.cuda.synchronize()
    log("profile: bw_predict x5, bw_loss_grad x3 done")
    del db, Tb, mb_
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)           # 1 GiB read + 1 GiB written per launch
    torch.cuda.synchronize()
    log("profile: reference copy x3 done (1073741824 bytes each way)")


def segments_leg(wm, synth, args, dev, tuned):
    """Workload segments: 2^20 applications of 1-12 segment rows (about 6.8
    million rows): application totals, and the application-level loss with
    its gradient."""
    import torch
    na = 1 << 20
    p = synth.param_set(0)
    q = synth.seg_params(7)
    sg, d = synth.segments(na, 150)
    rows = int(sg.app_off[-1])
    dd = wm.DeviceDescriptors.from_host(d, dev)
    ds = wm.DeviceSegments.from_host(sg, dev)
    Ta = torch.empty(na, dtype=torch.float32, device=dev)
    if not args.no_tune:
        tuned["predict_apps"] = wm.autotune_apps(wm.OP_PREDICT_APPS, dd, ds, None, p, q)
        log(f"autotuned predict_apps: {tuned['predict_apps']}")
    fa = lambda: wm.predict_apps(dd, ds, p, q, out=Ta)
    wall_f, ev_f = timed(fa, args.steps, args.warmup)
    meas = (Ta * torch.from_numpy(synth.lognormal_noise(na, 151, 0.05).astype(np.float32)).to(dev)).contiguous()
    p0 = synth.perturb_theta(p, 152, factor=1.2)
    ws = wm._workspace(wm.apps_workspace_bytes(rows, na), dev)
    out = torch.empty(33, dtype=torch.float64, device=dev)
    if not args.no_tune:
        tuned["apps_loss_grad"] = wm.autotune_apps(wm.OP_APPS_LOSS_GRAD, dd, ds, meas, p0, q)
        log(f"autotuned apps_loss_grad: {tuned['apps_loss_grad']}")
    fg = lambda: wm.apps_loss_grad(dd, ds, meas, p0, q, ws=ws, out=out)
    wall_g, ev_g = timed(fg, max(args.steps // 2, 3), 2)
    alg = SEG_ROW_BYTES * rows + APP_BYTES * na
    fa_gbs = alg / (ev_f * 1e-3) / 1e9
    fg_gbs = alg / (ev_g * 1e-3) / 1e9
    cf = wm.get_launch(wm.OP_PREDICT_APPS, na)
    cg = wm.get_launch(wm.OP_APPS_LOSS_GRAD, na)
    log(f"segments: predict_apps {ev_f:.4f} ms ({fa_gbs:.0f} GB/s), apps_loss_grad {ev_g:.4f} ms")
    return {"applications": na, "rows": rows,
            "predict_apps": {"ms_per_call": wall_f, "event_ms": ev_f, "rows_per_s": rows / (ev_f * 1e-3),
                             "apps_per_s": na / (ev_f * 1e-3), "achieved_GBs": fa_gbs,
                             "hbm_frac": fa_gbs / HBM_PEAK_GBS, "launch": cf,
                             "kernel": kernel_name("predict_apps", cf),
                             "traffic": counted_traffic(kernel_name("predict_apps", cf))},
            "apps_loss_grad": {"ms_per_call": wall_g, "event_ms": ev_g, "rows_per_s": rows / (ev_g * 1e-3),
                               "achieved_GBs_vs_one_pass": fg_gbs, "hbm_frac_vs_one_pass": fg_gbs / HBM_PEAK_GBS,
                               "launch": cg, "sweep_kernel": kernel_name("apps_loss_grad", cg),
                               "sweep_traffic": counted_traffic(kernel_name("apps_loss_grad", cg))},
            "bytes_per_row": SEG_ROW_BYTES, "bytes_per_app": APP_BYTES}


def planning_leg(wm, synth, args, dev, log):
    """Fusion planning over 2^16 synthetic kernel chains (2-16 kernels, runs up
    to 8) and per-group multipliers over 2^16 groups (1-40 rows)."""
    import torch
    p = synth.param_set(0)
    off, d, e = synth.chains(1 << 16, 164)
    dd = wm.DeviceDescriptors.from_host(d, dev)
    de = torch.from_numpy(e).to(dev)
    doff = torch.from_numpy(off).to(dev)
    R = 8
    ws = wm._workspace(wm.plan_workspace_bytes(d.n, R), dev)
    fp = lambda: wm.plan_fusion(dd, de, doff, p, R, ws=ws)
    wall_p, ev_p = timed(fp, args.steps, args.warmup)
    lens = np.diff(off).astype(np.int64)
    cands = int(sum(min(R, j + 1) for L in lens for j in range(L)))
    tot, unf, st = fp()
    redone = wm.plan_redone(ws)
    gain = float((unf / tot).double().mean().item())
    goff, fac, noise, train, d2 = synth.grouped_measurements(1 << 16, 172)
    dd2 = wm.DeviceDescriptors.from_host(d2, dev)
    T, _ = wm.predict(dd2, p, want_occ=False)
    g = torch.from_numpy(np.repeat(np.arange(1 << 16), np.diff(goff))).to(dev)
    meas = (T * torch.from_numpy(fac.astype(np.float32)).to(dev)[g] *
            torch.from_numpy(noise.astype(np.float32)).to(dev)).contiguous()
    dgoff = torch.from_numpy(goff).to(dev)
    dtrain = torch.from_numpy(train).to(dev)
    ws2 = wm._workspace(wm.workspace_bytes(wm.OP_FIT_MULTIPLIERS, d2.n), dev)
    fm = lambda: wm.fit_multipliers(T, meas, dgoff, dtrain, ws=ws2)
    wall_m, ev_m = timed(fm, args.steps, args.warmup)
    _, _, stt = fm()
    stt = stt.cpu().numpy()
    log(f"planning: fusion {ev_p:.3f} ms ({cands / (ev_p * 1e-3):.3g} candidate runs/s, "
        f"{redone} of {len(lens)} chains redone in float64), multipliers {ev_m:.3f} ms")
    return {"fusion": {"chains": len(lens), "rows": int(d.n), "max_run": R, "candidate_runs": cands,
                       "ms_per_call": wall_p, "event_ms": ev_p,
                       "candidate_runs_per_s": cands / (ev_p * 1e-3), "chains_per_s": len(lens) / (ev_p * 1e-3),
                       "chains_redone_fp64": redone,
                       "mean_unfused_over_planned": gain, "fused_share": float(1.0 - st.float().mean().item())},
            "multipliers": {"groups": 1 << 16, "rows": int(d2.n), "ms_per_call": wall_m, "event_ms": ev_m,
                            "rows_per_s": d2.n / (ev_m * 1e-3),
                            "train_mre": float(stt[0] / max(stt[1], 1)),
                            "holdout_mre": float(stt[2] / max(stt[3], 1))}}


BW_FWD_BYTES = 40    # 5 int32 + 3 float32 read, T f32 + cta i32 written
BW_ADJ_BYTES = 36    # 32 read + measured f32


def blackwell_leg(wm, synth, args, dev, log):
    """The Blackwell stage-centric family over 2^24 tile-kernel descriptors:
    forward sweep and forward + adjoint (loss and gradient)."""
    import torch
    n = 1 << 24
    p = synth.bw_param_set(0)
    d = synth.bw_descriptors(n, 230)
    dd = wm.DeviceBwDescriptors.from_host(d, dev)
    T = torch.empty(n, dtype=torch.float32, device=dev)
    fw = lambda: wm.bw_predict(dd, p, out_T=T)
    wall_f, ev_f = timed(fw, args.steps, args.warmup)
    Tm, _ = wm.bw_predict(dd, synth.bw_param_set(1), want_cta=False)
    meas = (Tm * torch.from_numpy(synth.lognormal_noise(n, 231, 0.02).astype(np.float32)).to(dev)).contiguous()
    del Tm
    ws = wm._workspace(wm.bw_workspace_bytes(wm.BW_OP_GRAD, n), dev)
    out = torch.empty(26, dtype=torch.float64, device=dev)
    lg = lambda: wm.bw_loss_grad(dd, meas, p, ws=ws, out=out)
    wall_g, ev_g = timed(lg, max(args.steps // 2, 3), 2)
    gf = BW_FWD_BYTES * n / (ev_f * 1e-3) / 1e9
    gg = BW_ADJ_BYTES * n / (ev_g * 1e-3) / 1e9
    log(f"blackwell: forward {ev_f:.4f} ms ({gf:.0f} GB/s), fwd+adjoint {ev_g:.4f} ms ({gg:.0f} GB/s)")
    return {"descriptors": n, "param_set": "Blackwell-style seed 0",
            "forward": {"evals_per_s": n / (ev_f * 1e-3), "event_ms": ev_f, "ms_per_call": wall_f,
                        "achieved_GBs": gf, "hbm_frac": gf / HBM_PEAK_GBS, "bytes_per_eval": BW_FWD_BYTES,
                        "traffic": counted_traffic("void wm::k_bw_predict<256>")},
            "fwd_adjoint": {"evals_per_s": n / (ev_g * 1e-3), "event_ms": ev_g, "ms_per_call": wall_g,
                            "achieved_GBs": gg, "hbm_frac": gg / HBM_PEAK_GBS, "bytes_per_eval": BW_ADJ_BYTES}}


def hardware_model_leg(wm, log):
    """Re-times the held-out validation kernels of the shipped MI355X
    parameter file on this GPU and scores the model with that file's
    microbenchmark and calibrated parameters, and the naive roofline."""
    from paper_2605_04178_amd import microbench as mb, recalibrate as rc
    path = os.path.join(ROOT, "paper_2605_04178_amd", "params", "mi355x.json")
    rec = json.load(open(path))
    names = {c["name"] for c in rec["cases"] if c["split"] == "hold"}
    cases = [c for c in mb.case_list() if c.name in names]
    mb.run_cases(cases, log=lambda *a: None)
    meas = np.array([c.seconds for c in cases])
    out = {"cases": len(cases), "params": "paper_2605_04178_amd/params/mi355x.json"}
    preds = {}
    for which in ("microbench", "calibrated"):
        T, _ = rc.predict(wm, rc.load_params(path, which), cases)
        out[f"mae_{which}"] = mb.mae(T, meas)
        preds[which] = T
    fm = rec.get("family_multipliers", {})
    if fm:
        out["mae_calibrated_multiplied"] = mb.mae(np.array([fm[c.kind] for c in cases]) * T, meas)
    out["mae_roofline"] = mb.mae(mb.roofline_naive(cases), meas)
    # adaptive tile selection against the measured best tile, live
    out["tile_choice"] = rc.tile_choice([dict(name=c.name, kind=c.kind, n=c.n, seconds=c.seconds,
                                              pred_microbench=float(preds["microbench"][i]),
                                              pred_calibrated=float(preds["calibrated"][i]))
                                         for i, c in enumerate(cases)])
    out["mae_recorded"] = {k: rec["mae"][k] for k in ("calibrated_holdout", "multipliers_holdout",
                                                       "roofline_holdout") if k in rec["mae"]}
    log(f"hardware model on held-out kernels: MAE calibrated {out['mae_calibrated']:.3f}, "
        f"microbench {out['mae_microbench']:.3f}, roofline {out['mae_roofline']:.3f}")
    return out


def platform(dev):
    """What the numbers were measured on: the GPU as the runtime reports it,
    its shader clock measured by wmb_clock, the host CPU."""
    import torch
    from paper_2605_04178_amd import microbench as mb
    pr = torch.cuda.get_device_properties(dev)
    cpu = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"gpu": pr.name, "arch": getattr(pr, "gcnArchName", ""), "cus": pr.multi_processor_count,
            "hbm_gib": pr.total_memory / 2 ** 30, "l2_mib": getattr(pr, "L2_cache_size", 0) / 2 ** 20,
            "hip_runtime": torch.version.hip, "torch": torch.__version__,
            "shader_clock_ghz": {"one_wave": mb.clock_hz(1) / 1e9,
                                 "loaded_32_waves_per_cu": mb.clock_hz(pr.multi_processor_count * 32) / 1e9},
            "host_cpu": cpu, "host_threads_visible": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--quick", action="store_true", help="forward sweep only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-steps", type=int, default=500)
    ap.add_argument("--no-tune", action="store_true",
                    help="time the default launch configurations instead of autotuned ones")
    ap.add_argument("--profile", action="store_true",
                    help="run each hot kernel a few times, then a plain 1 GiB device copy whose "
                         "known traffic scales the rocprofv3 FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--profile-summary", nargs="+", metavar="DIR",
                    help="KT_DIR FETCH_DIR WRITE_DIR [SQ_DIR]: summarise the rocprofv3 output folders "
                         "of a --profile run into profiles/traffic.json and markdown tables (no GPU "
                         "needed)")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(*args.profile_summary)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the batched model "
              "evaluation shards by descriptor range with no exchange, so run one process per GPU.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_04178_amd import synth, wavemodel as wm

    wm.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    props = torch.cuda.get_device_properties(dev)
    log(f"device {props.name} CUs={props.multi_processor_count}")

    n = args.n
    p = synth.param_set(0)
    log(f"generating {n} descriptors")
    d = synth.descriptors(n, 101)
    dd = wm.DeviceDescriptors.from_host(d, dev)
    T = torch.empty(n, dtype=torch.float32, device=dev)
    occ = torch.empty(n, dtype=torch.int32, device=dev)

    if args.profile:
        profile_run(wm, synth, dd, p, n, dev)
        return

    tuned = {}
    if not args.no_tune:
        tuned["predict"] = wm.autotune_predict(dd, p)
        log(f"autotuned predict: {tuned['predict']}")

    # ---- forward sweep (the step) ----
    fwd = lambda: wm.predict(dd, p, out_T=T, out_occ=occ)
    wall_ms, ev_ms = timed(fwd, args.steps, args.warmup)
    log(f"forward: {wall_ms:.4f} ms/step wall, {ev_ms:.4f} ms/launch (events)")
    value = n / (wall_ms * 1e-3)
    achieved = FWD_BYTES * n / (ev_ms * 1e-3) / 1e9
    res = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded PCG64 descriptor sweep, inputs resident in HBM)",
        "config": {"workload": "batched forward: 2^24 kernel descriptors, FP32 SoA "
                               "(8 f32 + 4 i32 each), one CDNA-style parameter set",
                   "n_descriptors": n, "param_set": "seed 0, 4 levels, HK_MAX"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counted_traffic(kernel_name("predict", wm.get_launch(wm.OP_PREDICT, n))),
                     "kernel": kernel_name("predict", wm.get_launch(wm.OP_PREDICT, n)),
                     "bytes_per_eval": FWD_BYTES, "avg_launch_us": ev_ms * 1e3},
        "launch": {"predict": wm.get_launch(wm.OP_PREDICT, n)},
    }

    if not args.quick:
        # ---- forward + adjoint (loss and gradient) over the same descriptors ----
        ps = synth.param_set(1)
        Tm, _ = wm.predict(dd, ps, want_occ=False)
        noise = torch.from_numpy(synth.lognormal_noise(n, 2, 0.02).astype(np.float32)).to(dev)
        meas = (Tm * noise).contiguous()
        del Tm, noise
        p0 = synth.perturb_theta(ps, 3)
        ws = wm._workspace(wm.workspace_bytes(wm.OP_LOSS_GRAD, n), dev)
        out = torch.empty(26, dtype=torch.float64, device=dev)
        if not args.no_tune:
            tuned["loss_grad"] = wm.autotune_grad(wm.OP_LOSS_GRAD, dd, meas, p0)
            log(f"autotuned loss_grad: {tuned['loss_grad']}")
        res["launch"]["loss_grad"] = wm.get_launch(wm.OP_LOSS_GRAD, n)
        lg = lambda: wm.loss_grad(dd, meas, p0, ws=ws, out=out)
        wall_a, ev_a = timed(lg, max(args.steps // 2, 3), 2)
        ach_a = ADJ_BYTES * n / (ev_a * 1e-3) / 1e9
        res["fwd_adjoint"] = {"value": n / (wall_a * 1e-3), "unit": "evals/s", "ms_per_step": wall_a,
                              "achieved_GBs": ach_a, "hbm_frac": ach_a / HBM_PEAK_GBS,
                              "bytes_per_eval": ADJ_BYTES, "dtype": "f32 + f64 reductions",
                              "traffic": counted_traffic(kernel_name("loss_grad", res["launch"]["loss_grad"]))}
        log(f"fwd+adjoint: {wall_a:.4f} ms/step, {ach_a:.0f} GB/s")
        # the float64-exact variant of the same call
        lx = lambda: wm.loss_grad(dd, meas, p0, ws=ws, out=out, exact=True)
        wall_x, ev_x = timed(lx, max(args.steps // 2, 3), 2)
        ach_x = ADJ_BYTES * n / (ev_x * 1e-3) / 1e9
        res["fwd_adjoint_exact"] = {"value": n / (wall_x * 1e-3), "unit": "evals/s", "ms_per_step": wall_x,
                                    "achieved_GBs": ach_x, "hbm_frac": ach_x / HBM_PEAK_GBS, "dtype": "f64"}
        log(f"fwd+adjoint, float64-exact call: {wall_x:.4f} ms/step, {ach_x:.0f} GB/s")
        del meas, ws

        # ---- tile selection ----
        sh = synth.shapes(1 << 16, 102)
        dsh = wm.DeviceShapes.from_host(sh, dev)
        if not args.no_tune:
            tuned["select_tile"] = wm.autotune_select_tile(dsh, p)
            log(f"autotuned select_tile: {tuned['select_tile']}")
        res["launch"]["select_tile"] = wm.get_launch(wm.OP_SELECT_TILE, sh.n)
        outs = (torch.empty(sh.n, dtype=torch.int32, device=dev),
                torch.empty(sh.n, dtype=torch.float64, device=dev),
                torch.empty(sh.n, dtype=torch.uint8, device=dev))
        sel = lambda: wm.select_tile(dsh, p, out=outs)
        wall_t, ev_t = timed(sel, args.steps, args.warmup)
        # the same launch replayed from a captured HIP graph
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            sel()
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(g):
            sel()
        wall_g, ev_g = timed(g.replay, args.steps, args.warmup)
        ncand = int(sh.cand_code.shape[0])
        res["select_tile"] = {"shapes": sh.n, "candidates": ncand, "ms_per_call": wall_t,
                              "ms_per_graph_replay": wall_g,
                              "candidates_per_s": ncand / (wall_g * 1e-3),
                              "shapes_per_s": sh.n / (wall_g * 1e-3)}
        log(f"select_tile: {wall_t:.4f} ms/call, {wall_g:.4f} ms/graph replay")

        # ---- calibration: 2^20 descriptors, Adam in captured graphs ----
        nc = 1 << 20
        dc = synth.calibration_descriptors(nc, 103)
        ddc = wm.DeviceDescriptors.from_host(dc, dev)
        Tc, _ = wm.predict(ddc, ps, want_occ=False)
        mc = (Tc * torch.from_numpy(synth.lognormal_noise(nc, 2, 0.02).astype(np.float32)).to(dev)).contiguous()
        mask = synth.fit_mask(ps.n_levels)
        p0c = synth.perturb_theta(ps, 3, mask=mask)
        if not args.no_tune:
            tuned["loss_grad_2^20"] = wm.autotune_grad(wm.OP_LOSS_GRAD, ddc, mc, p0c)
        res["launch"]["calibrate"] = wm.get_launch(wm.OP_CALIBRATE, nc)
        # one untimed call first (code-object loading, the allocator's first
        # workspace); the timed call runs every step, graph capture included
        wm.calibrate(ddc, mc, p0c, steps=args.calib_steps, free_mask=mask)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, th, hist = wm.calibrate(ddc, mc, p0c, steps=args.calib_steps, free_mask=mask)
        el = time.perf_counter() - t0
        idx = [j for j in range(24) if mask >> j & 1]
        err = float(np.max(np.abs(th[idx] / np.array(ps.theta)[idx] - 1)))
        res["calibrate"] = {"descriptors": nc, "steps": args.calib_steps, "seconds": el,
                            "timing": "second call (graph capture and instantiation included)",
                            "fwd_adj_evals_per_s": nc * args.calib_steps / el,
                            "max_recovery_err": err, "status": rc,
                            "loss_first_last": [float(hist[0]), float(hist[-1])]}
        log(f"calibrate: {el:.3f} s, max recovery err {err:.4f}")
        # the same problem under the Eq. (9)/(12) occupancy-overlap combine
        pe = ps.copy(combine=1)
        Te, _ = wm.predict(ddc, pe, want_occ=False)
        me = (Te * torch.from_numpy(synth.lognormal_noise(nc, 2, 0.02).astype(np.float32)).to(dev)).contiguous()
        p0e = synth.perturb_theta(pe, 3, mask=mask)
        t0 = time.perf_counter()
        rce, the, histe = wm.calibrate(ddc, me, p0e, steps=args.calib_steps, free_mask=mask)
        el_e = time.perf_counter() - t0
        err_e = float(np.max(np.abs(the[idx] / np.array(pe.theta)[idx] - 1)))
        res["calibrate_overlap_combine"] = {"descriptors": nc, "steps": args.calib_steps, "seconds": el_e,
                                            "max_recovery_err": err_e, "status": rce}
        log(f"calibrate (overlap combine): {el_e:.3f} s, max recovery err {err_e:.4f}")
        del ddc, mc, Tc, me, Te

        # ---- batched calibration of six architectures vs six plain launches ----
        sets = synth.multi_arch_sets()
        sizes = synth.multi_arch_sizes()
        descs, meas_l, p0s, opts = [], [], [], []
        for k, (pk, nk) in enumerate(zip(sets, sizes)):
            dk = synth.calibration_descriptors(nk, 120 + k)
            ddk = wm.DeviceDescriptors.from_host(dk, dev)
            Tk, _ = wm.predict(ddk, pk, want_occ=False)
            mk = (Tk * torch.from_numpy(synth.lognormal_noise(nk, 130 + k, 0.02).astype(np.float32)).to(dev)).contiguous()
            mk_mask = synth.fit_mask(pk.n_levels)
            descs.append(ddk)
            meas_l.append(mk)
            p0s.append(synth.perturb_theta(pk, 140 + k, mask=mk_mask))
            opts.append(wm.calib_opts(steps=args.calib_steps, free_mask=mk_mask))
        if not args.no_tune:
            tuned["batched"] = wm.autotune_batched(descs, meas_l, p0s, opts)
            log(f"autotuned batched: {tuned['batched']}")
        res["launch"]["batched"] = wm.get_launch(wm.OP_CALIBRATE_BATCHED, sum(sizes))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rcb, thb, histb = wm.calibrate_batched(descs, meas_l, p0s, opts)
        el_b = time.perf_counter() - t0
        t0 = time.perf_counter()
        for k in range(len(sets)):
            wm.calibrate(descs[k], meas_l[k], p0s[k], steps=args.calib_steps,
                         free_mask=opts[k].free_mask)
        el_p = time.perf_counter() - t0
        tot = sum(sizes) * args.calib_steps
        rec = []
        for k, pk in enumerate(sets):
            idx = [j for j in range(24) if opts[k].free_mask >> j & 1]
            rec.append(float(np.max(np.abs(thb[k][idx] / np.array(pk.theta)[idx] - 1))))
        res["batched"] = {"sets": len(sets), "sizes": sizes, "steps": args.calib_steps,
                          "persistent_evals_per_s": tot / el_b, "per_set_evals_per_s": tot / el_p,
                          "speedup": el_p / el_b, "per_set_recovery_err": rec, "status": rcb}
        log(f"batched: {el_b:.3f} s persistent vs {el_p:.3f} s per-set")
        del descs, meas_l

        res["segments"] = segments_leg(wm, synth, args, dev, tuned)
        res["planning"] = planning_leg(wm, synth, args, dev, log)
        res["blackwell"] = blackwell_leg(wm, synth, args, dev, log)
        res["mi355x_model"] = hardware_model_leg(wm, log)

    if tuned:
        res["autotune_us"] = {k: v["us"] for k, v in tuned.items()}
    res["platform"] = platform(dev)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(p, d, synth)
    res["paper_context"] = {
        "note": "the paper reports prediction accuracy on its hardware, not evaluation throughput",
        "MI300A_cdna_model_mae": "~0.09% calibrated with per-case multipliers (27 kernels); ~5-8% uncalibrated",
        "MI250X_parameter_port_mae": "4.69% (19 kernels)",
        "naive_roofline_mae": "99.6% MI300A, 97.9% MI250X",
        "B200_blackwell_model_mae": "1.31-1.33% (21 kernels)"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
