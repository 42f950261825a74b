"""Profiler-derived characterization of the validation kernels.

The paper finds (Discussion, Observation 3) that the model's accuracy depends
on where a kernel's flops and bytes come from: hardware counters or analysis
of the algorithm.  This module puts the validation kernels of the
recalibration suite through both.  Their first-principles bytes and reuse
fractions are the ones `microbench.case_list` derives from the algorithms.
Two profiler-derived readings come from rocprofv3 counters, each scaled by
what the same counter reads for a plain device copy of known size:

* L2-to-fabric bytes: FETCH_SIZE + WRITE_SIZE (Infinity-Cache hits
  included), with r1 = r2 = 0 since none of it is served by L1 or L2;
* L1-to-L2 bytes: the read and write requests the L1s send to the L2, with
  r1 = 0 and r2 the fraction of L2 requests that hit.

Both keep the footprint W, through which h_LLC(W) splits the traffic below L2
between the Infinity Cache and HBM.  Flops stay the algorithmic ones (the GPU
tests check every kernel's output, so they are the work done).  Each case's
counter value is the mean over its timed launches (the warm-up launch that
precedes them in `wmb_val_run`, and the warm-up launches before that, are
skipped).  The commands are in the summary
that `score --md` writes.
"""
from __future__ import annotations

import argparse
import csv
import dataclasses
import json
import sys
from collections import defaultdict
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import microbench as mb

COPY_BYTES = 1 << 30          # the reference device copy
COPY_REPS = 3
COPY_KERNEL = "copyBuffer"    # the runtime's device-to-device copy kernel
VAL_KERNEL = "k_val_"

# kernel-name stem of each validation family
STEM = {"copy": "k_val_copy", "triad": "k_val_triad", "reduce": "k_val_reduce", "fma": "k_val_fma",
        "stencil": "k_val_stencil", "transpose_naive": "k_val_transpose_naive",
        "transpose_lds": "k_val_transpose_lds", "gemm8": "k_val_gemm_tile", "gemm16": "k_val_gemm_tile",
        "gemm32": "k_val_gemm_tile", "gemm_mfma": "k_val_gemm_mfma", "bias": "k_val_bias",
        "gemm_mfma_bias": "k_val_gemm_mfma"}


# ---------------------------------------------------------------------------
# counter files (host logic, no GPU)
# ---------------------------------------------------------------------------
def read_dispatches(path: str, counter: str) -> List[Tuple[int, str, float]]:
    """(dispatch id, kernel name, counter value) per dispatch of a rocprofv3
    counter-collection CSV, in dispatch order; rows of one dispatch (several
    instances or dimensions) are summed."""
    val: Dict[int, float] = defaultdict(float)
    name: Dict[int, str] = {}
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            val[d] += float(r["Counter_Value"])
            name[d] = r["Kernel_Name"]
    return [(d, name[d], val[d]) for d in sorted(val)]


def per_case(dispatches: Sequence[Tuple[int, str, float]], kinds: Sequence[str], launches: int,
             warmup: int = 0) -> np.ndarray:
    """Mean counter value per case over its `launches` timed dispatches.
    Every case ran `warmup` + 1 + `launches` dispatches of its validation
    kernel (the warm-ups and one untimed launch first), cases in order; other
    kernels (the allocators' fills, the reference copy) are skipped."""
    val = [(n, v) for _, n, v in dispatches if VAL_KERNEL in n]
    per = warmup + 1 + launches
    if len(val) != per * len(kinds):
        raise ValueError(f"{len(val)} validation dispatches for {len(kinds)} cases x {per}")
    out = np.empty(len(kinds))
    for i, k in enumerate(kinds):
        chunk = val[i * per:(i + 1) * per]
        if not all(STEM[k] in n for n, _ in chunk):
            raise ValueError(f"case {i} ({k}): kernels {sorted({n for n, _ in chunk})}")
        out[i] = float(np.mean([v for _, v in chunk[per - launches:]]))
    return out


def copy_scale(dispatches: Sequence[Tuple[int, str, float]], bytes_per_copy: float = COPY_BYTES,
               unit: float = 1024.0) -> float:
    """True bytes per counted unit (FETCH_SIZE and WRITE_SIZE read KiB:
    unit = 1024; request counters: unit = 1): the reference copies' known
    traffic over what the counter read for them (their last COPY_REPS
    dispatches), so that the result multiplies counter x unit."""
    cp = [v for _, n, v in dispatches if COPY_KERNEL in n][-COPY_REPS:]
    if len(cp) < COPY_REPS or not min(cp) > 0:
        raise ValueError("reference copy missing from the counter file")
    return bytes_per_copy / (float(np.mean(cp)) * unit)


def profiler_bytes(fetch_csv: str, write_csv: str, kinds: Sequence[str], launches: int,
                   warmup: int = 0) -> Tuple[np.ndarray, dict]:
    """Scaled (FETCH_SIZE + WRITE_SIZE) bytes per launch of every case: the
    traffic between the L2 and the memory fabric."""
    fd = read_dispatches(fetch_csv, "FETCH_SIZE")
    wd = read_dispatches(write_csv, "WRITE_SIZE")
    fs, ws = copy_scale(fd), copy_scale(wd)
    rb = per_case(fd, kinds, launches, warmup) * 1024.0 * fs
    wb = per_case(wd, kinds, launches, warmup) * 1024.0 * ws
    return rb + wb, {"fetch_scale": fs, "write_scale": ws, "read_bytes": rb.tolist(), "write_bytes": wb.tolist()}


L2_COUNTERS = ("TCP_TCC_READ_REQ_sum", "TCP_TCC_WRITE_REQ_sum", "TCC_HIT_sum", "TCC_MISS_sum")


def l2_traffic(l2_csv: str, kinds: Sequence[str], launches: int,
               warmup: int = 0) -> Tuple[np.ndarray, np.ndarray, dict]:
    """Bytes requested from the L2 per launch (read and write requests from
    the L1s, each scaled by what the reference copy's requests carry) and
    the fraction of L2 requests that hit."""
    rd, wr, hit, miss = (read_dispatches(l2_csv, c) for c in L2_COUNTERS)
    rs = copy_scale(rd, unit=1.0)
    ws = copy_scale(wr, unit=1.0)
    B = per_case(rd, kinds, launches, warmup) * rs + per_case(wr, kinds, launches, warmup) * ws
    h, m = per_case(hit, kinds, launches, warmup), per_case(miss, kinds, launches, warmup)
    r2 = np.where(h + m > 0, h / np.maximum(h + m, 1.0), 0.0)
    return B, r2, {"read_req_bytes": rs, "write_req_bytes": ws}


# ---------------------------------------------------------------------------
# GPU steps
# ---------------------------------------------------------------------------
def run(out: str, quick: bool = False, launches: int = 100, warmup: int = 10) -> None:
    """Time every validation case, then make the reference copies."""
    import torch
    cases = mb.run_cases(mb.case_list(quick), launches=launches, warmup=warmup,
                         log=lambda *a: print(*a, flush=True))
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(COPY_REPS):
        b.copy_(a)
    torch.cuda.synchronize()
    with open(out, "w") as f:
        json.dump({"launches": launches, "warmup": warmup, "quick": quick,
                   "cases": [dataclasses.asdict(c) for c in cases]}, f)
    print(f"{len(cases)} cases timed, {COPY_REPS} reference copies of {COPY_BYTES} bytes", flush=True)


def _desc_with(cases: List[mb.Case], B: np.ndarray, r2=None):
    """Descriptors of the cases with bytes B served below L1 (r1 = 0) and
    the given L2 fraction (0 when the bytes are the traffic below L2)."""
    d = mb.descriptors_of(cases)
    d.B[:] = B.astype(np.float32)
    d.r1[:] = 0.0
    d.r2[:] = 0.0 if r2 is None else np.clip(r2, 0.0, 1.0).astype(np.float32)
    return d


def _predict(wm, p, d):
    import torch
    T, _ = wm.predict(wm.DeviceDescriptors.from_host(d), p)
    torch.cuda.synchronize()
    return T.cpu().numpy().astype(np.float64)


def _calibrate(wm, p0, d, meas, idx, steps):
    """Adam on the training cases (the slots the validation kernels inform)."""
    import torch
    from .recalibrate import FIT_MASK
    sub = type(d)(**{k: getattr(d, k)[idx] for k in d.__dataclass_fields__})
    m = torch.tensor(meas[idx], dtype=torch.float32, device="cuda")
    mask = FIT_MASK & ~sum(1 << j for j in range(24) if not p0.theta[j] > 0.0)
    rc, th, _ = wm.calibrate(wm.DeviceDescriptors.from_host(sub), m, p0, steps=steps, lr=0.02,
                             lr_final=1e-3, free_mask=mask)
    return rc, p0.copy(theta=[float(x) for x in th])


NAMES = {"first_principles": "first principles",
         "profiler_fabric": "profiler: L2-to-fabric bytes (FETCH_SIZE + WRITE_SIZE)",
         "profiler_l2": "profiler: L1-to-L2 request bytes, L2 hit fraction"}


def score(times: str, fetch_csv: str, write_csv: str, params: str, out: str, steps: int = 2000,
          md: str = None, l2_csv: str = None) -> dict:
    from . import wavemodel as wm
    from .recalibrate import load_params
    wm.lib()
    rec = json.load(open(times))
    cases = [mb.Case(**c) for c in rec["cases"]]
    kinds = [c.kind for c in cases]
    meas = np.array([c.seconds for c in cases])
    warm = rec.get("warmup", 0)
    B_fab, scales = profiler_bytes(fetch_csv, write_csv, kinds, rec["launches"], warm)
    B = {"first_principles": np.array([c.B for c in cases]), "profiler_fabric": B_fab}
    descs = {"first_principles": mb.descriptors_of(cases), "profiler_fabric": _desc_with(cases, B_fab)}
    r2_l2 = None
    if l2_csv:
        B_l2, r2_l2, sc2 = l2_traffic(l2_csv, kinds, rec["launches"], warm)
        scales.update(sc2)
        B["profiler_l2"] = B_l2
        descs["profiler_l2"] = _desc_with(cases, B_l2, r2_l2)
    train, hold = mb.split(cases)
    it = np.array([cases.index(c) for c in train])
    ih = np.array([cases.index(c) for c in hold])
    hold_set = set(ih.tolist())
    p_mb = load_params(params, "microbench")
    res = {"cases": [], "scales": scales, "params": params, "steps": steps, "tags": list(descs),
           "roofline": {}, "per_family": {}}
    preds = {}
    for tag, d in descs.items():
        T_mb = _predict(wm, p_mb, d)
        rc, p_cal = _calibrate(wm, p_mb, d, meas, it, steps)
        T_cal = _predict(wm, p_cal, d)
        roof = mb.roofline_naive([dataclasses.replace(c, B=float(b)) for c, b in zip(cases, B[tag])])
        preds[tag] = (T_mb, T_cal)
        res[tag] = {"calibration_status": rc, "theta_calibrated": list(p_cal.theta),
                    "mae_microbench_all": mb.mae(T_mb, meas), "mae_microbench_holdout": mb.mae(T_mb[ih], meas[ih]),
                    "mae_calibrated_train": mb.mae(T_cal[it], meas[it]),
                    "mae_calibrated_holdout": mb.mae(T_cal[ih], meas[ih]),
                    "mae_roofline_all": mb.mae(roof, meas), "mae_roofline_holdout": mb.mae(roof[ih], meas[ih])}
    for f in sorted(set(kinds)):
        ix = np.array([i for i, k in enumerate(kinds) if k == f])
        res["per_family"][f] = {
            **{f"bytes_ratio_{tag}": float(np.median(B[tag][ix] / B["first_principles"][ix])) for tag in descs},
            **{f"{tag}_{w}": mb.mae(preds[tag][j][ix], meas[ix])
               for tag in preds for j, w in enumerate(("microbench", "calibrated"))}}
    for i, c in enumerate(cases):
        row = {"name": c.name, "kind": c.kind, "split": "hold" if i in hold_set else "train", "seconds": c.seconds}
        for tag in descs:
            row[f"B_{tag}"] = float(B[tag][i])
            row[f"pred_{tag}_microbench"] = float(preds[tag][0][i])
            row[f"pred_{tag}_calibrated"] = float(preds[tag][1][i])
        if r2_l2 is not None:
            row["r2_profiler_l2"] = float(r2_l2[i])
        res["cases"].append(row)
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    if md:
        with open(md, "w") as f:
            f.write(summary_md(res))
    for tag in preds:
        print(tag, json.dumps({k: v for k, v in res[tag].items() if k.startswith("mae")}), flush=True)
    return res


def summary_md(res: dict) -> str:
    tags = res["tags"]
    L = ["# Validation kernels: first-principles against profiler-derived characterization\n",
         "The recalibration suite's validation kernels, characterized from their algorithms and from "
         "rocprofv3 counters; the same measured times, the shipped microbenchmark parameters and the same "
         f"calibration (Adam, {res['steps']} steps, training split) -- `paper_2605_04178_amd/characterize.py`.\n",
         "Commands (from /tmp with TMPDIR=/tmp and PYTHONPATH=$R; R = repository root; O = an output directory):\n",
         "```\n"
         "python -m paper_2605_04178_amd.characterize run --out $O/T.json\n"
         "rocprofv3 --pmc FETCH_SIZE --output-format csv -d $O/F -o fetch -- "
         "python -m paper_2605_04178_amd.characterize run --out $O/F.json\n"
         "rocprofv3 --pmc WRITE_SIZE --output-format csv -d $O/W -o write -- "
         "python -m paper_2605_04178_amd.characterize run --out $O/W.json\n"
         "rocprofv3 --pmc " + " ".join(L2_COUNTERS) + " --output-format csv -d $O/L -o l2 -- "
         "python -m paper_2605_04178_amd.characterize run --out $O/L.json\n"
         "python -m paper_2605_04178_amd.characterize score --times $O/T.json "
         "--fetch $O/F/fetch_counter_collection.csv --write $O/W/write_counter_collection.csv "
         "--l2 $O/L/l2_counter_collection.csv "
         "--params $R/paper_2605_04178_amd/params/mi355x.json --out $O/result.json --md $O/summary.md\n```\n",
         "Counter scales from the reference copy: " +
         ", ".join(f"{k} {v:.4g}" for k, v in res["scales"].items() if not isinstance(v, list)) + ".\n",
         f"## Mean absolute relative error (all {len(res['cases'])} kernels / held out)\n",
         "| characterization | naive roofline | model, microbenchmark theta | model, calibrated (train) | model, calibrated (held out) |",
         "|---|---|---|---|---|"]
    for tag in tags:
        r = res[tag]
        L.append(f"| {NAMES[tag]} | {r['mae_roofline_all']:.3f} / {r['mae_roofline_holdout']:.3f} | "
                 f"{r['mae_microbench_all']:.3f} / {r['mae_microbench_holdout']:.3f} | "
                 f"{r['mae_calibrated_train']:.3f} | {r['mae_calibrated_holdout']:.3f} |")
    L += ["\n## Per family: bytes against first principles (median ratio) and MAE (microbenchmark / calibrated theta)\n",
          "| family | " + " | ".join(NAMES[t] for t in tags) + " |", "|---|" + "---|" * len(tags)]
    for f, v in res["per_family"].items():
        cells = [f"x{v['bytes_ratio_' + t]:.3g}: {v[t + '_microbench']:.3f} / {v[t + '_calibrated']:.3f}" for t in tags]
        L.append(f"| {f} | " + " | ".join(cells) + " |")
    L += ["\n## Per kernel: bytes and calibrated prediction (us)\n",
          "| kernel | split | measured us | " + " | ".join(NAMES[t] for t in tags) + " |",
          "|---|---|---|" + "---|" * len(tags)]
    for c in res["cases"]:
        cells = [f"{c['B_' + t]:.3g} B, {c['pred_' + t + '_calibrated'] * 1e6:.1f}" for t in tags]
        L.append(f"| {c['name']} | {c['split']} | {c['seconds'] * 1e6:.1f} | " + " | ".join(cells) + " |")
    return "\n".join(L) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--out", required=True)
    r.add_argument("--quick", action="store_true")
    r.add_argument("--launches", type=int, default=100)
    r.add_argument("--warmup", type=int, default=10)
    s = sub.add_parser("score")
    for k in ("times", "fetch", "write", "params", "out"):
        s.add_argument("--" + k, required=True)
    s.add_argument("--steps", type=int, default=2000)
    s.add_argument("--md", default=None)
    s.add_argument("--l2", default=None, help="counter file of the L1-to-L2 requests and L2 hits")
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run(a.out, a.quick, a.launches, a.warmup)
    else:
        score(a.times, a.fetch, a.write, a.params, a.out, a.steps, a.md, a.l2)
    return 0


if __name__ == "__main__":
    sys.exit(main())
