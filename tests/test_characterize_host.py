"""Host logic of the profiler-derived characterization: mapping rocprofv3
counter rows to validation cases and scaling them by the reference copy
(no GPU; synthetic counter files)."""
import csv

import numpy as np
import pytest

from paper_2605_04178_amd import characterize as ch

FIELDS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _rows(counter, kinds, launches, per_case_kib, copy_kib, extra_rows=2, warmup=0):
    """Dispatches as the run step makes them: fills interleaved, each case's
    warm-up + timed launches, then the reference copies; one dispatch split
    over two rows (instances) to exercise the per-dispatch sum."""
    rows, d = [], 0
    for i, k in enumerate(kinds):
        for _ in range(extra_rows):
            d += 1
            rows.append(dict(Correlation_Id=d, Dispatch_Id=d, Kernel_Name="void at::native::fill_kernel(...)",
                             Counter_Name=counter, Counter_Value=123.0))
        for j in range(warmup + 1 + launches):
            d += 1
            v = 1e9 if j <= warmup else per_case_kib[i]     # the warm-ups are skipped
            name = f"(anonymous namespace)::{ch.STEM[k]}(float const*)"
            rows.append(dict(Correlation_Id=d, Dispatch_Id=d, Kernel_Name=name, Counter_Name=counter,
                             Counter_Value=v / 2))
            rows.append(dict(Correlation_Id=d, Dispatch_Id=d, Kernel_Name=name, Counter_Name=counter,
                             Counter_Value=v / 2))
    for _ in range(ch.COPY_REPS):
        d += 1
        rows.append(dict(Correlation_Id=d, Dispatch_Id=d, Kernel_Name="__amd_rocclr_copyBuffer",
                         Counter_Name=counter, Counter_Value=copy_kib))
    return rows


def test_counters_map_to_cases_and_scale(tmp_path):
    kinds = ["copy", "triad", "gemm16", "gemm_mfma"]
    launches = 3
    fk = [100.0, 200.0, 50.0, 10.0]
    wk = [40.0, 80.0, 20.0, 4.0]
    # the counters read half the true traffic for reads, all of it for writes
    _write(tmp_path / "f.csv", _rows("FETCH_SIZE", kinds, launches, fk, ch.COPY_BYTES / 1024 / 2))
    _write(tmp_path / "w.csv", _rows("WRITE_SIZE", kinds, launches, wk, ch.COPY_BYTES / 1024))
    B, info = ch.profiler_bytes(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), kinds, launches)
    assert info["fetch_scale"] == pytest.approx(2.0) and info["write_scale"] == pytest.approx(1.0)
    want = np.array(fk) * 1024 * 2 + np.array(wk) * 1024
    assert np.allclose(B, want)


def test_mismatched_dispatches_are_refused(tmp_path):
    kinds = ["copy", "triad"]
    _write(tmp_path / "f.csv", _rows("FETCH_SIZE", kinds, 3, [1.0, 2.0], 1000.0))
    d = ch.read_dispatches(str(tmp_path / "f.csv"), "FETCH_SIZE")
    with pytest.raises(ValueError):
        ch.per_case(d, kinds, 4)                    # wrong launch count
    with pytest.raises(ValueError):
        ch.per_case(d, ["triad", "copy"], 3)        # cases out of order
    with pytest.raises(ValueError):
        ch.copy_scale([x for x in d if "copyBuffer" not in x[1]])


def test_other_counters_are_ignored(tmp_path):
    rows = _rows("FETCH_SIZE", ["reduce"], 2, [7.0], 100.0)
    rows += [dict(r, Counter_Name="WRITE_SIZE", Counter_Value=1e12) for r in rows]
    _write(tmp_path / "f.csv", rows)
    d = ch.read_dispatches(str(tmp_path / "f.csv"), "FETCH_SIZE")
    assert np.allclose(ch.per_case(d, ["reduce"], 2), [7.0])


def test_l2_requests_and_hit_fraction(tmp_path):
    kinds = ["stencil", "gemm8"]
    launches = 2
    rows = []
    # per case: read / write requests and L2 hits / misses; the copy moves
    # 2^30 bytes each way in 2^24 read and 2^24 write requests (64 B each)
    vals = {"TCP_TCC_READ_REQ_sum": ([1000.0, 4000.0], 2.0 ** 24),
            "TCP_TCC_WRITE_REQ_sum": ([500.0, 100.0], 2.0 ** 24),
            "TCC_HIT_sum": ([300.0, 3000.0], 1.0), "TCC_MISS_sum": ([1200.0, 1100.0], 1.0)}
    for c, (pc, cp) in vals.items():
        rows += _rows(c, kinds, launches, pc, cp, extra_rows=1)
    _write(tmp_path / "l2.csv", rows)
    B, r2, sc = ch.l2_traffic(str(tmp_path / "l2.csv"), kinds, launches)
    assert sc["read_req_bytes"] == pytest.approx(64.0) and sc["write_req_bytes"] == pytest.approx(64.0)
    assert np.allclose(B, [(1000 + 500) * 64.0, (4000 + 100) * 64.0])
    assert np.allclose(r2, [300 / 1500, 3000 / 4100])


def test_warmup_dispatches_are_skipped(tmp_path):
    kinds = ["triad", "bias", "gemm_mfma_bias"]
    _write(tmp_path / "f.csv", _rows("FETCH_SIZE", kinds, 4, [3.0, 5.0, 7.0], 1000.0, warmup=10))
    d = ch.read_dispatches(str(tmp_path / "f.csv"), "FETCH_SIZE")
    assert np.allclose(ch.per_case(d, kinds, 4, warmup=10), [3.0, 5.0, 7.0])
    with pytest.raises(ValueError):
        ch.per_case(d, kinds, 4)                    # the warm-ups must be declared
