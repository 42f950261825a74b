"""The oracle's CPU pins re-run against a build of the oracle under
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code only), in a
child process that preloads the sanitizer runtimes.  Any out-of-bounds
access, use after free, signed overflow, misaligned access or invalid shift
in the oracle aborts that process and fails this test.  The two noisy
2^20-descriptor calibration runs are left out for time; the noiseless
calibration, identifiability and every other pin run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    from oracle import build as orc_build
    so = orc_build.build_variant(str(tmp_path / "liboracle_san.so"), extra_flags=SAN_FLAGS)
    env = dict(os.environ)
    env.update(WM_ORACLE_LIB=so, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    # the child loads the variant, and the variant is instrumented
    probe = ("import oracle, ctypes; L = oracle.lib(); print(L._name); "
             "print(hasattr(L, '__asan_report_load8'))")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    name, instrumented = r.stdout.split()
    assert name == so and instrumented == "True", r.stdout
    files = ["tests/test_oracle_pins.py", "tests/test_oracle_latency_overhead.py", "tests/test_oracle_segments.py",
             "tests/test_oracle_blackwell.py", "tests/test_oracle_planning.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-p", "no:xdist",
                        "-m", "not gpu", "-k", "not noisy_recovery and not planted_mistake"] + files,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    print(r.stdout.strip().splitlines()[-1])
