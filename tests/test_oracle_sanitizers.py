"""The CPU oracle under the address and undefined-behaviour sanitizers: a
driver (oracle/sanitize_check.c) runs every oracle entry point on small
channels (ghost rows at both walls, a 4-row lattice, unequal properties, a
perturbed start); the sanitized build must exit cleanly with no report.
Host code only (gcc); skipped where the toolchain lacks the sanitizer
runtimes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "sanitize_check")
    src = [os.path.join(ROOT, "oracle", "sanitize_check.c"), os.path.join(ROOT, "oracle", "lbm_oracle.c")]
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    r = subprocess.run([gcc] + flags + src + ["-o", exe, "-lm"], capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr or "ubsan" in r.stderr):
        pytest.skip("sanitizer runtimes not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr, run.stderr
    assert run.stdout.count("rc 0") == 3
