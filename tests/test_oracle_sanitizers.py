"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/oracle_driver.c drives every path of the oracle (both
precision forms and grid types, interactions with full record buffers, an
observer, far-flung fixed steps, refinement patches, the analytic field with
backtracking, per-step output past its capacity, cycle caps, and the
single-call entry points at non-finite and extreme values).  It is built twice
with gcc: with -fsanitize=address,undefined (any finding aborts the run) and
plainly as the oracle library is built; both must finish and print the same
counters and output checksums."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")
ORACLE = os.path.join(ROOT, "oracle", "crp_oracle.c")
COMMON = ["-std=gnu11", "-Wall", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-I", os.path.join(ROOT, "oracle"), DRIVER, ORACLE, "-lm"]


def _build(out, extra):
    subprocess.check_call(["gcc"] + extra + COMMON + ["-o", out])


@pytest.mark.slow
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    san = str(tmp_path / "driver_san")
    plain = str(tmp_path / "driver_plain")
    _build(san, ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=all"])
    _build(plain, ["-O2"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    rs = subprocess.run([san], capture_output=True, text=True, env=env, timeout=600)
    assert rs.returncode == 0, rs.stderr[-4000:]
    assert "runtime error" not in rs.stderr and "ERROR: AddressSanitizer" not in rs.stderr
    assert rs.stdout.rstrip().endswith("DRIVER DONE")
    rp = subprocess.run([plain], capture_output=True, text=True, timeout=600)
    assert rp.returncode == 0, rp.stderr[-2000:]
    # the same results with and without the sanitizers
    assert rs.stdout == rp.stdout
    # the scenarios did reach the paths they are meant to exercise
    lines = {ln.split(":")[0]: ln for ln in rs.stdout.splitlines() if ":" in ln}
    assert " neu_dropped 0 " not in lines["fp64_grid64"]
    assert " fin_dropped 0 " not in lines["fin_overflow"]
    assert " traj_dropped 0 " not in lines["traj_overflow"]
    assert " boundary 0 " not in lines["galactic_back"]
    assert " active 0 " not in lines["cycle_cap"]
    assert " forced 0 " not in lines["fixed_step_far"]
