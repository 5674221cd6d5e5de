"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer.

paper_1307_2643_amd/build.py (build_sanitized, run by __graft_entry__.build)
compiles the library's sources with their host code instrumented (device code
as in the library; sanitizers are host-only here) and links them with
tests/sanitize/runtime_driver.cpp, which drives the C-ABI on small problems:
argument checks and error paths, uploads, an all-or-nothing injection
refusal, propagation with a cycle budget and with an overflowing
neutral-record buffer, partial reads, checkpoint/restore against an
uninterrupted run (bitwise), trajectory output, the tuner and its cache,
field evaluation with and without per-call allocation, observables,
refinement patches, the neural field, backtracking with lenses.  Any
sanitizer finding stops the program with a non-zero status."""
import os
import subprocess

import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def test_runtime_clean_under_asan_and_ubsan():
    from paper_1307_2643_amd import build as B
    assert os.path.exists(B.SAN_EXE), "sanitized runtime driver not built (see build_sanitized)"
    env = dict(os.environ)
    # leak checking off: the HIP runtime keeps allocations until the process ends
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    print("running the sanitized runtime driver", flush=True)
    r = subprocess.run([B.SAN_EXE], capture_output=True, text=True, timeout=540, env=env)
    print(r.stdout[-3000:], flush=True)
    print(r.stderr[-6000:], flush=True)
    assert r.returncode == 0, r.returncode
    assert "runtime driver ok" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr
