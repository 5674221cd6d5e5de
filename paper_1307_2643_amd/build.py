"""Builds libcrp.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1307_2643_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcrp.so")
SOURCES = ["crp_kernels.hip", "crp_runtime.hip", "crp_nf.hip", "crp_observe.hip",
           "crp_lens.hip"]
ARCH = os.environ.get("CRP_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # every FP operation is one IEEE operation in source order
    "-ffp-contract=off", "-fno-fast-math",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc():
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


OBJ_DIR = os.path.join(HERE, "_obj")


def _run_parallel(cmds, verbose: bool) -> None:
    """Runs the commands, at most CRP_BUILD_JOBS (default: the CPU count, at
    most 16) at a time; raises CalledProcessError for the first that fails."""
    jobs = int(os.environ.get("CRP_BUILD_JOBS", os.cpu_count() or 4))
    jobs = max(1, min(jobs, 16, len(cmds)))
    pending, running, failed = list(cmds), [], None
    while pending or running:
        while pending and failed is None and len(running) < jobs:
            cmd = pending.pop(0)
            if verbose:
                print(" ".join(cmd), flush=True)
            running.append((cmd, subprocess.Popen(cmd)))
        cmd, proc = running.pop(0)
        if proc.wait() != 0 and failed is None:
            failed = subprocess.CalledProcessError(proc.returncode, cmd)
            pending.clear()
    if failed is not None:
        raise failed


def _lib_objects():
    """(compile commands, object paths) of libcrp.so's sources."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    flags = [f for f in FLAGS if f != "-shared"]
    inc = os.path.join(HERE, "..", "include")
    cmds, objs = [], []
    for s in SOURCES:
        obj = os.path.join(OBJ_DIR, s.replace(".hip", ".o"))
        cmds.append([hipcc()] + flags + ["-I", inc, "-c", "-o", obj, os.path.join(CSRC, s)])
        objs.append(obj)
    return cmds, objs


def _link_lib(objs, verbose: bool) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def build(verbose: bool = False) -> str:
    cmds, objs = _lib_objects()
    _run_parallel(cmds, verbose)
    return _link_lib(objs, verbose)


# The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer: the
# library's sources with their host code instrumented (device code as in the
# library: the sanitizers are host-only here), linked with the C-ABI driver
# tests/sanitize/runtime_driver.cpp into one executable for the GPU test.
SAN_DIR = os.path.join(HERE, "_sanitize")
SAN_EXE = os.path.join(SAN_DIR, "crp_runtime_sanitized")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]
SAN_LINK = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def _sanitized_objects():
    """(compile commands, object paths) of the sanitizer build's sources."""
    os.makedirs(SAN_DIR, exist_ok=True)
    inc = os.path.join(HERE, "..", "include")
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    cmds, objs = [], []
    for s in SOURCES:
        obj = os.path.join(SAN_DIR, s.replace(".hip", ".o"))
        cmds.append([hipcc()] + flags + SAN_HOST + ["-g", "-I", inc, "-c", "-o", obj,
                                                    os.path.join(CSRC, s)])
        objs.append(obj)
    return cmds, objs


def build_sanitized(verbose: bool = False) -> str:
    cmds, objs = _sanitized_objects()
    _run_parallel(cmds, verbose)
    return _link_sanitized(objs, verbose)


def _link_sanitized(objs, verbose: bool) -> str:
    inc = os.path.join(HERE, "..", "include")
    # host link (no HIP source on this line): ROCm's clang, whose sanitizer
    # runtime matches the instrumented objects
    clang = os.path.join(os.path.dirname(hipcc()), "..", "llvm", "bin", "clang++")
    driver = os.path.join(HERE, "..", "tests", "sanitize", "runtime_driver.cpp")
    rocm_lib = os.path.join(os.path.dirname(hipcc()), "..", "lib")
    tmp = SAN_EXE + ".tmp"
    link = [clang, "-std=c++17", "-O1", "-g"] + SAN_LINK + [
        "-I", inc, "-o", tmp, driver] + objs + [
        "-L" + rocm_lib, "-lamdhip64", "-Wl,-rpath," + rocm_lib]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, SAN_EXE)
    return SAN_EXE


def build_all(verbose: bool = False):
    """libcrp.so and the sanitizer build, their objects compiled in one pool."""
    lib_cmds, lib_objs = _lib_objects()
    san_cmds, san_objs = _sanitized_objects()
    _run_parallel(lib_cmds + san_cmds, verbose)
    return _link_lib(lib_objs, verbose), _link_sanitized(san_objs, verbose)


if __name__ == "__main__":
    if "--sanitized" in sys.argv:
        print(build_all(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
