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


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + ["-I", os.path.join(HERE, "..", "include"), "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


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


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(SAN_DIR, exist_ok=True)
    inc = os.path.join(HERE, "..", "include")
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    objs = []
    for s in SOURCES:
        obj = os.path.join(SAN_DIR, s.replace(".hip", ".o"))
        cmd = [hipcc()] + flags + SAN_HOST + ["-g", "-I", inc, "-c", "-o", obj,
                                              os.path.join(CSRC, s)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
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


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    if "--sanitized" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
