"""Build of the HIP libraries for gfx950 (hipcc, in-tree): libadg.so (the method) and
libadg_peaks.so (the copy and FP64 ceiling probes of the roofline)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libadg.so")
SOURCES = ["adg_api.hip", "adg_problem.hip", "adg_batch.hip", "adg_euler.hip", "adg_ns.hip"]
PEAKS_LIB = os.path.join(HERE, "libadg_peaks.so")
PEAKS_SOURCES = ["adg_peaks.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of all HIP code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _link(lib: str, sources: list[str], verbose: bool) -> str:
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = lib + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-o", tmp, *srcs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    _link(PEAKS_LIB, PEAKS_SOURCES, verbose)
    return _link(LIB, SOURCES, verbose)
