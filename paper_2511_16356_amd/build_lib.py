"""Build the gfx950 shared library ``libkc_mi355x.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkc_mi355x.so")
SOURCES = ["kc_device.hip", "kc_host.cpp", "kc_static.hip", "kc_batch.cpp", "kc_tune.cpp"]
# memory-ceiling probes used by the benchmark's roofline calibration
PROBE_LIB = os.path.join(HERE, "libkc_probe.so")
PROBE_SOURCES = ["kc_probe.hip"]
HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions (v_pk_add/mul/fma_f32): the library is built without them
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return exe


def build(verbose: bool = False) -> str:
    """Compile every HIP/C++ source of both libraries (always recompiles)."""
    _build_one(PROBE_LIB, PROBE_SOURCES, verbose)
    return _build_one(LIB, SOURCES, verbose)


def _build_one(lib: str, sources, verbose: bool) -> str:
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(HERE, "..", "include"), "-o", tmp] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature; that is expected
    noise = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(noise))
    if noise and verbose:
        print("\n".join(noise), file=sys.stderr)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
