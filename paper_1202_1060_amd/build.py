"""Build libndgsbp.so in-tree with hipcc for gfx950.

Usage: python -m paper_1202_1060_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "ndgsbp_host.cpp"),
           os.path.join(HERE, "csrc", "ndgsbp_kernels.hip"),
           os.path.join(HERE, "csrc", "ndgsbp_hbm.hip"),
           os.path.join(HERE, "csrc", "ndgsbp_noalloc.hip")]
OUT = os.path.join(HERE, "libndgsbp.so")
# issue-rate probes of the VALU (the bench's roofline calibration), a library of their own
PROBE_SRC = os.path.join(HERE, "csrc", "ndgsbp_probe.hip")
PROBE_OUT = os.path.join(HERE, "libndgsbp_probe.so")
OBJDIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _run(cmd):
    return subprocess.run(cmd, capture_output=True, text=True)


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.basename(src) + ".o") for src in SOURCES]
    cmds = [[HIPCC, *FLAGS, "-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
    cmds.append([HIPCC, *FLAGS, "-shared", PROBE_SRC, "-o", PROBE_OUT + ".tmp"])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(_run, cmds))
    for res in results:
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed")
        if verbose:
            sys.stderr.write(res.stderr)
    os.replace(PROBE_OUT + ".tmp", PROBE_OUT)
    tmp = OUT + ".tmp"
    res = _run([HIPCC, "--offload-arch=gfx950", "-shared", *objs, "-o", tmp])
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
