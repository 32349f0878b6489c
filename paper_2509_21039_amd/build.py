"""Builds libhfk.so for gfx950 with hipcc (in-tree, next to this file).

    python -m paper_2509_21039_amd.build

Each .hip source under csrc/ is compiled separately (parallel), then linked into one shared
library.  FP64 code is built without fast-math; packed FP32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libhfk.so")
PROBE = os.path.join(HERE, "valu_probe")
OBJDIR = os.path.join(HERE, "_build")

ARCH = os.environ.get("HFK_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]

SOURCES = ["hfk_api.hip", "hfk_prep.hip", "hfk_fock.hip", "hfk_grad.hip", "hfk_batched.hip", "hfk_scf.hip"]
# dense products and symmetric eigenproblems of the SCF loop
LIBS = ["-L/opt/rocm/lib", "-lrocblas", "-lrocsolver", "-Wl,-rpath,/opt/rocm/lib"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    if r.stderr.strip():
        # warnings other than the host pass not knowing the packed-fp32 feature
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, *LIBS]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, OUT)
    # the VALU throughput probe: a stand-alone measurement program (bench.py --valu-probe)
    probe_tmp = PROBE + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, os.path.join(CSRC, "valu_probe.hip"), "-o", probe_tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for valu_probe.hip:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(probe_tmp, PROBE)
    if verbose:
        print("built", OUT, "and", PROBE)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
