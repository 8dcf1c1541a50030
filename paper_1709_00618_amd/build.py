"""Build the gfx950 shared library libtpcca.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtpcca.so")
SOURCES = ["tpcca_kernels.hip", "tpcca_fit_rows.hip", "tpcca_runtime.hip", "tpcca_server.hip", "tpcca_phase2.hip"]
HEADERS = ["tpcca_internal.h", "tpcca_kernels.h", "tpcca_dev.h", "tpcca_kf.h", "tpcca_fit.h", "tpcca_runtime.h", "tpcca_phase2.h"]
ARCH = os.environ.get("TPCCA_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off and correctly rounded FP32 divide/sqrt: the kernels must
# reproduce the IEEE operation sequence of the tracker bit for bit.
# Packed FP32 instructions are disabled (-packed-fp32-ops).
HIPFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result", f"-I{INCLUDE}", f"-I{CSRC}",
]


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link libtpcca.so next to this file."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [_hipcc(), *HIPFLAGS, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
        objs.append(obj)
    for p, src in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{text}")
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


MEMBENCH = os.path.join(HERE, "membench")


def build_membench(verbose: bool = False) -> str:
    """The random-access ceilings microbenchmark: a measurement tool, not part
    of the library; built only by bench.py --ceilings."""
    tmp = MEMBENCH + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", os.path.join(CSRC, "membench.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if out.returncode != 0:
        raise RuntimeError("hipcc failed on membench.hip:\n" + out.stdout.decode(errors="replace"))
    os.replace(tmp, MEMBENCH)
    return MEMBENCH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
