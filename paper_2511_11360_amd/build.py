"""Build libpflbm.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2511_11360_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libpflbm.so")
OBJDIR = os.path.join(HERE, "_build")

# (source, object name, extra defines); the step kernel is instantiated once per
# lattice pair and phase-field model, each in its own compilation (in parallel)
PAIRS = (0, 1, 2)
MODELS = (0, 1, 2, 3, 4)
SOURCES = ([("kernels.hip", "kernels", []), ("adjoint.hip", "adjoint", []), ("pflbm.cpp", "pflbm", []),
            ("probe.hip", "probe", [])]
           + [("step_inst.hip", "step_p%d_m%d" % (p, m), ["-DPFK_PAIR=%d" % p, "-DPFK_MODEL=%d" % m])
              for p in PAIRS for m in MODELS])

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed fp32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _compile(item):
    src, name, defines = item
    obj = os.path.join(OBJDIR, name + ".o")
    cmd = [HIPCC, "-x", "hip"] + FLAGS + defines + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-8000:]))
    return obj


def build(verbose=True):
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-8000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
