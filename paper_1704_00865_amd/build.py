"""Build libwf.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

    python -m paper_1704_00865_amd.build        # or build() from Python
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libwf.so")
BUILD_DIR = os.path.join(PKG, "_build")

# (source, object, extra defines): the sweep kernels are compiled in three
# parts in parallel (float32 default tiling, float64, float32 other tilings)
SOURCES = [("wf_kernels.hip", "wf_kernels_f32.o", ("WF_PART=1",)),
           ("wf_kernels.hip", "wf_kernels_f64.o", ("WF_PART=2",)),
           ("wf_kernels.hip", "wf_kernels_tuned.o", ("WF_PART=4",)),
           ("wf_runtime.cpp", "wf_runtime.o", ()),
           ("wf_nn.hip", "wf_nn.o", ())]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 4, defines=(), out: str = LIB,
          build_dir: str = BUILD_DIR) -> str:
    """Compile every source for gfx950 and link the shared library.  Always
    recompiles (objects go to a temporary folder that is removed after).
    ``defines`` are extra -D options; ``out`` the library path."""
    hipcc = _hipcc()
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    procs = []
    for src, oname, part in SOURCES:
        obj = os.path.join(build_dir, oname)
        objs.append(obj)
        cmd = [hipcc, "-x", "hip", *HIPCC_FLAGS, *[f"-D{d}" for d in (*part, *defines)],
               "-I", INCLUDE, "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    while procs:
        _wait(procs.pop(0))
    tmp = out + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    _wait((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    os.replace(tmp, out)
    shutil.rmtree(build_dir, ignore_errors=True)
    return out


def _wait(item):
    cmd, p = item
    out, _ = p.communicate()
    if p.returncode != 0:
        sys.stderr.write(out)
        raise RuntimeError(f"build step failed ({p.returncode}): {' '.join(cmd)}")
    lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose=True))
