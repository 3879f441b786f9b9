"""Compile libcountgauss.so for gfx950 with hipcc (in-tree, no JIT cache).

Each HIP source is compiled to an object in _build/ (in parallel), then
linked into paper_1606_05732_amd/libcountgauss.so.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libcountgauss.so")
ARCH = os.environ.get("CG_OFFLOAD_ARCH", "gfx950")

SOURCES = ["cg_sx_atomic.hip", "cg_sx_sorted.hip", "cg_sx_binned.hip", "cg_gsx.hip", "cg_adjoint.hip",
           "cg_batched.hip", "cg_anchors.hip", "cg_lemma.hip",
           "cg_stream.hip", "cg_capi.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-munsafe-fp-atomics",
    # MFMA results in ordinary VGPRs: gfx950's register file is unified, and
    # with accumulators in AGPRs the allocator copies some of them between
    # register classes on every loop iteration (the FP32 contraction and
    # G^T dY lose those copies and gain occupancy this way)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    # no packed-FP32 instructions in the device code (the host pass does not
    # know the feature and warns; tests/test_build_no_packed_fp32.py checks
    # the device assembly)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return exe


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    # the host pass's warning about the packed-FP32 feature (device code is
    # checked by tests/test_build_no_packed_fp32.py)
    noise = "'-packed-fp32-ops' is not a recognized feature for this target"
    warn = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    return obj, warn


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 8)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = []
    for obj, warn in results:
        objs.append(obj)
        if verbose and warn.strip():
            print(warn, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
