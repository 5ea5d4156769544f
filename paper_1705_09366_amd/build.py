"""Compile the HIP sources into paper_1705_09366_amd/libstkde.so for gfx950.

Every HIP source is compiled with packed-FP32 instruction selection turned
off (``-Xclang -target-feature -Xclang -packed-fp32-ops``); the gather's FP32
accumulation is written as scalar FMA.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstkde.so")
SOURCES = ["ablation.hip", "api.hip", "bin.hip", "gather.hip", "pass.hip", "stats.hip"]
ARCH = os.environ.get("STKDE_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++20", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # matrix-core accumulators in VGPRs: the gather skips untouched blocks
          # with uniform branches, and AGPR accumulators would be copied to
          # VGPRs and back around every one of them
          "-mllvm", "-amdgpu-mfma-vgpr-form",
          "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False, save_temps_dir: str = None) -> str:
    """Compile every source and link the shared library; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()

    def one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = [cc, *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
        if save_temps_dir:
            cmd += ["-save-temps=obj"]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True, cwd=save_temps_dir or objdir)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
