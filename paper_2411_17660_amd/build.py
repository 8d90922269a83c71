"""Compile the HIP sources into paper_2411_17660_amd/libgsr.so for gfx950.

Every source is built with hipcc for gfx950 only, -O3, with the packed-FP32
instruction forms disabled (they are not used by this code and are kept out
of the binary on purpose).  The library is built in-tree so that it travels
with the source tree.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgsr.so")
SOURCES = ["runtime.hip", "preprocess.hip", "sort.hip", "raster.hip", "loss.hip", "ssim.hip", "densify.hip", "surfel.hip", "normals.hip", "adam.hip", "host_check.cpp"]
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _obj(src, outdir):
    return os.path.join(outdir, os.path.splitext(src)[0] + ".o")


def build(verbose=False, jobs=None):
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)

    def compile_one(src):
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", _obj(src, outdir)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return src

    with ThreadPoolExecutor(max_workers=jobs or min(len(SOURCES), os.cpu_count() or 4)) as ex:
        list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
        [_obj(s, outdir) for s in SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
