"""Host code under the address and undefined-behaviour sanitizers (CPU).

1. The host-side argument checks and frame-table layout of the C-ABI calls
   (paper_2411_17660_amd/csrc/host_check.cpp, the code runtime.hip runs
   before any device work) built with g++ -fsanitize=address,undefined and
   driven over valid, invalid and extreme arguments
   (tests/host_check_main.cpp).
2. The FP64 oracle (oracle/gsr_ref.c) built the same way and run, in a child
   process with the sanitizer runtime preloaded, over small scenes that reach
   its edge cases: empty and fully culled scenes, Gaussians outside the
   Jacobian guard, non-finite parameters, ragged multi-frame batches, every
   tile shape, the FP64-input and median-depth entry points, and the
   backward with its screen-space gradients.

A sanitizer report, or any check that fails, ends the child with a non-zero
status (-fno-sanitize-recover)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_17660_amd", "csrc")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=all"]


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                         text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.fixture(scope="module")
def asan_env():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=24"
    env["OMP_NUM_THREADS"] = "4"
    return env


def test_host_checks_under_sanitizers(tmp_path):
    exe = tmp_path / "host_check"
    cmd = ["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(ROOT, "tests", "host_check_main.cpp"),
           os.path.join(CSRC, "host_check.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().splitlines()[-1].startswith("ok ")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


ORACLE_RUN = r'''
import sys
import numpy as np
sys.path.insert(0, {root!r})
import oracle.ref as ref
from paper_2411_17660_amd import scenes
ref.use_library({lib!r})

def run(sc, **kw):
    fw = ref.forward(sc, threads=2, **kw)
    rec = fw.records(); start, ent = fw.tile_lists(); flags, nl, tf = fw.pixel_info()
    P = sc.n_pixels
    rng = np.random.default_rng(0)
    g = fw.backward(rng.normal(size=3 * P), rng.normal(size=P), rng.normal(size=P))
    sg = fw.screen_grads()
    for k, v in g.items():
        assert np.all(np.isfinite(v)), k
    return fw

cases = 0
for tile in [(16, 16), (8, 8), (32, 8), (16, 8), (32, 16)]:
    run(scenes.tiny_scene(seed=1, n=60, W=45, H=37, n_frames=2), tile=tile); cases += 1
run(scenes.tiny_scene(seed=2, n=0)); cases += 1
run(scenes.tiny_scene(seed=3, n=40, outside=(1.2, 3.0), ls_mean=-1.0)); cases += 1
sc = scenes.tiny_scene(seed=4, n=30, zrange=(-3.0, -1.0)); run(sc); cases += 1
sc = scenes.tiny_scene(seed=5, n=50, n_frames=3)
sc.means[3, 1] = np.nan; sc.log_scales[7, 0] = np.inf; sc.sh[9, 4, 2] = np.nan
run(sc); cases += 1
run(scenes.tiny_scene(seed=6, n=50, W=1, H=1)); cases += 1
run(scenes.tiny_scene(seed=7, n=80, W=61, H=29, n_frames=2), f64=True); cases += 1
run(scenes.tiny_scene(seed=8, n=80, W=50, H=40, n_frames=2), median=True); cases += 1
run(scenes.scene_c1(seed=0, n=400)); cases += 1
print("ok", cases)
'''


def test_oracle_under_sanitizers(tmp_path, asan_env):
    lib = tmp_path / "libgsr_ref_san.so"
    cmd = ["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", *SAN, os.path.join(ROOT, "oracle", "gsr_ref.c"),
           "-o", str(lib), "-lm"]
    subprocess.run(cmd, check=True)
    script = ORACLE_RUN.format(root=ROOT, lib=str(lib))
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True,
                       env=asan_env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip().splitlines()[-1].startswith("ok ")
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


CONTROL = r'''
import ctypes, sys
lib = ctypes.CDLL({lib!r})
lib.read_past_end.argtypes = [ctypes.c_int]
print(lib.read_past_end(4))
'''


def test_sanitizer_harness_catches_an_overrun(tmp_path, asan_env):
    """Control: the same build flags and preload report a heap overrun in a
    library loaded by a child Python process (so a clean run above means
    something)."""
    src = tmp_path / "overrun.c"
    src.write_text("#include <stdlib.h>\n"
                   "int read_past_end(int i) { int* p = malloc(4 * sizeof(int));\n"
                   "  for (int k = 0; k < 4; ++k) p[k] = k;\n"
                   "  int v = p[i]; free(p); return v; }\n")
    lib = tmp_path / "liboverrun.so"
    subprocess.run(["gcc", "-fPIC", "-shared", *SAN, str(src), "-o", str(lib)], check=True)
    r = subprocess.run([sys.executable, "-c", CONTROL.format(lib=str(lib))],
                       capture_output=True, text=True, env=asan_env, timeout=120)
    # either sanitizer may report it first (UBSan's object-size check, or
    # ASan's heap-buffer-overflow); both end the child with their exit code
    assert r.returncode in (23, 24), (r.returncode, r.stderr[-2000:])
    assert "heap-buffer-overflow" in r.stderr or "runtime error" in r.stderr
