"""Host-side parts of bench.py's output contract (no GPU).

- roofline.traffic comes from the committed HBM-counter summary only while the
  compositing sources are byte-identical to those the counters were taken
  on, and is None otherwise;
- more than one GPU is refused with a message (this build measures one);
- the sort object's arithmetic: algorithmic bytes per key over the stage time.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _copy_sources(dst):
    for rel in bench.COMPOSITING_SOURCES:
        os.makedirs(os.path.join(dst, os.path.dirname(rel)), exist_ok=True)
        shutil.copyfile(os.path.join(ROOT, rel), os.path.join(dst, rel))


def test_traffic_is_tied_to_the_compositing_sources(tmp_path, monkeypatch):
    root = str(tmp_path)
    _copy_sources(root)
    os.makedirs(os.path.join(root, "profiles"))
    sha = bench.compositing_sources_sha256(root)
    line = f"    traffic composite_bwd_kernel<16, 16> bytes_per_launch=123456 " \
           f"compositing_sources_sha256={sha}\n"
    with open(os.path.join(root, "profiles", "c3_hbm_traffic_pmc.md"), "w") as f:
        f.write("summary\n" + line)
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.measured_traffic("composite_bwd", (16, 16)) == 123456
    # another kernel or tile shape: no figure
    assert bench.measured_traffic("composite_fwd", (16, 16)) is None
    assert bench.measured_traffic("composite_bwd", (32, 16)) is None
    # one byte changed in a header the kernels include: the figure is stale
    hdr = os.path.join(root, "paper_2411_17660_amd", "csrc", "gsr_device.h")
    with open(hdr, "ab") as f:
        f.write(b"\n")
    assert bench.measured_traffic("composite_bwd", (16, 16)) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("K,t_sort,t_key,t_rng", [(85_237_737, 0.6107, 0.2049, 0.0449),
                                                  (1_000, 1.0, 1.0, 1.0)])
def test_sort_roofline_arithmetic(K, t_sort, t_key, t_rng):
    stages = {"tile_sort": (2 * t_sort, 2), "keygen": (t_key, 1), "ranges": (3 * t_rng, 3)}
    achievable = {"GBps": 6200.0}
    s = bench.sort_roofline(stages, K, achievable)
    gbs = 24 * K / (t_sort * 1e-3) / 1e9
    assert s["achieved_GBps"] == pytest.approx(gbs, abs=0.05)
    assert s["frac"] == pytest.approx(gbs / 8000.0, abs=1e-4)
    assert s["frac_of_achievable"] == pytest.approx(gbs / 6200.0, abs=1e-4)
    t_all = t_key + t_sort + t_rng
    assert s["lists"]["ms"] == pytest.approx(t_all, abs=1e-4)
    assert s["lists"]["achieved_GBps"] == pytest.approx(44 * K / (t_all * 1e-3) / 1e9, abs=0.05)
