"""Host logic of bench.py and of the benchmark workload (CPU only)."""
import subprocess
import sys
from pathlib import Path

import numpy as np

import bench
import scenes

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_measured_traffic_only_for_the_measured_kernels(monkeypatch):
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "source_sha256", bench.kernel_source_hash())
    assert bench.measured_traffic("bin_and_sort") == bench.MEASURED_TRAFFIC["bytes"]["bin_and_sort"]
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "source_sha256", "0" * 64)
    assert bench.measured_traffic("bin_and_sort") is None


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    for sub in ("paper_2506_21117_amd/csrc", "include"):
        (tmp_path / sub).mkdir(parents=True)
    (tmp_path / "include/clsplat.h").write_text("/* doc */ int f(int);\n")
    src = tmp_path / "paper_2506_21117_amd/csrc/k.hip"
    src.write_text("// a kernel\nint f(int x) { return x + 1; }\n")
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    h0 = bench.kernel_source_hash()
    src.write_text("// the kernel, reworded\nint f(int x) {\n  return x + 1;  // same code\n}\n")
    assert bench.kernel_source_hash() == h0
    src.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash() != h0


def test_local_change_ball_around_a_given_centre():
    c = (0.0, 0.0, 0.6)
    w = scenes.local_change(n=20_000, center=c)
    gt = w.scene_gt
    d = np.linalg.norm(gt.means.astype(np.float64) - np.asarray(c)[:, None], axis=0)
    a0 = w.active_begin
    assert np.all(d[a0:] <= 0.4) and np.all(d[:a0] > 0.4)      # static-first: the ball is the suffix
    assert w.name.endswith("-c0,0,0.6")
    w0 = scenes.local_change(n=20_000)
    assert w0.name == "local-20k-1280x720-16v"
