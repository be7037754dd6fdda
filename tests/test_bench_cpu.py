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


def _step_names(second_slab):
    return (["preprocess_kernel", "clear_kernel", "count_kernel", "rs_downsweep_kernel", "emit_kernel<true, true>",
             "render_forward_kernel<1>"]
            + (["emit_kernel<true, true>", "render_forward_kernel<2>"] if second_slab else [])
            + ["l1_loss_grad_kernel", "render_backward_kernel", "preprocess_backward_kernel", "adam_kernel"])


def _synthetic_trace():
    """Three steps (the second with a second depth slab) after a warm-up fragment and
    torch's own kernels, each dispatch 1000 ns long and 500 ns after the previous one."""
    names = ["adam_kernel", "at::native::fill"]
    for s in range(3):
        names += _step_names(s == 1) + ["at::native::copy"]
    names += ["preprocess_kernel", "clear_kernel"]  # an unfinished step
    rows, t = [], 0
    for n in names:
        rows.append((f"void clsp::(anonymous namespace)::{n}(int, float*)", t, t + 1000, 1000))
        t += 1500
    return rows


def test_step_split_assigns_each_kernel_to_its_call():
    seq = [(bench.short_kernel_name(n), s, e, d) for n, s, e, d in _synthetic_trace()]
    steps = bench.split_steps(seq, 10)
    assert len(steps) == 3
    for j, (disp, calls) in enumerate(steps):
        assert [x[0] for x in disp] == _step_names(j == 1)
        assert [x[0] for x in calls["bin_and_sort"]] == ["clear_kernel", "count_kernel", "rs_downsweep_kernel",
                                                         "emit_kernel<true, true>"]
        assert calls["render_forward"][0][0] == "render_forward_kernel<1>"
        assert calls["render_forward"][-1][0] == ("render_forward_kernel<2>" if j == 1 else "render_forward_kernel<1>")
        assert [x[0] for x in calls["render_backward"]] == ["render_backward_kernel", "preprocess_backward_kernel"]
    assert len(bench.split_steps(seq, 2)) == 2 and bench.split_steps(seq, 2)[0][0] == steps[1][0]


def test_trace_summary_of_a_synthetic_database(tmp_path):
    import sqlite3

    db = tmp_path / "t_results.db"
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, start integer, end integer, duration integer)")
    con.executemany("insert into kernels values (?, ?, ?, ?)", _synthetic_trace())
    con.commit()
    con.close()
    out = bench.summarize_trace(str(db), 3, ["a note"])
    lines = out.splitlines()
    assert lines[0] == "# a note"
    # 10, 12, 10 dispatches of 1 us each
    assert "(32 dispatches)" in lines[1] and "sum of kernel durations): 10.7 us" in lines[2]
    row = {ln.split()[0]: ln.split() for ln in lines if ln.startswith("emit_kernel")}
    assert row["emit_kernel<true,"][2] == "1.3"  # calls per step: 4 over 3 steps
    fwd = [ln for ln in lines if "render_forward " in ln and "kernels" in ln][0]
    # 1, 3 (phase 1, the second slab's listing, phase 2) and 1 kernels; spans 1, 4 and 1 us
    assert "1.7 kernels" in fwd and "sum      1.7 us" in fwd and "span      2.0 us" in fwd


def test_traffic_summary_scales_by_the_copy_calibration(tmp_path):
    import csv

    def write(folder, counter, seq):
        (tmp_path / folder / "box").mkdir(parents=True)
        with open(tmp_path / folder / "box" / "x_counter_collection.csv", "w", newline="") as fh:
            w = csv.DictWriter(fh, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for i, (n, v) in enumerate(seq):
                w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": n, "Counter_Name": counter, "Counter_Value": v})

    seq = [(n, 0) for n in ("adam_kernel",)]
    for s in range(2):
        seq += [(n, {"preprocess_kernel": 100, "count_kernel": 10, "render_forward_kernel<1>": 20,
                     "render_backward_kernel": 30, "adam_kernel": 5}.get(n, 1)) for n in _step_names(False)]
    write("f", "FETCH_SIZE", seq)
    write("w", "WRITE_SIZE", [(n, 2 * v) for n, v in seq])
    write("cf", "FETCH_SIZE", [("copyBuffer", 131072.0)] * 3)
    write("cw", "WRITE_SIZE", [("copyBuffer", 262144.0)] * 3)
    out = bench.summarize_traffic(*(str(tmp_path / d) for d in ("f", "w", "cf", "cw")), k=10)
    assert "factor 2.000" in out and "factor 1.000" in out
    rows = {ln.split()[0]: [float(x) for x in ln.split()[2::3][:3]] for ln in out.splitlines()
            if not ln.startswith("#")}
    # bin_and_sort: clear 1 + count 10 + downsweep 1 + emit 1 = 13 KiB fetch (x2), 26 KiB write (x1)
    assert rows["bin_and_sort"] == [round(13 * 1024 * 2 / 1e6, 3), round(26 * 1024 / 1e6, 3),
                                    round(2 * 26 * 1024 / 1e6, 3)]
    # render_backward: the raster backward (30) and the preprocess backward (1)
    assert rows["render_backward"][0] == round(31 * 1024 * 2 / 1e6, 3)
    step_fetch = (100 + 1 + 10 + 1 + 1 + 20 + 1 + 30 + 1 + 5) * 1024 * 2 / 1e6
    assert rows["step"][0] == round(step_fetch, 3)


def test_step_split_of_a_fused_local_step():
    """Local steps compute the L1 gradient in the forward and Adam in the preprocess
    backward: the step ends there and the backward call starts after the forward."""
    names = ["preprocess_kernel", "count_kernel", "emit_kernel<true, true>", "render_forward_kernel<1>",
             "recount_kernel", "render_forward_kernel<2>", "fill_u32_kernel", "render_backward_kernel",
             "preprocess_backward_adam_kernel"]
    seq = [(n, 1000 * i, 1000 * i + 500, 500) for i, n in enumerate(names * 2)]
    steps = bench.split_steps(seq, 10)
    assert len(steps) == 2
    disp, calls = steps[0]
    assert [x[0] for x in disp] == names
    assert [x[0] for x in calls["bin_and_sort"]] == ["count_kernel", "emit_kernel<true, true>"]
    assert [x[0] for x in calls["render_forward"]] == names[3:6]
    assert [x[0] for x in calls["render_backward"]] == names[6:]
