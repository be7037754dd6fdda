"""Benchmark: one local-optimisation step of CL-Splats' hot path on one MI355X.

Workload: 1M Gaussians (means uniform in [-1, 1]^3, SH degree 0), the Gaussians within
0.4 of the origin form the change set (re-initialised as new points and stored last),
16 ring views of 1280x720; targets are renders of the unchanged scene.  A step is one
view: zero grads -> preprocess -> mask + binning -> forward -> L1 gradient -> backward
-> masked Adam.  The local step (mask + change-set-only backward and Adam) is timed,
then the full-scene step on the same views for comparison.

Prints ONE JSON line.  `value` is local steps per second.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1_000_000, help="Gaussians (default: the 1M workload)")
    ap.add_argument("--no-full", action="store_true", help="skip the full-scene comparison")
    ap.add_argument("--only-full", action="store_true", help="time only the full-scene step (profiling)")
    ap.add_argument("--only-visible", action="store_true",
                    help="time only the local step with the change ball on the cube face z = +1 (profiling)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="time budget of the CPU oracle timing")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving latency leg")
    ap.add_argument("--no-visible", action="store_true",
                    help="skip the local leg whose change ball sits on the cube face z = +1 (visible)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests per arrival rate of the serving sweep (closed loop, then Poisson at 0.25, 0.5 "
                         "and 0.8 of the closed-loop rate)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the one-off timing of the full-scene (200k, SH3, 8 x 800x800) and differentiation "
                         "(3M, SH3, 4 x 1920x1080) workloads")
    ap.add_argument("--cpu-single", action="store_true",
                    help="also time one complete oracle local step on one thread")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 10 times (the reference kernel of known size for "
                         "the HBM byte counters) and exit")
    ap.add_argument("--summarize-trace", metavar="DB",
                    help="print per-step kernel averages and per-call sums from the results database of a "
                         "rocprofv3 --kernel-trace run of this script, and exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="print per-kernel averages of the counters in the output folders of rocprofv3 --pmc "
                         "--output-format csv runs of the step")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="print per-call HBM bytes from the output folders of four rocprofv3 --pmc runs "
                         "(FETCH_SIZE and WRITE_SIZE of this script, then of --copy-calibration), and exit")
    ap.add_argument("--summary-steps", type=int, default=10, help="steps (the last ones) a summary averages over")
    ap.add_argument("--summary-note", action="append", default=[], help="a header line of the summary (repeatable)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.summary_steps, args.summary_note))
        return 0
    if args.summarize_counters:
        print(summarize_counters(args.summarize_counters, k=args.summary_steps, notes=args.summary_note))
        return 0
    if args.summarize_traffic:
        print(summarize_traffic(*args.summarize_traffic, k=args.summary_steps, notes=args.summary_note))
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (this build runs on a single "
              "MI355X; see the design notes for how the step would shard).", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import scenes
    from paper_2506_21117_amd import api
    from paper_2506_21117_amd.optim import SplatOptimizer

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 10 copies of 256 MiB (268435456 B read and written per copy)")
        return 0
    t0 = time.time()
    w = scenes.local_change(n=args.n)
    sc, cams = w.scene, w.cameras
    a = (w.active_begin, sc.n)
    log(f"scene {w.name}: N={sc.n} active={a[1] - a[0]} built in {time.time() - t0:.1f}s")

    def render_targets(wl):
        """Renders of the unchanged scene (inputs, not timed)."""
        gt = api.GaussianTensors.from_scene(wl.scene_gt, dev)
        tg = torch.zeros(len(wl.cameras), 3, wl.cameras[0].height, wl.cameras[0].width, device=dev)
        proj = api.ProjectedBuffers.alloc(wl.scene.n, 1, dev)
        bins = None
        for v, cam in enumerate(wl.cameras):
            api.project_preprocess(gt, [cam], proj)
            bins = api.bin_and_sort(proj, [cam], bins=bins, capacity=120_000_000)
            api.render_forward(proj, bins, [cam], image=tg[v:v + 1],
                               T_final=torch.empty(1, cam.height, cam.width, device=dev),
                               n_contrib=torch.empty(1, cam.height, cam.width, dtype=torch.int32, device=dev))
            assert not bins.read_counters()["overflow"]
        torch.cuda.synchronize()
        return tg

    targets = render_targets(w)
    log("targets rendered")

    order = np.random.default_rng(0).permutation(len(cams))
    calls = SplatOptimizer.TIMED_CALLS

    def run(local, sc=sc, targets=targets, a=a, steps=args.steps):
        """Warm-up steps time every call with HIP events (recorded on the stream the
        calls run on) and pick the dominant one; the timed steps record events around
        that call only (events cost time of their own)."""
        params = api.GaussianTensors.from_scene(sc, dev)
        opt = SplatOptimizer(params, cams, targets, active=a, local=local)
        stream = torch.cuda.current_stream()
        mk = lambda: torch.cuda.Event(enable_timing=True)
        warm = max(args.warmup, 1)
        ev = [{c: (mk(), mk()) for c in calls} for _ in range(warm)]
        for i in range(warm):
            opt.step_timed(int(order[i % len(order)]), ev[i], stream)
        torch.cuda.synchronize()
        call_ms = {c: float(np.mean([e[c][0].elapsed_time(e[c][1]) for e in ev[warm // 2:]])) for c in calls}
        dom = max(call_ms, key=call_ms.get)
        ev = [{dom: (mk(), mk())} for _ in range(steps)]
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for i in range(steps):
            opt.step_timed(int(order[(warm + i) % len(order)]), ev[i], stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t_start
        if opt.overflowed():
            raise RuntimeError("pair capacity overflow during the timed steps")
        call_ms[dom] = float(np.mean([e[dom][0].elapsed_time(e[dom][1]) for e in ev]))
        # algorithmic units of a step: the timed steps cycle over the views, so a step's
        # work is averaged over one more (untimed) step on every view
        per_view = []
        for vi in range(len(cams)):
            opt.step(vi, stream)
            torch.cuda.synchronize()
            per_view.append(opt.render_stats())
        stats = {k: float(np.mean([st[k] for st in per_view])) for k in per_view[0]}
        return dt, call_ms, stats, opt

    if args.only_visible:
        del targets
        wv = scenes.local_change(n=args.n, center=(0.0, 0.0, 1.0))
        tv = render_targets(wv)
        t_v, ms_v, st_v, _ = run(True, sc=wv.scene, targets=tv, a=(wv.active_begin, wv.scene.n))
        log(f"visible: {args.steps / t_v:.1f} it/s, calls {ms_v}, {st_v}")
        return 0
    if args.only_full:
        t_full, ms_full, st_full, _ = run(False)
        log(f"full: {args.steps / t_full:.1f} it/s, calls {ms_full}, {st_full}")
        return 0
    t_local, ms_local, st_local, opt_local = run(True)
    it_local = args.steps / t_local
    log(f"local: {it_local:.1f} it/s, calls {ms_local}, {st_local}")
    res_full = None
    if not args.no_full:
        del opt_local
        torch.cuda.empty_cache()
        t_full, ms_full, st_full, opt_full = run(False)
        res_full = (args.steps / t_full, ms_full, st_full)
        log(f"full: {res_full[0]:.1f} it/s, calls {ms_full}, {st_full}")
        del opt_full
    del targets
    torch.cuda.empty_cache()

    visible = None
    if not args.no_visible:
        wv = scenes.local_change(n=args.n, center=(0.0, 0.0, 1.0))
        tv = render_targets(wv)
        av = (wv.active_begin, wv.scene.n)
        t_v, ms_v, st_v, opt_v = run(True, sc=wv.scene, targets=tv, a=av, steps=max(args.steps // 2, 1))
        it_v = max(args.steps // 2, 1) / t_v
        log(f"visible change set {wv.name}: {it_v:.1f} it/s, calls {ms_v}, {st_v}")
        over_v = None if res_full is None else it_v / res_full[0]
        visible = {"workload": wv.name, "active_gaussians": av[1] - av[0], "it_s": round(it_v, 3),
                   "over_full": None if over_v is None else round(over_v, 3),
                   "target_over_full": TARGET_LOCAL_OVER_FULL,
                   "gap_to_target": None if over_v is None else round(TARGET_LOCAL_OVER_FULL / over_v, 3),
                   "call_ms": {k: round(v, 4) for k, v in ms_v.items()}, "work_per_step": st_v,
                   "roofline": roofline_of(ms_v, st_v, wv.scene.n)}
        del opt_v, tv
        torch.cuda.empty_cache()

    roofline = roofline_of(ms_local, st_local, sc.n)
    serving = None
    if not args.no_serve:
        serving = serving_leg(dev, args.serve_requests, log)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sc, cams, a, w.scene_gt, order, args.cpu_seconds, log)
        if args.cpu_single:
            cpu["single_thread"] = cpu_single_thread(sc, cams, a, w.scene_gt, order, log)

    others = None if args.no_configs else other_configs(dev, log)
    mpix = st_local["pixels"] * it_local / 1e6
    out = {
        "metric": "fwd+bwd it/s local vs full at 1M Gaussians 720p; render p50/p99 ms",
        "value": round(it_local, 3),
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 / it_local, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n_gaussians": sc.n, "width": cams[0].width, "height": cams[0].height,
                   "views": len(cams), "active_gaussians": a[1] - a[0], "mode": "local",
                   "masked_tile_frac": round(st_local["tiles"] / st_local["tiles_total"], 4),
                   "pairs_local": round(st_local["pairs"])},
        "local_mpix_s": round(mpix, 2),
        "full_it_s": None if res_full is None else round(res_full[0], 3),
        "local_over_full": None if res_full is None else round(it_local / res_full[0], 3),
        # the stated change set is hidden from every view (no record of it is ever
        # composited, pixel_records_active = 0), so its local step computes no gradient;
        # the visible-change leg below is the one whose local step does gradient work
        "local_over_full_note": "stated change set occluded in all views (no gradient work); see "
                                "visible_change_variant for the leg with gradient work and its gap to the 5x target",
        "full_pairs": None if res_full is None else round(res_full[2]["pairs"]),
        "local_work_per_step": st_local,
        "full_work_per_step": None if res_full is None else res_full[2],
        "visible_change_variant": visible,
        "other_configs": others,
        # the dominant call over the timed steps, the others over the second half of warm-up
        "call_ms_local": {k: round(v, 4) for k, v in ms_local.items()},
        "call_ms_full": None if res_full is None else {k: round(v, 4) for k, v in res_full[1].items()},
        "serving": serving,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


# HBM bytes per call of the local step, from two rocprofv3 counter runs (FETCH_SIZE, then
# WRITE_SIZE, summed over the call's kernels and averaged over 10 steps), each scaled by
# what the counter reads for a plain 256 MiB device copy (fetch x2.000, write x1.000).
# They describe the kernels whose sources hash to `source_sha256` and are reported only
# while the sources still do (profiles/traffic_local_step_1M_1280x720.txt).
MEASURED_TRAFFIC = {
    "source_sha256": "3008baab7da9acbd15d0f483f73876ed3ebf9597763c4bbd0521af40a08b3a58",
    "bytes": {"bin_and_sort": 83.640e6, "render_forward": 18.101e6, "render_backward": 17.452e6},
}


def kernel_source_hash():
    """SHA-256 of the kernel sources with comments and whitespace removed (so that a
    comment-only edit keeps the measurement; the sources hold no // or /* in strings)."""
    import re
    h = hashlib.sha256()
    for p in sorted((ROOT / "paper_2506_21117_amd" / "csrc").glob("*")) + [ROOT / "include" / "clsplat.h"]:
        text = re.sub(r"/\*.*?\*/", " ", p.read_text(), flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(p.name.encode())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_traffic(call):
    if MEASURED_TRAFFIC["source_sha256"] != kernel_source_hash():
        return None
    return MEASURED_TRAFFIC["bytes"].get(call)


# The target ratio of the local step's rate to the full-scene step's on the same views.
TARGET_LOCAL_OVER_FULL = 5.0

# FP32 operations per (pixel, record) evaluation, counted from the model's formulas:
# the Gaussian weight (offset 2, quadratic form 9, exp 1, opacity product and clamp 2),
# the transmittance update (2) and the colour sums (3 multiply-adds = 6) ...
FLOP_EVAL = 22
# ... and, for a record of the active range in the backward, its gradient terms: dL/dalpha
# (3 x (2 mul + 1 sub) + 2 add + 1 reciprocal = 12), colour (3), opacity (1), power (1),
# centre (2 x 4), conic (8) and the reduction over the pixels of the tile (9 adds per
# pixel) = 42.
FLOP_GRAD = 42
# Peak of the FP32 vector units without packed math: 256 CUs x 4 SIMDs x 16 lanes x
# 2 (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 78.6


def roofline_of(ms, st, n):
    """Roofline of the local step's dominant call (by measured time)."""
    dom = max(ms, key=ms.get)
    t = ms[dom] * 1e-3
    if dom == "render_backward":
        flops = FLOP_EVAL * st["pixel_records"] + FLOP_GRAD * st["pixel_records_active"]
        ach = flops / t / 1e12
        return {"bound": "alu", "kernel": "render_backward (raster backward + preprocess backward)",
                "achieved": round(ach, 3), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / ALU_PEAK_TFLOPS, 5), "traffic": measured_traffic(dom),
                "units": {"pixel_records": st["pixel_records"], "pixel_records_active": st["pixel_records_active"],
                          "flop_per_eval": FLOP_EVAL, "flop_per_active_eval": FLOP_GRAD}}
    if dom == "render_forward":
        flops = FLOP_EVAL * st["pixel_records"]
        ach = flops / t / 1e12
        return {"bound": "alu", "kernel": "render_forward (both depth slabs)", "achieved": round(ach, 3),
                "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / ALU_PEAK_TFLOPS, 5),
                "traffic": measured_traffic(dom),
                "units": {"pixel_records": st["pixel_records"], "flop_per_eval": FLOP_EVAL}}
    # binning: read the projected rectangles, flags and depths of all N entries
    # (16 B), then per pair it lists (the first slab's) 44 B (emit 12 B, one sort read +
    # write 24 B, range scan 8 B)
    pairs = st["pairs_first_slab"]
    byts = 16 * n + 44 * pairs
    ach = byts / t / 1e9
    return {"bound": "hbm", "kernel": "bin_and_sort", "achieved": round(ach, 2), "peak": 8000.0, "unit": "GB/s",
            "frac": round(ach / 8000.0, 5), "traffic": measured_traffic(dom),
            "units": {"entries": n, "pairs": pairs, "algorithmic_bytes": byts}}


def serving_leg(dev, n_requests, log):
    """Render latency of stored scene states (the 2M-Gaussian base with 7 change steps;
    resolutions 640x480, 1280x720, 1920x1080): the closed-loop rate X (every request
    waiting at the start), then Poisson arrivals at 0.25 X, 0.5 X and 0.8 X, each with
    ``n_requests`` requests; the headline is p50/p99 at 0.5 X."""
    import numpy as np
    import torch

    import scenes
    from paper_2506_21117_amd.serve import Engine, GpuBackend, Request, StateStore, poisson_requests

    t0 = time.time()
    states, history = scenes.serving_history(seed=5)
    store = StateStore.from_history(states[-1], history)
    del states, history
    store.to_device(dev)
    log(f"serving store: {store.n_rows} resident rows, {store.timesteps} timesteps, built in {time.time() - t0:.1f}s")
    camfn = lambda r, W, H: scenes.sphere_camera(r, 4.0, width=W, height=H, fx=H / (2 * np.tan(np.radians(20))))
    be = GpuBackend(store, dev, max_slots=4)
    eng = Engine(be, hbm_budget_bytes=64 << 30, max_slots=4, max_batch=4)
    # warm-up: one request per (timestep, resolution)
    rng = np.random.default_rng(50)
    warm = [Request(i, k, camfn(rng, W, H), 0.0)
            for i, (k, (W, H)) in enumerate((k, res) for k in range(store.timesteps) for res in scenes.RESOLUTIONS)]
    eng.run(warm)
    torch.cuda.synchronize()

    def leg(qps, seed):
        reqs = poisson_requests(np.random.default_rng(seed), n_requests, qps, store.timesteps, scenes.RESOLUTIONS,
                                camfn)
        _, st = eng.run(reqs)
        torch.cuda.synchronize()
        sm = st.summary()
        return {"qps": None if qps == 0 else round(qps, 1), "requests": n_requests, "p50_ms": round(sm["p50_ms"], 3),
                "p99_ms": round(sm["p99_ms"], 3), "mean_ms": round(sm["mean_ms"], 3),
                "frames_per_s": round(sm["frames_per_s"], 1), "groups": sm["groups"], "retries": sm["retries"],
                "mean_group": round(sm["completed"] / max(sm["groups"], 1), 2), "peak_inflight": sm["peak_inflight"]}

    closed = leg(0.0, 51)          # all arrivals at t = 0: the saturation rate
    X = closed["frames_per_s"]
    log(f"serving closed loop: {closed}")
    sweep = []
    for i, f in enumerate((0.25, 0.5, 0.8)):
        r = leg(f * X, 52 + i)
        r["fraction_of_saturation"] = f
        log(f"serving at {f} X = {r['qps']} QPS: {r}")
        sweep.append(r)
    head = sweep[1]
    return {"saturation_frames_per_s": X, "closed_loop": closed, "poisson": sweep,
            "headline": {"qps": head["qps"], "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
                         "frames_per_s": head["frames_per_s"]},
            "workload": "2M-Gaussian base + 7 change steps, SH3, resolutions 640x480/1280x720/1920x1080 uniform, "
                        "random timestep, camera uniform on the radius-4 sphere, max 4 views per call, 4 slots"}


def other_configs(dev, log):
    """One-off timing of the other two workloads: full-scene optimisation (200k
    Gaussians, SH degree 3, 8 ring views of 800x800; every row active, Adam over all
    rows) and differentiation at scale (3M Gaussians, SH degree 3, a batch of 4
    1920x1080 views through the autograd wrapper in recompute mode, L1 loss)."""
    import numpy as np
    import torch

    import scenes
    from paper_2506_21117_amd import api
    from paper_2506_21117_amd.autograd import render
    from paper_2506_21117_amd.optim import SplatOptimizer

    out = {}
    w = scenes.full_scene()
    params = api.GaussianTensors.from_scene(w.scene, dev)
    tg = torch.as_tensor(w.targets, device=dev)
    opt = SplatOptimizer(params, w.cameras, tg, local=False)
    for i in range(8):
        opt.step(i % len(w.cameras))
    torch.cuda.synchronize()
    steps = 64
    t = time.perf_counter()
    for i in range(steps):
        opt.step(i % len(w.cameras))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    if opt.overflowed():
        raise RuntimeError("pair capacity overflow in the full-scene leg")
    out["full_scene_200k_sh3_800x800_8v"] = {"it_s": round(steps / dt, 2), "ms_per_step": round(1000 * dt / steps, 3),
                                            "steps": steps, "mode": "full (every row active), one view per step"}
    log(f"config full-scene: {out['full_scene_200k_sh3_800x800_8v']}")
    del opt, params, tg, w
    torch.cuda.empty_cache()

    w = scenes.differentiation()
    g = api.GaussianTensors.from_scene(w.scene, dev)
    leaves = [t.clone().requires_grad_(True) for t in g.tensors()]
    tg = torch.as_tensor(w.targets, device=dev)

    def it():
        img = render(*leaves, w.cameras, mode="recompute")
        loss = (img - tg).abs().mean()
        loss.backward()
        for x in leaves:
            x.grad = None

    for _ in range(2):
        it()
    torch.cuda.synchronize()
    steps = 6
    t = time.perf_counter()
    for _ in range(steps):
        it()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    out["differentiation_3m_sh3_1920x1080_4v"] = {
        "it_s": round(steps / dt, 3), "ms_per_iteration": round(1000 * dt / steps, 2), "steps": steps,
        "mode": "autograd recompute: forward of 4 views, L1 loss, backward (re-runs preprocess, binning, forward)"}
    log(f"config differentiation: {out['differentiation_3m_sh3_1920x1080_4v']}")
    del leaves, g, tg, w
    torch.cuda.empty_cache()
    return out


def cpu_baseline(sc, cams, a, scene_gt, order, budget_s, log, threads=None):
    """The CPU oracle (float64, brute force per pixel) running complete local steps of
    the same workload until ``budget_s`` seconds have passed: project every Gaussian,
    build the render mask from the change set, render every masked pixel, L1 gradient
    against the oracle's own render of the unchanged scene at those pixels, render again
    with that gradient, preprocess backward, Adam on the change set."""
    import numpy as np

    import oracle

    names = ("means", "log_scales", "quats", "opacity_logit", "sh")
    lrs = {"means": 1.6e-4, "log_scales": 5e-3, "quats": 1e-3, "opacity_logit": 5e-2, "sh": 2.5e-3}
    params = {k: np.asarray(x, dtype=np.float64) for k, x in zip(names, sc.param_arrays())}
    m = {k: np.zeros_like(x) for k, x in params.items()}
    v = {k: np.zeros_like(x) for k, x in params.items()}
    if threads is None:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rows = slice(a[0], a[1])
    steps = 0
    t_start = time.perf_counter()
    t_target = 0.0
    while True:
        cam = cams[int(order[steps % len(order)])]
        pt = tuple(params[k] for k in names)
        # the target pixels are rendered from the unchanged scene (not timed)
        pp = oracle.preprocess(sc, cam, params=pt)
        f32 = lambda k: pp[k].astype(np.float32)
        x0, x1, y0, y1 = oracle.tile_rects(f32("u"), f32("v"), f32("rx"), f32("ry"), cam.width, cam.height)
        TX, TY = oracle.tile_grid(cam.width, cam.height)
        mask = np.zeros((TY, TX), bool)
        for i in np.nonzero(pp["visible"][a[0]:a[1]])[0] + a[0]:
            mask[y0[i]:y1[i], x0[i]:x1[i]] = True
        ys, xs = np.nonzero(np.kron(mask, np.ones((16, 16), bool))[:cam.height, :cam.width])
        pix = np.stack([xs, ys], 1).astype(np.int32)
        t1 = time.perf_counter()
        tgt = oracle.render(scene_gt, cam, pixels=pix)["rgb"]
        t_target += time.perf_counter() - t1
        img = oracle.render(sc, cam, pixels=pix, params=pt)["rgb"]
        dl = np.sign(img - tgt) / (3.0 * cam.width * cam.height)
        r = oracle.render(sc, cam, pixels=pix, dL_dC=dl, params=pt)
        g = oracle.preprocess_backward(sc, cam, r["grad2d"], params=pt)
        params, m, v = oracle.adam_step(params, g, m, v, steps + 1, lrs, rows=rows)
        steps += 1
        if time.perf_counter() - t_start - t_target >= budget_s:
            break
    dt = time.perf_counter() - t_start - t_target
    log(f"cpu oracle: {steps} complete local steps in {dt:.1f}s ({threads} threads)")
    return {"value": round(steps / dt, 6), "unit": "it/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} complete local steps (views in the bench's order) of the 1M-Gaussian 1280x720 "
                      f"workload: fp64 projection of all Gaussians, render mask of the change set, brute-force "
                      f"forward of every masked pixel, L1 gradient, brute-force forward+backward, preprocess "
                      f"backward, Adam on the change set; {dt:.1f}s measured, no extrapolation (the render of "
                      f"the targets at the masked pixels is excluded)"}


def cpu_single_thread(sc, cams, a, scene_gt, order, log):
    """One complete oracle local step (as in ``cpu_baseline``) on one OpenMP thread."""
    import ctypes

    import oracle
    gomp = ctypes.CDLL("libgomp.so.1")
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.lib()
    gomp.omp_set_num_threads(1)
    try:
        r = cpu_baseline(sc, cams, a, scene_gt, order, 0.0, log, threads=1)
    finally:
        gomp.omp_set_num_threads(threads)
    r["sample"] = "one complete local step on one thread; " + r["sample"].split("; ", 1)[0]
    return r


# ---- summaries of rocprofv3 output (host only) ----------------------------------------
# A step of this script's timed loop starts at preprocess_kernel and ends with the Adam
# update: adam_kernel (full steps), or preprocess_backward_adam_kernel, which holds it
# (local steps).  Within it the C-ABI calls are: bin_and_sort = the kernels after
# preprocess_kernel up to the first phase-1 forward kernel; render_forward = that one
# up to the last render_forward_kernel (the second depth slab's listing runs between the
# two phases; local steps compute the L1 gradient inside the forward); render_backward =
# the kernels after l1_loss_grad_kernel (or after the forward) up to the preprocess
# backward.
CALLS = ("bin_and_sort", "render_forward", "render_backward")


def short_kernel_name(name):
    return name.replace("clsp::(anonymous namespace)::", "").split("(")[0].replace("void ", "").strip()


def split_steps(seq, k):
    """``seq``: dispatches in order, each a tuple whose first item is the short kernel name.
    Returns the last ``k`` complete steps, each as (all dispatches, {call: dispatches})."""
    seq = [x for x in seq if not (x[0].startswith("at::") or "rocclr" in x[0])]
    starts = [i for i, x in enumerate(seq) if x[0] == "preprocess_kernel"]
    out = []
    for j, s0 in enumerate(starts):
        s1 = starts[j + 1] if j + 1 < len(starts) else len(seq)
        st = seq[s0:s1]
        names = [x[0] for x in st]
        ends = [i for i, nm in enumerate(names) if nm in ("adam_kernel", "preprocess_backward_adam_kernel")]
        if not ends:
            continue
        st = st[:ends[0] + 1]
        names = names[:len(st)]
        try:
            i_f1 = next(i for i, nm in enumerate(names) if nm.startswith("render_forward_kernel<1"))
            i_f2 = max(i for i, nm in enumerate(names) if nm.startswith("render_forward_kernel"))
            i_l1 = names.index("l1_loss_grad_kernel") if "l1_loss_grad_kernel" in names else i_f2
            i_pb = max(i for i, nm in enumerate(names) if nm.startswith("preprocess_backward"))
        except ValueError:
            continue
        out.append((st, {"bin_and_sort": st[1:i_f1], "render_forward": st[i_f1:i_f2 + 1],
                         "render_backward": st[i_l1 + 1:i_pb + 1]}))
    return out[-k:]


def summarize_trace(db, k, notes=()):
    """Per-step kernel averages of a kernel trace (rocprofv3 results database)."""
    import collections
    import sqlite3

    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end, duration from kernels order by start").fetchall()
    con.close()
    steps = split_steps([(short_kernel_name(n), s, e, d) for n, s, e, d in rows], k)
    if not steps:
        raise SystemExit(f"{db}: no complete step found")
    k = len(steps)
    st = collections.defaultdict(lambda: [0, 0, float("inf"), 0])
    for disp, _ in steps:
        for n, _, _, d in disp:
            x = st[n]
            x[0] += 1; x[1] += d; x[2] = min(x[2], d); x[3] = max(x[3], d)
    tot = sum(v[1] for v in st.values())
    span = sum(disp[-1][2] - disp[0][1] for disp, _ in steps)
    lines = [f"# {n}" for n in notes]
    lines.append(f"# rocprofv3 kernel trace; averages over the last {k} steps "
                 f"({sum(len(d) for d, _ in steps)} dispatches)")
    lines.append(f"# GPU time per step (sum of kernel durations): {tot / k / 1e3:.1f} us; "
                 f"span per step (first start -> last end): {span / k / 1e3:.1f} us")
    lines.append(f"{'kernel':34s} {'calls/step':>10s} {'us/step':>9s} {'avg_us':>8s} {'min_us':>8s} "
                 f"{'max_us':>8s} {'share':>6s}")
    for n, (c, d, mn, mx) in sorted(st.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"{n:34s} {c / k:10.1f} {d / k / 1e3:9.1f} {d / c / 1e3:8.1f} {mn / 1e3:8.1f} "
                     f"{mx / 1e3:8.1f} {100 * d / tot:5.1f}%")
    lines.append("# per call (average over steps): kernels, sum of kernel durations, span first start -> last end")
    for call in CALLS:
        segs = [c[call] for _, c in steps]
        lines.append(f"#   {call:16s} {sum(len(s) for s in segs) / k:5.1f} kernels  "
                     f"sum {sum(sum(x[3] for x in s) for s in segs) / k / 1e3:8.1f} us  "
                     f"span {sum(s[-1][2] - s[0][1] for s in segs) / k / 1e3:8.1f} us")
    return "\n".join(lines)


def read_counter_csv(folder, counter):
    """Dispatches in order as (short kernel name, counter value) from the
    counter_collection.csv that rocprofv3 --pmc --output-format csv wrote under ``folder``."""
    import csv

    files = sorted(Path(folder).rglob("*counter_collection.csv"))
    if not files:
        raise SystemExit(f"{folder}: no counter_collection.csv")
    rows = {}
    with open(files[0]) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                rows[int(r["Dispatch_Id"])] = (short_kernel_name(r["Kernel_Name"]), float(r["Counter_Value"]))
    return [rows[i] for i in sorted(rows)]


def summarize_counters(folders, k=10, notes=()):
    """Per-kernel averages (per dispatch, over the last ``k`` steps) of every counter in the
    counter_collection.csv files under ``folders`` (one rocprofv3 --pmc run each), and the
    ratios that read them: VALU instructions per wave, the share of wave-cycles a wave
    waited for any instruction, and LDS bank-conflict cycles per LDS instruction."""
    import collections
    import csv

    per_kernel = collections.defaultdict(lambda: collections.defaultdict(list))
    order = []
    for folder in folders:
        files = sorted(Path(folder).rglob("*counter_collection.csv"))
        if not files:
            raise SystemExit(f"{folder}: no counter_collection.csv")
        disp = collections.OrderedDict()
        with open(files[0]) as fh:
            for r in csv.DictReader(fh):
                d = disp.setdefault(int(r["Dispatch_Id"]), (short_kernel_name(r["Kernel_Name"]), {}))
                d[1][r["Counter_Name"]] = d[1].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        seq = [(name, vals) for _, (name, vals) in sorted(disp.items())]
        steps = split_steps(seq, k)
        if not steps:
            raise SystemExit(f"{folder}: no complete step found")
        for st, _ in steps:
            for name, vals in st:
                if name not in order:
                    order.append(name)
                for c, v in vals.items():
                    per_kernel[name][c].append(v)
    counters = sorted({c for kv in per_kernel.values() for c in kv})
    mean = lambda x: sum(x) / len(x) if x else float("nan")
    lines = [f"# {n}" for n in notes]
    lines.append(f"# averages per dispatch over the last {k} steps; kernels in step order")
    lines.append("kernel".ljust(34) + "".join(f"{c[:18]:>19s}" for c in counters))
    for name in order:
        kv = per_kernel[name]
        lines.append(name[:34].ljust(34) + "".join(f"{mean(kv[c]):19.6g}" if c in kv else f"{'-':>19s}"
                                                 for c in counters))
    ratios = []
    for name in order:
        kv = {c: mean(v) for c, v in per_kernel[name].items()}
        parts = []
        if kv.get("SQ_WAVES") and "SQ_INSTS_VALU" in kv:
            parts.append(f"VALU insts/wave {kv['SQ_INSTS_VALU'] / kv['SQ_WAVES']:.0f}")
        if kv.get("SQ_WAVE_CYCLES") and "SQ_WAIT_INST_ANY" in kv:
            parts.append(f"waiting {100 * kv['SQ_WAIT_INST_ANY'] / kv['SQ_WAVE_CYCLES']:.0f}% of wave-cycles")
        if kv.get("SQ_WAVE_CYCLES") and "SQ_ACTIVE_INST_VALU" in kv:
            parts.append(f"issuing VALU {100 * kv['SQ_ACTIVE_INST_VALU'] / kv['SQ_WAVE_CYCLES']:.0f}% of wave-cycles")
        if kv.get("SQ_INSTS_LDS") and "SQ_LDS_BANK_CONFLICT" in kv:
            parts.append(f"LDS bank-conflict cycles/LDS inst {kv['SQ_LDS_BANK_CONFLICT'] / kv['SQ_INSTS_LDS']:.3f}")
        if parts:
            ratios.append(f"#   {name}: " + "; ".join(parts))
    if ratios:
        lines.append("# ratios of the averages above")
        lines += ratios
    return "\n".join(lines)


COPY_KIB = 262144.0  # the 256 MiB calibration copy, in KiB


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, k=10, notes=()):
    """HBM bytes per C-ABI call of the step: FETCH_SIZE and WRITE_SIZE (KiB per dispatch)
    summed over each call's kernels, averaged over the last ``k`` steps, and scaled by the
    factor that makes the counter read 256 MiB for a plain 256 MiB device copy."""
    def per_call(folder, counter):
        steps = split_steps(read_counter_csv(folder, counter), k)
        if not steps:
            raise SystemExit(f"{folder}: no complete step found")
        avg = {c: sum(sum(v for _, v in cs[c]) for _, cs in steps) / len(steps) for c in CALLS}
        avg["step"] = sum(sum(v for _, v in d) for d, _ in steps) / len(steps)
        return avg, len(steps)

    def factor(folder, counter):
        v = [x for n, x in read_counter_csv(folder, counter) if "copyBuffer" in n]
        if not v:
            raise SystemExit(f"{folder}: no copy dispatch")
        m = sum(v) / len(v)
        return COPY_KIB / m, m

    ff, fm = factor(copy_fetch_dir, "FETCH_SIZE")
    wf, wm = factor(copy_write_dir, "WRITE_SIZE")
    fetch, kf = per_call(fetch_dir, "FETCH_SIZE")
    write, kw = per_call(write_dir, "WRITE_SIZE")
    lines = [f"# {n}" for n in notes]
    lines.append(f"# copy calibration: 256 MiB device copy reads FETCH_SIZE {fm:.0f} KiB (factor {ff:.3f}), "
                 f"WRITE_SIZE {wm:.0f} KiB (factor {wf:.3f})")
    lines.append(f"# averages over {min(kf, kw)} steps; bytes = KiB x 1024 x factor")
    for call in CALLS + ("step",):
        f = fetch[call] * 1024 * ff
        w = write[call] * 1024 * wf
        lines.append(f"{call:16s} fetch {f / 1e6:9.3f} MB  write {w / 1e6:9.3f} MB  total {(f + w) / 1e6:9.3f} MB")
    return "\n".join(lines)


if __name__ == "__main__":
    sys.exit(main())
