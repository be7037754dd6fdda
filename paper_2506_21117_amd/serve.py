"""Serving: render any stored scene state for a stream of requests.

State store (Supp. "History Recovery", Alg. 4 alg:example): the paper keeps the latest
reconstruction G^T and, for every step k, the changed Gaussians O^k (their values before
the change) and the 0/1 indicator I^k over G^{k-1}; G^{k-1} is rebuilt by placing the
first #static Gaussians of G^k where I^k = 0 and O^k where I^k = 1.  Here every state
stays resident at once: one pool holds G^T's rows followed by every O^k, and the same
scatter is applied to int32 row lists instead of to Gaussian data, giving each timestep
a gather list into the pool.  A state is rendered by passing its gather list to
clsp_project_preprocess; nothing is copied per request.

Engine: requests (timestep, camera) arrive over time; waiting requests with the same
timestep and resolution are grouped into one multi-view call; a group is admitted when a
slot (its own HIP stream) is free and its memory estimate fits the HBM budget; work of
admitted groups overlaps on the device; completed groups free their slot and memory at
once, so new arrivals are admitted while others are still on the GPU (continuous
batching).  The scheduling logic is backend-agnostic; ``GpuBackend`` runs the C-ABI.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


# ------------------------------------------------------------------ state store
class StateStore:
    """Resident pool + per-timestep gather lists (host arrays until ``to_device``)."""

    def __init__(self, pool_arrays, sh_degree, gathers):
        self.pool_arrays = pool_arrays      # [means, log_scales, quats, opacity_logit, sh] numpy, last axis = row
        self.sh_degree = sh_degree
        self.gathers = gathers              # list of int32 numpy arrays, index = timestep
        self.device_pool = None
        self.device_gathers = None

    @property
    def n_rows(self):
        return int(self.pool_arrays[0].shape[-1])

    @property
    def timesteps(self):
        return len(self.gathers)

    @classmethod
    def from_history(cls, latest, history):
        """latest: the scene G^T (a ``scenes.Scene``); history[k-1] = (I^k, O^k) for
        k = 1..T with I^k a bool array over G^{k-1} and O^k the changed Gaussians'
        values before step k (stored before optimisation)."""
        arrays = [np.asarray(a) for a in latest.param_arrays()]
        n = latest.n
        gathers = [None] * (len(history) + 1)
        gathers[-1] = np.arange(n, dtype=np.int32)
        chunks = [arrays]
        rows = n
        for k in range(len(history), 0, -1):
            ind, old = history[k - 1]
            ind = np.asarray(ind, dtype=bool)
            m = old.n
            assert int(ind.sum()) == m
            o_rows = np.arange(rows, rows + m, dtype=np.int32)
            rows += m
            chunks.append([np.asarray(a) for a in old.param_arrays()])
            n_static = int((~ind).sum())          # #static: the zeros of I^k
            prev = np.empty(len(ind), dtype=np.int32)
            prev[ind] = o_rows                     # changed Gaussians where I^k = 1
            prev[~ind] = gathers[k][:n_static]     # the static prefix of G^k where I^k = 0
            gathers[k - 1] = prev
        pool = [np.concatenate([c[i] for c in chunks], axis=-1) for i in range(5)]
        return cls(pool, latest.sh_degree, gathers)

    def state_arrays(self, k):
        """The Gaussians of timestep k as arrays (host; for checks)."""
        g = self.gathers[k]
        return [a[..., g] for a in self.pool_arrays]

    def to_device(self, device):
        import torch

        from . import api
        self.device_pool = api.GaussianTensors(*[torch.as_tensor(np.ascontiguousarray(a), device=device)
                                                 for a in self.pool_arrays], self.sh_degree)
        self.device_gathers = [torch.as_tensor(g, device=device) for g in self.gathers]
        return self


# ------------------------------------------------------------------ requests
@dataclass
class Request:
    rid: int
    timestep: int
    camera: object
    arrival: float = 0.0      # seconds after the start of the run

    @property
    def key(self):
        return (self.timestep, self.camera.width, self.camera.height)


@dataclass
class Completed:
    rid: int
    latency_ms: float
    image: object = None
    group_size: int = 1


@dataclass
class _Group:
    reqs: list
    slot: int
    bytes: int
    handle: object = None
    launched: float = 0.0


@dataclass
class EngineStats:
    completed: int = 0
    groups: int = 0
    retries: int = 0
    peak_bytes: int = 0
    peak_inflight: int = 0
    wall_s: float = 0.0
    latencies_ms: list = field(default_factory=list)

    def summary(self):
        lat = np.asarray(self.latencies_ms) if self.latencies_ms else np.zeros(1)
        return {"completed": self.completed, "groups": self.groups, "retries": self.retries,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "frames_per_s": self.completed / max(self.wall_s, 1e-9),
                "peak_bytes": self.peak_bytes, "peak_inflight": self.peak_inflight, "wall_s": self.wall_s}


class Engine:
    """Continuous-batching render loop over a backend with ``estimate_bytes(reqs)``,
    ``launch(reqs, slot) -> handle``, ``done(handle) -> bool`` and
    ``finish(handle) -> list of images, or None to retry`` (retry after growing its
    pair capacity)."""

    def __init__(self, backend, hbm_budget_bytes, max_slots=8, max_batch=4, keep_images=False):
        self.backend = backend
        self.budget = int(hbm_budget_bytes)
        self.max_slots = int(max_slots)
        self.max_batch = int(max_batch)
        self.keep_images = keep_images

    def run(self, requests, clock=time.perf_counter, idle=None):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()
        inflight: list[_Group] = []
        free = list(range(self.max_slots))[::-1]
        used = 0
        stats = EngineStats()
        out = []
        t0 = clock()
        while pending or waiting or inflight:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            progressed = False
            # admission: oldest waiting request first, grouped with same-key arrivals
            while waiting and free:
                head = waiting[0]
                group = [r for r in waiting if r.key == head.key][:self.max_batch]
                need = self.backend.estimate_bytes(group)
                if need > self.budget:
                    raise MemoryError(f"request {head.rid} needs {need} bytes, more than the whole budget")
                if used + need > self.budget:
                    break
                for r in group:
                    waiting.remove(r)
                slot = free.pop()
                used += need
                g = _Group(group, slot, need, launched=clock() - t0)
                g.handle = self.backend.launch(group, slot)
                inflight.append(g)
                stats.groups += 1
                stats.peak_bytes = max(stats.peak_bytes, used)
                stats.peak_inflight = max(stats.peak_inflight, len(inflight))
                progressed = True
            # completion
            for g in list(inflight):
                if not self.backend.done(g.handle):
                    continue
                imgs = self.backend.finish(g.handle)
                if imgs is None:                  # pair capacity grown: run again
                    stats.retries += 1
                    g.handle = self.backend.launch(g.reqs, g.slot)
                    continue
                t_done = clock() - t0
                for r, im in zip(g.reqs, imgs):
                    lat = 1000.0 * (t_done - r.arrival)
                    out.append(Completed(r.rid, lat, im if self.keep_images else None, len(g.reqs)))
                    stats.latencies_ms.append(lat)
                    stats.completed += 1
                inflight.remove(g)
                free.append(g.slot)
                used -= g.bytes
                progressed = True
            if not progressed:
                if idle is not None:
                    idle(pending[0].arrival if (pending and not waiting and not inflight) else None)
                elif pending and not waiting and not inflight:
                    dt = pending[0].arrival - (clock() - t0)
                    if dt > 0:
                        time.sleep(min(dt, 0.001))
        stats.wall_s = clock() - t0
        return out, stats


# ------------------------------------------------------------------ GPU backend
class GpuBackend:
    """Renders request groups through the C-ABI, one HIP stream per slot."""

    def __init__(self, store: StateStore, device, max_slots=8, bg=(0.0, 0.0, 0.0)):
        import torch

        from . import api
        self.torch, self.api = torch, api
        self.store = store if store.device_pool is not None else store.to_device(device)
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max_slots)]
        self.bg = bg
        self.pairs_per_view = {}      # (timestep, W, H) -> largest pair count seen for one view

    def _capacity(self, reqs):
        """Pair capacity for the admission estimate: the largest per-view count seen for
        this (timestep, resolution), or 4 per Gaussian before any was seen.  The lists
        themselves are sized exactly (see ``launch``)."""
        key = reqs[0].key
        n = len(self.store.gathers[key[0]])
        per = self.pairs_per_view.get(key, 4 * n)
        return int(per * len(reqs) * 1.2) + 4096

    def estimate_bytes(self, reqs):
        n = len(self.store.gathers[reqs[0].timestep])
        V = len(reqs)
        W, H = reqs[0].camera.width, reqs[0].camera.height
        cap = self._capacity(reqs)
        ws = self.api.lib().clsp_bin_and_sort_workspace_bytes(n, V, W, H, cap)
        TX, TY = self.api.tile_grid(W, H)
        proj = n * V * (48 + 4 + 8 + 4)
        bins = cap * 8 + V * TX * TY * 24 + 128
        images = V * H * W * (12 + 4 + 4)
        return int(proj + bins + ws + images)

    def launch(self, reqs, slot):
        """Stage 1 on the slot's stream: project the state's Gaussians and count the
        pairs of the complete lists (a binning call with no pair capacity, which reports
        the count and emits nothing).  Stage 2 (``done`` starts it once stage 1 has
        finished): lists with exactly that capacity, which bounds the depth-sliced
        lists' pairs, and the forward.  No request is rendered twice."""
        torch, api = self.torch, self.api
        s = self.streams[slot]
        ts = reqs[0].timestep
        cams = [r.camera for r in reqs]
        gather = self.store.device_gathers[ts]
        n = int(gather.numel())
        W, H = cams[0].width, cams[0].height
        with torch.cuda.stream(s):
            proj = api.ProjectedBuffers.alloc(n, len(cams), self.device)
            probe = api.BinBuffers.alloc(n, len(cams), W, H, 1, self.device, api._ffi.BINS_COMPLETE)
            api.project_preprocess(self.store.device_pool, cams, proj, gather=gather, stream=s)
            api.bin_and_sort(proj, cams, None, False, probe, stream=s)
            count = torch.empty(1, dtype=torch.int32, pin_memory=True)
            count.copy_(probe.counters[0:1], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"reqs": reqs, "ev": ev, "stage": 1, "proj": proj, "probe": probe, "count": count, "stream": s,
                "cams": cams}

    def _stage2(self, h):
        torch, api = self.torch, self.api
        s, cams, proj = h["stream"], h["cams"], h["proj"]
        pairs = int(h["count"].numpy().view(np.uint32)[0])
        W, H = cams[0].width, cams[0].height
        with torch.cuda.stream(s):
            bins = api.BinBuffers.alloc(proj.n, len(cams), W, H, max(pairs, 1), self.device)
            api.bin_and_sort(proj, cams, None, False, bins, stream=s)
            img, T, nc = api.render_forward(proj, bins, cams, self.bg, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        h.update(stage=2, ev=ev, img=img, bins=bins, keep=(T, nc), probe=None, pairs=pairs)

    def done(self, h):
        if not h["ev"].query():
            return False
        if h["stage"] == 1:
            self._stage2(h)
            return False
        return True

    def finish(self, h):
        c = h["bins"].read_counters()
        key = h["reqs"][0].key
        per = -(-h["pairs"] // len(h["reqs"]))
        self.pairs_per_view[key] = max(self.pairs_per_view.get(key, 0), per)
        if c["overflow"]:
            return None
        return [h["img"][i] for i in range(len(h["reqs"]))]

    def render_alone(self, req):
        """The same request rendered by itself on the default stream (for checks)."""
        api = self.api
        gather = self.store.device_gathers[req.timestep]
        n = int(gather.numel())
        proj = api.project_preprocess(self.store.device_pool, [req.camera], gather=gather)
        cap = self._capacity([req])
        while True:
            bins = api.bin_and_sort(proj, [req.camera], capacity=cap)
            img, _, _ = api.render_forward(proj, bins, [req.camera], self.bg)
            c = bins.read_counters()
            if not c["overflow"]:
                return img[0]
            cap = int(c["pairs"] * 1.2) + 4096


def poisson_requests(rng, n_requests, qps, timesteps, resolutions, camera_fn):
    """Arrival process: exponential gaps at rate ``qps``; timestep and resolution drawn
    uniformly; ``camera_fn(rng, width, height)`` draws the camera."""
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / qps) if qps > 0 else 0.0
        W, H = resolutions[int(rng.integers(len(resolutions)))]
        out.append(Request(i, int(rng.integers(timesteps)), camera_fn(rng, W, H), t))
    return out
