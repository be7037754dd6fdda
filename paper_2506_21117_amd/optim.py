"""Local and full-scene optimisation steps over the C-ABI.

One step (one view, the 3D Gaussian Splatting convention) runs, all on one stream:
project all Gaussians -> render mask and per-tile depth order (masked tiles only in
local mode) -> forward render with the L1 loss gradient -> backward render, then the
preprocess backward for the change set, which in local steps applies each changed
row's Adam update from the gradients it has just computed (full steps: a separate
masked Adam call, which also clears the gradient rows for the next step).  This is the local optimisation of CL-Splats (Sec. 3.3 "Local Optimization
Kernel"; Supp. "3DGS Optimization in Changed Regions"); the full-scene step is the same
with no mask and every row active.
"""
from __future__ import annotations

import ctypes

import torch

from . import _ffi, api
from ._ffi import C_STICKY, check


class SplatOptimizer:
    def __init__(self, params: api.GaussianTensors, cams, targets, active=None, local=True, bg=(0.0, 0.0, 0.0),
                 capacity=None, lr=api.DEFAULT_LR, projection_cache_bytes=32 << 30, loss="l1", frozen_order=True):
        """params: device parameters (updated in place); cams: list of cameras of one
        size; targets: [V, 3, H, W] float32 device tensor; active: (a0, a1) change set
        (default: all rows); local: restrict rendering to the change set's tile mask.

        Local steps keep each view's projection of all Gaussians (64 B per Gaussian per
        view, when that fits in ``projection_cache_bytes``) and re-project only the
        change set's rows: the other rows are frozen, so their projection for a view is
        the same every time the view comes back.  Call ``invalidate_projections()`` after
        changing rows outside the change set.

        loss: "l1" (the benchmark's loss), or "l1_dssim", the default 3D Gaussian Splatting
        loss the paper trains with, 0.8 L1 + 0.2 (1 - SSIM); its gradient on a masked tile
        reads pixels around the tile, which local steps take from a render of the unchanged
        Gaussians alone, made once per view (they never change).

        frozen_order: local steps whose change set is the suffix [a0, n) keep each view's
        depth order of the unchanged rows (16 B per entry, made on the view's first step)
        and sort only the change set's entries into it (clsp_bin_and_sort_frozen; the
        same lists as a full sort)."""
        if loss not in ("l1", "l1_dssim"):
            raise ValueError("loss must be 'l1' or 'l1_dssim'")
        self.loss = loss
        self._frozen_images = {}
        self._frozen_orders = {}
        self.params = params
        self.cams = list(cams)
        self.targets = targets
        self.n = params.n
        self.local = bool(local)
        self.active = (0, self.n) if (active is None or not local) else (int(active[0]), int(active[1]))
        self.frozen_order = bool(frozen_order) and self.local
        self.bg = tuple(float(x) for x in bg)
        self.lr = lr
        dev = params.means.device
        W, H = self.cams[0].width, self.cams[0].height
        # full steps keep a gradient buffer for the separate Adam call (see step())
        self.grads = None if self.local else params.zeros_like()
        self.m = params.zeros_like()
        self.v = params.zeros_like()
        self.proj = api.ProjectedBuffers.alloc(self.n, 1, dev)
        cache = self.local and self.n * len(self.cams) * api.ProjectedBuffers.BYTES_PER_ENTRY <= projection_cache_bytes
        self.proj_views = [api.ProjectedBuffers.alloc(self.n, 1, dev) for _ in self.cams] if cache else None
        self._projected = [False] * len(self.cams)
        self.image = torch.zeros(1, 3, H, W, dtype=torch.float32, device=dev)
        self.T = torch.zeros(1, H, W, dtype=torch.float32, device=dev)
        self.nc = torch.zeros(1, H, W, dtype=torch.int32, device=dev)
        self.dL = torch.zeros(1, 3, H, W, dtype=torch.float32, device=dev)
        self.loss_sum = torch.zeros(1, dtype=torch.float32, device=dev)
        self.bwd_ws = api.render_backward_workspace(self.active[1] - self.active[0], 1, dev)
        self.state = api.render_state(self.cams[:1], dev)
        self.step_count = 0
        self.bins = None
        self._capacity = capacity
        self.ensure_capacity()

    def ensure_capacity(self, headroom=1.15):
        """Size the pair buffers for every view at the current parameters (reads the
        device pair counts once per view; not part of a step).  The complete lists'
        pair count bounds the depth-sliced lists' for the same parameters."""
        need = 1
        dev = self.params.means.device
        W, H = self.cams[0].width, self.cams[0].height
        probe = None
        for vi in range(len(self.cams)):
            cam = [self.cams[vi]]
            api.project_preprocess(self.params, cam, self.proj)
            if probe is None:
                probe = api.BinBuffers.alloc(self.n, 1, W, H, self._capacity or 1 << 20, dev, _ffi.BINS_COMPLETE)
            while True:
                api.bin_and_sort(self.proj, cam, self.active, self.local, probe)
                c = probe.read_counters()
                if not c["overflow"]:
                    break
                probe = api.BinBuffers.alloc(self.n, 1, W, H, int(c["pairs"] * 1.05) + 1024, dev, _ffi.BINS_COMPLETE)
            need = max(need, c["pairs"])
        del probe
        cap = int(need * headroom) + 1024
        if self.bins is None or self.bins.capacity < cap:
            # local steps: few tiles need the second depth slab
            mode = _ffi.BINS_DEPTH_SLICED_LOCAL if self.local else _ffi.BINS_DEPTH_SLICED
            self.bins = api.BinBuffers.alloc(self.n, 1, W, H, cap, dev, mode)
        self.bins.counters.zero_()
        self._prepare_calls()
        return need

    def _prepare_calls(self):
        """Build every ctypes argument of a step once (buffers never move)."""
        a0, a1 = self.active
        self._cams = [api.camera_array([c]) for c in self.cams]
        self._g = self.params.as_gaussians()
        self._pp = self.params.as_params()
        self._m = self.m.as_params()
        self._v = self.v.as_params()
        self._proj = self.proj.struct()
        self._proj_views = None if self.proj_views is None else [pv.struct() for pv in self.proj_views]
        self._bins = self.bins.struct()
        self._range = _ffi.Range(a0, a1)
        self._bg = (ctypes.c_float * 3)(*self.bg)
        self._hp = _ffi.AdamHParams()
        self._hp.lr = (ctypes.c_float * 6)(*[float(x) for x in self.lr])
        self._hp.beta1, self._hp.beta2, self._hp.eps = 0.9, 0.999, 1e-15
        # the separate Adam call clears the gradient rows it used (full steps), and skips
        # the update of a step whose lists overflowed the pair capacity
        self._hp.zero_grads = 1
        self._hp.skip_flag = ctypes.c_void_p(self.bins.counters.data_ptr() + 4 * _ffi.C_OVERFLOW)
        self._gr = None if self.grads is None else self.grads.as_params()
        p = lambda t: ctypes.c_void_p(t.data_ptr())
        self._ptrs = {"image": p(self.image), "T": p(self.T), "nc": p(self.nc), "dL": p(self.dL),
                      "loss": p(self.loss_sum), "ws": p(self.bins.ws), "bws": p(self.bwd_ws), "state": p(self.state),
                      "targets": [p(self.targets[v:v + 1]) for v in range(len(self.cams))]}
        self._sizes = (self.bins.ws.numel(), self.bwd_ws.numel(), self.state.numel())

    def prune(self, centers, radii):
        """Remove the changed Gaussians whose centre has left every sphere (Sec. 3.3
        "Sphere Pruning"; the paper checks every 15 iterations): the membership test and
        the compaction of parameters and Adam moments run in the library
        (clsp_sphere_keep, clsp_compact_rows); the change set stays the contiguous suffix
        after the unchanged rows.  ``centers`` [S, 3], ``radii`` [S] (device float32, e.g.
        from ``api.fit_spheres``).  Reads the kept count back (synchronises) and returns
        how many rows were removed.  The parameter tensors of ``params`` (and the
        moments) are replaced by the shorter ones; frozen rows keep their cached
        projections, and the pair buffers keep their capacity (removing Gaussians only
        removes pairs)."""
        if not self.local:
            raise ValueError("pruning applies to the change set of local optimisation")
        a0, a1 = self.active
        keep, kept = api.sphere_keep(self.params.means, (a0, a1), centers, radii)
        k = int(kept.item())
        if k == a1 - a0:
            return 0
        n_new = a0 + k
        dev = self.params.means.device
        deg = self.params.sh_degree
        newp, newm, newv = (api.GaussianTensors.zeros(n_new, deg, dev) for _ in range(3))
        api.compact_rows(self.params, (a0, a1), keep, newp, moments=(self.m, self.v, newm, newv))
        for old, new in ((self.params, newp), (self.m, newm), (self.v, newv)):
            for name in api.GaussianTensors.NAMES:
                setattr(old, name, getattr(new, name))
        self.n = n_new
        self.active = (a0, n_new)
        cut = lambda pb: api.ProjectedBuffers(pb.splat[:n_new], pb.depth[:n_new], pb.rect[:n_new], pb.flags[:n_new],
                                              n_new, 1)
        self.proj = cut(self.proj)
        if self.proj_views is not None:
            self.proj_views = [cut(pv) for pv in self.proj_views]
        self.bins.n = n_new
        self._frozen_orders = {}
        self.bwd_ws = api.render_backward_workspace(k, 1, dev)
        self._prepare_calls()
        return (a1 - a0) - k

    def _frozen_image(self, view):
        """Device pointer of the render of the unchanged rows [0, a0) from view ``view``
        (made on first use, not part of a step)."""
        if view not in self._frozen_images:
            a0 = self.active[0]
            dev = self.params.means.device
            cam = [self.cams[view]]
            g = api.GaussianTensors(*[getattr(self.params, k)[..., :a0].contiguous() for k in api.GaussianTensors.NAMES],
                                    self.params.sh_degree)
            proj = api.project_preprocess(g, cam)
            cap = 1 << 20
            while True:
                bins = api.bin_and_sort(proj, cam, capacity=cap)
                img, _, _ = api.render_forward(proj, bins, cam, self.bg)
                c = bins.read_counters()
                if not c["overflow"]:
                    break
                cap = int(c["pairs"] * 1.1) + 1024
            self._frozen_images[view] = img
        return ctypes.c_void_p(self._frozen_images[view].data_ptr())

    def _frozen_order(self, view, proj, st):
        """(pointer, bytes) of view ``view``'s stored depth order of the unchanged rows,
        made from ``proj`` (the view's projection) on the step's stream on first use."""
        if view not in self._frozen_orders:
            L = api.lib()
            a0 = self.active[0]
            nb = L.clsp_frozen_order_bytes(self.n, 1, a0)
            buf = torch.empty(max(1, nb), dtype=torch.uint8, device=self.params.means.device)
            check(L.clsp_frozen_order(ctypes.byref(proj), self._cams[view], 1, self.n, a0, ctypes.c_void_p(buf.data_ptr()),
                                      nb, self._ptrs["ws"], self._sizes[0], st))
            self._frozen_orders[view] = (buf, ctypes.c_void_p(buf.data_ptr()), nb)
        _, ptr, nb = self._frozen_orders[view]
        return ptr, nb

    def invalidate_projections(self):
        """The next step on each view projects every row again, and renders the unchanged
        rows again for the D-SSIM term and sorts them again (needed after rows outside the
        change set were modified)."""
        self._projected = [False] * len(self.cams)
        self._frozen_images = {}
        self._frozen_orders = {}

    def overflowed(self) -> bool:
        """True if any step since the last check ran out of pair capacity (sticky
        device flag; reading it synchronises)."""
        c = self.bins.counters
        flag = bool(c[C_STICKY].item())
        c[C_STICKY] = 0
        return flag

    TIMED_CALLS = ("bin_and_sort", "render_forward", "render_backward")

    def step_timed(self, view: int, events, stream=None):
        """``step`` with a pair of events recorded around each call named in
        ``events`` (a dict: call name -> (start, end); names from TIMED_CALLS), on the
        step's stream."""
        self.step(view, stream if stream is not None else torch.cuda.current_stream(), events)

    def render_stats(self):
        """Work of the last step: rendered tiles and pixels, pairs, entries (views x
        Gaussians with at least one pair), records each tile must read (the largest
        contributor count of its pixels), (pixel, record) evaluations (sum of
        contributor counts) and those of them whose record belongs to the active range
        (the evaluations whose gradient the backward computes)."""
        c = self.bins.read_counters()
        W, H = self.cams[0].width, self.cams[0].height
        TX, TY = api.tile_grid(W, H)
        dev = self.nc.device
        tiles = self.bins.tile_list[:c["tiles"]].long()
        nc = torch.zeros(1, TY * 16, TX * 16, dtype=torch.int64, device=dev)
        nc[:, :H, :W] = self.nc.long()
        per_tile = nc.reshape(TY, 16, TX, 16).permute(0, 2, 1, 3).reshape(TY * TX, 256)[tiles]
        inside = torch.zeros(TY * 16, TX * 16, dtype=torch.bool, device=dev)
        inside[:H, :W] = True
        pix = inside.reshape(TY, 16, TX, 16).permute(0, 2, 1, 3).reshape(TY * TX, 256)[tiles].sum()
        # active records among each pixel's first n_contrib list entries: prefix counts
        # of the active flag over the pair buffer, read at the two ranges of the list
        a0, a1 = self.active
        vals = self.bins.values[:max(c["pairs"], 1)].long()
        act = ((vals >= a0) & (vals < a1)).long()
        cum = torch.zeros(act.numel() + 1, dtype=torch.int64, device=dev)
        cum[1:] = torch.cumsum(act, 0)
        r1 = self.bins.ranges.view(-1, 2)[tiles].long()
        r2 = self.bins.ranges2.view(-1, 2)[tiles].long()
        len1 = (r1[:, 1] - r1[:, 0])[:, None]
        k1 = torch.minimum(per_tile, len1)
        k2 = (per_tile - len1).clamp(min=0)
        n_act = (cum[r1[:, 0:1] + k1] - cum[r1[:, 0:1]]) + (cum[r2[:, 0:1] + k2] - cum[r2[:, 0:1]])
        return {"tiles": c["tiles"], "tiles_total": TX * TY, "pairs": c["pairs"], "pairs_first_slab": c["pairs1"],
                "entries_first_slab": c["slab1"], "tiles_second_slab": c["alive"], "entries": c["entries"],
                "pixels": int(pix), "records": int(per_tile.max(dim=1).values.sum()),
                "pixel_records": int(per_tile.sum()), "pixel_records_active": int(n_act.sum())}

    def step(self, view: int, stream=None, events=None):
        """One step on view ``view``: the C-ABI calls in order, all on ``stream``
        (default: the current torch stream)."""
        L = api.lib()
        st = api._stream(stream)
        cam = self._cams[view]
        P = self._ptrs
        by = ctypes.byref
        use_mask = 1 if self.local else 0
        if self._proj_views is None:
            proj = self._proj
            check(L.clsp_project_preprocess(by(self._g), cam, 1, by(proj), st))
        else:
            proj = self._proj_views[view]
            if self._projected[view]:
                check(L.clsp_project_preprocess_rows(by(self._g), cam, 1, self._range, by(proj), st))
            else:
                check(L.clsp_project_preprocess(by(self._g), cam, 1, by(proj), st))
                self._projected[view] = True
        ev = events or {}
        mark = lambda name, i: ev[name][i].record(stream) if name in ev else None
        if self.frozen_order and self.active[1] == self.n:
            optr, onb = self._frozen_order(view, proj, st)
            mark("bin_and_sort", 0)
            check(L.clsp_bin_and_sort_frozen(by(proj), cam, 1, self.active[0], optr, onb, by(self._bins), st))
            mark("bin_and_sort", 1)
        else:
            mark("bin_and_sort", 0)
            check(L.clsp_bin_and_sort(by(proj), cam, 1, self._range, use_mask, by(self._bins), st))
            mark("bin_and_sort", 1)
        mark("render_forward", 0)
        if self.loss == "l1":
            # the forward also writes the L1 loss gradient of the pixels it renders
            check(L.clsp_render_forward_l1(by(proj), by(self._bins), cam, 1, self._bg, P["targets"][view],
                                           P["image"], P["T"], P["nc"], P["state"], self._sizes[2], P["dL"],
                                           P["loss"], st))
        else:
            check(L.clsp_render_forward(by(proj), by(self._bins), cam, 1, self._bg, P["image"], P["T"], P["nc"],
                                        P["state"], self._sizes[2], st))
            frozen = self._frozen_image(view) if self.local else None
            check(L.clsp_l1_dssim_loss_grad(P["image"], P["targets"][view], frozen, by(self._bins), cam, 1,
                                            ctypes.c_float(api.LAMBDA_DSSIM), P["dL"], P["loss"], st))
        mark("render_forward", 1)
        self.step_count += 1
        self._hp.step = self.step_count
        mark("render_backward", 0)
        if self.local:
            # the preprocess backward applies each changed row's Adam update from the
            # gradients it has just computed (no gradient buffer, no Adam launch)
            check(L.clsp_render_backward_adam(by(self._g), by(proj), by(self._bins), cam, 1, self._bg, self._range,
                                              P["T"], P["nc"], P["state"], self._sizes[2], P["dL"], by(self._pp),
                                              by(self._m), by(self._v), by(self._hp), P["bws"], self._sizes[1], st))
            mark("render_backward", 1)
        else:
            # every row: Adam's own kernel streams the rows faster than the fused update
            check(L.clsp_render_backward(by(self._g), by(proj), by(self._bins), cam, 1, self._bg, self._range,
                                         P["T"], P["nc"], P["state"], self._sizes[2], P["dL"], by(self._gr), P["bws"],
                                         self._sizes[1], st))
            mark("render_backward", 1)
            check(L.clsp_masked_adam_step(by(self._pp), by(self._gr), by(self._m), by(self._v), self._range, None,
                                          by(self._hp), st))
