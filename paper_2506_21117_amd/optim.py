"""Local and full-scene optimisation steps over the C-ABI.

One step (one view, the 3D Gaussian Splatting convention) runs, all on one stream:
zero the change set's gradient rows -> project all Gaussians -> render mask and per-tile
depth order (masked tiles only in local mode) -> forward render -> L1 loss gradient ->
backward render and preprocess backward for the change set -> masked Adam on the
change set.  This is the local optimisation of CL-Splats (Sec. 3.3 "Local Optimization
Kernel"; Supp. "3DGS Optimization in Changed Regions"); the full-scene step is the same
with no mask and every row active.
"""
from __future__ import annotations

import torch

from . import api
from ._ffi import C_OVERFLOW, C_PAIRS, C_STICKY


class SplatOptimizer:
    def __init__(self, params: api.GaussianTensors, cams, targets, active=None, local=True, bg=(0.0, 0.0, 0.0),
                 capacity=None, lr=api.DEFAULT_LR):
        """params: device parameters (updated in place); cams: list of cameras of one
        size; targets: [V, 3, H, W] float32 device tensor; active: (a0, a1) change set
        (default: all rows); local: restrict rendering to the change set's tile mask."""
        self.params = params
        self.cams = list(cams)
        self.targets = targets
        self.n = params.n
        self.local = bool(local)
        self.active = (0, self.n) if (active is None or not local) else (int(active[0]), int(active[1]))
        self.bg = tuple(float(x) for x in bg)
        self.lr = lr
        dev = params.means.device
        W, H = self.cams[0].width, self.cams[0].height
        self.grads = params.zeros_like()
        self.m = params.zeros_like()
        self.v = params.zeros_like()
        self.proj = api.ProjectedBuffers.alloc(self.n, 1, dev)
        self.image = torch.zeros(1, 3, H, W, dtype=torch.float32, device=dev)
        self.T = torch.zeros(1, H, W, dtype=torch.float32, device=dev)
        self.nc = torch.zeros(1, H, W, dtype=torch.int32, device=dev)
        self.dL = torch.zeros(1, 3, H, W, dtype=torch.float32, device=dev)
        self.loss_sum = torch.zeros(1, dtype=torch.float32, device=dev)
        self.bwd_ws = api.render_backward_workspace(self.active[1] - self.active[0], 1, dev)
        self.step_count = 0
        self.bins = None
        self._capacity = capacity
        self.ensure_capacity()

    def ensure_capacity(self, headroom=1.15):
        """Size the pair buffers for every view at the current parameters (reads the
        device pair counts once per view; not part of a step)."""
        need = 1
        for vi in range(len(self.cams)):
            cam = [self.cams[vi]]
            api.project_preprocess(self.params, cam, self.proj)
            b = self.bins if self.bins is not None else api.BinBuffers.alloc(
                self.n, 1, cam[0].width, cam[0].height, self._capacity or 1 << 20, self.params.means.device)
            api.bin_and_sort(self.proj, cam, self.active, self.local, b)
            need = max(need, b.read_counters()["pairs"])
            self.bins = b
        if self.bins.capacity < need:
            cap = int(need * headroom) + 1024
            self.bins = api.BinBuffers.alloc(self.n, 1, self.cams[0].width, self.cams[0].height, cap,
                                             self.params.means.device)
        self.bins.counters.zero_()
        return need

    def overflowed(self) -> bool:
        """True if any step since the last check ran out of pair capacity (sticky
        device flag; reading it synchronises)."""
        c = self.bins.counters
        flag = bool(c[C_STICKY].item())
        c[C_STICKY] = 0
        return flag

    def step_timed(self, view: int, events, stream=None):
        """``step`` with the two events recorded around the forward render call on
        the step's stream."""
        self.step(view, stream, events)

    def render_stats(self):
        """Work of the last step's forward render: rendered tiles and pixels, pairs,
        records each tile must read (the largest contributor count of its pixels) and
        (pixel, record) evaluations (sum of contributor counts)."""
        c = self.bins.read_counters()
        W, H = self.cams[0].width, self.cams[0].height
        TX, TY = api.tile_grid(W, H)
        tiles = self.bins.tile_list[:c["tiles"]].long()
        nc = torch.zeros(1, TY * 16, TX * 16, dtype=torch.int64, device=self.nc.device)
        nc[:, :H, :W] = self.nc.long()
        per_tile = nc.reshape(TY, 16, TX, 16).permute(0, 2, 1, 3).reshape(TY * TX, 256)[tiles]
        inside = torch.zeros(TY * 16, TX * 16, dtype=torch.bool, device=nc.device)
        inside[:H, :W] = True
        pix = inside.reshape(TY, 16, TX, 16).permute(0, 2, 1, 3).reshape(TY * TX, 256)[tiles].sum()
        return {"tiles": c["tiles"], "tiles_total": TX * TY, "pairs": c["pairs"], "pixels": int(pix),
                "records": int(per_tile.max(dim=1).values.sum()), "pixel_records": int(per_tile.sum())}

    def step(self, view: int, stream=None, events=None):
        cam = [self.cams[view]]
        a = self.active
        api.zero_grads(self.grads, a, stream)
        api.project_preprocess(self.params, cam, self.proj, stream=stream)
        api.bin_and_sort(self.proj, cam, a, self.local, self.bins, stream=stream)
        if events is not None:
            events[0].record(stream)
        api.render_forward(self.proj, self.bins, cam, self.bg, self.image, self.T, self.nc, stream=stream)
        if events is not None:
            events[1].record(stream)
        api.l1_loss_grad(self.image, self.targets[view:view + 1], self.bins, cam, self.dL, self.loss_sum,
                         stream=stream)
        api.render_backward(self.params, self.proj, self.bins, cam, self.bg, a, self.T, self.nc, self.dL, self.grads,
                            self.bwd_ws, stream=stream)
        self.step_count += 1
        api.masked_adam_step(self.params, self.grads, self.m, self.v, a, self.step_count, self.lr, stream=stream)
