"""Python face of the clsplat C-ABI: the same calls, taking torch tensors.

Every function here only checks shapes, packs ctypes structs from tensor pointers and
calls the library on the current torch stream (or the stream given).  All computation
happens in the HIP kernels; there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _ffi
from ._ffi import check

TILE = _ffi.TILE


def lib():
    return _ffi.load()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _f32(t, device=None):
    t = torch.as_tensor(t, dtype=torch.float32, device=device)
    return t.contiguous()


def tile_grid(width, height):
    return (width + TILE - 1) // TILE, (height + TILE - 1) // TILE


# ------------------------------------------------------------------ cameras
def camera_array(cams):
    """ctypes array of clsp_camera from objects with R, t, fx, fy, cx, cy, width,
    height (e.g. ``scenes.Camera``)."""
    arr = (_ffi.Camera * len(cams))()
    for i, c in enumerate(cams):
        R = np.asarray(c.R, dtype=np.float32).reshape(9)
        t = np.asarray(c.t, dtype=np.float32).reshape(3)
        arr[i].R = (ctypes.c_float * 9)(*R.tolist())
        arr[i].t = (ctypes.c_float * 3)(*t.tolist())
        arr[i].fx, arr[i].fy, arr[i].cx, arr[i].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[i].width, arr[i].height = int(c.width), int(c.height)
    return arr


# ------------------------------------------------------------------ parameter sets
@dataclass
class GaussianTensors:
    """Raw parameters on the device, component-major: means [3, N], log_scales [3, N],
    quats [4, N], opacity_logit [N], sh [K, 3, N]."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logit: torch.Tensor
    sh: torch.Tensor
    sh_degree: int

    NAMES = ("means", "log_scales", "quats", "opacity_logit", "sh")

    @property
    def n(self) -> int:
        return int(self.means.shape[-1])

    @classmethod
    def from_scene(cls, scene, device):
        return cls(*[_f32(a, device) for a in scene.param_arrays()], scene.sh_degree)

    @classmethod
    def zeros(cls, n, sh_degree, device):
        K = (sh_degree + 1) ** 2
        z = lambda *s: torch.zeros(*s, dtype=torch.float32, device=device)
        return cls(z(3, n), z(3, n), z(4, n), z(n), z(K, 3, n), sh_degree)

    def zeros_like(self):
        return GaussianTensors(*[torch.zeros_like(getattr(self, k)) for k in self.NAMES], self.sh_degree)

    def clone(self):
        return GaussianTensors(*[getattr(self, k).clone() for k in self.NAMES], self.sh_degree)

    def tensors(self):
        return [getattr(self, k) for k in self.NAMES]

    def check(self):
        n = self.n
        K = (self.sh_degree + 1) ** 2
        shapes = {"means": (3, n), "log_scales": (3, n), "quats": (4, n), "opacity_logit": (n,), "sh": (K, 3, n)}
        for k, s in shapes.items():
            t = getattr(self, k)
            if tuple(t.shape[-len(s):]) != s or t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError(f"{k}: expected contiguous float32 CUDA tensor of shape {s}, got "
                                 f"{tuple(t.shape)} {t.dtype} contiguous={t.is_contiguous()} cuda={t.is_cuda}")

    def as_gaussians(self, gather=None, n=None):
        self.check()
        g = _ffi.Gaussians()
        g.means, g.log_scales, g.quats = _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats)
        g.opacity_logit, g.sh = _ptr(self.opacity_logit), _ptr(self.sh)
        g.n_rows = self.n
        if gather is not None:
            if gather.dtype != torch.int32 or not gather.is_contiguous():
                raise ValueError("gather must be a contiguous int32 tensor")
            g.gather = _ptr(gather)
            g.n = int(gather.numel())
        else:
            g.gather = None
            g.n = self.n if n is None else int(n)
        g.sh_degree = self.sh_degree
        return g

    def as_params(self):
        self.check()
        p = _ffi.Params()
        p.means, p.log_scales, p.quats = _ptr(self.means), _ptr(self.log_scales), _ptr(self.quats)
        p.opacity_logit, p.sh = _ptr(self.opacity_logit), _ptr(self.sh)
        p.n = self.n
        p.sh_degree = self.sh_degree
        return p


# ------------------------------------------------------------------ buffers
@dataclass
class ProjectedBuffers:
    splat: torch.Tensor   # [V*N, 12] float32
    depth: torch.Tensor   # [V*N] float32
    rect: torch.Tensor    # [V*N, 2] int32 (uint32 bit patterns)
    flags: torch.Tensor   # [V*N] int32
    n: int
    views: int
    BYTES_PER_ENTRY = 64   # splat 48 + depth 4 + rect 8 + flags 4

    @classmethod
    def alloc(cls, n, views, device):
        e = max(1, n * views)
        return cls(torch.empty(e, 12, dtype=torch.float32, device=device),
                   torch.empty(e, dtype=torch.float32, device=device),
                   torch.empty(e, 2, dtype=torch.int32, device=device),
                   torch.empty(e, dtype=torch.int32, device=device), n, views)

    def struct(self):
        p = _ffi.Projected()
        p.splat, p.depth, p.rect, p.flags = _ptr(self.splat), _ptr(self.depth), _ptr(self.rect), _ptr(self.flags)
        return p


@dataclass
class BinBuffers:
    values: torch.Tensor      # [capacity] int32 (entry index)
    keys: torch.Tensor        # [capacity] int32 (global tile)
    ranges: torch.Tensor      # [V*T, 2] int32, first lists
    ranges2: torch.Tensor     # [V*T, 2] int32, second lists (depth-sliced mode)
    tile_mask: torch.Tensor   # [V, ceil(T/32)] int32
    alive_mask: torch.Tensor  # [V, ceil(T/32)] int32
    tile_list: torch.Tensor   # [V*T] int32
    counters: torch.Tensor    # [16] int32
    ws: torch.Tensor          # workspace bytes
    capacity: int
    n: int
    views: int
    width: int
    height: int
    mode: int = _ffi.BINS_DEPTH_SLICED

    @classmethod
    def alloc(cls, n, views, width, height, capacity, device, mode=_ffi.BINS_DEPTH_SLICED):
        TX, TY = tile_grid(width, height)
        T = TX * TY
        cap = max(1, int(capacity))
        wsb = lib().clsp_bin_and_sort_workspace_bytes(n, views, width, height, cap)
        i32 = lambda *s: torch.zeros(*s, dtype=torch.int32, device=device)
        wpv = (T + 31) // 32
        return cls(i32(cap), i32(cap), i32(views * T, 2), i32(views * T, 2), i32(views, wpv), i32(views, wpv),
                   i32(views * T), i32(_ffi.N_COUNTERS), torch.empty(max(1, wsb), dtype=torch.uint8, device=device),
                   cap, n, views, width, height, int(mode))

    def struct(self):
        b = _ffi.Bins()
        b.values, b.keys, b.ranges, b.ranges2 = _ptr(self.values), _ptr(self.keys), _ptr(self.ranges), _ptr(self.ranges2)
        b.tile_mask, b.alive_mask = _ptr(self.tile_mask), _ptr(self.alive_mask)
        b.tile_list, b.counters = _ptr(self.tile_list), _ptr(self.counters)
        b.ws, b.ws_bytes = _ptr(self.ws), self.ws.numel()
        b.capacity, b.n, b.mode = self.capacity, self.n, self.mode
        return b

    def read_counters(self):
        c = self.counters.cpu().numpy().view(np.uint32)
        return {"pairs": int(c[_ffi.C_PAIRS]), "overflow": bool(c[_ffi.C_OVERFLOW]), "tiles": int(c[_ffi.C_TILES]),
                "written": int(c[_ffi.C_WRITTEN]), "entries": int(c[_ffi.C_ENTRIES]), "slab1": int(c[_ffi.C_SLAB1]),
                "pairs1": int(c[_ffi.C_PAIRS1]), "alive": int(c[_ffi.C_ALIVE])}


# ------------------------------------------------------------------ calls
def project_preprocess(g: GaussianTensors, cams, out: ProjectedBuffers | None = None, gather=None, stream=None):
    n = g.n if gather is None else int(gather.numel())
    if out is None:
        out = ProjectedBuffers.alloc(n, len(cams), g.means.device)
    if out.n != n or out.views != len(cams):
        raise ValueError("projected buffers sized for another scene")
    gs = g.as_gaussians(gather)
    ca = camera_array(cams)
    check(lib().clsp_project_preprocess(ctypes.byref(gs), ca, len(cams), ctypes.byref(out.struct()), _stream(stream)))
    return out


def project_preprocess_rows(g: GaussianTensors, cams, rows, out: ProjectedBuffers, stream=None):
    """Re-project rows [rows[0], rows[1]) of every view into ``out`` (the other entries
    keep their values)."""
    if out.n != g.n or out.views != len(cams):
        raise ValueError("projected buffers sized for another scene")
    gs = g.as_gaussians()
    check(lib().clsp_project_preprocess_rows(ctypes.byref(gs), camera_array(cams), len(cams),
                                             _ffi.Range(int(rows[0]), int(rows[1])), ctypes.byref(out.struct()),
                                             _stream(stream)))
    return out


def bin_and_sort(proj: ProjectedBuffers, cams, active=None, use_mask=False, bins: BinBuffers | None = None,
                 capacity=None, mode=_ffi.BINS_DEPTH_SLICED, stream=None):
    """Render mask and per-tile depth order.  With depth-sliced bins (the default) the
    forward call completes the lists of the tiles that need more than the first slab."""
    n = proj.n
    a0, a1 = (0, n) if active is None else (int(active[0]), int(active[1]))
    if bins is None:
        cap = capacity if capacity is not None else max(1024, 64 * n * len(cams))
        bins = BinBuffers.alloc(n, len(cams), cams[0].width, cams[0].height, cap, proj.splat.device, mode)
    if bins.n != n or bins.views != len(cams):
        raise ValueError("bins sized for another projection")
    ca = camera_array(cams)
    check(lib().clsp_bin_and_sort(ctypes.byref(proj.struct()), ca, len(cams), _ffi.Range(a0, a1), 1 if use_mask else 0,
                                  ctypes.byref(bins.struct()), _stream(stream)))
    return bins


@dataclass
class FrozenOrder:
    """Stored depth order of the unchanged rows [0, a0) (clsp_frozen_order): valid for
    the projection rows, cameras and image size it was built from."""
    buf: torch.Tensor   # device bytes
    n: int
    views: int
    a0: int
    width: int
    height: int


def frozen_order(proj: ProjectedBuffers, cams, a0, ws: torch.Tensor | None = None, stream=None) -> FrozenOrder:
    """Depth order of the entries of rows [0, a0) of ``proj`` (made once per camera set
    during local optimisation of the change set [a0, n)).  ``ws``: scratch of at least
    ``clsp_bin_and_sort_workspace_bytes(n, views, w, h, 0)`` bytes (allocated when None)."""
    n, V, W, H = proj.n, len(cams), cams[0].width, cams[0].height
    L = lib()
    nb = L.clsp_frozen_order_bytes(n, V, int(a0))
    if nb == 0:
        raise ValueError(f"a0 = {a0} not in [0, {n}]")
    dev = proj.splat.device
    buf = torch.empty(nb, dtype=torch.uint8, device=dev)
    need = L.clsp_bin_and_sort_workspace_bytes(n, V, W, H, 0)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(1, need), dtype=torch.uint8, device=dev)
    check(L.clsp_frozen_order(ctypes.byref(proj.struct()), camera_array(cams), V, n, int(a0), _ptr(buf), nb, _ptr(ws),
                              ws.numel(), _stream(stream)))
    return FrozenOrder(buf, n, V, int(a0), W, H)


def bin_and_sort_frozen(proj: ProjectedBuffers, cams, order: FrozenOrder, bins: BinBuffers | None = None,
                        capacity=None, mode=_ffi.BINS_DEPTH_SLICED, stream=None):
    """``bin_and_sort(proj, cams, (order.a0, n), use_mask=True, ...)`` with the unchanged
    rows' depth order taken from ``order`` (the same lists)."""
    n, V = proj.n, len(cams)
    if (order.n, order.views, order.width, order.height) != (n, V, cams[0].width, cams[0].height):
        raise ValueError("frozen order built for another projection or camera set")
    if bins is None:
        cap = capacity if capacity is not None else max(1024, 64 * n * V)
        bins = BinBuffers.alloc(n, V, cams[0].width, cams[0].height, cap, proj.splat.device, mode)
    if bins.n != n or bins.views != V:
        raise ValueError("bins sized for another projection")
    check(lib().clsp_bin_and_sort_frozen(ctypes.byref(proj.struct()), camera_array(cams), V, order.a0, _ptr(order.buf),
                                         order.buf.numel(), ctypes.byref(bins.struct()), _stream(stream)))
    return bins


def render_state(cams, device):
    """Device buffer for the forward's compositing state (needed by the backward)."""
    b = lib().clsp_render_state_bytes(len(cams), cams[0].width, cams[0].height)
    return torch.empty(max(1, b), dtype=torch.uint8, device=device)


def render_forward(proj, bins, cams, bg=(0.0, 0.0, 0.0), image=None, T_final=None, n_contrib=None, state=None,
                   stream=None):
    """Returns (image, T_final, n_contrib).  ``state`` (from ``render_state``) is
    filled when given; pass it to ``render_backward``."""
    V, H, W = len(cams), cams[0].height, cams[0].width
    dev = proj.splat.device
    if image is None:
        image = torch.zeros(V, 3, H, W, dtype=torch.float32, device=dev)
    if T_final is None:
        T_final = torch.zeros(V, H, W, dtype=torch.float32, device=dev)
    if n_contrib is None:
        n_contrib = torch.zeros(V, H, W, dtype=torch.int32, device=dev)
    for t, shape in ((image, (V, 3, H, W)), (T_final, (V, H, W)), (n_contrib, (V, H, W))):
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"output of shape {tuple(t.shape)}, expected contiguous {shape}")
    bgc = (ctypes.c_float * 3)(*[float(x) for x in bg])
    check(lib().clsp_render_forward(ctypes.byref(proj.struct()), ctypes.byref(bins.struct()), camera_array(cams), V, bgc,
                                    _ptr(image), _ptr(T_final), _ptr(n_contrib), _ptr(state),
                                    0 if state is None else state.numel(), _stream(stream)))
    return image, T_final, n_contrib


def render_forward_l1(proj, bins, cams, target, bg=(0.0, 0.0, 0.0), image=None, T_final=None, n_contrib=None,
                      state=None, dL=None, loss_sum=None, stream=None):
    """``render_forward`` and ``l1_loss_grad`` in one pass.  Returns (image, T_final,
    n_contrib, dL)."""
    V, H, W = len(cams), cams[0].height, cams[0].width
    dev = proj.splat.device
    image = torch.zeros(V, 3, H, W, dtype=torch.float32, device=dev) if image is None else image
    T_final = torch.zeros(V, H, W, dtype=torch.float32, device=dev) if T_final is None else T_final
    n_contrib = torch.zeros(V, H, W, dtype=torch.int32, device=dev) if n_contrib is None else n_contrib
    dL = torch.zeros(V, 3, H, W, dtype=torch.float32, device=dev) if dL is None else dL
    for t, shape in ((image, (V, 3, H, W)), (T_final, (V, H, W)), (n_contrib, (V, H, W)), (target, (V, 3, H, W)),
                     (dL, (V, 3, H, W))):
        if tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"tensor of shape {tuple(t.shape)}, expected contiguous {shape}")
    bgc = (ctypes.c_float * 3)(*[float(x) for x in bg])
    check(lib().clsp_render_forward_l1(ctypes.byref(proj.struct()), ctypes.byref(bins.struct()), camera_array(cams), V,
                                       bgc, _ptr(target), _ptr(image), _ptr(T_final), _ptr(n_contrib), _ptr(state),
                                       0 if state is None else state.numel(), _ptr(dL), _ptr(loss_sum),
                                       _stream(stream)))
    return image, T_final, n_contrib, dL


def l1_loss_grad(image, target, bins, cams, dL=None, loss_sum=None, stream=None):
    if dL is None:
        dL = torch.zeros_like(image)
    if tuple(target.shape) != tuple(image.shape) or target.dtype != torch.float32 or not target.is_contiguous():
        raise ValueError("target must be a contiguous float32 tensor shaped like image")
    check(lib().clsp_l1_loss_grad(_ptr(image), _ptr(target), ctypes.byref(bins.struct()), camera_array(cams), len(cams),
                                  _ptr(dL), _ptr(loss_sum), _stream(stream)))
    return dL


LAMBDA_DSSIM = 0.2


def l1_dssim_loss_grad(image, target, bins, cams, frozen=None, lam=LAMBDA_DSSIM, dL=None, loss_sum=None, stream=None):
    """dL/dimage of (1 - lam) L1 + lam (1 - SSIM) on the rendered tiles; ``frozen`` (like
    image) supplies the pixels of tiles that were not rendered (local steps)."""
    if dL is None:
        dL = torch.zeros_like(image)
    for t in (target, frozen):
        if t is not None and (tuple(t.shape) != tuple(image.shape) or t.dtype != torch.float32
                              or not t.is_contiguous()):
            raise ValueError("target and frozen must be contiguous float32 tensors shaped like image")
    check(lib().clsp_l1_dssim_loss_grad(_ptr(image), _ptr(target), _ptr(frozen), ctypes.byref(bins.struct()),
                                        camera_array(cams), len(cams), float(lam), _ptr(dL), _ptr(loss_sum),
                                        _stream(stream)))
    return dL


def render_backward_workspace(n_active, views, device):
    """Zero-filled (render_backward_adam needs a zero workspace and leaves it zero)."""
    b = lib().clsp_render_backward_workspace_bytes(int(n_active), int(views))
    return torch.zeros(max(1, b), dtype=torch.uint8, device=device)


def render_backward(g: GaussianTensors, proj, bins, cams, bg, active, T_final, n_contrib, state, dL,
                    grads: GaussianTensors, ws=None, stream=None):
    """Adds the gradients of the Gaussians in ``active`` to ``grads``; ``T_final``,
    ``n_contrib`` and ``state`` come from the ``render_forward`` call on ``bins``."""
    a0, a1 = (0, g.n) if active is None else (int(active[0]), int(active[1]))
    if ws is None:
        ws = render_backward_workspace(a1 - a0, len(cams), g.means.device)
    bgc = (ctypes.c_float * 3)(*[float(x) for x in bg])
    check(lib().clsp_render_backward(ctypes.byref(g.as_gaussians()), ctypes.byref(proj.struct()),
                                     ctypes.byref(bins.struct()), camera_array(cams), len(cams), bgc,
                                     _ffi.Range(a0, a1), _ptr(T_final), _ptr(n_contrib), _ptr(state),
                                     0 if state is None else state.numel(), _ptr(dL),
                                     ctypes.byref(grads.as_params()), _ptr(ws), ws.numel(), _stream(stream)))
    return grads


def render_backward_noalloc(g: GaussianTensors, proj, bins, cams, bg, active, T_final, n_contrib, state, dL,
                            grads: GaussianTensors, stream=None):
    """``render_backward`` with the library's static scratch instead of a workspace (the
    call allocates no device memory); calls that overlap on one GPU race."""
    a0, a1 = (0, g.n) if active is None else (int(active[0]), int(active[1]))
    bgc = (ctypes.c_float * 3)(*[float(x) for x in bg])
    check(lib().clsp_render_backward_noalloc(ctypes.byref(g.as_gaussians()), ctypes.byref(proj.struct()),
                                             ctypes.byref(bins.struct()), camera_array(cams), len(cams), bgc,
                                             _ffi.Range(a0, a1), _ptr(T_final), _ptr(n_contrib), _ptr(state),
                                             0 if state is None else state.numel(), _ptr(dL),
                                             ctypes.byref(grads.as_params()), _stream(stream)))
    return grads


def zero_grads(grads: GaussianTensors, active=None, stream=None):
    a0, a1 = (0, grads.n) if active is None else (int(active[0]), int(active[1]))
    check(lib().clsp_zero_grads(ctypes.byref(grads.as_params()), _ffi.Range(a0, a1), _stream(stream)))


# Published 3D Gaussian Splatting default learning rates (position scaled by the scene
# extent, 1.0 here), in the C-ABI group order.
DEFAULT_LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 2.5e-3 / 20.0)


def masked_adam_step(params: GaussianTensors, grads, exp_avg, exp_avg_sq, active, step, lr=DEFAULT_LR, beta1=0.9,
                     beta2=0.999, eps=1e-15, row_mask=None, stream=None, step_device=None, zero_grads=False,
                     skip_flag=None):
    """``step`` (host int) or ``step_device`` (int32 device tensor [1]) gives the 1-based
    step count of the bias corrections.  With ``zero_grads`` the gradient rows of
    ``active`` are set to zero after use.  ``skip_flag`` (a one-element 32-bit device
    tensor, e.g. ``bins.counters[1:2]``, the pair-capacity overflow): when it is nonzero
    on the device, nothing is updated."""
    a0, a1 = (0, params.n) if active is None else (int(active[0]), int(active[1]))
    hp = _ffi.AdamHParams()
    hp.lr = (ctypes.c_float * 6)(*[float(x) for x in lr])
    hp.beta1, hp.beta2, hp.eps, hp.step = float(beta1), float(beta2), float(eps), int(step or 0)
    hp.zero_grads = 1 if zero_grads else 0
    if step_device is not None:
        if step_device.dtype != torch.int32 or step_device.numel() != 1 or not step_device.is_cuda:
            raise ValueError("step_device must be an int32 CUDA tensor of one element")
        hp.step_device = step_device.data_ptr()
    if skip_flag is not None:
        if skip_flag.element_size() != 4 or skip_flag.numel() != 1 or not skip_flag.is_cuda:
            raise ValueError("skip_flag must be a 32-bit CUDA tensor of one element")
        hp.skip_flag = skip_flag.data_ptr()
    if row_mask is not None and (row_mask.dtype != torch.uint8 or row_mask.numel() != params.n):
        raise ValueError("row_mask must be uint8 [N]")
    check(lib().clsp_masked_adam_step(ctypes.byref(params.as_params()), ctypes.byref(grads.as_params()),
                                      ctypes.byref(exp_avg.as_params()), ctypes.byref(exp_avg_sq.as_params()),
                                      _ffi.Range(a0, a1), _ptr(row_mask), ctypes.byref(hp), _stream(stream)))


def render_backward_adam(g: GaussianTensors, proj, bins, cam, bg, active, T_final, n_contrib, state, dL, exp_avg,
                         exp_avg_sq, step, lr=DEFAULT_LR, beta1=0.9, beta2=0.999, eps=1e-15, ws=None, stream=None):
    """One view's backward and one Adam step of the rows in ``active`` (``g`` is updated
    in place): zero_grads + render_backward + masked_adam_step in one call, without a
    gradient buffer.  ``ws`` must be zero (as ``render_backward_workspace`` returns it);
    the call leaves it zero, so one workspace serves every step."""
    a0, a1 = (0, g.n) if active is None else (int(active[0]), int(active[1]))
    if ws is None:
        ws = render_backward_workspace(a1 - a0, 1, g.means.device)
    bgc = (ctypes.c_float * 3)(*[float(x) for x in bg])
    hp = _ffi.AdamHParams()
    hp.lr = (ctypes.c_float * 6)(*[float(x) for x in lr])
    hp.beta1, hp.beta2, hp.eps, hp.step = float(beta1), float(beta2), float(eps), int(step)
    check(lib().clsp_render_backward_adam(ctypes.byref(g.as_gaussians()), ctypes.byref(proj.struct()),
                                          ctypes.byref(bins.struct()), camera_array([cam]), 1, bgc,
                                          _ffi.Range(a0, a1), _ptr(T_final), _ptr(n_contrib), _ptr(state),
                                          0 if state is None else state.numel(), _ptr(dL),
                                          ctypes.byref(g.as_params()), ctypes.byref(exp_avg.as_params()),
                                          ctypes.byref(exp_avg_sq.as_params()), ctypes.byref(hp), _ptr(ws), ws.numel(),
                                          _stream(stream)))
    return g


# ------------------------------------------------------------------ change-region spheres
def _means_ptr(means):
    if means.dtype != torch.float32 or means.dim() != 2 or means.shape[0] != 3 or not means.is_contiguous():
        raise ValueError("means must be a contiguous float32 tensor [3, N]")
    return _ptr(means), int(means.shape[1])


def fit_spheres(means, rows, labels, n_spheres, stream=None):
    """Centres [S, 3] and radii [S] of the clusters ``labels`` (int32 [rows[1] -
    rows[0]], -1: none) of the rows ``rows`` of ``means`` [3, N]."""
    mp, nr = _means_ptr(means)
    r0, r1 = int(rows[0]), int(rows[1])
    if labels.dtype != torch.int32 or labels.numel() != r1 - r0 or not labels.is_contiguous():
        raise ValueError("labels must be a contiguous int32 tensor of one entry per row")
    centers = torch.empty(int(n_spheres), 3, dtype=torch.float32, device=means.device)
    radii = torch.empty(int(n_spheres), dtype=torch.float32, device=means.device)
    check(lib().clsp_fit_spheres(mp, nr, _ffi.Range(r0, r1), _ptr(labels), int(n_spheres), _ptr(centers), _ptr(radii),
                                 _stream(stream)))
    return centers, radii


def sphere_keep(means, rows, centers, radii, keep=None, kept=None, stream=None):
    """(keep uint8 [rows[1] - rows[0]], kept int32 [1]): which rows' centres lie in the
    union of the spheres, and how many."""
    mp, nr = _means_ptr(means)
    r0, r1 = int(rows[0]), int(rows[1])
    centers = centers.contiguous()
    radii = radii.contiguous()
    if keep is None:
        keep = torch.empty(max(r1 - r0, 1), dtype=torch.uint8, device=means.device)
    if kept is None:
        kept = torch.empty(1, dtype=torch.int32, device=means.device)
    check(lib().clsp_sphere_keep(mp, nr, _ffi.Range(r0, r1), _ptr(centers), _ptr(radii), int(radii.numel()),
                                 _ptr(keep), _ptr(kept), _stream(stream)))
    return keep, kept


def compact_workspace(n_changed, device):
    b = lib().clsp_compact_rows_workspace_bytes(int(n_changed))
    return torch.empty(max(1, b), dtype=torch.uint8, device=device)


def compact_rows(src: GaussianTensors, rows, keep, dst: GaussianTensors, moments=None, ws=None, stream=None):
    """Copy ``src`` to ``dst`` without the rows of [rows[0], N) whose ``keep`` is 0; with
    ``moments`` = (src_m, src_v, dst_m, dst_v) the Adam moments too."""
    r0, r1 = int(rows[0]), int(rows[1])
    if ws is None:
        ws = compact_workspace(r1 - r0, src.means.device)
    mo = [None] * 4 if moments is None else [ctypes.byref(m.as_params()) for m in moments]
    check(lib().clsp_compact_rows(ctypes.byref(src.as_params()), mo[0], mo[1], _ffi.Range(r0, r1), _ptr(keep),
                                  ctypes.byref(dst.as_params()), mo[2], mo[3], _ptr(ws), ws.numel(), _stream(stream)))
    return dst


# ------------------------------------------------------------------ change lifting
DILATE_FRACTION = 0.02


def dilation_radius(width):
    """The paper's dilation half-width: 2% of the image width, rounded (halves up)."""
    return int(DILATE_FRACTION * width + 0.5)


def dilate_masks(masks, radius, out=None, stream=None):
    """masks: uint8 [V, H, W] (nonzero = changed) -> uint8 [V, H, W] dilated by a square
    of half-width ``radius``."""
    if masks.dtype != torch.uint8 or masks.dim() != 3 or not masks.is_contiguous():
        raise ValueError("masks must be a contiguous uint8 tensor [V, H, W]")
    V, H, W = (int(x) for x in masks.shape)
    if out is None:
        out = torch.empty_like(masks)
    b = lib().clsp_dilate_masks_workspace_bytes(V, W, H)
    ws = torch.empty(max(1, b), dtype=torch.uint8, device=masks.device)
    check(lib().clsp_dilate_masks(_ptr(masks), V, W, H, int(radius), _ptr(out), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def majority_vote(means, cams, masks, n=None, stream=None):
    """(changed uint8 [n], in_count uint8 [n], out_count uint8 [n], n_changed int32 [1])
    for the centres ``means`` [3, N] (the first ``n`` rows) against the masks [V, H, W]."""
    mp, nr = _means_ptr(means)
    n = nr if n is None else int(n)
    if masks.dtype != torch.uint8 or masks.dim() != 3 or not masks.is_contiguous() or masks.shape[0] != len(cams):
        raise ValueError("masks must be a contiguous uint8 tensor [V, H, W], one per camera")
    if (int(masks.shape[1]), int(masks.shape[2])) != (cams[0].height, cams[0].width):
        raise ValueError("masks must have the cameras' size")
    dev = means.device
    changed = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    cin = torch.empty_like(changed)
    cout = torch.empty_like(changed)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    check(lib().clsp_majority_vote(mp, nr, n, camera_array(cams), len(cams), _ptr(masks), _ptr(cin), _ptr(cout),
                                   _ptr(changed), _ptr(cnt), _stream(stream)))
    return changed[:n], cin[:n], cout[:n], cnt


# ------------------------------------------------------------------ history
def _history_ws(device):
    return torch.empty(max(1, lib().clsp_history_workspace_bytes()), dtype=torch.uint8, device=device)


def _u8(t, n, what):
    if t.dtype != torch.uint8 or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous uint8 tensor of {n} entries")
    return _ptr(t)


def reorder_static_first(src: GaussianTensors, changed, stream=None):
    """(dst, n_static int32 [1]): src's rows with changed = 0 first, then those with 1."""
    dev = src.means.device
    dst = GaussianTensors.zeros(src.n, src.sh_degree, dev)
    ns = torch.empty(1, dtype=torch.int32, device=dev)
    ws = _history_ws(dev)
    check(lib().clsp_reorder_static_first(ctypes.byref(src.as_params()), _u8(changed, src.n, "changed"),
                                          ctypes.byref(dst.as_params()), _ptr(ns), _ptr(ws), ws.numel(),
                                          _stream(stream)))
    return dst, ns


def recover_previous(latest: GaussianTensors, indicator, changed_before: GaussianTensors, stream=None):
    """G^{k-1} from G^k, I^k and O^k."""
    dev = latest.means.device
    n = int(indicator.numel())
    dst = GaussianTensors.zeros(n, latest.sh_degree, dev)
    ws = _history_ws(dev)
    check(lib().clsp_recover_previous(ctypes.byref(latest.as_params()), _u8(indicator, n, "indicator"),
                                      ctypes.byref(changed_before.as_params()), ctypes.byref(dst.as_params()),
                                      _ptr(ws), ws.numel(), _stream(stream)))
    return dst


def merge_updates(prev: GaussianTensors, ind1, ind2, o1: GaussianTensors, o2: GaussianTensors, n_out, stream=None):
    """The rows of ``prev`` neither update marks, then o1's, then o2's (``n_out`` rows)."""
    dev = prev.means.device
    dst = GaussianTensors.zeros(int(n_out), prev.sh_degree, dev)
    ws = _history_ws(dev)
    check(lib().clsp_merge_updates(ctypes.byref(prev.as_params()), _u8(ind1, prev.n, "ind1"), _u8(ind2, prev.n, "ind2"),
                                   ctypes.byref(o1.as_params()), ctypes.byref(o2.as_params()),
                                   ctypes.byref(dst.as_params()), _ptr(ws), ws.numel(), _stream(stream)))
    return dst
