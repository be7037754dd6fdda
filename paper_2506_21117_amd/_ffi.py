"""ctypes declarations of the clsplat C-ABI (include/clsplat.h)."""
from __future__ import annotations

import ctypes
from ctypes import POINTER, c_char_p, c_float, c_int32, c_int64, c_size_t, c_uint8, c_uint32, c_void_p
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libclsplat.so"

CLSP_OK = 0
CLSP_ERR_INVALID_ARG = -1
CLSP_ERR_HIP = -3
CLSP_ERR_UNSUPPORTED = -4
TILE = 16

FLAG_VISIBLE, FLAG_CLAMP_X, FLAG_CLAMP_Y, FLAG_SHCLAMP_R = 1, 2, 4, 8
C_PAIRS, C_OVERFLOW, C_TILES, C_WRITTEN, C_ENTRIES, C_STICKY, C_SLAB1, C_PAIRS1, C_ALIVE = 0, 1, 2, 3, 4, 5, 6, 7, 8
N_COUNTERS = 16
BINS_COMPLETE, BINS_DEPTH_SLICED, BINS_DEPTH_SLICED_LOCAL = 0, 1, 2

EXPORTED = (
    "clsp_version", "clsp_last_error", "clsp_project_preprocess", "clsp_project_preprocess_rows",
    "clsp_bin_and_sort_workspace_bytes",
    "clsp_bin_and_sort", "clsp_frozen_order_bytes", "clsp_frozen_order", "clsp_bin_and_sort_frozen",
    "clsp_render_state_bytes", "clsp_render_forward", "clsp_render_forward_l1",
    "clsp_l1_loss_grad",
    "clsp_render_backward_workspace_bytes",
    "clsp_render_backward", "clsp_masked_adam_step", "clsp_zero_grads", "clsp_render_backward_adam",
    "clsp_render_backward_noalloc", "clsp_fit_spheres", "clsp_sphere_keep", "clsp_compact_rows_workspace_bytes",
    "clsp_compact_rows", "clsp_dilate_masks_workspace_bytes", "clsp_dilate_masks", "clsp_majority_vote",
    "clsp_history_workspace_bytes", "clsp_reorder_static_first", "clsp_recover_previous", "clsp_merge_updates",
    "clsp_l1_dssim_loss_grad",
)


class Camera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("width", c_int32), ("height", c_int32)]


class Gaussians(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logit", c_void_p),
                ("sh", c_void_p), ("gather", c_void_p), ("n", c_int64), ("n_rows", c_int64), ("sh_degree", c_int32),
                ("reserved", c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("log_scales", c_void_p), ("quats", c_void_p), ("opacity_logit", c_void_p),
                ("sh", c_void_p), ("n", c_int64), ("sh_degree", c_int32), ("reserved", c_int32)]


class Range(ctypes.Structure):
    _fields_ = [("begin", c_int64), ("end", c_int64)]


class Projected(ctypes.Structure):
    _fields_ = [("splat", c_void_p), ("depth", c_void_p), ("rect", c_void_p), ("flags", c_void_p)]


class Bins(ctypes.Structure):
    _fields_ = [("values", c_void_p), ("keys", c_void_p), ("ranges", c_void_p), ("ranges2", c_void_p),
                ("tile_mask", c_void_p), ("alive_mask", c_void_p), ("tile_list", c_void_p), ("counters", c_void_p),
                ("ws", c_void_p), ("ws_bytes", c_size_t), ("capacity", c_int64), ("n", c_int64), ("mode", c_int32),
                ("reserved", c_int32)]


class AdamHParams(ctypes.Structure):
    _fields_ = [("lr", c_float * 6), ("beta1", c_float), ("beta2", c_float), ("eps", c_float), ("step", c_int32),
                ("step_device", c_void_p), ("zero_grads", c_int32), ("reserved", c_int32),
                ("skip_flag", c_void_p)]


_lib = None


class LibraryMissing(RuntimeError):
    pass


def load(path: Path | None = None):
    """Load libclsplat.so (built by ``paper_2506_21117_amd.build``).  Raises
    ``LibraryMissing`` when it is not built: there is no fallback path."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise LibraryMissing(f"{p} is not built; run `python -m paper_2506_21117_amd.build` "
                             "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(str(p))
    st = c_int32
    L.clsp_version.restype = c_char_p
    L.clsp_version.argtypes = []
    L.clsp_last_error.restype = c_char_p
    L.clsp_last_error.argtypes = []
    L.clsp_project_preprocess.restype = st
    L.clsp_project_preprocess.argtypes = [POINTER(Gaussians), POINTER(Camera), c_int32, POINTER(Projected), c_void_p]
    L.clsp_project_preprocess_rows.restype = st
    L.clsp_project_preprocess_rows.argtypes = [POINTER(Gaussians), POINTER(Camera), c_int32, Range, POINTER(Projected),
                                               c_void_p]
    L.clsp_bin_and_sort_workspace_bytes.restype = c_size_t
    L.clsp_bin_and_sort_workspace_bytes.argtypes = [c_int64, c_int32, c_int32, c_int32, c_int64]
    L.clsp_bin_and_sort.restype = st
    L.clsp_bin_and_sort.argtypes = [POINTER(Projected), POINTER(Camera), c_int32, Range, c_int32, POINTER(Bins),
                                    c_void_p]
    L.clsp_frozen_order_bytes.restype = c_size_t
    L.clsp_frozen_order_bytes.argtypes = [c_int64, c_int32, c_int64]
    L.clsp_frozen_order.restype = st
    L.clsp_frozen_order.argtypes = [POINTER(Projected), POINTER(Camera), c_int32, c_int64, c_int64, c_void_p, c_size_t,
                                    c_void_p, c_size_t, c_void_p]
    L.clsp_bin_and_sort_frozen.restype = st
    L.clsp_bin_and_sort_frozen.argtypes = [POINTER(Projected), POINTER(Camera), c_int32, c_int64, c_void_p, c_size_t,
                                           POINTER(Bins), c_void_p]
    L.clsp_render_state_bytes.restype = c_size_t
    L.clsp_render_state_bytes.argtypes = [c_int32, c_int32, c_int32]
    L.clsp_render_forward.restype = st
    L.clsp_render_forward.argtypes = [POINTER(Projected), POINTER(Bins), POINTER(Camera), c_int32, POINTER(c_float),
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.clsp_render_forward_l1.restype = st
    L.clsp_render_forward_l1.argtypes = [POINTER(Projected), POINTER(Bins), POINTER(Camera), c_int32, POINTER(c_float),
                                         c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p, c_void_p,
                                         c_void_p]
    L.clsp_l1_loss_grad.restype = st
    L.clsp_l1_loss_grad.argtypes = [c_void_p, c_void_p, POINTER(Bins), POINTER(Camera), c_int32, c_void_p, c_void_p,
                                    c_void_p]
    L.clsp_render_backward_workspace_bytes.restype = c_size_t
    L.clsp_render_backward_workspace_bytes.argtypes = [c_int64, c_int32]
    L.clsp_render_backward.restype = st
    L.clsp_render_backward.argtypes = [POINTER(Gaussians), POINTER(Projected), POINTER(Bins), POINTER(Camera), c_int32,
                                       POINTER(c_float), Range, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p,
                                       POINTER(Params), c_void_p, c_size_t, c_void_p]
    L.clsp_render_backward_noalloc.restype = st
    L.clsp_render_backward_noalloc.argtypes = [POINTER(Gaussians), POINTER(Projected), POINTER(Bins), POINTER(Camera),
                                               c_int32, POINTER(c_float), Range, c_void_p, c_void_p, c_void_p,
                                               c_size_t, c_void_p, POINTER(Params), c_void_p]
    L.clsp_masked_adam_step.restype = st
    L.clsp_masked_adam_step.argtypes = [POINTER(Params), POINTER(Params), POINTER(Params), POINTER(Params), Range,
                                        c_void_p, POINTER(AdamHParams), c_void_p]
    L.clsp_zero_grads.restype = st
    L.clsp_zero_grads.argtypes = [POINTER(Params), Range, c_void_p]
    L.clsp_render_backward_adam.restype = st
    L.clsp_render_backward_adam.argtypes = [POINTER(Gaussians), POINTER(Projected), POINTER(Bins), POINTER(Camera),
                                            c_int32, POINTER(c_float), Range, c_void_p, c_void_p, c_void_p, c_size_t,
                                            c_void_p, POINTER(Params), POINTER(Params), POINTER(Params),
                                            POINTER(AdamHParams), c_void_p, c_size_t, c_void_p]
    L.clsp_fit_spheres.restype = st
    L.clsp_fit_spheres.argtypes = [c_void_p, c_int64, Range, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]
    L.clsp_sphere_keep.restype = st
    L.clsp_sphere_keep.argtypes = [c_void_p, c_int64, Range, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                   c_void_p]
    L.clsp_compact_rows_workspace_bytes.restype = c_size_t
    L.clsp_compact_rows_workspace_bytes.argtypes = [c_int64]
    L.clsp_compact_rows.restype = st
    L.clsp_compact_rows.argtypes = [POINTER(Params), POINTER(Params), POINTER(Params), Range, c_void_p, POINTER(Params),
                                    POINTER(Params), POINTER(Params), c_void_p, c_size_t, c_void_p]
    L.clsp_dilate_masks_workspace_bytes.restype = c_size_t
    L.clsp_dilate_masks_workspace_bytes.argtypes = [c_int32, c_int32, c_int32]
    L.clsp_dilate_masks.restype = st
    L.clsp_dilate_masks.argtypes = [c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p, c_size_t,
                                    c_void_p]
    L.clsp_majority_vote.restype = st
    L.clsp_majority_vote.argtypes = [c_void_p, c_int64, c_int64, POINTER(Camera), c_int32, c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p]
    L.clsp_history_workspace_bytes.restype = c_size_t
    L.clsp_history_workspace_bytes.argtypes = []
    L.clsp_reorder_static_first.restype = st
    L.clsp_reorder_static_first.argtypes = [POINTER(Params), c_void_p, POINTER(Params), c_void_p, c_void_p, c_size_t,
                                            c_void_p]
    L.clsp_recover_previous.restype = st
    L.clsp_recover_previous.argtypes = [POINTER(Params), c_void_p, POINTER(Params), POINTER(Params), c_void_p,
                                        c_size_t, c_void_p]
    L.clsp_merge_updates.restype = st
    L.clsp_merge_updates.argtypes = [POINTER(Params), c_void_p, c_void_p, POINTER(Params), POINTER(Params),
                                     POINTER(Params), c_void_p, c_size_t, c_void_p]
    L.clsp_l1_dssim_loss_grad.restype = st
    L.clsp_l1_dssim_loss_grad.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(Bins), POINTER(Camera), c_int32,
                                          c_float, c_void_p, c_void_p, c_void_p]
    if path is None:
        _lib = L
    return L


class ClspError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"clsplat status {status}: {message}")
        self.status = status


def check(status: int):
    if status != CLSP_OK:
        raise ClspError(status, load().clsp_last_error().decode(errors="replace"))
