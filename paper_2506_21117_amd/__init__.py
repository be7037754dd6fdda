"""MI355X (gfx950) hot path of CL-Splats' local optimisation: a differentiable
tile-based Gaussian-splatting rasteriser whose backward pass and Adam step touch only the
changed Gaussians and the tiles they cover.

The kernels live in ``libclsplat.so`` (C-ABI in ``include/clsplat.h``); ``api`` calls it
with torch tensors, ``optim`` runs local and full-scene steps, ``autograd`` wraps the
renderer as a ``torch.autograd.Function`` and ``serve`` renders stored scene states for
a stream of requests.
"""
from ._ffi import LibraryMissing, load  # noqa: F401

__all__ = ["load", "LibraryMissing"]
