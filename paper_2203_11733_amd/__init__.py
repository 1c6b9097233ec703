"""MI355X (gfx950) Galerkin boundary element capacitance extractor (arXiv 2203.11733).

The numerical path lives in libgbem.so (C ABI in include/gbem.h, HIP kernels in
csrc/); ``binding`` is its ctypes wrapper.
"""
from . import binding  # noqa: F401
from .binding import Context, GbemError, make_opts, mesh_boxes, mesh_layout  # noqa: F401

__all__ = ["binding", "Context", "GbemError", "make_opts", "mesh_boxes", "mesh_layout"]
