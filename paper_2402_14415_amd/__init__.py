"""MI355X (gfx950) TaylorGrid query path: HIP kernels behind a C ABI, with a thin binding.

    from paper_2402_14415_amd import TaylorGrid, sdf_loss, taylor_grid, Server

The native library (``libtaylorgrid.so``) is loaded on first use; the seeded input
generators in ``synth`` import nothing from it.
"""
from __future__ import annotations

__all__ = ["TaylorGrid", "sdf_loss", "query", "taylor_grid", "TaylorGridFn", "Server", "coeffs_per_vertex"]


def __getattr__(name):
    if name in ("TaylorGrid", "sdf_loss", "query", "coeffs_per_vertex"):
        from . import grid

        return getattr(grid, name)
    if name in ("taylor_grid", "TaylorGridFn"):
        from . import autograd

        return getattr(autograd, name)
    if name == "Server":
        from .serving import Server

        return Server
    raise AttributeError(name)
