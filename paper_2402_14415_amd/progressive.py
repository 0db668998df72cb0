"""Progressive (coarse-to-fine) SDF fitting, the training schedule of Sec. 4.1: the grid is
fitted at a coarse resolution first, then each finer level starts from the field the previous
level represents (``tg_upsample``: value, gradient and Hessian of the coarse field at the fine
vertices) and is fitted further.

Argument marshalling only: every step is ``tg_train_step`` and every transfer ``tg_upsample``.
"""
from __future__ import annotations

from .grid import TaylorGrid


class ProgressiveFit:
    """One TaylorGrid per resolution level over the same box; ``advance`` moves to the next
    level.  The objective's weights (``eik_weight``, ``surface_k``, ``tv_weight``) and Adam's
    learning rate are passed to every step."""

    def __init__(self, dim, levels, order, lo, hi, device="cuda", storage="f32", coeffs=None,
                 eik_weight=0.1, surface_k=0.0, tv_weight=0.0, lr=1e-2):
        if not levels:
            raise ValueError("at least one resolution level is needed")
        self.levels = [tuple(r) if hasattr(r, "__len__") else (int(r),) * dim for r in levels]
        self.dim, self.order, self.lo, self.hi = dim, order, lo, hi
        self.device, self.storage = device, storage
        self.objective = dict(eik_weight=eik_weight, surface_k=surface_k, tv_weight=tv_weight)
        self.lr = lr
        self.level = 0
        self.grid = TaylorGrid(dim, self.levels[0], order, lo, hi, storage=storage, coeffs=coeffs, device=device)
        self._ws = {}

    def workspace(self, n):
        """The current level's workspace for n queries (kept per level and size)."""
        key = (self.level, n)
        if key not in self._ws:
            self._ws = {k: v for k, v in self._ws.items() if k[0] == self.level}
            self._ws[key] = self.grid.workspace(n)
        return self._ws[key]

    def step(self, q, d, **kw):
        """One fitting step of the current level; returns the loss (device float64)."""
        args = dict(self.objective, lr=self.lr)
        args.update(kw)
        return self.grid.train_step(q, d, self.workspace(q.shape[0]), **args)

    def advance(self):
        """Move to the next level: a new grid starts from the current field; the Adam moments
        start at zero."""
        if self.level + 1 >= len(self.levels):
            raise IndexError("already at the finest level")
        fine = TaylorGrid(self.dim, self.levels[self.level + 1], self.order, self.lo, self.hi, storage=self.storage,
                          device=self.device)
        fine.upsample_from(self.grid)
        self.grid = fine
        self.level += 1
        return fine
