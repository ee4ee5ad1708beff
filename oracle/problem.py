"""Whole-problem driver of the oracle (test infrastructure only).

Builds, for a workload description, the fine system (immersed formulation
section), the Galerkin hierarchy (coarsening subsection), the factored
additive Schwarz smoothers on every level above the coarsest (smoothers
subsection) and the V-cycle preconditioner (Algorithm alg:MGV).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import assemble as AS
from . import geometry as G
from . import hierarchy as H
from . import multigrid as MG
from . import schwarz as SW


@dataclass
class OracleProblem:
    w: object
    leaf: np.ndarray
    system: AS.System
    hier: H.Hierarchy
    smoothers: list
    vcycle: MG.VCycle

    @property
    def A(self):
        return self.system.A

    @property
    def b(self):
        return self.system.b

    def solve(self, b=None, tol=1e-8, max_iter=1000, flexible=False):
        b = self.b if b is None else b
        return MG.pcg(self.A, b, self.vcycle.apply, tol=tol, max_iter=max_iter, flexible=flexible)


def make_smoother(w, A, lev, fine):
    """The smoother of one level: w.smoother ("as" additive / "ms"
    multiplicative Schwarz) on the finest level, and on the coarser levels
    too unless w.coarse_smoother asks for diagonal smoothing there (Remark
    rem:coarseGS): "jacobi" (additive, one block per function) or "gs"
    (multiplicative, one block per function)."""
    kind = w.smoother if (fine or w.coarse_smoother == "same") else w.coarse_smoother
    if kind == "as":
        return SW.Smoother(A, lev)
    if kind == "ms":
        return SW.MultiplicativeSmoother(A, lev)
    if kind == "jacobi":
        return SW.DiagonalSmoother(A, lev)
    if kind == "gs":
        return SW.MultiplicativeSmoother(A, lev, kind="diagonal")
    raise ValueError(kind)


def build(w, orders=None, smoothers=True) -> OracleProblem:
    leaf = G.leaf_values(w, w.n, w.depth)
    sysf = AS.assemble(w, leaf, w.n, w.depth, orders=orders)
    hier = H.Hierarchy(w, sysf, leaf)
    sm = [None] * w.levels
    vc = None
    if smoothers:
        for l in range(1, w.levels):
            sm[l] = make_smoother(w, hier.A[l], hier.levels[l], fine=(l == w.levels - 1))
        vc = MG.VCycle(hier.A, hier.R, sm, nu_pre=w.nu, nu_post=w.nu, cycle=w.cycle)
    return OracleProblem(w=w, leaf=leaf, system=sysf, hier=hier, smoothers=sm, vcycle=vc)
