"""Pins of multigrid as a standalone solver and of full multigrid
(oracle/multigrid.py: mg_solve, fmg).

* the paper prints the standalone two-level rate of the additive Schwarz
  cycle on its star domain (0.5-0.6): the solver's error contraction per
  cycle must approach it;
* the solver reaches the direct solution;
* full multigrid with one (multiplicative Schwarz) cycle per level reaches
  the discretization error: its H1 error against the manufactured solution
  is within 1.1x of the Galerkin solution's, where one cycle from zero is
  far worse.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assemble as AS
from oracle import multigrid as MG
from oracle import problem as P
from oracle import quadrature as Q

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("n", [16])
def test_standalone_rate_matches_paper(n):
    op = P.build(W.star(n=n, depth=3))
    A = op.A
    rng = np.random.default_rng(3)
    e0 = rng.standard_normal(A.shape[0])
    # b = 0: the iterate is the error, e_k = (I - B A)^k e_0
    b = np.zeros_like(e0)
    errs = []
    x = e0.copy()
    for _ in range(40):
        x = x + op.vcycle.apply(b - A @ x)
        errs.append(math.sqrt(x @ (A @ x)))
    rate = (errs[-1] / errs[-11]) ** 0.1
    lo, hi = GOLD["two_level_as_standalone_rate_range"]["value"]
    assert lo < rate < hi, rate
    # the solver reaches the direct solution
    bb = A @ rng.standard_normal(A.shape[0])
    xs, k, rel = MG.mg_solve(A, bb, op.vcycle.apply, tol=1e-10)
    xd = spla.spsolve(A.tocsc(), bb)
    e = xs - xd
    # energy norm (the condition number here is ~5e10, so entrywise agreement
    # is limited by the direct solve, not by the iteration)
    assert rel <= 1e-10 and math.sqrt(e @ (A @ e)) <= 1e-8 * math.sqrt(xd @ (A @ xd))


def _h1_error(op, x):
    """H1-seminorm error of coefficients x against the manufactured u*."""
    sysf = op.system
    lev = sysf.level
    w = op.w
    pos = {int(L): i for i, L in enumerate(lev.active)}
    h1 = 0.0
    for e in zip(*np.nonzero(lev.active_el)):
        fl = lev.elem_funcs[AS.element_lin(e, lev.n)]
        vp, vw, _, _, _ = Q.element_quadrature(op.leaf, e, w.depth, lev.lo, lev.h, w.degree + 4, 2 * w.degree + 4, 2)
        if not len(vw):
            continue
        _, Gr = AS.tensor_eval(lev, e, vp)
        cf = np.array([x[pos[L]] if L in pos else 0.0 for L in fl])
        _, _, g = AS.manufactured(vp)
        h1 += np.sum(vw * np.sum((np.einsum("a,aqc->qc", cf, Gr) - g) ** 2, axis=1))
    return math.sqrt(h1)


def test_full_multigrid_reaches_discretization_error():
    """With the paper's multiplicative Schwarz cycle (a contraction of about
    0.2 per cycle), one FMG pass lands within 1.1x of the Galerkin
    solution's H1 error (measured 1.02x), while one cycle from zero is 40x
    off: a wrong restriction of b, a missing prolongation or a skipped
    level's cycle each leave FMG far from the discretization error."""
    import dataclasses
    w = dataclasses.replace(W.small_discs(seed=4, n=32, degree=2, levels=4, n_discs=3, rhs="manufactured"),
                            smoother="ms")
    op = P.build(w)
    xh = spla.spsolve(op.A.tocsc(), op.b)
    e_h = _h1_error(op, xh)
    e_fmg = _h1_error(op, MG.fmg(op.vcycle, op.b))
    e_v = _h1_error(op, op.vcycle.apply(op.b))
    assert e_fmg <= 1.1 * e_h, (e_fmg, e_h)
    assert e_v >= 10.0 * e_h, (e_v, e_h)
