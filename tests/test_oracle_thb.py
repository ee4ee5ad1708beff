"""Pins of the THB oracle (oracle/thb.py): truncated hierarchical B-splines
(Figure fig:THB), Algorithm alg:coarsen and the THB multigrid hierarchy.

Each pin is fixed by the mathematics, not by re-running the oracle's steps:
partition of unity, non-negativity and linear independence of the truncated
basis, equal span with the non-truncated hierarchical basis, the uniform
special cases, the characterization of the coarse mesh (one level of
refinement away from the fine mesh, and the coarsest such mesh), nestedness
of the coarse THB space (an exact R), Galerkin = direct coarse assembly, the
energy ordering of nested spaces, and equality with the pinned uniform
oracle when no cell is refined.
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import assemble as AS
from oracle import geometry as G
from oracle import hierarchy as H
from oracle import schwarz as SW
from oracle import thb as T


def random_mesh(seed, n0, M, frac=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    dom = [np.ones((n0, n0), dtype=bool)]
    for m in range(M):
        mark = dom[m] & (rng.random(dom[m].shape) < frac)
        dom.append(T.children(mark))
    return T.HMesh(n0, M, dom)


@pytest.fixture(scope="module")
def small():
    w = W.thb_discs(n=16, local_levels=2, levels=3)
    return T.build(w)


@pytest.mark.parametrize("seed,n0,M", [(0, 4, 1), (1, 4, 2), (2, 6, 2), (3, 3, 3)])
def test_truncated_basis_partition_nonneg_independent(seed, n0, M):
    mesh = random_mesh(seed, n0, M)
    p = 2
    funcs = T.thb_functions(mesh, p)
    C = T.coefficients(mesh, p, funcs, mesh.cells(M)).toarray()
    assert np.abs(C.sum(axis=0) - 1.0).max() < 1e-13      # sum of all functions = 1
    assert C.min() >= 0.0
    assert np.linalg.matrix_rank(C) == len(funcs)          # linearly independent
    Chb = T.coefficients(mesh, p, funcs, mesh.cells(M), truncate=False).toarray()
    assert np.linalg.matrix_rank(np.vstack([C, Chb])) == len(funcs)   # same span as the HB basis
    # truncation only removes parts: support of a THB function within its HB function's
    assert np.all((C > 0) <= (Chb > 0))
    # where truncation removed a (non-negative) part, the non-truncated
    # functions add up to more than one: the HB basis is no partition of unity
    if np.abs(C - Chb).max() > 0.0:
        assert Chb.sum(axis=0).max() > 1.0 + 1e-12
    if seed == 3:
        assert np.abs(C - Chb).max() > 0.0   # this mesh does truncate


def test_uniform_special_cases():
    p = 2
    # no refinement: the level-0 B-splines
    m0 = T.HMesh(5, 0, [np.ones((5, 5), dtype=bool)])
    f0 = T.thb_functions(m0, p)
    assert f0 == [(0, ix, iy) for iy in range(7) for ix in range(7)]
    C0 = T.coefficients(m0, p, f0, 5).toarray()
    assert np.array_equal(C0, np.eye(49))
    # everything refined once: exactly the level-1 B-splines, untruncated
    m1 = T.HMesh(4, 1, [np.ones((4, 4), dtype=bool), np.ones((8, 8), dtype=bool)])
    f1 = T.thb_functions(m1, p)
    assert f1 == [(1, ix, iy) for iy in range(10) for ix in range(10)]
    assert np.array_equal(T.coefficients(m1, p, f1, 8).toarray(), np.eye(100))


@pytest.mark.parametrize("seed,n0,M", [(4, 8, 1), (5, 8, 2), (6, 4, 3)])
def test_coarsen_is_the_coarsest_one_level_parent(seed, n0, M):
    fine = random_mesh(seed, n0, M, frac=0.25)
    coarse = T.coarsen(fine)
    assert coarse.n0 == n0 // 2 and coarse.M == M

    def one_level_away(cm):
        # every fine element is a coarse element or a child of one (same
        # absolute width: coarse level m+1 = fine level m)
        ok = True
        for m in range(fine.M + 1):
            fa = fine.active_cells(m)
            same = cm.active_cells(m + 1) if m + 1 <= cm.M else np.zeros_like(fa)
            par = T.children(cm.active_cells(m)) if m <= cm.M else np.zeros_like(fa)
            ok &= bool(np.all(fa <= (same | par)))
        return ok

    assert one_level_away(coarse)
    # coarsest: undoing any refinement of a coarse cell breaks the property
    for m in range(coarse.M):
        ref = coarse.refined(m)
        for ex, ey in zip(*np.nonzero(ref)):
            dom = [d.copy() for d in coarse.dom]
            # remove the cell's descendants at every finer level
            for k in range(m + 1, coarse.M + 1):
                s = 2 ** (k - m)
                dom[k][ex * s:(ex + 1) * s, ey * s:(ey + 1) * s] = False
            assert not one_level_away(T.HMesh(coarse.n0, coarse.M, dom))
    # nested regions: coarse Omega^{m+1} (width of fine level m) within fine Omega^m
    for m in range(M):
        assert np.all(coarse.dom[m + 1] <= fine.dom[m])
    # a uniform fine mesh coarsens to a uniform mesh
    uni = T.HMesh(n0, M, [np.ones((n0, n0), dtype=bool)] + [np.zeros((n0 * 2 ** k,) * 2, dtype=bool)
                                                          for k in range(1, M + 1)])
    cu = T.coarsen(uni)
    assert all(not d.any() for d in cu.dom[1:])


def test_coarse_space_nested_and_galerkin(small):
    h = small.hier
    for k in range(len(h.R)):
        lc, lf = h.levels[k], h.levels[k + 1]
        Cf, Cc = lf.C_all.toarray(), lc.C_all.toarray()
        # exact representation of every coarse function in the fine THB basis
        X = np.linalg.lstsq(Cf.T, Cc.T, rcond=None)[0].T
        assert np.abs(X @ Cf - Cc).max() < 1e-12
        # the restricted R of the oracle equals the active block of X
        Xa = X[np.ix_(np.nonzero(lc.act)[0], np.nonzero(lf.act)[0])]
        assert np.abs(h.R[k].toarray() - Xa).max() < 1e-11
        # partition of unity is kept: every fine column of X sums to one
        assert np.abs(X.sum(axis=0) - 1.0).max() < 1e-12
        # Galerkin product = the coarse THB space assembled directly on the grid
        D = h.A_direct[k]
        assert abs(h.A[k] - D).max() <= 1e-12 * abs(D).max()


def test_energy_ordering_of_nested_spaces(small):
    """Base uniform space within the THB space within the grid space: the
    discrete energy min_u 1/2 a(u,u) - b(u) = -1/2 b^T A^-1 b decreases."""
    h = small.hier
    w = small.w
    grid = h.grid
    nf1 = h.n_grid + w.degree
    Ag = T.embed(grid.level, grid.A, nf1)
    bg = np.zeros(nf1 * nf1)
    bg[grid.level.active] = grid.b

    def energy(C):
        A = (C @ Ag @ C.T).toarray()
        b = C @ bg
        keep = np.diag(A) > 0
        return -0.5 * b[keep] @ np.linalg.solve(A[np.ix_(keep, keep)], b[keep])

    J_thb = -0.5 * h.b @ np.linalg.solve(h.A[-1].toarray(), h.b)
    base = T.HMesh(w.n, 0, [np.ones((w.n, w.n), dtype=bool)])
    C0 = T.coefficients(base, w.degree, T.thb_functions(base, w.degree), h.n_grid)
    C0 = C0[np.nonzero(T.build_level(base, w.degree, h.n_grid, grid.level).act)[0]]
    J_base = energy(C0)
    J_grid = -0.5 * grid.b @ np.linalg.solve(grid.A.toarray(), grid.b)
    assert J_grid < J_thb < J_base


def test_without_refinement_equals_uniform_oracle():
    w = dataclasses.replace(W.thb_discs(n=16, local_levels=0, levels=3), name="thb-uniform")
    th = T.THBHierarchy(w)
    leaf = G.leaf_values(w, w.n, w.depth)
    sysf = AS.assemble(w, leaf, w.n, w.depth)
    hu = H.Hierarchy(w, sysf, leaf)
    for l in range(w.levels):
        assert th.A[l].shape == hu.A[l].shape
        assert abs(th.A[l] - hu.A[l]).max() <= 1e-13 * abs(hu.A[l]).max()
    for k in range(w.levels - 1):
        assert abs(th.R[k] - hu.R[k]).max() < 1e-13
    bu = SW.select_blocks(hu.levels[-1])[0]
    bt = SW.select_blocks(th.levels[-1])[0]
    assert len(bu) == len(bt) and all(np.array_equal(a, b) for a, b in zip(bu, bt))


def test_thb_pcg_converges(small):
    x, it, _ = small.solve()
    rel = np.linalg.norm(small.b - small.A @ x) / np.linalg.norm(small.b)
    assert rel <= 1e-8 and it < 60
    # blocks: every block holds its own function, and functions with their
    # whole support inside Omega on level-M cells form singleton blocks
    sm = small.smoothers[-1]
    assert all(j in set(b.tolist()) for j, b in zip(sm.assoc, sm.raw_blocks))


def test_thb_multiplicative_colours_and_symmetry():
    """Multiplicative Schwarz on THB levels (greedy colours, R-reading in the
    smoother's docstring): no two blocks of one colour share an element; on
    an unrefined mesh the greedy colouring of the (singleton) uncut blocks
    needs exactly (p+1)^d = 9 colours; the V-cycle with the forward sweep
    before and the reversed sweep after the coarse correction is symmetric
    (u.Bv = v.Bu); PCG converges in fewer iterations than with the additive
    smoother."""
    w = dataclasses.replace(W.thb_discs(n=16, local_levels=2, levels=3), smoother="ms")
    ob = T.build(w)
    for l in range(1, w.levels):
        sm = ob.smoothers[l]
        lev = ob.hier.levels[l]
        els = SW.block_elements(lev, sm.blocks)
        for c in set(sm.colours):
            seen = set()
            for j, cj in enumerate(sm.colours):
                if cj == c:
                    assert not (els[j] & seen)
                    seen |= els[j]
    rng = np.random.default_rng(5)
    n = ob.A.shape[0]
    for _ in range(3):
        u, v = rng.standard_normal(n), rng.standard_normal(n)
        a, b = u @ ob.vcycle.apply(v), v @ ob.vcycle.apply(u)
        assert abs(a - b) <= 1e-10 * max(abs(a), 1e-300)
    x, it, _ = ob.solve()
    assert np.linalg.norm(ob.b - ob.A @ x) / np.linalg.norm(ob.b) <= 1e-8
    wa = W.thb_discs(n=16, local_levels=2, levels=3)
    _, it_as, _ = T.build(wa).solve()
    assert it < it_as
    # an unrefined mesh away from the discs: 9 greedy colours for the interior blocks
    wu = dataclasses.replace(W.thb_discs(n=16, local_levels=0, levels=2), smoother="ms", discs=[[0.5, 0.5, 0.05]])
    ou = T.build(wu)
    smu = ou.smoothers[-1]
    single = [j for j, b in enumerate(smu.blocks) if len(b) == 1]
    assert len({smu.colours[j] for j in single}) == 9


# ---------------------------------------------------------------- elasticity
# Pins of the vector THB levels (2D linear elasticity on the star domain).

def test_elasticity_without_refinement_equals_uniform_vector_assembly():
    """No local refinement: the THB functions are the level-0 B-splines, so
    the finest vector operator, load and mass equal the uniform vector
    assembly of oracle/elasticity.py (a separate code path: lattice
    elements instead of grid coefficients; the star leaves the box-face
    functions inactive, so both keep the same functions)."""
    from oracle import elasticity as EL
    w = W.thb_star_elasticity(n=16, local_levels=0, levels=2)
    th = T.THBHierarchy(w)
    leaf = G.leaf_values(w, w.n, w.depth)
    vs = EL.assemble_elasticity(w, leaf, w.n, w.depth)
    assert th.ncomp == 2 and th.A[-1].shape == vs.A.shape
    assert abs(th.A[-1] - vs.A).max() <= 1e-12 * abs(vs.A).max()
    assert np.abs(th.b - vs.b).max() <= 1e-13 * np.abs(vs.b).max()
    assert abs(th.M - vs.M).max() <= 1e-13 * abs(vs.M).max()


def _greville(m, k, n0, p, lo, hi):
    """Greville abscissa of B-spline k of level m (open uniform knots)."""
    n = n0 * 2 ** m
    h = (hi - lo) / n
    t = np.concatenate([np.full(p, lo), lo + h * np.arange(n + 1), np.full(p, hi)])
    return float(np.mean(t[k + 1:k + p + 1]))


@pytest.mark.parametrize("M", [1, 2])
def test_elasticity_rigid_motions_in_the_kernel(M):
    """Without the penalty term (beta = 0) the elasticity operator of the
    refined THB space annihilates the rigid motions: the THB basis keeps the
    partition of unity and reproduces linear functions with the Greville
    abscissae of each function's own level as coefficients, so the
    translations and the rotation (-y, x) are exactly representable and have
    zero strain.  A wrong component block, a transposed coupling or a
    truncation error leaves a residual."""
    w = dataclasses.replace(W.thb_star_elasticity(n=16, local_levels=M, levels=2), penalty_factor=0.0)
    th = T.THBHierarchy(w)
    lev = th.levels[-1]
    funcs = [f for f, a in zip(lev.funcs, lev.act) if a]
    N = len(funcs)
    gx = np.array([_greville(m, ix, w.n, w.degree, w.box_lo, w.box_hi) for (m, ix, iy) in funcs])
    gy = np.array([_greville(m, iy, w.n, w.degree, w.box_lo, w.box_hi) for (m, ix, iy) in funcs])
    A = th.A[-1]
    scale = abs(A).max()
    modes = {"x": np.concatenate([np.ones(N), np.zeros(N)]), "y": np.concatenate([np.zeros(N), np.ones(N)]),
             "rotation": np.concatenate([-gy, gx])}
    for name, u in modes.items():
        assert np.abs(A @ u).max() <= 1e-10 * scale * np.abs(u).max(), name
    # and a strain-carrying linear field is not in the kernel
    ux = np.concatenate([gx, np.zeros(N)])
    assert np.abs(A @ ux).max() > 1e-3 * scale


def test_elasticity_multiplicative_colours_and_symmetry():
    """Vector THB levels with multiplicative Schwarz: blocks of one colour
    are uncoupled (A has no entry between any two of them, so their updates
    commute), the V-cycle is symmetric, and PCG converges in fewer
    iterations than with the additive smoother; gamma of the additive
    smoother counts the blocks of both components (twice the scalar N_K of
    the same level)."""
    from oracle import elasticity as EL
    w = dataclasses.replace(W.thb_star_elasticity(n=16, local_levels=2, levels=4), smoother="ms")
    ob = T.build(w)
    for l in range(1, w.levels):
        sm = ob.smoothers[l]
        A = ob.hier.A[l].tocsr()
        by_colour = {}
        for j, c in enumerate(sm.colours):
            by_colour.setdefault(c, []).append(np.asarray(sm.blocks[j]))
        for blocks in by_colour.values():
            owner = np.full(A.shape[0], -1)
            for j, b in enumerate(blocks):
                owner[b] = j
            for j, b in enumerate(blocks):
                cols = A[b].indices
                other = owner[cols]
                assert np.all((other == -1) | (other == j)), (l, j)
    # symmetry to 1e-6: the vector blocks of cut elements reach kappa ~ 1e8,
    # so rounding leaves up to ~5e-9; a post-sweep in forward order instead of
    # reversed leaves 4e-3 .. 4e-2 on the same vectors
    rng = np.random.default_rng(6)
    n = ob.A.shape[0]
    for _ in range(3):
        u, v = rng.standard_normal(n), rng.standard_normal(n)
        a, b = u @ ob.vcycle.apply(v), v @ ob.vcycle.apply(u)
        assert abs(a - b) <= 1e-6 * max(abs(a), 1e-300)
    _, it_ms, _ = ob.solve()
    wa = dataclasses.replace(w, smoother="as")
    oa = T.build(wa)
    _, it_as, _ = oa.solve()
    assert it_ms < it_as
    for l in range(1, w.levels):
        lev = ob.hier.levels[l]
        scalar = SW.max_NK(lev, SW.select_blocks(lev)[0])
        vec = EL.max_NK_vector(lev, EL.vector_blocks(lev, 2)[0], 2)
        assert vec == 2 * scalar
