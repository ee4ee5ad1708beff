"""Pins of the oracle's assembly, hierarchy, Schwarz smoother, V-cycle and CG.

Each test checks a property fixed by the paper or by the mathematics, through
a route that does not retype the oracle's own formula.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assemble as AS
from oracle import basis as B
from oracle import geometry as G
from oracle import hierarchy as H
from oracle import multigrid as MG
from oracle import problem as P
from oracle import quadrature as Q
from oracle import schwarz as SW

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _w(**kw):
    base = dict(name="t", dim=2, degree=2, n=8, depth=1, levels=2, geometry="discs",
                discs=[[0.47, 0.52, 0.26]], rhs="one")
    base.update(kw)
    return W.Workload(**base)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_stiffness_symmetric_psd_and_constant_kernel(p):
    # pure Neumann problem: constants are in the kernel (partition of unity)
    w = _w(degree=p, bc="neumann")
    leaf = G.leaf_values(w, w.n, w.depth)
    s = AS.assemble(w, leaf, w.n, w.depth)
    A = s.A.toarray()
    assert np.array_equal(A, A.T)
    assert np.abs(A @ np.ones(len(A))).max() < 1e-12 * np.abs(A).max()
    lam = np.linalg.eigvalsh(A)
    assert lam[0] > -1e-12 * lam[-1]
    # mass matrix sums to the measure of Omega_h
    assert s.M.sum() == pytest.approx(s.omega_measure, rel=1e-12)


@pytest.mark.parametrize("p", [2, 3])
def test_dirichlet_system_is_spd(p):
    w = _w(degree=p, discs=[[0.5, 0.5, 0.2]])
    leaf = G.leaf_values(w, w.n, w.depth)
    A = AS.assemble(w, leaf, w.n, w.depth).A.toarray()
    lam = np.linalg.eigvalsh(A)
    assert lam[0] > 0


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 2)])
def test_divergence_theorem_volume_vs_boundary(dim, p):
    """For u = x y (exactly reproduced: coefficients xi_i xi_j, Greville
    abscissae) -lap u = 0, so (A u)_i = int_{dOmega_h} phi_i grad u . n; for
    functions whose support avoids the box this is the immersed-boundary
    integral.  Volume quadrature is checked against boundary quadrature."""
    if dim == 2:
        w = _w(degree=p, bc="neumann", n=8, depth=1)
    else:
        w = W.Workload(name="t3", dim=3, degree=p, n=4, depth=0, levels=1, geometry="gyroid",
                       phase=[0.3, 1.1, 2.0], bc="neumann", rhs="zero")
    leaf = G.leaf_values(w, w.n, w.depth)
    s = AS.assemble(w, leaf, w.n, w.depth, with_rhs=False)
    lev = s.level
    gr = H.greville(w.n, p, 0.0, 1.0)
    m = [np.array([lev.lat_to_multi(int(L))[a] for L in lev.active]) for a in range(dim)]
    u = gr[m[0]] * gr[m[1]]

    def g(x, nrm):
        return x[:, 1] * nrm[:, 0] + x[:, 0] * nrm[:, 1]

    _, v = AS.load_vector(w, leaf, w.n, w.depth, g=g, strong_box=False)
    Au = s.A @ u
    interior = np.all([(mi >= p) & (mi <= w.n - 1) for mi in m], axis=0)
    # interior: support inside the open box (B-spline i spans elements i-p..i)
    assert interior.sum() > 5
    assert np.allclose(Au[interior], v[interior], atol=1e-12, rtol=1e-10)


def test_two_scale_relation_and_binomial_rows():
    rng = np.random.default_rng(3)
    for p in (1, 2, 3):
        nc = 6
        R = H.two_scale_1d("bspline", nc, p, 0.0, 1.0)
        x = rng.uniform(0, 1, 300)
        assert np.allclose(B.bspline_all(nc, p, x), R @ B.bspline_all(2 * nc, p, x), atol=1e-13)
        # interior coarse function p+1: coefficients 2^-p binom(p+1, k)
        i = p + 1
        row = R[i]
        nz = row[row != 0]
        expect = np.array([math.comb(p + 1, k) for k in range(p + 2)]) / 2 ** p
        assert np.allclose(nz, expect, atol=1e-15)
        # partition of unity: every column of R sums to one
        assert np.allclose(R.sum(axis=0), 1.0, atol=1e-14)
    # Lagrange: coarse functions sampled at fine nodes
    R = H.two_scale_1d("lagrange", 4, 2, 0.0, 1.0)
    x = rng.uniform(0, 1, 200)
    assert np.allclose(B.lagrange_all(4, 2, x), R @ B.lagrange_all(8, 2, x), atol=1e-13)


@pytest.mark.parametrize("p", [2, 3])
def test_galerkin_equals_direct_coarse_assembly(p):
    """Remark rem:gridParamCorr: R A R^T must equal the coarse stiffness
    assembled directly on the coarse grid with one more bisection level (same
    integrated geometry, rules exact for the stiffness integrand)."""
    w = _w(degree=p, n=8, depth=1, levels=2)
    leaf = G.leaf_values(w, w.n, w.depth)
    fine = AS.assemble(w, leaf, w.n, w.depth, with_rhs=False)
    hier = H.Hierarchy(w, fine, leaf)
    direct = AS.assemble(w, leaf, w.n // 2, w.depth + 1, with_rhs=False)
    assert np.array_equal(direct.level.active, hier.levels[0].active)
    D = direct.A.toarray()
    Gm = hier.A[0].toarray()
    assert np.abs(D - Gm).max() < 1e-12 * np.abs(D).max()
    # same structural pattern
    assert np.array_equal(direct.A.indptr, hier.A[0].indptr)
    assert np.array_equal(direct.A.indices, hier.A[0].indices)


def test_blocks_uncut_bspline_are_singletons_and_gamma():
    for p, d in ((2, 2), (3, 2)):
        w = W.Workload(name="u", dim=d, degree=p, n=8, depth=0, levels=2, geometry="none")
        op = P.build(w)
        sm = op.smoothers[-1]
        lev = op.hier.levels[-1]
        # functions p+1..n-2 per axis have full supports that contain no
        # other support (the open-knot boundary functions have shorter ones)
        for blk, j in zip(sm.blocks, sm.assoc):
            m = lev.lat_to_multi(int(lev.active[j]))
            if all(p + 1 <= mi <= w.n - 2 for mi in m):
                assert list(blk) == [j]
        assert sm.gamma == pytest.approx((p + 1) ** (-d))


def test_blocks_uncut_lagrange_size_and_gamma():
    p, d = 2, 2
    w = W.Workload(name="u", dim=d, degree=p, n=6, depth=0, levels=2, geometry="none",
                   basis="lagrange", bc="box_dirichlet")
    leaf = G.leaf_values(w, w.n, w.depth)
    lev = AS.make_level(w, leaf, w.n, w.depth, True)
    blocks, assoc = SW.select_blocks(lev)
    # vertex patches away from the box: (2p-1)^d functions
    sizes = []
    for blk, j in zip(blocks, assoc):
        m = lev.lat_to_multi(int(lev.active[j]))
        if all(2 * p <= mi <= p * w.n - 2 * p for mi in m):
            sizes.append(len(blk))
    assert sizes and set(sizes) == {(2 * p - 1) ** d}
    assert 1.0 / SW.max_NK(lev, blocks) == pytest.approx(GOLD["as_relaxation_2d_lagrange"]["value"])


def test_blocks_match_pointwise_support_containment():
    """Brute force on sample points: phi_k is in block j iff phi_k vanishes at
    every sample point of Omega_h where phi_j vanishes."""
    w = _w(degree=2, n=6, depth=2, discs=[[0.5, 0.45, 0.3]])
    leaf = G.leaf_values(w, w.n, w.depth)
    s = AS.assemble(w, leaf, w.n, w.depth, with_rhs=False)
    lev = s.level
    blocks, assoc = SW.select_blocks(lev)
    from oracle import quadrature as Q
    pts = []
    for e in zip(*np.nonzero(lev.active_el)):
        vp, vw, *_ = Q.element_quadrature(leaf, e, w.depth, 0.0, lev.h, 3, 3, 3)
        pts.append(vp[vw > 0])
    X = np.concatenate(pts)
    V1 = [B.bspline_all(w.n, 2, X[:, a]) for a in range(2)]
    vals = np.zeros((len(lev.active), len(X)))
    for i, L in enumerate(lev.active):
        mx, my = lev.lat_to_multi(int(L))
        vals[i] = V1[0][mx] * V1[1][my]
    nz = np.abs(vals) > 1e-13
    for blk, j in zip(blocks, assoc):
        brute = [k for k in range(len(lev.active)) if not np.any(nz[k] & ~nz[j])]
        assert list(blk) == brute


def test_removal_rule_on_exact_null_vector():
    import scipy.sparse as sp
    A = sp.csr_matrix(np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 2.0]]))
    keep, inv, lam, removed = SW.factor_block(A, np.array([0, 1, 2]))
    # null vector (1, -1, 0)/sqrt2: tie between local 0 and 1 -> lowest removed
    assert removed == [0]
    assert list(keep) == [1, 2]
    assert np.allclose(inv, np.diag([1.0, 0.5]))


def test_c1_smoother_bound_and_block_inverses():
    op = P.build(W.c1())
    for l in (1, 2):
        A = op.hier.A[l].toarray()
        sm = op.smoothers[l]
        assert sm.gamma == pytest.approx(1 / 9)
        kmax = 1.0
        for k, inv in zip(sm.blocks, sm.inv):
            Aj = A[np.ix_(k, k)]
            lam = np.linalg.eigvalsh(Aj)
            kappa = lam[-1] / lam[0]
            kmax = max(kmax, kappa)
            assert np.abs(inv @ Aj - np.eye(len(k))).max() < 1e3 * kappa * 1e-16 + 1e-10
        # eq:applyCS: gamma * lambda_max(M^-1 A) <= 1 (eigenvalues of S A, S = gamma M^-1),
        # up to the rounding of the block inverses (relative error ~ kappa_j * eps)
        S = sm.dense()
        lam = np.linalg.eigvals(S @ A).real
        assert lam.max() <= 1.0 + 10 * kmax * 1.1e-16 + 1e-8
        assert lam.min() > -1e-8


def test_two_level_error_propagation_identity():
    """eq:eigenMulti: I - B A = (I - S A)(I - R^T A_c^{-1} R A)(I - S A) for the
    two-level V-cycle with a symmetric smoother S = gamma M^{-1}."""
    w = _w(degree=2, n=8, depth=2, levels=2, discs=[[0.45, 0.55, 0.23]])
    op = P.build(w)
    A = op.hier.A[1].toarray()
    Ac = op.hier.A[0].toarray()
    R = op.hier.R[0].toarray()
    S = op.smoothers[1].dense()
    I = np.eye(len(A))
    Bm = op.vcycle.dense()
    rhs = (I - S @ A) @ (I - R.T @ np.linalg.solve(Ac, R @ A)) @ (I - S @ A)
    assert np.abs((I - Bm @ A) - rhs).max() < 1e-8
    assert np.abs(Bm - Bm.T).max() < 1e-8 * np.abs(Bm).max()
    lam = np.sort(np.linalg.eigvals(Bm @ A).real)
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-8


@pytest.mark.parametrize("nu", [1, 2])
def test_multilevel_error_propagation_recursion(nu):
    """eq:eigenMulti applied level by level (Algorithm alg:MGV is recursive):
    with nu smoothing steps on either side, the error propagation of the
    l-level cycle is E_l = (I - S_l A_l)^nu (I - R_l^T B_{l-1} R_l A_l)
    (I - S_l A_l)^nu with B_{l-1} = (I - E_{l-1}) A_{l-1}^{-1} and
    B_0 = A_0^{-1}.  Built here from the level matrices, compared with the
    oracle's V-cycle probed by unit vectors on a three-level hierarchy.  A
    dropped or extra smoothing step, a wrong level index or a missing
    residual update breaks the equality."""
    w = _w(degree=2, n=16, depth=1, levels=3, nu=nu, discs=[[0.45, 0.55, 0.23]])
    op = P.build(w)
    A = [a.toarray() for a in op.hier.A]
    R = [r.toarray() for r in op.hier.R]
    B = np.linalg.inv(A[0])
    for l in (1, 2):
        I = np.eye(len(A[l]))
        Sm = np.linalg.matrix_power(I - op.smoothers[l].dense() @ A[l], nu)
        E = Sm @ (I - R[l - 1].T @ B @ R[l - 1] @ A[l]) @ Sm
        B = (I - E) @ np.linalg.inv(A[l])
        Bv = op.vcycle.dense(l)
        scale = np.abs(B).max()
        assert np.abs(Bv - B).max() < 1e-8 * scale, (l, np.abs(Bv - B).max() / scale)
    # the symmetric cycle is SPD-preconditioning: spectrum of B A in (0, 1]
    lam = np.sort(np.linalg.eigvals(Bv @ A[2]).real)
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-8


def _manufactured_errors(p, n, leaf_n, discs):
    """L2 and H1-seminorm errors of the Galerkin solution (direct solve) of the
    manufactured problem on the level with n elements, on the Omega_h of a
    fixed leaf lattice with leaf_n cells per axis."""
    depth = int(round(math.log2(leaf_n // n)))
    w = W.Workload(name="ph", dim=2, degree=p, n=n, depth=depth, levels=1, geometry="discs",
                   discs=discs, rhs="manufactured")
    leaf = G.leaf_values(w, n, depth)
    s = AS.assemble(w, leaf, n, depth)
    x = spla.spsolve(s.A.tocsc(), s.b)
    lev = s.level
    pos = {int(L): i for i, L in enumerate(lev.active)}
    l2 = h1 = 0.0
    for e in zip(*np.nonzero(lev.active_el)):
        fl = lev.elem_funcs[AS.element_lin(e, n)]
        # rules well above the integrands' polynomial degree
        vp, vw, _, _, _ = Q.element_quadrature(leaf, e, depth, lev.lo, lev.h, p + 4, 2 * p + 4, 2)
        if not len(vw):
            continue
        V, Gr = AS.tensor_eval(lev, e, vp)
        cf = np.array([x[pos[L]] if L in pos else 0.0 for L in fl])
        u, _, g = AS.manufactured(vp)
        l2 += np.sum(vw * (cf @ V - u) ** 2)
        h1 += np.sum(vw * np.sum((np.einsum("a,aqc->qc", cf, Gr) - g) ** 2, axis=1))
    return math.sqrt(l2), math.sqrt(h1)


@pytest.mark.parametrize("p", [2, 3])
def test_manufactured_solution_rates(p):
    """u* = sin(2 pi x) sin(2 pi y) solves -lap u = f with f = 8 pi^2 u*, u = 0
    on the box and the Neumann data grad u* . n_h on the immersed boundary of
    Omega_h, so on a fixed Omega_h (leaf lattice held at 1/256 while the grid
    is refined) the Galerkin error must fall at the optimal rates of degree-p
    B-splines: L2 ~ h^(p+1), H1 ~ h^p.  A sign or factor error in f, in g or
    in the boundary normal leaves the error at a plateau (slope ~0)."""
    discs = [[0.46, 0.53, 0.21], [0.17, 0.2, 0.08]]
    e = [_manufactured_errors(p, n, 256, discs) for n in (8, 16, 32)]
    for k in (1, 2):
        s_l2 = math.log2(e[k - 1][0] / e[k][0])
        s_h1 = math.log2(e[k - 1][1] / e[k][1])
        assert p + 1 - 0.2 < s_l2 < p + 1 + 0.4, (k, s_l2)
        assert p - 0.2 < s_h1 < p + 0.4, (k, s_h1)


@pytest.mark.parametrize("n", [16, 32])
def test_star_domain_spectra_match_paper(n):
    """Smoothers subsection (Additive Schwarz): star domain, quadratic
    Lagrange, penalty 2/h, gamma = 1/4.  Printed: AS double iteration has
    nodal modes near 7/16 and maximum about 1; the two-level V-cycle spectrum
    has 0.4 < lambda_min < 0.5 and lambda_max = 1; standalone rate 0.5-0.6."""
    op = P.build(W.star(n=n, depth=3))
    A = op.A.toarray()
    sm = op.smoothers[-1]
    assert sm.gamma == GOLD["as_relaxation_2d_lagrange"]["value"]
    I = np.eye(len(A))
    S = sm.dense()
    E = (I - S @ A) @ (I - S @ A)
    lam = np.sort(np.linalg.eigvals(I - E).real)
    assert lam[-1] == pytest.approx(GOLD["as_double_largest_eigenvalue"]["value"], abs=0.02)
    near = np.sum(np.abs(lam - GOLD["as_double_nodal_eigenvalue"]["value"]) < 0.03)
    assert near >= 5
    Bm = op.vcycle.dense()
    lv = np.sort(np.linalg.eigvals(Bm @ A).real)
    lo, hi = GOLD["two_level_as_lambda_min_range"]["value"]
    assert lo < lv[0] < hi
    assert lv[-1] == pytest.approx(GOLD["two_level_as_lambda_max"]["value"], abs=1e-3)
    rate = np.abs(np.linalg.eigvals(I - Bm @ A)).max()
    lo, hi = GOLD["two_level_as_standalone_rate_range"]["value"]
    assert lo < rate < hi


def test_pcg_matches_direct_solve_c1():
    op = P.build(W.c1())
    x, it, hist = op.solve(tol=1e-8)
    b = op.b
    assert np.linalg.norm(b - op.A @ x) / np.linalg.norm(b) <= 1e-8
    xd = spla.spsolve(op.A.tocsc(), b)
    M = op.system.M
    e = x - xd
    assert math.sqrt(e @ (M @ e)) / math.sqrt(xd @ (M @ xd)) < 1e-6
    assert it < 60


def test_pcg_from_a_far_start_meets_the_true_residual():
    """CG from an x0 whose residual is 1e3 times ||b||: the solve must end with
    the true relative residual ||b - A x|| / ||b|| <= tol (the criterion the
    solve reports) and equal the direct solve (P-j); with too few iterations
    it must say that it did not converge."""
    op = P.build(W.c1())
    b = op.b
    rng = np.random.Generator(np.random.PCG64(7))
    x0 = rng.standard_normal(len(b))
    x0 *= 1e3 * np.linalg.norm(b) / np.linalg.norm(b - op.A @ x0)
    info = {}
    x, it, _ = MG.pcg(op.A, b, op.vcycle.apply, tol=1e-8, x0=x0, info=info)
    assert info["converged"] and info["true_rel"] <= 1e-8
    assert np.linalg.norm(b - op.A @ x) / np.linalg.norm(b) == pytest.approx(info["true_rel"], rel=1e-12)
    xd = spla.spsolve(op.A.tocsc(), b)
    M = op.system.M
    e = x - xd
    assert math.sqrt(e @ (M @ e)) / math.sqrt(xd @ (M @ xd)) < 1e-6
    # the far start needs more iterations than x0 = 0 (the residual falls by 1e11)
    assert it > op.solve(tol=1e-8)[1]
    info2 = {}
    MG.pcg(op.A, b, op.vcycle.apply, tol=1e-8, x0=x0, max_iter=5, info=info2)
    assert not info2["converged"] and info2["true_rel"] > 1e-8


def test_flexible_pcg_equals_standard_for_the_fixed_vcycle():
    """The V-cycle is one fixed SPD operator (the paragraph after Algorithm
    alg:MGV), so r_{k+1}.z_k = 0 in exact arithmetic and the Polak-Ribiere
    beta equals the Hestenes-Stiefel one: same iterates up to rounding, same
    iteration count, and the cross term is rounding-small against r_k.z_k."""
    op = P.build(W.c1())
    xs, its, hs = op.solve(tol=1e-8)
    xf, itf, hf = op.solve(tol=1e-8, flexible=True)
    assert itf == its
    k = min(10, len(hs))
    assert np.allclose(hf[:k], hs[:k], rtol=1e-8, atol=0.0)
    M = op.system.M
    e = xf - xs
    assert math.sqrt(e @ (M @ e)) / math.sqrt(xs @ (M @ xs)) < 1e-9
    # the cross term along the standard iteration
    A, B = op.A, op.vcycle.apply
    r = op.b.copy()
    z = B(r)
    p = z.copy()
    for _ in range(5):
        q = A @ p
        a = (r @ z) / (p @ q)
        r_new = r - a * q
        z_new = B(r_new)
        assert abs(r_new @ z) <= 1e-8 * abs(r @ z)
        p = z_new + ((r_new @ z_new) / (r @ z)) * p
        r, z = r_new, z_new


@pytest.mark.slow
def test_iterations_mesh_independent():
    """Numerical examples: iteration counts virtually independent of the grid."""
    its = []
    for n in (16, 32, 64):
        w = W.Workload(name="mi", dim=2, degree=2, n=n, depth=int(math.log2(128 // n)),
                       levels=int(math.log2(n // 4)) + 1, geometry="discs",
                       discs=[[0.47, 0.52, 0.26], [0.15, 0.2, 0.07]], rhs="one")
        op = P.build(w)
        its.append(op.solve(tol=1e-8)[1])
    assert max(its) - min(its) <= max(3, 0.2 * min(its)), its


def test_apple_active_counts_match_paper():
    """Numerical examples, apple: 80^3 quadratic, depth 0 -> 667k B-spline and
    4.87M Lagrange DOFs (3 components each)."""
    gold = GOLD["apple_dofs_80"]
    w = W.Workload(name="apple", dim=3, degree=2, n=80, depth=0, levels=1, geometry="apple",
                   box_lo=-2.0, box_hi=2.0)
    leaf = G.leaf_values(w, 80, 0)
    act = G.active_elements(leaf, 80, 0)
    nb = 3 * AS.active_function_mask(act, "bspline", 2).sum()
    nl = 3 * AS.active_function_mask(act, "lagrange", 2).sum()
    assert abs(nb / gold["bspline"] - 1) < 0.002
    assert abs(nl / gold["lagrange"] - 1) < 0.002


def test_helix_active_counts_match_paper():
    """Numerical examples, triple helix: 128^3 quadratic, depth 0 -> 1.11M
    B-spline and 6.96M Lagrange DOFs (3 components each), printed to three
    significant figures: the counts must round to the printed values."""
    gold = GOLD["helix_dofs_128"]
    w = W.Workload(name="helix", dim=3, degree=2, n=128, depth=0, levels=1, geometry="helix",
                   box_lo=-2.0, box_hi=2.0)
    leaf = G.leaf_values(w, 128, 0)
    act = G.active_elements(leaf, 128, 0)
    nb = 3 * AS.active_function_mask(act, "bspline", 2).sum()
    nl = 3 * AS.active_function_mask(act, "lagrange", 2).sum()
    assert abs(nb - gold["bspline"]) <= 0.005e6
    assert abs(nl - gold["lagrange"]) <= 0.005e6


def test_vectorised_activation_matches_element_loop():
    w = _w(degree=3, n=8, depth=1)
    leaf = G.leaf_values(w, w.n, w.depth)
    lev = AS.make_level(w, leaf, w.n, w.depth, False)
    mask = AS.active_function_mask(lev.active_el, "bspline", 3)
    # mask is indexed [x, y]; lattice index is x fastest
    lat = np.array(sorted(int(i + lev.nf1 * j) for i, j in zip(*np.nonzero(mask))))
    assert np.array_equal(lat, lev.active)


def test_assemble_rows_equals_full_assembly():
    """The row-restricted assembly (used for full-size spot checks) adds the
    same element contributions as the full assembly."""
    import workloads as W
    from oracle import assemble as AS
    from oracle import geometry as G
    w = W.small_discs(seed=11, n=32, degree=3, levels=3, n_discs=6, depth=1, rhs="manufactured", nu=2)
    leaf = G.leaf_values(w, w.n, w.depth)
    sysf = AS.assemble(w, leaf, w.n, w.depth)
    lev = sysf.level
    pick = np.random.default_rng(0).choice(len(lev.active), 25, replace=False)
    rows = [int(lev.active[i]) for i in pick]
    _, A, b = AS.assemble_rows(w, leaf, w.n, w.depth, rows)
    pos = {int(L): i for i, L in enumerate(lev.active)}
    for L in rows:
        i = pos[L]
        full = sysf.A.getrow(i).toarray().ravel()
        mine = np.zeros_like(full)
        for Lc, v in A[L].items():
            mine[pos[Lc]] = v
        assert np.abs(full - mine).max() <= 1e-13 * np.abs(full).max()
        assert abs(sysf.b[i] - b[L]) <= 1e-13 * max(abs(sysf.b[i]), np.abs(sysf.b).max())
