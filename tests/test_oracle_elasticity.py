"""Pins of the oracle's linear elasticity (immersed finite element formulation:
eq:strongMulti, eq:weakMulti, eq:operatorsMulti; smoothers subsection for the
per-component blocks) against what the mechanics and the mathematics fix:

* rigid body motions (three translations, three rotations) produce no
  strain, so the volume part of a_h annihilates their coefficient vectors;
* consistency (patch test): a linear displacement u = a + B x lies in the
  quadratic spline space, and with the boundary traction sigma(u) n on the
  whole approximate boundary, the Dirichlet data g_D = u on the bite and no
  body load, b_h(v) = a_h(v, u) holds exactly by the divergence theorem on
  Omega_h (sigma constant, quadrature exact for the degrees involved);
* the penalty term on constant fields (no strain): summed over the
  components, (lambda + 6 mu) beta |Gamma_D| since |n| = 1;
* partition of unity: the loads of a constant body force sum to f |Omega_h|;
* the additive Schwarz bound gamma lambda_max(M^{-1} A) <= 1 (eq:applyCS)
  with the per-component blocks and gamma = 1 / max_K N_K;
* the two-level error propagation identity of eq:eigenMulti for the vector
  operator.
Each of these fails for a dropped term, a wrong sign, a transposed index
(d_c phi_a d_c' phi_b against d_c' phi_a d_c phi_b) or a wrong factor.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import assemble as AS
from oracle import elasticity as E
from oracle import geometry as G
from oracle import hierarchy as H
from oracle import quadrature as Q


def _apple(n=8, levels=2):
    return W.apple(n=n, levels=levels)


def _greville_coeffs(lev, fn):
    """Coefficients of a linear vector field fn(points) -> (m, d) in the
    B-spline basis: its values at the Greville points (exact for degree 1)."""
    g = H.greville(lev.n, lev.p, lev.lo, lev.hi)
    m = np.array([lev.lat_to_multi(int(L)) for L in lev.active])
    pts = np.stack([g[m[:, a]] for a in range(lev.dim)], axis=1)
    u = fn(pts)
    return np.concatenate([u[:, c] for c in range(lev.dim)])


@pytest.fixture(scope="module")
def apple8():
    w = _apple()
    leaf = G.leaf_values(w, w.n, w.depth)
    return w, leaf


@pytest.fixture(scope="module")
def built(apple8):
    """The oracle problem (2 levels) and the volume-only operator (beta = 0)."""
    w, leaf = apple8
    P = E.build(w)
    S0 = E.assemble_elasticity(w, leaf, w.n, w.depth, beta=0.0)
    return P, S0


def test_rigid_body_motions_produce_no_force(built):
    _, S = built
    lev = S.level
    modes = [lambda P, c=c: np.eye(3)[c][None, :] * np.ones((P.shape[0], 1)) for c in range(3)]
    for axis in range(3):
        om = np.eye(3)[axis]
        modes.append(lambda P, om=om: np.cross(om[None, :], P))
    scale = abs(S.A).max()
    for k, fn in enumerate(modes):
        c = _greville_coeffs(lev, fn)
        r = S.A @ c
        assert np.abs(r).max() <= 1e-11 * scale * np.abs(c).max(), (k, np.abs(r).max())
    # a pure strain is not in the kernel
    c = _greville_coeffs(lev, lambda P: np.stack([P[:, 0], 0 * P[:, 0], 0 * P[:, 0]], axis=1))
    assert np.abs(S.A @ c).max() > 1e-3 * scale


def test_patch_test_linear_displacement_is_reproduced(apple8):
    w, leaf = apple8
    rng = np.random.default_rng(11)
    a = rng.standard_normal(3)
    Bm = rng.standard_normal((3, 3))
    lam, mu = 2.5e3, 0.7e3   # unequal, so that their roles are checked (the apple has lambda = mu)
    eps = 0.5 * (Bm + Bm.T)
    sigma = lam * np.trace(eps) * np.eye(3) + 2.0 * mu * eps

    def u_lin(P):
        return a[None, :] + P @ Bm.T

    p = w.degree
    orders = (p + 1, 3 * p + 1, 3 * p + 1)   # exact for the volume and boundary integrands
    S = E.assemble_elasticity(w, leaf, w.n, w.depth, orders=orders, force=lambda P: np.zeros_like(P),
                              g_dirichlet=u_lin, traction=lambda P, nn: nn @ sigma.T, traction_on="all",
                              lam=lam, mu=mu)
    c = _greville_coeffs(S.level, u_lin)
    r = S.A @ c - S.b
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(S.b), np.linalg.norm(r) / np.linalg.norm(S.b)
    assert S.gamma_d_measure > 0.5   # the bite (penalty and its traction) is part of the test


def test_penalty_trace_on_constant_fields(apple8, built):
    """Constant fields e_c have no strain, so e_c^T A e_c is the penalty term
    alone: lambda beta int (n_c)^2 + 2 mu beta |Gamma_D|; summed over c that is
    (lambda + 6 mu) beta |Gamma_D| because |n| = 1."""
    w, _ = apple8
    P, S0 = built
    S = P.system
    beta = w.penalty_factor / ((w.box_hi - w.box_lo) / w.n)
    N = len(S.level.active)
    Pm = S.A - S0.A
    tot = 0.0
    for c in range(3):
        e = np.zeros(3 * N)
        e[c * N:(c + 1) * N] = 1.0
        tot += e @ (Pm @ e)
        assert abs(e @ (S0.A @ e)) <= 1e-9 * abs(S0.A).max()
    gd = S.gamma_d_measure
    assert gd > 0.5
    ref = (w.lame_lambda + 6.0 * w.lame_mu) * beta * gd
    assert abs(tot - ref) <= 1e-11 * ref


def test_body_force_sums_to_force_times_volume(apple8, built):
    w, _ = apple8
    S = built[0].system
    f = np.asarray(w.force)
    N = len(S.level.active)
    for c in range(3):
        assert abs(S.b[c * N:(c + 1) * N].sum() - f[c] * S.omega_measure) <= 1e-12 * S.omega_measure * 3


def test_operator_symmetric_positive_definite_and_vector_mass(built):
    S = built[0].system
    A = S.A.toarray()
    assert np.array_equal(A, A.T)
    # positive definite: Cholesky succeeds on the shifted-by-nothing matrix
    # in the energy of every random vector (tiny cut modes aside)
    x = np.random.default_rng(2).standard_normal((A.shape[0], 8))
    assert np.all(np.einsum("ij,ij->j", x, A @ x) > 0)
    N = len(S.level.active)
    Ms = S.M[:N, :N]
    assert abs(S.M[N:2 * N, N:2 * N] - Ms).max() == 0.0
    assert abs(S.M[:N, N:2 * N]).max() == 0.0
    assert abs(np.ones(N) @ (Ms @ np.ones(N)) - S.omega_measure) <= 1e-12 * S.omega_measure


def test_per_component_blocks_and_additive_bound(built):
    P = built[0]
    sm = P.smoothers[1]
    N = len(P.hier.levels[1].active)
    # every block lies in one component and the components repeat the scalar blocks
    comp = [set((np.asarray(b) // N).tolist()) for b in sm.raw_blocks]
    assert all(len(c) == 1 for c in comp)
    nb = len(sm.raw_blocks) // 3
    for k in range(nb):
        for c in (1, 2):
            assert np.array_equal(sm.raw_blocks[k] + c * N, sm.raw_blocks[c * nb + k])
    # gamma counts the blocks of every component: 1 / (3 (p+1)^3) on this grid
    assert sm.gamma == pytest.approx(1.0 / (3 * 27))
    S = sm.dense()
    A = P.hier.A[1].toarray()
    ev = np.linalg.eigvals(S @ A).real
    assert ev.max() <= 1.0 + 1e-8


def test_two_level_error_propagation_vector(built):
    """I - B A = (I - S A)(I - R^T A_c^{-1} R A)(I - S A) on random vectors,
    compared in the energy norm (rounding in the cut blocks' inverses grows
    like sqrt(cond) there, not like cond)."""
    P = built[0]
    A = P.hier.A[1]
    Ac = P.hier.A[0].toarray()
    R = P.hier.R[0]
    S = P.smoothers[1]
    rng = np.random.default_rng(5)
    for _ in range(3):
        v = rng.standard_normal(A.shape[0])
        y1 = v - P.vcycle.apply(A @ v)
        t = v - S.apply(A @ v)
        t = t - R.T @ np.linalg.solve(Ac, R @ (A @ t))
        y2 = t - S.apply(A @ t)
        e = y1 - y2
        assert np.sqrt(e @ (A @ e)) <= 1e-6 * np.sqrt(v @ (A @ v))
        # the identity is not vacuous: the propagated error is not tiny
        assert np.sqrt(y1 @ (A @ y1)) > 1e-3 * np.sqrt(v @ (A @ v))


def test_vector_multiplicative_colours_and_symmetric_cycle():
    """Per-component multiplicative Schwarz on the clamped slab: three times
    the scalar colour count (3 (p+1)^3 = 81), no two blocks of one colour
    share an element (brute force over all pairs, components included: they
    are coupled by A), the symmetric V-cycle (forward sweep before, reversed
    after) is a symmetric operator, and it needs fewer PCG iterations than
    the additive form."""
    import dataclasses
    w = W.slab(n=8, levels=2)
    wm = dataclasses.replace(w, smoother="ms")
    P = E.build(wm)
    sm = P.smoothers[1]
    lev = P.hier.levels[1]
    N = len(lev.active)
    assert len(set(sm.colours)) == 81
    from oracle import schwarz as SW
    els = SW.block_elements(lev, [np.asarray(b) % N for b in sm.blocks])
    by_colour = {}
    for j, c in enumerate(sm.colours):
        by_colour.setdefault(c, []).append(j)
    for c, js in by_colour.items():
        seen = set()
        for j in js:
            assert not (els[j] & seen), c
            seen |= els[j]
    rng = np.random.default_rng(3)
    for _ in range(3):
        u, v = rng.standard_normal((2, P.A.shape[0]))
        a, b = v @ P.vcycle.apply(u), u @ P.vcycle.apply(v)
        assert abs(a - b) <= 1e-10 * (abs(a) + abs(b))
    _, it_ms, _ = P.solve(tol=1e-8)
    _, it_as, _ = E.build(w).solve(tol=1e-8)
    assert it_ms < it_as, (it_ms, it_as)
