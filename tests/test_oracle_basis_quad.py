"""Pins of the oracle's bases and cut-cell quadrature against closed forms.

Bases (immersed formulation section): open uniform B-splines and Lagrange
polynomials.  Quadrature (Figure 1 caption): bisection, triangulation, Gauss
rules on the clipped subcells and on the approximate boundary.
"""
import math

import numpy as np
import pytest

from oracle import basis as B
from oracle import quadrature as Q
from oracle import geometry as G
import workloads as W


@pytest.mark.parametrize("p", [1, 2, 3])
def test_bspline_partition_of_unity(p):
    n = 7
    x = np.random.default_rng(0).uniform(0, 1, 200)
    V = B.bspline_all(n, p, x)
    assert np.allclose(V.sum(axis=0), 1.0, atol=1e-14)
    assert V.min() >= -1e-15
    for e in range(n):
        xs = (e + np.linspace(0.01, 0.99, 9)) / n
        _, D = B.bspline_eval(n, p, e, xs)
        assert np.allclose(D.sum(axis=0), 0.0, atol=1e-11)


def test_bspline_uniform_closed_forms():
    # uniform quadratic B-spline: 1/2 at its inner knots, 3/4 at its centre
    n, p = 8, 2
    V = B.bspline_all(n, p, np.array([3 / n, 3.5 / n, 4 / n]))
    i = 4  # supported on elements 2..4, centre of element 3
    assert V[i, 0] == pytest.approx(0.5, abs=1e-15)
    assert V[i, 1] == pytest.approx(0.75, abs=1e-15)
    assert V[i, 2] == pytest.approx(0.5, abs=1e-15)
    # uniform cubic: 1/6, 2/3, 1/6 at consecutive inner knots
    n, p = 10, 3
    i = 6  # elements 3..6
    V = B.bspline_all(n, p, np.array([4 / n, 5 / n, 6 / n]))
    assert np.allclose(V[i], [1 / 6, 2 / 3, 1 / 6], atol=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_lagrange_kronecker_and_unity(p):
    n = 5
    nodes = B.lagrange_nodes_1d(n, p)
    V = B.lagrange_all(n, p, nodes)
    assert np.allclose(V, np.eye(len(nodes)), atol=1e-12)
    x = np.random.default_rng(1).uniform(0, 1, 100)
    assert np.allclose(B.lagrange_all(n, p, x).sum(axis=0), 1.0, atol=1e-12)


def test_linear_reproduction_by_greville():
    from oracle.hierarchy import greville
    for p in (1, 2, 3):
        n = 6
        x = np.linspace(0, 1, 31)
        V = B.bspline_all(n, p, x)
        assert np.allclose(greville(n, p, 0, 1) @ V, x, atol=1e-14)


@pytest.mark.parametrize("q,deg", [(3, 4), (4, 6), (6, 10)])
def test_triangle_rule_monomials(q, deg):
    # int over {0 <= y <= x <= 1} of x^a y^b = 1 / ((b+1)(a+b+2))
    P = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0]])
    p, w = Q.triangle_rule(P, q)
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            exact = 1.0 / ((b + 1) * (a + b + 2))
            assert np.dot(w, p[:, 0] ** a * p[:, 1] ** b) == pytest.approx(exact, rel=1e-13)


def test_tet_rule_monomials():
    # unit simplex {x,y,z >= 0, x+y+z <= 1}: int x^a y^b z^c = a! b! c! / (a+b+c+3)!
    P = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0], [0.0, 0, 1]])
    q = 7
    p, w = Q.tet_rule(P, q)
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                exact = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
                got = np.dot(w, p[:, 0] ** a * p[:, 1] ** b * p[:, 2] ** c)
                assert got == pytest.approx(exact, rel=1e-12)


def _single_cell_leaf(psi, depth, d):
    s = 2 ** depth
    c = G.leaf_coords(0.0, 1.0, s)
    grids = np.meshgrid(*([c] * d), indexing="ij")
    return G.snap(psi(np.stack(grids, -1)))


@pytest.mark.parametrize("depth", [0, 2])
@pytest.mark.parametrize("c", [0.3, 0.77, 1.4])
def test_clipped_square_area_and_boundary(depth, c):
    # Omega = {x + y < c}: linear psi is reproduced exactly by the leaf interpolant
    leaf = _single_cell_leaf(lambda P: c - P[..., 0] - P[..., 1], depth, 2)
    vp, vw, bp, bw, bn = Q.element_quadrature(leaf, (0, 0), depth, 0.0, 1.0, 3, 4, 3)
    area = c * c / 2 if c <= 1 else 1 - (2 - c) ** 2 / 2
    length = c * math.sqrt(2) if c <= 1 else (2 - c) * math.sqrt(2)
    assert vw.sum() == pytest.approx(area, rel=1e-13)
    assert bw.sum() == pytest.approx(length, rel=1e-13)
    assert np.allclose(bn, [1 / math.sqrt(2), 1 / math.sqrt(2)], atol=1e-13)
    # first moment: int x over the region
    mx = c ** 3 / 6 if c <= 1 else None
    if mx is not None:
        assert np.dot(vw, vp[:, 0]) == pytest.approx(mx, rel=1e-12)


@pytest.mark.parametrize("c", [0.5, 1.3, 2.6])
def test_clipped_cube_volume_and_area(c):
    leaf = _single_cell_leaf(lambda P: c - P[..., 0] - P[..., 1] - P[..., 2], 0, 3)
    vp, vw, bp, bw, bn = Q.element_quadrature(leaf, (0, 0, 0), 0, 0.0, 1.0, 3, 4, 4)

    def vol(t):  # volume of {x+y+z < t} in the unit cube
        f = lambda s: max(s, 0.0) ** 3
        return (f(t) - 3 * f(t - 1) + 3 * f(t - 2) - f(t - 3)) / 6

    def area(t):  # area of the plane section x+y+z = t, = sqrt(3) d/dt vol
        f = lambda s: max(s, 0.0) ** 2
        return math.sqrt(3) * (f(t) - 3 * f(t - 1) + 3 * f(t - 2) - f(t - 3)) / 2

    assert vw.sum() == pytest.approx(vol(c), rel=1e-13)
    assert bw.sum() == pytest.approx(area(c), rel=1e-12)
    assert np.allclose(bn, np.full(3, 1 / math.sqrt(3)), atol=1e-13)


def test_disc_area_converges_with_depth():
    # |Omega_h| of the unit square minus one disc approaches 1 - pi r^2 at O(h_leaf^2)
    w = W.c1()
    r = w.discs[0][2]
    exact = 1 - math.pi * r * r
    errs = []
    for depth in (0, 1, 2, 3):
        leaf = G.leaf_values(w, 8, depth)
        tot = 0.0
        for e in zip(*np.nonzero(G.active_elements(leaf, 8, depth))):
            _, vw, _, _, _ = Q.element_quadrature(leaf, e, depth, 0.0, 1 / 8, 2, 2, 2)
            tot += vw.sum()
        errs.append(abs(tot - exact))
    assert errs[3] < errs[0] / 20
    assert errs[3] < 2e-3


def test_snap_and_sign_convention():
    v = G.snap(np.array([1e-14, -1e-14, 2e-13, -0.5]))
    assert list(v > 0) == [False, False, True, False]
    # discs are removed: the disc centre is outside, the square corner inside
    psi = G.level_set(W.c1())
    c = W.c1().discs[0]
    assert psi(np.array([[c[0], c[1]]]))[0] < 0
    assert psi(np.array([[0.01, 0.01]]))[0] > 0
