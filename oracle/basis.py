"""Univariate bases (oracle; test infrastructure only).

Immersed formulation section: uniform B-splines with open knot vectors and
maximal smoothness, and traditional C0 Lagrange functions, both posed on the
tensor background grid.  Multivariate functions are tensor products.

B-splines: degree p on n uniform elements of [lo, hi]; open knot vector with
p+1 repeated end knots; n + p functions; function i is supported on elements
max(0, i-p) .. min(n-1, i).  Evaluation follows the Cox-de Boor recursion
written out literally (no triangular-table tricks).

Lagrange: degree p on n elements; node lattice of p n + 1 equidistant nodes;
node i is a vertex node when i % p == 0 (support: the one or two elements
sharing that vertex), otherwise interior to element i // p.
"""
from __future__ import annotations

import numpy as np


def open_knots(n: int, p: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    inner = lo + (hi - lo) * np.arange(n + 1, dtype=np.float64) / n
    return np.concatenate([np.full(p, lo), inner, np.full(p, hi)])


def _cox_de_boor(t: np.ndarray, i: int, k: int, x: np.ndarray, span: int) -> np.ndarray:
    """N_{i,k}(x) for points x known to lie in knot span [t_span, t_span+1]
    (closed on both sides: the span is passed explicitly so the right end of
    the interval is handled without half-open ambiguities)."""
    if k == 0:
        return np.full(x.shape, 1.0 if i == span else 0.0)
    out = np.zeros(x.shape)
    d1 = t[i + k] - t[i]
    if d1 > 0.0:
        out = out + (x - t[i]) / d1 * _cox_de_boor(t, i, k - 1, x, span)
    d2 = t[i + k + 1] - t[i + 1]
    if d2 > 0.0:
        out = out + (t[i + k + 1] - x) / d2 * _cox_de_boor(t, i + 1, k - 1, x, span)
    return out


def bspline_eval(n: int, p: int, e: int, x: np.ndarray, lo: float = 0.0, hi: float = 1.0):
    """Values and first derivatives of the p+1 B-splines that are non-zero on
    element e, at points x (array) inside that element.

    Returns (vals, ders), each of shape (p+1, len(x)); row a is function e + a.
    The derivative uses the standard recursion
    N'_{i,p} = p/(t_{i+p}-t_i) N_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) N_{i+1,p-1}.
    """
    t = open_knots(n, p, lo, hi)
    x = np.asarray(x, dtype=np.float64)
    span = e + p  # knot span index of element e in the open knot vector
    vals = np.zeros((p + 1, x.size))
    ders = np.zeros((p + 1, x.size))
    for a in range(p + 1):
        i = e + a
        vals[a] = _cox_de_boor(t, i, p, x.ravel(), span)
        if p > 0:
            d = np.zeros(x.size)
            d1 = t[i + p] - t[i]
            if d1 > 0.0:
                d += p / d1 * _cox_de_boor(t, i, p - 1, x.ravel(), span)
            d2 = t[i + p + 1] - t[i + 1]
            if d2 > 0.0:
                d -= p / d2 * _cox_de_boor(t, i + 1, p - 1, x.ravel(), span)
            ders[a] = d
    return vals, ders


def bspline_all(n: int, p: int, x: np.ndarray, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """All n + p B-splines at points x (any location in [lo, hi]); shape (n+p, len(x))."""
    x = np.asarray(x, dtype=np.float64).ravel()
    h = (hi - lo) / n
    e = np.clip(np.floor((x - lo) / h).astype(np.int64), 0, n - 1)
    out = np.zeros((n + p, x.size))
    for el in np.unique(e):
        m = e == el
        v, _ = bspline_eval(n, p, int(el), x[m], lo, hi)
        out[el:el + p + 1, m] = v
    return out


def bspline_support(n: int, p: int, i: int):
    """Elements (1D) on which B-spline i is non-zero."""
    return range(max(0, i - p), min(n - 1, i) + 1)


def lagrange_nodes_1d(n: int, p: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    return lo + (hi - lo) * np.arange(p * n + 1, dtype=np.float64) / (p * n)


def lagrange_eval(n: int, p: int, e: int, x: np.ndarray, lo: float = 0.0, hi: float = 1.0):
    """Values and derivatives of the p+1 Lagrange polynomials on element e
    (nodes p e .. p e + p) at points x in that element; shapes (p+1, len(x))."""
    x = np.asarray(x, dtype=np.float64).ravel()
    h = (hi - lo) / n
    xi = lo + h * e + h * np.arange(p + 1) / p
    vals = np.ones((p + 1, x.size))
    ders = np.zeros((p + 1, x.size))
    for a in range(p + 1):
        for b in range(p + 1):
            if b != a:
                vals[a] *= (x - xi[b]) / (xi[a] - xi[b])
        for c in range(p + 1):
            if c == a:
                continue
            term = np.full(x.size, 1.0 / (xi[a] - xi[c]))
            for b in range(p + 1):
                if b != a and b != c:
                    term = term * (x - xi[b]) / (xi[a] - xi[b])
            ders[a] += term
    return vals, ders


def lagrange_all(n: int, p: int, x: np.ndarray, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64).ravel()
    h = (hi - lo) / n
    e = np.clip(np.floor((x - lo) / h).astype(np.int64), 0, n - 1)
    out = np.zeros((p * n + 1, x.size))
    for el in np.unique(e):
        m = e == el
        v, _ = lagrange_eval(n, p, int(el), x[m], lo, hi)
        out[p * el:p * el + p + 1, m] = v
    return out


def lagrange_support(n: int, p: int, i: int):
    if i % p == 0:
        v = i // p
        return range(max(0, v - 1), min(n - 1, v) + 1)
    return range(i // p, i // p + 1)


def nfuncs_1d(basis: str, n: int, p: int) -> int:
    return n + p if basis == "bspline" else p * n + 1


def eval_1d(basis: str, n: int, p: int, e: int, x, lo, hi):
    if basis == "bspline":
        return bspline_eval(n, p, e, x, lo, hi)
    return lagrange_eval(n, p, e, x, lo, hi)


def first_func_1d(basis: str, p: int, e: int) -> int:
    """Index of the first of the p+1 functions non-zero on element e."""
    return e if basis == "bspline" else p * e


def support_1d(basis: str, n: int, p: int, i: int):
    return bspline_support(n, p, i) if basis == "bspline" else lagrange_support(n, p, i)


def all_1d(basis: str, n: int, p: int, x, lo, hi):
    return bspline_all(n, p, x, lo, hi) if basis == "bspline" else lagrange_all(n, p, x, lo, hi)
