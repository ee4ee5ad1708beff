"""Native generator vs the CPU oracle (no GPU).

Integer structures (active sets, CSR patterns, restriction patterns, block
lists) must agree bit-exactly; floating-point values to 1e-12 relative per row.
"""
import numpy as np
import pytest

import workloads as W
from oracle import problem as P
from oracle import schwarz as SW

GN = pytest.importorskip("paper_1903_10977_amd.generator")


def _lib_ok():
    try:
        GN._load()
        return True
    except RuntimeError:
        return False


pytestmark = pytest.mark.skipif(not _lib_ok(), reason="libimsmg_gen.so not built")

CASES = [
    W.c1(),
    W.small_discs(seed=11, n=16, degree=3, levels=3, n_discs=5, depth=1, rhs="manufactured", nu=2),
    W.small_discs(seed=12, n=16, degree=1, levels=3, n_discs=8, depth=2),
    W.small_gyroid(seed=5, n=8, degree=2, levels=2),
    W.star(n=16, depth=3),
    W.Workload(name="neumann-p2", dim=2, degree=2, n=8, depth=2, levels=2, geometry="discs",
               discs=[[0.5, 0.5, 0.3]], bc="neumann", rhs="one"),
]


def _rowrel(A, B):
    d = abs(A - B)
    rm = abs(A).max(axis=1).toarray().ravel()
    rm[rm == 0] = 1.0
    return float((d.max(axis=1).toarray().ravel() / rm).max())


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_generator_matches_oracle(w):
    g = GN.generate(w, with_mass=True)
    op = P.build(w, smoothers=False)
    for l in range(w.levels):
        ol, gl = op.hier.levels[l], g.levels[l]
        assert np.array_equal(ol.active, gl.dof_to_lattice)
        A, B = op.hier.A[l], gl.A
        assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
        assert _rowrel(A, B) < 1e-12
        if l > 0:
            R, GR = op.hier.R[l - 1], gl.R
            assert np.array_equal(R.indptr, GR.indptr) and np.array_equal(R.indices, GR.indices)
            assert abs(R - GR).max() < 1e-14
            ob, oassoc = SW.select_blocks(ol)
            gb = gl.blocks()
            assert len(ob) == len(gb)
            assert all(np.array_equal(a, b) for a, b in zip(ob, gb))
            assert np.array_equal(np.array(oassoc), gl.block_assoc)
    assert np.abs(op.b - g.b).max() <= 1e-12 * max(np.abs(op.b).max(), 1e-300)
    assert _rowrel(op.system.M, g.M) < 1e-12


def test_generator_rejects_bad_spec():
    w = W.c1()
    w.n = 30  # not divisible by 2^(levels-1) = 4
    with pytest.raises(RuntimeError):
        GN.generate(w)


@pytest.mark.parametrize("w", [W.apple(n=8, levels=2), W.slab(n=8, levels=2),
                               W.thb_star_elasticity(n=16, local_levels=0, levels=2)], ids=lambda w: w.name)
def test_generator_elasticity_matches_oracle(w):
    """Linear elasticity on the apple with a bite and on the clamped slab (8^3,
    two levels), and in 2D on the clamped star (16^2, uniform B-splines: the
    grid operator of the THB levels): vector operators (component-major) on
    the structural pattern of every component pair, load, vector mass,
    R = I (x) R_scalar and the per-component blocks against the oracle's
    independent assembly (1e-12 per row)."""
    from oracle import elasticity as E
    g = GN.generate(w, with_mass=True)
    op = E.build(w, smoothers=False)
    d = w.dim
    assert g.fine.ncomp == d
    for l in range(w.levels):
        ol, gl = op.hier.levels[l], g.levels[l]
        assert np.array_equal(ol.active, gl.dof_to_lattice)
        Pv = E.vector_pattern(ol, d)
        B = gl.A
        assert np.array_equal(Pv.indptr, B.indptr) and np.array_equal(Pv.indices, B.indices)
        assert _rowrel(op.hier.A[l], B) < 1e-12
        assert abs(B - B.T).max() == 0.0 if l == w.levels - 1 else True
        if l > 0:
            R, GR = op.hier.R[l - 1], gl.R
            assert abs(R - GR).max() < 1e-14
            ob, _ = E.vector_blocks(ol, d)
            gb = gl.blocks()
            assert len(ob) == len(gb)
            assert all(np.array_equal(a, b) for a, b in zip(ob, gb))
    bo = op.system.b
    assert np.abs(g.b - bo).max() <= 1e-12 * np.abs(bo).max()
    assert abs(g.M - op.system.M).max() <= 1e-14 * abs(op.system.M).max()
