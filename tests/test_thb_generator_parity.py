"""The THB problem builder of the package (paper_1903_10977_amd/thb.py)
against the THB oracle: meshes, operators, restrictions, load vector,
Schwarz blocks and element incidence on every level.  The two share only
the seeded workload; the builder's grid system comes from the native
generator, the oracle's from its own assembly."""
import numpy as np
import pytest

import workloads as W
from oracle import thb as T
from paper_1903_10977_amd import thb as P

CASES = [dict(n=16, local_levels=2, levels=3), dict(n=32, local_levels=1, levels=3, seed=3),
         dict(n=16, local_levels=3, levels=2, seed=5), dict(n=16, local_levels=0, levels=3, seed=11)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c['n']}-m{c['local_levels']}-l{c['levels']}")
def test_thb_builder_matches_oracle(case):
    w = W.thb_discs(**case)
    pr = P.generate(w)
    ob = T.build(w)
    h = ob.hier
    assert len(pr.levels) == w.levels
    for l in range(w.levels):
        lp = pr.levels[l]
        lo = h.levels[l]
        assert lp.dof_to_lattice is None
        Ap, Ao = lp.A, h.A[l]
        assert Ap.shape == Ao.shape
        assert abs(Ap - Ao).max() <= 1e-12 * abs(Ao).max()
        # element incidence over the elements meeting Omega (same order)
        on = np.nonzero(lo.elem_on)[0]
        assert lp.elem_ptr is not None and len(lp.elem_ptr) - 1 == len(on)
        for q, e in enumerate(on):
            got = lp.elem_idx[lp.elem_ptr[q]:lp.elem_ptr[q + 1]].tolist()
            assert got == sorted(lo.elem_funcs.get(int(e), []))
        if l > 0:
            Rp, Ro = lp.R, h.R[l - 1]
            assert Rp.shape == Ro.shape and abs(Rp - Ro).max() <= 1e-12
            bp = lp.blocks()
            bo = ob.smoothers[l].raw_blocks
            assert len(bp) == len(bo) and all(np.array_equal(a, b) for a, b in zip(bp, bo))
    assert np.abs(pr.b - h.b).max() <= 1e-14 * np.abs(h.b).max()


@pytest.mark.parametrize("case", [dict(n=16, local_levels=1, levels=4), dict(n=12, local_levels=2, levels=3)],
                         ids=lambda c: f"n{c['n']}-m{c['local_levels']}-l{c['levels']}")
def test_thb_elasticity_builder_matches_oracle(case):
    """Vector THB levels (2D linear elasticity on the star): operators,
    restrictions, load vector, per-component blocks and the element lists
    holding the DOFs of both components."""
    w = W.thb_star_elasticity(**case)
    pr = P.generate(w)
    ob = T.build(w)
    h = ob.hier
    assert h.ncomp == 2
    for l in range(w.levels):
        lp, lo = pr.levels[l], h.levels[l]
        N = lo.C.shape[0]
        Ap, Ao = lp.A, h.A[l]
        assert Ap.shape == Ao.shape == (2 * N, 2 * N)
        assert abs(Ap - Ao).max() <= 1e-12 * abs(Ao).max()
        on = np.nonzero(lo.elem_on)[0]
        assert len(lp.elem_ptr) - 1 == len(on)
        for q, e in enumerate(on):
            got = lp.elem_idx[lp.elem_ptr[q]:lp.elem_ptr[q + 1]].tolist()
            f = sorted(lo.elem_funcs.get(int(e), []))
            assert got == f + [k + N for k in f]
        if l > 0:
            Rp, Ro = lp.R, h.R[l - 1]
            assert Rp.shape == Ro.shape and abs(Rp - Ro).max() <= 1e-12
            bp = lp.blocks()
            bo = ob.smoothers[l].raw_blocks
            assert len(bp) == len(bo) and all(np.array_equal(a, b) for a, b in zip(bp, bo))
    assert np.abs(pr.b - h.b).max() <= 1e-14 * np.abs(h.b).max()
