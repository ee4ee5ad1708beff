"""The measured choice of lanes per general Schwarz row (autotune option).

The lane count only changes the summation order of the general-row product,
so a tuned context must agree with the default (4 lanes) to rounding: one
V-cycle to 1e-12 relative, PCG to a true relative residual <= 1e-8 with the
same iteration count (+-1) and solutions within 1e-6 relative in L2(Omega)
(the coefficient vectors of cut problems are dominated by near-null modes,
so they are compared in the mass norm, as in the oracle parity tests); every
level reports 2, 4 or 8 lanes, the default context 4 on every level.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "cubic-discs": lambda: W.small_discs(seed=11, n=32, degree=3, levels=3, n_discs=6, depth=1,
                                         rhs="manufactured", nu=2),
    "discs-256": lambda: W.c2(n=256, levels=4),
}


@pytest.mark.parametrize("name", list(CASES))
def test_tuned_lanes_agree_with_default(name):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10977_amd import generator as GN
    from paper_1903_10977_amd import solver as S
    S.load()
    w = CASES[name]()
    print(f"[case {name}] n={w.n} p={w.degree} levels={w.levels}", flush=True)
    g = GN.generate(w, with_mass=True)
    sols = {}
    for tune in (0, 1):
        o = S.default_options(nu_pre=w.nu, nu_post=w.nu, precision=S.MIXED, autotune=tune)
        sols[tune] = S.Solver(0).setup(g, o).factor()
    lanes = [sols[1].level_stats(l)["general_lanes"] for l in range(1, len(g.levels))]
    print(f"[case {name}] tuned lanes per level {lanes}", flush=True)
    assert all(x in (2, 4, 8) for x in lanes)
    assert all(sols[0].level_stats(l)["general_lanes"] == 4 for l in range(1, len(g.levels)))
    rng = np.random.Generator(np.random.PCG64(7))
    r = torch.tensor(rng.standard_normal(g.fine.n), device="cuda:0")
    z0 = sols[0].vcycle(r).cpu().numpy()
    z1 = sols[1].vcycle(r).cpu().numpy()
    assert np.abs(z0 - z1).max() <= 1e-12 * np.abs(z0).max()
    b = torch.tensor(g.b, device="cuda:0")
    xs, its = [], []
    for tune in (0, 1):
        x = torch.zeros_like(b)
        info = sols[tune].pcg(b, x, rtol=1e-8)
        assert info.true_rel_res <= 1e-8, (tune, info)
        xs.append(x.cpu().numpy())
        its.append(info.iterations)
    assert abs(its[0] - its[1]) <= 1, its
    e = xs[0] - xs[1]
    assert np.sqrt(e @ (g.M @ e)) <= 1e-6 * np.sqrt(xs[0] @ (g.M @ xs[0]))
    for s in sols.values():
        s.close()
