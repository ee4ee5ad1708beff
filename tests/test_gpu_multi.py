"""GPU parity of the multi-right-hand-side path (several systems with one
matrix, columns interleaved on the lattice) through the C ABI.

Bars: one V-cycle on nrhs columns equals nrhs single-column V-cycles to 1e-12
relative (same arithmetic except the coarsest dense product's summation
order; 1e-9 on the penalty star, whose near-singular Schwarz blocks amplify
that rounding difference by ~|z| / |r| ~ 1e9).  PCG: every column reaches a
true relative residual <= 1e-8; the finite-element right-hand side takes the
oracle's iteration count (+-1) and lands within relative L2(Omega) 1e-6 of the
oracle's solution; random right-hand sides (not finite-element consistent,
dominated by near-null cut modes whose recursive residual drifts) take the
single-column GPU solve's iteration count (+-1) (both restart CG from the
current iterate while the true residual is above rtol, as the oracle does);
a zero column stays zero.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10977_amd import solver as S
    S.load()
    return S


CASES = {
    "cubic-discs": lambda: W.small_discs(seed=11, n=32, degree=3, levels=3, n_discs=6, depth=1,
                                         rhs="manufactured", nu=2),
    "linear-discs": lambda: W.small_discs(seed=12, n=32, degree=1, levels=3, n_discs=8, depth=2),
    "star-lagrange": lambda: W.star(n=16, depth=3),
}
_cache = {}


def _problem(name):
    if name not in _cache:
        from paper_1903_10977_amd import generator as GN
        from oracle import problem as P
        w = CASES[name]()
        print(f"[case {name}] n={w.n} p={w.degree} levels={w.levels}", flush=True)
        _cache[name] = (w, GN.generate(w, with_mass=True), P.build(w))
    return _cache[name]


def _solver(S, g, **opt):
    w = g.workload
    o = S.default_options(nu_pre=w.nu, nu_post=w.nu, **opt)
    return S.Solver(0).setup(g, o).factor()


@pytest.mark.parametrize("nrhs", [3, 8, 16])
@pytest.mark.parametrize("name", list(CASES))
def test_multi_vcycle_equals_single_columns(name, nrhs):
    S = _gpu()
    w, g, op = _problem(name)
    sol = _solver(S, g)
    n = g.fine.n
    rng = np.random.Generator(np.random.PCG64(31 + nrhs))
    Rm = torch.tensor(rng.standard_normal((nrhs, n)), device="cuda:0")
    Zm = sol.vcycle_multi(Rm).cpu().numpy()
    for k in range(nrhs):
        z = sol.vcycle(Rm[k].contiguous()).cpu().numpy()
        tol = 1e-9 if name == "star-lagrange" else 1e-12
        assert np.abs(Zm[k] - z).max() <= tol * np.abs(z).max(), (name, nrhs, k)
    sol.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_multi_pcg_matches_oracle_per_column(name, precision):
    S = _gpu()
    from oracle import multigrid as MG
    w, g, op = _problem(name)
    sol = _solver(S, g, precision=S.FP64 if precision == "fp64" else S.MIXED)
    n = g.fine.n
    nrhs = 5
    rng = np.random.Generator(np.random.PCG64(41))
    B = rng.standard_normal((nrhs, n))
    B[2] = 0.0  # a zero right-hand side stays zero
    B[0] = g.b
    Bm = torch.tensor(B, device="cuda:0")
    Xm = torch.zeros_like(Bm)
    infos = sol.pcg_multi(Bm, Xm, rtol=1e-8)
    X = Xm.cpu().numpy()
    M = op.system.M
    for k in range(nrhs):
        if k == 2:
            assert infos[k].iterations == 0 and np.all(X[k] == 0.0)
            continue
        assert infos[k].true_rel_res <= 1e-8, (name, k, infos[k])
        if k == 0:
            x_ref, it_ref, _ = MG.pcg(op.A, B[k], op.vcycle.apply, tol=1e-8)
            assert abs(infos[k].iterations - it_ref) <= 1, (name, k, infos[k].iterations, it_ref)
            e = X[k] - x_ref
            assert np.sqrt(e @ (M @ e)) <= 1e-6 * np.sqrt(x_ref @ (M @ x_ref)), (name, k)
        else:
            x1 = torch.zeros(n, dtype=torch.float64, device="cuda:0")
            info1 = sol.pcg(Bm[k].contiguous(), x1, rtol=1e-8)
            assert abs(infos[k].iterations - info1.iterations) <= 1, (name, k, infos[k].iterations,
                                                                      info1.iterations)
    # repeated solves are bitwise identical
    Xm2 = torch.zeros_like(Bm)
    sol.pcg_multi(Bm, Xm2, rtol=1e-8)
    assert torch.equal(Xm, Xm2)
    sol.close()


def test_multi_pcg_sixteen_columns_match_single_solves():
    S = _gpu()
    w, g, op = _problem("cubic-discs")
    sol = _solver(S, g, precision=S.MIXED)
    n = g.fine.n
    rng = np.random.Generator(np.random.PCG64(43))
    # load vectors M u of random data u: standard-normal coefficient vectors
    # carry components along the near-null cut modes whose solutions are
    # ~kappa |b| large, and the FP64 true residual then stalls above 1e-8
    # (reported as NOT_CONVERGED)
    Bm = torch.tensor(np.stack([g.M @ u for u in rng.standard_normal((16, n))]), device="cuda:0")
    Xm = torch.zeros_like(Bm)
    infos = sol.pcg_multi(Bm, Xm, rtol=1e-8)
    for k in (0, 7, 15):
        x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
        info = sol.pcg(Bm[k].contiguous(), x, rtol=1e-8)
        assert abs(info.iterations - infos[k].iterations) <= 1
        d = (Xm[k] - x).cpu().numpy()
        assert np.linalg.norm(d) <= 1e-6 * np.linalg.norm(x.cpu().numpy())
    sol.close()
