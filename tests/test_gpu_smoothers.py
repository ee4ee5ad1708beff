"""GPU parity of the multiplicative Schwarz smoother (with colouring), the
diagonal coarse smoothers (Jacobi, Gauss-Seidel) and the W-cycle against the
oracle, through the C ABI.

Bars (as the additive smoother's): colours bit-exact; the forward sweep row
by row within the blocks' conditioning bound on random r and in L2(Omega)
within 1e-6 on load vectors r = M u; one cycle in L2(Omega) within 1e-7 on
M u; PCG to a true relative residual <= 1e-8 with the oracle's iteration count
(+-1 in FP64, +-2 with FP32 operators) and L2(Omega) within 1e-6 of its
solution.  The convergence-flag path (every level reads the flag) gives the
same solve bit for bit.
"""
import dataclasses
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = 2.0 ** -52


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10977_amd import solver as S
    S.load()
    return S


BASE = {
    "C1": lambda: W.c1(),
    "cubic-discs": lambda: W.small_discs(seed=11, n=32, degree=3, levels=3, n_discs=6, depth=1,
                                         rhs="manufactured", nu=2),
    "gyroid-3d": lambda: W.small_gyroid(seed=5, n=16, degree=2, levels=2),
    "star-lagrange": lambda: W.star(n=16, depth=3),
}
VARIANTS = {
    "ms": dict(smoother="ms"),
    "as+gs": dict(smoother="as", coarse_smoother="gs"),
    "ms+jacobi": dict(smoother="ms", coarse_smoother="jacobi"),
    "as-w": dict(cycle=2),
    "ms-w": dict(smoother="ms", cycle=2),
}
CASES = [("C1", "ms"), ("C1", "as+gs"), ("C1", "ms+jacobi"), ("C1", "as-w"), ("C1", "ms-w"),
         ("cubic-discs", "ms"), ("cubic-discs", "as+gs"), ("cubic-discs", "ms-w"),
         ("gyroid-3d", "ms"), ("star-lagrange", "ms")]
_cache = {}


def _problem(name, var):
    key = (name, var)
    if key not in _cache:
        from oracle import problem as P
        from paper_1903_10977_amd import generator as GN
        w = dataclasses.replace(BASE[name](), **VARIANTS[var])
        print(f"[case {name}/{var}] n={w.n} p={w.degree} levels={w.levels}", flush=True)
        _cache[key] = (w, GN.generate(w, with_mass=True), P.build(w))
    return _cache[key]


def _solver(S, g, **opt):
    w = g.workload
    o = S.default_options(nu_pre=w.nu, nu_post=w.nu, **S.smoother_options(w), **opt)
    return S.Solver(0).setup(g, o).factor()


def _t(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda:0")


def _level_mass(op, l):
    M = op.system.M
    for ll in range(len(op.hier.A) - 1, l, -1):
        R = op.hier.R[ll - 1]
        M = R @ M @ R.T
    return M


def _mrel(e, ref, M):
    return math.sqrt(max(e @ (M @ e), 0.0)) / math.sqrt(ref @ (M @ ref))


@pytest.mark.parametrize("name,var", CASES)
def test_colours_and_forward_sweep(name, var):
    from oracle import schwarz as SW
    S = _gpu()
    w, g, op = _problem(name, var)
    sol = _solver(S, g)
    rng = np.random.default_rng(21)
    for l in range(1, w.levels):
        sm = op.smoothers[l]
        if not isinstance(sm, SW.MultiplicativeSmoother):
            continue
        ptr, idx = sol.get_patches(l)
        gblocks = [idx[ptr[j]:ptr[j + 1]] for j in range(len(ptr) - 1)]
        if len(gblocks) != len(sm.blocks) or any(not np.array_equal(a, b) for a, b in zip(gblocks, sm.blocks)):
            # a removal decision in the ambiguous band (checked by the
            # additive parity test) changes this level's sweep: compare the
            # other levels
            print(f"[{name}/{var}] level {l}: block lists differ in the removal band, sweep not compared")
            continue
        nc, col = sol.get_patch_colours(l)
        assert np.array_equal(col, np.asarray(sm.colours)), (name, var, l)
        assert nc == max(sm.colours) + 1
        A = op.hier.A[l]
        r = rng.standard_normal(A.shape[0])
        y = sol.apply_smoother(l, _t(r)).cpu().numpy()
        ref = sm.forward(r)
        # a sweep propagates each block's rounding through the later
        # residuals: bound by the blocks' (kappa_j + 1) eps / lambda_min,j |r|
        bar = np.zeros(len(r))
        for k, lam in zip(sm.blocks, sm.lam):
            if len(k):
                bar[k] += 100 * EPS * (lam.max() / lam.min() + 1.0) / lam.min() * np.linalg.norm(r)
        worst = float(np.max(np.abs(y - ref) / (bar + 1e-12 * np.abs(ref).max())))
        M = _level_mass(op, l)
        rm = M @ rng.standard_normal(A.shape[0])
        ym = sol.apply_smoother(l, _t(rm)).cpu().numpy()
        refm = sm.forward(rm)
        d = _mrel(ym - refm, refm, M)
        print(f"[{name}/{var}] level {l}: {nc} colours, sweep row err/bar {worst:.2e}, L2 rel on M u {d:.2e}")
        assert worst <= 1.0 and d <= 1e-6, (name, var, l, worst, d)
    sol.close()


@pytest.mark.parametrize("name,var", CASES)
def test_cycle_matches_oracle(name, var):
    S = _gpu()
    w, g, op = _problem(name, var)
    sol = _solver(S, g)
    rng = np.random.default_rng(22)
    M = op.system.M
    r = M @ rng.standard_normal(op.A.shape[0])
    z = sol.vcycle(_t(r)).cpu().numpy()
    zr = op.vcycle.apply(r)
    d = _mrel(z - zr, zr, M)
    print(f"[{name}/{var}] cycle L2 rel diff on M u {d:.3e}")
    assert d <= 1e-7, (name, var, d)
    sol.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name,var", CASES)
def test_pcg_matches_oracle(name, var, precision):
    S = _gpu()
    w, g, op = _problem(name, var)
    b = op.b if w.rhs != "zero" else np.random.default_rng(10).standard_normal(op.A.shape[0])
    xo, ito, _ = op.solve(b=b, tol=1e-8)
    sol = _solver(S, g, precision=precision)
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda:0")
    info = sol.pcg(_t(g.b if w.rhs != "zero" else b), x, rtol=1e-8)
    xg = x.cpu().numpy()
    res = np.linalg.norm(b - op.A @ xg) / np.linalg.norm(b)
    M = op.system.M
    e = xg - xo
    rel = math.sqrt(e @ (M @ e)) / math.sqrt(xo @ (M @ xo))
    print(f"[{name}/{var}/p{precision}] iterations gpu {info.iterations} oracle {ito}, residual {res:.2e}, L2 {rel:.2e}")
    assert res <= 1.01e-8 and rel <= 1e-6
    assert abs(info.iterations - ito) <= (1 if precision == 0 else 2), (info.iterations, ito)
    # the convergence-flag path on every level: the same solve bit for bit
    sol2 = _solver(S, g, precision=precision, flag_min_rows=0)
    x2 = torch.zeros_like(x)
    sol2.pcg(_t(g.b if w.rhs != "zero" else b), x2, rtol=1e-8)
    assert torch.equal(x, x2)
    sol.close()
    sol2.close()


def test_multiplicative_rejections():
    S = _gpu()
    w, g, op = _problem("C1", "ms")
    sol = _solver(S, g)
    Bm = torch.zeros((4, g.fine.n), dtype=torch.float64, device="cuda:0")
    with pytest.raises(S.SolverError) as ei:
        sol.pcg_multi(Bm, torch.zeros_like(Bm), rtol=1e-8)
    assert ei.value.code == -1
    sol.close()
    with pytest.raises(S.SolverError) as ei:
        _solver(S, g, use_learned=1)
    assert ei.value.code == -1
