"""Degenerate inputs of the solve path, through the C ABI.

* b = 0: the initial residual is zero, so CG stops before its first
  iteration with x = 0 (single column, and one zero column among others in
  the multi-column solve, whose other columns still converge);
* one level: the V-cycle is the coarsest direct solve (Algorithm alg:MGV at
  l = 1), B = A^{-1}, so PCG reaches the solution in one iteration (as the
  oracle does) and one V-cycle equals the dense solve;
* empty or inconsistent setup arrays are rejected with INVALID_ARG.
"""
import ctypes as C
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10977_amd import solver as S
    S.load()
    return S


def _small(levels=3):
    return W.small_discs(seed=11, n=32, degree=3, levels=levels, n_discs=6, depth=1, rhs="manufactured", nu=2)


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_rhs_stops_at_once(precision):
    S = _gpu()
    from paper_1903_10977_amd import generator as GN
    w = _small()
    print(f"[case zero-rhs precision={precision}]", flush=True)
    g = GN.generate(w)
    o = S.default_options(nu_pre=w.nu, nu_post=w.nu, precision=precision)
    sol = S.Solver(0).setup(g, o).factor()
    b = torch.zeros(g.fine.n, dtype=torch.float64, device="cuda:0")
    x = torch.zeros_like(b)
    info = sol.pcg(b, x, rtol=1e-8)
    assert info.status == 0 and info.iterations == 0, info
    assert not torch.any(x != 0)
    # one zero column among three
    Bm = torch.zeros((3, g.fine.n), dtype=torch.float64, device="cuda:0")
    Bm[0] = torch.tensor(g.b, device="cuda:0")
    Bm[2] = 2.0 * Bm[0]
    Xm = torch.zeros_like(Bm)
    infos = sol.pcg_multi(Bm, Xm, rtol=1e-8)
    assert infos[1].status == 0 and infos[1].iterations == 0
    assert not torch.any(Xm[1] != 0)
    for k in (0, 2):
        assert infos[k].status == 0 and infos[k].true_rel_res <= 1e-8, infos[k]
    sol.close()


def test_single_level_is_the_direct_solve():
    S = _gpu()
    from paper_1903_10977_amd import generator as GN
    from oracle import problem as P
    w = W.small_discs(seed=11, n=16, degree=2, levels=1, n_discs=4, depth=1)
    print("[case one-level] n=16 p=2", flush=True)
    g = GN.generate(w, with_mass=True)
    op = P.build(w)
    xo, ito, _ = op.solve(tol=1e-8)
    sol = S.Solver(0).setup(g, S.default_options()).factor()
    A = op.A.tocsc()
    rng = np.random.Generator(np.random.PCG64(3))
    r = rng.standard_normal(g.fine.n)
    z = sol.vcycle(torch.tensor(r, device="cuda:0")).cpu().numpy()
    zd = spla.spsolve(A, r)
    assert np.linalg.norm(A @ z - r) <= 1e-10 * np.linalg.norm(r)
    b = torch.tensor(g.b, device="cuda:0")
    x = torch.zeros_like(b)
    info = sol.pcg(b, x, rtol=1e-8)
    print(f"[case one-level] iterations gpu {info.iterations} oracle {ito}", flush=True)
    assert info.status == 0 and info.iterations == ito == 1
    xg = x.cpu().numpy()
    M = op.system.M
    e = xg - xo
    assert math.sqrt(e @ (M @ e)) <= 1e-8 * math.sqrt(xo @ (M @ xo))
    e = z - zd
    assert math.sqrt(e @ (M @ e)) <= 1e-8 * math.sqrt(zd @ (M @ zd))
    sol.close()


def test_empty_setup_arrays_are_rejected():
    S = _gpu()
    sol = S.Solver(0)
    opt = S.default_options()
    A = S.Csr(nrows=0, ncols=0, nnz=0)
    lat = S.Lattice(dim=2, reach=1)
    lat.shape[0] = lat.shape[1] = lat.shape[2] = 1
    rc = sol.lib.imsmg_setup(sol.h, 1, C.byref(A), None, None, C.byref(lat), None, C.byref(opt))
    assert rc == -1
    assert b"non-empty" in sol.lib.imsmg_last_error(sol.h)
    rc = sol.lib.imsmg_setup(sol.h, 0, C.byref(A), None, None, C.byref(lat), None, C.byref(opt))
    assert rc == -1
    # the context is still usable for nothing but another setup: a solve is a state error
    x = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    rc = sol.lib.imsmg_pcg_solve(sol.h, C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()), C.c_double(1e-8), None)
    assert rc == -7
    sol.close()


def test_nan_right_hand_side_then_a_valid_solve():
    """A NaN in b is reported as IMSMG_ERR_NAN (single and multi-column); the
    next solve on the same context, with a valid b, must converge: the NaN
    status of one call does not leak into the next."""
    S = _gpu()
    from paper_1903_10977_amd import generator as GN
    w = _small()
    print("[case nan-rhs]", flush=True)
    g = GN.generate(w)
    sol = S.Solver(0).setup(g, S.default_options(nu_pre=w.nu, nu_post=w.nu)).factor()
    b = torch.tensor(g.b, device="cuda:0")
    bn = b.clone()
    bn[len(bn) // 2] = float("nan")
    x = torch.zeros_like(b)
    info = sol.pcg(bn, x, rtol=1e-8, raise_on_error=False)
    assert info.status == -6, info
    x.zero_()
    info = sol.pcg(b, x, rtol=1e-8)
    assert info.status == 0 and info.true_rel_res <= 1e-8, info
    Bm = torch.stack([b, bn, 2.0 * b])
    Xm = torch.zeros_like(Bm)
    infos = sol.pcg_multi(Bm, Xm, rtol=1e-8, raise_on_error=False)
    assert infos[1].status == -6, infos
    Bm[1] = 3.0 * b
    Xm.zero_()
    infos = sol.pcg_multi(Bm, Xm, rtol=1e-8)
    for i in infos:
        assert i.status == 0 and i.true_rel_res <= 1e-8, infos
    sol.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_far_start_meets_the_true_residual(precision):
    """x0 whose residual is 1e3 ||b||: the stopping threshold is rtol min(||r0||,
    ||b||), so the solve ends at a true relative residual <= rtol, with the
    oracle's iteration count (+-1) and its solution (L2 1e-6); with max_iter
    too small it reports IMSMG_ERR_NOT_CONVERGED and fills info."""
    S = _gpu()
    from oracle import multigrid as MG
    from oracle import problem as P
    from paper_1903_10977_amd import generator as GN
    w = W.c1()
    print(f"[case far-start precision={precision}]", flush=True)
    g = GN.generate(w, with_mass=True)
    op = P.build(w)
    rng = np.random.Generator(np.random.PCG64(7))
    x0 = rng.standard_normal(g.fine.n)
    x0 *= 1e3 * np.linalg.norm(op.b) / np.linalg.norm(op.b - op.A @ x0)
    oinfo = {}
    xo, ito, _ = MG.pcg(op.A, op.b, op.vcycle.apply, tol=1e-8, x0=x0, info=oinfo)
    assert oinfo["converged"]
    sol = S.Solver(0).setup(g, S.default_options(precision=precision)).factor()
    b = torch.tensor(g.b, device="cuda:0")
    x = torch.tensor(x0, device="cuda:0")
    info = sol.pcg(b, x, rtol=1e-8)
    xg = x.cpu().numpy()
    res = np.linalg.norm(op.b - op.A @ xg) / np.linalg.norm(op.b)
    print(f"[case far-start] iterations gpu {info.iterations} oracle {ito}, true residual {res:.2e}", flush=True)
    assert info.status == 0 and res <= 1.01e-8
    assert abs(info.iterations - ito) <= 1
    M = op.system.M
    e = xg - xo
    assert math.sqrt(e @ (M @ e)) <= 1e-6 * math.sqrt(xo @ (M @ xo))
    sol.close()
    sol = S.Solver(0).setup(g, S.default_options(precision=precision, max_iter=5)).factor()
    x = torch.tensor(x0, device="cuda:0")
    info = sol.pcg(b, x, rtol=1e-8, raise_on_error=False)
    assert info.status == -5 and info.true_rel_res > 1e-8, info
    sol.close()


def test_non_positive_diagonal_is_not_spd():
    """A flipped diagonal entry of the fine operator is rejected at setup with
    IMSMG_ERR_NOT_SPD (the operator is not SPD; nothing is launched on it)."""
    S = _gpu()
    from paper_1903_10977_amd import generator as GN
    w = _small()
    print("[case flipped-diagonal]", flush=True)
    g = GN.generate(w)
    A = g.fine.A.tocsr(copy=True)
    i = A.shape[0] // 3
    k = A.indptr[i] + int(np.nonzero(A.indices[A.indptr[i]:A.indptr[i + 1]] == i)[0][0])
    A.data[k] = -A.data[k]
    g.fine.A = A
    with pytest.raises(S.SolverError) as ei:
        S.Solver(0).setup(g, S.default_options(nu_pre=w.nu, nu_post=w.nu)).factor()
    assert ei.value.code == -4
