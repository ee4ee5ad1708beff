"""Batched form through the C ABI (imsmg_setup_batched /
imsmg_pcg_solve_batched): independent problems of mixed size and degree, 16
right-hand sides each, driven concurrently (one child context and stream per
problem, the library's pool of host threads); a batch problem equals the same
problem in a stand-alone context bit for bit.  Bars: every column reaches a true relative
residual <= 1e-8, and the concurrent run gives bit-for-bit the results of a
sequential run (no state is shared between contexts); with the general
blocks as BF16 patch GEMMs every column still reaches 1e-8."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# batched problems with 64^2 or 128^2 elements and p = 1, 2, 3
INDICES = [1, 2, 5, 7, 8, 12]


def test_concurrent_batch_matches_sequential_and_converges():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10977_amd import batch as BT
    from paper_1903_10977_amd import generator as GN
    from paper_1903_10977_amd import solver as S
    S.load()
    probs = [GN.generate(W.batched_c4(i), with_mass=True) for i in INDICES]
    print(f"[case batch] sizes {[g.fine.n for g in probs]}", flush=True)
    bs = BT.BatchSolver(probs, nrhs=16, precision=S.MIXED, workers=4)
    B = bs.rhs()
    Xc, infos_c, _ = bs.solve(B)
    bs.workers = 1
    Xs, infos_s, _ = bs.solve(B)
    for i, (a, b) in enumerate(zip(Xc, Xs)):
        assert torch.equal(a, b), INDICES[i]
        assert all(x.status == 0 and x.true_rel_res <= 1e-8 for x in infos_c[i]), \
            (INDICES[i], [(x.status, x.iterations, x.true_rel_res) for x in infos_c[i]])
        assert [x.iterations for x in infos_c[i]] == [x.iterations for x in infos_s[i]]
    # the batch context's problem 1 against a stand-alone context of the same
    # problem (same kernels, its own stream): bitwise the same columns
    g1 = probs[1]
    o1 = S.default_options(nu_pre=g1.workload.nu, nu_post=g1.workload.nu, precision=S.MIXED, max_iter=2000)
    alone = S.Solver(0).setup(g1, o1).factor()
    X1 = torch.zeros_like(B[1])
    alone.pcg_multi(B[1], X1, rtol=1e-8)
    assert torch.equal(X1, Xc[1])
    alone.close()
    # one problem against the stand-alone single-column solve of column 3
    g = probs[0]
    sol = S.Solver(0).setup(g, S.default_options(nu_pre=1, nu_post=1, precision=S.MIXED, max_iter=2000)).factor()
    x = torch.zeros(g.fine.n, dtype=torch.float64, device="cuda:0")
    info = sol.pcg(B[0][3].contiguous(), x, rtol=1e-8)
    assert abs(info.iterations - infos_c[0][3].iterations) <= 1
    r = g.fine.A @ Xc[0][3].cpu().numpy() - B[0][3].cpu().numpy()
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(B[0][3].cpu().numpy()) * 1.0001
    sol.close()
    bs.close()
    # the same batch with the general blocks as BF16 patch GEMMs on the matrix
    # cores (FP32 accumulation): every column still reaches 1e-8
    bs2 = BT.BatchSolver(probs, nrhs=16, precision=S.MIXED, workers=4, block_gemm=2)
    X2, infos2, _ = bs2.solve(B)
    for i, inf in enumerate(infos2):
        assert all(x.status == 0 and x.true_rel_res <= 1e-8 for x in inf), \
            (INDICES[i], [(x.status, x.iterations, x.true_rel_res) for x in inf])
    print(f"[case batch] BF16 patch GEMM iterations {[max(x.iterations for x in inf) for inf in infos2]} "
          f"(CSR {[max(x.iterations for x in inf) for inf in infos_c]})", flush=True)
    bs2.close()


@pytest.mark.parametrize("index", [16, 48, 17])
def test_batch_problem_matches_the_oracle(index):
    """One batch problem per degree p = 1, 2, 3 (64^2 elements, depth 4,
    3 levels) in a 3-problem batch, columns 0 and 5 of its 16 load vectors
    M u, against the oracle's PCG on the same right-hand sides (the oracle's
    M is its own mass matrix; both sides draw u from the same seed):
    residual <= 1e-8 with the oracle's A, iterations within one of the
    oracle's, L2(Omega) within 1e-6 of its solution."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import multigrid as MG
    from oracle import problem as P
    from paper_1903_10977_amd import batch as BT
    from paper_1903_10977_amd import generator as GN
    from paper_1903_10977_amd import solver as S
    S.load()
    idx = [index, 1, 2]
    probs = [GN.generate(W.batched_c4(i), with_mass=True) for i in idx]
    w = W.batched_c4(index)
    print(f"[case batch-oracle {index}] n={w.n} p={w.degree}", flush=True)
    op = P.build(w)
    bs = BT.BatchSolver(probs, nrhs=16, precision=S.FP64, workers=3)
    rng = np.random.Generator(np.random.PCG64(1000 + index))
    U = rng.standard_normal((16, probs[0].fine.n))
    B = bs.rhs()
    B[0] = torch.tensor(np.stack([op.system.M @ u for u in U]), device="cuda:0")
    X, infos, _ = bs.solve(B)
    M = op.system.M
    for k in (0, 5):
        b = B[0][k].cpu().numpy()
        xo, ito, _ = MG.pcg(op.A, b, op.vcycle.apply, tol=1e-8)
        xg = X[0][k].cpu().numpy()
        res = np.linalg.norm(b - op.A @ xg) / np.linalg.norm(b)
        e = xg - xo
        rel = np.sqrt(e @ (M @ e)) / np.sqrt(xo @ (M @ xo))
        print(f"[case batch-oracle {index}] column {k}: iterations gpu {infos[0][k].iterations} oracle {ito}, "
              f"residual {res:.2e}, L2 {rel:.2e}", flush=True)
        assert res <= 1.01e-8 and rel <= 1e-6
        assert abs(infos[0][k].iterations - ito) <= 1
    bs.close()
