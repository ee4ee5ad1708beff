"""Kernel timing of the finest plain smoothing step (timing option).

With timing = n the context runs without graphs and launches the finest
level's fused residual + trivial-row kernel n times inside each event pair.
The step only reads x_a and r, so the repeats must leave the solve unchanged:
the solution is bitwise that of the graph-replayed solve without timing, the
iteration count the same, and the reported launch count a multiple of n.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("reps", [1, 4])
def test_repeated_timed_launches_leave_the_solve_unchanged(reps):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10977_amd import generator as GN
    from paper_1903_10977_amd import solver as S
    S.load()
    w = W.small_discs(seed=11, n=32, degree=3, levels=3, n_discs=6, depth=1, rhs="manufactured", nu=2)
    print(f"[case reps={reps}] n={w.n} p={w.degree} levels={w.levels}", flush=True)
    g = GN.generate(w)
    b = torch.tensor(g.b, device="cuda:0")
    xs, its = [], []
    for timing in (0, reps):
        o = S.default_options(nu_pre=w.nu, nu_post=w.nu, precision=S.MIXED, timing=timing,
                              use_graph=0 if timing else 1)
        sol = S.Solver(0).setup(g, o).factor()
        sol.kernel_time(reset=True)
        x = torch.zeros_like(b)
        info = sol.pcg(b, x, rtol=1e-8)
        assert info.status == 0 and info.true_rel_res <= 1e-8, info
        ms, cnt = sol.kernel_time()
        if timing:
            # nu - 1 plain pre-steps and nu - 1 plain post-steps per V-cycle
            assert cnt > 0 and cnt % reps == 0 and ms > 0, (ms, cnt)
        else:
            assert cnt == 0
        xs.append(x.cpu().numpy())
        its.append(info.iterations)
        sol.close()
    assert its[0] == its[1]
    assert np.array_equal(xs[0], xs[1])
