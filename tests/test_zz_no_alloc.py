"""The allocation-free loss/gradient entry point (imsmg_mlp_loss_grad_noalloc,
for callers that cannot allocate device memory) against the entry point with
a caller workspace (imsmg_mlp_loss_grad), through the C ABI: the same kernels
in the same order, so loss and gradient must be bitwise equal, on two calls
in a row (the second with fewer samples, so that stale workspace contents of
the first call would show), and sizes beyond the cap are rejected."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_10977_amd import solver as S
    return S, S.load()


def _p(t):
    return C.c_void_p(t.data_ptr())


def _case(S, lib, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = torch.tensor(0.2 * rng.standard_normal(S.MLP_PARAMS), dtype=torch.float32, device="cuda:0")
    X = torch.tensor(rng.standard_normal((n, S.NFEAT)), dtype=torch.float32, device="cuda:0")
    t = torch.tensor(rng.standard_normal(n), dtype=torch.float32, device="cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    work = torch.empty(int(lib.imsmg_mlp_workspace_bytes(n)), dtype=torch.uint8, device="cuda:0")
    loss_ref = torch.zeros(1, dtype=torch.float32, device="cuda:0")
    grad_ref = torch.zeros(S.MLP_PARAMS, dtype=torch.float32, device="cuda:0")
    assert lib.imsmg_mlp_loss_grad(stream, _p(params), _p(X), _p(t), n, _p(work), _p(loss_ref), _p(grad_ref)) == 0
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda:0")
    grad = torch.full((S.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda:0")
    assert lib.imsmg_mlp_loss_grad_noalloc(stream, _p(params), _p(X), _p(t), n, _p(loss), _p(grad)) == 0
    torch.cuda.synchronize()
    return loss_ref, grad_ref, loss, grad


def test_noalloc_loss_grad_equals_the_workspace_entry_point():
    S, lib = _lib()
    lib.imsmg_mlp_loss_grad_noalloc.argtypes = [C.c_void_p] * 4 + [C.c_int32] + [C.c_void_p] * 2
    for n, seed in ((S.NOALLOC_MAX_SAMPLES - 37, 1), (700, 2)):
        print(f"[case noalloc n={n} seed={seed}]", flush=True)
        loss_ref, grad_ref, loss, grad = _case(S, lib, n, seed)
        assert torch.isfinite(loss_ref).all() and torch.isfinite(grad_ref).all()
        assert torch.equal(loss, loss_ref), (n, loss.item(), loss_ref.item())
        assert torch.equal(grad, grad_ref), (n, (grad - grad_ref).abs().max().item())
    # the Python binding (marshalling only) gives the same numbers
    rng = np.random.Generator(np.random.PCG64(2))
    params = torch.tensor(0.2 * rng.standard_normal(S.MLP_PARAMS), dtype=torch.float32, device="cuda:0")
    X = torch.tensor(rng.standard_normal((700, S.NFEAT)), dtype=torch.float32, device="cuda:0")
    t = torch.tensor(rng.standard_normal(700), dtype=torch.float32, device="cuda:0")
    lb, gb = S.mlp_loss_grad_noalloc(params, X, t)
    torch.cuda.synchronize()
    assert torch.equal(lb, loss) and torch.equal(gb, grad)


def test_noalloc_rejects_sizes_beyond_the_cap():
    S, lib = _lib()
    lib.imsmg_mlp_loss_grad_noalloc.argtypes = [C.c_void_p] * 4 + [C.c_int32] + [C.c_void_p] * 2
    x = torch.zeros(16, dtype=torch.float32, device="cuda:0")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n in (0, S.NOALLOC_MAX_SAMPLES + 1):
        assert lib.imsmg_mlp_loss_grad_noalloc(stream, _p(x), _p(x), _p(x), n, _p(x), _p(x)) == -1
    assert lib.imsmg_mlp_loss_grad_noalloc(stream, None, _p(x), _p(x), 4, _p(x), _p(x)) == -1
