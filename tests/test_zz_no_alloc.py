"""The allocation-free gradient entry point (lbs_grad_noalloc) against the
surrogate's lbs_grad, through the C ABI: same loss and gradient on two calls
in a row (the second with fewer samples, after the first left its partial
gradients in the library's fixed scratch array), and sizes beyond the array
rejected."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    from paper_2403_05443_amd import lbell
    lbell.load()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lbell


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def test_grad_noalloc_matches_lbs_grad(lb):
    import torch
    from paper_2403_05443_amd import workloads
    lib = lb.load()
    dev = torch.device("cuda:0")
    params = workloads.xavier_params(workloads.SplitMix64(2403054430 + 71)).astype(np.float32)
    rng = np.random.default_rng(5)
    sur = lb.Surrogate(max_samples=4096, params=params)
    P = torch.from_numpy(params).to(dev)
    stream = torch.cuda.current_stream(dev)
    for n in (3000, 37):   # the second call: smaller, over the first call's scratch contents
        X = rng.standard_normal((n, 8)).astype(np.float32)
        Y = rng.standard_normal((n, 6)).astype(np.float32)
        loss_ref, g_ref = sur.grad(X, Y)
        Xd, Yd = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
        g = torch.full((lb.Surrogate.N_PARAMS,), float("nan"), dtype=torch.float32, device=dev)
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device=dev)
        st = lib.lbs_grad_noalloc(_ptr(P), _ptr(Xd), _ptr(Yd), n, _ptr(g), _ptr(loss),
                                  C.c_void_p(stream.cuda_stream))
        assert st == 0
        torch.cuda.synchronize()
        # the same kernels and the same summation order: equal bit for bit
        assert np.array_equal(g.cpu().numpy(), g_ref), n
        assert loss.item() == loss_ref, n
        assert np.isfinite(g_ref).all() and loss_ref > 0


def test_grad_noalloc_rejects_sizes_beyond_its_scratch(lb):
    import torch
    lib = lb.load()
    dev = torch.device("cuda:0")
    n = 4097
    P = torch.zeros(lb.Surrogate.N_PARAMS, dtype=torch.float32, device=dev)
    X = torch.zeros((n, 8), dtype=torch.float32, device=dev)
    Y = torch.zeros((n, 6), dtype=torch.float32, device=dev)
    g = torch.zeros_like(P)
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    assert lib.lbs_grad_noalloc(_ptr(P), _ptr(X), _ptr(Y), n, _ptr(g), None, stream) == -1
    assert lib.lbs_grad_noalloc(_ptr(P), _ptr(X), _ptr(Y), 0, _ptr(g), None, stream) == -1
    assert lib.lbs_grad_noalloc(None, _ptr(X), _ptr(Y), 16, _ptr(g), None, stream) == -1
