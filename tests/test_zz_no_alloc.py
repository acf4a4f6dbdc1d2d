"""The allocation-free gradient entry point (crkdg_mlp_grad_noalloc) against
crkdg_mlp_grad, through the C ABI: two calls in a row, the second with a
smaller batch, each bit-identical to the entry point with caller work
memory (same kernels, same reduction order); the batch limit is enforced."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2307_06471_amd import crkdg
    return crkdg


def test_noalloc_gradient_equals_the_work_memory_entry_point(K):
    import torch
    rng = np.random.default_rng(11)
    P = torch.from_numpy((0.3 * rng.standard_normal(1505)).astype(np.float32)).cuda()
    for B in (K.MLP_NOALLOC_MAX_B, 1000):  # the largest batch, then a smaller ragged one
        X = torch.from_numpy(rng.standard_normal((B, 12)).astype(np.float32)).cuda()
        y = torch.from_numpy((rng.random(B) < 0.25).astype(np.uint8)).cuda()
        g_ref, l_ref = K.crkdg_mlp_grad(P, X, y, 2.5)
        g = torch.full((1505,), float("nan"), device="cuda")
        l = torch.full((1,), float("nan"), device="cuda")
        K.crkdg_mlp_grad_noalloc(P, X, y, 2.5, g, l)
        torch.cuda.synchronize()
        print(f"[noalloc] B={B} max|dg|={float((g - g_ref).abs().max()):.3g}", flush=True)
        assert torch.equal(g, g_ref) and torch.equal(l, l_ref), B


def test_noalloc_rejects_batches_beyond_its_buffer(K):
    import torch
    lib = K.lib()
    B = K.MLP_NOALLOC_MAX_B + 1
    X = torch.zeros((B, 12), dtype=torch.float32, device="cuda")
    y = torch.zeros(B, dtype=torch.uint8, device="cuda")
    P = torch.zeros(1505, dtype=torch.float32, device="cuda")
    g = torch.zeros(1505, dtype=torch.float32, device="cuda")
    ptr = lambda t: C.c_void_p(t.data_ptr())
    rc = lib.crkdg_mlp_grad_noalloc(ptr(P), ptr(X), ptr(y), B, 1.0, ptr(g), None, None)
    assert rc == K.CRKDG_EINVAL
    rc = lib.crkdg_mlp_grad_noalloc(ptr(P), ptr(X), ptr(y), 0, 1.0, ptr(g), None, None)
    assert rc == K.CRKDG_EINVAL
