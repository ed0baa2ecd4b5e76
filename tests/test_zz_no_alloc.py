"""The allocation-free gradient entry point (pf_mlp_loss_grad_noalloc)
against the entry point with a caller-owned work buffer (pf_mlp_loss_grad):
two calls in a row, the second with fewer rows, each bit-identical to the
work-buffer call (same launch shape, same fixed-order reduction) and within
the gradient tolerance of the FP64 oracle at the bfloat16-rounded parameters
(relative L2 below 1e-2, cosine above 0.999: the GPU rounds hidden
activations and layer errors to bfloat16)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def pf(torch_mod):
    import paper_1407_8071_amd as pf
    pf.lib()
    return pf


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _params(orc, rng, in_dim, out_dim):
    p = np.zeros(orc.mlp_nparams(in_dim, out_dim))
    W1, b1, W2, b2, W3, b3 = orc.mlp_unpack(p, in_dim, out_dim)
    W1[:] = rng.standard_normal(W1.shape) * np.sqrt(2 / in_dim)
    W2[:] = rng.standard_normal(W2.shape) * np.sqrt(2 / 64)
    W3[:] = rng.standard_normal(W3.shape) * np.sqrt(1 / 64)
    b1[:] = rng.standard_normal(64) * 0.05
    b2[:] = rng.standard_normal(64) * 0.05
    b3[:] = rng.standard_normal(out_dim) * 0.05
    return p.astype(np.float32).astype(np.float64)


def test_noalloc_gradient_equals_work_buffer_gradient(pf, orc, torch_mod):
    torch = torch_mod
    in_dim, out_dim = 22, 2
    rng = np.random.default_rng(2024)
    p = _params(orc, rng, in_dim, out_dim)
    pd = _dev(p)
    n = pf.mlp_nparams(in_dim, out_dim)
    # the larger call first (near the static buffer's row limit for this
    # network), then a smaller one whose partials cover only part of what
    # the first call left in the buffer
    for rows in (46000, 1000):
        print(f"noalloc gradient: in_dim {in_dim} out_dim {out_dim} rows {rows}", flush=True)
        X = orc.bf16(rng.standard_normal((rows, in_dim)).astype(np.float32))
        T = rng.standard_normal((rows, out_dim)).astype(np.float32).astype(np.float64)
        Xd, Td = _dev(X), _dev(T)
        grad = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        pf.mlp_loss_grad_noalloc(pd, Xd, Td, grad, loss)
        ref_loss, ref_grad = pf.mlp_loss_grad(pd, Xd, Td)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        assert np.array_equal(g, ref_grad.cpu().numpy())
        assert loss.item() == ref_loss.item()
        rloss, rg = orc.mlp_loss_grad(orc.bf16(p), X, T)
        assert abs(loss.item() - rloss) <= 1e-2 * rloss
        g64 = g.astype(np.float64)
        rel = np.linalg.norm(g64 - rg) / np.linalg.norm(rg)
        cos = g64 @ rg / (np.linalg.norm(g64) * np.linalg.norm(rg))
        assert rel < 1e-2 and cos > 0.999, (rows, rel, cos)


def test_noalloc_rejects_rows_beyond_the_static_buffer(pf, torch_mod):
    import ctypes as C
    torch = torch_mod
    n = pf.mlp_nparams(22, 2)
    dummy = torch.zeros(16, dtype=torch.float32, device="cuda")
    ptr = C.c_void_p(dummy.data_ptr())
    st = pf.lib().pf_mlp_loss_grad_noalloc(ptr, 22, 2, ptr, ptr, 46337, ptr, None, None)
    assert st == 3
    assert "static buffer holds" in pf.lib().pf_last_error().decode()
    del n
