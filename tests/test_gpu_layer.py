"""GPU parity of the circulant layer (forward with a shared row, hand-written backward)
against FP64 references: dense autograd and finite differences at n = 64, the DFT-identity
oracle at the full size (batch 256, n = 2^14)."""
import numpy as np
import pytest

from oracle import grad as OG
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


def rel(got, want):
    return np.linalg.norm(got - want) / np.linalg.norm(want)


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available()
    return fcirc


def test_real_n64_against_dense_autograd_and_finite_differences(F):
    import torch
    rng = np.random.default_rng(64)
    n, batch = 64, 5
    a = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal((batch, n)).astype(np.float32)
    g = rng.standard_normal((batch, n)).astype(np.float32)
    ta = torch.from_numpy(a).cuda().requires_grad_(True)
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    y = F.circulant(ta, tx)
    y.backward(torch.from_numpy(g).cuda())
    y_ref, ga_ref, gx_ref = OG.dense_autograd(a.astype(np.float64), x.astype(np.float64), g.astype(np.float64))
    fa, fx = OG.finite_differences(a, x, g)
    assert rel(y.detach().cpu().numpy(), y_ref) <= TOL
    assert rel(ta.grad.cpu().numpy(), ga_ref) <= TOL
    assert rel(tx.grad.cpu().numpy(), gx_ref) <= TOL
    assert rel(ta.grad.cpu().numpy(), fa) <= TOL
    assert rel(tx.grad.cpu().numpy(), fx) <= TOL


@pytest.mark.parametrize("n,batch", [(16, 1), (64, 3), (1024, 7), (1 << 13, 4), (1 << 14, 33), (1 << 14, 64), (1 << 16, 2), (1 << 21, 1),
                                     # grad_a by 13-level accumulating blocks: no top split at 2^13
                                     # (512 complex instances), one top level at 2^14 (256)
                                     (1 << 13, 512), (1 << 14, 256),
                                     # 11 top levels: two top passes (5 + 6 levels) in every product
                                     (1 << 24, 1)])
def test_complex_layer(F, n, batch):
    import torch
    rng = np.random.default_rng(n + batch)
    c = lambda *s: (rng.standard_normal(s) + 1j * rng.standard_normal(s)).astype(np.complex64)
    a, x, g = c(n), c(batch, n), c(batch, n)
    ta = torch.from_numpy(a).cuda().requires_grad_(True)
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    y = F.circulant(ta, tx)
    y.backward(torch.from_numpy(g).cuda())
    y_ref, ga_ref, gx_ref = OG.grads_fft(a.astype(np.complex128), x.astype(np.complex128), g.astype(np.complex128))
    if n <= 64:
        y_d, ga_d, gx_d = OG.dense_autograd(a.astype(np.complex128), x.astype(np.complex128), g.astype(np.complex128))
        np.testing.assert_allclose(ga_ref, ga_d, rtol=1e-9, atol=1e-9)
    assert rel(y.detach().cpu().numpy(), y_ref) <= TOL
    assert rel(ta.grad.cpu().numpy(), ga_ref) <= TOL
    assert rel(tx.grad.cpu().numpy(), gx_ref) <= TOL


@pytest.mark.parametrize("batch", [1, 2, 3, 8])
def test_real_odd_batches(F, batch):
    import torch
    rng = np.random.default_rng(batch)
    n = 256
    a = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal((batch, n)).astype(np.float32)
    g = rng.standard_normal((batch, n)).astype(np.float32)
    y = F.layer_forward(torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
    ga, gx = F.layer_backward(torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda())
    y_ref, ga_ref, gx_ref = OG.grads_fft(a.astype(np.float64), x.astype(np.float64), g.astype(np.float64))
    assert rel(y, y_ref) <= TOL
    assert rel(ga.cpu().numpy(), ga_ref) <= TOL
    assert rel(gx.cpu().numpy(), gx_ref) <= TOL


def test_real_13_level_accumulation(F):
    """Real batch of 1024 at n = 2^13: 512 packed pairs, enough for 13-level accumulating
    blocks; packed pairs take one top level and 12-level blocks there instead (the 13-level
    pass reading pairs directly would spill registers)."""
    import torch
    rng = np.random.default_rng(13)
    n, batch = 1 << 13, 1024
    a = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal((batch, n)).astype(np.float32)
    g = rng.standard_normal((batch, n)).astype(np.float32)
    ga, gx = F.layer_backward(torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda())
    _, ga_ref, gx_ref = OG.grads_fft(a.astype(np.float64), x.astype(np.float64), g.astype(np.float64))
    assert rel(ga.cpu().numpy(), ga_ref) <= TOL
    assert rel(gx.cpu().numpy(), gx_ref) <= TOL


def test_c5_config(F):
    """Batch 256 of x in R^(2^14), shared a, float32 N(0,1), upstream gradient N(0,1)."""
    import torch
    a, x, g = W.circ_layer_f32()
    ta = torch.from_numpy(a).cuda().requires_grad_(True)
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    y = F.circulant(ta, tx)
    y.backward(torch.from_numpy(g).cuda())
    y_ref, ga_ref, gx_ref = OG.grads_fft(a.astype(np.float64), x.astype(np.float64), g.astype(np.float64))
    assert rel(y.detach().cpu().numpy(), y_ref) <= TOL
    assert rel(ta.grad.cpu().numpy(), ga_ref) <= TOL
    assert rel(tx.grad.cpu().numpy(), gx_ref) <= TOL
    # per-row accuracy of the forward and grad_x as well
    yh = y.detach().cpu().numpy()
    gxh = tx.grad.cpu().numpy()
    assert max(rel(yh[b], y_ref[b]) for b in range(256)) <= TOL
    assert max(rel(gxh[b], gx_ref[b]) for b in range(256)) <= TOL
