"""Repeated products over rotating buffers, as a serving loop or the benchmark runs them.

The passes of a product hand their outputs to the next pass through memory written with
streaming (non-temporal) and agent-scope stores. These tests run many products back to
back over several input and output buffers, with unrelated torch work (FFTs, elementwise
kernels) in between, and check every output: Z/p products bit-exact against the oracle's
level form of Algorithm 1, complex64 products bit-identical to the first product of the
same inputs, which itself lies within 1e-5 of an FP64 FFT evaluation of the definition
(Definition 2 with f = 1: a cyclic correlation).
"""
import numpy as np
import pytest

from oracle import fcirc as O
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fcirc.set_split(-1)
    return fcirc


def dev(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.int32)).cuda()


def test_rotating_buffers_bit_exact(F):
    import torch
    p = W.P1
    L = 21
    n = 1 << L
    fs = [1, 1, p - 1, 1]  # one negacyclic set: its tables are built between the others
    sets = []
    for k, f in enumerate(fs):
        a, x = W.modp_pair(n, p, seed=W.SEED_HEADLINE + 1000 * k)
        want = O.levels_matvec_modp(a, x, f, p).astype(np.uint32)
        sets.append((dev(a), dev(x), f, want))
    outs = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in range(3)]
    ca, cx = W.complex_pair(n, seed=W.SEED_HEADLINE)
    tca, tcx = torch.from_numpy(ca).cuda(), torch.from_numpy(cx).cuda()
    cy0 = F.matvec(tca, tcx)
    cy = torch.empty_like(cy0)
    noise = torch.randn(n, dtype=torch.complex64, device="cuda")
    got = []
    for r in range(12):
        a, x, f, _ = sets[r % 4]
        y = outs[r % 3]
        F.matvec(a, x, f=f, p=p, out=y)
        got.append((r % 4, y.clone()))
        F.matvec(tca, tcx, out=cy)  # another ring's tables and workspace in between
        assert torch.equal(cy, cy0), f"complex product changed at repeat {r}"
        noise = torch.fft.ifft(torch.fft.fft(noise) * 0.5) + 1.0  # unrelated device work
    torch.cuda.synchronize()
    for r, (k, y) in enumerate(got):
        np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32), sets[k][3], err_msg=f"repeat {r}, set {k}")
    # the complex product itself against the definition (cyclic correlation via FP64 FFT)
    idx = (-np.arange(n)) % n
    yd = np.fft.ifft(np.fft.fft(ca.astype(np.complex128)[idx]) * np.fft.fft(cx.astype(np.complex128)))
    rel = np.linalg.norm(cy0.cpu().numpy() - yd) / np.linalg.norm(yd)
    assert rel < 1e-5, rel
