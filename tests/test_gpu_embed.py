"""GPU parity of the products of any size (Corollary 1) and of Toeplitz products, both
through one power-of-two cyclic product, against the CPU oracle.

Z/p results must be bit-exact; complex and real FP32 results within relative L2 error
1e-5 of the FP64 oracle on the same FP32 inputs.
"""
import numpy as np
import pytest

from oracle import embed as OE
from oracle import fcirc as O
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu

PRIMES = (W.P1, W.P2, W.P3)
TOL = 1e-5


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield fcirc


def dev(arr):
    import torch
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.int64)


def rel(got, want):
    return float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-30))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 100, 1000, 4096, 4097, 65537, 300001])
def test_fcirc_any_n_modp(F, n):
    rng = np.random.default_rng(31 + n)
    for p in PRIMES:
        a = rng.integers(0, p, n, dtype=np.uint32)
        x = rng.integers(0, p, n, dtype=np.uint32)
        for f in (1, p - 1, int(rng.integers(2, p)), 0):
            got = host_u32(F.matvec_any(dev(a), dev(x), f=f, p=p))
            if n <= 2048:
                want = OE.toeplitz_matvec_dense(a, OE.fcirc_col(list(a.astype(np.int64)), f, p), x, p)
                np.testing.assert_array_equal(got, want, err_msg=f"p={p} f={f}")
            elif p == PRIMES[0] and f in (1, 0):
                np.testing.assert_array_equal(got, OE.fcirc_any_matvec_modp(a, x, f, p), err_msg=f"f={f}")
            else:  # sampled outputs from the dense definition
                for i in (0, 1, n // 2, n - 1):
                    assert got[i] == O.matvec_entry_modp(a, x, f, p, i), (p, f, i)


def test_fcirc_any_power_of_two_f_without_root(F):
    """A power-of-two n whose f has no square root in Z/p falls back to the embedding."""
    p = W.P1
    n = 1024
    rng = np.random.default_rng(5)
    a = rng.integers(0, p, n, dtype=np.uint32)
    x = rng.integers(0, p, n, dtype=np.uint32)
    f = 3  # a primitive root: no square root in Z/p
    got = host_u32(F.matvec_any(dev(a), dev(x), f=f, p=p))
    np.testing.assert_array_equal(got, O.dense_matvec_modp(a, x, f, p))


@pytest.mark.parametrize("n", [1, 3, 100, 5000, 100003])
def test_fcirc_any_n_complex(F, n):
    rng = np.random.default_rng(77 + n)
    c = lambda: (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    a, x = c(), c()
    for f in (1.0, 1j, np.exp(0.3j), 0.5 - 2j):
        got = F.matvec_any(dev(a), dev(x), f=f).cpu().numpy()
        want = OE.fcirc_any_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), f)
        assert rel(got, want) <= TOL, (f, rel(got, want))


@pytest.mark.parametrize("n", [7, 1000, 9999])
def test_fcirc_any_n_real(F, n):
    rng = np.random.default_rng(5 + n)
    a = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    for f in (1.0, -1.0, 0.25):
        got = F.matvec_any(dev(a), dev(x), f=f).cpu().numpy()
        want = OE.fcirc_any_matvec_c128(a.astype(np.float64), x.astype(np.float64), f).real
        assert rel(got, want) <= TOL, (f, rel(got, want))


@pytest.mark.parametrize("n", [1, 2, 6, 257, 3000, 70000])
def test_toeplitz(F, n):
    rng = np.random.default_rng(900 + n)
    for p in PRIMES:
        row = rng.integers(0, p, n, dtype=np.uint32)
        col = rng.integers(0, p, n, dtype=np.uint32)
        x = rng.integers(0, p, n, dtype=np.uint32)
        got = host_u32(F.toeplitz_matvec(dev(row), dev(col), dev(x), p=p))
        if n <= 3000:
            np.testing.assert_array_equal(got, OE.toeplitz_matvec_dense(row, col, x, p))
        else:
            np.testing.assert_array_equal(got, OE.toeplitz_matvec_modp(row, col, x, p))
    c = lambda: (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    row, col, x = c(), c(), c()
    got = F.toeplitz_matvec(dev(row), dev(col), dev(x)).cpu().numpy()
    want = OE.toeplitz_matvec_c128(row.astype(np.complex128), col.astype(np.complex128), x.astype(np.complex128))
    assert rel(got, want) <= TOL


def test_embed_errors(F):
    import torch
    from paper_2103_02605_amd._lib import FcircError
    p = W.P1
    a = dev(np.ones(5, dtype=np.uint32))
    with pytest.raises(FcircError, match="EINVAL"):
        F.matvec_any(a, a, f=1, p=p, out=a)  # output aliases the input
    with pytest.raises(FcircError, match="EINVAL"):
        F.toeplitz_matvec(a, a, dev(np.ones(5, dtype=np.uint32)), p=p, out=a)
    big = torch.zeros((1 << 22) + 1, dtype=torch.int32, device="cuda")  # N = 2^24 > 2^23
    with pytest.raises(FcircError, match="ESIZE"):
        F.matvec_any(big, big, f=1, p=p)


def test_largest_embedding_sampled(F):
    """n = 2^22 - 1 over Z/998244353: the embedded cyclic length is 2^23, the prime's limit.
    Sampled entries of the f-circulant (f = 3, no 2^22-th root needed) and Toeplitz
    definitions; one more element (N = 2^24) is refused."""
    from paper_2103_02605_amd._lib import FcircError
    p = W.P1
    n = (1 << 22) - 1
    rng = np.random.default_rng(23)
    a, x, col = (rng.integers(0, p, n, dtype=np.uint32) for _ in range(3))
    y = host_u32(F.matvec_any(dev(a), dev(x), f=3, p=p))
    t = host_u32(F.toeplitz_matvec(dev(a), dev(col), dev(x), p=p))
    for i in (0, 1, n // 2, n - 1, 3141592):
        assert y[i] == O.matvec_entry_modp(a, x, 3, p, i), i
        assert t[i] == OE.toeplitz_entry_modp(a, col, x, p, i), i
    big = dev(np.zeros((1 << 22) + 1, dtype=np.uint32))
    with pytest.raises(FcircError, match="ESIZE"):
        F.matvec_any(big, big.clone(), f=3, p=p)
