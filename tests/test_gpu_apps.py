"""GPU parity of the applications (section 3): exact integer polynomial products and
large-integer products, bit-exact against the CPU oracle."""
import numpy as np
import pytest

from oracle import bigint as OB
from oracle import polymul as OP
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu
PRIMES = (W.P1, W.P2, W.P3)


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available()
    fcirc.set_split(-1)
    return fcirc


def d(arr):
    import torch
    arr = np.ascontiguousarray(arr)
    if arr.dtype == np.uint16:
        arr = arr.view(np.int16)
    return torch.from_numpy(arr).cuda()


@pytest.mark.parametrize("na,nb", [(1, 1), (1, 7), (5, 3), (100, 37), (1000, 1000), (4096, 4096), (3000, 70000),
                                   (1, 1 << 16)])
def test_polymul_small(F, na, nb):
    rng = np.random.default_rng(na * 31 + nb)
    a = rng.integers(-(1 << 15), 1 << 15, na).astype(np.int32)
    b = rng.integers(-(1 << 15), 1 << 15, nb).astype(np.int32)
    got = F.polymul_i64(d(a), d(b)).cpu().numpy()
    want = OP.poly_kronecker(a, b) if na * nb > 10**6 else np.array(OP.poly_schoolbook(a, b), dtype=np.int64)
    np.testing.assert_array_equal(got, want)
    F.check()


@pytest.mark.parametrize("L", list(range(1, 15)))
def test_polymul_bigint_every_size(F, L):
    """Factors of 2^(L-1) coefficients (limbs), so that the three-prime products have
    exactly 2^L elements: every schedule form of the product (small-product kernel, block
    pass, top passes) meets the row-reversing and padding loaders."""
    m = 1 << (L - 1)
    rng = np.random.default_rng(1000 + L)
    a = rng.integers(-(1 << 15), 1 << 15, m).astype(np.int32)
    b = rng.integers(-(1 << 15), 1 << 15, m).astype(np.int32)
    want = OP.poly_kronecker(a, b) if m * m > 10**6 else np.array(OP.poly_schoolbook(a, b), dtype=np.int64)
    np.testing.assert_array_equal(F.polymul_i64(d(a), d(b)).cpu().numpy(), want)
    ua = rng.integers(0, 1 << 16, m).astype(np.uint16)
    ub = rng.integers(0, 1 << 16, m).astype(np.uint16)
    np.testing.assert_array_equal(F.bigint_mul(d(ua), d(ub)).cpu().numpy().view(np.uint16), OB.bigint_mul_pyint(ua, ub))
    F.check()


def test_polymul_full_config(F):
    """2 x 2^20 int32 coefficients in [-2^15, 2^15) (seed 4): every coefficient against the
    oracle's three circulant products and textbook CRT."""
    a, b = W.poly_i32(1 << 20, W.SEED_POLY)
    got = F.polymul_i64(d(a), d(b)).cpu().numpy()
    F.check()
    want = np.array(OP.poly_via_circulant(a, b, PRIMES), dtype=np.int64)
    np.testing.assert_array_equal(got, want)


def test_polymul_extremes_in_range(F):
    a = np.array([2**31 - 1, -(2**31), 7], dtype=np.int32)
    b = np.array([1 << 26, -(1 << 26)], dtype=np.int32)  # |c_1| = 2^58 - 2^26 < p1 p2 ~ 2^58.7
    got = F.polymul_i64(d(a), d(b)).cpu().numpy()
    F.check()
    np.testing.assert_array_equal(got, np.array(OP.poly_schoolbook(a, b), dtype=np.int64))


def test_polymul_out_of_range_flag(F):
    from paper_2103_02605_amd._lib import FcircError
    a = np.array([2**31 - 1, -(2**31), 7], dtype=np.int32)
    b = np.array([1 << 27, -(1 << 27)], dtype=np.int32)  # |c_1| ~ 2^59 > p1 p2
    got = F.polymul_i64(d(a), d(b)).cpu().numpy()
    with pytest.raises(FcircError, match="ERANGE"):
        F.check()
    want = np.array(OP.poly_schoolbook(a, b), dtype=object)
    inrange = np.abs(want) < W.P1 * W.P2
    assert (got[~inrange] == 0).all() and (got[inrange] == want[inrange].astype(np.int64)).all()
    a = np.full(4, -(2**31), dtype=np.int32)
    got = F.polymul_i64(d(a), d(a)).cpu().numpy()
    with pytest.raises(FcircError, match="ERANGE"):
        F.check()
    assert (got == 0).all()
    F.check()  # the sticky status was cleared


@pytest.mark.parametrize("na,nb", [(1, 1), (2, 3), (64, 64), (1000, 333), (4096, 4096), (1 << 14, 5), (1 << 15, 1 << 15)])
def test_bigint_small(F, na, nb):
    rng = np.random.default_rng(na + 7 * nb)
    a = rng.integers(0, 1 << 16, na).astype(np.uint16)
    b = rng.integers(0, 1 << 16, nb).astype(np.uint16)
    got = F.bigint_mul(d(a), d(b)).cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got, OB.bigint_mul_pyint(a, b))


@pytest.mark.parametrize("n", [1, 3, 4096, 5000, 1 << 16, 1 << 18])
def test_bigint_carry_chains(F, n):
    """All-ones limbs give the longest carry chains; (2^k - 1)^2 = 2^2k - 2^(k+1) + 1."""
    a = np.full(n, 0xFFFF, dtype=np.uint16)
    got = F.bigint_mul(d(a), d(a)).cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got, OB.bigint_mul_pyint(a, a))
    one = np.zeros(n, dtype=np.uint16)
    one[0] = 1
    got = F.bigint_mul(d(a), d(one)).cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got[:n], a)
    assert (got[n:] == 0).all()


def test_bigint_full_config(F):
    """Two 2^24-bit integers (2^20 uniform limbs, seed 5) against Python's integer multiply."""
    a, b = W.bigint_u16(1 << 20, W.SEED_BIGINT)
    got = F.bigint_mul(d(a), d(b)).cpu().numpy().view(np.uint16)
    F.check()
    np.testing.assert_array_equal(got, OB.bigint_mul_pyint(a, b))


def test_polymul_max_size_sampled(F):
    """na = nb = 2^22: 2^23 - 1 coefficients, the largest cyclic length of the first prime;
    sampled coefficients from the O(n) definition."""
    import torch
    from oracle import polymul as OP
    na = nb = 1 << 22
    rng = np.random.default_rng(41)
    a = rng.integers(-(1 << 15), 1 << 15, na, dtype=np.int32)
    b = rng.integers(-(1 << 15), 1 << 15, nb, dtype=np.int32)
    c = F.polymul_i64(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()).cpu().numpy()
    F.check()
    nc = na + nb - 1
    for k in [0, 1, nc // 2, nc - 2, nc - 1] + [int(v) for v in rng.integers(0, nc, 5)]:
        assert int(c[k]) == OP.poly_coef(a, b, k), k


def test_bigint_max_size_both_routes(F):
    """na + nb - 1 = 2^23 - 1 limbs with min(na, nb) = 2^20: the three-prime route at its
    limit, and section 3.2's route on the same factors, against Python's product."""
    import torch
    na, nb = 1 << 20, (1 << 23) - (1 << 20)
    rng = np.random.default_rng(42)
    ua = rng.integers(0, 1 << 16, na, dtype=np.uint16)
    vb = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
    want = int.from_bytes(ua.tobytes(), "little") * int.from_bytes(vb.tobytes(), "little")
    ta, tb = torch.from_numpy(ua.view(np.int16)).cuda(), torch.from_numpy(vb.view(np.int16)).cuda()
    for fn in (F.bigint_mul, F.bigint_mul_fermat):
        got = fn(ta, tb).cpu().numpy().view(np.uint16)
        assert int.from_bytes(got.tobytes(), "little") == want, fn.__name__
