"""GPU parity of the product over Z/(2^K + 1) (section 3.2's ring: roots are shifts) against
the CPU oracle, bit for bit, and of the large-integer product by that route against
Python's integer product."""
import random

import numpy as np
import pytest

from oracle import fermat as OF

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return fcirc


def to_words(vals, K):
    """Python ints in [0, 2^K] -> (n, K/32 + 1) uint32 element array."""
    W = K // 32
    out = np.zeros((len(vals), W + 1), dtype=np.uint32)
    for i, v in enumerate(vals):
        v = int(v)
        if v == 1 << K:
            out[i, W] = 1
        else:
            out[i, :W] = np.frombuffer(v.to_bytes(4 * W, "little"), dtype=np.uint32)
    return out


def from_words(arr, K):
    W = K // 32
    return [int.from_bytes(row[:W].astype(np.uint32).tobytes(), "little") + (int(row[W]) << K) for row in arr]


def dev(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.int32)).cuda()


def rand_elems(n, K, rng, edge=True):
    M = OF.modulus(K)
    vals = [rng.randrange(M) for _ in range(n)]
    if edge and n >= 4:
        vals[0], vals[1], vals[2], vals[3] = 1 << K, 0, (1 << K) - 1, 1
    return vals


def run(F, a, x, K, f_shift):
    y = F.fermat_matvec(dev(to_words(a, K)), dev(to_words(x, K)), K, f_shift)
    return from_words(y.cpu().numpy().view(np.uint32), K)


@pytest.mark.parametrize("K", [2048, 4096, 8192, 16384])
@pytest.mark.parametrize("n", [1, 2, 4, 8, 32])
def test_fermat_small_against_definition(F, K, n):
    rng = random.Random(K + n)
    a, x = rand_elems(n, K, rng), rand_elems(n, K, rng)
    M = OF.modulus(K)
    for f_shift in sorted({0, K, (2 * n * 3) % (2 * K)}):
        want = OF.dense_matvec(a, x, pow(2, f_shift, M), K) if n <= 8 else OF.levels_matvec(a, x, f_shift, K)
        assert run(F, a, x, K, f_shift) == want, (K, n, f_shift)


@pytest.mark.parametrize("K,L", [(2048, 10), (2048, 12), (4096, 11), (8192, 9), (16384, 7)])
def test_fermat_larger_against_levels(F, K, L):
    n = 1 << L
    rng = random.Random(7 * K + L)
    a, x = rand_elems(n, K, rng), rand_elems(n, K, rng)
    for f_shift in (0, K):
        if f_shift % n:  # -1 = 2^K has no power-of-two n-th root unless n | K
            from paper_2103_02605_amd._lib import FcircError
            with pytest.raises(FcircError, match="ENOROOT"):
                run(F, a, x, K, f_shift)
            with pytest.raises(ValueError):
                OF.node_exponents(L, f_shift, K)
            continue
        assert run(F, a, x, K, f_shift) == OF.levels_matvec(a, x, f_shift, K), (K, L, f_shift)


def test_fermat_edge_values(F):
    """Every element 2^K (= -1), 0, 2^K - 1 and 1: the special top word through shifts,
    sums, differences and products."""
    K, n = 2048, 16
    M = OF.modulus(K)
    for av, xv in ((1 << K, 1 << K), ((1 << K) - 1, (1 << K) - 1), (0, 1 << K), (1, (1 << K) - 1)):
        a, x = [av] * n, [xv] * n
        for f_shift in (0, K):
            assert run(F, a, x, K, f_shift) == OF.dense_matvec(a, x, pow(2, f_shift, M), K), (av, xv, f_shift)


def test_fermat_errors(F):
    from paper_2103_02605_amd._lib import FcircError
    K = 2048
    a = dev(to_words([1] * 8, K))
    with pytest.raises(FcircError, match="ENOROOT"):
        F.fermat_matvec(a, a.clone(), K, 4)  # 8 does not divide 4
    with pytest.raises(FcircError, match="EINVAL"):
        F.fermat_matvec(a, a.clone(), K, 2 * K)
    big = dev(np.zeros((1 << 13, K // 32 + 1), dtype=np.uint32))
    with pytest.raises(FcircError, match="ESIZE"):
        F.fermat_matvec(big, big.clone(), K, 0)  # 2^12 does not divide 2048
    import torch
    with pytest.raises(ValueError):
        F.fermat_matvec(a, a.clone(), 4096, 0)
    bad = torch.zeros((8, 3000 // 32 + 1), dtype=torch.int32, device="cuda")
    from paper_2103_02605_amd import _lib
    import ctypes as C
    ctx = F.context(bad.device)
    assert _lib.lib().fcirc_fermat_matvec(ctx.handle, C.c_void_p(bad.data_ptr()), C.c_void_p(bad.data_ptr()),
                                          C.c_void_p(bad.data_ptr() + 4096), 8, 3000, 0, None) == 1  # EINVAL


def limbs_of(v, nl):
    return np.frombuffer(v.to_bytes(2 * nl, "little"), dtype=np.uint16).copy()


def int_of(limbs):
    return int.from_bytes(np.ascontiguousarray(limbs).astype(np.uint16).tobytes(), "little")


def bigint_gpu(F, u_limbs, v_limbs):
    import torch
    a = torch.from_numpy(u_limbs.view(np.int16)).cuda()
    b = torch.from_numpy(v_limbs.view(np.int16)).cuda()
    return F.bigint_mul_fermat(a, b).cpu().numpy().view(np.uint16)


@pytest.mark.parametrize("na,nb", [(1, 1), (3, 5), (64, 64), (1000, 37), (4096, 4095), (30000, 70001), (1 << 17, 1 << 17)])
def test_bigint_fermat_against_python(F, na, nb):
    rng = random.Random(na * 31 + nb)
    u, v = rng.getrandbits(16 * na), rng.getrandbits(16 * nb)
    got = bigint_gpu(F, limbs_of(u, na), limbs_of(v, nb))
    assert got.shape[0] == na + nb
    assert int_of(got) == u * v


def test_bigint_fermat_all_ones_and_c3_size(F):
    """All-ones factors (every piece at its maximum, the largest coefficients), then the
    C3 size: two 2^24-bit integers, against Python's product and the NTT route."""
    import torch
    na = 1 << 12
    top = (1 << (16 * na)) - 1
    assert int_of(bigint_gpu(F, limbs_of(top, na), limbs_of(top, na))) == top * top
    na = nb = 1 << 20
    rng = np.random.default_rng(5)
    ua = rng.integers(0, 1 << 16, na, dtype=np.uint16)
    vb = rng.integers(0, 1 << 16, nb, dtype=np.uint16)
    got = bigint_gpu(F, ua, vb)
    assert int_of(got) == int_of(ua) * int_of(vb)
    ntt = F.bigint_mul(torch.from_numpy(ua.view(np.int16)).cuda(), torch.from_numpy(vb.view(np.int16)).cuda())
    np.testing.assert_array_equal(ntt.cpu().numpy().view(np.uint16), got)


def test_fermat_max_size_sampled(F):
    """K = 16384 at its largest n = 2^15 (2^(L-1) | K): sampled entries of the definition."""
    K, n = 16384, 1 << 15
    rng = random.Random(99)
    a, x = rand_elems(n, K, rng), rand_elems(n, K, rng)
    y = run(F, a, x, K, 0)
    for i in (0, n - 1, 12345):
        assert y[i] == OF.matvec_entry(a, x, 1, K, i), i


def test_fermat_input_check(F):
    """With the input check on, a non-canonical element (top word 2, or top word 1 with a
    nonzero word) is refused with EINVAL and nothing is written; canonical ones pass."""
    import torch
    from paper_2103_02605_amd._lib import FcircError
    K, n = 4096, 16
    rng = random.Random(5)
    a, x = rand_elems(n, K, rng), rand_elems(n, K, rng)
    good_a, good_x = to_words(a, K), to_words(x, K)
    want = OF.levels_matvec(a, x, 0, K)
    F.set_checks(F.CHECK_INPUTS)
    try:
        assert from_words(F.fermat_matvec(dev(good_a), dev(good_x), K, 0).cpu().numpy().view(np.uint32), K) == want
        for bad_k, top, word in ((3, 2, None), (9, 1, 17)):
            bad = good_x.copy()
            bad[bad_k, K // 32] = top
            if word is not None:
                bad[bad_k, word] = 5
            y = torch.full((n, K // 32 + 1), 7, dtype=torch.int32, device="cuda")
            with pytest.raises(FcircError, match="EINVAL"):
                F.fermat_matvec(dev(good_a), dev(bad), K, 0, out=y)
            assert (y.cpu().numpy() == 7).all()
    finally:
        F.set_checks(0)
