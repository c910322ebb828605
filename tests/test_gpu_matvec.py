"""GPU parity of the f-circulant product against the CPU oracle.

Z/p results must be bit-exact. Complex/real FP32 results must be within relative L2
error 1e-5 of the FP64 oracle evaluated on the same (FP32) inputs.
"""
import random

import numpy as np
import pytest

from oracle import fcirc as O
from oracle import gfp2 as OG
from paper_2103_02605_amd import _lib
from paper_2103_02605_amd import workloads as W

GP = OG.P  # 2^31 - 1, the ring of section 3.1

pytestmark = pytest.mark.gpu

P1, P2, P3 = W.P1, W.P2, W.P3
PRIMES = (P1, P2, P3)
TOL = 1e-5


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fcirc.set_split(-1)
    yield fcirc
    fcirc.set_split(-1)


def dev64(arr):
    """(n, 2) residues of Z/p[sqrt 3] as the int32 pairs the binding takes."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr.astype(np.int32))).cuda()


def dev(arr):
    import torch
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.int64)


def rand_f(n, p, seed):
    return pow(random.Random(seed).randrange(1, p), n, p)


def oracle_modp(a, x, f, p):
    n = len(a)
    if n <= 2048:
        return O.dense_matvec_modp(a, x, f, p)
    return O.levels_matvec_modp(a, x, f, p)


# C1: n = 1024 over Z/998244353, f = 1 (cyclic) and f = p - 1 (negacyclic), bit-exact -------

@pytest.mark.parametrize("f,seed", [(1, W.SEED_C1_CYCLIC), (P1 - 1, W.SEED_C1_NEGACYCLIC)])
def test_c1_n1024_bit_exact(F, f, seed):
    a, x = W.modp_pair(1024, P1, seed)
    y = F.matvec(dev(a), dev(x), f=f, p=P1)
    np.testing.assert_array_equal(host_u32(y), O.dense_matvec_modp(a, x, f, P1))


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("L", list(range(0, 15)))
def test_all_sizes_bit_exact(F, p, L):
    n = 1 << L
    a, x = W.modp_pair(n, p, seed=100 + L)
    for f in (1, p - 1, rand_f(n, p, L)):
        if f == p - 1 and L >= 23:
            continue
        y = F.matvec(dev(a), dev(x), f=f, p=p)
        np.testing.assert_array_equal(host_u32(y), oracle_modp(a, x, f, p), err_msg=f"p={p} n={n} f={f}")


@pytest.mark.parametrize("ring", ["p1", "p2", "p3", "c64", "r32", "gfp2"])
@pytest.mark.parametrize("L", list(range(6, 13)))
def test_small_kernel_and_block_pass(F, ring, L):
    """Products of 2^6..2^12 with no top pass run as the several-wave small-product kernel
    by default (FCIRC_SCHED_SMALL) and as the single-wave block pass otherwise; both
    against the oracle (bit-exact over Z/p for f = 1, p - 1 and a random f; complex within
    1e-5 of the FP64 definition), alone and as a batch of 3."""
    import torch
    n = 1 << L
    ring_id = {"p1": 0, "p2": 1, "p3": 2, "c64": 3, "r32": _lib.FCIRC_R32, "gfp2": _lib.FCIRC_GFP2}[ring]
    try:
        for flags in (F.SCHED_XCD | F.SCHED_SMALL, F.SCHED_XCD):
            F.set_schedule(n, ring_id, 0, -1, flags)
            if ring == "r32":
                rng = np.random.default_rng(600 + L)
                a = rng.standard_normal(n).astype(np.float32)
                x = rng.standard_normal(n).astype(np.float32)
                y = F.matvec(torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
                want = O.dense_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), 1.0).real
                assert np.linalg.norm(y - want) / np.linalg.norm(want) < 1e-5, (L, flags)
                continue
            if ring == "gfp2":
                a = np.random.default_rng(700 + L).integers(0, GP, (n, 2)).astype(np.uint64)
                x = np.random.default_rng(800 + L).integers(0, GP, (n, 2)).astype(np.uint64)
                y = F.matvec(dev64(a), dev64(x), f=1, p=GP).cpu().numpy().astype(np.uint64)
                np.testing.assert_array_equal(y, OG.levels_matvec(a, x, OG.ONE), err_msg=f"L={L} flags={flags}")
                continue
            if ring == "c64":
                a, x = W.complex_pair(n, seed=300 + L)
                y = F.matvec(torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda()).cpu().numpy()
                want = O.dense_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), 1.0)
                assert np.linalg.norm(y - want) / np.linalg.norm(want) < 1e-5, (L, flags)
                continue
            p = PRIMES[ring_id]
            a, x = W.modp_pair(n, p, seed=200 + L)
            for f in (1, p - 1, rand_f(n, p, 7 * L)):
                y = F.matvec(dev(a), dev(x), f=f, p=p)
                np.testing.assert_array_equal(host_u32(y), oracle_modp(a, x, f, p), err_msg=f"p={p} n={n} f={f} flags={flags}")
            am = np.stack([W.modp_pair(n, p, seed=400 + 10 * L + k)[0] for k in range(3)])
            xm = np.stack([W.modp_pair(n, p, seed=400 + 10 * L + k)[1] for k in range(3)])
            ym = F.matvec_many(dev(am), dev(xm), f=1, p=p).cpu().numpy().view(np.uint32).astype(np.int64)
            for k in range(3):
                np.testing.assert_array_equal(ym[k], oracle_modp(am[k], xm[k], 1, p), err_msg=f"batch row {k} flags={flags}")
    finally:
        F.set_schedule(n, ring_id, -1, -1, F.SCHED_XCD | F.SCHED_SMALL)


@pytest.mark.parametrize("count", [2, 300])
def test_block_twiddle_forms(F, count):
    """2^13-element block passes with at most one workgroup per CU and with more (300
    blocks on 256 CUs, two blocks resident per CU) bit-exact, on a batch of 2^13 products
    forced to one block pass."""
    L = 13
    n = 1 << L
    p = P1
    rows = [W.modp_pair(n, p, seed=500 + k) for k in range(count)]
    am = np.stack([r[0] for r in rows])
    xm = np.stack([r[1] for r in rows])
    F.set_schedule(n, 0, 0, -1, F.SCHED_XCD)
    try:
        ym = F.matvec_many(dev(am), dev(xm), f=p - 1, p=p).cpu().numpy().view(np.uint32).astype(np.int64)
    finally:
        F.set_schedule(n, 0, -1, -1, F.SCHED_XCD | F.SCHED_SMALL)
    for k in sorted({0, count // 2, count - 1}):
        np.testing.assert_array_equal(ym[k], O.levels_matvec_modp(am[k], xm[k], p - 1, p), err_msg=f"row {k}")


def test_zero_sizes(F):
    """Empty inputs through the C-ABI: n = 0 is ESIZE; an empty batch (count 0) enqueues
    nothing and returns OK; an empty factor (na = 0) or an empty layer batch is EINVAL."""
    import ctypes as C
    import torch
    from paper_2103_02605_amd import _lib
    lib, ctx = _lib.lib(), F.context(0).handle
    buf = torch.full((64,), 7, dtype=torch.int32, device="cuda")
    out = torch.full((64,), 7, dtype=torch.int32, device="cuda")
    p, q = C.c_void_p(buf.data_ptr()), C.c_void_p(out.data_ptr())
    one = C.c_uint32(1)
    OK, EINVAL, ESIZE = 0, 1, 2
    assert lib.fcirc_matvec(ctx, p, p, q, 0, C.byref(one), _lib.FCIRC_ZP_998244353, None) == ESIZE
    assert lib.fcirc_matvec_any(ctx, p, p, q, 0, C.byref(one), _lib.FCIRC_ZP_998244353, None) == ESIZE
    assert lib.fcirc_toeplitz_matvec(ctx, p, p, p, q, 0, _lib.FCIRC_ZP_998244353, None) == ESIZE
    assert lib.fcirc_fermat_matvec(ctx, p, p, q, 0, 2048, 0, None) == ESIZE
    assert lib.fcirc_matvec_many(ctx, p, p, q, 16, 0, C.byref(one), _lib.FCIRC_ZP_998244353, None) == OK
    assert lib.fcirc_matvec_many(ctx, None, p, q, 16, 0, C.byref(one), _lib.FCIRC_ZP_998244353, None) == EINVAL
    items = (_lib.fcirc_item * 1)()
    assert lib.fcirc_matvec_batched(ctx, p, p, q, items, 0, C.byref(one), _lib.FCIRC_ZP_998244353, None) == OK
    assert lib.fcirc_polymul_i64(ctx, p, 0, p, 4, q, None) == EINVAL
    assert lib.fcirc_bigint_mul(ctx, p, 4, p, 0, q, None) == EINVAL
    assert lib.fcirc_bigint_mul_fermat(ctx, p, 0, p, 0, q, None) == EINVAL
    assert lib.fcirc_matvec_fwd_shared(ctx, p, p, q, 16, 0, _lib.FCIRC_R32, None) == EINVAL
    assert lib.fcirc_matvec_backward(ctx, p, p, p, q, None, 16, 0, _lib.FCIRC_R32, None) == EINVAL
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == 7).all()  # nothing was written
    # through the binding: an empty batch gives an empty result
    y = F.matvec_many(torch.empty((0, 16), dtype=torch.int32, device="cuda"),
                      torch.empty((0, 16), dtype=torch.int32, device="cuda"), f=1, p=P1)
    assert y.shape == (0, 16)


@pytest.mark.parametrize("L,top", [(8, 2), (8, 7), (13, 1), (13, 9), (15, 3), (16, 12), (17, 14), (18, 5)])
def test_forced_splits_bit_exact(F, L, top):
    """Every split point of the recursion between HBM passes and the LDS block gives the
    same bits (covers one and two top passes, narrow and wide tiles)."""
    n = 1 << L
    a, x = W.modp_pair(n, P1, seed=7 + L)
    want = oracle_modp(a, x, 1, P1)
    F.set_split(top)
    try:
        y = F.matvec(dev(a), dev(x), f=1, p=P1)
    finally:
        F.set_split(-1)
    np.testing.assert_array_equal(host_u32(y), want)


def test_many_instances(F):
    import torch
    for L, count in [(0, 3), (5, 7), (10, 4), (14, 3)]:
        n = 1 << L
        a, x = W.modp_batch(count, n, P2, seed=L)
        y = F.matvec_many(dev(a), dev(x), f=P2 - 1, p=P2)
        got = host_u32(y)
        for k in range(count):
            np.testing.assert_array_equal(got[k], oracle_modp(a[k], x[k], P2 - 1, P2))


@pytest.mark.parametrize("p,L", [(P1, 21), (P1, 23), (P3, 25), (P2, 26)])
def test_large_sampled(F, p, L):
    """Full sizes up to each prime's limit: sampled outputs from the O(n) definition."""
    n = 1 << L
    a, x = W.modp_pair(n, p, seed=W.SEED_HEADLINE)
    y = host_u32(F.matvec(dev(a), dev(x), f=1, p=p))
    rng = np.random.default_rng(L)
    for i in list(rng.integers(0, n, 12)) + [0, n - 1]:
        assert y[i] == O.matvec_entry_modp(a, x, 1, p, int(i)), f"y[{i}]"
    assert y.max() < p


def test_headline_levels_oracle_full(F):
    """The n = 2^21 headline product against the level-by-level oracle, every element."""
    n = 1 << 21
    a, x = W.modp_pair(n, P1, seed=W.SEED_HEADLINE)
    y = host_u32(F.matvec(dev(a), dev(x), f=1, p=P1))
    np.testing.assert_array_equal(y, O.levels_matvec_modp(a, x, 1, P1))


def test_deterministic(F):
    n = 1 << 18
    a, x = W.modp_pair(n, P1, seed=9)
    y1 = host_u32(F.matvec(dev(a), dev(x), f=1, p=P1))
    y2 = host_u32(F.matvec(dev(a), dev(x), f=1, p=P1))
    np.testing.assert_array_equal(y1, y2)


# Complex FP32 ---------------------------------------------------------------------------

def rel_l2(got, want):
    return np.linalg.norm(got - want) / np.linalg.norm(want)


@pytest.mark.parametrize("L", list(range(0, 17)))
def test_complex_sizes(F, L):
    n = 1 << L
    a, x = W.complex_pair(n, seed=L)
    want = O.matvec_c128(a.astype(np.complex128), x.astype(np.complex128), 1.0)
    got = F.matvec(dev(a), dev(x)).cpu().numpy()
    assert rel_l2(got, want) <= TOL


@pytest.mark.parametrize("L", [18, 21, 24])
def test_complex_large(F, L):
    """Large complex products (f = 1) against the DFT identity in complex128."""
    n = 1 << L
    a, x = W.complex_pair(n, seed=L)
    want = O.cyclic_matvec_fft_c128(a.astype(np.complex128), x.astype(np.complex128))
    got = F.matvec(dev(a), dev(x)).cpu().numpy()
    assert rel_l2(got, want) <= TOL


def test_complex_and_real_large_negacyclic(F):
    n = 1 << 20
    a, x = W.complex_pair(n, seed=20)
    want = O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), -1.0)
    assert rel_l2(F.matvec(dev(a), dev(x), f=-1.0).cpu().numpy(), want) <= TOL
    ar, xr = a.real.copy(), x.real.copy()
    want = O.levels_matvec_c128(ar.astype(np.complex128), xr.astype(np.complex128), -1.0).real
    assert rel_l2(F.matvec(dev(ar), dev(xr), f=-1.0).cpu().numpy(), want) <= TOL


@pytest.mark.parametrize("f", [-1.0, 1j, np.exp(0.3j), np.exp(-2.0j)])
def test_complex_unit_f(F, f):
    for L in (1, 6, 12, 15):
        n = 1 << L
        a, x = W.complex_pair(n, seed=L + 50)
        want = O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), f)
        got = F.matvec(dev(a), dev(x), f=f).cpu().numpy()
        assert rel_l2(got, want) <= TOL, (L, f)


@pytest.mark.parametrize("f", [2.0, 0.5j, 1.5 + 0.5j])
def test_complex_non_unit_f(F, f):
    """f off the unit circle (accepted by the ABI; the node roots then have moduli
    |f|^(1/2^(d+1))): every entry against the FP64 oracle, whose error measure is taken
    relative to the result's own norm as for unit f."""
    for L in (1, 6, 12, 15):
        n = 1 << L
        a, x = W.complex_pair(n, seed=L + 70)
        want = O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), f)
        got = F.matvec(dev(a), dev(x), f=f).cpu().numpy()
        assert rel_l2(got, want) <= TOL, (L, f, rel_l2(got, want))


@pytest.mark.parametrize("L", [0, 1, 5, 6, 7, 8, 9, 10, 11, 12, 14, 16])
def test_real_ring(F, L):
    n = 1 << L
    rng = np.random.default_rng(L)
    a = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    want = O.matvec_c128(a.astype(np.complex128), x.astype(np.complex128), 1.0).real
    got = F.matvec(dev(a), dev(x)).cpu().numpy()
    assert rel_l2(got, want) <= TOL


# (20, 16..20): two top passes of 8, 9 and 10 levels each way, so the inner merge passes
# (workspace to workspace, agent-scope stores) of 8..10 levels run; blocks of 2^4 .. 2^0
@pytest.mark.parametrize("L,top", [(12, 3), (14, 10), (16, 13), (20, 16), (20, 18), (20, 20)])
def test_complex_forced_splits(F, L, top):
    n = 1 << L
    a, x = W.complex_pair(n, seed=3)
    want = O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), 1.0)
    F.set_split(top)
    try:
        got = F.matvec(dev(a), dev(x)).cpu().numpy()
    finally:
        F.set_split(-1)
    assert rel_l2(got, want) <= TOL


# Errors raised before anything is enqueued ------------------------------------------------

def test_errors(F):
    import torch
    from paper_2103_02605_amd._lib import FcircError
    a = dev(np.zeros(12, np.uint32))
    with pytest.raises(FcircError, match="ESIZE"):
        F.matvec(a, a.clone(), f=1, p=P1)
    a = dev(np.zeros(1 << 24, np.uint32))
    with pytest.raises(FcircError, match="ESIZE"):
        F.matvec(a, a.clone(), f=1, p=P1)
    a = dev(np.zeros(8, np.uint32))
    with pytest.raises(FcircError, match="ENOROOT"):
        F.matvec(a, a.clone(), f=0, p=P1)
    # 3 is a generator, so it has no square root, hence no 8-th root
    with pytest.raises(FcircError, match="ENOROOT"):
        F.matvec(a, a.clone(), f=3, p=P1)
    with pytest.raises(FcircError, match="EINVAL"):
        F.matvec(a, a, f=1, p=P1, out=a)  # output aliases the input


@pytest.mark.parametrize("L", [14, 18, 21])
def test_schedule_variants_bit_exact(F, L):
    """Every top-pass tile size, tile order and row/vector grouping the tuner may pick gives
    the same bits."""
    from paper_2103_02605_amd import _lib
    n = 1 << L
    a, x = W.modp_pair(n, P3, seed=L)
    want = oracle_modp(a, x, 1, P3)
    ring = _lib.FCIRC_ZP_167772161
    try:
        for top in (L - 13, L - 11, L - 9):
            for tile_log in (10, 11, 12, 13, 14):
                for flags in (0, 1, 2, 3):
                    F.set_schedule(n, ring, top, tile_log, flags)
                    got = host_u32(F.matvec(dev(a), dev(x), f=1, p=P3))
                    np.testing.assert_array_equal(got, want, err_msg=f"{top} {tile_log} {flags}")
        F.tune(n, ring)
        np.testing.assert_array_equal(host_u32(F.matvec(dev(a), dev(x), f=1, p=P3)), want)
    finally:
        F.set_schedule(n, ring, -1, -1, 1)
