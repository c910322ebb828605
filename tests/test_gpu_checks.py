"""GPU tests of the debugging checks (canonical-input check, per-kernel sync), of the
products at the edge values of the rings, and a property test over random (ring, n, f)."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

from oracle import fcirc as O
from oracle import gfp2 as G
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu

PRIMES = (W.P1, W.P2, W.P3)
SENTINEL = 12345


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fcirc.set_split(-1)
    yield fcirc
    fcirc.set_checks(0)
    fcirc.set_split(-1)


def dev(arr):
    import torch
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.int64)


def sentinel_like(t):
    import torch
    return torch.full_like(t, SENTINEL)


def constant_product(c, d, f, p, n):
    """A(c 1, f) (d 1): row i holds n - i entries c and i entries f c (Definition 2)."""
    k = np.arange(n, dtype=np.int64)
    coef = ((n - k) + (f % p) * k) % p  # < 2^31 * 2^26: fits int64
    return coef * (c * d % p) % p


# --- canonical-input check ------------------------------------------------------------

@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("where", ["a_first", "a_last", "x_mid"])
def test_input_check_rejects_and_writes_nothing(F, p, where):
    from paper_2103_02605_amd._lib import FcircError
    n = 1 << 13
    a, x = W.modp_pair(n, p, seed=5)
    if where == "a_first":
        a[0] = p
    elif where == "a_last":
        a[-1] = 0xFFFFFFFF
    else:
        x[n // 2] = p + 7
    A, X = dev(a), dev(x)
    y = sentinel_like(A)
    F.set_checks(F.CHECK_INPUTS)
    try:
        with pytest.raises(FcircError, match="EINVAL"):
            F.matvec(A, X, f=1, p=p, out=y)
    finally:
        F.set_checks(0)
    assert (host_u32(y) == SENTINEL).all()
    # without the check the call goes through (the result is unspecified)
    F.matvec(A, X, f=1, p=p, out=y)


def test_input_check_accepts_canonical_and_matches(F):
    p = W.P1
    n = 1 << 16
    a, x = W.modp_pair(n, p, seed=6)
    a[0], x[-1] = p - 1, p - 1
    plain = host_u32(F.matvec(dev(a), dev(x), f=1, p=p))
    F.set_checks(F.CHECK_INPUTS)
    try:
        checked = host_u32(F.matvec(dev(a), dev(x), f=1, p=p))
    finally:
        F.set_checks(0)
    np.testing.assert_array_equal(checked, plain)
    np.testing.assert_array_equal(checked, O.levels_matvec_modp(a, x, 1, p))


def test_input_check_many_any_toeplitz(F):
    from paper_2103_02605_amd._lib import FcircError
    p = W.P2
    a, x = W.modp_batch(6, 1 << 10, p, seed=8)
    a[5, 1023] = p
    A, X = dev(a), dev(x)
    y = sentinel_like(A)
    F.set_checks(F.CHECK_INPUTS)
    try:
        with pytest.raises(FcircError, match="EINVAL"):
            F.matvec_many(A, X, f=1, p=p, out=y)
        assert (host_u32(y) == SENTINEL).all()
        n = 1000
        r, v = W.modp_pair(n, p, seed=9)
        col = r.copy()
        col[999] = p + 1
        y1 = sentinel_like(dev(r))
        with pytest.raises(FcircError, match="EINVAL"):
            F.toeplitz_matvec(dev(r), dev(col), dev(v), p=p, out=y1)
        v_bad = v.copy()
        v_bad[0] = p
        with pytest.raises(FcircError, match="EINVAL"):
            F.matvec_any(dev(r), dev(v_bad), f=1, p=p, out=y1)
        assert (host_u32(y1) == SENTINEL).all()
        got = host_u32(F.matvec_any(dev(r), dev(v), f=3, p=p))
    finally:
        F.set_checks(0)
    np.testing.assert_array_equal(got, O.dense_matvec_modp(r, v, 3, p))


def test_input_check_batched(F):
    from paper_2103_02605_amd import batched
    from paper_2103_02605_amd._lib import FcircError
    p = W.P3
    sizes = [1 << k for k in (0, 3, 7, 12, 5)]
    a_list = [W.modp_pair(n, p, seed=20 + k)[0] for k, n in enumerate(sizes)]
    x_list = [W.modp_pair(n, p, seed=40 + k)[1] for k, n in enumerate(sizes)]
    plan = batched.BatchPlan(a_list, x_list, p=p, f=1)
    F.set_checks(F.CHECK_INPUTS)
    try:
        plan.run()
        for k, y in enumerate(plan.outputs()):
            np.testing.assert_array_equal(y, O.dense_matvec_modp(a_list[k], x_list[k], 1, p))
        x_list[3][4095] = p
        plan.load(a_list, x_list)
        plan.y.fill_(SENTINEL)
        with pytest.raises(FcircError, match="EINVAL"):
            plan.run()
        assert all((y == SENTINEL).all() for y in plan.outputs())
    finally:
        F.set_checks(0)


def test_input_check_gfp2(F):
    from paper_2103_02605_amd._lib import FcircError
    n = 1 << 11
    rng = np.random.default_rng(3)
    a = rng.integers(0, G.P, (n, 2), dtype=np.int64).astype(np.uint32)
    x = rng.integers(0, G.P, (n, 2), dtype=np.int64).astype(np.uint32)
    a[17, 1] = G.P
    y = sentinel_like(dev(a))
    F.set_checks(F.CHECK_INPUTS)
    try:
        with pytest.raises(FcircError, match="EINVAL"):
            F.matvec(dev(a), dev(x), f=1, p=G.P, out=y)
    finally:
        F.set_checks(0)
    assert (host_u32(y) == SENTINEL).all()


def test_check_flags(F):
    from paper_2103_02605_amd._lib import FcircError
    with pytest.raises(FcircError, match="EINVAL"):
        F.set_checks(4)


def test_sync_after_every_kernel_same_bits(F):
    p = W.P1
    n = 1 << 21
    a, x = W.modp_pair(n, p, seed=W.SEED_HEADLINE)
    A, X = dev(a), dev(x)
    plain = host_u32(F.matvec(A, X, f=1, p=p))
    F.set_checks(F.CHECK_SYNC | F.CHECK_INPUTS)
    try:
        synced = host_u32(F.matvec(A, X, f=1, p=p))
    finally:
        F.set_checks(0)
    np.testing.assert_array_equal(synced, plain)


# --- edge values of the rings -----------------------------------------------------------

@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("L", [0, 1, 4, 10, 13, 16, 20])
def test_constant_edge_values(F, p, L):
    """Inputs all 0, all 1 and all p-1 (the largest canonical value, which drives every
    lazy intermediate to its upper bound) against the closed form of a constant product."""
    n = 1 << L
    for f in (1, p - 1):
        for c, d in ((0, 5), (1, 1), (p - 1, p - 1), (p - 1, 1)):
            a = np.full(n, c, dtype=np.uint32)
            x = np.full(n, d, dtype=np.uint32)
            y = host_u32(F.matvec(dev(a), dev(x), f=f, p=p))
            np.testing.assert_array_equal(y, constant_product(c, d, f, p, n), err_msg=f"n={n} f={f} c={c} d={d}")


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("L", [1, 5, 11, 14])
def test_alternating_edge_values(F, p, L):
    n = 1 << L
    a = np.where(np.arange(n) % 2 == 0, 0, p - 1).astype(np.uint32)
    x = np.where(np.arange(n) % 3 == 0, p - 1, 1).astype(np.uint32)
    f = p - 1
    y = host_u32(F.matvec(dev(a), dev(x), f=f, p=p))
    want = O.dense_matvec_modp(a, x, f, p) if n <= 2048 else O.levels_matvec_modp(a, x, f, p)
    np.testing.assert_array_equal(y, want)


def test_gfp2_edge_values(F):
    n = 1 << 12
    m = G.P - 1
    for c, d in (((m, m), (m, m)), ((0, m), (0, m)), ((m, 0), (1, 0))):
        a = np.tile(np.array(c, dtype=np.uint32), (n, 1))
        x = np.tile(np.array(d, dtype=np.uint32), (n, 1))
        for f in (1, m):
            y = F.matvec(dev(a), dev(x), f=f, p=G.P).cpu().numpy().view(np.uint32).reshape(n, 2)
            cd = G.mul(c, d)
            for i in (0, 1, n // 2, n - 1):
                coef = ((n - i) + f * i) % G.P
                assert tuple(int(v) for v in y[i]) == G.scale(cd, coef), (c, d, f, i)


# --- property test -----------------------------------------------------------------------

@settings(max_examples=60, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.function_scoped_fixture, HealthCheck.too_slow])
@given(ring=st.sampled_from(PRIMES), L=st.integers(0, 17), phi=st.integers(1, 2**31), seed=st.integers(0, 2**31))
def test_random_ring_size_root(F, ring, L, phi, seed):
    """f = phi^n always has the n-th root phi (Theorem 1's condition); any such f works."""
    p = ring
    n = 1 << L
    f = pow(phi % (p - 1) + 1, n, p)
    a, x = W.modp_pair(n, p, seed=seed)
    y = host_u32(F.matvec(dev(a), dev(x), f=f, p=p))
    want = O.dense_matvec_modp(a, x, f, p) if n <= 1024 else O.levels_matvec_modp(a, x, f, p)
    np.testing.assert_array_equal(y, want, err_msg=f"p={p} n={n} f={f}")
