"""Pins for the CPU oracle: each test checks it against something other than itself
(the paper's worked example, closed forms, invariants, library routines, brute force).
"""
import os
import random

import numpy as np
import pytest

from oracle import fcirc as O
from oracle import ring
from oracle import polymul as OP
from oracle import bigint as OB
from oracle import grad as OG
from oracle import embed as OE

P1, P2, P3 = 998244353, 469762049, 167772161
PRIMES = (P1, P2, P3)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_f_with_root(n, p, rng):
    """A random f that has an n-th root: phi**n for a random unit phi."""
    phi = rng.randrange(1, p)
    return pow(phi, n, p)


# P1: the worked 3x3 example of Definition 2 -------------------------------------------

def _read_golden_3x3():
    a, f, rows = None, None, []
    with open(os.path.join(GOLDEN, "paper_3x3.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            vals = [int(v) for v in vals]
            if key == "a":
                a = vals
            elif key == "f":
                f = vals[0]
            elif key == "row":
                rows.append(vals)
    return a, f, rows


def test_p1_paper_3x3_example():
    a, f, rows = _read_golden_3x3()
    assert O.fcirc_matrix(a, f) == rows
    assert O.fcirc_matrix_np(a, f, 10**9 + 7).tolist() == rows


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 64, 256])
def test_closed_form_matrix_matches_definition(n):
    rng = random.Random(n)
    for p in PRIMES:
        a = [rng.randrange(p) for _ in range(n)]
        f = rng.randrange(p)
        assert O.fcirc_matrix_np(a, f, p).tolist() == O.fcirc_matrix(a, f, p)


# P2: closed forms at n = 1 and n = 2 ---------------------------------------------------

@pytest.mark.parametrize("p", PRIMES)
def test_p2_closed_forms(p):
    rng = random.Random(p)
    for _ in range(20):
        a0, a1, x0, x1 = (rng.randrange(p) for _ in range(4))
        f = pow(rng.randrange(1, p), 2, p)  # n = 2 needs a square root of f
        want = [(a0 * x0 + a1 * x1) % p, (f * a1 * x0 + a0 * x1) % p]
        assert O.alg1_modp([a0, a1], [x0, x1], f, p) == want
        assert O.levels_matvec_modp([a0, a1], [x0, x1], f, p).tolist() == want
        assert O.dense_matvec_py([a0, a1], [x0, x1], f, p) == want
        assert O.alg1_modp([a0], [x0], f, p) == [a0 * x0 % p]


# P3: recursion == definition, brute force -----------------------------------------------

@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("L", range(0, 9))
def test_p3_alg1_equals_dense(p, L):
    n = 1 << L
    rng = random.Random(1000 * L + p % 1000)
    for f in (1, p - 1, _rand_f_with_root(n, p, rng)):
        a = [rng.randrange(p) for _ in range(n)]
        x = [rng.randrange(p) for _ in range(n)]
        want = O.dense_matvec_py(a, x, f, p) if n <= 64 else O.dense_matvec_modp(a, x, f, p).tolist()
        assert O.alg1_modp(a, x, f, p) == want


@pytest.mark.parametrize("p", PRIMES)
@pytest.mark.parametrize("L", range(0, 12))
def test_p3_levels_equals_dense(p, L):
    n = 1 << L
    rng = np.random.default_rng(L * 7 + p % 97)
    prng = random.Random(L)
    for f in (1, p - 1, _rand_f_with_root(n, p, prng)):
        a = rng.integers(0, p, n)
        x = rng.integers(0, p, n)
        np.testing.assert_array_equal(O.levels_matvec_modp(a, x, f, p), O.dense_matvec_modp(a, x, f, p))


def test_dense_numpy_equals_python():
    rng = random.Random(5)
    for n in (1, 3, 8, 17, 32):
        for p in PRIMES:
            a = [rng.randrange(p) for _ in range(n)]
            x = [rng.randrange(p) for _ in range(n)]
            f = rng.randrange(p)
            assert O.dense_matvec_modp(a, x, f, p).tolist() == O.dense_matvec_py(a, x, f, p)


# P4: special cases that reduce to library routines ---------------------------------------

def _fft_correlation_exact(a, x, sign=1):
    """sum_k a_k x_{i+k} (times sign on wrap) for small integers, via numpy.fft and rounding."""
    n = len(a)
    ap = np.concatenate([np.asarray(a, float), np.zeros(n)])
    xp = np.concatenate([np.asarray(x, float), sign * np.asarray(x, float)])
    y = np.fft.ifft(np.conj(np.fft.fft(ap)) * np.fft.fft(xp))[:n]
    return np.rint(y.real).astype(np.int64)


@pytest.mark.parametrize("L", [3, 8, 12, 15])
def test_p4_cyclic_and_negacyclic_match_fft(L):
    n = 1 << L
    rng = np.random.default_rng(L)
    a = rng.integers(0, 64, n)
    x = rng.integers(0, 64, n)
    for p in PRIMES:
        cyc = _fft_correlation_exact(a, x, +1) % p
        neg = _fft_correlation_exact(a, x, -1) % p
        np.testing.assert_array_equal(O.levels_matvec_modp(a, x, 1, p), cyc)
        np.testing.assert_array_equal(O.levels_matvec_modp(a, x, p - 1, p), neg)


def test_p4_negacyclic_transpose_is_convolution():
    """For f = -1 the transpose of A(a) multiplies polynomials mod z^n + 1 (schoolbook)."""
    rng = np.random.default_rng(3)
    for n in (1, 2, 4, 8, 32):
        a = rng.integers(-50, 50, n)
        x = rng.integers(-50, 50, n)
        A = np.array(O.fcirc_matrix(a.tolist(), -1))
        full = np.convolve(a, x)
        want = full[:n].copy()
        want[: len(full) - n] -= full[n:]
        np.testing.assert_array_equal(A.T @ x, want)


def test_p4_complex_matches_fft_identity():
    rng = np.random.default_rng(9)
    for n in (1, 2, 8, 64, 1024, 4096):
        a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        want = np.fft.ifft(np.conj(np.fft.fft(np.conj(a))) * np.fft.fft(x))
        got = O.levels_matvec_c128(a, x, 1.0)
        assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
        if n <= 1024:
            assert np.linalg.norm(O.dense_matvec_c128(a, x) - want) <= 1e-12 * np.linalg.norm(want)
        if n <= 64:
            assert np.linalg.norm(np.array(O.alg1_c128(a, x)) - want) <= 1e-12 * np.linalg.norm(want)


def test_fft_oracle_matches_recursion():
    rng = np.random.default_rng(12)
    for n in (1, 2, 16, 256, 8192):
        a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        want = O.levels_matvec_c128(a, x, 1.0)
        got = O.cyclic_matvec_fft_c128(a, x)
        assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


def test_p4_complex_general_unit_f():
    rng = np.random.default_rng(10)
    for n in (2, 16, 128):
        a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        for f in (1.0, -1.0, 1j, np.exp(0.7j), 2.5 - 0.3j):
            want = O.dense_matvec_c128(a, x, f)
            for got in (O.levels_matvec_c128(a, x, f), np.array(O.alg1_c128(a, x, f))):
                assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)


# P5: invariants -------------------------------------------------------------------------

@pytest.mark.parametrize("p", PRIMES)
def test_p5_linearity_and_unit_vectors(p):
    n = 64
    rng = np.random.default_rng(p % 1000)
    prng = random.Random(p)
    f = _rand_f_with_root(n, p, prng)
    a, a2, x, x2 = (rng.integers(0, p, n) for _ in range(4))
    c = int(rng.integers(0, p))
    mv = lambda u, v: O.levels_matvec_modp(u, v, f, p)
    np.testing.assert_array_equal(mv((a + c * a2) % p, x), (mv(a, x) + c * mv(a2, x)) % p)
    np.testing.assert_array_equal(mv(a, (x + c * x2) % p), (mv(a, x) + c * mv(a, x2)) % p)
    e0 = np.zeros(n, np.int64)
    e0[0] = 1
    np.testing.assert_array_equal(mv(e0, x), x % p)
    for k in (1, 5, 63):
        ek = np.zeros(n, np.int64)
        ek[k] = 1
        # (P^k x)_i = x_{i+k}, times f when the index wraps
        idx = np.arange(n) + k
        want = np.where(idx < n, x[idx % n], x[idx % n] * f % p) % p
        np.testing.assert_array_equal(mv(ek, x), want)
    A = O.fcirc_matrix_np(a, f, p)
    for j in (0, 7, 63):
        ej = np.zeros(n, np.int64)
        ej[j] = 1
        np.testing.assert_array_equal(mv(a, ej), A[:, j])


# P6: ring homomorphism A(a) A(b) = A(a b mod z^n - f) ------------------------------------

@pytest.mark.parametrize("p", PRIMES)
def test_p6_homomorphism(p):
    n = 32
    rng = np.random.default_rng(1 + p % 100)
    f = _rand_f_with_root(n, p, random.Random(p + 1))
    a, b, x = (rng.integers(0, p, n) for _ in range(3))
    full = [0] * (2 * n - 1)
    for i in range(n):
        for j in range(n):
            full[i + j] += int(a[i]) * int(b[j])
    c = [(full[r] + (f * full[r + n] if r + n < 2 * n - 1 else 0)) % p for r in range(n)]
    lhs = O.levels_matvec_modp(a, O.levels_matvec_modp(b, x, f, p), f, p)
    np.testing.assert_array_equal(lhs, O.levels_matvec_modp(np.array(c), x, f, p))


# P7: any choice of square root gives the same product ------------------------------------

@pytest.mark.parametrize("p", PRIMES)
def test_p7_root_choice_invariance(p):
    n = 64
    rng = random.Random(p)
    a = [rng.randrange(p) for _ in range(n)]
    x = [rng.randrange(p) for _ in range(n)]
    for f in (1, p - 1, _rand_f_with_root(n, p, rng)):
        base = O.alg1_modp(a, x, f, p)
        for s in range(6):
            assert O.alg1_modp(a, x, f, p, random.Random(s)) == base


# P8: the children are (+-sqrt f)-circulant with rows a_lo +- g a_hi ------------------------

@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_p8_children_are_fcirculant(n):
    p = P1
    rng = random.Random(n)
    f = _rand_f_with_root(n, p, rng)
    a = [rng.randrange(p) for _ in range(n)]
    A = np.array(O.fcirc_matrix(a, f, p), dtype=object)
    h = n // 2
    A1, A2 = A[:h, :h], A[:h, h:]
    g = ring.sqrt_mod(f, p)
    R = O.ModP(p)
    r1, r2 = O.alg1_children_rows(a, g, R)
    M1 = np.array(O.fcirc_matrix(r1, g, p), dtype=object)
    M2 = np.array(O.fcirc_matrix(r2, (p - g) % p, p), dtype=object)
    assert ((A1 + A2 * g) % p == M1).all()
    assert ((A1 - A2 * g) % p == M2).all()
    # the lower blocks are A2 f and A1 (block form in the proof of Theorem 1)
    assert ((A[h:, :h] - A2 * f) % p == 0).all()
    assert (A[h:, h:] == A1).all()


# P9: Corollary 1, arbitrary n by padding ---------------------------------------------------

@pytest.mark.parametrize("n", [3, 5, 6, 7])
def test_p9_corollary1_padding(n):
    d = 0
    while (1 << d) <= n:
        d += 1
    N = 1 << (d + 1)  # the paper's N = 2^(d+1) with 2^d > n
    rng = random.Random(n)
    p = P1
    a = [rng.randrange(p) for _ in range(n)]
    b = [rng.randrange(p) for _ in range(n)]
    a_pad = a + [0] * (N - 2 * n + 1) + a[1:]
    b_pad = b + [0] * (N - n)
    assert len(a_pad) == N
    got = O.alg1_modp(a_pad, b_pad, 1, p)[:n]
    assert got == O.dense_matvec_py(a, b, 1, p)


# P10: polynomial and integer products against library routines ------------------------------

def test_p10_polymul_small():
    rng = np.random.default_rng(4)
    for na, nb in [(1, 1), (1, 5), (3, 4), (17, 9), (100, 100), (257, 31)]:
        a = rng.integers(-(1 << 15), 1 << 15, na)
        b = rng.integers(-(1 << 15), 1 << 15, nb)
        want = OP.poly_schoolbook(a, b)
        np.testing.assert_array_equal(np.convolve(a.astype(object), b.astype(object)), want)
        assert OP.poly_kronecker(a, b).tolist() == want
        assert OP.poly_via_circulant(a, b, PRIMES) == want


def test_p10_polymul_medium_kronecker_vs_circulant():
    rng = np.random.default_rng(44)
    n = 1 << 12
    a = rng.integers(-(1 << 15), 1 << 15, n)
    b = rng.integers(-(1 << 15), 1 << 15, n)
    kr = OP.poly_kronecker(a, b)
    np.testing.assert_array_equal(np.convolve(a, b), kr)  # int64 exact: |c| < 2^42
    assert OP.poly_via_circulant(a, b, PRIMES) == kr.tolist()


def test_p10_bigint():
    rng = np.random.default_rng(5)
    for na, nb in [(1, 1), (2, 3), (64, 64), (1000, 333), (1 << 11, 1 << 11)]:
        a = rng.integers(0, 1 << 16, na).astype(np.uint16)
        b = rng.integers(0, 1 << 16, nb).astype(np.uint16)
        want = OB.bigint_mul_pyint(a, b)
        assert OB.limbs_to_int(want) == OB.limbs_to_int(a) * OB.limbs_to_int(b)
        np.testing.assert_array_equal(OB.bigint_mul_via_circulant(a, b, PRIMES), want)
    ff = np.full(300, 0xFFFF, np.uint16)
    np.testing.assert_array_equal(OB.bigint_mul_via_circulant(ff, ff, PRIMES), OB.bigint_mul_pyint(ff, ff))


# P11: CRT round trip -----------------------------------------------------------------------

def test_p11_crt_round_trip():
    rng = random.Random(11)
    M = P1 * P2 * P3
    vals = [rng.randrange(-(M // 2) + 1, M // 2) for _ in range(200)]
    vals += [0, 1, -1, P1 * P2 - 1, -(P1 * P2), M // 2, -(M // 2) + 1]
    res = [[v % q for v in vals] for q in PRIMES]
    assert OP.crt_textbook(res, PRIMES) == vals


# P13: gradients: dense autograd against finite differences ----------------------------------

def test_p13_grad_dense_vs_finite_differences():
    rng = np.random.default_rng(13)
    n, batch = 64, 2
    a = rng.standard_normal(n)
    x = rng.standard_normal((batch, n))
    g = rng.standard_normal((batch, n))
    y, ga, gx = OG.dense_autograd(a, x, g)
    fa, fx = OG.finite_differences(a, x, g)
    assert np.abs(ga - fa).max() <= 1e-6 * max(1.0, np.abs(fa).max())
    assert np.abs(gx - fx).max() <= 1e-6 * max(1.0, np.abs(fx).max())
    # and the forward is the f = 1 product
    for b in range(batch):
        np.testing.assert_allclose(y[b], O.dense_matvec_c128(a, x[b]).real, rtol=0, atol=1e-10)


def test_complex_grad_is_adjoint():
    """For complex data, grad_x = A^H g and grad_a_k = sum_i conj(x_{i+k}) g_i."""
    rng = np.random.default_rng(14)
    n = 16
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = rng.standard_normal((1, n)) + 1j * rng.standard_normal((1, n))
    g = rng.standard_normal((1, n)) + 1j * rng.standard_normal((1, n))
    _, ga, gx = OG.dense_autograd(a, x, g)
    A = O.fcirc_matrix_np(a, 1.0)
    np.testing.assert_allclose(gx[0], A.conj().T @ g[0], atol=1e-12)
    want_a = np.array([sum(np.conj(x[0][(i + k) % n]) * g[0][i] for i in range(n)) for k in range(n)])
    np.testing.assert_allclose(ga, want_a, atol=1e-12)


# Ring helpers --------------------------------------------------------------------------------

@pytest.mark.parametrize("p", PRIMES)
def test_ring_roots(p):
    assert ring.primitive_root(p) == 3  # 3 generates all three multiplicative groups
    two_adic = {P1: 23, P2: 26, P3: 25}[p]
    assert (p - 1) % (1 << two_adic) == 0 and (p - 1) % (1 << (two_adic + 1)) != 0
    w = ring.root_of_unity(1 << two_adic, p)
    assert pow(w, 1 << (two_adic - 1), p) == p - 1
    with pytest.raises(ValueError):
        ring.root_of_unity(1 << (two_adic + 1), p)


@pytest.mark.parametrize("p", PRIMES)
def test_ring_inverse_root_identity(p):
    """Section 3.1: the inverse of the fourth root of i is -i sqrt(i) fourth-root(i)."""
    i = pow(3, (p - 1) // 4, p)
    assert i * i % p == p - 1
    s = ring.sqrt_mod(i, p)
    r = ring.sqrt_mod(s, p)
    assert r * r % p == s
    assert (-i * s * r) % p == ring.inv(r, p)


@pytest.mark.parametrize("cplx", [False, True])
def test_fft_grads_match_dense_autograd(cplx):
    rng = np.random.default_rng(15)
    n, batch = 32, 3
    def draw(*shape):
        v = rng.standard_normal(shape)
        return v + 1j * rng.standard_normal(shape) if cplx else v
    a, x, g = draw(n), draw(batch, n), draw(batch, n)
    y, ga, gx = OG.dense_autograd(a, x, g)
    y2, ga2, gx2 = OG.grads_fft(a, x, g)
    for u, v in ((y, y2), (ga, ga2), (gx, gx2)):
        np.testing.assert_allclose(v, u, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("cplx", [False, True])
def test_layer_entries_match_dense_autograd(cplx):
    """The O(n) entry formulas (used for sampled checks at sizes the dense and FFT
    references cannot reach) against torch autograd on the dense matrix, every entry."""
    rng = np.random.default_rng(16)
    n, batch = 32, 3
    def draw(*shape):
        v = rng.standard_normal(shape)
        return v + 1j * rng.standard_normal(shape) if cplx else v
    a, x, g = draw(n), draw(batch, n), draw(batch, n)
    y, ga, gx = OG.dense_autograd(a, x, g)
    y2, ga2, gx2 = OG.layer_entries(a, x, g, np.arange(n))
    for u, v in ((y, y2), (ga, ga2), (gx, gx2)):
        np.testing.assert_allclose(v, u, rtol=1e-10, atol=1e-10)


# P9b: Toeplitz products and the f-circulant of any size by embedding ----------------------

def test_p9b_toeplitz_matrix_is_scipy_toeplitz():
    import scipy.linalg
    rng = np.random.default_rng(91)
    for n in (1, 2, 5, 12):
        row = rng.standard_normal(n)
        col = rng.standard_normal(n)
        col[0] = row[0]
        assert np.array_equal(np.array(OE.toeplitz_matrix(row, col)), scipy.linalg.toeplitz(col, row))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 7, 9, 12])
def test_p9b_fcirc_is_toeplitz_with_wrapped_column(n):
    """Definition 2's builder (any n) equals the Toeplitz matrix whose first column is
    f times the row's tail in reverse."""
    rng = random.Random(9 * n)
    p = P2
    a = [rng.randrange(p) for _ in range(n)]
    for f in (1, p - 1, rng.randrange(2, p), 0):
        assert O.fcirc_matrix(a, f, p) == OE.toeplitz_matrix(a, OE.fcirc_col(a, f, p), p)


def test_p9b_library_length_is_the_corollarys():
    for n in range(2, 5000):
        if n & (n - 1):
            assert OE.cyclic_length(n) == OE.corollary_length(n)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 17, 100, 333])
def test_p9b_embedded_products_match_the_definition(n):
    rng = np.random.default_rng(700 + n)
    for p in PRIMES:
        row = rng.integers(0, p, n)
        col = rng.integers(0, p, n)
        x = rng.integers(0, p, n)
        want = OE.toeplitz_matvec_dense(row, col, x, p)
        assert np.array_equal(OE.toeplitz_matvec_modp(row, col, x, p), want)
        for f in (1, p - 1, int(rng.integers(2, p)), 0):
            want_f = np.array(O.dense_matvec_py([int(v) for v in row], [int(v) for v in x], f, p))
            assert np.array_equal(OE.fcirc_any_matvec_modp(row, x, f, p), want_f)
    c = lambda: rng.standard_normal(n) + 1j * rng.standard_normal(n)
    row, col, x = c(), c(), c()
    np.testing.assert_allclose(OE.toeplitz_matvec_c128(row, col, x), OE.toeplitz_matvec_dense(row, col, x),
                               rtol=1e-9, atol=1e-9)
    for f in (1.0, 1j, 0.5 - 2j):
        np.testing.assert_allclose(OE.fcirc_any_matvec_c128(row, x, f), O.dense_matvec_c128(row, x, f),
                                   rtol=1e-9, atol=1e-9)


# P15: the ring of section 3.1, Z/p[sqrt 3] with p = 2^31 - 1 -----------------------------

from oracle import gfp2 as OG2  # noqa: E402


def test_p15_ring_is_a_field_and_the_generator_has_order_2_31():
    p = OG2.P
    assert p == 2**31 - 1 and pow(2, p - 1, p) == 1
    assert pow(3, (p - 1) // 2, p) == p - 1          # 3 is not a square: Z/p[sqrt 3] = GF(p^2)
    assert OG2.norm(OG2.GEN) == 1                       # 2 + sqrt 3 has norm 4 - 3 = 1
    assert OG2.power(OG2.GEN, 1 << 31) == OG2.ONE       # order divides p + 1 = 2^31
    assert OG2.power(OG2.GEN, 1 << 30) != OG2.ONE       # ... and is exactly 2^31
    for k in (1, 2, 5, 16, 31):
        w = OG2.root_of_unity(1 << k)
        assert OG2.power(w, 1 << k) == OG2.ONE
        assert OG2.power(w, 1 << (k - 1)) == (p - 1, 0)  # primitive: w^(N/2) = -1


def test_p15_paper_inverse_root_identity():
    """(fourth root of i)^-1 = -i sqrt(i) (fourth root of i), with the precomputed roots."""
    z = OG2.root_of_unity(16)     # a fourth root of i
    s = OG2.mul(z, z)             # a square root of i
    i = OG2.mul(s, s)
    assert OG2.mul(i, i) == (OG2.P - 1, 0)
    assert OG2.inv(z) == OG2.neg(OG2.mul(OG2.mul(i, s), z))


def test_p15_field_operations():
    rng = random.Random(15)
    for _ in range(200):
        u = (rng.randrange(OG2.P), rng.randrange(OG2.P))
        v = (rng.randrange(OG2.P), rng.randrange(OG2.P))
        if u != (0, 0):
            assert OG2.mul(u, OG2.inv(u)) == OG2.ONE
        assert OG2.mul(u, v) == OG2.mul(v, u)
        sq = OG2.mul(u, u)
        r = OG2.sqrt(sq)
        assert OG2.mul(r, r) == sq
        arr_u, arr_v = OG2.as_array([u]), OG2.as_array([v])
        assert tuple(int(c) for c in OG2.vmul(arr_u, arr_v)[0]) == OG2.mul(u, v)
        if u != (0, 0):
            assert tuple(int(c) for c in OG2.vinv(arr_u)[0]) == OG2.inv(u)
    with pytest.raises(ValueError):
        OG2.sqrt(OG2.Z_NONSQ)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32])
def test_p15_recursion_matches_definition(n):
    rng = random.Random(150 + n)
    a = [(rng.randrange(OG2.P), rng.randrange(OG2.P)) for _ in range(n)]
    x = [(rng.randrange(OG2.P), rng.randrange(OG2.P)) for _ in range(n)]
    for f in (OG2.ONE, (OG2.P - 1, 0)):
        want = OG2.dense_matvec(a, x, f)
        assert O.alg1_matvec(a, x, f, OG2.GFp2(random.Random(n))) == want  # random root choices
        assert [tuple(int(c) for c in r) for r in OG2.levels_matvec(a, x, f)] == want


def test_p15_levels_sampled_at_2_14():
    n = 1 << 14
    g = np.random.default_rng(16)
    a = g.integers(0, OG2.P, (n, 2)).astype(np.uint64)
    x = g.integers(0, OG2.P, (n, 2)).astype(np.uint64)
    for f in (OG2.ONE, (OG2.P - 1, 0)):
        y = OG2.levels_matvec(a, x, f)
        for i in (0, 1, 777, n - 1):
            assert tuple(int(c) for c in y[i]) == OG2.matvec_entry(a, x, f, i)


# ----------------------------------------------------------------------------------
# P16: section 3.2's ring Z/(2^K + 1), roots of unity as powers of two
# ----------------------------------------------------------------------------------
from oracle import fermat as OF  # noqa: E402


@pytest.mark.parametrize("K", [8, 64, 2048])
def test_p16_two_has_order_2k(K):
    """2^K = -1, so 2 is a primitive 2K-th root of unity: 2^e != 1 for 0 < e < 2K
    (checked at the divisors of 2K, which suffice since 2K is a power of two times K)."""
    M = OF.modulus(K)
    assert pow(2, K, M) == M - 1
    assert pow(2, 2 * K, M) == 1
    for e in range(1, 2 * K):
        if (2 * K) % e == 0:
            assert pow(2, e, M) != 1 or e == 2 * K


def test_p16_square_roots_are_shifts():
    K = 64
    R = OF.Fermat(K, random.Random(1))
    M = OF.modulus(K)
    for e in range(0, 2 * K, 2):
        r = R.sqrt(pow(2, e, M))
        assert r * r % M == pow(2, e, M)
        assert R.log2(r) in (e // 2, e // 2 + K)
    with pytest.raises(ValueError):
        R.sqrt(2)
    with pytest.raises(ValueError):
        R.sqrt(3)  # not a power of two


@pytest.mark.parametrize("K,n", [(16, 8), (64, 16), (64, 32), (256, 32), (2048, 16)])
def test_p16_recursion_matches_definition(K, n):
    """Definition 2 (dense), Algorithm 1 with random choices of the roots, and the level
    form with shift counts agree for f = 1, f = -1 = 2^K and f = 2^e (e a multiple of 2n)."""
    rng = random.Random(K + n)
    M = OF.modulus(K)
    a = [rng.randrange(M) for _ in range(n)]
    x = [rng.randrange(M) for _ in range(n)]
    a[0], x[-1] = M - 1, M - 1  # the value 2^K itself
    for f_exp in (0, K, 2 * n):
        f = pow(2, f_exp, M)
        want = OF.dense_matvec(a, x, f, K)
        assert O.alg1_matvec(a, x, f, OF.Fermat(K, random.Random(n))) == want
        assert OF.levels_matvec(a, x, f_exp, K) == want


def test_p16_odd_exponent_has_no_root():
    with pytest.raises(ValueError):
        OF.levels_matvec([1, 2], [3, 4], 1, 64)
    with pytest.raises(ValueError):
        OF.node_exponents(6, 0, 16)  # 2^6 = 64 > 2K = 32: the ladder runs out of halvings


@pytest.mark.parametrize("P,N,K", [(16, 8, 64), (64, 16, 256), (96, 64, 256), (1008, 64, 2048)])
def test_p16_bigint_through_one_cyclic_product(P, N, K):
    """Section 3.2: the product of two integers split into pieces of P bits is one cyclic
    product over Z/(2^K + 1), recomposed; it equals Python's integer product."""
    rng = random.Random(P * N)
    for _ in range(3):
        u = rng.getrandbits(P * (N // 2))
        v = rng.getrandbits(P * (N // 2))
        assert OF.bigint_mul_ssa(u, v, P, N, K) == u * v
    top = (1 << (P * (N // 2))) - 1
    assert OF.bigint_mul_ssa(top, top, P, N, K) == top * top
    assert OF.bigint_mul_ssa(0, top, P, N, K) == 0


def test_sampled_entry_helpers_match_full_definitions():
    """The O(n) one-entry forms used for sampled checks at large n agree with the full
    definitions on small inputs (Toeplitz, polynomial product, Z/(2^K + 1))."""
    rng = np.random.default_rng(77)
    p = 998244353
    for n in (1, 2, 7, 33):
        row, col, x = (rng.integers(0, p, n) for _ in range(3))
        full = OE.toeplitz_matvec_dense(row.tolist(), col.tolist(), x.tolist(), p)
        assert [OE.toeplitz_entry_modp(row, col, x, p, i) for i in range(n)] == [int(v) for v in full]
    for na, nb in ((1, 1), (5, 3), (40, 17)):
        a = rng.integers(-(1 << 15), 1 << 15, na)
        b = rng.integers(-(1 << 15), 1 << 15, nb)
        full = OP.poly_schoolbook(a.tolist(), b.tolist())
        assert [OP.poly_coef(a, b, k) for k in range(na + nb - 1)] == [int(v) for v in full]
    K, n = 64, 8
    M = OF.modulus(K)
    r = random.Random(78)
    a = [r.randrange(M) for _ in range(n)]
    x = [r.randrange(M) for _ in range(n)]
    full = OF.dense_matvec(a, x, 5, K)
    assert [OF.matvec_entry(a, x, 5, K, i) for i in range(n)] == full
