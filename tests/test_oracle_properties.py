"""Property tests of the oracle (CPU): random (prime, n, f, seed) with f = phi^n, so that
f has the n-th root phi that Theorem 1 asks for. Each property is fixed by Definition 2
or by linear algebra, not by the recursion under test."""
import random

import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import fcirc as O
from paper_2103_02605_amd import workloads as W

PRIMES = (W.P1, W.P2, W.P3)
SETTINGS = settings(max_examples=80, deadline=None, derandomize=True)


def _case(p, L, phi, seed):
    n = 1 << L
    f = pow(phi % (p - 1) + 1, n, p)
    a, x = W.modp_pair(n, p, seed=seed)
    return n, f, a.astype(np.int64), x.astype(np.int64)


@SETTINGS
@given(p=st.sampled_from(PRIMES), L=st.integers(0, 9), phi=st.integers(0, 2**40), seed=st.integers(0, 2**31))
def test_recursions_equal_definition(p, L, phi, seed):
    """Algorithm 1 (literal recursion, random square-root signs) and its level-by-level
    form both give the dense product of Definition 2."""
    n, f, a, x = _case(p, L, phi, seed)
    want = O.dense_matvec_modp(a, x, f, p)
    np.testing.assert_array_equal(O.levels_matvec_modp(a, x, f, p), want)
    if n <= 64:
        got = O.alg1_modp([int(v) for v in a], [int(v) for v in x], f, p, rng=random.Random(seed))
        np.testing.assert_array_equal(np.array(got, dtype=np.int64), want)


@SETTINGS
@given(p=st.sampled_from(PRIMES), L=st.integers(1, 11), phi=st.integers(0, 2**40), seed=st.integers(0, 2**31),
       k=st.integers(0, 2**31))
def test_linear_in_a_and_x(p, L, phi, seed, k):
    """y is bilinear in (a, x): A(a, f)(x + k x') = y + k y' and A(a + k a', f) x likewise."""
    n, f, a, x = _case(p, L, phi, seed)
    _, _, a2, x2 = _case(p, L, phi, seed + 1)
    k %= p
    y = O.levels_matvec_modp(a, x, f, p)
    lhs = O.levels_matvec_modp(a, (x + k * x2) % p, f, p)
    np.testing.assert_array_equal(lhs, (y + k * O.levels_matvec_modp(a, x2, f, p)) % p)
    lhs = O.levels_matvec_modp((a + k * a2) % p, x, f, p)
    np.testing.assert_array_equal(lhs, (y + k * O.levels_matvec_modp(a2, x, f, p)) % p)


@SETTINGS
@given(p=st.sampled_from(PRIMES), L=st.integers(1, 10), phi=st.integers(0, 2**40), seed=st.integers(0, 2**31))
def test_f_shift_of_the_vector(p, L, phi, seed):
    """By Definition 2, A(a, f) = sum_k a_k S^k for the f-shift S, (S v)_i = v_{i+1} and
    (S v)_{n-1} = f v_0; so A commutes with S: A (S x) = S (A x)."""
    n, f, a, x = _case(p, L, phi, seed)
    sx = np.concatenate([x[1:], [f * x[0] % p]])
    y = O.levels_matvec_modp(a, x, f, p)
    sy = np.concatenate([y[1:], [f * y[0] % p]])
    np.testing.assert_array_equal(O.levels_matvec_modp(a, sx, f, p), sy)


@SETTINGS
@given(p=st.sampled_from(PRIMES), L=st.integers(0, 10), phi=st.integers(0, 2**40), seed=st.integers(0, 2**31),
       i=st.integers(0, 2**20))
def test_single_entry(p, L, phi, seed, i):
    """One output by the O(n) definition equals the recursion's."""
    n, f, a, x = _case(p, L, phi, seed)
    i %= n
    assert O.matvec_entry_modp(a, x, f, p, i) == int(O.levels_matvec_modp(a, x, f, p)[i])


@SETTINGS
@given(p=st.sampled_from(PRIMES), L=st.integers(2, 12), phi=st.integers(0, 2**40), phi2=st.integers(0, 2**40),
       d0=st.integers(0, 11), blk=st.integers(0, 2**20))
def test_block_factors_of_the_root_ladder(p, L, phi, phi2, d0, blk):
    """Inside any block of the recursion (depth d0, index blk), the square root at local
    level l and index g is the block's first root of that level times a factor that
    depends on (l, g) only: not on the block, its depth, or f. The factors of level l are
    the powers w_l^brev_l(g) of one primitive 2^(l+1)-th root of unity. (The GPU path
    forms the roots of its block passes this way.)"""
    n = 1 << L
    d0 %= L
    blk %= 1 << d0
    fs = [pow(v % (p - 1) + 1, n, p) for v in (phi, phi2)]
    ladders = [O.node_roots_modp(n, f, p) for f in fs]

    def brev(g, l):
        return int(format(g, f"0{l}b")[::-1], 2) if l else 0

    for l in range(L - d0):
        d = d0 + l
        per_case = []
        for gs in ladders:
            for b in {blk, (blk + 1) % (1 << d0), 0}:
                first = int(gs[d][b << l])
                inv = pow(first, p - 2, p)
                per_case.append([int(gs[d][(b << l) + g]) * inv % p for g in range(1 << l)])
        for r in per_case[1:]:
            assert r == per_case[0], (l, d0)
        ratio = per_case[0]
        if l == 0:
            assert ratio == [1]
            continue
        w = ratio[brev(1, l)]  # the factor of exponent 1
        assert pow(w, 1 << l, p) == p - 1  # primitive 2^(l+1)-th root of unity
        assert ratio == [pow(w, brev(g, l), p) for g in range(1 << l)]
