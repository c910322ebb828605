"""Algorithm 1 over Z/(2^K + 1), the ring of section 3.2 (test infrastructure only).

Section 3.2 applies Algorithm 1 to Schoenhage-Strassen multiplication: the pieces of two
large integers are coefficients of two polynomials over a ring Z/(2^K + 1), in which the
roots of unity are powers of two, so a multiplication by a root is a shift and the
roots need not be computed, only the shift counts. The polynomial product is then one
circulant product of Algorithm 1, with the pointwise products computed by any method.

In Z/(2^K + 1), 2^K = -1, so 2 has order 2K and every power of two 2^e (0 <= e < 2K) is
a unit whose square roots include 2^(e/2) and -2^(e/2) = 2^(e/2 + K) when e is even.
Algorithm 1 over this ring therefore only needs f = 2^e with e even at every level of
the recursion: here the square root of a node value is taken among powers of two, and a
node value with an odd exponent has no such root (ValueError).

Functions:
  * ``Fermat``: the ring for ``fcirc.alg1_matvec`` (literal recursion, random root choice).
  * ``dense_matvec``: Definition 2 written out with Python integers.
  * ``node_exponents`` / ``levels_matvec``: the recursion one level at a time, roots as
    shift counts (Python integers; every multiplication by a root is a multiplication
    by pow(2, e, M), not a shift, so it does not share the shift logic it checks).
  * ``bigint_pieces`` / ``bigint_recompose`` / ``bigint_mul_ssa``: the large-integer
    product of section 3.2 through one cyclic product (f = 1, zero-padded so nothing
    wraps), for comparison with Python's own integer product.
"""
from __future__ import annotations

import random


def modulus(K: int) -> int:
    return (1 << K) + 1


class Fermat:
    """Z/(2^K + 1) for ``fcirc.alg1_matvec``; square roots among +-powers of two."""

    def __init__(self, K: int, rng: random.Random | None = None):
        self.K = K
        self.M = modulus(K)
        self.rng = rng
        self._log = {pow(2, e, self.M): e for e in range(2 * K)}

    def add(self, u, v):
        return (u + v) % self.M

    def sub(self, u, v):
        return (u - v) % self.M

    def mul(self, u, v):
        return u * v % self.M

    def neg(self, u):
        return (-u) % self.M

    def div(self, u, v):
        return u * pow(v % self.M, -1, self.M) % self.M

    def log2(self, v) -> int:
        """e in [0, 2K) with 2^e = v, or ValueError if v is not a power of two."""
        try:
            return self._log[v % self.M]
        except KeyError:
            raise ValueError("not a power of two in Z/(2^K + 1)") from None

    def sqrt(self, v):
        e = self.log2(v)
        if e % 2:
            raise ValueError("odd exponent: no power-of-two square root")
        h = e // 2
        if self.rng is not None and self.rng.random() < 0.5:
            h += self.K  # the other root, -2^(e/2)
        return pow(2, h, self.M)


def dense_matvec(a, x, f, K: int):
    """y = A(a, f) x from Definition 2: A[i][j] = a[j-i] (j >= i), else f a[n+j-i]."""
    M = modulus(K)
    n = len(a)
    y = []
    for i in range(n):
        s = 0
        for j in range(n):
            e = a[j - i] if j >= i else f * a[n + j - i]
            s += e * x[j]
        y.append(s % M)
    return y


def node_exponents(L: int, f_exp: int, K: int):
    """Shift counts of the node values, level by level: node (0, 0) holds f = 2^f_exp; the
    children of a node 2^e are 2^(e/2) (first child) and -2^(e/2) = 2^(e/2 + K)."""
    levels = [[f_exp % (2 * K)]]
    for _ in range(L):
        nxt = []
        for e in levels[-1]:
            if e % 2:
                raise ValueError("odd exponent: no power-of-two square root")
            nxt += [e // 2, (e // 2 + K) % (2 * K)]
        levels.append(nxt)
    return levels


def levels_matvec(a, x, f_exp: int, K: int):
    """Algorithm 1 over Z/(2^K + 1), one level at a time; f = 2^f_exp."""
    M = modulus(K)
    A = [int(v) % M for v in a]
    X = [int(v) % M for v in x]
    n = len(A)
    L = n.bit_length() - 1
    assert 1 << L == n
    nodes = node_exponents(L, f_exp, K)
    for d in range(L):
        m = n >> d
        h = m // 2
        for b in range(1 << d):
            g = pow(2, nodes[d + 1][2 * b], M)  # the root used at node (d, b)
            for k in range(b * m, b * m + h):
                u, v = A[k], A[k + h]
                A[k], A[k + h] = (u + g * v) % M, (u - g * v) % M
                u, v = X[k], X[k + h]
                X[k], X[k + h] = (g * u + v) % M, (g * u - v) % M
    Y = [A[k] * X[k] % M for k in range(n)]
    inv2 = pow(2, -1, M)
    for d in reversed(range(L)):
        m = n >> d
        h = m // 2
        for b in range(1 << d):
            g = pow(2, nodes[d + 1][2 * b], M)
            inv_2g = pow(2 * g, -1, M)
            for k in range(b * m, b * m + h):
                m1, m2 = Y[k], Y[k + h]
                s = m1 + m2
                Y[k], Y[k + h] = s * inv_2g % M, (s * inv2 - m2) % M
    return Y


def bigint_pieces(v: int, P: int, N: int):
    """v as N pieces of P bits (least significant first); v must fit."""
    assert v >= 0 and v.bit_length() <= P * N
    mask = (1 << P) - 1
    return [(v >> (P * j)) & mask for j in range(N)]


def bigint_recompose(c, P: int) -> int:
    return sum(int(cj) << (P * j) for j, cj in enumerate(c))


def bigint_mul_ssa(u: int, v: int, P: int, N: int, K: int) -> int:
    """u v through one cyclic product of length N over Z/(2^K + 1) (section 3.2).

    The row convention makes the product a correlation, so the defining row is the
    reversed piece vector r_k = a_((-k) mod N); the pieces of u and v together must fit
    in N pieces (no wrap), and every coefficient must stay below 2^K."""
    na, nb = max(1, -(-u.bit_length() // P)), max(1, -(-v.bit_length() // P))
    assert na + nb - 1 <= N, "the product must fit in N pieces"
    assert min(na, nb) << (2 * P) < 1 << K, "a coefficient must stay below 2^K"
    a = bigint_pieces(u, P, N)
    b = bigint_pieces(v, P, N)
    r = [a[(-k) % N] for k in range(N)]
    c = levels_matvec(r, b, 0, K)
    return bigint_recompose(c, P)


def matvec_entry(a, x, f, K: int, i: int) -> int:
    """One output y_i of Definition 2 over Z/(2^K + 1), O(n) big-integer products."""
    M = modulus(K)
    n = len(a)
    s = 0
    for j in range(n):
        e = a[j - i] if j >= i else f * a[n + j - i]
        s += e * x[j]
    return s % M
