"""The f-circulant matrix-vector product, written plainly (test infrastructure only).

Conventions fixed by the paper:
* Definition 2 (section 1.2, after Pan) defines an f-circulant n x n matrix by two
  properties: (1) entries repeat down each diagonal, and (2) the entry that wraps from
  the last column of row i to the first column of row i+1 is multiplied by f.
* Section 1.2 then states that matrices are identified by their first ROW, not their
  first column. So the defining vector a is row 1, and the product is A times a column
  vector (Algorithm 1 writes A b with b = (b1, b2)^T).
* Algorithm 1 (section 2, in the proof of Theorem 1) splits A = [[A1, A2], [A2 f, A1]]
  into M1 = (A1 + A2 sqrt f)(b1 sqrt f + b2) and M2 = (A1 - A2 sqrt f)(b1 sqrt f - b2),
  and returns c1 = (M1 + M2) / (2 sqrt f), c2 = (M1 + M2) / 2 - M2. The proof shows that
  A1 + A2 sqrt f is sqrt(f)-circulant and A1 - A2 sqrt f is (-sqrt f)-circulant, so the
  split recurses. The recursion ends at 1 x 1 matrices, whose product is a scalar one.

Everything here works either over Z/p (Python ints, or numpy int64 with products below
2**63) or over the complex numbers (Python complex / numpy complex128).
"""
from __future__ import annotations

import cmath
import random

import numpy as np

from . import ring


# ----------------------------------------------------------------------------------
# O1: the dense definition
# ----------------------------------------------------------------------------------

def fcirc_matrix(a, f, p: int | None = None):
    """The f-circulant matrix with first row a, built from Definition 2's two properties.

    Row 1 is a. Row i+1 is row i shifted one place to the right (property (1)), and its
    first entry is the last entry of row i times f (property (2)). Returns a list of rows
    (Python ints reduced mod p when p is given, else the values' own type).
    """
    n = len(a)
    rows = [list(a)]
    for _ in range(n - 1):
        prev = rows[-1]
        first = prev[n - 1] * f
        if p is not None:
            first %= p
        rows.append([first] + prev[: n - 1])
    if p is not None:
        rows = [[int(v) % p for v in r] for r in rows]
    return rows


def dense_matvec_py(a, x, f, p: int | None = None):
    """y = A x with A = fcirc_matrix(a, f): O(n^2), Python arithmetic."""
    A = fcirc_matrix(a, f, p)
    y = []
    for row in A:
        s = 0
        for aij, xj in zip(row, x):
            s += aij * xj
        y.append(s % p if p is not None else s)
    return y


def fcirc_matrix_np(a, f, p: int | None = None):
    """Closed form of Definition 2 (0-indexed): A[i][j] = a[j-i] if j >= i else f a[n+j-i].

    numpy version of ``fcirc_matrix``, used for n up to a few thousand. The tests pin it
    to the property-by-property builder above.
    """
    a = np.asarray(a)
    n = a.shape[0]
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    k = j - i
    wrap = k < 0
    if p is not None:
        av = a.astype(np.int64) % p
        A = av[np.where(wrap, k + n, k)]
        A = np.where(wrap, A * (int(f) % p) % p, A)
        return A
    av = a.astype(np.complex128) if np.iscomplexobj(a) or np.iscomplexobj(f) else a.astype(np.float64)
    A = av[np.where(wrap, k + n, k)]
    return np.where(wrap, A * f, A)


def dense_matvec_modp(a, x, f, p: int):
    """y = A x over Z/p with numpy int64, exact.

    Entries of A are below 2**30 and x is split into 15-bit halves, so every partial sum
    stays below 2**63 for n up to 2**18.
    """
    A = fcirc_matrix_np(a, f, p)
    xv = np.asarray(x).astype(np.int64) % p
    lo = xv & 0x7FFF
    hi = xv >> 15
    y_lo = (A @ lo) % p
    y_hi = (A @ hi) % p
    return (y_lo + y_hi * (1 << 15)) % p


def dense_matvec_c128(a, x, f=1.0):
    """y = A x in complex128 from the closed-form matrix."""
    A = fcirc_matrix_np(np.asarray(a, dtype=np.complex128), complex(f))
    return A @ np.asarray(x, dtype=np.complex128)


# ----------------------------------------------------------------------------------
# O2: Algorithm 1, literally
# ----------------------------------------------------------------------------------

class ModP:
    """Z/p for the literal recursion; square roots by Tonelli-Shanks."""

    def __init__(self, p: int, rng: random.Random | None = None):
        self.p, self.rng = p, rng

    def add(self, u, v):
        return (u + v) % self.p

    def sub(self, u, v):
        return (u - v) % self.p

    def mul(self, u, v):
        return u * v % self.p

    def div(self, u, v):
        return u * ring.inv(v, self.p) % self.p

    def neg(self, u):
        return (-u) % self.p

    def sqrt(self, v):
        return ring.sqrt_mod(v, self.p, self.rng)


class Complex:
    """The complex field for the literal recursion; principal square roots."""

    def __init__(self, rng: random.Random | None = None):
        self.rng = rng

    add = staticmethod(lambda u, v: u + v)
    sub = staticmethod(lambda u, v: u - v)
    mul = staticmethod(lambda u, v: u * v)
    div = staticmethod(lambda u, v: u / v)
    neg = staticmethod(lambda u: -u)

    def sqrt(self, v):
        r = cmath.sqrt(v)
        if self.rng is not None and self.rng.random() < 0.5:
            r = -r
        return r


def alg1_matvec(a, b, f, R):
    """Algorithm 1 applied recursively: the product of the f-circulant matrix with first
    row a and the column vector b (section 2, Theorem 1 and its proof).

    A1 is the top-left and A2 the top-right n/2 x n/2 block of A, so their first rows are
    the two halves of a. The children A1 +- A2 sqrt f are (+-sqrt f)-circulant and are
    handed down by their first rows. The base case n = 1 is the 1 x 1 product.
    """
    n = len(a)
    if n == 1:
        return [R.mul(a[0], b[0])]
    h = n // 2
    g = R.sqrt(f)  # sqrt f
    a1, a2 = a[:h], a[h:]
    b1, b2 = b[:h], b[h:]
    row_m1 = [R.add(a1[k], R.mul(a2[k], g)) for k in range(h)]  # A1 + A2 sqrt f
    row_m2 = [R.sub(a1[k], R.mul(a2[k], g)) for k in range(h)]  # A1 - A2 sqrt f
    vec_m1 = [R.add(R.mul(b1[k], g), b2[k]) for k in range(h)]  # b1 sqrt f + b2
    vec_m2 = [R.sub(R.mul(b1[k], g), b2[k]) for k in range(h)]  # b1 sqrt f - b2
    M1 = alg1_matvec(row_m1, vec_m1, g, R)          # f' = sqrt f
    M2 = alg1_matvec(row_m2, vec_m2, R.neg(g), R)   # f'' = -sqrt f
    two_g = R.add(g, g)
    c1 = [R.div(R.add(M1[k], M2[k]), two_g) for k in range(h)]
    c2 = [R.sub(R.div(R.add(M1[k], M2[k]), 2), M2[k]) for k in range(h)]
    return c1 + c2


def alg1_children_rows(a, g, R):
    """First rows of the two children A1 + A2 g and A1 - A2 g (proof of Theorem 1)."""
    h = len(a) // 2
    return ([R.add(a[k], R.mul(a[k + h], g)) for k in range(h)],
            [R.sub(a[k], R.mul(a[k + h], g)) for k in range(h)])


def alg1_modp(a, x, f, p, rng: random.Random | None = None):
    return alg1_matvec([int(v) % p for v in a], [int(v) % p for v in x], int(f) % p, ModP(p, rng))


def alg1_c128(a, x, f=1.0, rng: random.Random | None = None):
    return alg1_matvec([complex(v) for v in a], [complex(v) for v in x], complex(f), Complex(rng))


# ----------------------------------------------------------------------------------
# O2 level by level (numpy), for large n
# ----------------------------------------------------------------------------------

def _pow_vec(base: int, exps: np.ndarray, p: int) -> np.ndarray:
    """base ** exps mod p for an int64 array of exponents (square and multiply)."""
    exps = exps.astype(np.int64).copy()
    out = np.ones_like(exps)
    b = np.full_like(exps, base % p)
    while np.any(exps):
        odd = (exps & 1).astype(bool)
        out = np.where(odd, out * b % p, out)
        b = b * b % p
        exps >>= 1
    return out


def _inv_vec(v: np.ndarray, p: int) -> np.ndarray:
    """Elementwise inverse mod p (Fermat), v nonzero."""
    e = p - 2
    out = np.ones_like(v)
    b = v % p
    while e:
        if e & 1:
            out = out * b % p
        b = b * b % p
        e >>= 1
    return out


def node_roots_modp(n: int, f: int, p: int):
    """The square roots taken at every node of the recursion, level by level.

    Theorem 1 assumes an n-th root phi of f and an n-th root of unity w (read as a
    primitive one). Writing a node value at depth d as phi^(n/2^d) w^(e n/2^d), its
    square root is g = phi^(n/2^(d+1)) w^(e n/2^(d+1)); the two children carry +g
    (same e) and -g (e + 2^d, since w^(n/2) = -1). Returns the list of per-level arrays
    g_d (length 2^d, in block order).
    """
    L = n.bit_length() - 1
    phi = ring.nth_root_pow2(f, n, p)
    w = ring.root_of_unity(n, p)
    e = np.zeros(1, dtype=np.int64)
    gs = []
    for d in range(L):
        h = n >> (d + 1)
        g = pow(phi, h, p) * _pow_vec(pow(w, h, p), e, p) % p
        gs.append(g)
        e = np.stack([e, e + (1 << d)], axis=1).reshape(-1)
    return gs


def levels_matvec_modp(a, x, f, p: int, gs=None):
    """Algorithm 1 over Z/p, one recursion level at a time on whole arrays.

    At depth d the vector holds 2^d independent subproblems of size m = n/2^d, child
    2b in the low half and child 2b+1 in the high half of block b. Split (per block, with
    that block's sqrt g): row -> (lo + g hi, lo - g hi), vector -> (g lo + hi, g lo - hi).
    At the leaves (1 x 1) multiply. Merge back up: c1 = (M1+M2)/(2g), c2 = (M1+M2)/2 - M2.
    Exact with int64 since every product is of two residues below 2**30.
    """
    A = np.asarray(a).astype(np.int64) % p
    X = np.asarray(x).astype(np.int64) % p
    n = A.shape[0]
    f = int(f) % p
    if n == 1:
        return A * X % p
    if gs is None:
        gs = node_roots_modp(n, f, p)
    L = len(gs)
    for d in range(L):
        m = n >> d
        h = m // 2
        g = gs[d][:, None]
        A2 = A.reshape(1 << d, m)
        lo, hi = A2[:, :h], A2[:, h:]
        t = hi * g % p
        A = np.concatenate([(lo + t) % p, (lo - t) % p], axis=1).reshape(-1)
        X2 = X.reshape(1 << d, m)
        lo, hi = X2[:, :h], X2[:, h:]
        t = lo * g % p
        X = np.concatenate([(t + hi) % p, (t - hi) % p], axis=1).reshape(-1)
    Y = A * X % p
    inv2 = ring.inv(2, p)
    for d in reversed(range(L)):
        m = n >> d
        h = m // 2
        inv_2g = _inv_vec(2 * gs[d] % p, p)[:, None]
        Y2 = Y.reshape(1 << d, m)
        M1, M2 = Y2[:, :h], Y2[:, h:]
        s = (M1 + M2) % p
        c1 = s * inv_2g % p
        c2 = (s * inv2 - M2) % p
        Y = np.concatenate([c1, c2], axis=1).reshape(-1)
    return Y


def levels_matvec_c128(a, x, f=1.0):
    """Algorithm 1 over the complex numbers, level by level in complex128.

    The square root at each node is numpy's principal root of that node's value; the
    children carry +g and -g.
    """
    A = np.asarray(a, dtype=np.complex128).copy()
    X = np.asarray(x, dtype=np.complex128).copy()
    n = A.shape[0]
    F = np.array([complex(f)], dtype=np.complex128)
    gs = []
    L = n.bit_length() - 1
    for d in range(L):
        m = n >> d
        h = m // 2
        g = np.sqrt(F)
        gs.append(g)
        gc = g[:, None]
        A2 = A.reshape(1 << d, m)
        lo, hi = A2[:, :h], A2[:, h:]
        A = np.concatenate([lo + gc * hi, lo - gc * hi], axis=1).reshape(-1)
        X2 = X.reshape(1 << d, m)
        lo, hi = X2[:, :h], X2[:, h:]
        X = np.concatenate([gc * lo + hi, gc * lo - hi], axis=1).reshape(-1)
        F = np.stack([g, -g], axis=1).reshape(-1)
    Y = A * X
    for d in reversed(range(L)):
        m = n >> d
        h = m // 2
        gc = gs[d][:, None]
        Y2 = Y.reshape(1 << d, m)
        M1, M2 = Y2[:, :h], Y2[:, h:]
        Y = np.concatenate([(M1 + M2) / (2 * gc), (M1 + M2) / 2 - M2], axis=1).reshape(-1)
    return Y


def cyclic_matvec_fft_c128(a, x):
    """The f = 1 product through the discrete Fourier transform, in complex128.

    Section 1.2 recalls that a circulant is diagonalised by the DFT (A = F^-1 diag(F a) F
    for the usual column convention). For the row convention used here,
    y_i = sum_k a_k x_((i+k) mod n), which is ifft(conj(fft(conj(a))) * fft(x)). The pins
    tie this identity to the recursion of Algorithm 1 at several sizes.
    """
    a = np.asarray(a, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128)
    return np.fft.ifft(np.conj(np.fft.fft(np.conj(a))) * np.fft.fft(x))


def matvec_modp(a, x, f, p: int):
    """y = A(a, f) x over Z/p: dense definition for small n, else the level form."""
    n = len(a)
    if n <= 2048:
        return dense_matvec_modp(a, x, f, p)
    return levels_matvec_modp(a, x, f, p)


def matvec_c128(a, x, f=1.0):
    n = len(a)
    if n <= 1024:
        return dense_matvec_c128(a, x, f)
    return levels_matvec_c128(a, x, f)


def matvec_entry_modp(a, x, f, p: int, i: int) -> int:
    """One output y_i of the dense definition, O(n): sum_j A[i][j] x_j with
    A[i][j] = a[j-i] (j >= i) else f a[n+j-i]. Used to check sampled outputs at sizes
    where the full product is too slow on the CPU."""
    av = np.asarray(a).astype(np.int64) % p
    xv = np.asarray(x).astype(np.int64) % p
    n = av.shape[0]
    j = np.arange(n)
    k = j - i
    row = np.where(k >= 0, av[k % n], av[k % n] * (int(f) % p) % p)
    lo = int(((row * (xv & 0x7FFF)) % p).sum() % p)
    hi = int(((row * (xv >> 15)) % p).sum() % p)
    return (lo + hi * (1 << 15)) % p
