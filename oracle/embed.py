"""Products of any size n through one power-of-two cyclic product (test infrastructure only).

Corollary 1 (section 2): for an n x n circulant A with first row (a_1, ..., a_n) and n not
a power of two, let 2^d be the smallest power of two above n and N = 2^(d+1); with the row
a' = (a_1, ..., a_n, 0, ..., 0, a_2, ..., a_n) and the vector b' = (b, 0, ..., 0) of
length N, the first n entries of A' b' (A' the circulant with first row a') are A b.

The introduction recalls that a Toeplitz product is a circulant product the same way.
With T[i][j] = t_(j-i) (0-indexed; first row t_0 .. t_(n-1), first column t_0, t_-1, ...,
t_-(n-1)), the row (t_0, ..., t_(n-1), 0, ..., 0, t_-(n-1), ..., t_-1) of any length
N >= 2n - 1 works: entry (i, j) of the cyclic matrix is row'[(j - i) mod N], which is
t_(j-i) for j >= i and row'[N - (i - j)] = t_-(i-j) for j < i. An f-circulant is the
Toeplitz matrix with t_-m = f a_(n-m) (Definition 2: the entry that wraps is times f),
which gives the corollary's row for f = 1.

Functions follow these definitions; the pins compare them with the dense definitions
and a library routine (scipy.linalg.toeplitz).
"""
from __future__ import annotations

import numpy as np

from . import fcirc as O


def toeplitz_matrix(row, col, p: int | None = None):
    """T[i][j] = row[j - i] for j >= i, col[i - j] for j < i (col[0] unused), as lists."""
    n = len(row)
    T = [[row[j - i] if j >= i else col[i - j] for j in range(n)] for i in range(n)]
    if p is not None:
        T = [[int(v) % p for v in r] for r in T]
    return T


def toeplitz_matvec_dense(row, col, x, p: int | None = None):
    """y = T x from the definition, O(n^2): exact over Z/p (numpy int64 with x split in
    15-bit halves), complex128 otherwise."""
    n = len(row)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    k = j - i
    if p is not None:
        r = np.asarray(row).astype(np.int64) % p
        c = np.asarray(col).astype(np.int64) % p
        T = np.where(k >= 0, r[np.clip(k, 0, n - 1)], c[np.clip(-k, 0, n - 1)])
        xv = np.asarray(x).astype(np.int64) % p
        return ((T @ (xv & 0x7FFF)) % p + ((T @ (xv >> 15)) % p) * (1 << 15)) % p
    r = np.asarray(row, dtype=np.complex128)
    c = np.asarray(col, dtype=np.complex128)
    T = np.where(k >= 0, r[np.clip(k, 0, n - 1)], c[np.clip(-k, 0, n - 1)])
    return T @ np.asarray(x, dtype=np.complex128)


def cyclic_length(n: int) -> int:
    """Smallest power of two >= 2n - 1 (for n not a power of two: the corollary's N)."""
    N = 1
    while N < 2 * n - 1:
        N *= 2
    return N


def corollary_length(n: int) -> int:
    """The corollary's N = 2^(d+1) with 2^d the smallest power of two above n."""
    d = 0
    while (1 << d) <= n:
        d += 1
    return 1 << (d + 1)


def embedded_row(row, col, N: int):
    """(t_0, ..., t_(n-1), 0, ..., 0, t_-(n-1), ..., t_-1) of length N."""
    n = len(row)
    assert N >= 2 * n - 1
    tail = [col[m] for m in range(n - 1, 0, -1)]  # positions N-(n-1) .. N-1 hold t_-(n-1) .. t_-1
    return list(row) + [0] * (N - 2 * n + 1) + tail


def fcirc_col(a, f, p: int | None = None):
    """First column of the f-circulant with first row a: col[m] = f a[n - m] (m >= 1)."""
    n = len(a)
    col = [a[0]] + [f * a[n - m] for m in range(1, n)]
    if p is not None:
        col = [int(v) % p for v in col]
    return col


def toeplitz_matvec_modp(row, col, x, p: int):
    """T x over Z/p through the embedding and one cyclic product (Algorithm 1, f = 1)."""
    n = len(row)
    N = cyclic_length(n)
    rp = np.array([int(v) % p for v in embedded_row(list(row), list(col), N)], dtype=np.int64)
    xp = np.zeros(N, dtype=np.int64)
    xp[:n] = np.asarray(x).astype(np.int64) % p
    return np.asarray(O.matvec_modp(rp, xp, 1, p), dtype=np.int64)[:n]


def toeplitz_matvec_c128(row, col, x):
    """T x in complex128 through the embedding and one cyclic product."""
    n = len(row)
    N = cyclic_length(n)
    rp = np.asarray(embedded_row(list(np.asarray(row, dtype=np.complex128)), list(np.asarray(col, dtype=np.complex128)),
                                 N), dtype=np.complex128)
    xp = np.zeros(N, dtype=np.complex128)
    xp[:n] = np.asarray(x, dtype=np.complex128)
    if N <= 1024:
        return O.dense_matvec_c128(rp, xp, 1.0)[:n]
    return O.cyclic_matvec_fft_c128(rp, xp)[:n]


def fcirc_any_matvec_modp(a, x, f, p: int):
    """A(a, f) x over Z/p for any n (Corollary 1 with the f-wrapped column)."""
    return toeplitz_matvec_modp(a, fcirc_col(list(np.asarray(a).astype(np.int64)), int(f) % p, p), x, p)


def fcirc_any_matvec_c128(a, x, f=1.0):
    a = np.asarray(a, dtype=np.complex128)
    return toeplitz_matvec_c128(a, fcirc_col(list(a), complex(f)), x)


def toeplitz_entry_modp(row, col, x, p: int, i: int) -> int:
    """One output y_i = sum_j t_(j-i) x_j of the Toeplitz definition (t_k = row[k] for
    k >= 0, col[-k] for k < 0), O(n), for sampled checks at large n."""
    r = np.asarray(row).astype(np.int64) % p
    c = np.asarray(col).astype(np.int64) % p
    xv = np.asarray(x).astype(np.int64) % p
    n = r.shape[0]
    j = np.arange(n)
    k = j - i
    t = np.where(k >= 0, r[np.clip(k, 0, n - 1)], c[np.clip(-k, 0, n - 1)])
    lo = int(((t * (xv & 0x7FFF)) % p).sum() % p)
    hi = int(((t * (xv >> 15)) % p).sum() % p)
    return (lo + hi * (1 << 15)) % p
