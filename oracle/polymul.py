"""Integer polynomial multiplication (section 3.1), written plainly (test infrastructure only).

Section 3.1 multiplies two integer polynomials as a circulant matrix-vector product of
power-of-two size, after filling the inputs up (Corollary 1). The paper computes modulo
one prime; here the exact integer product is recovered from three primes by the
Chinese remainder theorem, the textbook construction (sum of r_i M_i (M_i^-1 mod p_i)).

Readings (the paper is silent or garbled here):
* The cyclic length is the smallest power of two >= deg a + deg b + 1 (the paper's
  "N = (d_a + 1)(d_b + 1) - 1" counts coefficients wrongly; a product of polynomials with
  na and nb coefficients has na + nb - 1 of them).
* "In a natural way": the matrix row is the index-reversed first polynomial,
  r_k = a_((-k) mod N), and the vector is the second one. Then (C(r) b)_i is the cyclic
  convolution sum_j a_j b_((i-j) mod N).
* A signed coefficient v is taken to the residue v mod p in [0, p).
"""
from __future__ import annotations

import numpy as np

from .fcirc import levels_matvec_modp, dense_matvec_modp


def poly_schoolbook(a, b):
    """c_k = sum_{i+j=k} a_i b_j with Python integers, O(na nb)."""
    a = [int(v) for v in a]
    b = [int(v) for v in b]
    c = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j, bj in enumerate(b):
            c[i + j] += ai * bj
    return c


def poly_kronecker(a, b, offset: int = 1 << 15, slot_bits: int = 64):
    """Exact product by Kronecker substitution with Python big integers.

    Coefficients are shifted by ``offset`` to be non-negative, packed into ``slot_bits``
    slots of one integer each, multiplied by Python's integer multiply, unpacked, and the
    shift is removed with the closed form
        a*b = (a+o)*(b+o) - o*(a conv 1_nb) - o*(1_na conv b) - o^2 (1_na conv 1_nb).
    Needs every shifted product coefficient below 2**slot_bits.
    """
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    na, nb = a.shape[0], b.shape[0]
    nbytes = slot_bits // 8
    sa = (a + offset).astype(np.uint64)
    sb = (b + offset).astype(np.uint64)
    A = int.from_bytes(sa.astype("<u8").tobytes(), "little")
    B = int.from_bytes(sb.astype("<u8").tobytes(), "little")
    C = A * B
    nc = na + nb - 1
    raw = np.frombuffer(C.to_bytes(nc * nbytes, "little"), dtype="<u8").astype(np.int64)
    # sliding sums: (a conv 1_nb)_k = sum_{i = max(0, k-nb+1)}^{min(k, na-1)} a_i
    k = np.arange(nc)
    pa = np.concatenate([[0], np.cumsum(a)])
    pb = np.concatenate([[0], np.cumsum(b)])
    a_hi = np.minimum(k, na - 1) + 1
    a_lo = np.maximum(0, k - nb + 1)
    sum_a = pa[a_hi] - pa[a_lo]
    b_hi = np.minimum(k, nb - 1) + 1
    b_lo = np.maximum(0, k - na + 1)
    sum_b = pb[b_hi] - pb[b_lo]
    count = a_hi - a_lo
    return raw - offset * sum_a - offset * sum_b - offset * offset * count


def cyclic_length(na: int, nb: int) -> int:
    m = na + nb - 1
    N = 1
    while N < m:
        N *= 2
    return N


def circulant_row_and_vector(a, b, N: int):
    """(r, x) with r_k = a_((-k) mod N) and x = b, both zero-filled to length N."""
    ap = np.zeros(N, dtype=np.int64)
    ap[: len(a)] = np.asarray(a, dtype=np.int64)
    x = np.zeros(N, dtype=np.int64)
    x[: len(b)] = np.asarray(b, dtype=np.int64)
    r = ap[(-np.arange(N)) % N]
    return r, x


def poly_residues(a, b, p: int):
    """The product's coefficients mod p through one circulant product of length N."""
    N = cyclic_length(len(a), len(b))
    r, x = circulant_row_and_vector(a, b, N)
    r %= p
    x %= p
    if N <= 1024:
        y = dense_matvec_modp(r, x, 1, p)
    else:
        y = levels_matvec_modp(r, x, 1, p)
    return y[: len(a) + len(b) - 1]


def crt_textbook(residues, primes):
    """Signed integers from residues: the CRT sum, then the symmetric lift (-M/2, M/2]."""
    M = 1
    for q in primes:
        M *= q
    terms = []
    for q in primes:
        Mq = M // q
        terms.append((Mq, Mq * pow(Mq % q, q - 2, q)))
    out = []
    for vals in zip(*[np.asarray(r).tolist() for r in residues]):
        c = 0
        for v, (_, coef) in zip(vals, terms):
            c += int(v) * coef
        c %= M
        if c > M // 2:
            c -= M
        out.append(c)
    return out


def poly_via_circulant(a, b, primes):
    """Exact product: one circulant product per prime, then the CRT."""
    return crt_textbook([poly_residues(a, b, q) for q in primes], primes)


def poly_coef(a, b, k: int) -> int:
    """c_k = sum_i a_i b_(k-i) of the polynomial product, O(n) in int64; refuses inputs
    whose partial sums could leave int64."""
    av = np.asarray(a).astype(np.int64)
    bv = np.asarray(b).astype(np.int64)
    bound = int(np.abs(av).max(initial=0)) * int(np.abs(bv).max(initial=0)) * min(len(av), len(bv))
    if bound >= 1 << 62:
        raise ValueError("inputs too large for an int64 coefficient")
    lo, hi = max(0, k - (len(bv) - 1)), min(k, len(av) - 1)
    if lo > hi:
        return 0
    return int((av[lo:hi + 1] * bv[k - hi:k - lo + 1][::-1]).sum())
