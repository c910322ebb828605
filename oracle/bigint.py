"""Large-integer multiplication (section 3.2 application), plainly (test infrastructure only).

Section 3.2 proposes Algorithm 1 for multiplying large integers. Here an integer is a
little-endian vector of 16-bit limbs; the product of na and nb limbs always has
na + nb limbs (leading zeros kept).
"""
from __future__ import annotations

import numpy as np

from .polymul import crt_textbook, poly_residues


def limbs_to_int(limbs) -> int:
    return int.from_bytes(np.asarray(limbs, dtype="<u2").tobytes(), "little")


def int_to_limbs(v: int, nlimbs: int) -> np.ndarray:
    return np.frombuffer(v.to_bytes(2 * nlimbs, "little"), dtype="<u2").astype(np.uint16)


def bigint_mul_pyint(a, b) -> np.ndarray:
    """The product by Python's own integer multiply."""
    return int_to_limbs(limbs_to_int(a) * limbs_to_int(b), len(a) + len(b))


def carry_propagate(coeffs, nlimbs: int) -> np.ndarray:
    """Limbs of sum_k c_k 2^(16k) for non-negative integer coefficients c_k, one limb at a
    time with a running carry (Python integers)."""
    out = np.zeros(nlimbs, dtype=np.uint16)
    carry = 0
    coeffs = [int(c) for c in coeffs]
    for k in range(nlimbs):
        v = carry + (coeffs[k] if k < len(coeffs) else 0)
        out[k] = v & 0xFFFF
        carry = v >> 16
    if carry:
        raise OverflowError("product does not fit in the limb count")
    return out


def bigint_mul_via_circulant(a, b, primes) -> np.ndarray:
    """Convolution of the limb vectors through circulant products mod three primes,
    the CRT, then carries."""
    res = [poly_residues(np.asarray(a, np.int64), np.asarray(b, np.int64), q) for q in primes]
    c = crt_textbook(res, primes)
    return carry_propagate(c, len(a) + len(b))
