"""Seeded synthetic inputs for every workload the library is tested and measured on.

This module only draws random numbers. It holds none of the method's arithmetic, so
both the CPU oracle checks and the GPU path can take their inputs from it without
sharing any computation. Every generator uses ``numpy.random.default_rng(seed)``
(PCG64) and returns host numpy arrays.

Workloads (sizes as measured):

* ``modp_pair``: one f-circulant product over Z/p, defining row ``a`` and vector
  ``x`` uniform in [0, p) as uint32. The n = 1024 case with f = 1 and f = p - 1 is the
  small exactness case; n = 2**21 with p = 998244353 is the headline product.
* ``poly_i32``: two integer polynomials of 2**20 coefficients uniform in
  [-2**15, 2**15) (int32), multiplied exactly (cyclic length 2**21).
* ``bigint_u16``: two 2**24-bit integers as 2**20 little-endian uint16 limbs with
  uniform bits (leading zero limbs allowed).
* ``batched_c64``: 4096 complex64 instances whose lengths are 2**e with e uniform on
  {6, ..., 16}; real and imaginary parts i.i.d. N(0, 1).
* ``circ_layer_f32``: a shared defining row a in R**(2**14), a batch of 256 vectors x
  and 256 upstream gradients, all float32 N(0, 1).

The paper's own benchmark inputs (its polynomial-multiplication timing in section 3.1)
were not published; these seeded draws stand in for them.
"""
from __future__ import annotations

import numpy as np

P1 = 998244353
P2 = 469762049
P3 = 167772161
PRIMES = (P1, P2, P3)

SEED_C1_CYCLIC = 1
SEED_C1_NEGACYCLIC = 2
SEED_HEADLINE = 3
SEED_POLY = 4
SEED_BIGINT = 5
SEED_BATCHED = 6
SEED_LAYER = 7


def modp_pair(n: int, p: int = P1, seed: int = SEED_HEADLINE):
    """(a, x): two uint32 vectors of length n, uniform in [0, p)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, p, n, dtype=np.uint32)
    x = rng.integers(0, p, n, dtype=np.uint32)
    return a, x


def modp_batch(count: int, n: int, p: int = P1, seed: int = 11):
    """(a, x): two uint32 arrays of shape (count, n), uniform in [0, p)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, p, (count, n), dtype=np.uint32)
    x = rng.integers(0, p, (count, n), dtype=np.uint32)
    return a, x


def poly_i32(n: int = 1 << 20, seed: int = SEED_POLY, lo: int = -(1 << 15), hi: int = 1 << 15):
    """(a, b): two int32 coefficient vectors of length n, uniform in [lo, hi)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(lo, hi, n, dtype=np.int32)
    b = rng.integers(lo, hi, n, dtype=np.int32)
    return a, b


def bigint_u16(nlimbs: int = 1 << 20, seed: int = SEED_BIGINT):
    """(a, b): two uint16 little-endian limb vectors of length nlimbs, uniform bits."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 1 << 16, nlimbs, dtype=np.uint16)
    b = rng.integers(0, 1 << 16, nlimbs, dtype=np.uint16)
    return a, b


def batched_sizes(count: int = 4096, seed: int = SEED_BATCHED, emin: int = 6, emax: int = 16):
    """log2 of each instance length: uniform integers on {emin, ..., emax}."""
    rng = np.random.default_rng(seed)
    return rng.integers(emin, emax + 1, count)


def batched_c64(count: int = 4096, seed: int = SEED_BATCHED, emin: int = 6, emax: int = 16):
    """(log2n, a_list, x_list): complex64 instances with N(0,1) real and imaginary parts.

    The size draw uses the same stream as ``batched_sizes`` so the two agree.
    """
    rng = np.random.default_rng(seed)
    e = rng.integers(emin, emax + 1, count)
    a_list, x_list = [], []
    for k in range(count):
        n = 1 << int(e[k])
        a = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
        x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
        a_list.append(a)
        x_list.append(x)
    return e, a_list, x_list


def complex_pair(n: int, seed: int = 21):
    """(a, x): complex64 vectors of length n with N(0,1) real and imaginary parts."""
    rng = np.random.default_rng(seed)
    a = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)).astype(np.complex64)
    return a, x


def circ_layer_f32(batch: int = 256, n: int = 1 << 14, seed: int = SEED_LAYER):
    """(a, x, g): shared row a (n,), inputs x (batch, n), upstream gradient g (batch, n)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((batch, n), dtype=np.float32)
    g = rng.standard_normal((batch, n), dtype=np.float32)
    a = rng.standard_normal(n, dtype=np.float32)
    return a, x, g
