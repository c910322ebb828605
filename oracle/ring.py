"""Z/p helpers for the oracle (test infrastructure only).

Theorem 1 (section 2) needs, in the ring R: an n-th root of f, an n-th root of unity,
and the inverses of 2 and of f. For R = Z/p these are found here with textbook
number theory on Python integers: trial-division factoring of p - 1, a primitive-root
search, Tonelli-Shanks square roots, and repeated square roots for n-th roots.
"""
from __future__ import annotations

import random


def inv(v: int, p: int) -> int:
    """Multiplicative inverse modulo the prime p (Fermat)."""
    v %= p
    if v == 0:
        raise ZeroDivisionError("0 has no inverse")
    return pow(v, p - 2, p)


def prime_factors(m: int) -> list[int]:
    """Distinct prime factors of m by trial division."""
    out, d = [], 2
    while d * d <= m:
        if m % d == 0:
            out.append(d)
            while m % d == 0:
                m //= d
        d += 1 if d == 2 else 2
    if m > 1:
        out.append(m)
    return out


def primitive_root(p: int) -> int:
    """Smallest generator of (Z/p)^*: g^((p-1)/q) != 1 for every prime q | p - 1."""
    qs = prime_factors(p - 1)
    for g in range(2, p):
        if all(pow(g, (p - 1) // q, p) != 1 for q in qs):
            return g
    raise ValueError("no primitive root")


def is_square(v: int, p: int) -> bool:
    """Euler's criterion."""
    v %= p
    return v == 0 or pow(v, (p - 1) // 2, p) == 1


def sqrt_mod(v: int, p: int, rng: random.Random | None = None) -> int:
    """A square root of v modulo the odd prime p (Tonelli-Shanks).

    Returns one of the two roots; with ``rng`` the branch is picked at random, which the
    tests use to show that the product does not depend on which root is taken.
    Raises ValueError when v is not a square.
    """
    v %= p
    if v == 0:
        return 0
    if not is_square(v, p):
        raise ValueError(f"{v} is not a square mod {p}")
    q, s = p - 1, 0
    while q % 2 == 0:
        q //= 2
        s += 1
    z = 2
    while is_square(z, p):
        z += 1
    m, c, t, r = s, pow(z, q, p), pow(v, q, p), pow(v, (q + 1) // 2, p)
    while t != 1:
        i, t2 = 0, t
        while t2 != 1:
            t2 = t2 * t2 % p
            i += 1
        b = pow(c, 1 << (m - i - 1), p)
        m, c, t, r = i, b * b % p, t * b * b % p, r * b % p
    assert r * r % p == v
    if rng is not None and rng.random() < 0.5:
        r = (p - r) % p
    return r


def nth_root_pow2(f: int, n: int, p: int) -> int:
    """An n-th root of f (n a power of two) by log2(n) successive square roots.

    Any branch works once Z/p holds a primitive n-th root of unity: if phi**n = f then
    both square roots of f have an (n/2)-th root.
    """
    r = f % p
    m = n
    while m > 1:
        r = sqrt_mod(r, p)
        m //= 2
    assert pow(r, n, p) == f % p
    return r


def root_of_unity(n: int, p: int) -> int:
    """A primitive n-th root of unity mod p (requires n | p - 1)."""
    if (p - 1) % n:
        raise ValueError(f"no primitive {n}-th root of unity mod {p}")
    w = pow(primitive_root(p), (p - 1) // n, p)
    assert pow(w, n, p) == 1 and (n == 1 or pow(w, n // 2, p) != 1)
    return w


def has_nth_root(f: int, n: int, p: int) -> bool:
    """Whether f is an n-th power in Z/p (n | p - 1 assumed)."""
    f %= p
    if f == 0:
        return False
    return pow(f, (p - 1) // n, p) == 1
