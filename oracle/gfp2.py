"""The ring of section 3.1 (test infrastructure only): Z/p[sqrt 3] with p = 2^31 - 1.

Section 3.1 avoids complex numbers by computing modulo the Mersenne prime p = 2^31 - 1.
Since p + 1 is a power of two, it works in Z/p[sqrt 3], where 2 + sqrt 3 is a generator
(of the roots of unity of two-power order), and takes (2 + sqrt 3)^((p+1)/N) as the N-th
root of unity. 3 is not a square modulo p (p = 7 mod 12), so the ring is the field
GF(p^2); its elements a + b sqrt 3 are pairs (a, b) with a, b in [0, p).

Here: the field operations with Python integers, a ring object for the literal
recursion of ``fcirc.alg1_matvec`` (square roots by Tonelli-Shanks in the multiplicative
group of order p^2 - 1), the dense definition of the f-circulant product, and the
recursion one level at a time in numpy (uint64 with Mersenne reduction) for large n.
"""
from __future__ import annotations

import random

import numpy as np

P = (1 << 31) - 1
ONE = (1, 0)
GEN = (2, 1)  # 2 + sqrt 3
GROUP_ORDER = P * P - 1  # multiplicative group of GF(p^2): 2^32 times an odd number


def add(u, v):
    return ((u[0] + v[0]) % P, (u[1] + v[1]) % P)


def sub(u, v):
    return ((u[0] - v[0]) % P, (u[1] - v[1]) % P)


def neg(u):
    return ((-u[0]) % P, (-u[1]) % P)


def mul(u, v):
    a, b = u
    c, d = v
    return ((a * c + 3 * b * d) % P, (a * d + b * c) % P)


def scale(u, k: int):
    return (u[0] * k % P, u[1] * k % P)


def norm(u) -> int:
    return (u[0] * u[0] - 3 * u[1] * u[1]) % P


def inv(u):
    """(a - b sqrt 3) / (a^2 - 3 b^2)."""
    ni = pow(norm(u), P - 2, P)
    return (u[0] * ni % P, (-u[1]) * ni % P)


def power(u, e: int):
    out, b = ONE, u
    while e:
        if e & 1:
            out = mul(out, b)
        b = mul(b, b)
        e >>= 1
    return out


def root_of_unity(N: int):
    """The paper's N-th root of unity (2 + sqrt 3)^((p+1)/N), N a power of two <= 2^31."""
    assert N & (N - 1) == 0 and (P + 1) % N == 0
    return power(GEN, (P + 1) // N)


def _two_adic():
    s, m = 0, GROUP_ORDER
    while m % 2 == 0:
        m //= 2
        s += 1
    return s, m


S2, ODD = _two_adic()  # p^2 - 1 = 2^S2 * ODD


def _non_square():
    k = 0
    while True:
        z = (k, 1)
        if power(z, GROUP_ORDER // 2) == (P - 1, 0):
            return z
        k += 1


Z_NONSQ = _non_square()


def sqrt(v, rng: random.Random | None = None):
    """A square root of v in GF(p^2) (Tonelli-Shanks in the cyclic group of order
    p^2 - 1); raises ValueError if v is not a square. With rng, the sign is random."""
    if v == (0, 0):
        return (0, 0)
    if power(v, GROUP_ORDER // 2) != ONE:
        raise ValueError("not a square in GF(p^2)")
    M, c, t, x = S2, power(Z_NONSQ, ODD), power(v, ODD), power(v, (ODD + 1) // 2)
    while t != ONE:
        i, t2 = 0, t
        while t2 != ONE:
            t2 = mul(t2, t2)
            i += 1
        b = c
        for _ in range(M - i - 1):
            b = mul(b, b)
        x = mul(x, b)
        c = mul(b, b)
        t = mul(t, c)
        M = i
    assert mul(x, x) == v
    if rng is not None and rng.random() < 0.5:
        x = neg(x)
    return x


class GFp2:
    """GF(p^2) for ``fcirc.alg1_matvec``."""

    def __init__(self, rng: random.Random | None = None):
        self.rng = rng

    add = staticmethod(add)
    sub = staticmethod(sub)
    mul = staticmethod(mul)
    neg = staticmethod(neg)

    def div(self, u, v):
        if isinstance(v, int):
            v = (v % P, 0)
        return mul(u, inv(v))

    def sqrt(self, v):
        return sqrt(v, self.rng)


def dense_matvec(a, x, f):
    """y = A(a, f) x from Definition 2's closed form: A[i][j] = a[j-i] (j >= i), else
    f a[n+j-i]. Python integers, O(n^2)."""
    n = len(a)
    y = []
    for i in range(n):
        s = (0, 0)
        for j in range(n):
            e = a[j - i] if j >= i else mul(f, a[n + j - i])
            s = add(s, mul(e, x[j]))
        y.append(s)
    return y


# ----------------------------------------------------------------------------------
# numpy: arrays of shape (..., 2) of uint64 components in [0, p)
# ----------------------------------------------------------------------------------

def _red(t):
    """t < 2^64 (uint64) -> t mod p, using 2^31 = 1 mod p."""
    t = (t & np.uint64(P)) + (t >> np.uint64(31))
    t = (t & np.uint64(P)) + (t >> np.uint64(31))
    return np.where(t >= np.uint64(P), t - np.uint64(P), t)


def vmul(u, v):
    """Componentwise field product of two arrays (..., 2)."""
    a, b = u[..., 0], u[..., 1]
    c, d = v[..., 0], v[..., 1]
    re = _red(_red(a * c) + np.uint64(3) * _red(b * d))
    im = _red(_red(a * d) + _red(b * c))
    return np.stack([re, im], axis=-1)


def vadd(u, v):
    s = u + v
    return np.where(s >= np.uint64(P), s - np.uint64(P), s)


def vsub(u, v):
    return np.where(u >= v, u - v, u + np.uint64(P) - v)


def _vmulp(x, y):
    return _red(x * y)


def vinv(u):
    """Componentwise inverse (a - b sqrt 3) / (a^2 - 3 b^2) of an array (..., 2)."""
    a, b = u[..., 0], u[..., 1]
    x = _red(a * a)
    y = _red(np.uint64(3) * _red(b * b))
    nrm = np.where(x >= y, x - y, x + np.uint64(P) - y)
    out = np.ones_like(nrm)
    base = nrm.copy()
    e = P - 2
    while e:
        if e & 1:
            out = _vmulp(out, base)
        base = _vmulp(base, base)
        e >>= 1
    nb = np.where(b == 0, b, np.uint64(P) - b)
    return np.stack([_vmulp(a, out), _vmulp(nb, out)], axis=-1)


def vpower(base, exps: np.ndarray):
    """base ** exps (base one element, exps a uint64 array) as an array (len, 2)."""
    exps = exps.astype(np.uint64).copy()
    out = np.zeros((exps.shape[0], 2), dtype=np.uint64)
    out[:, 0] = 1
    b = np.tile(np.array(base, dtype=np.uint64), (exps.shape[0], 1))
    while np.any(exps):
        odd = (exps & np.uint64(1)).astype(bool)
        out = np.where(odd[:, None], vmul(out, b), out)
        b = vmul(b, b)
        exps >>= np.uint64(1)
    return out


def as_array(vals):
    return np.array([[int(v[0]) % P, int(v[1]) % P] for v in vals], dtype=np.uint64).reshape(-1, 2)


# The 2-Sylow subgroup of the multiplicative group is cyclic of order 2^32; GAMMA generates
# it. A node value in it is GAMMA^e; its square roots are GAMMA^(e/2) and GAMMA^(e/2 + 2^31).
GAMMA = power(Z_NONSQ, ODD)


def dlog2(v) -> int:
    """e with GAMMA^e = v for v in the 2-Sylow subgroup (Pohlig-Hellman, bit by bit)."""
    assert power(v, 1 << S2) == ONE
    e = 0
    for k in range(S2):
        # is GAMMA^(-e) v an element whose 2^(S2-1-k)-th power is 1?
        w = mul(v, inv(power(GAMMA, e)))
        if power(w, 1 << (S2 - 1 - k)) != ONE:
            e |= 1 << k
    assert power(GAMMA, e) == v
    return e


def node_roots(n: int, f):
    """Square roots taken at every node, level by level: the node value of (d, b) is
    GAMMA^e; child 2b takes GAMMA^(e/2), child 2b+1 takes -GAMMA^(e/2)."""
    L = n.bit_length() - 1
    e = np.array([dlog2(f)], dtype=np.uint64)
    half = np.uint64(1 << (S2 - 1))
    mask = np.uint64((1 << S2) - 1)
    gs = []
    for _ in range(L):
        assert not np.any(e & np.uint64(1)), "node value without a square root"
        g_e = e >> np.uint64(1)
        gs.append(vpower(GAMMA, g_e))
        e = np.stack([g_e, (g_e + half) & mask], axis=1).reshape(-1)
    return gs


def levels_matvec(a, x, f):
    """Algorithm 1 over GF(p^2), one level at a time; a, x arrays (n, 2) or lists of pairs."""
    A = as_array(a) if not isinstance(a, np.ndarray) else a.astype(np.uint64) % np.uint64(P)
    X = as_array(x) if not isinstance(x, np.ndarray) else x.astype(np.uint64) % np.uint64(P)
    n = A.shape[0]
    if n == 1:
        return vmul(A, X)
    gs = node_roots(n, f)
    L = len(gs)
    for d in range(L):
        m = n >> d
        h = m // 2
        g = gs[d][:, None, :]
        A2 = A.reshape(1 << d, m, 2)
        lo, hi = A2[:, :h], A2[:, h:]
        t = vmul(hi, g)
        A = np.concatenate([vadd(lo, t), vsub(lo, t)], axis=1).reshape(-1, 2)
        X2 = X.reshape(1 << d, m, 2)
        lo, hi = X2[:, :h], X2[:, h:]
        t = vmul(lo, g)
        X = np.concatenate([vadd(t, hi), vsub(t, hi)], axis=1).reshape(-1, 2)
    Y = vmul(A, X)
    inv2 = np.array([pow(2, P - 2, P), 0], dtype=np.uint64)
    for d in reversed(range(L)):
        m = n >> d
        h = m // 2
        inv_2g = vinv(vadd(gs[d], gs[d]))[:, None, :]
        Y2 = Y.reshape(1 << d, m, 2)
        M1, M2 = Y2[:, :h], Y2[:, h:]
        s = vadd(M1, M2)
        c1 = vmul(s, inv_2g)
        c2 = vsub(vmul(s, inv2[None, None, :]), M2)
        Y = np.concatenate([c1, c2], axis=1).reshape(-1, 2)
    return Y


def matvec_entry(a, x, f, i: int):
    """One output y_i of the definition, O(n) with numpy."""
    A = a.astype(np.uint64)
    X = x.astype(np.uint64)
    n = A.shape[0]
    j = np.arange(n)
    k = j - i
    row = A[k % n]
    fa = np.array(f, dtype=np.uint64)
    wrapped = vmul(row, np.broadcast_to(fa, row.shape))
    row = np.where((k >= 0)[:, None], row, wrapped)
    prod = vmul(row, X)
    s0 = int(prod[:, 0].sum() % P)
    s1 = int(prod[:, 1].sum() % P)
    return (s0, s1)
