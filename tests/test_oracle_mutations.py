"""Plant plausible mistakes in the oracle (on the CPU, via monkeypatch) and check that the
pins catch every one of them: a dropped term, a wrong sign, a wrong index, a transposed
operand, a wrong root."""
import random

import numpy as np
import pytest

from oracle import fcirc as O
from oracle import ring

P = 998244353


def _pins_pass() -> bool:
    """A compact re-run of the pins: closed form at n = 2, brute force and FFT at larger n."""
    rng = random.Random(0)
    try:
        for _ in range(3):
            a0, a1, x0, x1 = (rng.randrange(P) for _ in range(4))
            f = pow(rng.randrange(2, P), 2, P)
            want = [(a0 * x0 + a1 * x1) % P, (f * a1 * x0 + a0 * x1) % P]
            if O.alg1_modp([a0, a1], [x0, x1], f, P) != want:
                return False
            if O.levels_matvec_modp([a0, a1], [x0, x1], f, P).tolist() != want:
                return False
        n = 16
        a = [rng.randrange(64) for _ in range(n)]
        x = [rng.randrange(64) for _ in range(n)]
        cyc = [sum(a[k] * x[(i + k) % n] for k in range(n)) % P for i in range(n)]
        neg = [sum(a[k] * x[(i + k) % n] * (-1 if i + k >= n else 1) for k in range(n)) % P
               for i in range(n)]
        for f, want in ((1, cyc), (P - 1, neg)):
            if O.alg1_modp(a, x, f, P) != want:
                return False
            if O.levels_matvec_modp(a, x, f, P).tolist() != want:
                return False
            if O.dense_matvec_modp(a, x, f, P).tolist() != want:
                return False
        return O.fcirc_matrix([10, 100, 1000], 7) == [[10, 100, 1000], [7000, 10, 100], [700, 7000, 10]]
    except (ValueError, AssertionError, ZeroDivisionError):
        return False


def test_unmutated_oracle_passes():
    assert _pins_pass()


def _mut_sub_is_add(mp):
    mp.setattr(O.ModP, "sub", lambda self, u, v: (u + v) % self.p)


def _mut_merge_drops_half(mp):
    mp.setattr(O.ModP, "div", lambda self, u, v: u * ring.inv(v, self.p) % self.p if v != 2 else u)


def _mut_wrong_root(mp):
    real = ring.sqrt_mod
    mp.setattr(ring, "sqrt_mod", lambda v, p, rng=None: real(v, p, rng) * 3 % p)


def _mut_transposed_matrix(mp):
    real = O.fcirc_matrix_np
    mp.setattr(O, "fcirc_matrix_np", lambda a, f, p=None: real(a, f, p).T)


def _mut_dense_drops_f(mp):
    real = O.fcirc_matrix_np
    mp.setattr(O, "fcirc_matrix_np", lambda a, f, p=None: real(a, 1, p))


def _mut_levels_swapped_children(mp):
    real = O.node_roots_modp

    def swapped(n, f, p):
        return [(p - g) % p if d == 1 else g for d, g in enumerate(real(n, f, p))]
    mp.setattr(O, "node_roots_modp", swapped)


def _mut_levels_inverse_wrong(mp):
    mp.setattr(O, "_inv_vec", lambda v, p: v % p)


def _mut_definition_shift_left(mp):
    def bad(a, f, p=None):
        n = len(a)
        rows = [list(a)]
        for _ in range(n - 1):
            prev = rows[-1]
            last = prev[0] * f
            rows.append(prev[1:] + [last % p if p else last])
        return [[int(v) % p for v in r] for r in rows] if p else rows
    mp.setattr(O, "fcirc_matrix", bad)


@pytest.mark.parametrize("mutation", [
    _mut_sub_is_add, _mut_merge_drops_half, _mut_wrong_root, _mut_transposed_matrix,
    _mut_dense_drops_f, _mut_levels_swapped_children, _mut_levels_inverse_wrong,
    _mut_definition_shift_left,
])
def test_pins_catch_mutation(mutation, monkeypatch):
    mutation(monkeypatch)
    assert not _pins_pass()


# Embedding (Corollary 1, Toeplitz): the same idea, with its own compact pin set.
from oracle import embed as OE  # noqa: E402


def _embed_pins_pass() -> bool:
    rng = random.Random(5)
    try:
        for n in (3, 5, 6):
            row = [rng.randrange(P) for _ in range(n)]
            col = [rng.randrange(P) for _ in range(n)]
            x = [rng.randrange(P) for _ in range(n)]
            want = [sum((row[j - i] if j >= i else col[i - j]) * x[j] for j in range(n)) % P for i in range(n)]
            if OE.toeplitz_matvec_modp(row, col, x, P).tolist() != want:
                return False
            for f in (1, 7):
                want_f = [sum((row[j - i] if j >= i else f * row[n + j - i]) * x[j] for j in range(n)) % P
                          for i in range(n)]
                if OE.fcirc_any_matvec_modp(row, x, f, P).tolist() != want_f:
                    return False
        return True
    except (ValueError, AssertionError, IndexError):
        return False


def test_unmutated_embedding_passes():
    assert _embed_pins_pass()


def _mut_embed_tail_not_reversed(mp):
    real = OE.embedded_row
    def bad(row, col, N):
        r = real(row, col, N)
        n = len(row)
        return r[: N - n + 1] + r[N - n + 1:][::-1]
    mp.setattr(OE, "embedded_row", bad)


def _mut_embed_drops_f(mp):
    mp.setattr(OE, "fcirc_col", lambda a, f, p=None: [a[0]] + [a[len(a) - m] % P for m in range(1, len(a))])


def _mut_embed_short_length(mp):
    mp.setattr(OE, "cyclic_length", lambda n: max(1, 1 << ((n - 1).bit_length())))


@pytest.mark.parametrize("mutation", [_mut_embed_tail_not_reversed, _mut_embed_drops_f, _mut_embed_short_length])
def test_embedding_pins_catch_mutation(mutation, monkeypatch):
    mutation(monkeypatch)
    assert not _embed_pins_pass()


# --- section 3.2's ring Z/(2^K + 1) ------------------------------------------------------
from oracle import fermat as OF  # noqa: E402


def _fermat_pins_pass() -> bool:
    """A compact re-run of the P16 pins: level form against the definition, and the
    large-integer product against Python's."""
    rng = random.Random(16)
    try:
        K, n = 64, 16
        M = OF.modulus(K)
        a = [rng.randrange(M) for _ in range(n)]
        x = [rng.randrange(M) for _ in range(n)]
        for f_exp in (0, K):
            if OF.levels_matvec(a, x, f_exp, K) != OF.dense_matvec(a, x, pow(2, f_exp, M), K):
                return False
        u, v = rng.getrandbits(96 * 32), rng.getrandbits(96 * 32)
        return OF.bigint_mul_ssa(u, v, 96, 64, 256) == u * v
    except (ValueError, AssertionError):
        return False


def test_unmutated_fermat_passes():
    assert _fermat_pins_pass()


def _mut_fermat_second_child(mp):
    def bad(L, f_exp, K):
        levels = [[f_exp % (2 * K)]]
        for _ in range(L):
            levels.append([c for e in levels[-1] for c in (e // 2, e // 2)])  # -sqrt dropped
        return levels
    mp.setattr(OF, "node_exponents", bad)


def _mut_fermat_merge_without_half(mp):
    real_pow = pow

    def levels(a, x, f_exp, K):  # the merge divides by g instead of 2g
        M = OF.modulus(K)
        n = len(a)
        L = n.bit_length() - 1
        nodes = OF.node_exponents(L, f_exp, K)
        A, X = [v % M for v in a], [v % M for v in x]
        for d in range(L):
            m, h = n >> d, n >> (d + 1)
            for b in range(1 << d):
                g = real_pow(2, nodes[d + 1][2 * b], M)
                for k in range(b * m, b * m + h):
                    u, w = A[k], A[k + h]
                    A[k], A[k + h] = (u + g * w) % M, (u - g * w) % M
                    u, w = X[k], X[k + h]
                    X[k], X[k + h] = (g * u + w) % M, (g * u - w) % M
        Y = [A[k] * X[k] % M for k in range(n)]
        for d in reversed(range(L)):
            m, h = n >> d, n >> (d + 1)
            for b in range(1 << d):
                g = real_pow(2, nodes[d + 1][2 * b], M)
                for k in range(b * m, b * m + h):
                    s = Y[k] + Y[k + h]
                    Y[k], Y[k + h] = s * real_pow(g, -1, M) % M, (s * real_pow(2, -1, M) - Y[k + h]) % M
        return Y
    mp.setattr(OF, "levels_matvec", levels)


def _mut_fermat_row_not_reversed(mp):
    def bad(u, v, P, N, K):
        a, b = OF.bigint_pieces(u, P, N), OF.bigint_pieces(v, P, N)
        return OF.bigint_recompose(OF.levels_matvec(a, b, 0, K), P)
    mp.setattr(OF, "bigint_mul_ssa", bad)


@pytest.mark.parametrize("mutation", [_mut_fermat_second_child, _mut_fermat_merge_without_half,
                                      _mut_fermat_row_not_reversed])
def test_fermat_pins_catch_mutation(mutation, monkeypatch):
    mutation(monkeypatch)
    assert not _fermat_pins_pass()
