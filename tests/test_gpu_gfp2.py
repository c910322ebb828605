"""GPU parity of the product over the ring of section 3.1, GF(p^2) = Z/p[sqrt 3] with
p = 2^31 - 1, against the CPU oracle: bit-exact."""
import random

import numpy as np
import pytest

from oracle import gfp2 as G

pytestmark = pytest.mark.gpu

P = G.P
FS = {1: G.ONE, -1: (P - 1, 0)}


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield fcirc


def dev(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr.astype(np.int32))).cuda()


def rand(n, seed):
    return np.random.default_rng(seed).integers(0, P, (n, 2)).astype(np.uint64)


@pytest.mark.parametrize("L", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 16])
def test_gfp2_sizes_bit_exact(F, L):
    n = 1 << L
    a, x = rand(n, 100 + L), rand(n, 200 + L)
    for fs, fe in FS.items():
        got = F.matvec(dev(a), dev(x), f=fs, p=P).cpu().numpy().astype(np.uint64)
        if n <= 32:
            want = G.as_array(G.dense_matvec([tuple(int(c) for c in r) for r in a],
                                             [tuple(int(c) for c in r) for r in x], fe))
        else:
            want = G.levels_matvec(a, x, fe)
        np.testing.assert_array_equal(got, want, err_msg=f"L={L} f={fs}")


def test_gfp2_full_size_sampled(F):
    n = 1 << 21
    a, x = rand(n, 7), rand(n, 8)
    for fs, fe in FS.items():
        got = F.matvec(dev(a), dev(x), f=fs, p=P).cpu().numpy().astype(np.uint64)
        rng = random.Random(fs)
        for i in [0, 1, n // 2, n - 1] + [rng.randrange(n) for _ in range(4)]:
            assert tuple(int(c) for c in got[i]) == G.matvec_entry(a, x, fe, i), (fs, i)


def test_gfp2_many_and_forced_splits(F):
    import torch
    n, count = 1 << 14, 3
    a = np.stack([rand(n, 30 + k) for k in range(count)])
    x = np.stack([rand(n, 40 + k) for k in range(count)])
    got = F.matvec_many(dev(a), dev(x), f=-1, p=P).cpu().numpy().astype(np.uint64)
    for k in range(count):
        np.testing.assert_array_equal(got[k], G.levels_matvec(a[k], x[k], FS[-1]))
    base = F.matvec(dev(a[0]), dev(x[0]), f=1, p=P).cpu().numpy()
    try:
        for top in (0, 2, 5):
            F.set_split(top)
            np.testing.assert_array_equal(F.matvec(dev(a[0]), dev(x[0]), f=1, p=P).cpu().numpy(), base)
    finally:
        F.set_split(-1)
    del torch


def test_gfp2_two_top_passes(F):
    """Forced schedules of 16, 18 and 20 top levels at 2^20: two top passes of 8, 9 and 10
    levels each way (inner merges write the workspace), blocks of 2^4, 2^2 and 2^0."""
    n = 1 << 20
    a, x = rand(n, 61), rand(n, 62)
    want = G.levels_matvec(a, x, G.ONE)
    try:
        for top in (16, 18, 20):
            F.set_split(top)
            got = F.matvec(dev(a), dev(x), f=1, p=P).cpu().numpy().astype(np.uint64)
            np.testing.assert_array_equal(got, want, err_msg=f"top={top}")
    finally:
        F.set_split(-1)


def test_gfp2_errors(F):
    from paper_2103_02605_amd._lib import FcircError
    a = dev(rand(16, 1))
    with pytest.raises(FcircError, match="ENOROOT"):
        F.matvec(a, a.clone(), f=3, p=P)
    bad = rand(16, 2)
    bad[0, 0] = P  # the ABI checks f, not the data; data must be canonical
    with pytest.raises(FcircError, match="EINVAL"):
        F.matvec(a, a, f=1, p=P, out=a)


def test_gfp2_max_size_sampled(F):
    """n = 2^26, the largest size the ring's tables serve: sampled entries from the O(n)
    definition, f = 1 and f = -1."""
    n = 1 << 26
    a, x = rand(n, 61), rand(n, 62)
    da, dx = dev(a), dev(x)
    for (fs, fe), rows in zip(FS.items(), ((0, n - 1), (12345677,))):  # each entry is an O(n) CPU sum
        got = F.matvec(da, dx, f=fs, p=P).cpu().numpy()
        for i in rows:
            assert tuple(int(c) for c in got[i]) == G.matvec_entry(a, x, fe, i), (fs, i)
