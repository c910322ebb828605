"""GPU parity of whole products at the headline size and above, every output element.

* n = 2^21 over Z/998244353 with f = p - 1 (the negacyclic form of the headline product)
  and with f = phi^n for a random phi (all three primes, 2^20 and 2^21), against the
  oracle's level-by-level form of Algorithm 1, run in the test.
* The largest sizes of each prime (2^22 .. 2^26, f = 1 and f = p - 1), against SHA-256
  digests of the oracle's products stored in tests/golden/large_products.txt (written by
  tests/golden/make_large_digests.py, which calls only the oracle): the full output must
  match bit for bit.
"""
import hashlib
import os
import random

import numpy as np
import pytest

from oracle import fcirc as O
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_products.txt")


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fcirc.set_split(-1)
    return fcirc


def dev(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.int32)).cuda()


def host_u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("L", [18, 21])
def test_negacyclic_headline_full(F, L):
    """f = p - 1 over Z/998244353 (a negacyclic correlation), every element."""
    p = W.P1
    n = 1 << L
    a, x = W.modp_pair(n, p, seed=W.SEED_HEADLINE)
    got = host_u32(F.matvec(dev(a), dev(x), f=p - 1, p=p)).astype(np.int64)
    np.testing.assert_array_equal(got, O.levels_matvec_modp(a, x, p - 1, p))


@pytest.mark.parametrize("p", W.PRIMES)
@pytest.mark.parametrize("L", [20, 21])
def test_random_f_full(F, p, L):
    """f = phi^n for a random phi: every root of the ladder differs from the f = 1 and
    f = -1 closed forms (Tonelli-Shanks chain), every element checked."""
    n = 1 << L
    f = pow(random.Random(1000 * L + p % 997).randrange(2, p), n, p)
    a, x = W.modp_pair(n, p, seed=40 + L)
    got = host_u32(F.matvec(dev(a), dev(x), f=f, p=p)).astype(np.int64)
    np.testing.assert_array_equal(got, O.levels_matvec_modp(a, x, f, p), err_msg=f"p={p} n=2^{L} f={f}")


def _golden_cases():
    cases = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        p, L, fs, seed, sha, *samples = line.split()
        cases.append(pytest.param(int(p), int(L), fs, int(seed), sha,
                                  [tuple(map(int, s.split(":"))) for s in samples], id=f"p{p}-2^{L}-f{fs}"))
    return cases


@pytest.mark.parametrize("p,L,fs,seed,sha,samples", _golden_cases())
def test_largest_sizes_full_digest(F, p, L, fs, seed, sha, samples):
    """Largest product of each prime: the whole output's digest equals the oracle's."""
    n = 1 << L
    f = 1 if fs == "1" else p - 1
    a, x = W.modp_pair(n, p, seed=seed)
    y = F.matvec(dev(a), dev(x), f=f, p=p)
    del a, x
    got = host_u32(y)
    for i, want in samples:
        assert int(got[i]) == want, f"y[{i}]"
    assert int(got.max()) < p
    assert hashlib.sha256(np.ascontiguousarray(got.astype("<u4")).tobytes()).hexdigest() == sha
