"""Write large_products.txt: SHA-256 digests of full f-circulant products over Z/p at sizes
where running the CPU oracle inside a GPU test would take minutes (2^22 .. 2^26 elements).

Every digest comes from the oracle alone: the row a and vector x are the seeded draws of
``paper_2103_02605_amd.workloads.modp_pair`` (which holds no arithmetic of the method), the
product y = A(a, f) x is the oracle's level-by-level form of Algorithm 1
(``oracle.fcirc.levels_matvec_modp``), and the digest is taken over y as little-endian
uint32. Each line also stores a few entries of y, checked against the O(n) definition of
one entry (Definition 2) before the line is written.

    python tests/golden/make_large_digests.py            # rewrites large_products.txt
"""
from __future__ import annotations

import hashlib
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fcirc as O  # noqa: E402
from paper_2103_02605_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_products.txt")

# (prime, log2 n, f as "1" or "p-1", seed): the largest size of each prime with f = 1 and
# f = p - 1 (for f = p - 1 a 2n-th root of unity is needed, so the limit halves)
CASES = [
    (W.P1, 22, "p-1", 31),
    (W.P1, 23, "1", 32),
    (W.P3, 24, "p-1", 33),
    (W.P3, 25, "1", 34),
    (W.P2, 25, "p-1", 35),
    (W.P2, 26, "1", 36),
]


def digest(y: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(y.astype("<u4")).tobytes()).hexdigest()


def main() -> None:
    lines = ["# prime log2n f seed sha256(y as little-endian uint32) i:y_i ...",
             "# written by tests/golden/make_large_digests.py from oracle.fcirc.levels_matvec_modp"]
    for p, L, fs, seed in CASES:
        n = 1 << L
        f = 1 if fs == "1" else p - 1
        a, x = W.modp_pair(n, p, seed=seed)
        y = O.levels_matvec_modp(a, x, f, p)
        idx = [0, 1, n // 3, n - 1]
        for i in idx:
            assert int(y[i]) == O.matvec_entry_modp(a, x, f, p, i), (p, L, fs, i)
        samples = " ".join(f"{i}:{int(y[i])}" for i in idx)
        lines.append(f"{p} {L} {fs} {seed} {digest(y)} {samples}")
        print(lines[-1], flush=True)
        del a, x, y
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
