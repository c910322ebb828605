"""Every pass schedule on every ring, against the CPU oracle.

The top passes are compiled once per number of levels (1..10) and per loader (plain, real,
packed real pairs, the polynomial and large-integer loaders), the block pass once per block
size. The schedule (fcirc_set_schedule: top levels, tile size, tile order, joint or separate
row/vector split) picks which of them run, so sweeping it reaches each of them: at
n = 2^14, top levels 0..14 give blocks of 14..0 levels (clamped to what fits in LDS), one top
pass of 1..10 levels or two of 5..7. Z/p and GF(p^2) results are bit-exact; FP32 within
relative L2 1e-5 of the FP64 oracle. The layer (shared row, f = 1) is swept over every
size and a few batch counts, which moves its own top/block split."""
import numpy as np
import pytest

from oracle import fcirc as O
from oracle import gfp2 as G
from oracle import grad as OG
from oracle import polymul as OP
from oracle import bigint as OB
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5
TILES = (-1, 4, 10, 14)


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fcirc.set_split(-1)
    return fcirc


def dev(arr):
    import torch
    a = np.ascontiguousarray(arr)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    if a.dtype == np.uint16:
        a = a.view(np.int16)
    return torch.from_numpy(a).cuda()


def rel(got, want):
    return np.linalg.norm(got - want) / np.linalg.norm(want)


def sweep(F, ring, n, run, check):
    """Run every (top levels, tile, flags) schedule for (ring, n); check each result."""
    L = n.bit_length() - 1
    try:
        for top in range(0, L + 1):
            for tile_log in TILES:
                for flags in range(4):
                    F.set_schedule(n, ring, top, min(tile_log, 13 if ring >= 3 else 14), flags)
                    check(run(), f"top={top} tile={tile_log} flags={flags}")
    finally:
        F.set_schedule(n, ring, -1, -1, 1)


@pytest.mark.parametrize("L", [6, 14])
def test_zp_every_schedule(F, L):
    from paper_2103_02605_amd import _lib
    n, p = 1 << L, W.P2
    a, x = W.modp_pair(n, p, seed=300 + L)
    f = p - 1
    want = O.levels_matvec_modp(a, x, f, p)
    da, dx = dev(a), dev(x)
    sweep(F, _lib.FCIRC_ZP_469762049, n, lambda: F.matvec(da, dx, f=f, p=p).cpu().numpy().view(np.uint32),
          lambda got, msg: np.testing.assert_array_equal(got.astype(np.int64), want, err_msg=msg))


@pytest.mark.parametrize("L", [6, 14])
def test_complex_every_schedule(F, L):
    from paper_2103_02605_amd import _lib
    n = 1 << L
    a, x = W.complex_pair(n, seed=400 + L)
    want = O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), -1.0)
    da, dx = dev(a), dev(x)

    def check(got, msg):
        assert rel(got, want) <= TOL, msg

    sweep(F, _lib.FCIRC_C64, n, lambda: F.matvec(da, dx, f=-1.0).cpu().numpy(), check)


@pytest.mark.parametrize("L", [6, 14])
def test_real_every_schedule(F, L):
    from paper_2103_02605_amd import _lib
    n = 1 << L
    rng = np.random.default_rng(500 + L)
    a = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    want = O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), 1.0).real
    da, dx = dev(a), dev(x)

    def check(got, msg):
        assert rel(got, want) <= TOL, msg

    sweep(F, _lib.FCIRC_R32, n, lambda: F.matvec(da, dx).cpu().numpy(), check)


@pytest.mark.parametrize("L", [6, 14])
def test_gfp2_every_schedule(F, L):
    from paper_2103_02605_amd import _lib
    n = 1 << L
    rng = np.random.default_rng(600 + L)
    a = rng.integers(0, G.P, (n, 2)).astype(np.uint64)
    x = rng.integers(0, G.P, (n, 2)).astype(np.uint64)
    want = G.levels_matvec(a, x, (G.P - 1, 0))
    da, dx = dev(a.astype(np.int32)), dev(x.astype(np.int32))
    sweep(F, _lib.FCIRC_GFP2, n, lambda: F.matvec(da, dx, f=-1, p=G.P).cpu().numpy().astype(np.uint64),
          lambda got, msg: np.testing.assert_array_equal(got, want, err_msg=msg))


def test_polymul_and_bigint_every_schedule(F):
    """The products of both applications run at 2^14 (8000 + 8000 coefficients or limbs)
    under every schedule: their loaders reverse the row and zero-pad the vector."""
    from paper_2103_02605_amd import _lib
    rng = np.random.default_rng(700)
    a = rng.integers(-(1 << 15), 1 << 15, 8000).astype(np.int32)
    b = rng.integers(-(1 << 15), 1 << 15, 8000).astype(np.int32)
    want_poly = OP.poly_kronecker(a, b)
    u = rng.integers(0, 1 << 16, 8000).astype(np.uint16)
    v = rng.integers(0, 1 << 16, 8000).astype(np.uint16)
    want_big = OB.limbs_to_int(u) * OB.limbs_to_int(v)
    da, db, du, dv = dev(a), dev(b), dev(u), dev(v)

    def run():
        return (F.polymul_i64(da, db).cpu().numpy(), F.bigint_mul(du, dv).cpu().numpy().view(np.uint16))

    def check(got, msg):
        np.testing.assert_array_equal(got[0], want_poly, err_msg=msg)
        assert OB.limbs_to_int(got[1]) == want_big, msg

    sweep(F, _lib.FCIRC_ZP_998244353, 1 << 14, run, check)


@pytest.mark.parametrize("L", list(range(0, 14)))
def test_polymul_and_bigint_every_size(F, L):
    """Products of length 2^L (2^(L-1) and 2^(L-1) + 1 coefficients or limbs): up to 2^12 the block
    pass alone reads the inputs through the reversing and zero-padding loaders, one block
    size per L; at 2^13 the 13-level block is forced (no top levels) as well."""
    from paper_2103_02605_amd import _lib
    ma, mb = (1, 1) if L == 0 else (1 << (L - 1), (1 << (L - 1)) + 1)
    rng = np.random.default_rng(900 + L)
    a = rng.integers(-(1 << 15), 1 << 15, ma).astype(np.int32)
    b = rng.integers(-(1 << 15), 1 << 15, mb).astype(np.int32)
    u = rng.integers(0, 1 << 16, ma).astype(np.uint16)
    v = rng.integers(0, 1 << 16, mb).astype(np.uint16)
    want_poly = np.array(OP.poly_schoolbook(a, b), dtype=np.int64) if ma <= 512 else OP.poly_kronecker(a, b)
    want_big = OB.limbs_to_int(u) * OB.limbs_to_int(v)
    assert OP.cyclic_length(ma, mb) == 1 << L
    tops = (-1, 0) if L == 13 else (-1,)
    try:
        for top in tops:
            F.set_schedule(1 << L, _lib.FCIRC_ZP_998244353, top, -1, 1)
            np.testing.assert_array_equal(F.polymul_i64(dev(a), dev(b)).cpu().numpy(), want_poly, err_msg=f"top={top}")
            assert OB.limbs_to_int(F.bigint_mul(dev(u), dev(v)).cpu().numpy().view(np.uint16)) == want_big, top
    finally:
        F.set_schedule(1 << L, _lib.FCIRC_ZP_998244353, -1, -1, 1)


@pytest.mark.parametrize("L", list(range(0, 17)))
def test_real_every_size(F, L):
    """The real-input product (float32 in and out) at every size up to 2^16, f = 1 and -1."""
    n = 1 << L
    rng = np.random.default_rng(950 + L)
    a = rng.standard_normal(n).astype(np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    for f in (1.0, -1.0):
        want = O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), f).real
        got = F.matvec(dev(a), dev(x), f=f).cpu().numpy()
        assert rel(got, want) <= TOL, (L, f)


def layer_case(F, n, batch, real, seed):
    import torch
    rng = np.random.default_rng(seed)
    if real:
        a, x, g = (rng.standard_normal(s).astype(np.float32) for s in (n, (batch, n), (batch, n)))
    else:
        a, x, g = ((rng.standard_normal(s) + 1j * rng.standard_normal(s)).astype(np.complex64)
                   for s in (n, (batch, n), (batch, n)))
    ta, tx, tg = (torch.from_numpy(v).cuda() for v in (a, x, g))
    y = F.layer_forward(ta, tx).cpu().numpy()
    ga, gx = F.layer_backward(ta, tx, tg)
    hi = np.complex128 if not real else np.float64
    y_ref, ga_ref, gx_ref = OG.grads_fft(a.astype(hi), x.astype(hi), g.astype(hi))
    assert rel(y, y_ref) <= TOL, (n, batch, real)
    assert rel(ga.cpu().numpy(), ga_ref) <= TOL, (n, batch, real)
    assert rel(gx.cpu().numpy(), gx_ref) <= TOL, (n, batch, real)


@pytest.mark.parametrize("L,batch,real", [
    # grad_a's accumulating blocks read the batch directly (no top split): 11 and 12 levels
    (11, 512, False), (12, 512, False), (11, 1024, True), (12, 1024, True),
    # forward and grad_x with two and three top levels over packed real pairs
    (15, 256, True), (16, 128, True)])
def test_layer_large_batches(F, L, batch, real):
    layer_case(F, 1 << L, batch, real, seed=1000 + L + batch)


@pytest.mark.parametrize("real", [False, True])
def test_layer_2p23_sampled(F, real):
    """One instance of 2^23, where the forward, grad_x and grad_a each take 10 top levels:
    sampled entries of all three against their O(n) definitions, each within 1e-5 of the
    sampled entries' RMS (the FFT references cost tens of seconds per vector here)."""
    import torch
    n = 1 << 23
    rng = np.random.default_rng(2323 + real)
    if real:
        a, x, g = (rng.standard_normal(s).astype(np.float32) for s in (n, (1, n), (1, n)))
    else:
        a, x, g = ((rng.standard_normal(s) + 1j * rng.standard_normal(s)).astype(np.complex64)
                   for s in (n, (1, n), (1, n)))
    ta, tx, tg = (torch.from_numpy(v).cuda() for v in (a, x, g))
    y = F.layer_forward(ta, tx).cpu().numpy()
    ga, gx = F.layer_backward(ta, tx, tg)
    ga, gx = ga.cpu().numpy(), gx.cpu().numpy()
    idx = np.array([0, 1, n // 2, n - 1] + list(rng.integers(0, n, 4)))
    y_ref, ga_ref, gx_ref = OG.layer_entries(a, x, g, idx)
    for got, want in ((y[:, idx], y_ref), (gx[:, idx], gx_ref), (ga[idx], ga_ref)):
        scale = np.sqrt(np.mean(np.abs(want) ** 2))
        assert np.max(np.abs(got - want)) <= TOL * scale, (np.max(np.abs(got - want)) / scale)


@pytest.mark.parametrize("real", [False, True])
@pytest.mark.parametrize("L", list(range(4, 21)))
def test_layer_every_size(F, L, real):
    """Forward, grad_x and grad_a at every size, for one instance and a small batch."""
    for batch in (1, 3):
        layer_case(F, 1 << L, batch, real, seed=800 + L + 100 * real + batch)
