#!/usr/bin/env python3
"""Benchmark of libfcirc on one MI355X.

Headline workload: one f-circulant product over Z/998244353 of size n = 2^21 with f = 1
(defining row a and vector x uniform in [0, p), seed 3). One step = one fcirc_matvec
call, i.e. the whole path: top split passes -> LDS block pass -> top merge passes.
Inputs rotate over 24 resident (a, x, y) sets (576 MiB, more than twice the 256 MB
Infinity Cache), so each step reads its inputs from HBM.

Printed (rank 0, one JSON line): throughput in output coefficients per second, the
roofline of the dominant kernel (per-kernel times from HIP events recorded by the
library on the stream it launches on), the CPU oracle timed on this host, and the
secondary workloads (polynomial and integer products, batched and forward+backward
forms against their one-call-per-instance equivalents).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

P1 = 998244353
W_SEED_GF = 3
HBM_PEAK_GBS = 8000.0
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz: 32-bit VALU lane-operations per second (T/s)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic cost model (lane-operations), from the operation counts of a product of
# length n = 2^L: (1.5 L + 1) n modular multiplies and 3 L n modular additions. A multiply
# by a precomputed constant (Shoup: mul_hi, mul_lo, mul_lo, sub) = 4, a lazy modular
# add/sub (add, conditional correction) = 2; one coefficient per level per transform does
# half a multiply and one add/sub = 4; the leaf (product of two variables, then the
# constant 1/n) = 2 multiplies = 8. For n = 2^21 that is 3 * 21 * 4 + 8 = 260 per coefficient.
OPS_PER_COEF_LEVEL = 4.0
OPS_LEAF = 8.0
# Schedule bytes per coefficient of each kernel (uint32 data): split reads a, x and writes
# both; the block reads both and writes y; the merge reads and writes y.
BYTES_PER_COEF = {"fcirc_top_split": 16, "fcirc_block": 12, "fcirc_top_merge": 8}
# Secondary rows. Garner CRT of three residues to one coefficient (three Shoup products,
# their corrections and the 64-bit combination) and the carry passes of the large-integer
# product, in lane-operations per output coefficient (limb).
OPS_CRT = 30.0
OPS_CARRY = 20.0
# Complex FP32 rows: FP32 operations per coefficient per level of one transform (split of
# a, split of x or merge of y: half a complex product by the twiddle, 4 operations with
# fused multiply-adds, plus a complex sum and difference, 4 operations; 13 for all three).
FP32_OPS_PER_COEF_LEVEL_TRANSFORM = 13.0 / 3.0


# The sources the headline product's kernels and launches are built from (the Z/p plan and
# driver, the host schedule and launch code, the tile kernels and the ring arithmetic).
HEADLINE_SOURCES = ("host.hpp", "ring.hpp", "tile.hpp", "zp.hip")


def source_digest() -> str:
    """Digest of the headline kernels' sources: a traffic summary taken on other sources
    is not reported."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2103_02605_amd", "csrc")
    for f in HEADLINE_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, digest: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary, if it was taken
    on the current kernel sources (null otherwise)."""
    path = os.path.join(ROOT, "profiles", "traffic_zp_n2p21.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_digest") != digest:
        return None
    key = f"{kernel}_bytes_per_launch"
    return float(vals[key]) if key in vals else None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_steps(torch, fn, steps, warmup):
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        fn(i)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps  # ms per step


def headline(torch, F, W, steps, warmup, nsets=24):
    L = 21
    n = 1 << L
    sets = []
    for k in range(nsets):
        a, x = W.modp_pair(n, P1, seed=W.SEED_HEADLINE + 1000 * k)
        sets.append((torch.from_numpy(a.view(np.int32)).cuda(), torch.from_numpy(x.view(np.int32)).cuda(),
                     torch.empty(n, dtype=torch.int32, device="cuda")))

    def step(i):
        a, x, y = sets[i % nsets]
        F.matvec(a, x, f=1, p=P1, out=y)

    ms = time_steps(torch, step, steps, warmup)
    # per-step spread (separate pass: one event pair per step)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(100)]
    for i, (e0, e1) in enumerate(evs):
        e0.record()
        step(i)
        e1.record()
    torch.cuda.synchronize()
    per = sorted(e0.elapsed_time(e1) * 1e3 for e0, e1 in evs)
    spread = {"median_us": round(per[len(per) // 2], 2), "min_us": round(per[0], 2), "steps": len(per)}
    # per-kernel durations: HIP events around each kernel, on the stream it runs on
    F.set_timing(True)
    for i in range(steps):
        step(i)
    stages = F.stage_times()
    F.set_timing(False)
    T = F.get_split(n, 0)
    return n, ms, stages, T, spread


def negacyclic_headline(torch, F, W, steps, warmup, nsets=24):
    """The headline product with f = p - 1 (a negacyclic correlation): n = 2^21 over
    Z/998244353, same inputs (seed 3 + 1000 k), same 24 rotating sets."""
    n = 1 << 21
    sets = []
    for k in range(nsets):
        a, x = W.modp_pair(n, P1, seed=W.SEED_HEADLINE + 1000 * k)
        sets.append((torch.from_numpy(a.view(np.int32)).cuda(), torch.from_numpy(x.view(np.int32)).cuda(),
                     torch.empty(n, dtype=torch.int32, device="cuda")))

    def step(i):
        a, x, y = sets[i % nsets]
        F.matvec(a, x, f=P1 - 1, p=P1, out=y)
    ms = time_steps(torch, step, steps, warmup)
    return {"ms": ms, "Gcoeff_per_s": n / ms / 1e6, **fractions(12 * n, ALU_OPS_PER_COEF_ZP(21) * n, ms)}


def fractions(bytes_compulsory: float, lane_ops: float | None, ms: float) -> dict:
    """HBM fraction (compulsory bytes over the whole call against 8 TB/s) and VALU fraction
    (modelled 32-bit lane-operations against 39.3 T/s) of one measured call."""
    out = {"hbm_frac": round(bytes_compulsory / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "compulsory_bytes": int(bytes_compulsory)}
    if lane_ops is not None:
        out["valu_frac"] = round(lane_ops / (ms * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4)
        out["model_lane_ops"] = int(lane_ops)
    return out


def ALU_OPS_PER_COEF_ZP(L: int) -> float:  # noqa: N802 - a model constant, written as a function of L
    """Lane-operations per coefficient of one Z/p product of length 2^L (cost model above)."""
    return 3 * L * OPS_PER_COEF_LEVEL + OPS_LEAF


def copy_ceiling(torch) -> float:
    """GB/s (read + write) of a plain 64 MiB device copy: the same-box HBM reference."""
    src = torch.ones(1 << 24, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    ms = time_steps(torch, lambda i: dst.copy_(src), 50, 5)
    return 2 * src.numel() * 4 / (ms * 1e-3) / 1e9


def c1_latency(torch, F, W):
    """n = 1024 over Z/998244353 (seeds 1 and 2 for f = 1 and f = p - 1): one call per
    product, and 1024 products of that size (seed 11) in one batched launch and in one
    uniform-size call."""
    from paper_2103_02605_amd.batched import BatchPlan
    out = {}
    for f, seed, name in ((1, W.SEED_C1_CYCLIC, "f1"), (P1 - 1, W.SEED_C1_NEGACYCLIC, "f_pm1")):
        a, x = W.modp_pair(1024, P1, seed=seed)
        ta, tx = torch.from_numpy(a.view(np.int32)).cuda(), torch.from_numpy(x.view(np.int32)).cuda()
        ty = torch.empty_like(ta)
        ms = time_steps(torch, lambda i: F.matvec(ta, tx, f=f, p=P1, out=ty), 200, 20)
        out[f"plain_us_per_call_{name}"] = round(ms * 1e3, 3)
        if name == "f1":
            out.update(fractions(12 * 1024, ALU_OPS_PER_COEF_ZP(10) * 1024, ms))
    ab, xb = W.modp_batch(1024, 1024, P1)
    al, xl = list(ab), list(xb)
    plan = BatchPlan(al, xl, p=P1, f=1)
    ms = time_steps(torch, lambda i: plan.run(), 50, 5)
    out["batched_1024x1024_us_per_product"] = round(ms * 1e3 / 1024, 4)
    out["batched_1024x1024_us_per_launch"] = round(ms * 1e3, 2)
    # the same 1024 products as one uniform-size call (fcirc_matvec_many: one block launch)
    da, dx = torch.from_numpy(ab.view(np.int32)).cuda(), torch.from_numpy(xb.view(np.int32)).cuda()
    dy = torch.empty_like(da)
    ms = time_steps(torch, lambda i: F.matvec_many(da, dx, f=1, p=P1, out=dy), 50, 5)
    out["many_1024x1024_us_per_product"] = round(ms * 1e3 / 1024, 4)
    out["many_1024x1024_us_per_call"] = round(ms * 1e3, 2)
    return out


SECONDARY_ROWS = ("polymul", "bigint", "fermat", "c1", "negacyclic", "fft", "gfp2", "batched", "layer")


def secondary(torch, F, W, quick: bool, rows=SECONDARY_ROWS, plain: bool = True):
    """The secondary workloads named in `rows`; plain=False skips the one-call-per-instance
    comparisons of the batched and layer rows (for profiling runs)."""
    out = {}
    N, nc = 1 << 21, (1 << 21) - 1
    if "polymul" in rows:  # C2: exact polynomial product, 2 x 2^20 int32 -> 2^21 - 1 int64
        a, b = W.poly_i32(1 << 20, W.SEED_POLY)
        ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
        c = torch.empty(nc, dtype=torch.int64, device="cuda")
        ms = time_steps(torch, lambda i: F.polymul_i64(ta, tb, out=c), 20 if quick else 100, 5)
        out["polymul_i64_2x2^20"] = {"ms": ms, "Gcoeff_per_s": nc / ms / 1e6,
                                     **fractions(2 * (1 << 20) * 4 + nc * 8,
                                                 3 * ALU_OPS_PER_COEF_ZP(21) * N + OPS_CRT * nc, ms)}
    if "bigint" in rows or "fermat" in rows:  # C3: big integers, 2 x 2^24 bits -> 2^21 limbs
        a, b = W.bigint_u16(1 << 20, W.SEED_BIGINT)
        ta, tb = torch.from_numpy(a.view(np.int16)).cuda(), torch.from_numpy(b.view(np.int16)).cuda()
        c = torch.empty(1 << 21, dtype=torch.int16, device="cuda")
        ms = time_steps(torch, lambda i: F.bigint_mul(ta, tb, out=c), 20 if quick else 100, 5)
        out["bigint_mul_2x2^24bit"] = {"ms": ms, "Glimb_per_s": N / ms / 1e6,
                                       **fractions(2 * (1 << 20) * 2 + N * 2,
                                                   3 * ALU_OPS_PER_COEF_ZP(21) * N + (OPS_CRT + OPS_CARRY) * N, ms)}
        if "fermat" in rows:
            out["bigint_fermat_2x2^24bit"] = bigint_fermat(torch, F, ta, tb, ms, quick)
    if "c1" in rows:
        out["c1_n1024_latency"] = c1_latency(torch, F, W)
    if "negacyclic" in rows:
        out["headline_negacyclic_f_p-1_2^21"] = negacyclic_headline(torch, F, W, 20 if quick else 200, 10)
    if "fft" in rows:
        out["circulant_vs_fft_c64_2^21"] = circulant_vs_fft(torch, F, W, quick)
    if "gfp2" in rows:
        out["gfp2_section3_ring_2^21"] = gfp2_product(torch, F, quick)
    if "batched" in rows:
        out["batched_c64_4096"] = batched_vs_plain(torch, F, W, quick, plain)
    if "layer" in rows:
        out["layer_fwd_bwd_256x2^14"] = layer_vs_plain(torch, F, W, quick, plain)
    return out


def bigint_fermat(torch, F, ta, tb, ms_ntt, quick: bool):
    """Section 3.2's route for the C3 integers (2 x 2^24 bits, seed 5): pieces as
    coefficients over Z/(2^K + 1), one cyclic product with shift-only roots. Compared with
    the three-prime route on the same inputs; both give the same limbs."""
    c = torch.empty(1 << 21, dtype=torch.int16, device="cuda")
    ms = time_steps(torch, lambda i: F.bigint_mul_fermat(ta, tb, out=c), 5 if quick else 30, 2)
    F.set_timing(True)
    F.bigint_mul_fermat(ta, tb, out=c)
    st = F.stage_times()
    F.set_timing(False)
    ref = F.bigint_mul(ta, tb)
    same = bool(torch.equal(ref, c))
    kern = {k: round(v[1] * 1e3, 1) for k, v in st.items() if k.startswith("fcirc_fermat") and v[0]}
    return {"ms": ms, "Glimb_per_s": (1 << 21) / ms / 1e6, "over_three_prime": ms / ms_ntt, "same_limbs": same,
            "kernel_us": kern}


def circulant_vs_fft(torch, F, W, quick: bool):
    """The paper's comparison (circulant product against the classic three-FFT cyclic
    convolution), on this GPU: complex64, n = 2^21, f = 1 (seed 3). The classic side is
    torch.fft (hipFFT): y = ifft(fft(b) * fft(x)) with b_k = a_(-k mod n)."""
    n = 1 << 21
    a, x = W.complex_pair(n, seed=W.SEED_HEADLINE)
    ta, tx = torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda()
    ty = torch.empty_like(ta)
    idx = (-torch.arange(n, device="cuda")) % n
    tb = ta[idx].contiguous()
    ms_c = time_steps(torch, lambda i: F.matvec(ta, tx, out=ty), 20 if quick else 200, 10)

    def classic(i):
        return torch.fft.ifft(torch.fft.fft(tb) * torch.fft.fft(tx))
    torch.cuda.synchronize()
    yh = ty.cpu().numpy()  # the circulant product, copied out before the FFT side runs
    ms_f = time_steps(torch, classic, 20 if quick else 200, 10)
    yc = classic(0).cpu().numpy()
    # both results against the FP64 evaluation of the definition (cyclic correlation by a
    # host FFT), and against each other, on host copies
    yd = np.fft.ifft(np.fft.fft(a.astype(np.complex128)[(-np.arange(n)) % n]) * np.fft.fft(x.astype(np.complex128)))
    nd = np.linalg.norm(yd)
    return {"circulant_ms": ms_c, "fft_ms": ms_f, "fft_over_circulant": ms_f / ms_c,
            "rel_l2_between": float(np.linalg.norm(yh - yc) / np.linalg.norm(yc)),
            "rel_l2_circulant_vs_fp64": float(np.linalg.norm(yh - yd) / nd),
            "rel_l2_fft_vs_fp64": float(np.linalg.norm(yc - yd) / nd),
            "output_changed_after": bool(not np.array_equal(ty.cpu().numpy(), yh)),
            **fractions(24 * n, 3 * FP32_OPS_PER_COEF_LEVEL_TRANSFORM * 21 * n, ms_c)}


def gfp2_product(torch, F, quick: bool):
    """The ring of section 3.1, GF(p^2) = Z/p[sqrt 3] with p = 2^31 - 1: one product of
    n = 2^21 (f = 1), inputs uniform (seed 3), 8 rotating sets."""
    n = 1 << 21
    p = (1 << 31) - 1
    rng = np.random.default_rng(W_SEED_GF)
    sets = [(torch.from_numpy(rng.integers(0, p, (n, 2)).astype(np.int32)).cuda(),
             torch.from_numpy(rng.integers(0, p, (n, 2)).astype(np.int32)).cuda()) for _ in range(8)]
    ty = torch.empty_like(sets[0][0])
    ms = time_steps(torch, lambda i: F.matvec(sets[i % 8][0], sets[i % 8][1], f=1, p=p, out=ty), 20 if quick else 200, 10)
    return {"ms": ms, "Gcoeff_per_s": n / ms / 1e6, **fractions(24 * n, None, ms)}


def batched_vs_plain(torch, F, W, quick: bool, with_plain: bool = True):
    """4096 complex64 products of sizes 2^6..2^16 (seed 6): one persistent launch (its work
    queue reused) against one fcirc_matvec call per instance, on the same device buffers."""
    from paper_2103_02605_amd.batched import BatchPlan
    from paper_2103_02605_amd import _lib
    e, a_list, x_list = W.batched_c64(4096, W.SEED_BATCHED)
    plan = BatchPlan(a_list, x_list, dtype=np.complex64)
    total = int(plan.offsets[-1])
    ms_default = time_steps(torch, lambda i: plan.run(), 5 if quick else 20, 2)
    # the launch's parameters per instance size picked by the autotuner (fcirc_tune), then
    # the timed runs of the same batch
    t0 = time.perf_counter()
    for L in range(int(min(e)), int(max(e)) + 1):
        F.tune(1 << L, _lib.FCIRC_C64)
    tune_s = time.perf_counter() - t0
    params = {f"2^{L}": F.get_batch_schedule(1 << L, _lib.FCIRC_C64) for L in range(int(min(e)), int(max(e)) + 1)}
    ms_b = time_steps(torch, lambda i: plan.run(), 5 if quick else 20, 2)
    plan.check()
    views = [(plan.a[plan.offsets[k]:plan.offsets[k + 1]], plan.x[plan.offsets[k]:plan.offsets[k + 1]],
              plan.y[plan.offsets[k]:plan.offsets[k + 1]]) for k in range(len(a_list))]

    def plain(i):
        for a, x, y in views:
            F.matvec(a, x, out=y)
    ms_p = time_steps(torch, plain, 1 if quick else 3, 1) if with_plain else float("nan")
    ops = sum(3 * FP32_OPS_PER_COEF_LEVEL_TRANSFORM * int(L) * (1 << int(L)) for L in e)
    return {"coefficients": total, "batched_ms": ms_b, "plain_ms": ms_p,
            "batched_Gcoeff_per_s": total / ms_b / 1e6, "plain_Gcoeff_per_s": total / ms_p / 1e6,
            "batched_over_plain": ms_p / ms_b, "batched_ms_default_parameters": ms_default,
            "tuned_parameters": params, "tuning_s": round(tune_s, 2), **fractions(24 * total, ops, ms_b)}


def layer_vs_plain(torch, F, W, quick: bool, with_plain: bool = True):
    """Circulant layer, batch 256 x 2^14 float32 (seed 7): library forward + backward against
    one product per row for y, grad_x and grad_a plus a torch sum."""
    a, x, g = W.circ_layer_f32()
    ta, tx, tg = torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda(), torch.from_numpy(g).cuda()
    n = a.shape[0]

    def fused(i):
        F.layer_forward(ta, tx)
        F.layer_backward(ta, tx, tg)
    ms_f = time_steps(torch, fused, 5 if quick else 20, 2)
    rev = ta[(-torch.arange(n, device="cuda")) % n].contiguous()
    y = torch.empty_like(tx)
    gx = torch.empty_like(tx)
    parts = torch.empty_like(tx)

    def plain(i):
        for b in range(tx.shape[0]):
            F.matvec(ta, tx[b], out=y[b])
            F.matvec(rev, tg[b], out=gx[b])
            F.matvec(tg[b], tx[b], out=parts[b])
        parts.sum(0)
    ms_p = time_steps(torch, plain, 1 if quick else 3, 1) if with_plain else float("nan")
    # compulsory: forward reads x, writes y; backward reads x and gy, writes gx (float32),
    # plus the row and its gradient; work: per row, the forward splits x and merges y, the
    # backward splits gy twice, x once, and merges grad_x (grad_a's merge is shared)
    rows, L = tx.shape[0], n.bit_length() - 1
    nbytes = 4 * (5 * rows * n + 3 * n)
    ops = rows * 6 * FP32_OPS_PER_COEF_LEVEL_TRANSFORM * L * n
    return {"fwd_bwd_ms": ms_f, "plain_ms": ms_p, "fused_over_plain": ms_p / ms_f,
            "coefficients_per_pass": int(tx.numel()), **fractions(nbytes, ops, ms_f)}


def _pool_cores() -> int:
    """Worker processes for the pooled oracle runs: the cores this process may use, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _oracle_residues(args):
    """One prime's residues of the polynomial product (pool worker; oracle only)."""
    a, b, p = args
    from oracle import polymul as OP
    return OP.poly_residues(a, b, p)


def _oracle_c128(args):
    """One complex product by the oracle's level form (pool worker)."""
    a, x = args
    from oracle import fcirc as O
    O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128))
    return a.shape[0]


def _timed(fn):
    t0 = time.perf_counter()
    r = fn()
    return r, time.perf_counter() - t0


def cpu_baselines_secondary(W) -> dict:
    """The oracle on each secondary configuration, timed on this host (reported baselines,
    not targets). Runs before the GPU is touched, so the spawned pool workers start from a
    process with no device state. Single products run on 1 core; the independent parts of
    a configuration (the three primes of C2 and C3, the instances of C4) also run on a
    process pool."""
    import multiprocessing as mp

    from oracle import bigint as OB
    from oracle import fcirc as O
    from oracle import polymul as OP
    host = cpu_model()
    cores = _pool_cores()
    spawn = mp.get_context("spawn")
    out = {}
    # C1: the dense O(n^2) definition, n = 1024, f = 1 and f = p - 1
    vals = {}
    for f, seed, name in ((1, W.SEED_C1_CYCLIC, "f1"), (P1 - 1, W.SEED_C1_NEGACYCLIC, "f_pm1")):
        a, x = W.modp_pair(1024, P1, seed=seed)
        runs, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 1.0:
            O.dense_matvec_modp(a, x, f, P1)
            runs += 1
        vals[name] = (time.perf_counter() - t0) / runs
    out["c1_n1024_latency"] = {"value": round(vals["f1"] * 1e6, 1), "unit": "us per product", "cores": 1, "kind": "oracle",
                               "f_pm1_us": round(vals["f_pm1"] * 1e6, 1),
                               "sample": f"dense definition (Definition 2) in numpy int64, n=1024, repeated for 1 s per f; {host}"}
    # C2: three circulant products + the textbook CRT, full size; then the primes on a pool
    a, b = W.poly_i32(1 << 20, W.SEED_POLY)
    nc = (1 << 21) - 1
    _, dt1 = _timed(lambda: OP.poly_via_circulant(a, b, W.PRIMES))
    with spawn.Pool(3) as pool:
        _, dtp = _timed(lambda: OP.crt_textbook(pool.map(_oracle_residues, [(a, b, p) for p in W.PRIMES]), W.PRIMES))
    out["polymul_i64_2x2^20"] = {"value": nc / dt1 / 1e9, "unit": "Gcoeff/s", "cores": 1, "kind": "oracle",
                                 "pool": {"value": nc / dtp / 1e9, "cores": 3, "what": "one prime per process, CRT in the parent"},
                                 "sample": f"one full C2 product (3 level-form products of 2^21 + textbook CRT), {dt1:.1f} s; {host}"}
    # C3: Python's integer multiply (1 core); the circulant route with its primes on a pool
    a, b = W.bigint_u16(1 << 20, W.SEED_BIGINT)
    _, dt1 = _timed(lambda: OB.bigint_mul_pyint(a, b))
    a64, b64 = a.astype(np.int64), b.astype(np.int64)
    with spawn.Pool(3) as pool:
        _, dtp = _timed(lambda: OB.carry_propagate(
            OP.crt_textbook(pool.map(_oracle_residues, [(a64, b64, p) for p in W.PRIMES]), W.PRIMES), 1 << 21))
    out["bigint_mul_2x2^24bit"] = {"value": (1 << 21) / dt1 / 1e9, "unit": "Glimb/s", "cores": 1, "kind": "oracle",
                                   "pool": {"value": (1 << 21) / dtp / 1e9, "cores": 3,
                                            "what": "circulant route: one prime per process, CRT and carries in the parent"},
                                   "sample": f"one full C3 product by Python int multiply, {dt1:.1f} s; {host}"}
    # C4: a seeded sample of 512 of the 4096 instances (all sizes), 1 core and a pool
    e, a_list, x_list = W.batched_c64(4096, W.SEED_BATCHED)
    pick = np.random.default_rng(0).choice(len(a_list), 512, replace=False)
    work = [(a_list[k], x_list[k]) for k in pick]
    coefs = sum(int(a.shape[0]) for a, _ in work)
    _, dt1 = _timed(lambda: [_oracle_c128(w) for w in work])
    with spawn.Pool(cores) as pool:
        pool.map(_oracle_c128, work[:cores])  # workers started and warm
        _, dtp = _timed(lambda: pool.map(_oracle_c128, work, chunksize=4))
    out["batched_c64_4096"] = {"value": coefs / dt1 / 1e9, "unit": "Gcoeff/s", "cores": 1, "kind": "oracle",
                               "pool": {"value": coefs / dtp / 1e9, "cores": cores, "what": "instances over a process pool"},
                               "sample": f"512 of the 4096 instances (seeded choice, {coefs} coefficients), complex128 level form; {host}"}
    # C5: forward and backward of 16 of the 256 rows (one product each for y, grad_x, grad_a)
    ra, rx, rg = W.circ_layer_f32()
    n = ra.shape[0]
    rev = ra[(-np.arange(n)) % n]
    rows = 16

    def layer_rows():
        for b in range(rows):
            O.levels_matvec_c128(ra.astype(np.complex128), rx[b].astype(np.complex128))
            O.levels_matvec_c128(rev.astype(np.complex128), rg[b].astype(np.complex128))
            O.levels_matvec_c128(rg[b].astype(np.complex128), rx[b].astype(np.complex128))
    _, dt1 = _timed(layer_rows)
    out["layer_fwd_bwd_256x2^14"] = {"value": dt1 * 256 / rows * 1e3, "unit": "ms per forward+backward (256 rows)",
                                     "cores": 1, "kind": "oracle",
                                     "sample": f"{rows} of 256 rows, 3 complex128 level-form products each, scaled to 256; {host}"}
    return out


def cpu_baseline(W, budget_s: float = 15.0):
    from oracle import fcirc as O
    n = 1 << 21
    a, x = W.modp_pair(n, P1, seed=W.SEED_HEADLINE)
    runs, t0 = 0, time.perf_counter()
    while True:
        O.levels_matvec_modp(a, x, 1, P1)
        runs += 1
        if time.perf_counter() - t0 >= budget_s or runs >= 8:
            break
    dt = (time.perf_counter() - t0) / runs
    return {"value": n / dt / 1e9, "unit": "Gcoeff/s", "cores": 1, "kind": "oracle",
            "sample": f"{runs} full n=2^21 Z/998244353 products with the level-by-level numpy oracle "
                      f"(single-threaded numpy), {dt:.2f} s each, host CPU: {cpu_model()}"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip timing the CPU oracle")
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--quick-secondary", action="store_true", help="time the secondary workloads with fewer steps")
    ap.add_argument("--rows", default=",".join(SECONDARY_ROWS),
                    help="comma-separated secondary workloads to run (default: all of " + ", ".join(SECONDARY_ROWS) + ")")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the one-call-per-instance comparisons of the batched and layer rows (profiling runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run 3 plain 64 MiB device copies (torch), the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs each product on a single device "
              "(multi-GPU sharding is a design note, not built). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    from paper_2103_02605_amd import workloads as W
    # the pooled oracle runs start worker processes: do them before the GPU is touched
    sec_cpu = cpu_baselines_secondary(W) if not (args.no_cpu_baseline or args.no_secondary) else {}

    import torch
    from paper_2103_02605_amd import fcirc as F

    torch.cuda.set_device(0)
    if args.calib_copy:
        src = torch.ones(1 << 24, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n, ms, stages, T, spread = headline(torch, F, W, args.steps, args.warmup)
    copy_gbs = copy_ceiling(torch)
    value = n / ms / 1e6  # Gcoeff/s
    L = 21
    B = L - T
    ops_coef = {"fcirc_top_split": 2 * T * OPS_PER_COEF_LEVEL,
                "fcirc_block": 3 * B * OPS_PER_COEF_LEVEL + OPS_LEAF,
                "fcirc_top_merge": T * OPS_PER_COEF_LEVEL}
    kern = {}
    for name, (launches, tot) in stages.items():
        avg_ms = tot / max(launches, 1)
        kern[name] = {"launches": launches, "avg_us": avg_ms * 1e3,
                      "alu_Tops": ops_coef.get(name, 0) * n / (avg_ms * 1e-3) / 1e12,
                      "sched_GBs": BYTES_PER_COEF.get(name, 0) * n / (avg_ms * 1e-3) / 1e9}
    dom = max(kern, key=lambda k: kern[k]["avg_us"] * kern[k]["launches"])
    digest = source_digest()
    dk = kern[dom]
    traffic = read_traffic(dom, digest)
    hbm_frac = round(12 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(dk["alu_Tops"], 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "Tops/s (32-bit VALU lane-ops)", "frac": round(dk["alu_Tops"] / VALU_PEAK_TOPS, 4),
                "hbm_frac": hbm_frac,
                "hbm_frac_is": "the metric's % HBM roofline: 12 compulsory bytes per coefficient over the whole "
                               "step (all kernels) against 8 TB/s",
                "traffic": traffic,
                "per_unit": f"{ops_coef[dom]} lane-ops per coefficient x {n} coefficients per launch",
                "hbm": {"achieved_GBs": round(12 * n / (ms * 1e-3) / 1e9, 1), "peak_GBs": HBM_PEAK_GBS,
                        "frac": hbm_frac,
                        "copy_ceiling_GBs": round(copy_gbs, 1),
                        "per_unit": "12 compulsory bytes per coefficient (a, x read, y written), whole step"},
                "kernels": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in kern.items()},
                "source_digest": digest}
    line = {"metric": "Gcoeff/s for n=2^21 mod-p product, % HBM roofline; batched/fwd+bwd vs plain",
            "value": round(value, 3), "unit": "Gcoeff/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(ms, 5), "step_spread": spread, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32", "data": "synthetic",
            "config": {"workload": "fcirc_matvec over Z/998244353, n=2^21, f=1, a and x uniform in [0,p) (seed 3), "
                                   "24 rotating input sets", "n": n, "ring": "Z/998244353", "f": 1,
                       "split": {"top_levels": T, "block_levels": B}},
            "roofline": roofline}
    if not args.no_secondary:
        rows = tuple(r for r in args.rows.split(",") if r)
        unknown = set(rows) - set(SECONDARY_ROWS)
        if unknown:
            raise SystemExit(f"unknown secondary rows: {sorted(unknown)}")
        line["secondary"] = secondary(torch, F, W, quick=args.quick_secondary, rows=rows, plain=not args.no_plain)
        for row, cb in sec_cpu.items():
            if row in line["secondary"]:
                line["secondary"][row]["cpu_baseline"] = cb
    if not args.no_cpu_baseline:
        cb = cpu_baseline(W)
        line["cpu_baseline"] = cb
        line["gpu_over_cpu_oracle"] = round(value / cb["value"], 1)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
