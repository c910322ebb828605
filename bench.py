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


def secondary(torch, F, W, quick: bool):
    out = {}
    # C2: exact polynomial product, 2 x 2^20 int32 -> 2^21 - 1 int64
    a, b = W.poly_i32(1 << 20, W.SEED_POLY)
    ta, tb = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    c = torch.empty((1 << 21) - 1, dtype=torch.int64, device="cuda")
    ms = time_steps(torch, lambda i: F.polymul_i64(ta, tb, out=c), 20 if quick else 100, 5)
    out["polymul_i64_2x2^20"] = {"ms": ms, "Gcoeff_per_s": ((1 << 21) - 1) / ms / 1e6}
    # C3: big integers, 2 x 2^24 bits -> 2^21 limbs
    a, b = W.bigint_u16(1 << 20, W.SEED_BIGINT)
    ta, tb = torch.from_numpy(a.view(np.int16)).cuda(), torch.from_numpy(b.view(np.int16)).cuda()
    c = torch.empty(1 << 21, dtype=torch.int16, device="cuda")
    ms = time_steps(torch, lambda i: F.bigint_mul(ta, tb, out=c), 20 if quick else 100, 5)
    out["bigint_mul_2x2^24bit"] = {"ms": ms, "Glimb_per_s": (1 << 21) / ms / 1e6}
    out["bigint_fermat_2x2^24bit"] = bigint_fermat(torch, F, ta, tb, ms, quick)
    out["c1_n1024_latency"] = c1_latency(torch, F, W)
    out["circulant_vs_fft_c64_2^21"] = circulant_vs_fft(torch, F, W, quick)
    out["gfp2_section3_ring_2^21"] = gfp2_product(torch, F, quick)
    out["batched_c64_4096"] = batched_vs_plain(torch, F, W, quick)
    out["layer_fwd_bwd_256x2^14"] = layer_vs_plain(torch, F, W, quick)
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
    ms_f = time_steps(torch, classic, 20 if quick else 200, 10)
    yc = classic(0)
    rel = float(torch.linalg.vector_norm(ty - yc) / torch.linalg.vector_norm(yc))
    return {"circulant_ms": ms_c, "fft_ms": ms_f, "fft_over_circulant": ms_f / ms_c, "rel_l2_between": rel}


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
    return {"ms": ms, "Gcoeff_per_s": n / ms / 1e6}


def batched_vs_plain(torch, F, W, quick: bool):
    """4096 complex64 products of sizes 2^6..2^16 (seed 6): one persistent launch (its work
    queue reused) against one fcirc_matvec call per instance, on the same device buffers."""
    from paper_2103_02605_amd.batched import BatchPlan
    e, a_list, x_list = W.batched_c64(4096, W.SEED_BATCHED)
    plan = BatchPlan(a_list, x_list, dtype=np.complex64)
    total = int(plan.offsets[-1])
    ms_b = time_steps(torch, lambda i: plan.run(), 5 if quick else 20, 2)
    views = [(plan.a[plan.offsets[k]:plan.offsets[k + 1]], plan.x[plan.offsets[k]:plan.offsets[k + 1]],
              plan.y[plan.offsets[k]:plan.offsets[k + 1]]) for k in range(len(a_list))]

    def plain(i):
        for a, x, y in views:
            F.matvec(a, x, out=y)
    ms_p = time_steps(torch, plain, 1 if quick else 3, 1)
    return {"coefficients": total, "batched_ms": ms_b, "plain_ms": ms_p,
            "batched_Gcoeff_per_s": total / ms_b / 1e6, "plain_Gcoeff_per_s": total / ms_p / 1e6,
            "batched_over_plain": ms_p / ms_b}


def layer_vs_plain(torch, F, W, quick: bool):
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
    ms_p = time_steps(torch, plain, 1 if quick else 3, 1)
    return {"fwd_bwd_ms": ms_f, "plain_ms": ms_p, "fused_over_plain": ms_p / ms_f,
            "coefficients_per_pass": int(tx.numel())}


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
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run 3 plain 64 MiB device copies (torch), the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs each product on a single device "
              "(multi-GPU sharding is a design note, not built). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_02605_amd import fcirc as F
    from paper_2103_02605_amd import workloads as W

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
    roofline = {"bound": "alu", "kernel": dom, "achieved": round(dk["alu_Tops"], 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "Tops/s (32-bit VALU lane-ops)", "frac": round(dk["alu_Tops"] / VALU_PEAK_TOPS, 4),
                "traffic": traffic,
                "per_unit": f"{ops_coef[dom]} lane-ops per coefficient x {n} coefficients per launch",
                "hbm": {"achieved_GBs": round(12 * n / (ms * 1e-3) / 1e9, 1), "peak_GBs": HBM_PEAK_GBS,
                        "frac": round(12 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
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
        line["secondary"] = secondary(torch, F, W, quick=args.quick_secondary)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(W)
        line["cpu_baseline"] = cb
        line["gpu_over_cpu_oracle"] = round(value / cb["value"], 1)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
