// The f-circulant product over Z/(2^K + 1), the ring that section 3.2 of Rosowski (arXiv
// 2103.02605) proposes for Schoenhage-Strassen multiplication of large integers. There
// 2^K = -1, so 2 has order 2K, the roots of unity are powers of two, and a multiplication
// by a root is a shift: Algorithm 1 needs only the shift counts, no modular multiply and
// no root tables. The pointwise products at the leaves are full K-bit products.
//
// Element layout in device memory: K/32 words, least significant first, then one word
// that is 1 only for the value 2^K (= -1); canonical values lie in [0, 2^K], so an element
// takes W + 1 words, W = K/32 = 64 Q. In registers one wave holds one element: lane l has
// words [l Q, l Q + Q), and the top word is uniform over the wave. Carries cross lanes
// through a carry-lookahead on wave ballots (generate / propagate bits per lane).
//
// Node roots: the value at node (d, b) of the recursion is 2^v with
// v = (f_shift + 2K brev_d(b)) / 2^d mod 2K (the first child of a node 2^e takes 2^(e/2),
// the second -2^(e/2) = 2^(e/2 + K)); node (d, b) uses the root g = 2^(v/2). This needs
// 2^L | f_shift and 2^(L-1) | K.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <initializer_list>

#include "host.hpp"

namespace fcirc {

namespace {

constexpr int FM_WAVES = 4;  // waves (elements or butterflies) per workgroup

template <int Q>
struct FE {
  uint32_t w[Q];
  uint32_t hi;  // uniform: 1 only for the value 2^K
};

// The physical lane (workgroups are whole waves). Not a count of active lanes, so it stays
// right inside branches.
__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// r = a + b + cin over the wave's K-bit numbers; returns the carry out of bit K (uniform).
// Each lane adds its Q words with carry-in 0; a lane generates a carry (G) or, being all
// ones, propagates one (P). With A = G | P and B = G, the carries into the lanes are the
// carries of the 64-bit sum A + B + cin (bit l of (A + B + cin) ^ A ^ B).
template <int Q>
__device__ __forceinline__ uint32_t wadd(uint32_t (&r)[Q], const uint32_t (&a)[Q], const uint32_t (&b)[Q], uint32_t cin) {
  // (64-bit sums: the same chain written with 32-bit carry compares, which the compiler
  // turns into add-with-carry instructions, gave wrong results for a constant operand)
  uint32_t c = 0, all = 0xffffffffu;
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    const uint64_t t = (uint64_t)a[s] + b[s] + c;
    r[s] = (uint32_t)t;
    c = (uint32_t)(t >> 32);
    all &= r[s];
  }
  const uint64_t G = __ballot(c != 0);
  const uint64_t A = G | __ballot(all == 0xffffffffu && c == 0);
  const uint64_t S = A + G;
  const uint64_t S2 = S + (uint64_t)cin;
  const uint32_t cout = (S < A ? 1u : 0u) | (S2 < S ? 1u : 0u);
  uint32_t ci = (uint32_t)((S2 ^ A ^ G) >> lane_id()) & 1u;
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    const uint64_t t = (uint64_t)r[s] + ci;
    r[s] = (uint32_t)t;
    ci = (uint32_t)(t >> 32);
  }
  return cout;
}

// r = a + T, T a two's complement 96-bit value (t2:t1:t0) sign-extended to K bits.
template <int Q>
__device__ __forceinline__ uint32_t wadd_s96(uint32_t (&r)[Q], const uint32_t (&a)[Q], uint32_t t0, uint32_t t1,
                                             uint32_t t2) {
  const uint32_t ext = (int32_t)t2 < 0 ? 0xffffffffu : 0u;
  uint32_t b[Q];
  if constexpr (Q >= 4) {  // words 0..2 all sit in lane 0
    const bool l0 = lane_id() == 0;
#pragma unroll
    for (int s = 0; s < Q; ++s) b[s] = (l0 && s < 3) ? (s == 0 ? t0 : (s == 1 ? t1 : t2)) : ext;
  } else {
    const uint32_t base = lane_id() * Q;
#pragma unroll
    for (int s = 0; s < Q; ++s) {
      const uint32_t j = base + s;
      b[s] = j == 0 ? t0 : (j == 1 ? t1 : (j == 2 ? t2 : ext));
    }
  }
  return wadd<Q>(r, a, b, 0);
}

// The canonical element of r + T (r a K-bit number, |T| far below 2^K), using 2^K = -1:
// r + T either fits in K bits, or overflows by 2^K (then the value is its low part - 1),
// or goes below zero (then it is its low part + 2^K, i.e. low part + 1).
template <int Q>
__device__ __forceinline__ FE<Q> reduce96(const uint32_t (&r)[Q], uint32_t t0, uint32_t t1, uint32_t t2) {
  FE<Q> o;
  o.hi = 0;
  const bool tneg = (int32_t)t2 < 0;
  const uint32_t c = wadd_s96<Q>(o.w, r, t0, t1, t2);
  const int u = (!tneg && c) ? -1 : ((tneg && !c) ? 1 : 0);
  if (u != 0) {
    uint32_t w2[Q];
    const uint32_t e = u < 0 ? 0xffffffffu : 0u;
    const uint32_t c2 = wadd_s96<Q>(w2, o.w, (uint32_t)u, e, e);
    // -1 from 0, or +1 from 2^K - 1, lands on 2^K itself
    const bool top = u < 0 ? c2 == 0 : c2 != 0;
#pragma unroll
    for (int s = 0; s < Q; ++s) o.w[s] = top ? 0u : w2[s];
    o.hi = top ? 1u : 0u;
  }
  return o;
}

// The canonical element of r + h 2^K = r - h (h small).
template <int Q>
__device__ __forceinline__ FE<Q> reduce_hi(const uint32_t (&r)[Q], int32_t h) {
  const uint32_t t = (uint32_t)(-h), e = -h < 0 ? 0xffffffffu : 0u;
  return reduce96<Q>(r, t, e, e);
}

template <int Q>
__device__ __forceinline__ FE<Q> fadd(const FE<Q>& a, const FE<Q>& b) {
  uint32_t r[Q];
  const uint32_t c = wadd<Q>(r, a.w, b.w, 0);
  return reduce_hi<Q>(r, (int32_t)(c + a.hi + b.hi));
}

// a - b: a + (~b) + 1 = a - b + 2^K over K bits, with carry c: a - b = r + (c - 1) 2^K.
template <int Q>
__device__ __forceinline__ FE<Q> fsub(const FE<Q>& a, const FE<Q>& b) {
  uint32_t nb[Q], r[Q];
#pragma unroll
  for (int s = 0; s < Q; ++s) nb[s] = ~b.w[s];
  const uint32_t c = wadd<Q>(r, a.w, nb, 1);
  return reduce_hi<Q>(r, (int32_t)c - 1 + (int32_t)a.hi - (int32_t)b.hi);
}

template <int Q>
__device__ __forceinline__ FE<Q> fneg(const FE<Q>& a) {
  FE<Q> z;
#pragma unroll
  for (int s = 0; s < Q; ++s) z.w[s] = 0;
  z.hi = 0;
  return fsub<Q>(z, a);
}

// y[s] = x[(s - ds) mod Q] for a uniform ds in [0, Q).
template <int Q>
__device__ __forceinline__ void rot_regs(uint32_t (&y)[Q], const uint32_t (&x)[Q], uint32_t ds) {
#pragma unroll
  for (int s = 0; s < Q; ++s) y[s] = x[s];
#pragma unroll
  for (int r = 1; r < Q; ++r)
    if (ds == (uint32_t)r) {
#pragma unroll
      for (int s = 0; s < Q; ++s) y[s] = x[(s - r + Q) % Q];
    }
}

// m[s] = word (j - d) mod W of x, where j = l Q + s is the word this lane holds (d uniform,
// 0 <= d < W): register slot (s - d) mod Q of lane l - floor(d / Q) (one lane further
// when s < d mod Q).
template <int Q>
__device__ __forceinline__ void fetch_rot(uint32_t (&m)[Q], const uint32_t (&x)[Q], uint32_t d) {
  const uint32_t dl = d / Q, ds = d % Q, l = lane_id();
  uint32_t y[Q];
  rot_regs<Q>(y, x, ds);
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    const uint32_t delta = dl + ((uint32_t)s < ds ? 1u : 0u);
    m[s] = __shfl(y[s], (int)((l - delta) & 63u), 64);
  }
}

// x 2^e for 0 <= e < 2K. For e < K: x 2^e = lo + hp 2^K = lo - hp, where lo holds the low
// K bits of the shifted value and hp the bits shifted past bit K; for e >= K the result is
// negated (2^K = -1).
template <int Q>
__device__ __forceinline__ FE<Q> fshl(const FE<Q>& x, uint32_t e) {
  constexpr uint32_t K = 32u * 64u * Q;
  const bool negate = e >= K;
  const uint32_t ee = negate ? e - K : e;
  const uint32_t l = lane_id();
  if (x.hi) {  // x = -1: x 2^ee = -2^ee
    FE<Q> p;
    p.hi = 0;
#pragma unroll
    for (int s = 0; s < Q; ++s) p.w[s] = (l * Q + s == (ee >> 5)) ? (1u << (ee & 31u)) : 0u;
    return negate ? p : fneg<Q>(p);
  }
  if (ee == 0) return negate ? fneg<Q>(x) : x;
  const uint32_t ws = ee >> 5, bs = ee & 31u;
  uint32_t M[Q], F[Q];
  fetch_rot<Q>(M, x.w, ws);  // word j - ws (mod W) of x
  F[0] = __shfl(M[Q - 1], (int)((l + 63u) & 63u), 64);
#pragma unroll
  for (int s = 1; s < Q; ++s) F[s] = M[s - 1];  // word j - ws - 1 (mod W)
  uint32_t lo[Q], hp[Q];
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    const uint32_t j = l * Q + s;
    const bool w1 = j < ws, w2 = j <= ws;  // the source word wrapped past the top
    const uint32_t mv = M[s] << bs;
    const uint32_t fv = bs ? (F[s] >> (32u - bs)) : 0u;
    lo[s] = (w1 ? 0u : mv) | (w2 ? 0u : fv);
    hp[s] = (w1 ? mv : 0u) | (w2 ? fv : 0u);
  }
  uint32_t nb[Q], r[Q];
  uint32_t c;
  if (!negate) {
#pragma unroll
    for (int s = 0; s < Q; ++s) nb[s] = ~hp[s];
    c = wadd<Q>(r, lo, nb, 1);
  } else {
#pragma unroll
    for (int s = 0; s < Q; ++s) nb[s] = ~lo[s];
    c = wadd<Q>(r, hp, nb, 1);
  }
  return reduce_hi<Q>(r, (int32_t)c - 1);
}

// acc (96 bits: lo64, hi32) += a b. The product and the low 64 bits come from one 64-bit
// multiply-add; it wrapped exactly when the new low part is below the old one.
__device__ __forceinline__ void mac96(uint64_t& lo, uint32_t& hi, uint32_t a, uint32_t b) {
  const uint64_t t = (uint64_t)a * b + lo;
  hi += t < lo ? 1u : 0u;
  lo = t;
}

// Sum of the three shifted word arrays X0 + X1 2^32 + X2 2^64 (each W words in LDS) as a
// K-bit number r plus the part at or above 2^K, returned as a 96-bit value (uniform).
template <int Q>
__device__ __forceinline__ void combine3(uint32_t (&r)[Q], const uint32_t* x0, const uint32_t* x1, const uint32_t* x2,
                                         uint32_t& s0, uint32_t& s1, uint32_t& s2) {
  constexpr uint32_t W = 64u * Q;
  const uint32_t l = lane_id();
  uint32_t v0[Q], v1[Q], v2[Q], t[Q];
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    const uint32_t j = l * Q + s;
    v0[s] = x0[j];
    v1[s] = j >= 1 ? x1[j - 1] : 0u;
    v2[s] = j >= 2 ? x2[j - 2] : 0u;
  }
  const uint32_t c1 = wadd<Q>(t, v0, v1, 0);
  const uint32_t c2 = wadd<Q>(r, t, v2, 0);
  // spill at 2^K: x1[W-1] + x2[W-2] + x2[W-1] 2^32 + the two carries
  const uint64_t lo = (uint64_t)x1[W - 1] + x2[W - 2] + c1 + c2;
  const uint64_t hi = (uint64_t)x2[W - 1] + (lo >> 32);
  s0 = (uint32_t)lo;
  s1 = (uint32_t)hi;
  s2 = (uint32_t)(hi >> 32);
}

// a b mod 2^K + 1. The 32-bit word products are summed per column of the negacyclic
// convolution: a_i b_j lands in column (i + j) mod W, with a minus sign when i + j >= W
// (2^(32 W) = 2^K = -1). Lane l owns columns l + 64 m (m < Q); every column has exactly W
// terms, so the lanes stay balanced. Positive and negative parts are kept apart in 96-bit
// accumulators, moved to LDS, and recombined as K-bit numbers. sm: 8 W words of LDS (a,
// then b twice while the columns are summed; the six column arrays afterwards).
template <int Q>
__device__ __forceinline__ FE<Q> fmul(const FE<Q>& a, const FE<Q>& b, uint32_t* sm) {
  constexpr uint32_t W = 64u * Q;
  const uint32_t l = lane_id();
  if (a.hi || b.hi) {
    if (a.hi && b.hi) {  // (-1)(-1) = 1
      FE<Q> one;
      one.hi = 0;
#pragma unroll
      for (int s = 0; s < Q; ++s) one.w[s] = (l * Q + s == 0) ? 1u : 0u;
      return one;
    }
    return fneg<Q>(a.hi ? b : a);
  }
  uint32_t* sa = sm;
  uint32_t* sb = sm + W;  // b twice: sb[j] = sb[j + W] = b_j, so (c - i) mod W needs no wrap
#pragma unroll
  for (int s = 0; s < Q; ++s) {
    sa[l * Q + s] = a.w[s];
    sb[l * Q + s] = b.w[s];
    sb[W + l * Q + s] = b.w[s];
  }
  wave_lds_sync();
  uint64_t pl[Q], nl[Q];  // low 64 bits of the positive and negative column sums
  uint32_t ph[Q], nh[Q];  // their bits 64..95
#pragma unroll
  for (int m = 0; m < Q; ++m) pl[m] = nl[m] = 0, ph[m] = nh[m] = 0;
  // i = 64 t + u; column c_m = l + 64 m receives a_i b_((c_m - i) mod W), positive when
  // i <= c_m: for t < m always, for t > m never, for t == m when u <= l.
  constexpr int UNROLL_U = Q <= 4 ? 4 : 1;  // beyond Q = 4 the unrolled body only adds registers
#pragma unroll
  for (int t = 0; t < Q; ++t) {
#pragma unroll UNROLL_U
    for (uint32_t u = 0; u < 64u; ++u) {
      const uint32_t i = 64u * t + u;
      const uint32_t ai = sa[i];
      const uint32_t* sbi = sb + (l + W - i);  // column c_m reads sbi[64 m], index in [1, 2W)
#pragma unroll
      for (int m = 0; m < Q; ++m) {
        const uint32_t bj = sbi[64 * m];
        if (m > t) {
          mac96(pl[m], ph[m], ai, bj);
        } else if (m < t) {
          mac96(nl[m], nh[m], ai, bj);
        } else {
          const uint32_t bp = u <= l ? bj : 0u;
          mac96(pl[m], ph[m], ai, bp);
          mac96(nl[m], nh[m], ai, bj - bp);
        }
      }
    }
  }
  wave_lds_sync();  // all reads of sa, sb done before the columns overwrite them
  uint32_t* c0 = sm;  // [p0 p1 p2 n0 n1 n2], W words each
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    const uint32_t col = l + 64u * m;
    c0[col] = (uint32_t)pl[m];
    c0[W + col] = (uint32_t)(pl[m] >> 32);
    c0[2 * W + col] = ph[m];
    c0[3 * W + col] = (uint32_t)nl[m];
    c0[4 * W + col] = (uint32_t)(nl[m] >> 32);
    c0[5 * W + col] = nh[m];
  }
  wave_lds_sync();
  uint32_t rp[Q], rn[Q];
  uint32_t sp0, sp1, sp2, sn0, sn1, sn2;
  combine3<Q>(rp, c0, c0 + W, c0 + 2 * W, sp0, sp1, sp2);
  combine3<Q>(rn, c0 + 3 * W, c0 + 4 * W, c0 + 5 * W, sn0, sn1, sn2);
  wave_lds_sync();  // the next call may overwrite this wave's LDS
  // value = (rp - sp) - (rn - sn); rp - rn = d + (c - 1) 2^K = d + 1 - c
  uint32_t nb[Q], d[Q];
#pragma unroll
  for (int s = 0; s < Q; ++s) nb[s] = ~rn[s];
  const uint32_t c = wadd<Q>(d, rp, nb, 1);
  // T = sn - sp + 1 - c as a two's complement 96-bit value
  const unsigned __int128 spv = ((unsigned __int128)sp2 << 64) | ((uint64_t)sp1 << 32) | sp0;
  const unsigned __int128 snv = ((unsigned __int128)sn2 << 64) | ((uint64_t)sn1 << 32) | sn0;
  const unsigned __int128 T = snv - spv + 1u - c;
  return reduce96<Q>(d, (uint32_t)T, (uint32_t)(T >> 32), (uint32_t)(T >> 64));
}

template <int Q>
__device__ __forceinline__ FE<Q> fload(const uint32_t* p) {
  FE<Q> e;
  const uint32_t l = lane_id();
#pragma unroll
  for (int s = 0; s < Q; ++s) e.w[s] = p[l * Q + s];
  e.hi = p[64u * Q];
  return e;
}

template <int Q>
__device__ __forceinline__ void fstore(uint32_t* p, const FE<Q>& e) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int s = 0; s < Q; ++s) p[l * Q + s] = e.w[s];
  if (l == 0) p[64u * Q] = e.hi;
}

__device__ __forceinline__ uint32_t brev_bits(uint32_t v, uint32_t bits) {
  return bits == 0 ? 0u : (__brev(v) >> (32u - bits));
}

// Shift count of the root g used at node (d, b): (f_shift + 2K brev_d(b)) / 2^(d+1) mod 2K.
__device__ __forceinline__ uint32_t root_shift(uint32_t f_shift, uint32_t K, uint32_t d, uint32_t b) {
  const uint32_t v = f_shift + 2u * K * brev_bits(b, d);
  return (v >> (d + 1)) % (2u * K);
}

// R split levels d .. d + R - 1 in one pass. A wave takes the E = 2^R elements
// k + j q (j < E, q = n / 2^(d+R)) of one depth-d block b: at level d + l the pairs
// (j, j + E / 2^(l+1)) of sub-block s use the root of node (d + l, b 2^l + s). Row
// (IS_X false): (u, v) -> (u + g v, u - g v); vector: (u, v) -> (g u + v, g u - v).
// src may equal dst.
// Split level l of a pass (then the levels below it), with compile-time indices so that
// the E elements stay in registers.
template <int Q, int R, int l, bool IS_X>
__device__ __forceinline__ void fm_split_from(FE<Q>* v, uint32_t b, uint32_t d, uint32_t f_shift) {
  if constexpr (l < R) {
    constexpr uint32_t K = 32u * 64u * Q;
    constexpr int E = 1 << R, h = E >> (l + 1);
#pragma unroll
    for (int sb = 0; sb < (1 << l); ++sb) {
      const uint32_t e = root_shift(f_shift, K, d + l, (b << l) + sb);
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const int j = sb * 2 * h + i;
        if constexpr (IS_X) {
          const FE<Q> g = fshl<Q>(v[j], e);
          v[j] = fadd<Q>(g, v[j + h]);
          v[j + h] = fsub<Q>(g, v[j + h]);
        } else {
          const FE<Q> g = fshl<Q>(v[j + h], e);
          v[j + h] = fsub<Q>(v[j], g);
          v[j] = fadd<Q>(v[j], g);
        }
      }
    }
    fm_split_from<Q, R, l + 1, IS_X>(v, b, d, f_shift);
  }
}

template <int Q, int R, bool IS_X>
__device__ __forceinline__ void fm_split_levels(const uint32_t* src, uint32_t* dst, uint32_t k, uint32_t q, uint32_t b,
                                                uint32_t d, uint32_t f_shift) {
  constexpr uint32_t S = 64u * Q + 1;
  constexpr int E = 1 << R;
  FE<Q> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = fload<Q>(src + (size_t)(k + j * q) * S);
  fm_split_from<Q, R, 0, IS_X>(v, b, d, f_shift);
#pragma unroll
  for (int j = 0; j < E; ++j) fstore<Q>(dst + (size_t)(k + j * q) * S, v[j]);
}

template <int Q, int R>
__global__ void __launch_bounds__(64 * FM_WAVES) k_fm_split(const uint32_t* a_in, const uint32_t* x_in, uint32_t* wa,
                                                            uint32_t* wx, uint32_t n, uint32_t d, uint32_t f_shift) {
  constexpr int E = 1 << R;
  const uint32_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * FM_WAVES + (threadIdx.x >> 6));  // one per wave
  if (t >= (n >> R)) return;
  const uint32_t q = n >> (d + R), b = t / q, k = b * E * q + (t - b * q);
  fm_split_levels<Q, R, false>(a_in, wa, k, q, b, d, f_shift);
  fm_split_levels<Q, R, true>(x_in, wx, k, q, b, d, f_shift);
}

// Four levels d .. d + 3 in one pass, exchanged through LDS: a workgroup of four waves
// takes the 16 elements k + j q (j < 16, q = n / 2^(d+4)) of one depth-d block b. For
// levels d and d + 1, wave w holds elements w + 4i (i < 4): a two-level pass over block b.
// For levels d + 2 and d + 3 it holds elements 4w + i: a two-level pass over the
// depth-(d+2) block 4b + w. Every element is read from memory and written back once per
// four levels (twice per two-level pass).
static_assert(FM_WAVES == 4, "a four-level pass takes one wave per quarter of its 16 elements");

template <int Q, bool IS_X>
__device__ __forceinline__ void fm_split4_array(const uint32_t* src, uint32_t* dst, uint32_t* sm, uint32_t k, uint32_t q,
                                                uint32_t b, uint32_t d, uint32_t f_shift, uint32_t w) {
  constexpr uint32_t S = 64u * Q + 1;
  FE<Q> v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = fload<Q>(src + (size_t)(k + (w + 4u * i) * q) * S);
  fm_split_from<Q, 2, 0, IS_X>(v, b, d, f_shift);
#pragma unroll
  for (int i = 0; i < 4; ++i) fstore<Q>(sm + (w + 4u * i) * S, v[i]);
  __syncthreads();  // also: every element of the group has been read before any is written
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = fload<Q>(sm + (4u * w + i) * S);
  fm_split_from<Q, 2, 0, IS_X>(v, 4u * b + w, d + 2, f_shift);
#pragma unroll
  for (int i = 0; i < 4; ++i) fstore<Q>(dst + (size_t)(k + (4u * w + i) * q) * S, v[i]);
}

// grid: 2 n / 16 workgroups of 4 waves, the row's groups then the vector's.
template <int Q>
__global__ void __launch_bounds__(64 * FM_WAVES) k_fm_split4(const uint32_t* a_in, const uint32_t* x_in, uint32_t* wa,
                                                             uint32_t* wx, uint32_t n, uint32_t d, uint32_t f_shift) {
  constexpr uint32_t S = 64u * Q + 1;
  __shared__ uint32_t sm[16 * S];
  const uint32_t groups = n >> 4;
  const bool is_x = blockIdx.x >= groups;
  const uint32_t t = is_x ? blockIdx.x - groups : blockIdx.x;
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t q = n >> (d + 4), b = t / q, k = b * 16u * q + (t - b * q);
  if (is_x)
    fm_split4_array<Q, true>(x_in, wx, sm, k, q, b, d, f_shift, w);
  else
    fm_split4_array<Q, false>(a_in, wa, sm, k, q, b, d, f_shift, w);
}

// Leaves: y_k = a_k x_k / n (1/n = 2^(2K - L)), one wave per element.
template <int Q>
__global__ void __launch_bounds__(64 * FM_WAVES) k_fm_leaf(const uint32_t* a, const uint32_t* x, uint32_t* y, uint32_t n,
                                                           uint32_t L) {
  constexpr uint32_t W = 64u * Q, K = 32u * W, S = W + 1;
  __shared__ uint32_t sm[FM_WAVES * 8 * W];
  const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t k = blockIdx.x * FM_WAVES + wv;
  if (k >= n) return;
  const FE<Q> p = fmul<Q>(fload<Q>(a + (size_t)k * S), fload<Q>(x + (size_t)k * S), sm + wv * 8 * W);
  fstore<Q>(y + (size_t)k * S, fshl<Q>(p, (2u * K - L) % (2u * K)));
}

// R merge levels d + R - 1 .. d in one pass (the inverse order of k_fm_split; the 1/2 of
// each level is folded into the leaves): (M1, M2) -> ((M1 + M2) / g, M1 - M2), in place.
// Merge level l of a pass (then the levels above it), compile-time indices as above.
template <int Q, int R, int l>
__device__ __forceinline__ void fm_merge_from(FE<Q>* v, uint32_t b, uint32_t d, uint32_t f_shift) {
  if constexpr (l >= 0) {
    constexpr uint32_t K = 32u * 64u * Q;
    constexpr int E = 1 << R, h = E >> (l + 1);
#pragma unroll
    for (int sb = 0; sb < (1 << l); ++sb) {
      const uint32_t e = root_shift(f_shift, K, d + l, (b << l) + sb);
#pragma unroll
      for (int i = 0; i < h; ++i) {
        const int j = sb * 2 * h + i;
        const FE<Q> sum = fadd<Q>(v[j], v[j + h]);
        v[j + h] = fsub<Q>(v[j], v[j + h]);
        v[j] = fshl<Q>(sum, (2u * K - e) % (2u * K));
      }
    }
    fm_merge_from<Q, R, l - 1>(v, b, d, f_shift);
  }
}

template <int Q, int R>
__global__ void __launch_bounds__(64 * FM_WAVES) k_fm_merge(uint32_t* y, uint32_t n, uint32_t d, uint32_t f_shift) {
  constexpr uint32_t S = 64u * Q + 1;
  constexpr int E = 1 << R;
  const uint32_t t = __builtin_amdgcn_readfirstlane(blockIdx.x * FM_WAVES + (threadIdx.x >> 6));  // one per wave
  if (t >= (n >> R)) return;
  const uint32_t q = n >> (d + R), b = t / q, k = b * E * q + (t - b * q);
  FE<Q> v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) v[j] = fload<Q>(y + (size_t)(k + j * q) * S);
  fm_merge_from<Q, R, R - 1>(v, b, d, f_shift);
#pragma unroll
  for (int j = 0; j < E; ++j) fstore<Q>(y + (size_t)(k + j * q) * S, v[j]);
}

// Four merge levels d + 3 .. d in one pass (the inverse of k_fm_split4), in place.
// grid: n / 16 workgroups of 4 waves.
template <int Q>
__global__ void __launch_bounds__(64 * FM_WAVES) k_fm_merge4(uint32_t* y, uint32_t n, uint32_t d, uint32_t f_shift) {
  constexpr uint32_t S = 64u * Q + 1;
  __shared__ uint32_t sm[16 * S];
  const uint32_t t = blockIdx.x;
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t q = n >> (d + 4), b = t / q, k = b * 16u * q + (t - b * q);
  FE<Q> v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = fload<Q>(y + (size_t)(k + (4u * w + i) * q) * S);
  fm_merge_from<Q, 2, 1>(v, 4u * b + w, d + 2, f_shift);
#pragma unroll
  for (int i = 0; i < 4; ++i) fstore<Q>(sm + (4u * w + i) * S, v[i]);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = fload<Q>(sm + (w + 4u * i) * S);
  fm_merge_from<Q, 2, 1>(v, b, d, f_shift);
#pragma unroll
  for (int i = 0; i < 4; ++i) fstore<Q>(y + (size_t)(k + (w + 4u * i) * q) * S, v[i]);
}

// Canonical form of n elements (the input check): the top word is 0 or 1, and 1 only
// with every other word 0. One thread per element; the words are read only when the top
// word is 1.
__global__ void k_fm_check(const uint32_t* __restrict__ v, uint32_t n, uint32_t W, uint32_t* flag) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t* e = v + (size_t)k * (W + 1);
  const uint32_t hi = e[W];
  bool bad = hi > 1;
  if (hi == 1) {
    uint32_t acc = 0;
    for (uint32_t w = 0; w < W; ++w) acc |= e[w];
    bad = acc != 0;
  }
  if (bad) atomicOr(flag, 1u);
}

// Pieces of a large integer (16-bit limbs) as ring elements: element k holds piece j of
// pw words (j = k, or j = (n - k) mod n for the reversed defining row), zero-extended.
__global__ void k_fm_pack(const uint16_t* __restrict__ src, uint64_t nlimbs, uint32_t pw, uint32_t n, uint32_t W,
                          uint32_t reverse, uint32_t* __restrict__ dst) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t S = (uint64_t)W + 1;
  if (idx >= (uint64_t)n * S) return;
  const uint32_t k = (uint32_t)(idx / S), w = (uint32_t)(idx % S);
  const uint32_t j = reverse ? (n - k) & (n - 1u) : k;
  uint32_t v = 0;
  if (w < pw) {
    const uint64_t l0 = 2 * ((uint64_t)j * pw + w);
    const uint32_t lo = l0 < nlimbs ? src[l0] : 0u;
    const uint32_t hi = l0 + 1 < nlimbs ? src[l0 + 1] : 0u;
    v = lo | (hi << 16);
  }
  dst[idx] = v;
}

// coef[k] = sum over pieces j of limb k - j p16 of y_j (each y_j < 2^K, 2 W limbs).
__global__ void k_fm_coef(const uint32_t* __restrict__ y, uint32_t n, uint32_t W, uint32_t p16, uint64_t nc,
                          uint64_t* __restrict__ coef) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nc) return;
  const uint64_t span = 2ull * W;  // limbs per element
  const uint64_t jhi = std::min<uint64_t>(n - 1, k / p16);
  const uint64_t jlo = k >= span ? (k - span) / p16 + 1 : 0;
  uint64_t s = 0;
  for (uint64_t j = jlo; j <= jhi; ++j) {
    const uint64_t off = k - j * p16;  // < 2 W
    const uint32_t word = y[j * ((uint64_t)W + 1) + (off >> 1)];
    s += (off & 1) ? (word >> 16) : (word & 0xFFFFu);
  }
  coef[k] = s;
}

// Levels per split or merge pass. A register pass holds 2^R elements of Q words per lane:
// measured on MI355X for the 2 x 2^24-bit product (K = 8192, 2^14 pieces), register passes
// of 3 and 4 levels took 545 and 720 us against 499 us with 2 levels, their registers (200
// and 256 per lane in the split) cutting occupancy more than the fewer passes save. Four
// levels go through LDS instead (k_fm_split4, k_fm_merge4: two 2-level steps per pass, the
// registers of a 2-level pass); the 1..3 levels left take register passes of 2 and 1.
template <int Q, int R>
hipError_t fm_split_pass(Ctx& c, const uint32_t* sa, const uint32_t* sx, uint32_t* wa, uint32_t* wx, uint32_t n, uint32_t d,
                         uint32_t f_shift, hipStream_t s) {
  const uint32_t grid = ((n >> R) + FM_WAVES - 1) / FM_WAVES;
  return launch(c, "fcirc_fermat_split", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, (k_fm_split<Q, R>), dim3(grid), dim3(64 * FM_WAVES), 0, s, sa, sx, wa, wx, n, d, f_shift);
  });
}

template <int Q, int R>
hipError_t fm_merge_pass(Ctx& c, uint32_t* y, uint32_t n, uint32_t d, uint32_t f_shift, hipStream_t s) {
  const uint32_t grid = ((n >> R) + FM_WAVES - 1) / FM_WAVES;
  return launch(c, "fcirc_fermat_merge", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, (k_fm_merge<Q, R>), dim3(grid), dim3(64 * FM_WAVES), 0, s, y, n, d, f_shift);
  });
}

template <int Q>
hipError_t fm_split4_pass(Ctx& c, const uint32_t* sa, const uint32_t* sx, uint32_t* wa, uint32_t* wx, uint32_t n, uint32_t d,
                          uint32_t f_shift, hipStream_t s) {
  return launch(c, "fcirc_fermat_split", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, k_fm_split4<Q>, dim3(2 * (n >> 4)), dim3(64 * FM_WAVES), 0, s, sa, sx, wa, wx, n, d, f_shift);
  });
}

template <int Q>
hipError_t fm_merge4_pass(Ctx& c, uint32_t* y, uint32_t n, uint32_t d, uint32_t f_shift, hipStream_t s) {
  return launch(c, "fcirc_fermat_merge", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, k_fm_merge4<Q>, dim3(n >> 4), dim3(64 * FM_WAVES), 0, s, y, n, d, f_shift);
  });
}

template <int Q>
hipError_t fm_product_q(Ctx& c, const uint32_t* a, const uint32_t* x, uint32_t* y, int L, uint32_t f_shift, uint32_t* wa,
                        uint32_t* wx, hipStream_t s) {
  const uint32_t n = 1u << L;
  // passes from the top: 4 levels while at least 4 are left, then 2, then 1
  int pd[32], pr[32], np = 0;
  for (int d = 0; d < L;) {
    const int r = L - d >= 4 ? 4 : std::min(2, L - d);
    pd[np] = d;
    pr[np] = r;
    ++np;
    d += r;
  }
  hipError_t e = hipSuccess;
  const uint32_t* sa = a;
  const uint32_t* sx = x;
  for (int i = 0; i < np && e == hipSuccess; ++i) {
    const uint32_t dd = (uint32_t)pd[i];
    if (pr[i] == 4) e = fm_split4_pass<Q>(c, sa, sx, wa, wx, n, dd, f_shift, s);
    else if (pr[i] == 2) e = fm_split_pass<Q, 2>(c, sa, sx, wa, wx, n, dd, f_shift, s);
    else e = fm_split_pass<Q, 1>(c, sa, sx, wa, wx, n, dd, f_shift, s);
    sa = wa;
    sx = wx;
  }
  if (e != hipSuccess) return e;
  const uint32_t LL = (uint32_t)L, gl = (n + FM_WAVES - 1) / FM_WAVES;
  e = launch(c, "fcirc_fermat_leaf", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, k_fm_leaf<Q>, dim3(gl), dim3(64 * FM_WAVES), 0, s, sa, sx, y, n, LL);
  });
  // the same passes in reverse order (none when n = 1)
  for (int i = np - 1; i >= 0 && e == hipSuccess; --i) {
    const uint32_t dd = (uint32_t)pd[i];
    if (pr[i] == 4) e = fm_merge4_pass<Q>(c, y, n, dd, f_shift, s);
    else if (pr[i] == 2) e = fm_merge_pass<Q, 2>(c, y, n, dd, f_shift, s);
    else e = fm_merge_pass<Q, 1>(c, y, n, dd, f_shift, s);
  }
  return e;
}

// Workspace: two arrays of n elements (the transformed row and vector).
hipError_t fm_product(Ctx& c, const uint32_t* a, const uint32_t* x, uint32_t* y, int L, int q, uint32_t f_shift,
                      uint32_t* wa, uint32_t* wx, hipStream_t s) {
  switch (q) {
    case 1: return fm_product_q<1>(c, a, x, y, L, f_shift, wa, wx, s);
    case 2: return fm_product_q<2>(c, a, x, y, L, f_shift, wa, wx, s);
    case 4: return fm_product_q<4>(c, a, x, y, L, f_shift, wa, wx, s);
    case 8: return fm_product_q<8>(c, a, x, y, L, f_shift, wa, wx, s);
    default: return hipErrorInvalidValue;
  }
}

// Parameters of the large-integer product: words per lane q (K = 2048 q), log2 of the
// number of pieces L, and piece size pw words. The coefficients of the product stay below
// 2^K when 32 pw 2 + L <= K (at most 2^(L-1) nonzero products of pieces < 2^(32 pw)), the
// pieces of both factors fit in 2^L, and 2^(L-1) | K. Among the feasible (q, L) the one
// with the fewest estimated operations wins (3 L levels of W-word butterflies, and W^2
// word products per leaf).
struct FmPlan {
  int q = 0, L = 0;
  uint32_t pw = 0;
};

FmPlan fm_plan(uint64_t na, uint64_t nb) {
  FmPlan best;
  double best_cost = 0;
  for (int q : {1, 2, 4, 8}) {
    const uint32_t K = 2048u * q, W = 64u * q;
    const int lmax = 12 + ilog2((uint64_t)q);
    for (int L = 1; L <= lmax; ++L) {
      const uint32_t pw = (K - (uint32_t)L) / 64u;  // 64 pw + L <= K
      if (pw == 0) break;
      const uint64_t pa = (na + 2ull * pw - 1) / (2ull * pw), pb = (nb + 2ull * pw - 1) / (2ull * pw);
      if (pa + pb - 1 > (1ull << L)) continue;
      const double cost = (double)(1ull << L) * W * (3.0 * L * 40.0 + 6.0 * W);
      if (best.q == 0 || cost < best_cost) {
        best = FmPlan{q, L, pw};
        best_cost = cost;
      }
      break;  // larger L with the same q only costs more
    }
  }
  return best;
}

}  // namespace

fcirc_status fermat_matvec(Ctx& c, const uint32_t* a, const uint32_t* x, uint32_t* y, int L, int q, uint32_t f_shift,
                           hipStream_t s) {
  const uint32_t n = 1u << L, W = 64u * q;
  if (c.check_inputs) {  // canonical inputs, checked before anything is written
    uint32_t* flag = c.d_status + 1;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(uint32_t), s);
    for (const uint32_t* v : {a, x}) {
      if (e != hipSuccess) break;
      e = launch(c, "fcirc_input_check", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
        FCIRC_LAUNCH(e0_, e1_, k_fm_check, dim3((n + 255) / 256), dim3(256), 0, s, v, n, W, flag);
      });
    }
    uint32_t bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof bad, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e);
    if (bad) return FCIRC_EINVAL;
  }
  const uint64_t elems = ((uint64_t)1 << L) * (64ull * q + 1);
  fcirc_status st = ws_reserve(c, 2 * elems * sizeof(uint32_t));
  if (st != FCIRC_OK) return st;
  uint32_t* wa = (uint32_t*)c.ws;
  return hip_status(fm_product(c, a, x, y, L, q, f_shift, wa, wa + elems, s));
}

fcirc_status fermat_bigint_mul(Ctx& c, const uint16_t* a, uint64_t na, const uint16_t* b, uint64_t nb, uint16_t* out,
                               hipStream_t s) {
  const FmPlan P = fm_plan(na, nb);
  if (P.q == 0) return FCIRC_ESIZE;
  const uint32_t n = 1u << P.L, W = 64u * P.q;
  const uint64_t elems = (uint64_t)n * (W + 1);
  // every limb position of the product (a coefficient y_j spans 2 W limbs from position
  // j p16 on, so its upper limbs land above position na + nb - 2)
  const uint64_t nl = na + nb, nc = nl, nblk = carry_blocks(nl);
  // layout (uint32 units): row | vector | y | transformed row | transformed vector | coef u64[nc] | u[nl] | summaries
  const uint64_t off_c = 5 * elems, off_u = off_c + 2 * nc, off_s = off_u + nl, total = off_s + 2 * nblk;
  fcirc_status st = ws_reserve(c, total * sizeof(uint32_t));
  if (st != FCIRC_OK) return st;
  uint32_t* base = (uint32_t*)c.ws;
  uint32_t *row = base, *vec = base + elems, *y = base + 2 * elems, *wa = base + 3 * elems, *wx = base + 4 * elems;
  uint64_t* coef = (uint64_t*)(base + off_c);
  const uint32_t grid_p = (uint32_t)((elems + 255) / 256);
  const uint32_t pw = P.pw;
  hipError_t e = launch(c, "fcirc_fermat_pack", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, k_fm_pack, dim3(grid_p), dim3(256), 0, s, a, na, pw, n, W, 1u, row);
  });
  if (e == hipSuccess)
    e = launch(c, "fcirc_fermat_pack", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
      FCIRC_LAUNCH(e0_, e1_, k_fm_pack, dim3(grid_p), dim3(256), 0, s, b, nb, pw, n, W, 0u, vec);
    });
  if (e == hipSuccess) e = fm_product(c, row, vec, y, P.L, P.q, 0u, wa, wx, s);
  if (e == hipSuccess)
    e = launch(c, "fcirc_fermat_coef", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
      FCIRC_LAUNCH(e0_, e1_, k_fm_coef, dim3((uint32_t)((nc + 255) / 256)), dim3(256), 0, s, y, n, W, 2u * pw, nc, coef);
    });
  if (e != hipSuccess) return hip_status(e);
  return carry_to_limbs(c, coef, nc, nl, base + off_u, base + off_s, out, s);
}

}  // namespace fcirc
