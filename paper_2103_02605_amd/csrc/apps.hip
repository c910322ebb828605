// Applications of the f-circulant product (Rosowski, arXiv 2103.02605, section 3):
// exact integer polynomial products (section 3.1) and large-integer products (the
// application of section 3.2), through three Z/p products and the Chinese remainder
// theorem.
//
// Section 3.1 fills both polynomials up to a power-of-two length N and multiplies them as
// one circulant product. The cyclic convolution sum_j a_j b_((i-j) mod N) equals
// (C(r) b)_i for the circulant whose first row is r_k = a_((-k) mod N), so the row loader
// reads a in reversed index order and the vector loader reads b; both fill with zeros.
// With N >= na + nb - 1 the cyclic and the plain product coincide.
//
// The CRT uses Garner's mixed-radix digits v1, v2, v3 (x = v1 + v2 p1 + v3 p1 p2) and
// reads a signed result with |c| < p1 p2 as v3 = 0 (c >= 0) or v3 = p3 - 1 (c < 0);
// any other v3 is a range error.
#include <hip/hip_runtime.h>

#include "host.hpp"

namespace fcirc {

namespace {

constexpr uint32_t Q1 = 998244353u, Q2 = 469762049u, Q3 = 167772161u;

// A signed 32-bit input enters as a residue in (0, 3p), not reduced further: every first
// operation of the product (split butterfly, or the leaf product of a one-element block)
// takes operands below 4p. v + 2^31 is brought to [0, 2p) by Shoup's method with w = 1,
// then 2^31 mod p is subtracted as p - (2^31 mod p) added.
template <class V>
__device__ __forceinline__ uint32_t residue_of(const Zp& R, V v) {
  if constexpr (sizeof(V) == 4) {
    const uint32_t u = (uint32_t)(int32_t)v ^ 0x80000000u;
    const uint32_t r = u - __umulhi(u, R.one.wp) * R.p;
    return r + (R.p - R.two31);
  } else {
    return (uint32_t)v;
  }
}
// Both loaders read unconditionally (element 0 when the index is past the data: na and nb
// are at least 1) and select zero afterwards, so the loads of a stage are all issued before
// the first wait instead of one branch, load and wait per element.
// Indices are 32-bit: N = 2^L <= 2^26 and na, nb <= N.
template <class V>
struct LdRowRev {  // r_k = a_((N - k) mod N), zero beyond na
  const V* a;
  uint32_t na, N;
  __device__ __forceinline__ uint32_t operator()(const Zp& R, uint32_t, uint32_t k) const {
    const uint32_t j = (N - k) & (N - 1);
    const bool in = j < na;
    const uint32_t r = residue_of(R, a[in ? j : 0u]);
    return in ? r : 0u;
  }
};
template <class V>
struct LdVecPad {  // b_k, zero beyond nb
  const V* b;
  uint32_t nb;
  __device__ __forceinline__ uint32_t operator()(const Zp& R, uint32_t, uint32_t k) const {
    const bool in = k < nb;
    const uint32_t r = residue_of(R, b[in ? k : 0]);
    return in ? r : 0u;
  }
};

struct CrtConsts {
  ZpTw one2, one3;           // reductions mod p2, p3
  ZpTw inv12, inv13, inv23;  // p1^-1 mod p2, p1^-1 mod p3, p2^-1 mod p3
};

__device__ __forceinline__ uint32_t shoup_mod(uint32_t v, ZpTw t, uint32_t p) {
  uint32_t r = v * t.w - __umulhi(v, t.wp) * p;  // [0, 2p)
  return min(r, r - p);
}

// Garner: residues (r1, r2, r3) -> digits; returns v3, writes c = v1 + v2 p1.
__device__ __forceinline__ uint32_t garner(uint32_t r1, uint32_t r2, uint32_t r3, const CrtConsts& K, uint64_t* c) {
  const uint32_t t2 = shoup_mod(r1, K.one2, Q2);
  uint32_t d2 = r2 + Q2 - t2;
  d2 = min(d2, d2 - Q2);
  const uint32_t v2 = shoup_mod(d2, K.inv12, Q2);
  const uint32_t t3 = shoup_mod(r1, K.one3, Q3);
  uint32_t d3 = r3 + Q3 - t3;
  d3 = min(d3, d3 - Q3);
  uint32_t e3 = shoup_mod(d3, K.inv13, Q3);
  const uint32_t w3 = shoup_mod(v2, K.one3, Q3);
  e3 = e3 + Q3 - w3;
  e3 = min(e3, e3 - Q3);
  const uint32_t v3 = shoup_mod(e3, K.inv23, Q3);
  *c = (uint64_t)r1 + (uint64_t)v2 * Q1;
  return v3;
}

// c_k for k < nc from residues res[i * N + k]; signed int64 (polymul).
__global__ void k_crt_i64(const uint32_t* __restrict__ res, uint64_t N, uint64_t nc, CrtConsts K, int64_t* __restrict__ out,
                          uint32_t* status) {
  const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nc) return;
  uint64_t c;
  const uint32_t v3 = garner(res[k], res[N + k], res[2 * N + k], K, &c);
  int64_t v;
  if (v3 == 0) {
    v = (int64_t)c;
  } else if (v3 == Q3 - 1) {
    v = (int64_t)c - (int64_t)((uint64_t)Q1 * Q2);
  } else {
    v = 0;
    atomicOr(status, FCIRC_STATUS_RANGE);
  }
  out[k] = v;
}

// Carries. The value is sum_k c_k 2^(16k) with c_k < 2^52. With digit_t(c) = 16-bit digit t,
// s_j = sum_{t<4} digit_t(c_(j-t)) < 2^18 and u_j = (s_j mod 2^16) + floor(s_(j-1) / 2^16)
// <= 2^16 + 2 keep the same value; then one carry-lookahead pass over u finishes it:
// limb_j = (u_j + cin_j) mod 2^16 with cin_(j+1) = [u_j >= 2^16] or ([u_j = 2^16 - 1] and cin_j).
constexpr int CARRY_PER_THREAD = 8;  // 8 against 16 (twice the workgroups): 2 x 2^24 bits 102.2 against 103.1 us
constexpr int CARRY_NT = 256;
constexpr int CARRY_BLOCK = CARRY_PER_THREAD * CARRY_NT;  // limbs per workgroup

// (generate, propagate) composition: right = later limb. Identity: (0, 1).
struct GP {
  uint32_t g, p;
};
__device__ __forceinline__ GP gp_combine(GP first, GP later) { return GP{later.g | (later.p & first.g), later.p & first.p}; }
__device__ __forceinline__ uint32_t gp_pack(GP a) { return a.g | (a.p << 1); }
__device__ __forceinline__ GP gp_unpack(uint32_t v) { return GP{v & 1u, (v >> 1) & 1u}; }
__device__ __forceinline__ GP gp_of(uint32_t u) { return GP{u >= 0x10000u ? 1u : 0u, u == 0xFFFFu ? 1u : 0u}; }

// Ordered inclusive scan of one GP per thread over the workgroup (thread order): wave64
// shuffles, then the wave totals in order. sh holds CARRY_NT / 64 words. *total = the
// composition over all threads.
__device__ __forceinline__ GP block_scan_gp(GP v, uint32_t* sh, GP* total) {
  constexpr int NW = CARRY_NT / 64;
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = gp_pack(v);
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x = gp_pack(gp_combine(gp_unpack(y), gp_unpack(x)));
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  GP pre{0u, 1u}, tot{0u, 1u};
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const GP t = gp_unpack(sh[q]);
    if ((uint32_t)q < w) pre = gp_combine(pre, t);
    tot = gp_combine(tot, t);
  }
  *total = tot;
  return gp_combine(pre, gp_unpack(x));
}

// LDS index of limb k of a block with one pad word per 16 (conflict-free per-thread runs).
__device__ __forceinline__ uint32_t padk(uint32_t k) { return k + (k >> 4); }
constexpr int CARRY_PAD = CARRY_BLOCK + CARRY_BLOCK / 16;

// Coefficient sources of the first carry pass: c_k from memory, or formed from the three
// residues by Garner's method (the large-integer product: no coefficient array at all).
// Each has load(k), which reads unconditionally (coefficient 0 past the end: nc >= 1), and
// value(k, raw, bad), which selects zero past the end; a thread issues all its loads before
// the first value. A coefficient out of range is noted in `bad` and reported once per
// thread (report).
struct CoefU64 {
  const uint64_t* c;
  uint64_t nc;
  using Raw = uint64_t;
  __device__ __forceinline__ Raw load(uint64_t k) const { return c[k < nc ? k : 0]; }
  __device__ __forceinline__ uint64_t value(uint64_t k, Raw v, uint32_t&) const { return k < nc ? v : 0ull; }
  __device__ __forceinline__ void report(uint32_t) const {}
};
struct CoefCrt {  // unsigned coefficients: v3 must be 0, else the range flag is raised
  const uint32_t* res;
  uint64_t N, nc;
  CrtConsts K;
  uint32_t* status;
  struct Raw {
    uint32_t r1, r2, r3;
  };
  __device__ __forceinline__ Raw load(uint64_t k) const {
    const uint64_t kk = k < nc ? k : 0;
    return Raw{res[kk], res[N + kk], res[2 * N + kk]};
  }
  __device__ __forceinline__ uint64_t value(uint64_t k, Raw r, uint32_t& bad) const {
    uint64_t c;
    const uint32_t v3 = garner(r.r1, r.r2, r.r3, K, &c);
    const bool in = k < nc;
    bad |= (in && v3 != 0) ? 1u : 0u;
    return in && v3 == 0 ? c : 0ull;
  }
  __device__ __forceinline__ void report(uint32_t bad) const {
    if (bad) atomicOr(status, FCIRC_STATUS_RANGE);
  }
};

// Pass 1: u_j into `u`, and each workgroup's (G, P) summary. The block's coefficients
// (plus 4 before it) are staged in LDS with coalesced loads; thread t computes u for limbs
// t + 256 i (consecutive lanes, consecutive words), then takes the GP summary of its own
// contiguous run of CARRY_PER_THREAD.
template <class Coef>
__global__ void __launch_bounds__(CARRY_NT) k_carry_scan1(Coef coef, uint64_t nl, uint32_t* __restrict__ u,
                                                          uint32_t* __restrict__ summ) {
  __shared__ uint64_t sc[CARRY_BLOCK + 4];
  __shared__ uint32_t su[CARRY_PAD];
  __shared__ uint32_t sh[CARRY_NT / 64];
  const uint64_t jb = (uint64_t)blockIdx.x * CARRY_BLOCK;
  // sc[k] = c_(jb + k - 4), k < CARRY_BLOCK + 4: the 4 coefficients before the block, then
  // its CARRY_BLOCK;
  // thread t < 4 also stages c_(jb + t - 4) (zero before the first limb)
  const uint64_t kx = jb + threadIdx.x >= 4 ? jb + threadIdx.x - 4 : coef.nc;
  typename Coef::Raw raw[CARRY_PER_THREAD], rx;
#pragma unroll
  for (int i = 0; i < CARRY_PER_THREAD; ++i) raw[i] = coef.load(jb + threadIdx.x + (uint32_t)i * CARRY_NT);
  if (threadIdx.x < 4) rx = coef.load(kx);
  uint32_t bad = 0;
#pragma unroll
  for (int i = 0; i < CARRY_PER_THREAD; ++i) {
    const uint64_t k = jb + threadIdx.x + (uint32_t)i * CARRY_NT;
    sc[threadIdx.x + (uint32_t)i * CARRY_NT + 4] = coef.value(k, raw[i], bad);
  }
  if (threadIdx.x < 4) sc[threadIdx.x] = coef.value(kx, rx, bad);
  coef.report(bad);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < CARRY_PER_THREAD; ++i) {
    const uint32_t k = threadIdx.x + (uint32_t)i * CARRY_NT;  // limb jb + k, coefficient sc[k + 4]
    const uint64_t c0 = sc[k + 4], c1 = sc[k + 3], c2 = sc[k + 2], c3 = sc[k + 1], c4 = sc[k];
    const uint32_t s = (uint32_t)(c0 & 0xFFFFu) + (uint32_t)((c1 >> 16) & 0xFFFFu) + (uint32_t)((c2 >> 32) & 0xFFFFu) +
                       (uint32_t)((c3 >> 48) & 0xFFFFu);
    const uint32_t sp = (uint32_t)(c1 & 0xFFFFu) + (uint32_t)((c2 >> 16) & 0xFFFFu) + (uint32_t)((c3 >> 32) & 0xFFFFu) +
                        (uint32_t)((c4 >> 48) & 0xFFFFu);
    su[padk(k)] = (s & 0xFFFFu) + (sp >> 16);
  }
  __syncthreads();
  GP acc{0u, 1u};
#pragma unroll
  for (int i = 0; i < CARRY_PER_THREAD; ++i) {
    const uint32_t k = threadIdx.x * CARRY_PER_THREAD + i;
    if (jb + k < nl) acc = gp_combine(acc, gp_of(su[padk(k)]));
  }
  for (uint32_t k = threadIdx.x; k < CARRY_BLOCK; k += CARRY_NT)
    if (jb + k < nl) u[jb + k] = su[padk(k)];
  GP tot;
  (void)block_scan_gp(acc, sh, &tot);
  if (threadIdx.x == 0) {
    summ[2 * blockIdx.x] = tot.g;
    summ[2 * blockIdx.x + 1] = tot.p;
  }
}

// Pass 2: carry into each workgroup from all earlier summaries (ordered), then limbs.
__global__ void __launch_bounds__(CARRY_NT) k_carry_scan2(const uint32_t* __restrict__ u, uint64_t nl,
                                                          const uint32_t* __restrict__ summ, uint16_t* __restrict__ out) {
  __shared__ uint32_t su[CARRY_PAD];
  __shared__ uint32_t sh[CARRY_NT / 64];
  const uint64_t jb = (uint64_t)blockIdx.x * CARRY_BLOCK;
  // Summaries of blocks [0, blockIdx.x): thread t composes its contiguous share in order.
  // All loads are issued before the first wait: the block's limbs (unconditional: limb
  // nl - 1 past the end) and the first two summaries of the share (a share has at most two
  // below 513 blocks; the rest, if any, follow in a loop).
  const uint32_t nb = blockIdx.x;
  const uint32_t per = (nb + CARRY_NT - 1) / CARRY_NT;
  const uint32_t b0 = threadIdx.x * per, b1 = min(b0 + per, nb);
  uint32_t lv[CARRY_PER_THREAD];
#pragma unroll
  for (int i = 0; i < CARRY_PER_THREAD; ++i) {
    const uint64_t j = jb + threadIdx.x + (uint32_t)i * CARRY_NT;
    lv[i] = u[j < nl ? j : nl - 1];
  }
  uint32_t sv[4];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const uint32_t b = b0 + q < b1 ? b0 + q : 0;  // summary 0 always exists
    sv[2 * q] = summ[2 * b];
    sv[2 * q + 1] = summ[2 * b + 1];
  }
#pragma unroll
  for (int i = 0; i < CARRY_PER_THREAD; ++i) {
    const uint32_t k = threadIdx.x + (uint32_t)i * CARRY_NT;
    su[padk(k)] = jb + k < nl ? lv[i] : 0u;
  }
  GP part{0u, 1u};
#pragma unroll
  for (int q = 0; q < 2; ++q)
    if (b0 + q < b1) part = gp_combine(part, GP{sv[2 * q], sv[2 * q + 1]});
  for (uint32_t b = b0 + 2; b < b1; ++b) part = gp_combine(part, GP{summ[2 * b], summ[2 * b + 1]});
  GP before;
  (void)block_scan_gp(part, sh, &before);
  const uint32_t cin_blk = before.g;  // carry out of all earlier limbs (initial carry 0)
  __syncthreads();                    // sh is reused, su is complete
  GP acc{0u, 1u};
  uint32_t uv[CARRY_PER_THREAD];
#pragma unroll
  for (int i = 0; i < CARRY_PER_THREAD; ++i) {
    uv[i] = su[padk(threadIdx.x * CARRY_PER_THREAD + i)];
    acc = gp_combine(acc, gp_of(uv[i]));
  }
  GP tot;
  const GP incl = block_scan_gp(acc, sh, &tot);
  // exclusive prefix of this thread = inclusive prefix of the previous thread
  const uint32_t prev = __shfl_up(gp_pack(incl), 1, 64);
  GP excl;
  if ((threadIdx.x & 63) != 0) {
    excl = gp_unpack(prev);
    // the wave scan is already offset by earlier waves (incl includes them)
  } else {
    // first lane of a wave: composition of the earlier waves only
    excl = GP{0u, 1u};
    const uint32_t w = threadIdx.x >> 6;
    for (uint32_t q = 0; q < w; ++q) excl = gp_combine(excl, gp_unpack(sh[q]));
  }
  uint32_t carry = excl.g | (excl.p & cin_blk);
  __syncthreads();  // every thread has read su and sh
#pragma unroll
  for (int i = 0; i < CARRY_PER_THREAD; ++i) {
    const uint32_t v = uv[i] + carry;
    su[padk(threadIdx.x * CARRY_PER_THREAD + i)] = v & 0xFFFFu;
    carry = v >> 16;
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < CARRY_BLOCK; k += CARRY_NT)
    if (jb + k < nl) out[jb + k] = (uint16_t)su[padk(k)];
}

uint32_t pw(uint64_t b, uint64_t e, uint32_t p) {
  uint64_t r = 1;
  b %= p;
  while (e) {
    if (e & 1) r = r * b % p;
    b = b * b % p;
    e >>= 1;
  }
  return (uint32_t)r;
}
ZpTw stw(uint32_t w, uint32_t p) { return ZpTw{w, (uint32_t)(((uint64_t)w << 32) / p)}; }

CrtConsts crt_consts() {
  CrtConsts K;
  K.one2 = stw(1, Q2);
  K.one3 = stw(1, Q3);
  K.inv12 = stw(pw(Q1, Q2 - 2, Q2), Q2);
  K.inv13 = stw(pw(Q1, Q3 - 2, Q3), Q3);
  K.inv23 = stw(pw(Q2, Q3 - 2, Q3), Q3);
  return K;
}

// Three cyclic products (one per prime) of length N = 2^L into res[3N].
template <class V>
fcirc_status three_prime_products(Ctx& c, const V* a, uint64_t na, const V* b, uint64_t nb, int L, uint32_t* res,
                                  uint32_t* ws, hipStream_t s) {
  const uint32_t ps[3] = {Q1, Q2, Q3};
  ZpParams rp[3];
  const ZpTw* tw[3];
  const ZpTw* twi[3];
  const uint32_t* U[3];
  const uint32_t* FT[3];
  const uint32_t* FTI[3];
  bool have_ft = true;
  for (int i = 0; i < 3; ++i) {
    const ZpTables* T = nullptr;
    fcirc_status st = zp_tables(c, ps[i], 1u, L, &T);
    if (st != FCIRC_OK) return st;
    rp[i] = zp_params(ps[i], L);
    tw[i] = T->tw;
    twi[i] = T->twi;
    U[i] = T->dU;
    st = zp_first_tables(c, T, L, &FT[i], &FTI[i]);
    if (st != FCIRC_OK) return st;
    have_ft = have_ft && FT[i] != nullptr;
  }
  const uint64_t N = (uint64_t)1 << L;
  const Schedule S = schedule_for(c, FCIRC_ZP_998244353, L);
  // The residues are read by the CRT kernel next: written through at agent scope (measured
  // 1.5 us faster per call than plain stores for 2 x 2^20 coefficients).
  return hip_status(run_product<Zp>(c, S, 3, rp, tw, twi, U, have_ft ? FT : nullptr, have_ft ? FTI : nullptr, true, LdRowRev<V>{a, (uint32_t)na, (uint32_t)N}, LdVecPad<V>{b, (uint32_t)nb},
                                    StPlain<uint32_t, ST_AGENT>{res, N}, res, ws, s));
}

// The two carry passes over nl limbs, coefficients from `coef`.
template <class Coef>
fcirc_status carry_passes(Ctx& c, Coef coef, uint64_t nl, uint32_t* u, uint32_t* summ, uint16_t* out, hipStream_t s) {
  const uint64_t nblk = (nl + CARRY_BLOCK - 1) / CARRY_BLOCK;
  hipError_t e = launch(c, "fcirc_carry", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, k_carry_scan1<Coef>, dim3((uint32_t)nblk), dim3(CARRY_NT), 0, s, coef, nl, u, summ);
  });
  if (e != hipSuccess) return hip_status(e);
  return hip_status(launch(c, "fcirc_carry", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, k_carry_scan2, dim3((uint32_t)nblk), dim3(CARRY_NT), 0, s, u, nl, summ, out);
  }));
}

}  // namespace

fcirc_status polymul_i64(Ctx& c, const int32_t* a, uint64_t na, const int32_t* b, uint64_t nb, int64_t* out, hipStream_t s) {
  const uint64_t nc = na + nb - 1;
  const int L = ilog2(nc);
  const uint64_t N = (uint64_t)1 << L;
  const Schedule S = schedule_for(c, FCIRC_ZP_998244353, L);
  const uint64_t wse = 3 * N + product_ws_elems(S, 3, false);
  fcirc_status st = ws_reserve(c, wse * sizeof(uint32_t));
  if (st != FCIRC_OK) return st;
  uint32_t* res = (uint32_t*)c.ws;
  st = three_prime_products<int32_t>(c, a, na, b, nb, L, res, res + 3 * N, s);
  if (st != FCIRC_OK) return st;
  const CrtConsts K = crt_consts();
  const uint32_t grid = (uint32_t)((nc + 255) / 256);
  return hip_status(launch(c, "fcirc_crt", s, [&](hipEvent_t e0_, hipEvent_t e1_) { FCIRC_LAUNCH(e0_, e1_, k_crt_i64, dim3(grid), dim3(256), 0, s, res, N, nc, K, out, c.d_status); }));
}

fcirc_status bigint_mul(Ctx& c, const uint16_t* a, uint64_t na, const uint16_t* b, uint64_t nb, uint16_t* out, hipStream_t s) {
  const uint64_t nc = na + nb - 1, nl = na + nb;
  const int L = ilog2(nc);
  const uint64_t N = (uint64_t)1 << L;
  const Schedule S = schedule_for(c, FCIRC_ZP_998244353, L);
  const uint64_t nblk = (nl + CARRY_BLOCK - 1) / CARRY_BLOCK;
  // layout (uint32 units): res[3N] | u[nl] | summaries[2 nblk] | product workspace
  const uint64_t off_u = 3 * N, off_s = off_u + nl, off_w = (off_s + 2 * nblk + 63) & ~63ull;
  const uint64_t wse = off_w + product_ws_elems(S, 3, false);
  fcirc_status st = ws_reserve(c, wse * sizeof(uint32_t));
  if (st != FCIRC_OK) return st;
  uint32_t* base = (uint32_t*)c.ws;
  uint32_t* res = base;
  uint32_t* u = base + off_u;
  uint32_t* summ = base + off_s;
  st = three_prime_products<uint16_t>(c, a, na, b, nb, L, res, base + off_w, s);
  if (st != FCIRC_OK) return st;
  // Garner's CRT runs inside the first carry pass, on the coefficients each workgroup
  // stages: the 8-byte coefficients never reach memory (measured on MI355X for 2 x 2^24
  // bits: a separate CRT kernel and pass took 9.1 + 12.3 us).
  return carry_passes(c, CoefCrt{res, N, nc, crt_consts(), c.d_status}, nl, u, summ, out, s);
}

uint64_t carry_blocks(uint64_t nl) { return (nl + CARRY_BLOCK - 1) / CARRY_BLOCK; }

fcirc_status carry_to_limbs(Ctx& c, const uint64_t* coef, uint64_t nc, uint64_t nl, uint32_t* u, uint32_t* summ,
                            uint16_t* out, hipStream_t s) {
  return carry_passes(c, CoefU64{coef, nc}, nl, u, summ, out, s);
}

}  // namespace fcirc
