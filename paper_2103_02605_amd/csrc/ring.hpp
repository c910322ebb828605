// Ring arithmetic for the f-circulant product kernels (gfx950).
//
// Algorithm 1 (section 2 of Rosowski, arXiv 2103.02605) needs +, -, x, 1/2 and the
// square roots of f in a ring R (Theorem 1). Three butterflies come out of it, one per
// direction of the recursion, for a pair (u, v) = (low half, high half) of a block whose
// node value has square root g:
//   row split    (A1 + A2 g, A1 - A2 g) on first rows:   (u, v) -> (u + g v, u - g v)
//   vector split (b1 g + b2, b1 g - b2):                 (u, v) -> (g u + v, g u - v)
//   merge        c1 = (M1 + M2)/(2g), c2 = (M1 - M2)/2:  (u, v) -> ((u + v) / g, u - v)
// The merge drops the factor 1/2 at every level; the leaves multiply by 1/n instead,
// which gives the same result (the recursion is linear in the leaf values).
//
// Z/p: values live in 32-bit lanes with lazy reduction (Harvey): split outputs in
// [0, 4p), merge values in [0, 2p), canonical [0, p) only at the final store. All three
// primes are below 2^30, so 4p < 2^32. Multiplication by a twiddle w uses Shoup's method
// with the precomputed companion w' = floor(w 2^32 / p): q = hi32(v w'), r = v w - q p
// lies in [0, 2p) for any 32-bit v. The leaf product of two variables uses a signed
// Montgomery reduction. On gfx950 the 32-bit v_mul_hi_u32 / v_mad_u64_u32 issue at
// full rate, which makes this cheaper than an FP64-FMA formulation.
//
// Complex FP32: float2 lanes, twiddles are FP32 roundings of FP64-computed roots.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcirc {

struct ZpTw {
  uint32_t w, wp;  // w in [0, p) and floor(w * 2^32 / p)
};

struct ZpParams {
  uint32_t p;
  uint32_t pinv;   // p^-1 mod 2^32
  uint32_t npinv;  // -p^-1 mod 2^32, from the host: formed on the device, t * (0 - pinv)
                   // is rewritten by the compiler as -(t * pinv), one instruction more
  ZpTw leaf;       // 2^32 / n mod p: undoes the Montgomery factor and applies 1/n
  ZpTw one;        // {1, floor(2^32 / p)}: reduces any 32-bit value to [0, 2p)
  uint32_t two31;  // 2^31 mod p
  ZpTw r32;        // 2^32 mod p: converts a twiddle to Montgomery form
};

struct Zp {
  using T = uint32_t;
  using Tw = ZpTw;
  using Params = ZpParams;
  uint32_t p, p2, pinv, npinv;
  ZpTw leafs, one;
  uint32_t two31;
  ZpTw r32;

  __device__ __forceinline__ explicit Zp(const ZpParams& q)
      : p(q.p), p2(2u * q.p), pinv(q.pinv), npinv(q.npinv), leafs(q.leaf), one(q.one), two31(q.two31), r32(q.r32) {}

  __device__ __forceinline__ uint32_t shoup(uint32_t v, ZpTw t) const {
    const uint32_t q = __umulhi(v, t.wp);
    return v * t.w - q * p;  // in [0, 2p)
  }
  // The negated product: q p - v w = -shoup(v, t) mod 2^32 (same cost). With it the row
  // split needs one subtraction and one three-operand addition.
  __device__ __forceinline__ uint32_t shoup_neg(uint32_t v, ZpTw t) const {
    const uint32_t q = __umulhi(v, t.wp);
    return q * p - v * t.w;
  }
  __device__ __forceinline__ uint32_t red2(uint32_t u) const { return min(u, u - p2); }  // [0,4p) -> [0,2p)

  __device__ __forceinline__ void split_a(T& u, T& v, Tw g) const {
    const uint32_t uu = red2(u);
    const uint32_t tn = shoup_neg(v, g);  // -g v, as 2^32 - [0, 2p)
    u = uu - tn;                          // uu + g v in [0, 4p)
    v = uu + p2 + tn;                     // uu - g v + 2p in (0, 4p)
  }
  __device__ __forceinline__ void split_x(T& u, T& v, Tw g) const {
    const uint32_t t = shoup(u, g);
    const uint32_t vv = red2(v);
    u = t + vv;
    v = t - vv + p2;
  }
  __device__ __forceinline__ void merge(T& u, T& v, Tw gi) const {
    const uint32_t s = u + v;       // [0, 4p)
    const uint32_t d = u - v + p2;  // (0, 4p)
    u = shoup(s, gi);
    v = red2(d);
  }
  // Butterflies whose twiddle is c * u with u from a small uniform table: two Shoup
  // multiplications (each result in [0, 2p), any 32-bit input), no derived companion.
  static constexpr bool kCheapDerive = false;
  __device__ __forceinline__ void split_a2(T& u, T& v, Tw tu, Tw c) const {
    const uint32_t uu = red2(u);
    const uint32_t tn = shoup_neg(shoup(v, tu), c);
    u = uu - tn;
    v = uu + p2 + tn;
  }
  __device__ __forceinline__ void split_x2(T& u, T& v, Tw tu, Tw c) const {
    const uint32_t t = shoup(shoup(u, tu), c);
    const uint32_t vv = red2(v);
    u = t + vv;
    v = t - vv + p2;
  }
  __device__ __forceinline__ void merge2(T& u, T& v, Tw tu, Tw c) const {
    const uint32_t s = u + v;
    const uint32_t d = u - v + p2;
    u = shoup(shoup(s, tu), c);
    v = red2(d);
  }
  __device__ __forceinline__ Tw derive(Tw c, Tw) const { return c; }  // unused (kCheapDerive false)

  // Deepest-stage twiddles in Montgomery form wM = w 2^32 mod p (in [0, p)). The product
  // mont(v, wM) = v wM 2^-32 mod p = v w needs no per-twiddle companion, so twiddles of the
  // deepest stage are formed once per item (a square, or the product with a uniform factor)
  // at the cost of one multiply. For v < 4p the result lies in [0, 2p), as Shoup's does.
  using DeepW = uint32_t;
  __device__ __forceinline__ uint32_t mont(uint32_t v, uint32_t wM) const {
    const uint64_t t = (uint64_t)v * wM;
    const uint32_t m = (uint32_t)t * npinv;
    return (uint32_t)(((uint64_t)m * p + t) >> 32);        // (t + m p) / 2^32, exact
  }
  __device__ __forceinline__ uint32_t canon1(uint32_t v) const { return min(v, v - p); }  // [0,2p) -> [0,p)
  __device__ __forceinline__ DeepW to_deep(Tw t) const { return canon1(shoup(t.w, r32)); }
  __device__ __forceinline__ DeepW deep_sq(DeepW c) const { return canon1(mont(c, c)); }
  __device__ __forceinline__ DeepW deep_derive(DeepW c, DeepW u) const { return canon1(mont(c, u)); }
  __device__ __forceinline__ void split_aD(T& u, T& v, DeepW w) const {
    const uint32_t uu = red2(u);
    const uint32_t t = mont(v, w);
    u = uu + t;
    v = uu - t + p2;
  }
  __device__ __forceinline__ void split_xD(T& u, T& v, DeepW w) const {
    const uint32_t t = mont(u, w);
    const uint32_t vv = red2(v);
    u = t + vv;
    v = t - vv + p2;
  }
  __device__ __forceinline__ void mergeD(T& u, T& v, DeepW w) const {
    const uint32_t s = u + v;
    const uint32_t d = u - v + p2;
    u = mont(s, w);
    v = red2(d);
  }
  // a x / n for a, x in [0, 4p); result in [0, 2p)
  __device__ __forceinline__ T leaf(T a, T x) const {
    a = red2(a);
    x = red2(x);
    const uint32_t lo = a * x, hi = __umulhi(a, x);  // a x < 4p^2 < p 2^32, so hi < p
    const uint32_t m = lo * pinv;
    const uint32_t r = hi - __umulhi(m, p) + p;  // (a x - m p) / 2^32 + p in (0, 2p)
    return shoup(r, leafs);
  }
  // [0, 4p) -> [0, p)
  __device__ __forceinline__ uint32_t canon(T v) const {
    v = red2(v);
    return min(v, v - p);
  }
  // any signed 32-bit integer -> its residue in [0, p)
  __device__ __forceinline__ uint32_t from_i32(int32_t v) const {
    const uint32_t u = (uint32_t)v ^ 0x80000000u;  // v + 2^31, in [0, 2^32)
    uint32_t r = shoup(u, one);                      // [0, 2p)
    r = min(r, r - p);                               // [0, p)
    r = r + p - two31;                               // [1, 2p)
    return min(r, r - p);
  }
};

struct C32Params {
  float scale;  // 1/n
};

struct C32 {
  using T = float2;
  using Tw = float2;
  using Params = C32Params;
  float scale;

  __device__ __forceinline__ explicit C32(const C32Params& q) : scale(q.scale) {}

  static __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
  }
  __device__ __forceinline__ void split_a(T& u, T& v, Tw g) const {
    const float2 t = cmul(g, v);
    const float2 uu = u;
    u = make_float2(uu.x + t.x, uu.y + t.y);
    v = make_float2(uu.x - t.x, uu.y - t.y);
  }
  __device__ __forceinline__ void split_x(T& u, T& v, Tw g) const {
    const float2 t = cmul(g, u);
    const float2 vv = v;
    u = make_float2(t.x + vv.x, t.y + vv.y);
    v = make_float2(t.x - vv.x, t.y - vv.y);
  }
  __device__ __forceinline__ void merge(T& u, T& v, Tw gi) const {
    const float2 s = make_float2(u.x + v.x, u.y + v.y);
    const float2 d = make_float2(u.x - v.x, u.y - v.y);
    u = cmul(s, gi);
    v = d;
  }
  // A twiddle c * u is formed once (one complex product) and used as any other twiddle.
  static constexpr bool kCheapDerive = true;
  __device__ __forceinline__ Tw derive(Tw c, Tw u) const { return cmul(c, u); }
  // Deepest-stage twiddles: the same values (see Zp).
  using DeepW = float2;
  __device__ __forceinline__ DeepW to_deep(Tw t) const { return t; }
  __device__ __forceinline__ DeepW deep_sq(DeepW c) const { return cmul(c, c); }
  __device__ __forceinline__ DeepW deep_derive(DeepW c, DeepW u) const { return cmul(c, u); }
  __device__ __forceinline__ void split_aD(T& u, T& v, DeepW w) const { split_a(u, v, w); }
  __device__ __forceinline__ void split_xD(T& u, T& v, DeepW w) const { split_x(u, v, w); }
  __device__ __forceinline__ void mergeD(T& u, T& v, DeepW w) const { merge(u, v, w); }
  __device__ __forceinline__ void split_a2(T& u, T& v, Tw tu, Tw c) const { split_a(u, v, cmul(c, tu)); }
  __device__ __forceinline__ void split_x2(T& u, T& v, Tw tu, Tw c) const { split_x(u, v, cmul(c, tu)); }
  __device__ __forceinline__ void merge2(T& u, T& v, Tw tu, Tw c) const { merge(u, v, cmul(c, tu)); }
  __device__ __forceinline__ T leaf(T a, T x) const {
    const float2 t = cmul(a, x);
    return make_float2(t.x * scale, t.y * scale);
  }
  static __device__ __forceinline__ T add(T a, T b) { return make_float2(a.x + b.x, a.y + b.y); }
  __device__ __forceinline__ T canon(T v) const { return v; }
};

// GF(p^2) = Z/p[sqrt 3] with the Mersenne prime p = 2^31 - 1, the ring section 3.1 computes
// in (3 is not a square mod p). An element a + b sqrt 3 is a uint2 (a, b), components
// canonical in [0, p) at every step; products use 2^31 = 1 mod p for the reduction.
struct Gp2Params {
  uint32_t ninv;  // 1/n mod p (= 2^(31 - log2 n))
};

struct Gp2 {
  using T = uint2;
  using Tw = uint2;
  using Params = Gp2Params;
  static constexpr uint32_t P = 0x7fffffffu;
  uint32_t ninv;

  __device__ __forceinline__ explicit Gp2(const Gp2Params& q) : ninv(q.ninv) {}

  // t < 2^64 -> t mod p
  static __device__ __forceinline__ uint32_t red64(uint64_t t) {
    const uint64_t s = (t & P) + (t >> 31);                      // < 2^34
    const uint32_t r = (uint32_t)((s & P) + (s >> 31));          // < p + 8
    return r >= P ? r - P : r;
  }
  static __device__ __forceinline__ uint32_t addm(uint32_t a, uint32_t b) {
    const uint32_t s = a + b;
    return min(s, s - P);
  }
  static __device__ __forceinline__ uint32_t subm(uint32_t a, uint32_t b) {
    const uint32_t d = a - b;
    return min(d, d + P);
  }
  // (a + b sqrt 3)(c + d sqrt 3) = (a c + 3 b d) + (a d + b c) sqrt 3; a c + 3 b d < 2^64
  static __device__ __forceinline__ T mul(T u, T v) {
    const uint64_t ac = (uint64_t)u.x * v.x, bd = (uint64_t)u.y * v.y;
    const uint64_t ad = (uint64_t)u.x * v.y, bc = (uint64_t)u.y * v.x;
    return make_uint2(red64(ac + 3 * bd), red64(ad + bc));
  }
  static __device__ __forceinline__ T add(T u, T v) { return make_uint2(addm(u.x, v.x), addm(u.y, v.y)); }
  static __device__ __forceinline__ T sub(T u, T v) { return make_uint2(subm(u.x, v.x), subm(u.y, v.y)); }

  __device__ __forceinline__ void split_a(T& u, T& v, Tw g) const {
    const T t = mul(g, v);
    const T uu = u;
    u = add(uu, t);
    v = sub(uu, t);
  }
  __device__ __forceinline__ void split_x(T& u, T& v, Tw g) const {
    const T t = mul(g, u);
    const T vv = v;
    u = add(t, vv);
    v = sub(t, vv);
  }
  __device__ __forceinline__ void merge(T& u, T& v, Tw gi) const {
    const T s = add(u, v), d = sub(u, v);
    u = mul(s, gi);
    v = d;
  }
  static constexpr bool kCheapDerive = true;
  __device__ __forceinline__ Tw derive(Tw c, Tw u) const { return mul(c, u); }
  __device__ __forceinline__ void split_a2(T& u, T& v, Tw tu, Tw c) const { split_a(u, v, mul(c, tu)); }
  __device__ __forceinline__ void split_x2(T& u, T& v, Tw tu, Tw c) const { split_x(u, v, mul(c, tu)); }
  __device__ __forceinline__ void merge2(T& u, T& v, Tw tu, Tw c) const { merge(u, v, mul(c, tu)); }
  using DeepW = uint2;
  __device__ __forceinline__ DeepW to_deep(Tw t) const { return t; }
  __device__ __forceinline__ DeepW deep_sq(DeepW c) const { return mul(c, c); }
  __device__ __forceinline__ DeepW deep_derive(DeepW c, DeepW u) const { return mul(c, u); }
  __device__ __forceinline__ void split_aD(T& u, T& v, DeepW w) const { split_a(u, v, w); }
  __device__ __forceinline__ void split_xD(T& u, T& v, DeepW w) const { split_x(u, v, w); }
  __device__ __forceinline__ void mergeD(T& u, T& v, DeepW w) const { merge(u, v, w); }
  // a x / n
  __device__ __forceinline__ T leaf(T a, T x) const {
    const T t = mul(a, x);
    return make_uint2(red64((uint64_t)t.x * ninv), red64((uint64_t)t.y * ninv));
  }
  __device__ __forceinline__ T canon(T v) const { return v; }
};

}  // namespace fcirc
