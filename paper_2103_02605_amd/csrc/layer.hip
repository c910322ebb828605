// The circulant layer y = C(a) x over a batch with one shared defining row (f = 1), and
// its gradients, in the leaf domain of the recursion (Algorithm 1, Rosowski arXiv
// 2103.02605, section 2).
//
// Algorithm 1 computes y = M(F_a(a) * F_x(x)): F_a runs the row splits
// (lo + g hi, lo - g hi) down to the leaves, F_x the vector splits (g lo + hi, g lo - hi),
// the leaves are multiplied, and M runs the merges back up. The three maps are linear,
// so the layer reuses them:
//   forward   y_b  = M(Fa(a) * Fx(x_b)), Fa(a) computed once for the batch;
//   gradient  gx_b = C(a)^H gy_b: the row conj(rev a) has leaves conj(Fa(a)) for f = 1,
//             so gx_b = M(conj(Fa(a)) * Fx(gy_b));
//   gradient  ga = sum_b C(gy_b) conj(x_b) = M(sum_b Fa(gy_b) * Fx(conj x_b)): the batch
//             sum is taken on the leaves, followed by one merge.
// Real data: two rows are packed as the real and imaginary parts of one complex row.
// C(a) is real for real a, so the packed product carries both results; for grad_a the
// vector side is conjugated, which leaves sum(C(gy_0) x_0 + C(gy_1) x_1) in the real part.
#include <hip/hip_runtime.h>

#include <cmath>

#include "host.hpp"

namespace fcirc {

namespace {

// Packed pairs of real rows: instance j holds rows 2j (real part) and 2j + 1 (imaginary).
struct LdPair {
  const float* p;
  uint32_t rows, n;
  float sign;  // -1: conjugate (imaginary part negated)
  template <class R>
  __device__ __forceinline__ float2 operator()(const R&, uint32_t j, uint32_t i) const {
    const uint64_t r0 = 2ull * j;
    const float re = p[r0 * n + i];
    const float im = r0 + 1 < rows ? p[(r0 + 1) * n + i] : 0.f;
    return make_float2(re, sign * im);
  }
};
struct StPair {
  float* p;
  uint32_t rows, n;
  __device__ __forceinline__ void operator()(uint32_t j, uint32_t i, float2 v) const {
    const uint64_t r0 = 2ull * j;
    p[r0 * n + i] = v.x;
    if (r0 + 1 < rows) p[(r0 + 1) * n + i] = v.y;
  }
};
struct LdConj {
  const float2* p;
  uint64_t stride;
  template <class R>
  __device__ __forceinline__ float2 operator()(const R&, uint32_t j, uint32_t i) const {
    const float2 v = p[(uint64_t)j * stride + i];
    return make_float2(v.x, -v.y);
  }
};

// Y[j][i] = leaf(A[i] or conj(A[i]), X[j][i]) for every instance j.
__global__ void k_leaf_mul(const float2* __restrict__ A, float2* __restrict__ X, uint32_t n, uint32_t count, int conj_a,
                           float scale) {
  const uint64_t total = (uint64_t)n * count;
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (uint64_t)gridDim.x * blockDim.x) {
    float2 a = A[k % n];
    if (conj_a) a.y = -a.y;
    const float2 x = X[k];
    X[k] = make_float2((a.x * x.x - a.y * x.y) * scale, (a.x * x.y + a.y * x.x) * scale);
  }
}

// S[i] = sum_j leaf(G[j][i], X[j][i]) (fixed summation order: deterministic).
__global__ void k_leaf_sum(const float2* __restrict__ G, const float2* __restrict__ X, float2* __restrict__ S, uint32_t n,
                           uint32_t count, float scale) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float sx = 0.f, sy = 0.f;
  for (uint32_t j = 0; j < count; ++j) {
    const float2 g = G[(uint64_t)j * n + i], x = X[(uint64_t)j * n + i];
    sx = fmaf(g.x, x.x, fmaf(-g.y, x.y, sx));
    sy = fmaf(g.x, x.y, fmaf(g.y, x.x, sy));
  }
  S[i] = make_float2(sx * scale, sy * scale);
}

// Passes of a whole transform or merge: top passes of at most 10 levels, then one pass of
// up to 12 levels over contiguous blocks (tile = one block, logc = 0).
struct LeafSchedule {
  int n = 0;
  int d0[4], r[4], c[4];
};

LeafSchedule leaf_schedule(int L) {
  LeafSchedule S;
  const int last = L < 12 ? L : 12;
  const int T = L - last;
  const int ntop = T == 0 ? 0 : (T + 9) / 10;
  int d0 = 0;
  for (int i = 0; i < ntop; ++i) {
    const int r = (T - d0) / (ntop - i);
    int c = 12 - r;
    if (c > L - d0 - r) c = L - d0 - r;
    S.d0[S.n] = d0;
    S.r[S.n] = r;
    S.c[S.n] = c;
    ++S.n;
    d0 += r;
  }
  if (last > 0) {
    S.d0[S.n] = d0;
    S.r[S.n] = last;
    S.c[S.n] = 0;
    ++S.n;
  }
  return S;
}

#define FCIRC_R12_SWITCH(R_, CALL)        \
  switch (R_) {                           \
    case 1: return CALL(1);               \
    case 2: return CALL(2);               \
    case 3: return CALL(3);               \
    case 4: return CALL(4);               \
    case 5: return CALL(5);               \
    case 6: return CALL(6);               \
    case 7: return CALL(7);               \
    case 8: return CALL(8);               \
    case 9: return CALL(9);               \
    case 10: return CALL(10);             \
    case 11: return CALL(11);             \
    case 12: return CALL(12);             \
    default: return hipErrorInvalidValue; \
  }

template <class Src, class Dst>
hipError_t split_pass_any(Ctx& c, const PassArgs<C32>& A, const C32Params* rp, Src src, Dst dst, uint32_t grid, uint32_t nt,
                          size_t lds, hipStream_t s) {
#define FCIRC_CALL(r) launch_split_r<C32, r>(c, A, rp, src, src, dst, dst, grid, nt, lds, s)
  FCIRC_R12_SWITCH(A.logr, FCIRC_CALL)
#undef FCIRC_CALL
}
template <class Src, class Dst>
hipError_t merge_pass_any(Ctx& c, const PassArgs<C32>& A, const C32Params* rp, Src src, Dst dst, uint32_t grid, uint32_t nt,
                          size_t lds, hipStream_t s) {
#define FCIRC_CALL(r) launch_merge_r<C32, r>(c, A, rp, src, dst, grid, nt, lds, s)
  FCIRC_R12_SWITCH(A.logr, FCIRC_CALL)
#undef FCIRC_CALL
}

PassArgs<C32> layer_args(const C32Tables* T, int L, uint32_t count) {
  PassArgs<C32> A{};
  for (int r = 0; r < 3; ++r) {
    A.tw[r] = T->tw;
    A.twi[r] = T->twi;
    A.tu[r] = T->dU;
    A.tui[r] = T->dU + 15;
  }
  A.logn = L;
  A.ninst = count;
  A.narr = 1;
  A.xcd = 1;
  return A;
}

// Leaves of `count` rows (arr 0) or vectors (arr 1) read by src, written to out (n each).
template <class Src>
hipError_t transform(Ctx& c, const C32Tables* T, int L, uint32_t count, int arr, Src src, float2* out, hipStream_t s) {
  const uint64_t n = 1ull << L;
  const C32Params rp[3] = {{1.f}, {1.f}, {1.f}};
  const LeafSchedule S = leaf_schedule(L);
  PassArgs<C32> A = layer_args(T, L, count);
  A.arr0 = arr;
  A.final_store = 0;
  const LdPlain<float2> lo{out, n};
  const StPlain<float2> so{out, n};
  for (int i = 0; i < S.n; ++i) {
    A.d0 = S.d0[i];
    A.logr = S.r[i];
    A.logc = S.c[i];
    A.tiles = (uint32_t)(n >> (A.logr + A.logc));
    const size_t tile = (size_t)1 << (A.logr + A.logc);
    const uint32_t grid = A.tiles * count, nt = (uint32_t)(tile >> EPT_LOG);
    const hipError_t e = i == 0 ? split_pass_any(c, A, rp, src, so, grid, nt, tile * sizeof(float2), s)
                                : split_pass_any(c, A, rp, lo, so, grid, nt, tile * sizeof(float2), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Merge `count` leaf vectors (in place in `leaves`) and write the results through dst.
template <class Dst>
hipError_t merge_leaves(Ctx& c, const C32Tables* T, int L, uint32_t count, float2* leaves, Dst dst, hipStream_t s) {
  const uint64_t n = 1ull << L;
  const C32Params rp[3] = {{1.f}, {1.f}, {1.f}};
  const LeafSchedule S = leaf_schedule(L);
  PassArgs<C32> A = layer_args(T, L, count);
  const LdPlain<float2> lo{leaves, n};
  const StPlain<float2> so{leaves, n};
  for (int i = S.n - 1; i >= 0; --i) {
    A.d0 = S.d0[i];
    A.logr = S.r[i];
    A.logc = S.c[i];
    A.tiles = (uint32_t)(n >> (A.logr + A.logc));
    A.final_store = i == 0;
    const size_t tile = (size_t)1 << (A.logr + A.logc);
    const uint32_t grid = A.tiles * count, nt = (uint32_t)(tile >> EPT_LOG);
    const hipError_t e = i == 0 ? merge_pass_any(c, A, rp, lo, dst, grid, nt, tile * sizeof(float2), s)
                                : merge_pass_any(c, A, rp, lo, so, grid, nt, tile * sizeof(float2), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t leaf_mul(Ctx& c, const float2* A, float2* X, uint32_t n, uint32_t count, bool conj_a, float scale, hipStream_t s) {
  const uint64_t total = (uint64_t)n * count;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((total + 255) / 256, 8192);
  return launch(c, "fcirc_leaf_mul", s, [&](hipEvent_t e0_, hipEvent_t e1_) { FCIRC_LAUNCH(e0_, e1_, k_leaf_mul, dim3(grid), dim3(256), 0, s, A, X, n, count, conj_a ? 1 : 0, scale); });
}

struct LayerWs {
  float2 *ahat, *v1, *v2;
};

fcirc_status layer_ws(Ctx& c, uint64_t n, uint32_t count, LayerWs* w) {
  const uint64_t elems = n + 2 * n * (uint64_t)count;
  const fcirc_status st = ws_reserve(c, elems * sizeof(float2));
  if (st != FCIRC_OK) return st;
  float2* base = (float2*)c.ws;
  w->ahat = base;
  w->v1 = base + n;
  w->v2 = base + n + n * (uint64_t)count;
  return FCIRC_OK;
}

fcirc_status check_layer(fcirc_ctx* ctx, const void* a, uint64_t n, uint32_t batch, fcirc_ring ring, int* L) {
  if (!ctx || !a || batch == 0 || (ring != FCIRC_C64 && ring != FCIRC_R32)) return FCIRC_EINVAL;
  if (n == 0 || (n & (n - 1))) return FCIRC_ESIZE;
  *L = ilog2(n);
  if (*L < 4 || *L > 24) return FCIRC_ESIZE;  // passes need at least one 16-element item
  return FCIRC_OK;
}

}  // namespace

}  // namespace fcirc

using namespace fcirc;

extern "C" fcirc_status fcirc_matvec_fwd_shared(fcirc_ctx* ctx, const void* a, const void* x, void* y, uint64_t n,
                                                uint32_t batch, fcirc_ring ring, void* stream) {
  int L = 0;
  fcirc_status st = check_layer(ctx, a, n, batch, ring, &L);
  if (st != FCIRC_OK) return st;
  if (!x || !y) return FCIRC_EINVAL;
  Ctx& c = ctx->c;
  if (hipSetDevice(c.device) != hipSuccess) return FCIRC_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  const C32Tables* T = nullptr;
  st = c32_tables(c, 1.0, 0.0, L, s, &T);
  if (st != FCIRC_OK) return st;
  const bool real = ring == FCIRC_R32;
  const uint32_t count = real ? (batch + 1) / 2 : batch;
  LayerWs w;
  st = layer_ws(c, n, count, &w);
  if (st != FCIRC_OK) return st;
  const float scale = (float)std::ldexp(1.0, -L);
  hipError_t e;
  if (real) {
    e = transform(c, T, L, 1, 0, LdR32{(const float*)a, n}, w.ahat, s);
    if (e == hipSuccess) e = transform(c, T, L, count, 1, LdPair{(const float*)x, batch, (uint32_t)n, 1.f}, w.v1, s);
  } else {
    e = transform(c, T, L, 1, 0, LdPlain<float2>{(const float2*)a, n}, w.ahat, s);
    if (e == hipSuccess) e = transform(c, T, L, count, 1, LdPlain<float2>{(const float2*)x, n}, w.v1, s);
  }
  if (e == hipSuccess) e = leaf_mul(c, w.ahat, w.v1, (uint32_t)n, count, false, scale, s);
  if (e == hipSuccess)
    e = real ? merge_leaves(c, T, L, count, w.v1, StPair{(float*)y, batch, (uint32_t)n}, s)
             : merge_leaves(c, T, L, count, w.v1, StPlain<float2>{(float2*)y, n}, s);
  return hip_status(e);
}

extern "C" fcirc_status fcirc_matvec_backward(fcirc_ctx* ctx, const void* a, const void* x, const void* gy, void* ga,
                                              void* gx, uint64_t n, uint32_t batch, fcirc_ring ring, void* stream) {
  int L = 0;
  fcirc_status st = check_layer(ctx, a, n, batch, ring, &L);
  if (st != FCIRC_OK) return st;
  if (!gy || (ga && !x)) return FCIRC_EINVAL;
  Ctx& c = ctx->c;
  if (hipSetDevice(c.device) != hipSuccess) return FCIRC_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  const C32Tables* T = nullptr;
  st = c32_tables(c, 1.0, 0.0, L, s, &T);
  if (st != FCIRC_OK) return st;
  const bool real = ring == FCIRC_R32;
  const uint32_t count = real ? (batch + 1) / 2 : batch;
  LayerWs w;
  st = layer_ws(c, n, count, &w);
  if (st != FCIRC_OK) return st;
  const float scale = (float)std::ldexp(1.0, -L);
  hipError_t e = hipSuccess;
  if (gx) {
    // gx_b = M(conj(Fa(a)) * Fx(gy_b))
    e = real ? transform(c, T, L, 1, 0, LdR32{(const float*)a, n}, w.ahat, s)
             : transform(c, T, L, 1, 0, LdPlain<float2>{(const float2*)a, n}, w.ahat, s);
    if (e == hipSuccess)
      e = real ? transform(c, T, L, count, 1, LdPair{(const float*)gy, batch, (uint32_t)n, 1.f}, w.v1, s)
               : transform(c, T, L, count, 1, LdPlain<float2>{(const float2*)gy, n}, w.v1, s);
    if (e == hipSuccess) e = leaf_mul(c, w.ahat, w.v1, (uint32_t)n, count, true, scale, s);
    if (e == hipSuccess)
      e = real ? merge_leaves(c, T, L, count, w.v1, StPair{(float*)gx, batch, (uint32_t)n}, s)
               : merge_leaves(c, T, L, count, w.v1, StPlain<float2>{(float2*)gx, n}, s);
  }
  if (ga && e == hipSuccess) {
    // ga = M(sum_b Fa(gy_b) * Fx(conj x_b))
    e = real ? transform(c, T, L, count, 0, LdPair{(const float*)gy, batch, (uint32_t)n, 1.f}, w.v1, s)
             : transform(c, T, L, count, 0, LdPlain<float2>{(const float2*)gy, n}, w.v1, s);
    if (e == hipSuccess)
      e = real ? transform(c, T, L, count, 1, LdPair{(const float*)x, batch, (uint32_t)n, -1.f}, w.v2, s)
               : transform(c, T, L, count, 1, LdConj{(const float2*)x, n}, w.v2, s);
    if (e == hipSuccess) {
      const uint32_t grid = (uint32_t)((n + 255) / 256);
      e = launch(c, "fcirc_leaf_sum", s, [&](hipEvent_t e0_, hipEvent_t e1_) { FCIRC_LAUNCH(e0_, e1_, k_leaf_sum, dim3(grid), dim3(256), 0, s, w.v1, w.v2, w.ahat, (uint32_t)n, count, scale); });
    }
    if (e == hipSuccess)
      e = real ? merge_leaves(c, T, L, 1, w.ahat, StR32{(float*)ga, n}, s)
               : merge_leaves(c, T, L, 1, w.ahat, StPlain<float2>{(float2*)ga, n}, s);
  }
  return hip_status(e);
}
