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

#include <algorithm>
#include <cmath>
#include <type_traits>

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

LeafSchedule leaf_schedule(int L, uint32_t count) {
  LeafSchedule S;
  // tiles of 2^12 elements, or of 2^10 when 2^12 would give fewer than 64 workgroups (the
  // shared row: one instance)
  const int tl = (L > 12 && ((uint64_t)count << (L - 12)) >= 64) ? 12 : 10;
  const int last = L < tl ? L : tl;
  const int T = L - last;
  const int ntop = T == 0 ? 0 : (T + 9) / 10;
  int d0 = 0;
  for (int i = 0; i < ntop; ++i) {
    const int r = (T - d0) / (ntop - i);
    int c = tl - r;
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

// Calls f(std::integral_constant<int, r>) for a pass of r levels, LO <= r <= HI (a kernel is
// compiled per level count; each call site names the counts its schedule can produce).
template <int LO, int HI, class F>
hipError_t with_levels(int r, F&& f) {
  if constexpr (LO > HI) {
    return hipErrorInvalidValue;
  } else {
    if (r == LO) return f(std::integral_constant<int, LO>{});
    return with_levels<LO + 1, HI>(r, f);
  }
}

// Top passes take at most 10 levels; the last pass of a leaf schedule (logc = 0) up to 12.
template <int HI, class Src, class Dst>
hipError_t split_pass_any(Ctx& c, const PassArgs<C32>& A, const C32Params* rp, Src src, Dst dst, uint32_t grid, uint32_t nt,
                          size_t lds, hipStream_t s) {
  return with_levels<1, HI>(A.logr, [&](auto r) {
    return launch_split_r<C32, decltype(r)::value>(c, A, rp, src, src, dst, dst, grid, nt, lds, s);
  });
}
template <int HI, class Src, class Dst>
hipError_t merge_pass_any(Ctx& c, const PassArgs<C32>& A, const C32Params* rp, Src src, Dst dst, uint32_t grid, uint32_t nt,
                          size_t lds, hipStream_t s) {
  return with_levels<1, HI>(A.logr, [&](auto r) {
    return launch_merge_r<C32, decltype(r)::value>(c, A, rp, src, dst, grid, nt, lds, s);
  });
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
  const LeafSchedule S = leaf_schedule(L, count);
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
    const hipError_t e = i == 0 ? split_pass_any<10>(c, A, rp, src, so, grid, nt, tile * sizeof(float2), s)
                                : split_pass_any<12>(c, A, rp, lo, so, grid, nt, tile * sizeof(float2), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Merge `count` leaf vectors (in place in `leaves`) and write the results through dst.
template <class Dst>
hipError_t merge_leaves(Ctx& c, const C32Tables* T, int L, uint32_t count, float2* leaves, Dst dst, hipStream_t s) {
  const uint64_t n = 1ull << L;
  const C32Params rp[3] = {{1.f}, {1.f}, {1.f}};
  const LeafSchedule S = leaf_schedule(L, count);
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
    const hipError_t e = i == 0 ? merge_pass_any<10>(c, A, rp, lo, dst, grid, nt, tile * sizeof(float2), s)
                                : merge_pass_any<12>(c, A, rp, lo, so, grid, nt, tile * sizeof(float2), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The row's leaves, shared by every instance (optionally conjugated).
struct LeafRow {
  const float2* p;
  template <bool CONJ>
  __device__ __forceinline__ float2 get(uint32_t i) const {
    const float2 v = p[i];
    return CONJ ? make_float2(v.x, -v.y) : v;
  }
};

// Levels [0, T) of `count` vectors (arr 1) or rows (arr 0): HBM tile passes of at most 10
// levels, tiles of 2^12 elements.
template <class Src>
hipError_t split_top(Ctx& c, const C32Tables* T, int L, int top, uint32_t count, int arr, Src src, float2* out,
                     hipStream_t s) {
  const uint64_t n = 1ull << L;
  const C32Params rp[3] = {{1.f}, {1.f}, {1.f}};
  PassArgs<C32> A = layer_args(T, L, count);
  A.arr0 = arr;
  A.final_store = 0;
  const LdPlain<float2> lo{out, n};
  const StPlain<float2> so{out, n};
  const int npass = (top + 9) / 10;
  int d0 = 0;
  for (int i = 0; i < npass; ++i) {
    const int r = (top - d0) / (npass - i);
    A.d0 = d0;
    A.logr = r;
    A.logc = std::min(12 - r, L - d0 - r);
    A.tiles = (uint32_t)(n >> (A.logr + A.logc));
    const size_t tile = (size_t)1 << (A.logr + A.logc);
    const uint32_t grid = A.tiles * count, nt = (uint32_t)(tile >> EPT_LOG);
    const hipError_t e = i == 0 ? split_pass_any<10>(c, A, rp, src, so, grid, nt, tile * sizeof(float2), s)
                                : split_pass_any<10>(c, A, rp, lo, so, grid, nt, tile * sizeof(float2), s);
    if (e != hipSuccess) return e;
    d0 += r;
  }
  return hipSuccess;
}

// Merge levels [0, T) of `count` vectors in ws (deepest first); the last pass writes dst.
template <class Dst>
hipError_t merge_top(Ctx& c, const C32Tables* T, int L, int top, uint32_t count, float2* ws, Dst dst, hipStream_t s) {
  const uint64_t n = 1ull << L;
  const C32Params rp[3] = {{1.f}, {1.f}, {1.f}};
  PassArgs<C32> A = layer_args(T, L, count);
  const LdPlain<float2> lo{ws, n};
  const StPlain<float2> so{ws, n};
  const int npass = (top + 9) / 10;
  int d0s[4], rs[4];
  int d0 = 0;
  for (int i = 0; i < npass; ++i) {
    rs[i] = (top - d0) / (npass - i);
    d0s[i] = d0;
    d0 += rs[i];
  }
  for (int i = npass - 1; i >= 0; --i) {
    A.d0 = d0s[i];
    A.logr = rs[i];
    A.logc = std::min(12 - rs[i], L - d0s[i] - rs[i]);
    A.tiles = (uint32_t)(n >> (A.logr + A.logc));
    A.final_store = i == 0;
    const size_t tile = (size_t)1 << (A.logr + A.logc);
    const uint32_t grid = A.tiles * count, nt = (uint32_t)(tile >> EPT_LOG);
    const hipError_t e = i == 0 ? merge_pass_any<10>(c, A, rp, lo, dst, grid, nt, tile * sizeof(float2), s)
                                : merge_pass_any<10>(c, A, rp, lo, so, grid, nt, tile * sizeof(float2), s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Levels below `top` of every instance in one leaf-domain block launch: split the vector,
// multiply by the row's leaves (conjugated if conj) and 1/n, merge back to level `top`.
template <int B, bool CONJ, class Src, class Dst>
hipError_t lf_block_b(Ctx& c, const PassArgs<C32>& A, float scale, Src src, const float2* ahat, Dst dst, hipStream_t s) {
  using S = BlockShape<B>;
  const uint64_t vwgs = (uint64_t)A.tiles * A.ninst;
  const uint32_t grid = (uint32_t)((vwgs + S::GROUPS - 1) / S::GROUPS);
  const size_t lds = lf_block_lds_bytes<C32, B>();
  auto k = k_lf_block<C32, B, CONJ, Src, LeafRow, Dst>;
  allow_lds(k, lds);
  const C32Params rp{scale};
  return launch(c, "fcirc_lf_block", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, k, dim3(grid), dim3(S::NT), lds, s, A, rp, src, LeafRow{ahat}, dst);
  });
}

template <class Src, class Dst>
hipError_t lf_block(Ctx& c, const C32Tables* T, int L, int top, uint32_t count, bool conj, Src src, const float2* ahat,
                    Dst dst, hipStream_t s) {
  PassArgs<C32> A = layer_args(T, L, count);
  A.d0 = top;
  A.logr = L - top;
  A.logc = 0;
  A.tiles = 1u << top;
  A.final_store = top == 0 ? 1 : 0;
  const float scale = (float)std::ldexp(1.0, -L);
#define FCIRC_LF(b)                                                                           \
  case b:                                                                                     \
    return conj ? lf_block_b<b, true>(c, A, scale, src, ahat, dst, s)                         \
                : lf_block_b<b, false>(c, A, scale, src, ahat, dst, s);
  switch (L - top) {  // the layer takes n >= 16; with top levels, at least 10 remain
    FCIRC_LF(4) FCIRC_LF(5) FCIRC_LF(6) FCIRC_LF(7)
    FCIRC_LF(8) FCIRC_LF(9) FCIRC_LF(10) FCIRC_LF(11) FCIRC_LF(12) FCIRC_LF(13) FCIRC_LF(14)
    default: return hipErrorInvalidValue;
  }
#undef FCIRC_LF
}

// Top levels of the leaf-domain product: at most 13 levels stay in the block (64 KiB of
// LDS for the vector), and the block shrinks to 2^10 while that keeps more workgroups busy.
int lf_top(int L, uint32_t count) {
  int b = std::min(L, 13);
  while (b > 10 && ((uint64_t)count << (L - b)) < 512) --b;
  return L - b;
}

// Top levels of the forward and grad_x products: none (one workgroup per instance runs
// every level in LDS, 1024 threads for 2^14 complex elements) when the instance fits,
// unless there are too few instances to fill the chip. Measured on MI355X for 2^11..2^14
// and 32..512 instances: one pass is faster except at 2^14 with fewer than 64 instances.
int lf_product_top(int L, uint32_t count) {
  if (L <= 13 || (L == 14 && count >= 64)) return 0;
  return lf_top(L, count);
}

// y_b = M(ahat (or its conjugate) * Fx(x_b)) for every instance: top split of the vectors,
// one leaf-domain block launch, top merge.
template <class Src, class Dst>
hipError_t lf_product(Ctx& c, const C32Tables* T, int L, uint32_t count, bool conj, Src src, const float2* ahat,
                      float2* ws, Dst dst, hipStream_t s) {
  const int top = lf_product_top(L, count);
  if (top == 0) return lf_block(c, T, L, 0, count, conj, src, ahat, dst, s);
  const uint64_t n = 1ull << L;
  hipError_t e = split_top(c, T, L, top, count, 1, src, ws, s);
  if (e == hipSuccess)
    e = lf_block(c, T, L, top, count, conj, LdPlain<float2>{ws, n}, ahat, StPlain<float2>{ws, n}, s);
  if (e == hipSuccess) e = merge_top(c, T, L, top, count, ws, dst, s);
  return e;
}

struct LayerWs {
  float2 *ahat, *v1, *v2, *part;
};

// ahat (n) | v1 (count n) | v2 (count n) | partial leaf sums (chunks n)
fcirc_status layer_ws(Ctx& c, uint64_t n, uint32_t count, uint32_t chunks, LayerWs* w) {
  const uint64_t elems = n + 2 * n * (uint64_t)count + n * (uint64_t)chunks;
  const fcirc_status st = ws_reserve(c, elems * sizeof(float2));
  if (st != FCIRC_OK) return st;
  float2* base = (float2*)c.ws;
  w->ahat = base;
  w->v1 = base + n;
  w->v2 = base + n + n * (uint64_t)count;
  w->part = base + n + 2 * n * (uint64_t)count;
  return FCIRC_OK;
}

// grad_a of the layer for n >= 2^10: the batch sum is taken in registers.
//   joint top split of g (row split) and conj x (vector split), levels [0, top);
//   k_acc_block: workgroup (block, chunk) splits both sides of the chunk's instances down
//   to the leaves and sums their leaf products; writes one partial per chunk;
//   k_chunk_sum: sums the partials in chunk order; then one merge.
struct PartialOut {
  float2* p;
  uint64_t n;
  __device__ __forceinline__ void operator()(uint32_t chunk, uint32_t i, float2 v) const { p[chunk * n + i] = v; }
};

// S[i] = sum over chunks of P[chunk][i], in chunk order: 32 leaves x 8 chunk ranges per
// workgroup, ranges combined in order through LDS.
__global__ void __launch_bounds__(256) k_chunk_sum(const float2* __restrict__ P, float2* __restrict__ S, uint32_t n,
                                                    uint32_t chunks) {
  __shared__ float2 part[8][32];
  const uint32_t li = threadIdx.x & 31, r = threadIdx.x >> 5;
  const uint32_t i = blockIdx.x * 32 + li;
  const uint32_t per = (chunks + 7) / 8, c0 = r * per, c1 = min(chunks, c0 + per);
  float sx = 0.f, sy = 0.f;
  if (i < n)
    for (uint32_t ch = c0; ch < c1; ++ch) {
      const float2 v = P[(uint64_t)ch * n + i];
      sx += v.x;
      sy += v.y;
    }
  part[r][li] = make_float2(sx, sy);
  __syncthreads();
  if (r == 0 && i < n) {
    float tx = 0.f, ty = 0.f;
    for (int q = 0; q < 8; ++q) {
      tx += part[q][li].x;
      ty += part[q][li].y;
    }
    S[i] = make_float2(tx, ty);
  }
}

template <class SrcA, class SrcX>
hipError_t split_top_ax(Ctx& c, const C32Tables* T, int L, int top, uint32_t count, SrcA srca, SrcX srcx, float2* outa,
                        float2* outx, hipStream_t s) {
  const uint64_t n = 1ull << L;
  const C32Params rp[3] = {{1.f}, {1.f}, {1.f}};
  PassArgs<C32> A = layer_args(T, L, count);
  A.final_store = 0;
  const LdPlain<float2> la{outa, n}, lx{outx, n};
  const StPlain<float2> sa{outa, n}, sx{outx, n};
  const int npass = (top + 9) / 10;
  int d0 = 0;
  for (int i = 0; i < npass; ++i) {
    const int r = (top - d0) / (npass - i);
    A.d0 = d0;
    A.logr = r;
    A.logc = std::min(12 - r, L - d0 - r);
    A.tiles = (uint32_t)(n >> (A.logr + A.logc));
    const size_t tile = (size_t)1 << (A.logr + A.logc);
    const uint32_t grid = A.tiles * count, nt = (uint32_t)(tile >> EPT_LOG);
    hipError_t e;
    if (i == 0) {
      e = with_levels<1, 10>(r, [&](auto rr) {
        return launch_split_ax_r<C32, decltype(rr)::value>(c, A, rp, srca, srcx, sa, sx, grid, nt, s);
      });
    } else {
      e = with_levels<1, 10>(r, [&](auto rr) {
        return launch_split_ax_r<C32, decltype(rr)::value>(c, A, rp, la, lx, sa, sx, grid, nt, s);
      });
    }
    if (e != hipSuccess) return e;
    d0 += r;
  }
  return hipSuccess;
}

template <int B, class SrcA, class SrcX>
hipError_t acc_block_b(Ctx& c, const PassArgs<C32>& A, float scale, uint32_t chunks, uint32_t per_chunk, SrcA sa, SrcX sx,
                       float2* part, hipStream_t s) {
  using S = BlockShape<B>;
  const size_t lds = block_lds_bytes<C32, B>();
  auto k = k_acc_block<C32, B, SrcA, SrcX, PartialOut>;
  allow_lds(k, lds);
  const C32Params rp{scale};
  const uint32_t grid = A.tiles * chunks;
  return launch(c, "fcirc_acc_block", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, k, dim3(grid), dim3(S::NT), lds, s, A, rp, per_chunk, sa, sx, PartialOut{part, (uint64_t)1 << A.logn});
  });
}

// Top levels of grad_a's accumulating pass: lf_top's, except for packed real pairs at 2^13,
// which take one top level instead of none. Reading pairs straight from the batch, the
// 13-level pass needs more registers than 512 threads allow and spills (81 registers);
// measured on MI355X for 512 pairs, one top level and a 12-level pass take 75 us against
// 82 us. Complex rows spill little there and keep the single pass (61 against 75 us).
int ga_top(int L, uint32_t count, bool packed_real) {
  const int t = lf_top(L, count);
  return (packed_real && t == 0 && L == 13) ? 1 : t;
}

// Chunks of the batch for grad_a: about 256 workgroups over (block, chunk).
uint32_t ga_chunks(int L, uint32_t count, bool packed_real) {
  const uint32_t blocks = 1u << ga_top(L, count, packed_real);
  return std::min<uint32_t>(count, std::max<uint32_t>(1, 256 / blocks));
}

template <class SrcA, class SrcX, class Dst>
hipError_t grad_a_acc(Ctx& c, const C32Tables* T, int L, uint32_t count, SrcA srca, SrcX srcx, const LayerWs& w, Dst dst,
                      hipStream_t s) {
  const uint64_t n = 1ull << L;
  constexpr bool packed_real = std::is_same_v<SrcA, LdPair>;
  const int top = ga_top(L, count, packed_real);
  const uint32_t chunks = ga_chunks(L, count, packed_real), per_chunk = (count + chunks - 1) / chunks;
  PassArgs<C32> A = layer_args(T, L, count);
  A.d0 = top;
  A.logr = L - top;
  A.logc = 0;
  A.tiles = 1u << top;
  A.final_store = 0;
  const float scale = (float)std::ldexp(1.0, -L);
  hipError_t e = hipSuccess;
  auto run = [&](auto sa, auto sx) -> hipError_t {
    switch (L - top) {
      case 10: return acc_block_b<10>(c, A, scale, chunks, per_chunk, sa, sx, w.part, s);
      case 11: return acc_block_b<11>(c, A, scale, chunks, per_chunk, sa, sx, w.part, s);
      case 12: return acc_block_b<12>(c, A, scale, chunks, per_chunk, sa, sx, w.part, s);
      case 13:
        if constexpr (std::is_same_v<decltype(sa), LdPair>) {
          return hipErrorInvalidValue;  // ga_top never leaves 13 levels to packed pairs
        } else {
          return acc_block_b<13>(c, A, scale, chunks, per_chunk, sa, sx, w.part, s);
        }
      default: return hipErrorInvalidValue;
    }
  };
  if (top > 0) {
    e = split_top_ax(c, T, L, top, count, srca, srcx, w.v1, w.v2, s);
    if (e == hipSuccess) e = run(LdPlain<float2>{w.v1, n}, LdPlain<float2>{w.v2, n});
  } else {
    e = run(srca, srcx);
  }
  if (e == hipSuccess) {
    const uint32_t grid = (uint32_t)((n + 31) / 32);
    e = launch(c, "fcirc_chunk_sum", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
      FCIRC_LAUNCH(e0_, e1_, k_chunk_sum, dim3(grid), dim3(256), 0, s, w.part, w.ahat, (uint32_t)n, chunks);
    });
  }
  if (e == hipSuccess) e = merge_leaves(c, T, L, 1, w.ahat, dst, s);
  return e;
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
  st = layer_ws(c, n, count, 0, &w);
  if (st != FCIRC_OK) return st;
  const float scale = (float)std::ldexp(1.0, -L);
  hipError_t e;
  (void)scale;
  e = real ? transform(c, T, L, 1, 0, LdR32{(const float*)a, n}, w.ahat, s)
           : transform(c, T, L, 1, 0, LdPlain<float2>{(const float2*)a, n}, w.ahat, s);
  if (e == hipSuccess)
    e = real ? lf_product(c, T, L, count, false, LdPair{(const float*)x, batch, (uint32_t)n, 1.f}, w.ahat, w.v1,
                          StPair{(float*)y, batch, (uint32_t)n}, s)
             : lf_product(c, T, L, count, false, LdPlain<float2>{(const float2*)x, n}, w.ahat, w.v1,
                          StPlain<float2>{(float2*)y, n}, s);
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
  st = layer_ws(c, n, count, (ga && L >= 10) ? ga_chunks(L, count, real) : 0, &w);
  if (st != FCIRC_OK) return st;
  const float scale = (float)std::ldexp(1.0, -L);
  hipError_t e = hipSuccess;
  if (gx) {
    // gx_b = M(conj(Fa(a)) * Fx(gy_b))
    e = real ? transform(c, T, L, 1, 0, LdR32{(const float*)a, n}, w.ahat, s)
             : transform(c, T, L, 1, 0, LdPlain<float2>{(const float2*)a, n}, w.ahat, s);
    if (e == hipSuccess)
      e = real ? lf_product(c, T, L, count, true, LdPair{(const float*)gy, batch, (uint32_t)n, 1.f}, w.ahat, w.v1,
                            StPair{(float*)gx, batch, (uint32_t)n}, s)
               : lf_product(c, T, L, count, true, LdPlain<float2>{(const float2*)gy, n}, w.ahat, w.v1,
                            StPlain<float2>{(float2*)gx, n}, s);
  }
  if (ga && e == hipSuccess && L >= 10) {
    // ga = M(sum_b Fa(gy_b) * Fx(conj x_b)), batch sum in registers
    e = real ? grad_a_acc(c, T, L, count, LdPair{(const float*)gy, batch, (uint32_t)n, 1.f},
                          LdPair{(const float*)x, batch, (uint32_t)n, -1.f}, w, StR32{(float*)ga, n}, s)
             : grad_a_acc(c, T, L, count, LdPlain<float2>{(const float2*)gy, n}, LdConj{(const float2*)x, n}, w,
                          StPlain<float2>{(float2*)ga, n}, s);
  } else if (ga && e == hipSuccess) {
    // small n: leaves of both sides, then the ordered batch sum
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
