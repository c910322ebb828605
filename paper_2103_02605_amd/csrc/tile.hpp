// Tile passes of the f-circulant recursion (Algorithm 1 of Rosowski, arXiv 2103.02605,
// unrolled level by level).
//
// Layout. Algorithm 1 splits a block of size m into its low and high halves, and the
// proof of Theorem 1 shows the children are again f-circulant, with first rows
// lo +- g hi. Keeping child 2b in the low half and child 2b+1 in the high half of
// parent b, the whole recursion runs in place in natural order: at depth d the array
// holds 2^d independent blocks of n/2^d elements, and no bit reversal is ever needed.
//
// Twiddles. g_{d,b} is the square root taken at node b of depth d. The tables hold the
// heap order tw[2^d + b] (split) and twi[2^d + b] = 1/g_{d,b} (merge).
//
// Tiles. A pass applies levels [d0, d0 + R) to one depth-d0 block. The block is viewed
// as 2^R rows of rs = n / 2^(d0+R) consecutive elements: every butterfly of those levels
// joins two elements of the same column. A workgroup takes C = 2^logc adjacent columns
// (the "tile"), so each global row segment it reads is C contiguous elements. The R
// levels run as radix-2^k stages: a thread owns 2^k elements of one column spaced to
// cover k consecutive levels, keeps them in registers through those k levels, and
// exchanges through LDS between stages. The bottom pass of a product (d0 + R = log2 n)
// has rs = 1 and C = 1, so a tile is one contiguous block; it also does the leaf
// products and runs the merge levels back up before it writes anything out.
#pragma once
#include <type_traits>

#include "ring.hpp"

namespace fcirc {

template <class Ring>
struct PassArgs {
  typename Ring::Tw const* tw[3];   // split twiddles per ring instance (heap order)
  typename Ring::Tw const* twi[3];  // merge twiddles
  uint32_t logn;                    // log2 of the product size
  uint32_t d0;                      // first level of the pass
  uint32_t logr;                    // levels in the pass (tile rows)
  uint32_t logc;                    // tile columns
  uint32_t tiles;                   // tiles per instance
  uint32_t narr;                    // arrays per instance handled by this launch (split: 1 or 2)
  uint32_t ring_per_inst;           // 1: instance z uses ring parameters [z % 3]
  uint32_t final_store;             // 1: canonicalise values on the way out
};

struct TilePos {
  uint32_t tile, arr, inst;
  uint32_t blk;      // depth-d0 block index
  uint64_t base;     // element index of (row 0, column 0) within the instance
  uint64_t rs;       // row stride in elements
};

template <class Ring>
__device__ __forceinline__ TilePos tile_pos(const PassArgs<Ring>& A) {
  TilePos t;
  uint32_t wg = blockIdx.x;
  t.tile = wg % A.tiles;
  uint32_t rest = wg / A.tiles;
  t.arr = rest % A.narr;
  t.inst = rest / A.narr;
  const uint32_t cols_log = A.logn - A.d0 - A.logr;  // log2 rs
  const uint32_t tpb_log = cols_log - A.logc;        // log2 tiles per block
  t.blk = t.tile >> tpb_log;
  const uint32_t col0 = (t.tile & ((1u << tpb_log) - 1)) << A.logc;
  t.base = ((uint64_t)t.blk << (A.logn - A.d0)) + col0;
  t.rs = (uint64_t)1 << cols_log;
  return t;
}

// Iterate this thread's items of a stage covering tile levels [l0, l0 + K).
// body(col, sb, row0, sh): element i of the item sits at row row0 + (i << sh), column col;
// sb is the item's sub-block index at tile level l0.
template <int K, int NT, class F>
__device__ __forceinline__ void for_items(uint32_t logr, uint32_t logc, uint32_t l0, F&& body) {
  const uint32_t sh = logr - l0 - K;
  const uint32_t items = 1u << (logr + logc - K);
  for (uint32_t item = threadIdx.x; item < items; item += NT) {
    const uint32_t col = item & ((1u << logc) - 1);
    const uint32_t rp = item >> logc;
    const uint32_t o = rp & ((1u << sh) - 1);
    const uint32_t sb = rp >> sh;
    body(col, sb, (sb << (logr - l0)) + o, sh);
  }
}

// Heap index of the twiddle used at tile level l (= l0 + j) by sub-group g of an item.
__device__ __forceinline__ uint32_t tw_index(uint32_t d0, uint32_t blk, uint32_t l0, uint32_t j, uint32_t sb, uint32_t g) {
  const uint32_t l = l0 + j;
  return (1u << (d0 + l)) + (blk << l) + (sb << j) + g;
}

// k split levels on the registers of one item, for the row (a) and/or the vector (x).
template <class Ring, int K, bool DA, bool DX>
__device__ __forceinline__ void split_levels(const Ring& R, typename Ring::T* va, typename Ring::T* vx,
                                             typename Ring::Tw const* tw, uint32_t d0, uint32_t blk,
                                             uint32_t l0, uint32_t sb) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int h = 1 << (K - 1 - j);
    const uint32_t ib = tw_index(d0, blk, l0, j, sb, 0);
#pragma unroll
    for (int g = 0; g < (1 << j); ++g) {
      const typename Ring::Tw t = tw[ib + g];
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const int i = g * 2 * h + q;
        if constexpr (DA) R.split_a(va[i], va[i + h], t);
        if constexpr (DX) R.split_x(vx[i], vx[i + h], t);
      }
    }
  }
}

// k merge levels, deepest first.
template <class Ring, int K>
__device__ __forceinline__ void merge_levels(const Ring& R, typename Ring::T* vy, typename Ring::Tw const* twi,
                                             uint32_t d0, uint32_t blk, uint32_t l0, uint32_t sb) {
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    const int h = 1 << (K - 1 - j);
    const uint32_t ib = tw_index(d0, blk, l0, j, sb, 0);
#pragma unroll
    for (int g = 0; g < (1 << j); ++g) {
      const typename Ring::Tw t = twi[ib + g];
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const int i = g * 2 * h + q;
        R.merge(vy[i], vy[i + h], t);
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Split pass: levels [d0, d0 + logr) of the row (arr 0) or the vector (arr 1), src -> dst.
// ---------------------------------------------------------------------------------------
template <class Ring, int LOGE, int NT, class SrcA, class SrcX, class Dst>
__global__ void __launch_bounds__(NT) k_split(PassArgs<Ring> A, typename Ring::Params rp0, typename Ring::Params rp1,
                                              typename Ring::Params rp2, SrcA srca, SrcX srcx, Dst dsta, Dst dstx) {
  using T = typename Ring::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const TilePos P = tile_pos(A);
  const uint32_t rsel = A.ring_per_inst ? P.inst % 3 : 0;
  const typename Ring::Params rp = rsel == 0 ? rp0 : (rsel == 1 ? rp1 : rp2);
  const Ring R(rp);
  const typename Ring::Tw* tw = A.tw[rsel];
  const uint32_t nst = (A.logr + LOGE - 1) / LOGE;

  auto stage = [&](auto kc, uint32_t s) {
    constexpr int K = decltype(kc)::value;
    const uint32_t l0 = s * LOGE;
    const bool first = s == 0, last = s + 1 == nst;
    for_items<K, NT>(A.logr, A.logc, l0, [&](uint32_t col, uint32_t sb, uint32_t row0, uint32_t sh) {
      T v[1 << K];
#pragma unroll
      for (int i = 0; i < (1 << K); ++i) {
        const uint32_t row = row0 + ((uint32_t)i << sh);
        if (first) {
          const uint64_t g = P.base + row * P.rs + col;
          v[i] = P.arr == 0 ? srca(R, P.inst, g) : srcx(R, P.inst, g);
        } else {
          v[i] = lds[(row << A.logc) + col];
        }
      }
      if (P.arr == 0)
        split_levels<Ring, K, true, false>(R, v, v, tw, A.d0, P.blk, l0, sb);
      else
        split_levels<Ring, K, false, true>(R, v, v, tw, A.d0, P.blk, l0, sb);
#pragma unroll
      for (int i = 0; i < (1 << K); ++i) {
        const uint32_t row = row0 + ((uint32_t)i << sh);
        if (last) {
          const uint64_t g = P.base + row * P.rs + col;
          if (P.arr == 0) dsta(P.inst, g, v[i]); else dstx(P.inst, g, v[i]);
        } else {
          lds[(row << A.logc) + col] = v[i];
        }
      }
    });
  };
  for (uint32_t s = 0; s < nst; ++s) {
    const uint32_t k = min((uint32_t)LOGE, A.logr - s * LOGE);
    if constexpr (LOGE >= 5) { if (k == 5) stage(std::integral_constant<int, 5>{}, s); }
    if constexpr (LOGE >= 4) { if (k == 4) stage(std::integral_constant<int, 4>{}, s); }
    if (k == 3) stage(std::integral_constant<int, 3>{}, s);
    if (k == 2) stage(std::integral_constant<int, 2>{}, s);
    if (k == 1) stage(std::integral_constant<int, 1>{}, s);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Merge pass: levels [d0 + logr - 1 .. d0] of the product, src -> dst (may alias: each
// workgroup reads its whole tile before it writes any of it).
// ---------------------------------------------------------------------------------------
template <class Ring, int LOGE, int NT, class Src, class Dst>
__global__ void __launch_bounds__(NT) k_merge(PassArgs<Ring> A, typename Ring::Params rp0, typename Ring::Params rp1,
                                              typename Ring::Params rp2, Src src, Dst dst) {
  using T = typename Ring::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  const TilePos P = tile_pos(A);
  const uint32_t rsel = A.ring_per_inst ? P.inst % 3 : 0;
  const typename Ring::Params rp = rsel == 0 ? rp0 : (rsel == 1 ? rp1 : rp2);
  const Ring R(rp);
  const typename Ring::Tw* twi = A.twi[rsel];
  const uint32_t nst = (A.logr + LOGE - 1) / LOGE;

  auto stage = [&](auto kc, uint32_t s) {
    constexpr int K = decltype(kc)::value;
    const uint32_t l0 = s * LOGE;
    const bool first = s + 1 == nst, last = s == 0;  // merge runs deepest stage first
    for_items<K, NT>(A.logr, A.logc, l0, [&](uint32_t col, uint32_t sb, uint32_t row0, uint32_t sh) {
      T v[1 << K];
#pragma unroll
      for (int i = 0; i < (1 << K); ++i) {
        const uint32_t row = row0 + ((uint32_t)i << sh);
        if (first)
          v[i] = src(R, P.inst, P.base + row * P.rs + col);
        else
          v[i] = lds[(row << A.logc) + col];
      }
      merge_levels<Ring, K>(R, v, twi, A.d0, P.blk, l0, sb);
#pragma unroll
      for (int i = 0; i < (1 << K); ++i) {
        const uint32_t row = row0 + ((uint32_t)i << sh);
        if (last)
          dst(P.inst, P.base + row * P.rs + col, A.final_store ? R.canon(v[i]) : v[i]);
        else
          lds[(row << A.logc) + col] = v[i];
      }
    });
  };
  for (int s = (int)nst - 1; s >= 0; --s) {
    const uint32_t k = min((uint32_t)LOGE, A.logr - s * LOGE);
    if constexpr (LOGE >= 5) { if (k == 5) stage(std::integral_constant<int, 5>{}, s); }
    if constexpr (LOGE >= 4) { if (k == 4) stage(std::integral_constant<int, 4>{}, s); }
    if (k == 3) stage(std::integral_constant<int, 3>{}, s);
    if (k == 2) stage(std::integral_constant<int, 2>{}, s);
    if (k == 1) stage(std::integral_constant<int, 1>{}, s);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Block pass (bottom of the recursion): one contiguous block of 2^logr elements per
// workgroup (d0 + logr = logn, logc = 0). Split levels on row and vector, leaf products,
// merge levels back up, all in LDS and registers; the deepest stage goes split -> leaf ->
// merge without leaving registers.
// ---------------------------------------------------------------------------------------
template <class Ring, int LOGE, int NT, class SrcA, class SrcX, class Dst>
__global__ void __launch_bounds__(NT) k_block(PassArgs<Ring> A, typename Ring::Params rp0, typename Ring::Params rp1,
                                              typename Ring::Params rp2, SrcA srca, SrcX srcx, Dst dst) {
  using T = typename Ring::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sa = reinterpret_cast<T*>(smem_raw);
  T* sx = sa + ((size_t)1 << A.logr);
  const TilePos P = tile_pos(A);
  const uint32_t rsel = A.ring_per_inst ? P.inst % 3 : 0;
  const typename Ring::Params rp = rsel == 0 ? rp0 : (rsel == 1 ? rp1 : rp2);
  const Ring R(rp);
  const typename Ring::Tw* tw = A.tw[rsel];
  const typename Ring::Tw* twi = A.twi[rsel];
  const uint32_t nst = (A.logr + LOGE - 1) / LOGE;

  if (A.logr == 0) {  // 1 x 1 product
    if (threadIdx.x == 0) {
      const T y = R.leaf(srca(R, P.inst, P.base), srcx(R, P.inst, P.base));
      dst(P.inst, P.base, A.final_store ? R.canon(y) : y);
    }
    return;
  }

  auto split_stage = [&](auto kc, uint32_t s) {
    constexpr int K = decltype(kc)::value;
    const uint32_t l0 = s * LOGE;
    const bool first = s == 0, deepest = s + 1 == nst;
    for_items<K, NT>(A.logr, 0, l0, [&](uint32_t, uint32_t sb, uint32_t row0, uint32_t sh) {
      T va[1 << K], vx[1 << K];
#pragma unroll
      for (int i = 0; i < (1 << K); ++i) {
        const uint32_t row = row0 + ((uint32_t)i << sh);
        if (first) {
          va[i] = srca(R, P.inst, P.base + row);
          vx[i] = srcx(R, P.inst, P.base + row);
        } else {
          va[i] = sa[row];
          vx[i] = sx[row];
        }
      }
      split_levels<Ring, K, true, true>(R, va, vx, tw, A.d0, P.blk, l0, sb);
      if (deepest) {
#pragma unroll
        for (int i = 0; i < (1 << K); ++i) va[i] = R.leaf(va[i], vx[i]);
        merge_levels<Ring, K>(R, va, twi, A.d0, P.blk, l0, sb);
      }
#pragma unroll
      for (int i = 0; i < (1 << K); ++i) {
        const uint32_t row = row0 + ((uint32_t)i << sh);
        if (deepest && first) {
          dst(P.inst, P.base + row, A.final_store ? R.canon(va[i]) : va[i]);
        } else {
          sa[row] = va[i];
          if (!deepest) sx[row] = vx[i];
        }
      }
    });
  };
  auto merge_stage = [&](auto kc, uint32_t s) {
    constexpr int K = decltype(kc)::value;
    const uint32_t l0 = s * LOGE;
    const bool last = s == 0;
    for_items<K, NT>(A.logr, 0, l0, [&](uint32_t, uint32_t sb, uint32_t row0, uint32_t sh) {
      T v[1 << K];
#pragma unroll
      for (int i = 0; i < (1 << K); ++i) v[i] = sa[row0 + ((uint32_t)i << sh)];
      merge_levels<Ring, K>(R, v, twi, A.d0, P.blk, l0, sb);
#pragma unroll
      for (int i = 0; i < (1 << K); ++i) {
        const uint32_t row = row0 + ((uint32_t)i << sh);
        if (last)
          dst(P.inst, P.base + row, A.final_store ? R.canon(v[i]) : v[i]);
        else
          sa[row] = v[i];
      }
    });
  };
  for (uint32_t s = 0; s < nst; ++s) {
    const uint32_t k = min((uint32_t)LOGE, A.logr - s * LOGE);
    if constexpr (LOGE >= 5) { if (k == 5) split_stage(std::integral_constant<int, 5>{}, s); }
    if constexpr (LOGE >= 4) { if (k == 4) split_stage(std::integral_constant<int, 4>{}, s); }
    if (k == 3) split_stage(std::integral_constant<int, 3>{}, s);
    if (k == 2) split_stage(std::integral_constant<int, 2>{}, s);
    if (k == 1) split_stage(std::integral_constant<int, 1>{}, s);
    __syncthreads();
  }
  for (int s = (int)nst - 2; s >= 0; --s) {
    const uint32_t k = min((uint32_t)LOGE, A.logr - s * LOGE);
    if constexpr (LOGE >= 5) { if (k == 5) merge_stage(std::integral_constant<int, 5>{}, s); }
    if constexpr (LOGE >= 4) { if (k == 4) merge_stage(std::integral_constant<int, 4>{}, s); }
    if (k == 3) merge_stage(std::integral_constant<int, 3>{}, s);
    if (k == 2) merge_stage(std::integral_constant<int, 2>{}, s);
    if (k == 1) merge_stage(std::integral_constant<int, 1>{}, s);
    __syncthreads();
  }
}

}  // namespace fcirc
