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
// levels run as radix-2^k stages (k <= 4): every thread owns 16 elements per stage, as
// 16 / 2^k items of 2^k elements of one column spaced to cover k consecutive levels.
// It issues all its twiddle and element loads first, runs the k levels in registers,
// and writes back; stages exchange through LDS. The first stage takes the remainder
// (k = R mod 4, or 4) so every later stage is a full radix-16 stage. The bottom pass of
// a product (d0 + R = log2 n, rs = 1, C = 1) is one contiguous block; it also does the
// leaf products and runs the merge levels back up before anything leaves the workgroup,
// and its deepest stage goes split -> leaf -> merge without leaving registers.
#pragma once
#include <type_traits>

#include "ring.hpp"

namespace fcirc {

constexpr int EPT_LOG = 4;  // log2 elements per thread per stage

// Largest top-pass workgroup: 1024 threads (2^14-element tiles) for 32-bit rings, whose
// top-pass kernels fit the 128 registers that allows; 512 for the complex ring.
template <class Ring>
struct TopThreads {
  static constexpr int value = sizeof(typename Ring::T) == 4 ? 1024 : 512;
};

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
  uint32_t arr0;                    // array of the first (split with narr 1: 0 row, 1 vector)
  uint32_t ninst;                   // instances
  uint32_t ring_per_inst;           // 1: instance z uses ring parameters [z % 3]
  uint32_t final_store;             // 1: canonicalise values on the way out
  uint32_t xcd;                     // 1: XCD-aware tile order
  // Uniform factors of the deepest block stage: for the 2^j consecutive nodes of level j
  // inside one radix-16 item, twiddle g = (twiddle of the first node) * tu[2^j - 1 + g],
  // tu[2^j - 1 + g] = rho_j^brev_j(g) (a root of unity that does not depend on f, the
  // block or the item). tui holds the inverses for the merge. Stored in the ring's
  // deepest-stage form (Montgomery form for Z/p).
  typename Ring::DeepW const* tu[3];   // 15 entries each, in device memory
  typename Ring::DeepW const* tui[3];
  // Last first-twiddle of the deepest radix-16 stage per item (may be null), deepest-stage
  // form: for the node b0 at depth logn - 4, ft[b0] = c_3 = g_{logn-1, 8 b0}; fti the
  // inverses. The other first twiddles follow by squaring: c_j = c_(j+1)^2, since the
  // first child's root is a square root of its parent's.
  typename Ring::DeepW const* ft[3];
  typename Ring::DeepW const* fti[3];
  // Block factors (may be null): the twiddle of node (local level l, index g) of any block
  // at depth d0 is the twiddle of the block's first node of level l times
  // ub[2^l - 1 + g] = rho_l^brev_l(g) (a root of unity that depends on neither f, d0 nor
  // the block; ubi the inverses), l < 13, in deepest-stage form. With them a block pass
  // reads one heap twiddle per level instead of 2^l, and no first-twiddle table.
  typename Ring::DeepW const* ub[3];
  typename Ring::DeepW const* ubi[3];
};

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup i runs on XCD i mod 8),
// and each XCD has its own L2. Remapping gives every XCD a contiguous range of tiles, so
// neighbouring column tiles, which share cache lines, are fetched through one L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t grid) {
  if ((grid & 7u) != 0) return bid;
  return (bid & 7u) * (grid >> 3) + (bid >> 3);
}

struct TilePos {
  uint32_t tile, arr, inst;
  uint32_t blk;   // depth-d0 block index
  uint32_t base;  // element index of (row 0, column 0) within the instance (n <= 2^26)
  uint32_t rs;    // row stride in elements
};

template <class Ring>
__device__ __forceinline__ TilePos tile_pos(const PassArgs<Ring>& A, uint32_t wg) {
  TilePos t;
  t.tile = wg % A.tiles;
  const uint32_t rest = wg / A.tiles;
  t.arr = rest % A.narr + A.arr0;
  t.inst = rest / A.narr;
  const uint32_t cols_log = A.logn - A.d0 - A.logr;  // log2 rs
  const uint32_t tpb_log = cols_log - A.logc;        // log2 tiles per block
  t.blk = t.tile >> tpb_log;
  const uint32_t col0 = (t.tile & ((1u << tpb_log) - 1)) << A.logc;
  t.base = (t.blk << (A.logn - A.d0)) + col0;
  t.rs = 1u << cols_log;
  return t;
}

// Position of a stage item: element i sits at row row0 + (i << sh), column col; sb is the
// item's sub-block index at tile level l0.
struct Item {
  uint32_t col, sb, row0, sh;
};

__device__ __forceinline__ Item item_at(uint32_t item, uint32_t logr, uint32_t logc, uint32_t l0, uint32_t k) {
  Item it;
  it.sh = logr - l0 - k;
  it.col = item & ((1u << logc) - 1);
  const uint32_t rp = item >> logc;
  it.sb = rp >> it.sh;
  it.row0 = (it.sb << (logr - l0)) + (rp & ((1u << it.sh) - 1));
  return it;
}

// Global element index (within the instance) of element i of an item of a top pass:
// (row0 + i 2^sh) rs + col + base, written as first + i step.
__device__ __forceinline__ uint32_t gidx(uint32_t base, uint32_t rs, const Item& it, int i) {
  return (base + it.row0 * rs + it.col) + (uint32_t)i * (rs << it.sh);
}

// Heap index of the twiddle used at tile level l0 + j by sub-group g of an item.
__device__ __forceinline__ uint32_t tw_index(uint32_t d0, uint32_t blk, uint32_t l0, uint32_t j, uint32_t sb) {
  const uint32_t l = l0 + j;
  return (1u << (d0 + l)) + (blk << l) + (sb << j);
}

// The 2^K - 1 twiddles of one item, stored level by level: level j, group g at (2^j - 1 + g).
template <class Ring, int K>
__device__ __forceinline__ void load_tw(typename Ring::Tw* t, typename Ring::Tw const* tw, uint32_t d0, uint32_t blk,
                                        uint32_t l0, uint32_t sb) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t ib = tw_index(d0, blk, l0, j, sb);
#pragma unroll
    for (int g = 0; g < (1 << j); ++g) t[(1 << j) - 1 + g] = tw[ib + g];
  }
}

// The first twiddle of each of the K levels of an item (heap index of group 0).
template <class Ring, int K>
__device__ __forceinline__ void load_tw_first(typename Ring::Tw* t, typename Ring::Tw const* tw, uint32_t d0, uint32_t blk,
                                              uint32_t l0, uint32_t sb) {
#pragma unroll
  for (int j = 0; j < K; ++j) t[j] = tw[tw_index(d0, blk, l0, j, sb)];
}

// The 2^K - 1 twiddles of an item from the LDS copy (levels l0 .. l0 + K - 1; level l of
// the copy, node b at 2^l - 1 + b).
template <class Ring, int K, class W>
__device__ __forceinline__ void lds_tw(W* t, const W* stw, uint32_t l0, uint32_t sb) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint32_t ib = (1u << (l0 + j)) - 1 + (sb << j);
#pragma unroll
    for (int g = 0; g < (1 << j); ++g) t[(1 << j) - 1 + g] = stw[ib + g];
  }
}

// The 2^K - 1 twiddles of a radix-2^K item in deepest-stage form, from the first twiddle
// of each level (c[j]) and the uniform factors (level j, group g: c[j] * tu[2^j - 1 + g]).
template <class Ring, int K>
__device__ __forceinline__ void deep_twiddles(const Ring& R, typename Ring::DeepW* w, const typename Ring::DeepW* c,
                                              const typename Ring::DeepW* tu) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    w[(1 << j) - 1] = c[j];
#pragma unroll
    for (int g = 1; g < (1 << j); ++g) w[(1 << j) - 1 + g] = R.deep_derive(c[j], tu[(1 << j) - 1 + g]);
  }
}

// K split levels with twiddles in the ring's deepest-stage form (Montgomery form for Z/p,
// which needs no per-twiddle companion), on the row (DA) and/or the vector (DX).
template <class Ring, int K, bool DA = true, bool DX = true>
__device__ __forceinline__ void split_levels_d(const Ring& R, typename Ring::T* va, typename Ring::T* vx,
                                               const typename Ring::DeepW* w) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int h = 1 << (K - 1 - j);
#pragma unroll
    for (int g = 0; g < (1 << j); ++g) {
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const int i = g * 2 * h + q;
        if constexpr (DA) R.split_aD(va[i], va[i + h], w[(1 << j) - 1 + g]);
        if constexpr (DX) R.split_xD(vx[i], vx[i + h], w[(1 << j) - 1 + g]);
      }
    }
  }
}

// K merge levels (deepest first) with twiddles in deepest-stage form.
template <class Ring, int K>
__device__ __forceinline__ void merge_levels_d(const Ring& R, typename Ring::T* vy, const typename Ring::DeepW* w) {
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    const int h = 1 << (K - 1 - j);
#pragma unroll
    for (int g = 0; g < (1 << j); ++g) {
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const int i = g * 2 * h + q;
        R.mergeD(vy[i], vy[i + h], w[(1 << j) - 1 + g]);
      }
    }
  }
}

// K split levels from the first twiddle per level and the uniform factors tu, on the row
// (DA) and/or the vector (DX).
template <class Ring, int K, bool DA = true, bool DX = true>
__device__ __forceinline__ void split_levels_first(const Ring& R, typename Ring::T* va, typename Ring::T* vx,
                                                   const typename Ring::DeepW* c, const typename Ring::DeepW* tu) {
  typename Ring::DeepW w[(1 << K) - 1];
  deep_twiddles<Ring, K>(R, w, c, tu);
  split_levels_d<Ring, K, DA, DX>(R, va, vx, w);
}

// K merge levels (deepest first) from the first twiddle per level and the factors tui.
template <class Ring, int K>
__device__ __forceinline__ void merge_levels_first(const Ring& R, typename Ring::T* vy, const typename Ring::DeepW* c,
                                                   const typename Ring::DeepW* tui) {
  typename Ring::DeepW w[(1 << K) - 1];
  deep_twiddles<Ring, K>(R, w, c, tui);
  merge_levels_d<Ring, K>(R, vy, w);
}

// Form of the twiddles a block pass stages in LDS. MONT: the ring's deepest-stage form
// (Montgomery words for Z/p: fewer instructions per butterfly and half the LDS, but more
// registers); otherwise its heap form (Shoup pairs).
template <class Ring, bool MONT>
using BlockTw = std::conditional_t<MONT, typename Ring::DeepW, typename Ring::Tw>;
template <class Ring, bool MONT>
__device__ __forceinline__ BlockTw<Ring, MONT> to_block_tw(const Ring& R, typename Ring::Tw t) {
  if constexpr (std::is_same_v<BlockTw<Ring, MONT>, typename Ring::Tw>)
    return t;
  else
    return R.to_deep(t);
}

// K split levels on the registers of one item, for the row (a) and/or the vector (x).
template <class Ring, int K, bool DA, bool DX>
__device__ __forceinline__ void split_levels(const Ring& R, typename Ring::T* va, typename Ring::T* vx,
                                             const typename Ring::Tw* t) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int h = 1 << (K - 1 - j);
#pragma unroll
    for (int g = 0; g < (1 << j); ++g) {
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const int i = g * 2 * h + q;
        if constexpr (DA) R.split_a(va[i], va[i + h], t[(1 << j) - 1 + g]);
        if constexpr (DX) R.split_x(vx[i], vx[i + h], t[(1 << j) - 1 + g]);
      }
    }
  }
}

// K merge levels, deepest first.
template <class Ring, int K>
__device__ __forceinline__ void merge_levels(const Ring& R, typename Ring::T* vy, const typename Ring::Tw* t) {
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    const int h = 1 << (K - 1 - j);
#pragma unroll
    for (int g = 0; g < (1 << j); ++g) {
#pragma unroll
      for (int q = 0; q < h; ++q) {
        const int i = g * 2 * h + q;
        R.merge(vy[i], vy[i + h], t[(1 << j) - 1 + g]);
      }
    }
  }
}

// K split (merge) levels with twiddles of either form: the heap form (Shoup pair) or the
// deepest-stage form.
template <class Ring, int K, bool DA, bool DX, class W>
__device__ __forceinline__ void split_levels_w(const Ring& R, typename Ring::T* va, typename Ring::T* vx, const W* t) {
  if constexpr (std::is_same_v<W, typename Ring::Tw>)
    split_levels<Ring, K, DA, DX>(R, va, vx, t);
  else
    split_levels_d<Ring, K, DA, DX>(R, va, vx, t);
}
template <class Ring, int K, class W>
__device__ __forceinline__ void merge_levels_w(const Ring& R, typename Ring::T* vy, const W* t) {
  if constexpr (std::is_same_v<W, typename Ring::Tw>)
    merge_levels<Ring, K>(R, vy, t);
  else
    merge_levels_d<Ring, K>(R, vy, t);
}

template <class Ring>
__device__ __forceinline__ Ring make_ring(const PassArgs<Ring>& A, uint32_t inst, const typename Ring::Params& rp0,
                                          const typename Ring::Params& rp1, const typename Ring::Params& rp2,
                                          uint32_t* rsel_out) {
  const uint32_t rsel = A.ring_per_inst ? inst % 3 : 0;
  *rsel_out = rsel;
  return Ring(rsel == 0 ? rp0 : (rsel == 1 ? rp1 : rp2));
}

// ---------------------------------------------------------------------------------------
// One split stage of a top pass (one array). FIRST: read from global; LAST: write global.
// PRE: the stage's elements were loaded ahead (pre); TWL: the twiddles come from the tile's
// LDS copy stw, in the ring's deepest-stage form (local heap order: level l of the tile,
// node b at 2^l - 1 + b); hook runs between the stage's arithmetic and its stores.
// ---------------------------------------------------------------------------------------
template <class Ring, int K>
struct StagePre {
  typename Ring::T v[1 << (EPT_LOG - K)][1 << K];
};

struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};

template <class Ring, int K, bool FIRST, bool LAST, bool IS_X, bool PRE = false, bool TWL = false, class Src, class Dst,
          class Hook = NoHook>
__device__ __forceinline__ void split_stage(const PassArgs<Ring>& A, const TilePos& P, const Ring& R,
                                            typename Ring::Tw const* tw, typename Ring::T* lds, uint32_t l0,
                                            uint32_t nt, uint32_t tid, const Src& src, const Dst& dst,
                                            const StagePre<Ring, K>* pre = nullptr, const Hook& hook = Hook{},
                                            const typename Ring::DeepW* stw = nullptr) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  constexpr int IPT = 1 << (EPT_LOG - K);
  constexpr int E = 1 << K;
  static_assert(!PRE || FIRST, "only a first stage takes preloaded elements");
  T v[IPT][E];
  using TwS = std::conditional_t<TWL, typename Ring::DeepW, Tw>;  // LDS copy or heap tables
  TwS t[IPT][E - 1];
  Item it[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    it[u] = item_at(tid + u * nt, A.logr, A.logc, l0, K);
    if constexpr (TWL)
      lds_tw<Ring, K>(t[u], stw, l0, it[u].sb);
    else
      load_tw<Ring, K>(t[u], tw, A.d0, P.blk, l0, it[u].sb);
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (PRE)
        v[u][i] = pre->v[u][i];
      else if constexpr (FIRST)
        v[u][i] = src(R, P.inst, gidx(P.base, P.rs, it[u], i));
      else
        v[u][i] = lds[(row << A.logc) + it[u].col];
    }
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    if constexpr (TWL)
      split_levels_d<Ring, K, !IS_X, IS_X>(R, v[u], v[u], t[u]);
    else
      split_levels<Ring, K, !IS_X, IS_X>(R, v[u], v[u], t[u]);
  }
  hook();
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (LAST)
        dst(P.inst, gidx(P.base, P.rs, it[u], i), v[u][i]);
      else
        lds[(row << A.logc) + it[u].col] = v[u][i];
    }
}

// The first-stage elements of a top pass's tile (one array), loaded ahead of the stage.
template <class Ring, int K, class Src>
__device__ __forceinline__ void stage_prefetch(const PassArgs<Ring>& A, const TilePos& P, const Ring& R, uint32_t nt,
                                               uint32_t tid, const Src& src, StagePre<Ring, K>& pre) {
#pragma unroll
  for (int u = 0; u < (1 << (EPT_LOG - K)); ++u) {
    const Item it = item_at(tid + u * nt, A.logr, A.logc, 0, K);
#pragma unroll
    for (int i = 0; i < (1 << K); ++i) pre.v[u][i] = src(R, P.inst, gidx(P.base, P.rs, it, i));
  }
}

// Stage plan of a pass of R levels: the first stage takes the remainder.
template <int R>
struct StagePlan {
  static constexpr int NST = (R + EPT_LOG - 1) / EPT_LOG;
  static constexpr int K0 = R - EPT_LOG * (NST - 1);
  static constexpr int k(int s) { return s == 0 ? K0 : EPT_LOG; }
  static constexpr int l0(int s) { return s == 0 ? 0 : K0 + EPT_LOG * (s - 1); }
};

template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

// ---------------------------------------------------------------------------------------
// Split pass: levels [d0, d0 + R) of the row (arr 0) or the vector (arr 1), src -> dst, by
// nt = tile elements / 16 threads (threads 0 .. nt-1 of the workgroup).
// ---------------------------------------------------------------------------------------
template <class Ring, int R, class SrcA, class SrcX, class Dst>
__device__ __forceinline__ void split_pass(const PassArgs<Ring>& A, const TilePos& P, const Ring& Rg, uint32_t rsel,
                                           uint32_t nt, uint32_t tid, typename Ring::T* lds, const SrcA& srca,
                                           const SrcX& srcx, const Dst& dsta, const Dst& dstx) {
  using SP = StagePlan<R>;
  const typename Ring::Tw* tw = A.tw[rsel];
  static_for<SP::NST>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    constexpr bool first = s == 0, last = s + 1 == SP::NST;
    if (P.arr == 0)
      split_stage<Ring, SP::k(s), first, last, false>(A, P, Rg, tw, lds, SP::l0(s), nt, tid, srca, dsta);
    else
      split_stage<Ring, SP::k(s), first, last, true>(A, P, Rg, tw, lds, SP::l0(s), nt, tid, srcx, dstx);
    if constexpr (!last) __syncthreads();
  });
}

template <class Ring, int R, class SrcA, class SrcX, class Dst>
__global__ void __launch_bounds__(TopThreads<Ring>::value) k_split(PassArgs<Ring> A, typename Ring::Params rp0, typename Ring::Params rp1,
                                               typename Ring::Params rp2, SrcA srca, SrcX srcx, Dst dsta, Dst dstx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TilePos P = tile_pos(A, A.xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x);
  uint32_t rsel;
  const Ring Rg = make_ring(A, P.inst, rp0, rp1, rp2, &rsel);
  split_pass<Ring, R>(A, P, Rg, rsel, blockDim.x, threadIdx.x, reinterpret_cast<typename Ring::T*>(smem_raw), srca, srcx,
                      dsta, dstx);
}

// ---------------------------------------------------------------------------------------
// Joint split pass: one workgroup takes the same tile of the row and of the vector, row
// first. It runs every stage of the row's tile, then every stage of the vector's; the
// vector's first-stage elements are loaded as soon as the row's first stage has its data,
// so those loads are in flight while the row's later stages compute and write, and the
// tile's reads of one array overlap the writes of the other (the outputs are streamed out
// with non-temporal stores, not held in L2 until the kernel ends). Every stage takes its
// twiddles from an LDS copy of the tile's 2^R - 1 (the row and the vector split of a node
// share g), converted to the ring's deepest-stage form (Montgomery form for Z/p, one
// instruction less per vector butterfly) and loaded behind the row's elements so that no
// global load waits behind the vector's. LDS holds two tiles and the twiddles.
// ---------------------------------------------------------------------------------------
template <class Ring, int R>
constexpr size_t split_ax_lds_bytes(size_t tile) {
  return 2 * tile * sizeof(typename Ring::T) + (((size_t)1 << R) - 1) * sizeof(typename Ring::DeepW);
}

template <class Ring, int R, class SrcA, class SrcX, class Dst>
__global__ void __launch_bounds__(TopThreads<Ring>::value) k_split_ax(PassArgs<Ring> A, typename Ring::Params rp0, typename Ring::Params rp1,
                                                  typename Ring::Params rp2, SrcA srca, SrcX srcx, Dst dsta, Dst dstx) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  using SP = StagePlan<R>;
  constexpr int K0 = SP::K0;
  const TilePos P = tile_pos(A, A.xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x);
  uint32_t rsel;
  const Ring Rg = make_ring(A, P.inst, rp0, rp1, rp2, &rsel);
  const size_t tile = (size_t)1 << (A.logr + A.logc);
  T* lda = reinterpret_cast<T*>(smem_raw);
  T* ldx = lda + tile;
  typename Ring::DeepW* stw = reinterpret_cast<typename Ring::DeepW*>(ldx + tile);
  const Tw* tw = A.tw[rsel];
  const uint32_t nt = blockDim.x, tid = threadIdx.x;
  StagePre<Ring, K0> pa, px;
  stage_prefetch<Ring, K0>(A, P, Rg, nt, tid, srca, pa);
  __builtin_amdgcn_sched_barrier(0);  // the row's loads first
  // level l of the tile is the contiguous heap range [2^(d0+l) + blk 2^l, + 2^l)
  for (uint32_t e = tid; e < (1u << R) - 1; e += nt) {
    const uint32_t l = 31u - __clz(e + 1);
    stw[e] = Rg.to_deep(tw[(1u << (A.d0 + l)) + (P.blk << l) + (e + 1 - (1u << l))]);
  }
  __syncthreads();
  const auto prefetch_x = [&] {
    __builtin_amdgcn_sched_barrier(0);
    stage_prefetch<Ring, K0>(A, P, Rg, nt, tid, srcx, px);
    __builtin_amdgcn_sched_barrier(0);
  };
  static_for<SP::NST>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    constexpr bool first = s == 0, last = s + 1 == SP::NST;
    if constexpr (first)
      split_stage<Ring, SP::k(s), first, last, false, true, true>(A, P, Rg, tw, lda, SP::l0(s), nt, tid, srca, dsta, &pa,
                                                                  prefetch_x, stw);
    else
      split_stage<Ring, SP::k(s), first, last, false, false, true>(A, P, Rg, tw, lda, SP::l0(s), nt, tid, srca, dsta,
                                                                   nullptr, NoHook{}, stw);
    if constexpr (!last) __syncthreads();
  });
  static_for<SP::NST>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    constexpr bool first = s == 0, last = s + 1 == SP::NST;
    if constexpr (first)
      split_stage<Ring, SP::k(s), first, last, true, true, true>(A, P, Rg, tw, ldx, SP::l0(s), nt, tid, srcx, dstx, &px,
                                                                 NoHook{}, stw);
    else
      split_stage<Ring, SP::k(s), first, last, true, false, true>(A, P, Rg, tw, ldx, SP::l0(s), nt, tid, srcx, dstx,
                                                                  nullptr, NoHook{}, stw);
    if constexpr (!last) __syncthreads();
  });
}

// ---------------------------------------------------------------------------------------
// One merge stage of a top pass. FIRST: read global (the deepest stage runs first).
// tpre: the stage's twiddles, loaded ahead (a stage at tile level 0, whose items all use
// sub-block 0), or null.
// ---------------------------------------------------------------------------------------
template <class Ring, int K, bool FIRST, bool LAST, class Src, class Dst>
__device__ __forceinline__ void merge_stage(const PassArgs<Ring>& A, const TilePos& P, const Ring& R,
                                            typename Ring::Tw const* twi, typename Ring::T* lds, uint32_t l0,
                                            uint32_t nt, uint32_t tid, const Src& src, const Dst& dst,
                                            const typename Ring::Tw* tpre = nullptr) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  constexpr int IPT = 1 << (EPT_LOG - K);
  constexpr int E = 1 << K;
  T v[IPT][E];
  Tw t[IPT][E - 1];
  Item it[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    it[u] = item_at(tid + u * nt, A.logr, A.logc, l0, K);
    if (tpre != nullptr) {
#pragma unroll
      for (int j = 0; j < E - 1; ++j) t[u][j] = tpre[j];
    } else {
      load_tw<Ring, K>(t[u], twi, A.d0, P.blk, l0, it[u].sb);
    }
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (FIRST)
        v[u][i] = src(R, P.inst, gidx(P.base, P.rs, it[u], i));
      else
        v[u][i] = lds[(row << A.logc) + it[u].col];
    }
#pragma unroll
  for (int u = 0; u < IPT; ++u) merge_levels<Ring, K>(R, v[u], t[u]);
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (LAST)
        dst(P.inst, gidx(P.base, P.rs, it[u], i), A.final_store ? R.canon(v[u][i]) : v[u][i]);
      else
        lds[(row << A.logc) + it[u].col] = v[u][i];
    }
}

// ---------------------------------------------------------------------------------------
// Merge pass: levels [d0 + R - 1 .. d0] of the product, src -> dst (may alias: a
// workgroup reads its whole tile before it writes any of it).
// ---------------------------------------------------------------------------------------
template <class Ring, int R, class Src, class Dst>
__device__ __forceinline__ void merge_pass(const PassArgs<Ring>& A, const TilePos& P, const Ring& Rg, uint32_t rsel,
                                           uint32_t nt, uint32_t tid, typename Ring::T* lds, const Src& src, const Dst& dst) {
  using SP = StagePlan<R>;
  const typename Ring::Tw* twi = A.twi[rsel];
  // The last stage (tile levels 0 .. K0-1) uses the same twiddles in every item: loaded at
  // the start from addresses uniform over the workgroup, so that they do not wait behind
  // the stage barriers.
  typename Ring::Tw t0[(1 << SP::K0) - 1];
  load_tw<Ring, SP::K0>(t0, twi, A.d0, P.blk, 0, 0);
  static_for<SP::NST>([&](auto sc) {
    constexpr int s = SP::NST - 1 - decltype(sc)::value;  // deepest stage first
    constexpr bool first = s + 1 == SP::NST, last = s == 0;
    merge_stage<Ring, SP::k(s), first, last>(A, P, Rg, twi, lds, SP::l0(s), nt, tid, src, dst, last ? t0 : nullptr);
    if constexpr (!last) __syncthreads();
  });
}

template <class Ring, int R, class Src, class Dst>
__global__ void __launch_bounds__(TopThreads<Ring>::value) k_merge(PassArgs<Ring> A, typename Ring::Params rp0, typename Ring::Params rp1,
                                               typename Ring::Params rp2, Src src, Dst dst) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TilePos P = tile_pos(A, A.xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x);
  uint32_t rsel;
  const Ring Rg = make_ring(A, P.inst, rp0, rp1, rp2, &rsel);
  merge_pass<Ring, R>(A, P, Rg, rsel, blockDim.x, threadIdx.x, reinterpret_cast<typename Ring::T*>(smem_raw), src, dst);
}

// Synchronisation between two stages of a block pass. In a radix-16 stage whose items (one
// per thread) have their elements 2^sh <= 64 rows apart, the 64 items of a wave cover the
// 1024 consecutive rows [1024 w, 1024 w + 1024) of the block, and that wave's items cover
// the same rows in every deeper stage: an exchange between such stages stays inside the
// wave, and only the wave's own LDS operations have to complete. A block of at most 2^10
// elements (at most 64 threads) lies in one wave altogether.
template <int LOGR, int EL = EPT_LOG>
constexpr bool block_in_one_wave() {
  return LOGR - EL <= 6;
}
template <int LOGR, int EL = EPT_LOG>
constexpr bool wave_region(int l0) {  // radix-2^EL stage at level l0
  return block_in_one_wave<LOGR, EL>() || LOGR - l0 - EL <= 6;
}
__device__ __forceinline__ void stage_sync(bool wave_local) {
  if (wave_local) {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// Block pass (bottom of the recursion): a contiguous block of 2^LOGR elements per thread
// group (d0 + LOGR = logn, logc = 0). Blocks of fewer than 1024 elements share a
// workgroup: 64 threads hold 64 / (2^LOGR / 16) groups, each its own block.
//
// Twiddle latency. A thread group holds the whole block, so there is one workgroup per
// CU and little else to hide a global load behind. The twiddles of every level above the
// deepest radix-16 stage (2^(LOGR-4) - 1 nodes per direction, contiguous per level in the
// heap) are therefore copied into LDS at the start, and the first twiddles of the deepest
// stage are loaded into registers at the start too; all of these loads overlap the
// element loads of the first stage.
// ---------------------------------------------------------------------------------------
// EL: log2 elements per thread (radix of the register stages).
template <int LOGR, int NT_ = 0, int EL = EPT_LOG>
struct BlockShape {
  static constexpr int ACTIVE_LOG = LOGR > EL ? LOGR - EL : 0;  // threads per block
  static constexpr int NT = NT_ ? NT_ : ((1 << ACTIVE_LOG) < 64 ? 64 : (1 << ACTIVE_LOG));
  static constexpr int GROUPS = NT >> ACTIVE_LOG;              // blocks per workgroup
  static constexpr int NST = LOGR == 0 ? 0 : (LOGR + EL - 1) / EL;
  static constexpr int K0 = LOGR - EL * (NST > 0 ? NST - 1 : 0);  // levels of the first stage
  static constexpr int EPT = LOGR < EL ? (1 << LOGR) : (1 << EL);
  static constexpr int NTW = LOGR > EL ? (1 << (LOGR - EL)) - 1 : 0;  // LDS twiddles per direction
};

// LDS of a block pass: [GROUPS][row, vector][2^LOGR] elements, then [GROUPS][split, merge][NTW]
// twiddles (local heap order: level l, node b at 2^l - 1 + b).
template <class Ring, int LOGR, int NT = 0, bool MONT = true, int EL = EPT_LOG>
constexpr size_t block_lds_bytes() {
  using S = BlockShape<LOGR, NT, EL>;
  return (size_t)S::GROUPS * (2 * (sizeof(typename Ring::T) << LOGR) + 2 * (size_t)S::NTW * sizeof(BlockTw<Ring, MONT>));
}

// First twiddles of the deepest radix-16 stage (one item per thread), split and merge,
// in deepest-stage form.
template <class Ring, int EL = EPT_LOG>
struct DeepTw {
  typename Ring::DeepW t[EL], ti[EL];
};

// A copy of D whose 32-bit twiddles are pinned as 32-bit registers where the deepest stage
// uses them. D is formed in one of two branches (the packed first-twiddle table or the heap
// tables); without the pin the compiler merges the two as zero-extended 64-bit values, and
// every Montgomery product with one of them becomes a 64 x 32-bit multiply (two multiplies
// and a move instead of one multiply).
template <class Ring, int EL>
__device__ __forceinline__ DeepTw<Ring, EL> pinned(const DeepTw<Ring, EL>& D) {
  DeepTw<Ring, EL> P = D;
  if constexpr (std::is_same_v<typename Ring::DeepW, uint32_t>) {
#pragma unroll
    for (int j = 0; j < EL; ++j) asm volatile("" : "+v"(P.t[j]), "+v"(P.ti[j]));
  }
  return P;
}

// From the heap tables (any block at depth d0, levels l0 .. l0 + 3, item sub-block sb).
template <class Ring, int EL>
__device__ __forceinline__ void load_deep_heap(DeepTw<Ring, EL>& D, const Ring& R, typename Ring::Tw const* tw,
                                               typename Ring::Tw const* twi, uint32_t d0, uint32_t blk, uint32_t l0,
                                               uint32_t sb) {
  typename Ring::Tw c[EL], ci[EL];
  load_tw_first<Ring, EL>(c, tw, d0, blk, l0, sb);
  load_tw_first<Ring, EL>(ci, twi, d0, blk, l0, sb);
#pragma unroll
  for (int j = 0; j < EL; ++j) {
    D.t[j] = R.to_deep(c[j]);
    D.ti[j] = R.to_deep(ci[j]);
  }
}

// The packed first-twiddle table ft serves radix-16 deepest stages only.
template <class Ring, int LOGR, int EL = EPT_LOG>
__device__ __forceinline__ void load_deep_tw(DeepTw<Ring, EL>& D, const Ring& R, const PassArgs<Ring>& A, const TilePos& P,
                                             uint32_t rsel, typename Ring::Tw const* tw, typename Ring::Tw const* twi,
                                             uint32_t ltid) {
  constexpr uint32_t l0 = LOGR - EL;
  const Item it = item_at(ltid, LOGR, 0, l0, EL);
  if constexpr (LOGR <= 13 && std::is_same_v<typename Ring::DeepW, uint32_t>) {
    if (A.ub[rsel] != nullptr) {  // c_(EL-1): node (LOGR - 1, sb 2^(EL-1)) from the block factors
      constexpr uint32_t l = LOGR - 1;
      const uint32_t g0 = (1u << (A.d0 + l)) + (P.blk << l);
      const uint32_t ge = (1u << l) - 1 + (it.sb << (EL - 1));
      D.t[EL - 1] = R.deep_derive(R.to_deep(tw[g0]), A.ub[rsel][ge]);
      D.ti[EL - 1] = R.deep_derive(R.to_deep(twi[g0]), A.ubi[rsel][ge]);
#pragma unroll
      for (int j = EL - 2; j >= 0; --j) {
        D.t[j] = R.deep_sq(D.t[j + 1]);
        D.ti[j] = R.deep_sq(D.ti[j + 1]);
      }
      return;
    }
  }
  if constexpr (EL == EPT_LOG) {
    if (A.ft[rsel] != nullptr && A.d0 + (uint32_t)LOGR == A.logn) {
      const uint32_t b0 = (P.blk << l0) + it.sb;  // node at depth logn - 4
      D.t[EL - 1] = A.ft[rsel][b0];
      D.ti[EL - 1] = A.fti[rsel][b0];
#pragma unroll
      for (int j = EL - 2; j >= 0; --j) {
        D.t[j] = R.deep_sq(D.t[j + 1]);
        D.ti[j] = R.deep_sq(D.ti[j + 1]);
      }
      return;
    }
  }
  load_deep_heap<Ring, EL>(D, R, tw, twi, A.d0, P.blk, l0, it.sb);
}

// One split stage of the block pass on row and vector. FIRST: elements come from global
// memory (twiddles too); otherwise from LDS. DEEPEST: the stage also forms the leaf
// products and runs its merge levels, leaving y in sa (or writing dst if also FIRST).
template <class Ring, int LOGR, int K, bool FIRST, bool DEEPEST, int EL = EPT_LOG, class W, class SrcA, class SrcX,
          class Dst>
__device__ __forceinline__ void block_split_stage(const PassArgs<Ring>& A, const TilePos& P, const Ring& R, uint32_t rsel,
                                                  typename Ring::Tw const* tw, typename Ring::Tw const* twi,
                                                  const W* stw, const DeepTw<Ring, EL>& D,
                                                  typename Ring::T* sa, typename Ring::T* sx, uint32_t l0, uint32_t ltid,
                                                  const SrcA& srca, const SrcX& srcx, const Dst& dst) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  using S = BlockShape<LOGR, 0, EL>;
  constexpr int E = 1 << K;
  constexpr int IPT = S::EPT / E;
  constexpr uint32_t ACTIVE = 1u << S::ACTIVE_LOG;
  // the deepest stage of a multi-stage pass takes its first twiddles from D (radix 16)
  constexpr bool FROM_D = DEEPEST && !FIRST;
  constexpr bool FIRSTS = DEEPEST && K == EL;
  static_assert(!FROM_D || K == EL, "deepest stage of a multi-stage block pass is a full radix-2^EL stage");
  T va[IPT][E], vx[IPT][E];
  // a first stage loads its twiddles from the heap tables (Shoup form), later stages from
  // the LDS copy (deepest-stage form)
  using TwS = std::conditional_t<FIRST, Tw, W>;
  TwS t[(FROM_D || FIRSTS) ? 1 : IPT][E - 1];
  Tw ti[(DEEPEST && !FROM_D && !FIRSTS) ? IPT : 1][E - 1];
  DeepTw<Ring, EL> Dl[FIRSTS && !FROM_D ? IPT : 1];  // single-stage radix-16 block: from the heap
  Item it[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    it[u] = item_at(ltid + u * ACTIVE, LOGR, 0, l0, K);
    if constexpr (FIRST) {
      if constexpr (FIRSTS) {
        load_deep_heap<Ring, EL>(Dl[u], R, tw, twi, A.d0, P.blk, l0, it[u].sb);
      } else {
        load_tw<Ring, K>(t[u], tw, A.d0, P.blk, l0, it[u].sb);
        if constexpr (DEEPEST) load_tw<Ring, K>(ti[u], twi, A.d0, P.blk, l0, it[u].sb);
      }
    } else if constexpr (!DEEPEST) {
      lds_tw<Ring, K>(t[u], stw, l0, it[u].sb);
    }
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (FIRST) {
        va[u][i] = srca(R, P.inst, P.base + row);
        vx[u][i] = srcx(R, P.inst, P.base + row);
      } else {
        va[u][i] = sa[row];
        vx[u][i] = sx[row];
      }
    }
  [[maybe_unused]] const DeepTw<Ring, EL> Dp = FROM_D ? pinned<Ring, EL>(D) : D;
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    if constexpr (FROM_D)
      split_levels_first<Ring, K>(R, va[u], vx[u], Dp.t, A.tu[rsel]);
    else if constexpr (FIRSTS)
      split_levels_first<Ring, K>(R, va[u], vx[u], Dl[u].t, A.tu[rsel]);
    else
      split_levels_w<Ring, K, true, true>(R, va[u], vx[u], t[u]);
  }
  if constexpr (DEEPEST) {
#pragma unroll
    for (int u = 0; u < IPT; ++u)
#pragma unroll
      for (int i = 0; i < E; ++i) va[u][i] = R.leaf(va[u][i], vx[u][i]);
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      if constexpr (FROM_D)
        merge_levels_first<Ring, K>(R, va[u], Dp.ti, A.tui[rsel]);
      else if constexpr (FIRSTS)
        merge_levels_first<Ring, K>(R, va[u], Dl[u].ti, A.tui[rsel]);
      else
        merge_levels<Ring, K>(R, va[u], ti[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (DEEPEST && FIRST) {
        dst(P.inst, P.base + row, A.final_store ? R.canon(va[u][i]) : va[u][i]);
      } else {
        sa[row] = va[u][i];
        if constexpr (!DEEPEST) sx[row] = vx[u][i];
      }
    }
}

// One radix-2^K merge stage of the block pass (twiddles from the LDS copy). LAST: write dst.
template <class Ring, int LOGR, int K, bool LAST, int EL = EPT_LOG, class W, class Dst>
__device__ __forceinline__ void block_merge_stage(const PassArgs<Ring>& A, const TilePos& P, const Ring& R,
                                                  const W* stwi, typename Ring::T* sa, uint32_t l0,
                                                  uint32_t ltid, const Dst& dst) {
  using T = typename Ring::T;
  using S = BlockShape<LOGR, 0, EL>;
  constexpr int E = 1 << K;
  constexpr int IPT = S::EPT / E;
  constexpr uint32_t ACTIVE = 1u << S::ACTIVE_LOG;
  W t[IPT][E - 1];
  T v[IPT][E];
  Item it[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    it[u] = item_at(ltid + u * ACTIVE, LOGR, 0, l0, K);
    lds_tw<Ring, K>(t[u], stwi, l0, it[u].sb);
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) v[u][i] = sa[it[u].row0 + ((uint32_t)i << it[u].sh)];
#pragma unroll
  for (int u = 0; u < IPT; ++u) merge_levels_w<Ring, K>(R, v[u], t[u]);
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (LAST)
        dst(P.inst, P.base + row, A.final_store ? R.canon(v[u][i]) : v[u][i]);
      else
        sa[row] = v[u][i];
    }
}

// The block pass for workgroup-local virtual workgroups vwg0 .. vwg0 + GROUPS - 1 (NT threads;
// each group of 2^(LOGR-4) threads owns one block). smem_raw holds block_lds_bytes<Ring,
// LOGR, NT>() bytes. tid is the thread's index in the workgroup.
template <class Ring, int LOGR, int NT, bool MONT = true, int EL = EPT_LOG, class SrcA, class SrcX, class Dst>
__device__ __forceinline__ void block_pass(const PassArgs<Ring>& A, uint32_t vwg0, uint32_t tid, unsigned char* smem_raw,
                                           const typename Ring::Params& rp0, const typename Ring::Params& rp1,
                                           const typename Ring::Params& rp2, const SrcA& srca, const SrcX& srcx,
                                           const Dst& dst) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  using S = BlockShape<LOGR, NT, EL>;
  const uint32_t group = tid >> S::ACTIVE_LOG;
  const uint32_t ltid = tid & ((1u << S::ACTIVE_LOG) - 1);
  const uint32_t vwg = vwg0 + group;
  const bool active = group < S::GROUPS && vwg < A.tiles * A.ninst;
  T* sa = reinterpret_cast<T*>(smem_raw) + ((size_t)group << (LOGR + 1));
  T* sx = sa + ((size_t)1 << LOGR);
  using DW = BlockTw<Ring, MONT>;
  DW* stw = reinterpret_cast<DW*>(smem_raw + (size_t)S::GROUPS * 2 * (sizeof(T) << LOGR)) + (size_t)group * 2 * S::NTW;
  DW* stwi = stw + S::NTW;
  const TilePos P = tile_pos(A, active ? vwg : 0);
  uint32_t rsel;
  const Ring R = make_ring(A, P.inst, rp0, rp1, rp2, &rsel);
  const Tw* tw = A.tw[rsel];
  const Tw* twi = A.twi[rsel];

  if constexpr (LOGR == 0) {
    if (active) {
      const T y = R.leaf(srca(R, P.inst, P.base), srcx(R, P.inst, P.base));
      dst(P.inst, P.base, A.final_store ? R.canon(y) : y);
    }
  } else {
    constexpr int NST = S::NST, K0 = S::K0;
    DeepTw<Ring, EL> D;
    if constexpr (NST > 1) {
      if (active) {
        // LDS copy of the twiddles above the deepest stage, in the ring's deepest-stage form
        // (Montgomery form for Z/p: the vector split and the merge then take one instruction
        // less per butterfly, and the copy is half the size): level l of the block is the
        // contiguous heap range [2^(d0+l) + blk 2^l, + 2^l)
        bool staged = false;
        if constexpr (MONT && LOGR <= 13 && std::is_same_v<typename Ring::DeepW, uint32_t>) {
          if (A.ub[rsel] != nullptr) {
            // from the block factors: one heap twiddle per level (the level's first node)
            for (uint32_t e = ltid; e < (uint32_t)S::NTW; e += 1u << S::ACTIVE_LOG) {
              const uint32_t l = 31u - __clz(e + 1);
              const uint32_t g0 = (1u << (A.d0 + l)) + (P.blk << l);
              stw[e] = R.deep_derive(R.to_deep(tw[g0]), A.ub[rsel][e]);
              stwi[e] = R.deep_derive(R.to_deep(twi[g0]), A.ubi[rsel][e]);
            }
            staged = true;
          }
        }
        if (!staged) {
          for (uint32_t e = ltid; e < (uint32_t)S::NTW; e += 1u << S::ACTIVE_LOG) {
            const uint32_t l = 31u - __clz(e + 1);
            const uint32_t gi = (1u << (A.d0 + l)) + (P.blk << l) + (e + 1 - (1u << l));
            stw[e] = to_block_tw<Ring, MONT>(R, tw[gi]);
            stwi[e] = to_block_tw<Ring, MONT>(R, twi[gi]);
          }
        }
        load_deep_tw<Ring, LOGR, EL>(D, R, A, P, rsel, tw, twi, ltid);
      }
    }
    // split stages (first takes K0 levels), the deepest also runs leaf + its merge levels
    if (active) block_split_stage<Ring, LOGR, K0, true, NST == 1, EL>(A, P, R, rsel, tw, twi, stw, D, sa, sx, 0, ltid, srca, srcx, dst);
    if constexpr (NST > 1) {
      stage_sync(block_in_one_wave<LOGR, EL>());  // also publishes the LDS twiddles
#pragma unroll
      for (int s = 1; s < NST; ++s) {
        const uint32_t l0 = K0 + EL * (s - 1);
        if (active) {
          if (s + 1 == NST)
            block_split_stage<Ring, LOGR, EL, false, true, EL>(A, P, R, rsel, tw, twi, stw, D, sa, sx, l0, ltid, srca, srcx, dst);
          else
            block_split_stage<Ring, LOGR, EL, false, false, EL>(A, P, R, rsel, tw, twi, stw, D, sa, sx, l0, ltid, srca, srcx, dst);
        }
        // next: split stage s + 1, or (after the deepest) merge stage NST - 2 in its layout
        const int nxt = s + 1 < NST ? s : NST - 2;
        stage_sync(nxt >= 1 && wave_region<LOGR, EL>(K0 + EL * (nxt - 1)) ? true : block_in_one_wave<LOGR, EL>());
      }
      // merge stages above the deepest one, then the first stage's K0 levels to dst
#pragma unroll
      for (int s = NST - 2; s >= 1; --s) {
        const uint32_t l0 = K0 + EL * (s - 1);
        if (active) block_merge_stage<Ring, LOGR, EL, false, EL>(A, P, R, stwi, sa, l0, ltid, dst);
        stage_sync(s - 1 >= 1 && wave_region<LOGR, EL>(K0 + EL * (s - 2)) ? true : block_in_one_wave<LOGR, EL>());
      }
      if (active) block_merge_stage<Ring, LOGR, K0, true, EL>(A, P, R, stwi, sa, 0, ltid, dst);
    }
  }
}

// ---------------------------------------------------------------------------------------
// Small product in one workgroup: the whole tree of an instance of 2^LOGR elements
// (LOGR <= 12, no top pass) by 2^(LOGR - K) threads, radix-2^K register stages (the first
// takes the remainder), every twiddle of the tree staged in LDS, a barrier between
// stages. A lone small product then runs on 2^(LOGR - K - 6) waves instead of the block
// pass's single wave, whose 16 elements per thread make it one long dependent stream.
// One workgroup per instance.
// ---------------------------------------------------------------------------------------
template <int LOGR, int K>
struct SmallShape {
  static constexpr int NST = (LOGR + K - 1) / K;
  static constexpr int K0 = LOGR - K * (NST - 1);  // levels of the first stage
  static constexpr int NT = 1 << (LOGR - K);       // threads; 2^K elements each per stage
  static constexpr int NTW = (1 << LOGR) - 1;      // twiddles per direction
};

template <class Ring, int LOGR, int K>
constexpr size_t small_lds_bytes() {
  return 2 * (sizeof(typename Ring::T) << LOGR) + 2 * (size_t)SmallShape<LOGR, K>::NTW * sizeof(typename Ring::Tw);
}

// One split stage of KS levels (the deepest also forms the leaves and merges back).
template <class Ring, int LOGR, int K, int KS, bool FIRST, bool DEEPEST, class SrcA, class SrcX, class Dst>
__device__ __forceinline__ void small_split_stage(const PassArgs<Ring>& A, const TilePos& P, const Ring& R,
                                                  const typename Ring::Tw* stw, const typename Ring::Tw* stwi,
                                                  typename Ring::T* sa, typename Ring::T* sx, uint32_t l0, uint32_t tid,
                                                  const SrcA& srca, const SrcX& srcx, const Dst& dst) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  constexpr int E = 1 << KS;
  constexpr int IPT = (1 << K) / E;
  constexpr uint32_t NT = SmallShape<LOGR, K>::NT;
  T va[IPT][E], vx[IPT][E];
  Tw t[IPT][E - 1];
  Tw ti[DEEPEST ? IPT : 1][E - 1];
  Item it[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    it[u] = item_at(tid + u * NT, LOGR, 0, l0, KS);
    lds_tw<Ring, KS>(t[u], stw, l0, it[u].sb);
    if constexpr (DEEPEST) lds_tw<Ring, KS>(ti[u], stwi, l0, it[u].sb);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (FIRST) {
        va[u][i] = srca(R, P.inst, P.base + row);
        vx[u][i] = srcx(R, P.inst, P.base + row);
      } else {
        va[u][i] = sa[row];
        vx[u][i] = sx[row];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    split_levels<Ring, KS, true, true>(R, va[u], vx[u], t[u]);
    if constexpr (DEEPEST) {
#pragma unroll
      for (int i = 0; i < E; ++i) va[u][i] = R.leaf(va[u][i], vx[u][i]);
      merge_levels<Ring, KS>(R, va[u], ti[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (DEEPEST && FIRST) {
        dst(P.inst, P.base + row, A.final_store ? R.canon(va[u][i]) : va[u][i]);
      } else {
        sa[row] = va[u][i];
        if constexpr (!DEEPEST) sx[row] = vx[u][i];
      }
    }
}

// One merge stage of KS levels. LAST: write dst.
template <class Ring, int LOGR, int K, int KS, bool LAST, class Dst>
__device__ __forceinline__ void small_merge_stage(const PassArgs<Ring>& A, const TilePos& P, const Ring& R,
                                                  const typename Ring::Tw* stwi, typename Ring::T* sa, uint32_t l0,
                                                  uint32_t tid, const Dst& dst) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  constexpr int E = 1 << KS;
  constexpr int IPT = (1 << K) / E;
  constexpr uint32_t NT = SmallShape<LOGR, K>::NT;
  T v[IPT][E];
  Tw t[IPT][E - 1];
  Item it[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    it[u] = item_at(tid + u * NT, LOGR, 0, l0, KS);
    lds_tw<Ring, KS>(t[u], stwi, l0, it[u].sb);
#pragma unroll
    for (int i = 0; i < E; ++i) v[u][i] = sa[it[u].row0 + ((uint32_t)i << it[u].sh)];
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u) merge_levels<Ring, KS>(R, v[u], t[u]);
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (LAST)
        dst(P.inst, P.base + row, A.final_store ? R.canon(v[u][i]) : v[u][i]);
      else
        sa[row] = v[u][i];
    }
}

template <class Ring, int LOGR, int K, class SrcA, class SrcX, class Dst>
__global__ void __launch_bounds__((SmallShape<LOGR, K>::NT)) k_small(PassArgs<Ring> A, typename Ring::Params rp0,
                                                                   typename Ring::Params rp1, typename Ring::Params rp2,
                                                                   SrcA srca, SrcX srcx, Dst dst) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  using S = SmallShape<LOGR, K>;
  static_assert(S::NST >= 2, "at least two stages");
  const uint32_t tid = threadIdx.x;
  T* sa = reinterpret_cast<T*>(smem_raw);
  T* sx = sa + (1u << LOGR);
  Tw* stw = reinterpret_cast<Tw*>(sx + (1u << LOGR));
  Tw* stwi = stw + S::NTW;
  const TilePos P = tile_pos(A, blockIdx.x);
  uint32_t rsel;
  const Ring R = make_ring(A, P.inst, rp0, rp1, rp2, &rsel);
  // the tree of one instance (d0 = 0, block 0): level l is heap range [2^l, 2^(l+1)),
  // local index 2^l - 1 + g, so the copy is contiguous
  const Tw* tw = A.tw[rsel] + 1;
  const Tw* twi = A.twi[rsel] + 1;
  for (uint32_t e = tid; e < (uint32_t)S::NTW; e += S::NT) {
    stw[e] = tw[e];
    stwi[e] = twi[e];
  }
  __syncthreads();
  small_split_stage<Ring, LOGR, K, S::K0, true, false>(A, P, R, stw, stwi, sa, sx, 0, tid, srca, srcx, dst);
  __syncthreads();
#pragma unroll
  for (int s = 1; s < S::NST; ++s) {
    const uint32_t l0 = S::K0 + K * (s - 1);
    if (s + 1 == S::NST)
      small_split_stage<Ring, LOGR, K, K, false, true>(A, P, R, stw, stwi, sa, sx, l0, tid, srca, srcx, dst);
    else
      small_split_stage<Ring, LOGR, K, K, false, false>(A, P, R, stw, stwi, sa, sx, l0, tid, srca, srcx, dst);
    __syncthreads();
  }
#pragma unroll
  for (int s = S::NST - 2; s >= 1; --s) {
    small_merge_stage<Ring, LOGR, K, K, false>(A, P, R, stwi, sa, S::K0 + K * (s - 1), tid, dst);
    __syncthreads();
  }
  small_merge_stage<Ring, LOGR, K, S::K0, true>(A, P, R, stwi, sa, 0, tid, dst);
}

// ---------------------------------------------------------------------------------------
// Leaf-domain block pass: the row's leaves are given (the row transform of the whole
// product, shared by every instance), so a block only splits the vector, multiplies each
// leaf by the row's leaf (conjugated if CONJ) and 1/n, and merges back up. Same stage plan
// and twiddle staging as block_pass; LDS holds the vector only.
// ---------------------------------------------------------------------------------------
template <class Ring, int LOGR, int NT = 0>
constexpr size_t lf_block_lds_bytes() {
  using S = BlockShape<LOGR, NT>;
  return (size_t)S::GROUPS * ((sizeof(typename Ring::T) << LOGR) + 2 * (size_t)S::NTW * sizeof(BlockTw<Ring, true>));
}

template <class Ring, int LOGR, int K, bool FIRST, bool DEEPEST, bool CONJ, class SrcX, class Lv, class Dst>
__device__ __forceinline__ void lf_split_stage(const PassArgs<Ring>& A, const TilePos& P, const Ring& R, uint32_t rsel,
                                               typename Ring::Tw const* tw, typename Ring::Tw const* twi,
                                               const BlockTw<Ring, true>* stw, const DeepTw<Ring>& D, typename Ring::T* sx,
                                               uint32_t l0, uint32_t ltid, const SrcX& srcx, const Lv& leaves,
                                               const Dst& dst) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  using S = BlockShape<LOGR>;
  constexpr int E = 1 << K;
  constexpr int IPT = S::EPT / E;
  constexpr uint32_t ACTIVE = 1u << S::ACTIVE_LOG;
  constexpr bool FROM_D = DEEPEST && !FIRST;
  constexpr bool FIRSTS = DEEPEST && K == EPT_LOG;
  static_assert(!FROM_D || K == EPT_LOG, "deepest stage of a multi-stage block pass is radix 16");
  T vx[IPT][E];
  using TwS = std::conditional_t<FIRST, Tw, BlockTw<Ring, true>>;  // heap (Shoup) or LDS copy
  TwS t[(FROM_D || FIRSTS) ? 1 : IPT][E - 1];
  Tw ti[(DEEPEST && !FROM_D && !FIRSTS) ? IPT : 1][E - 1];
  DeepTw<Ring> Dl[FIRSTS && !FROM_D ? IPT : 1];  // single-stage radix-16 block: from the heap
  Item it[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    it[u] = item_at(ltid + u * ACTIVE, LOGR, 0, l0, K);
    if constexpr (FIRST) {
      if constexpr (FIRSTS) {
        load_deep_heap<Ring>(Dl[u], R, tw, twi, A.d0, P.blk, l0, it[u].sb);
      } else {
        load_tw<Ring, K>(t[u], tw, A.d0, P.blk, l0, it[u].sb);
        if constexpr (DEEPEST) load_tw<Ring, K>(ti[u], twi, A.d0, P.blk, l0, it[u].sb);
      }
    } else if constexpr (!DEEPEST) {
      lds_tw<Ring, K>(t[u], stw, l0, it[u].sb);
    }
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (FIRST)
        vx[u][i] = srcx(R, P.inst, P.base + row);
      else
        vx[u][i] = sx[row];
    }
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    if constexpr (FROM_D)
      split_levels_first<Ring, K, false, true>(R, vx[u], vx[u], D.t, A.tu[rsel]);
    else if constexpr (FIRSTS)
      split_levels_first<Ring, K, false, true>(R, vx[u], vx[u], Dl[u].t, A.tu[rsel]);
    else
      split_levels_w<Ring, K, false, true>(R, vx[u], vx[u], t[u]);
  }
  if constexpr (DEEPEST) {
#pragma unroll
    for (int u = 0; u < IPT; ++u)
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
        vx[u][i] = R.leaf(leaves.template get<CONJ>(P.base + row), vx[u][i]);
      }
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      if constexpr (FROM_D)
        merge_levels_first<Ring, K>(R, vx[u], D.ti, A.tui[rsel]);
      else if constexpr (FIRSTS)
        merge_levels_first<Ring, K>(R, vx[u], Dl[u].ti, A.tui[rsel]);
      else
        merge_levels<Ring, K>(R, vx[u], ti[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < IPT; ++u)
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = it[u].row0 + ((uint32_t)i << it[u].sh);
      if constexpr (DEEPEST && FIRST)
        dst(P.inst, P.base + row, A.final_store ? R.canon(vx[u][i]) : vx[u][i]);
      else
        sx[row] = vx[u][i];
    }
}

template <class Ring, int LOGR, int NT, bool CONJ, class SrcX, class Lv, class Dst>
__device__ __forceinline__ void lf_block_pass(const PassArgs<Ring>& A, uint32_t vwg0, uint32_t tid, unsigned char* smem_raw,
                                              const typename Ring::Params& rp, const SrcX& srcx, const Lv& leaves,
                                              const Dst& dst) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  using S = BlockShape<LOGR, NT>;
  static_assert(LOGR >= 1, "at least one level");
  const uint32_t group = tid >> S::ACTIVE_LOG;
  const uint32_t ltid = tid & ((1u << S::ACTIVE_LOG) - 1);
  const uint32_t vwg = vwg0 + group;
  const bool active = group < S::GROUPS && vwg < A.tiles * A.ninst;
  T* sx = reinterpret_cast<T*>(smem_raw) + ((size_t)group << LOGR);
  using DW = BlockTw<Ring, true>;
  DW* stw = reinterpret_cast<DW*>(smem_raw + (size_t)S::GROUPS * (sizeof(T) << LOGR)) + (size_t)group * 2 * S::NTW;
  DW* stwi = stw + S::NTW;
  const TilePos P = tile_pos(A, active ? vwg : 0);
  const uint32_t rsel = 0;
  const Ring R(rp);
  const Tw* tw = A.tw[0];
  const Tw* twi = A.twi[0];
  constexpr int NST = S::NST, K0 = S::K0;
  DeepTw<Ring> D;
  if constexpr (NST > 1) {
    if (active) {
      for (uint32_t e = ltid; e < (uint32_t)S::NTW; e += 1u << S::ACTIVE_LOG) {
        const uint32_t l = 31u - __clz(e + 1);
        const uint32_t gi = (1u << (A.d0 + l)) + (P.blk << l) + (e + 1 - (1u << l));
        stw[e] = to_block_tw<Ring, true>(R, tw[gi]);
        stwi[e] = to_block_tw<Ring, true>(R, twi[gi]);
      }
      load_deep_tw<Ring, LOGR>(D, R, A, P, rsel, tw, twi, ltid);
    }
  }
  if (active) lf_split_stage<Ring, LOGR, K0, true, NST == 1, CONJ>(A, P, R, rsel, tw, twi, stw, D, sx, 0, ltid, srcx, leaves, dst);
  if constexpr (NST > 1) {
    stage_sync(block_in_one_wave<LOGR>());
#pragma unroll
    for (int s = 1; s < NST; ++s) {
      const uint32_t l0 = K0 + EPT_LOG * (s - 1);
      if (active) {
        if (s + 1 == NST)
          lf_split_stage<Ring, LOGR, EPT_LOG, false, true, CONJ>(A, P, R, rsel, tw, twi, stw, D, sx, l0, ltid, srcx, leaves, dst);
        else
          lf_split_stage<Ring, LOGR, EPT_LOG, false, false, CONJ>(A, P, R, rsel, tw, twi, stw, D, sx, l0, ltid, srcx, leaves, dst);
      }
      const int nxt = s + 1 < NST ? s : NST - 2;
      stage_sync(nxt >= 1 && wave_region<LOGR>(K0 + EPT_LOG * (nxt - 1)) ? true : block_in_one_wave<LOGR>());
    }
#pragma unroll
    for (int s = NST - 2; s >= 1; --s) {
      const uint32_t l0 = K0 + EPT_LOG * (s - 1);
      if (active) block_merge_stage<Ring, LOGR, EPT_LOG, false>(A, P, R, stwi, sx, l0, ltid, dst);
      stage_sync(s - 1 >= 1 && wave_region<LOGR>(K0 + EPT_LOG * (s - 2)) ? true : block_in_one_wave<LOGR>());
    }
    if (active) block_merge_stage<Ring, LOGR, K0, true>(A, P, R, stwi, sx, 0, ltid, dst);
  }
}

template <class Ring, int LOGR, bool CONJ, class SrcX, class Lv, class Dst>
__global__ void __launch_bounds__(BlockShape<LOGR>::NT) k_lf_block(PassArgs<Ring> A, typename Ring::Params rp, SrcX srcx,
                                                                    Lv leaves, Dst dst) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using S = BlockShape<LOGR>;
  lf_block_pass<Ring, LOGR, S::NT, CONJ>(A, blockIdx.x * S::GROUPS, threadIdx.x, smem_raw, rp, srcx, leaves, dst);
}

// ---------------------------------------------------------------------------------------
// Accumulating block pass: for one depth-(logn - LOGR) block and instances [b0, b1), split
// the row and the vector of each instance down to the leaves and add their leaf products
// into per-thread accumulators; no merge. Writes the sums for the block's leaves through
// out(chunk, index, value). One thread group per workgroup (LOGR >= 10).
// ---------------------------------------------------------------------------------------
template <class Ring, int LOGR, class SrcA, class SrcX, class Out>
__device__ __forceinline__ void acc_block_pass(const PassArgs<Ring>& A, uint32_t blk, uint32_t b0, uint32_t b1,
                                               uint32_t chunk, uint32_t tid, unsigned char* smem_raw,
                                               const typename Ring::Params& rp, const SrcA& srca, const SrcX& srcx,
                                               const Out& out) {
  using T = typename Ring::T;
  using Tw = typename Ring::Tw;
  using S = BlockShape<LOGR>;
  static_assert(S::GROUPS == 1 && S::NST > 1, "one block of at least 2^10 elements per workgroup");
  constexpr int NST = S::NST, K0 = S::K0;
  constexpr int K = EPT_LOG, E = 1 << K;
  const uint32_t ltid = tid;
  T* sa = reinterpret_cast<T*>(smem_raw);
  T* sx = sa + ((size_t)1 << LOGR);
  using DW = BlockTw<Ring, true>;
  DW* stw = reinterpret_cast<DW*>(smem_raw + 2 * (sizeof(T) << LOGR));
  DW* stwi = stw + S::NTW;
  const Ring R(rp);
  const Tw* tw = A.tw[0];
  const Tw* twi = A.twi[0];
  const TilePos P0 = tile_pos(A, blk);  // block position (instance 0)
  for (uint32_t e = ltid; e < (uint32_t)S::NTW; e += 1u << S::ACTIVE_LOG) {
    const uint32_t l = 31u - __clz(e + 1);
    const uint32_t gi = (1u << (A.d0 + l)) + (P0.blk << l) + (e + 1 - (1u << l));
    stw[e] = to_block_tw<Ring, true>(R, tw[gi]);
    stwi[e] = to_block_tw<Ring, true>(R, twi[gi]);
  }
  DeepTw<Ring> D;
  load_deep_tw<Ring, LOGR>(D, R, A, P0, 0, tw, twi, ltid);
  constexpr uint32_t l0d = LOGR - EPT_LOG;
  const Item itd = item_at(ltid, LOGR, 0, l0d, K);
  T acc[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = T{};
  for (uint32_t b = b0; b < b1; ++b) {
    TilePos P = P0;
    P.inst = b;
    block_split_stage<Ring, LOGR, K0, true, false>(A, P, R, 0, tw, twi, stw, D, sa, sx, 0, ltid, srca, srcx, out);
    stage_sync(block_in_one_wave<LOGR>());
#pragma unroll
    for (int s = 1; s + 1 < NST; ++s) {
      block_split_stage<Ring, LOGR, EPT_LOG, false, false>(A, P, R, 0, tw, twi, stw, D, sa, sx, K0 + EPT_LOG * (s - 1), ltid,
                                                           srca, srcx, out);
      stage_sync(wave_region<LOGR>(K0 + EPT_LOG * (s - 1)));
    }
    // deepest stage: split both, add the leaf products
    T va[E], vx[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const uint32_t row = itd.row0 + ((uint32_t)i << itd.sh);
      va[i] = sa[row];
      vx[i] = sx[row];
    }
    split_levels_first<Ring, K>(R, va, vx, D.t, A.tu[0]);
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] = R.add(acc[i], R.leaf(va[i], vx[i]));
    __syncthreads();  // LDS is refilled by the next instance
  }
#pragma unroll
  for (int i = 0; i < E; ++i) out(chunk, P0.base + itd.row0 + ((uint32_t)i << itd.sh), acc[i]);
}

template <class Ring, int LOGR, class SrcA, class SrcX, class Out>
__global__ void __launch_bounds__(BlockShape<LOGR>::NT) k_acc_block(PassArgs<Ring> A, typename Ring::Params rp,
                                                                     uint32_t per_chunk, SrcA srca, SrcX srcx, Out out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const uint32_t blk = blockIdx.x % A.tiles, chunk = blockIdx.x / A.tiles;
  const uint32_t b0 = chunk * per_chunk, b1 = min(A.ninst, b0 + per_chunk);
  acc_block_pass<Ring, LOGR>(A, blk, b0, b1, chunk, threadIdx.x, smem_raw, rp, srca, srcx, out);
}

template <class Ring, int LOGR, class SrcA, class SrcX, class Dst, bool MONT = true, int EL = EPT_LOG>
__global__ void __launch_bounds__((BlockShape<LOGR, 0, EL>::NT)) k_block(PassArgs<Ring> A, typename Ring::Params rp0,
                                                                 typename Ring::Params rp1, typename Ring::Params rp2,
                                                                 SrcA srca, SrcX srcx, Dst dst) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using S = BlockShape<LOGR, 0, EL>;
  block_pass<Ring, LOGR, S::NT, MONT, EL>(A, blockIdx.x * S::GROUPS, threadIdx.x, smem_raw, rp0, rp1, rp2, srca, srcx, dst);
}

}  // namespace fcirc
