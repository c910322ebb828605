// Host-side internals of libfcirc: context, twiddle plans, pass schedules, workspace,
// per-kernel event timing, and the driver that enqueues one f-circulant product (or a
// batch of equal-size products) as top split passes -> block pass -> top merge passes.
#pragma once
#include <hip/hip_ext.h>
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/fcirc.h"
#include "ring.hpp"
#include "tile.hpp"

namespace fcirc {

// ----------------------------------------------------------------------------------------
// Timing: HIP events around every kernel the library enqueues (opt-in).
// ----------------------------------------------------------------------------------------
struct Timer {
  bool enabled = false;
  struct Rec {
    int name;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<std::string> names;
  std::vector<uint64_t> launches;
  std::vector<double> ms;
  std::vector<hipEvent_t> pool;

  int name_id(const char* n) {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == n) return (int)i;
    names.emplace_back(n);
    launches.push_back(0);
    ms.push_back(0.0);
    return (int)names.size() - 1;
  }
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void collect() {
    for (auto& r : pending) {
      float t = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        launches[r.name] += 1;
        ms[r.name] += t;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  ~Timer() {
    for (auto& r : pending) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// ----------------------------------------------------------------------------------------
// Twiddle tables (heap order, index 2^d + b) for one ring and one f.
// ----------------------------------------------------------------------------------------
// Uniform radix-16 factors rho_j^brev_j(g), j < 4, and their inverses (host side).
template <class Ring>
struct Uniform16 {
  typename Ring::Tw tu[15], tui[15];
};

// Levels of the Z/p block factors (see PassArgs::ub): every block pass of at most 2^13.
constexpr int ZP_UB_LEVELS = 13;
constexpr size_t ZP_UB = ((size_t)1 << ZP_UB_LEVELS) - 1;

struct ZpTables {
  uint32_t p = 0, f = 0;
  int levels = 0;  // covers depths d < levels
  ZpTw* tw = nullptr;
  ZpTw* twi = nullptr;
  // uniform factors in Montgomery form (device): tu[15], tui[15], then the block factors
  // ub[ZP_UB] and ubi[ZP_UB]
  uint32_t* dU = nullptr;
  // last first-twiddle of the deepest radix-16 stage per item, Montgomery form, per log2 n
  // (see PassArgs::ft)
  uint32_t* ft[27] = {nullptr};
  uint32_t* fti[27] = {nullptr};
};

struct Gp2Tables {
  int fneg = 0;    // 0: f = 1, 1: f = -1
  int levels = 0;  // covers depths d < levels
  uint2* tw = nullptr;
  uint2* twi = nullptr;
  uint2* dU = nullptr;  // uniform radix-16 factors: tu[15] then tui[15]
};

struct C32Tables {
  double fre = 1.0, fim = 0.0;
  int levels = 0;
  float2* tw = nullptr;
  float2* twi = nullptr;
  Uniform16<C32> U;
  float2* dU = nullptr;  // device copy: tu[15] then tui[15]
};

// ----------------------------------------------------------------------------------------
// Pass schedule of one product of size 2^L.
// ----------------------------------------------------------------------------------------
struct Schedule {
  int L = 0;
  int flags = 1;         // FCIRC_SCHED_* bits: XCD-aware tile order, separate row/vector split
  int block_levels = 0;  // levels done in the LDS-resident block pass
  int ntop = 0;          // HBM-streamed top passes
  int top_d0[4] = {0, 0, 0, 0};
  int top_r[4] = {0, 0, 0, 0};
  int top_c[4] = {0, 0, 0, 0};  // log2 tile columns
};

struct TuneKey {
  int ring, L;
  bool operator<(const TuneKey& o) const { return ring != o.ring ? ring < o.ring : L < o.L; }
};
struct TuneVal {
  int top = -1;       // top levels (HBM-streamed), -1: default
  int tile_log = -1;  // log2 elements per top-pass tile, -1: default
  int flags = 1;      // FCIRC_SCHED_* bits
};

// A workspace the caller brings (fcirc_matvec_noalloc): the product then allocates nothing,
// so its twiddle tables must already be resident (FCIRC_ENOPLAN otherwise) and its
// workspace must fit in `bytes` (FCIRC_ESIZE otherwise).
struct FixedWs {
  void* ptr;
  size_t bytes;
};

// Bits of the sticky device status word (Ctx::d_status[0]), reported by fcirc_check.
constexpr uint32_t FCIRC_STATUS_RANGE = 1u;  // a CRT result fell outside the exact range (ERANGE)
constexpr uint32_t FCIRC_STATUS_SCHED = 2u;  // a batched launch's dependency wait gave up (ESCHED)

struct BatchEntry;  // cached batched launches: device item queue and kernel arguments (batched.hip)

// Parameters of the batched launch for one (ring, instance size), per workgroup size
// (index 0: 256 threads, 1: 512): the block levels of the three-pass form of an instance
// (0: the whole instance is one FULL item; -1: not set, the default applies) and the time
// per coefficient measured by fcirc_tune (ns; negative: not measured).
struct BatchTune {
  int blog[2] = {-1, -1};
  float ns[2] = {-1.f, -1.f};
};
// Parameters forced for one instance size while fcirc_tune times them.
struct BatchForce {
  int L, bt, blog;
};

struct Ctx {
  int device = 0;
  hipDeviceProp_t prop{};
  std::deque<ZpTables> zp;   // deque: references stay valid as plans are added
  std::deque<C32Tables> c32;
  std::deque<Gp2Tables> gp2;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* ws2 = nullptr;  // operands of the embedded (arbitrary-n, Toeplitz) products
  size_t ws2_bytes = 0;
  size_t ws_limit = SIZE_MAX;  // bound on ws_bytes + ws2_bytes
  uint32_t* d_status = nullptr;  // [0] sticky ERANGE word, [1] input-check flag
  bool check_inputs = false;     // FCIRC_CHECK_INPUTS
  int forced_top = -1;
  std::map<TuneKey, TuneVal> tuned;
  Timer timer;
  std::vector<BatchEntry*> batches;  // owned; freed by release_batches
  std::map<TuneKey, BatchTune> batch_tuned;
  uint64_t batch_gen = 0;  // bumped whenever batch_tuned changes (cached queues then rebuild)
  bool debug_sync = false;
  void* scratch = nullptr;  // device address of fcirc_matvec_noalloc's array on this device
};

// Launch wrapper. fn(e0, e1) enqueues one kernel; with timing on, e0/e1 are events that
// the kernel's own dispatch records (hipExtLaunchKernelGGL), so the measured interval is
// the kernel alone. Errors are checked; FCIRC_DEBUG_SYNC synchronises after each launch.
#define FCIRC_LAUNCH(e0, e1, kern, grid, block, lds, strm, ...)                                  \
  do {                                                                                        \
    if (e0)                                                                                   \
      hipExtLaunchKernelGGL(kern, grid, block, lds, strm, e0, e1, 0, __VA_ARGS__);            \
    else                                                                                      \
      hipLaunchKernelGGL(kern, grid, block, lds, strm, __VA_ARGS__);                          \
  } while (0)

template <class F>
inline hipError_t launch(Ctx& c, const char* name, hipStream_t s, F&& fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (c.timer.enabled) {
    a = c.timer.get();
    b = c.timer.get();
    if (!a || !b) a = b = nullptr;
  }
  fn(a, b);
  hipError_t e = hipGetLastError();
  if (a && b) c.timer.pending.push_back({c.timer.name_id(name), a, b});
  if (e == hipSuccess && c.debug_sync) e = hipStreamSynchronize(s);
  return e;
}

// Workspace: grows on demand, never shrinks while the context lives. Callers must have
// synchronised nothing: growth frees the old buffer only after a device synchronise.
// Grow one of the context's workspaces to at least `bytes` (contents are not kept).
inline fcirc_status ws_grow(Ctx& c, void** buf, size_t* have, size_t other, size_t bytes) {
  if (bytes <= *have) return FCIRC_OK;
  if (bytes > c.ws_limit || other > c.ws_limit - bytes) return FCIRC_ENOMEM;
  if (*buf) {
    if (hipDeviceSynchronize() != hipSuccess) return FCIRC_EDEVICE;
    (void)hipFree(*buf);
    *buf = nullptr;
    *have = 0;
  }
  size_t want = bytes + bytes / 4;
  if (want > c.ws_limit - other) want = bytes;
  if (hipMalloc(buf, want) != hipSuccess) {
    (void)hipGetLastError();
    return FCIRC_ENOMEM;
  }
  *have = want;
  return FCIRC_OK;
}
inline fcirc_status ws_reserve(Ctx& c, size_t bytes) { return ws_grow(c, &c.ws, &c.ws_bytes, c.ws2_bytes, bytes); }
inline fcirc_status ws2_reserve(Ctx& c, size_t bytes) { return ws_grow(c, &c.ws2, &c.ws2_bytes, c.ws_bytes, bytes); }

// ----------------------------------------------------------------------------------------
// Elementwise global access functors used by the tile kernels.
// ----------------------------------------------------------------------------------------
// Element i (32-bit, within one instance) of instance `inst` (wave-uniform). The byte
// offset of i is formed in 32 bits (an instance holds at most 2^26 elements of 8 bytes), so
// the access is a uniform 64-bit base plus a 32-bit per-lane offset: the global load/store
// form with a scalar base, no 64-bit address arithmetic per lane.
template <class T>
__device__ __forceinline__ const T* elem32(const T* base, uint32_t i) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ T* elem32(T* base, uint32_t i) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
struct LdPlain {
  const T* p;
  uint64_t stride;
  template <class R>
  __device__ __forceinline__ T operator()(const R&, uint32_t inst, uint32_t i) const {
    return *elem32(p + (uint64_t)inst * stride, i);
  }
};
// Store policy of a pass's output. Cached: plain stores (dirty lines stay in the XCD's L2
// and are written back when the kernel ends, after its last wave). Stream: non-temporal
// stores. Agent: relaxed stores at agent scope, written through the L2 as they are made.
// The two last policies move a pass's writes into its compute time instead of a drain
// after it.
enum StorePolicy : int { ST_CACHED = 0, ST_STREAM = 1, ST_AGENT = 2 };

template <class T, int POL = ST_CACHED>
struct StPlain {
  T* p;
  uint64_t stride;
  __device__ __forceinline__ void operator()(uint32_t inst, uint32_t i, T v) const {
    T* q = elem32(p + (uint64_t)inst * stride, i);
    using U = std::conditional_t<sizeof(T) == 4, uint32_t, uint64_t>;
    static_assert(sizeof(T) == sizeof(U), "4- or 8-byte elements");
    if constexpr (POL == ST_STREAM) {
      __builtin_nontemporal_store(__builtin_bit_cast(U, v), reinterpret_cast<U*>(q));
    } else if constexpr (POL == ST_AGENT) {
      __hip_atomic_store(reinterpret_cast<U*>(q), __builtin_bit_cast(U, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      *q = v;
    }
  }
};
struct LdR32 {  // real data promoted to complex
  const float* p;
  uint64_t stride;
  template <class R>
  __device__ __forceinline__ float2 operator()(const R&, uint32_t inst, uint32_t i) const {
    return make_float2(*elem32(p + (uint64_t)inst * stride, i), 0.f);
  }
};
struct StR32 {  // real part of a complex result
  float* p;
  uint64_t stride;
  __device__ __forceinline__ void operator()(uint32_t inst, uint32_t i, float2 v) const {
    *elem32(p + (uint64_t)inst * stride, i) = v.x;
  }
};

// ----------------------------------------------------------------------------------------
// Schedules.
// ----------------------------------------------------------------------------------------
inline int ilog2(uint64_t v) {
  int l = 0;
  while ((1ull << l) < v) ++l;
  return l;
}

// elem_log: log2 bytes per element (2 for uint32, 3 for complex64).
// top_levels < 0: default split; tile_log_in < 0: default tile (32 KiB of LDS).
inline Schedule make_schedule(int L, int elem_log, int top_levels, int tile_log_in = -1, int flags = 1) {
  Schedule s;
  s.L = L;
  s.flags = flags;
  // Largest block pass: row + vector of 2^B elements in LDS (64 KiB Z/p at B = 13, 64 KiB
  // complex at B = 12) plus its staged twiddles.
  const int block_max = elem_log == 2 ? 13 : 12;
  const int tile_max = elem_log == 2 ? 14 : 13;  // 1024 (512) threads x 16 elements per workgroup
  // Defaults measured on MI355X: at least 2^8 blocks (one per CU) once n allows it, blocks
  // of at most 2^block_max and at least 2^10 elements; top-pass tiles of 2^(L-8) elements,
  // within [2^11, 2^13], so that a top pass also has about 2^8 workgroups.
  int tile_log = tile_log_in >= 0 ? tile_log_in : std::min(13, std::max(11, L - 8));
  if (tile_log > tile_max) tile_log = tile_max;
  if (tile_log < 4) tile_log = 4;
  const int top_max = 10;
  int T = top_levels;
  if (T < 0) T = L <= 12 ? 0 : std::max(L - block_max, std::min(8, L - 10));
  // Z/p above 2^21 (every top-level count from L - 13 to L - 8 and tiles of 2^12..2^14
  // timed on MI355X at 2^22..2^26): 2^22 and 2^23 take 10 top levels in one pass over
  // 2^14-element tiles (2^23: 135 against 182 us with 2^13 tiles); from 2^24 on, two top
  // passes over blocks of 2^10 (2^25: 523 against 564 us; 2^26: 1.02 against 1.16 ms).
  if (elem_log == 2 && L >= 22) {
    if (tile_log_in < 0) tile_log = L <= 23 ? 14 : 13;
    if (top_levels < 0) T = L <= 23 ? 10 : L - 10;
  }
  // 8-byte elements from 2^23 on (same sweep, complex64 at 2^20..2^24): two top passes over
  // 2^12-element tiles and blocks of 2^10 (2^23: 218 against 233 us; 2^24: 434 against 445 us).
  if (elem_log == 3 && L >= 23) {
    if (tile_log_in < 0) tile_log = 12;
    if (top_levels < 0) T = L - 10;
  }
  if (T > L) T = L;
  if (L < 5) T = 0;                                // too small for a column tile of 16 elements
  if (L - T > 13 - (elem_log - 2)) T = L - (13 - (elem_log - 2));  // block must fit LDS
  s.block_levels = L - T;
  s.ntop = T == 0 ? 0 : (T + top_max - 1) / top_max;
  int d0 = 0;
  for (int i = 0; i < s.ntop; ++i) {
    const int r = (T - d0) / (s.ntop - i);
    s.top_d0[i] = d0;
    s.top_r[i] = r;
    const int cols_log = L - d0 - r;
    int c = tile_log - r;
    if (c > cols_log) c = cols_log;
    if (c < 0) c = 0;
    s.top_c[i] = c;
    d0 += r;
  }
  return s;
}

// Dynamic LDS above the 64 KiB default needs an explicit opt-in per kernel.
template <class K>
inline void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ----------------------------------------------------------------------------------------
// The product driver.
//   count instances, ring parameters rp[3] / tables tw[3], twi[3] (instance z uses index
//   z % 3 when ring_per_inst). srca/srcx read the inputs, dst receives the final
//   (canonical) values. ws must hold 2 * count * n elements of Ring::T when the schedule
//   has top passes, plus count * n more when `wy` is null (the result then stays in
//   workspace until the last merge pass writes it through dst).
// ----------------------------------------------------------------------------------------
template <class Ring, int LOGR, class SrcA, class SrcX, class Dst>
inline hipError_t launch_block_l(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, SrcA sa, SrcX sx, Dst d,
                                 hipStream_t s) {
  // Radix-16 register stages. Measured on MI355X at 2^13-element blocks against radix 8
  // (1024 threads, 47 VGPRs): one 2^21 product over Z/p, block pass 19.3 us against 21.5.
  constexpr int EL = EPT_LOG;
  using S = BlockShape<LOGR, 0, EL>;
  const uint64_t vwgs = (uint64_t)A.tiles * A.ninst;
  const uint32_t grid = (uint32_t)((vwgs + S::GROUPS - 1) / S::GROUPS);
  // Montgomery-form staged twiddles (fewer instructions than Shoup pairs). With the deepest
  // stage's twiddles pinned as 32-bit values the kernel needs 98 registers at 2^13 (148
  // before), so two 2^13-element blocks fit a CU in this form too; measured on MI355X for
  // three 2^21 products (polymul, bigint) against the Shoup-pair kernel then picked for
  // launches of more blocks than CUs: 95.9 against 96.6-97.5 us, and 103.5 against 104.5 us.
  const size_t lds = block_lds_bytes<Ring, LOGR, 0, true, EL>();
  const auto k = k_block<Ring, LOGR, SrcA, SrcX, Dst, true, EL>;
  allow_lds(k, lds);
  return launch(c, "fcirc_block", s, [&](hipEvent_t e0_, hipEvent_t e1_) { FCIRC_LAUNCH(e0_, e1_, k, dim3(grid), dim3(S::NT), lds, s, A, rp[0], rp[1], rp[2], sa, sx, d); });
}

template <class Ring, class SrcA, class SrcX, class Dst>
inline hipError_t launch_block(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, SrcA sa, SrcX sx, Dst d,
                               hipStream_t s) {
  switch (A.logr) {
#define FCIRC_BLOCK_CASE(l) \
  case l: return launch_block_l<Ring, l>(c, A, rp, sa, sx, d, s);
    FCIRC_BLOCK_CASE(0) FCIRC_BLOCK_CASE(1) FCIRC_BLOCK_CASE(2) FCIRC_BLOCK_CASE(3) FCIRC_BLOCK_CASE(4)
    FCIRC_BLOCK_CASE(5) FCIRC_BLOCK_CASE(6) FCIRC_BLOCK_CASE(7) FCIRC_BLOCK_CASE(8) FCIRC_BLOCK_CASE(9)
    FCIRC_BLOCK_CASE(10) FCIRC_BLOCK_CASE(11) FCIRC_BLOCK_CASE(12)
#undef FCIRC_BLOCK_CASE
    case 13:
      if constexpr (sizeof(typename Ring::T) == 4) return launch_block_l<Ring, 13>(c, A, rp, sa, sx, d, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// Small-product kernel for 6 <= L <= 12 (one workgroup per instance), radix-4 stages:
// measured on MI355X against radix 8, radix 4 was as fast or faster from 2^7 to 2^11.
template <class Ring, int LOGR, class SrcA, class SrcX, class Dst>
inline hipError_t launch_small_l(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, SrcA sa, SrcX sx, Dst d,
                                 hipStream_t s) {
  constexpr int K = 2;
  const size_t lds = small_lds_bytes<Ring, LOGR, K>();
  auto k = k_small<Ring, LOGR, K, SrcA, SrcX, Dst>;
  allow_lds(k, lds);
  const uint32_t grid = A.tiles * A.ninst;
  return launch(c, "fcirc_block", s, [&](hipEvent_t e0_, hipEvent_t e1_) { FCIRC_LAUNCH(e0_, e1_, k, dim3(grid), dim3(SmallShape<LOGR, K>::NT), lds, s, A, rp[0], rp[1], rp[2], sa, sx, d); });
}

template <class Ring, class SrcA, class SrcX, class Dst>
inline hipError_t launch_small(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, SrcA sa, SrcX sx, Dst d,
                               hipStream_t s) {
  switch (A.logr) {
#define FCIRC_SMALL_CASE(l) \
  case l: return launch_small_l<Ring, l>(c, A, rp, sa, sx, d, s);
    FCIRC_SMALL_CASE(6) FCIRC_SMALL_CASE(7) FCIRC_SMALL_CASE(8) FCIRC_SMALL_CASE(9) FCIRC_SMALL_CASE(10)
    FCIRC_SMALL_CASE(11) FCIRC_SMALL_CASE(12)
#undef FCIRC_SMALL_CASE
    default: return hipErrorInvalidValue;
  }
}

template <class Ring, int R, class SrcA, class SrcX, class Dst>
inline hipError_t launch_split_r(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, SrcA sa, SrcX sx, Dst da,
                                 Dst dx, uint32_t grid, uint32_t nt, size_t lds, hipStream_t s) {
  auto k = k_split<Ring, R, SrcA, SrcX, Dst>;
  allow_lds(k, lds);
  return launch(c, "fcirc_top_split", s, [&](hipEvent_t e0_, hipEvent_t e1_) { FCIRC_LAUNCH(e0_, e1_, k, dim3(grid), dim3(nt), lds, s, A, rp[0], rp[1], rp[2], sa, sx, da, dx); });
}
template <class Ring, int R, class SrcA, class SrcX, class Dst>
inline hipError_t launch_split_ax_r(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, SrcA sa, SrcX sx,
                                    Dst da, Dst dx, uint32_t grid, uint32_t nt, hipStream_t s) {
  auto k = k_split_ax<Ring, R, SrcA, SrcX, Dst>;
  const size_t lds = split_ax_lds_bytes<Ring, R>((size_t)1 << (A.logr + A.logc));
  allow_lds(k, lds);
  return launch(c, "fcirc_top_split", s, [&](hipEvent_t e0_, hipEvent_t e1_) { FCIRC_LAUNCH(e0_, e1_, k, dim3(grid), dim3(nt), lds, s, A, rp[0], rp[1], rp[2], sa, sx, da, dx); });
}
template <class Ring, int R, class Src, class Dst>
inline hipError_t launch_merge_r(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, Src src, Dst dst,
                                 uint32_t grid, uint32_t nt, size_t lds, hipStream_t s) {
  auto k = k_merge<Ring, R, Src, Dst>;
  allow_lds(k, lds);
  return launch(c, "fcirc_top_merge", s, [&](hipEvent_t e0_, hipEvent_t e1_) { FCIRC_LAUNCH(e0_, e1_, k, dim3(grid), dim3(nt), lds, s, A, rp[0], rp[1], rp[2], src, dst); });
}

#define FCIRC_R_SWITCH(R_, CALL)          \
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
    default: return hipErrorInvalidValue; \
  }

template <class Ring, class SrcA, class SrcX, class Dst>
inline hipError_t launch_split(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, SrcA sa, SrcX sx, Dst da,
                               Dst dx, uint32_t grid, uint32_t nt, size_t lds, hipStream_t s) {
#define FCIRC_CALL(r) launch_split_r<Ring, r>(c, A, rp, sa, sx, da, dx, grid, nt, lds, s)
  FCIRC_R_SWITCH(A.logr, FCIRC_CALL)
#undef FCIRC_CALL
}
template <class Ring, class SrcA, class SrcX, class Dst>
inline hipError_t launch_split_ax(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, SrcA sa, SrcX sx, Dst da,
                                  Dst dx, uint32_t grid, uint32_t nt, hipStream_t s) {
#define FCIRC_CALL(r) launch_split_ax_r<Ring, r>(c, A, rp, sa, sx, da, dx, grid, nt, s)
  FCIRC_R_SWITCH(A.logr, FCIRC_CALL)
#undef FCIRC_CALL
}
template <class Ring, class Src, class Dst>
inline hipError_t launch_merge(Ctx& c, const PassArgs<Ring>& A, const typename Ring::Params* rp, Src src, Dst dst,
                               uint32_t grid, uint32_t nt, size_t lds, hipStream_t s) {
#define FCIRC_CALL(r) launch_merge_r<Ring, r>(c, A, rp, src, dst, grid, nt, lds, s)
  FCIRC_R_SWITCH(A.logr, FCIRC_CALL)
#undef FCIRC_CALL
}

// The pass arguments every pass of one product shares (tables, size, instances).
template <class Ring>
inline PassArgs<Ring> product_pass_args(const Schedule& S, uint32_t count, typename Ring::Tw const* const* tw,
                                        typename Ring::Tw const* const* twi, typename Ring::DeepW const* const* U,
                                        typename Ring::DeepW const* const* FT, typename Ring::DeepW const* const* FTI,
                                        bool ring_per_inst) {
  PassArgs<Ring> A{};
  for (int r = 0; r < 3; ++r) {
    A.tu[r] = U[r];
    A.tui[r] = U[r] + 15;
    A.ft[r] = FT ? FT[r] : nullptr;
    A.fti[r] = FTI ? FTI[r] : nullptr;
    if constexpr (std::is_same_v<Ring, Zp>) {
      A.ub[r] = U[r] + 30;
      A.ubi[r] = U[r] + 30 + ZP_UB;
    }
  }
  for (int i = 0; i < 3; ++i) {
    A.tw[i] = tw[i];
    A.twi[i] = twi[i];
  }
  A.logn = S.L;
  A.ninst = count;
  A.ring_per_inst = ring_per_inst ? 1 : 0;
  A.xcd = (S.flags & FCIRC_SCHED_XCD) ? 1 : 0;
  return A;
}

template <class Ring, class SrcA, class SrcX, class Dst>
inline hipError_t run_product(Ctx& c, const Schedule& S, uint32_t count, const typename Ring::Params* rp,
                              typename Ring::Tw const* const* tw, typename Ring::Tw const* const* twi,
                              typename Ring::DeepW const* const* U, typename Ring::DeepW const* const* FT,
                              typename Ring::DeepW const* const* FTI, bool ring_per_inst, SrcA srca, SrcX srcx, Dst dst,
                              typename Ring::T* wy, typename Ring::T* ws, hipStream_t s) {
  using T = typename Ring::T;
  const int L = S.L;
  const uint64_t n = (uint64_t)1 << L;
  PassArgs<Ring> A = product_pass_args<Ring>(S, count, tw, twi, U, FT, FTI, ring_per_inst);
  hipError_t e;
  if (S.ntop == 0) {
    A.d0 = 0;
    A.logr = L;
    A.logc = 0;
    A.tiles = 1;
    A.narr = 1;
    A.final_store = 1;
    // The small-product kernel takes one workgroup of up to 1024 threads per instance; for
    // batches of more than 2^21 elements in all, the block pass's smaller workgroups fill the
    // chip better (measured: 1024 x 2^12 in 30.8 us against 39.4 us).
    if ((S.flags & FCIRC_SCHED_SMALL) && L >= 6 && L <= 12 && ((uint64_t)count << L) <= (1ull << 21))
      return launch_small<Ring>(c, A, rp, srca, srcx, dst, s);
    return launch_block<Ring>(c, A, rp, srca, srcx, dst, s);
  }
  T* wa = ws;
  T* wx = ws + (uint64_t)count * n;
  if (!wy) wy = ws + 2 * (uint64_t)count * n;
  const LdPlain<T> lwa{wa, n}, lwx{wx, n}, lwy{wy, n};
  // Split outputs are streamed out, the block pass's output is written through at agent
  // scope; the caller's dst keeps its own policy (measured on MI355X at n = 2^21).
  const StPlain<T, ST_STREAM> swa{wa, n}, swx{wx, n};
  const StPlain<T, ST_AGENT> swy{wy, n};
  for (int i = 0; i < S.ntop; ++i) {
    A.d0 = S.top_d0[i];
    A.logr = S.top_r[i];
    A.logc = S.top_c[i];
    A.tiles = (uint32_t)(n >> (A.logr + A.logc));
    A.final_store = 0;
    const size_t tile = (size_t)1 << (A.logr + A.logc);
    const uint32_t nt = (uint32_t)(tile >> EPT_LOG);
    if (S.flags & FCIRC_SCHED_SEPARATE) {  // row and vector tiles in separate workgroups
      A.narr = 2;
      const size_t lds = tile * sizeof(T);
      const uint32_t grid = A.tiles * 2 * count;
      if (i == 0)
        e = launch_split<Ring>(c, A, rp, srca, srcx, swa, swx, grid, nt, lds, s);
      else
        e = launch_split<Ring>(c, A, rp, lwa, lwx, swa, swx, grid, nt, lds, s);
    } else {  // one workgroup per tile of both
      A.narr = 1;
      const uint32_t grid = A.tiles * count;
      if (i == 0)
        e = launch_split_ax<Ring>(c, A, rp, srca, srcx, swa, swx, grid, nt, s);
      else
        e = launch_split_ax<Ring>(c, A, rp, lwa, lwx, swa, swx, grid, nt, s);
    }
    if (e != hipSuccess) return e;
  }
  A.d0 = L - S.block_levels;
  A.logr = S.block_levels;
  A.logc = 0;
  A.tiles = 1u << A.d0;
  A.narr = 1;
  A.final_store = 0;
  e = launch_block<Ring>(c, A, rp, lwa, lwx, swy, s);
  if (e != hipSuccess) return e;
  for (int i = S.ntop - 1; i >= 0; --i) {
    A.d0 = S.top_d0[i];
    A.logr = S.top_r[i];
    A.logc = S.top_c[i];
    A.tiles = (uint32_t)(n >> (A.logr + A.logc));
    A.narr = 1;
    A.final_store = i == 0 ? 1 : 0;
    const size_t tile = (size_t)1 << (A.logr + A.logc);
    const size_t lds = tile * sizeof(T);
    const uint32_t grid = A.tiles * count, nt = (uint32_t)(tile >> EPT_LOG);
    if (i == 0)
      e = launch_merge<Ring>(c, A, rp, lwy, dst, grid, nt, lds, s);
    else
      e = launch_merge<Ring>(c, A, rp, lwy, swy, grid, nt, lds, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Workspace elements run_product needs (Ring::T units).
inline uint64_t product_ws_elems(const Schedule& S, uint32_t count, bool need_wy) {
  if (S.ntop == 0) return 0;
  const uint64_t n = (uint64_t)1 << S.L;
  return (uint64_t)count * n * (need_wy ? 3 : 2);
}

// ----------------------------------------------------------------------------------------
// Plans (zp.hip, c32.hip) and helpers shared by the entry points.
// ----------------------------------------------------------------------------------------
uint32_t zp_prime(fcirc_ring r);
int zp_two_adic(uint32_t p);
// Tables for (p, f) covering at least L levels; ENOROOT if f has no 2^L-th root.
fcirc_status zp_tables(Ctx& c, uint32_t p, uint32_t f, int L, const ZpTables** out, bool build = true);
// Packed deepest-stage first twiddles for size 2^L (L >= 4), built on first use.
fcirc_status zp_first_tables(Ctx& c, const ZpTables* T, int L, const uint32_t** ft, const uint32_t** fti,
                             bool build = true);
ZpParams zp_params(uint32_t p, int L);
fcirc_status c32_tables(Ctx& c, double fre, double fim, int L, hipStream_t s, const C32Tables** out, bool build = true);


// With fx set the product allocates nothing (see FixedWs).
fcirc_status zp_matvec(Ctx& c, const uint32_t* a, const uint32_t* x, uint32_t* y, int L, uint32_t count, uint32_t p,
                       uint32_t f, hipStream_t s, const FixedWs* fx = nullptr);
fcirc_status c32_matvec(Ctx& c, const void* a, const void* x, void* y, int L, uint32_t count, double fre, double fim,
                        bool real_io, hipStream_t s, const FixedWs* fx = nullptr);

fcirc_status gp2_matvec(Ctx& c, const void* a, const void* x, void* y, int L, uint32_t count, int fneg, hipStream_t s,
                        const FixedWs* fx = nullptr);

// The workspace of a product: the context's (grown on demand), or the caller's fixed one.
inline fcirc_status product_ws(Ctx& c, const FixedWs* fx, size_t bytes, void** ws) {
  if (fx) {
    if (bytes > fx->bytes) return FCIRC_ESIZE;
    *ws = fx->ptr;
    return FCIRC_OK;
  }
  if (bytes) {
    const fcirc_status st = ws_reserve(c, bytes);
    if (st != FCIRC_OK) return st;
  }
  *ws = c.ws;
  return FCIRC_OK;
}
fcirc_status embed_product(Ctx& c, fcirc_ring ring, const void* r, const void* col, const void* f, const void* x, void* y,
                           uint64_t n, hipStream_t s);
fcirc_status polymul_i64(Ctx& c, const int32_t* a, uint64_t na, const int32_t* b, uint64_t nb, int64_t* out, hipStream_t s);
fcirc_status bigint_mul(Ctx& c, const uint16_t* a, uint64_t na, const uint16_t* b, uint64_t nb, uint16_t* out, hipStream_t s);
void release_batches(Ctx& c);
// The batched product (fcirc_matvec_batched after validation); `force` overrides one size's
// parameters (fcirc_tune).
fcirc_status batched_product(Ctx& c, const void* a_base, const void* x_base, void* y_base, const fcirc_item* items,
                             uint32_t count, const void* f, fcirc_ring ring, hipStream_t s,
                             const BatchForce* force = nullptr);
// Whether (workgroup size bt, block levels blog) is a valid batched form of size 2^L.
bool batch_param_ok(fcirc_ring ring, int L, int bt, int blog);
// Limbs of sum_k coef[k] 2^(16 k) (coef[k] < 2^64, k < nc) into out[0, nl); u holds nl and
// summ 2 carry_blocks(nl) words of scratch.
uint64_t carry_blocks(uint64_t nl);
fcirc_status carry_to_limbs(Ctx& c, const uint64_t* coef, uint64_t nc, uint64_t nl, uint32_t* u, uint32_t* summ,
                            uint16_t* out, hipStream_t s);
fcirc_status fermat_matvec(Ctx& c, const uint32_t* a, const uint32_t* x, uint32_t* y, int L, int q, uint32_t f_exp,
                           hipStream_t s);
fcirc_status fermat_bigint_mul(Ctx& c, const uint16_t* a, uint64_t na, const uint16_t* b, uint64_t nb, uint16_t* out,
                               hipStream_t s);

// The input range check of FCIRC_CHECK_INPUTS: one launch per span of 32-bit words,
// then one synchronisation in finish(), which returns FCIRC_EINVAL if a word was >= bound.
// With the check off, every member does nothing and finish() returns FCIRC_OK.
class InputCheck {
 public:
  InputCheck(Ctx& c, uint32_t bound, hipStream_t s);
  void span(const void* words, uint64_t count);
  fcirc_status finish();

 private:
  Ctx& c_;
  uint32_t bound_;
  hipStream_t s_;
  hipError_t err_ = hipSuccess;
};

inline fcirc_status hip_status(hipError_t e) {
  if (e == hipSuccess) return FCIRC_OK;
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory ? FCIRC_ENOMEM : FCIRC_EDEVICE;
}

// Schedule for (ring, L): a forced split wins, then a tuned entry, then the defaults.
inline Schedule schedule_for(Ctx& c, int ring, int L) {
  const int elem_log = ring == FCIRC_C64 || ring == FCIRC_R32 || ring == FCIRC_GFP2 ? 3 : 2;
  TuneVal v;
  auto it = c.tuned.find(TuneKey{ring, L});
  if (it != c.tuned.end())
    v = it->second;
  else if (L >= 6 && L <= 12)
    v.flags |= FCIRC_SCHED_SMALL;  // lone small products over several waves (measured on MI355X)
  if (c.forced_top >= 0) v.top = c.forced_top;
  return make_schedule(L, elem_log, v.top, v.tile_log, v.flags);
}

}  // namespace fcirc

struct fcirc_ctx {
  fcirc::Ctx c;
};
