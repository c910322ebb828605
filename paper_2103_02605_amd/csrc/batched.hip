// Many independent f-circulant products of different power-of-two sizes in one persistent
// launch (the recursion of Algorithm 1, Rosowski arXiv 2103.02605, section 2, applied to each
// instance). The queue built for an item list is kept and reused when the same list comes
// again, so a repeated batch costs two launches (counter reset, persistent kernel).
//
// Work items, issued from one queue:
//   SPLIT  one top-split tile (row or vector) of a large instance
//   FULL   a group of small instances of one size, each a whole product (split, leaf
//          products, merge) by one group of threads of the workgroup
//   BLOCK  LDS-resident blocks of a large instance (waits for all of its SPLIT tiles)
//   MERGE  one top-merge tile of a large instance (waits for all of its BLOCK items)
// Large instances are ordered largest first and taken in groups; the queue is pipelined
// over the groups (SPLITs of one group, BLOCKs of the previous, MERGEs of the one before,
// FULL items spread between). Every item waits only for items that sit earlier in the
// queue, which some running workgroup has already taken, so waits end; each wait is also
// bounded and reports an error instead of spinning forever.
//
// Parameters by size. The workgroup size of a launch (256 or 512 threads, 16 elements per
// thread per stage) fixes the largest FULL instance and the top-pass tile (2^12 or 2^13
// elements). Per instance size, an instance is either one FULL item or takes the
// three-pass form with a block of 2^10 .. 2^(log2 threads + 4) elements (at most 6 levels
// above it). fcirc_tune measures every valid choice per size and workgroup size
// (BatchTune); a launch takes 512 threads when the measured times of its sizes favour it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <utility>
#include <vector>

#include "host.hpp"

namespace fcirc {

namespace {

constexpr uint32_t SPIN_LIMIT = 1u << 24;
// Split outputs per group of large instances in the pipelined queue (see build_and_launch).
// Measured for 4096 complex instances of 2^6..2^16 on MI355X: 2, 4, 8, 16, 32, 64 MiB and one
// group gave 1344, 1089, 922, 795, 809, 856 and 851 us per batch. Smaller groups leave the
// BLOCK items of a group waiting for its SPLIT tiles; larger ones let the intermediates
// leave the last-level cache before they are read back.
constexpr size_t GROUP_WS_BYTES = (size_t)16 << 20;

enum : uint32_t { IT_SPLIT = 0, IT_FULL = 1, IT_BLOCK = 2, IT_MERGE = 3 };

struct BItem {
  uint32_t type, L;
  uint32_t inst;  // FULL: first instance; else: instance
  uint32_t arg;   // FULL: instance count; SPLIT/MERGE: virtual workgroup; BLOCK: first block
};

struct BInst {
  uint64_t a, x, y;  // element offsets into a_base, x_base, y_base
  uint64_t ws;       // element offset of this instance's workspace (large instances)
  uint32_t L, big;   // log2 size; index among large instances (or ~0)
  uint32_t blog;     // large instances: levels of the LDS block
  uint32_t nsplit;   // large instances: SPLIT items (row and vector tiles)
  uint32_t nblock;   // large instances: BLOCK items
  uint32_t pad;
};

template <int BT>
constexpr int elog_of() {  // log2 elements held by one workgroup (16 per thread)
  return BT == 512 ? 13 : 12;
}

template <class Ring>
struct BatchArgs {
  const typename Ring::T* a;
  const typename Ring::T* x;
  typename Ring::T* y;
  typename Ring::T* ws;
  const BItem* items;
  const BInst* insts;
  uint32_t nitems;
  uint32_t* head;        // queue head
  uint32_t* cnt;         // per large instance: [2j] SPLIT items done, [2j+1] BLOCK items done
  uint32_t* status;      // sticky error bits
  typename Ring::Tw const* tw;
  typename Ring::Tw const* twi;
  typename Ring::Params rp[17];  // per log2 size (the leaf scale depends on n)
  typename Ring::DeepW const* U;  // uniform radix-16 factors (deepest-stage form): tu[15] then tui[15]
};

// Data passed between workgroups (the top-split workspace and the block results) goes
// through device-coherent accesses: relaxed agent-scope atomic loads and stores, which
// read and write at the level shared by all XCDs. With every such store coherent, a
// producer only has to wait for its stores to complete before it bumps a counter, and a
// consumer only has to read the counter; neither needs an agent-scope fence, which on
// this chip writes back or invalidates the whole L2 of an XCD.
template <class T>
struct Coh;
template <>
struct Coh<uint32_t> {
  static __device__ __forceinline__ uint32_t ld(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  static __device__ __forceinline__ void st(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};
template <>
struct Coh<float2> {
  static __device__ __forceinline__ float2 ld(const float2* p) {
    const uint64_t u = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((uint32_t)u), __uint_as_float((uint32_t)(u >> 32)));
  }
  static __device__ __forceinline__ void st(float2* p, float2 v) {
    const uint64_t u = (uint64_t)__float_as_uint(v.x) | ((uint64_t)__float_as_uint(v.y) << 32);
    __hip_atomic_store(reinterpret_cast<uint64_t*>(p), u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};

// Element access for one instance (uniform per workgroup).
template <class T>
struct LdInst {
  const T* base;
  const BInst* insts;
  int which;  // 0: a, 1: x
  template <class R>
  __device__ __forceinline__ T operator()(const R&, uint32_t inst, uint32_t i) const {
    const BInst& b = insts[inst];
    return base[(which == 0 ? b.a : b.x) + i];
  }
};
template <class T>
struct StInstY {
  T* base;
  const BInst* insts;
  __device__ __forceinline__ void operator()(uint32_t inst, uint32_t i, T v) const { base[insts[inst].y + i] = v; }
};
// One large instance's y, written by its BLOCK items and read by its MERGE items (coherent),
// or written plainly by the last merge pass.
template <class T, bool COH>
struct InstY {
  T* p;  // y of the instance
  template <class R>
  __device__ __forceinline__ T operator()(const R&, uint32_t, uint32_t i) const {
    if constexpr (COH) return Coh<T>::ld(p + i);
    else return p[i];
  }
  __device__ __forceinline__ void operator()(uint32_t, uint32_t i, T v) const {
    if constexpr (COH) Coh<T>::st(p + i, v);
    else p[i] = v;
  }
};
// Workspace of a large instance: row at [ws, ws + n), vector at [ws + n, ws + 2n) (coherent).
template <class T>
struct WsArr {
  T* p;
  template <class R>
  __device__ __forceinline__ T operator()(const R&, uint32_t, uint32_t i) const { return Coh<T>::ld(p + i); }
  __device__ __forceinline__ void operator()(uint32_t, uint32_t i, T v) const { Coh<T>::st(p + i, v); }
};
// Plain input of one instance.
template <class T>
struct InstIn {
  const T* p;
  template <class R>
  __device__ __forceinline__ T operator()(const R&, uint32_t, uint32_t i) const { return p[i]; }
};

// Counters: every thread waits for its own (coherent) stores, the workgroup meets, then one
// thread publishes with a relaxed agent-scope add. A waiter polls with relaxed loads; the
// workgroup barrier after the poll orders the item's loads after it.
// Returns false (for every thread of the workgroup) when the wait gave up; the item is then
// skipped and the launch's status gets FCIRC_STATUS_SCHED.
__device__ __forceinline__ bool wait_count(uint32_t* c, uint32_t target, uint32_t* status, uint32_t* s_ok) {
  if (threadIdx.x == 0) {
    uint32_t spins = 0, ok = 1;
    while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > SPIN_LIMIT) {
        atomicOr(status, FCIRC_STATUS_SCHED);
        ok = 0;
        break;
      }
    }
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

__device__ __forceinline__ void signal_done(uint32_t* c) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have completed
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class Ring>
__device__ __forceinline__ PassArgs<Ring> batch_pass_args(const BatchArgs<Ring>& B) {
  PassArgs<Ring> A{};
  for (int r = 0; r < 3; ++r) {
    A.tw[r] = B.tw;
    A.twi[r] = B.twi;
    A.tu[r] = B.U;
    A.tui[r] = B.U + 15;
  }
  A.narr = 1;
  A.ring_per_inst = 0;
  A.xcd = 0;
  return A;
}

template <class Ring, int L, int BT>
__device__ __forceinline__ void do_full(const BatchArgs<Ring>& B, const BItem& it, uint32_t tid, unsigned char* smem) {
  PassArgs<Ring> A = batch_pass_args(B);
  A.logn = L;
  A.d0 = 0;
  A.logr = L;
  A.logc = 0;
  A.tiles = 1;
  A.ninst = it.inst + it.arg;
  A.final_store = 1;
  const typename Ring::Params& rp = B.rp[L];
  block_pass<Ring, L, BT>(A, it.inst, tid, smem, rp, rp, rp, LdInst<typename Ring::T>{B.a, B.insts, 0},
                          LdInst<typename Ring::T>{B.x, B.insts, 1}, StInstY<typename Ring::T>{B.y, B.insts});
}

// Top passes of a large instance: R levels on tiles of 2^elog elements (one per workgroup).
template <class Ring, int R, int BT>
__device__ __forceinline__ PassArgs<Ring> top_args(const BatchArgs<Ring>& B, uint32_t L) {
  constexpr int TL = elog_of<BT>();
  PassArgs<Ring> A = batch_pass_args(B);
  A.logn = L;
  A.d0 = 0;
  A.logr = R;
  A.logc = TL - R;
  A.tiles = 1u << (L - TL);
  A.ninst = 1;
  return A;
}

template <class Ring, int R, int BT>
__device__ __forceinline__ void do_split(const BatchArgs<Ring>& B, const BItem& it, const BInst& bi, uint32_t tid,
                                         unsigned char* smem) {
  const uint32_t L = it.L;
  PassArgs<Ring> A = top_args<Ring, R, BT>(B, L);
  A.narr = 2;
  A.final_store = 0;
  TilePos P = tile_pos(A, it.arg);
  P.inst = 0;
  const Ring Rg(B.rp[L]);
  using T = typename Ring::T;
  split_pass<Ring, R>(A, P, Rg, 0, BT, tid, reinterpret_cast<T*>(smem), InstIn<T>{B.a + bi.a}, InstIn<T>{B.x + bi.x},
                      WsArr<T>{B.ws + bi.ws}, WsArr<T>{B.ws + bi.ws + (1ull << L)});
}

template <class Ring, int R, int BT>
__device__ __forceinline__ void do_merge(const BatchArgs<Ring>& B, const BItem& it, const BInst& bi, uint32_t tid,
                                         unsigned char* smem) {
  const uint32_t L = it.L;
  PassArgs<Ring> A = top_args<Ring, R, BT>(B, L);
  A.final_store = 1;
  TilePos P = tile_pos(A, it.arg);
  P.inst = 0;
  const Ring Rg(B.rp[L]);
  using T = typename Ring::T;
  T* y = B.y + bi.y;
  merge_pass<Ring, R>(A, P, Rg, 0, BT, tid, reinterpret_cast<T*>(smem), InstY<T, true>{y}, InstY<T, false>{y});
}

template <class Ring, int BLOG, int BT>
__device__ __forceinline__ void do_block(const BatchArgs<Ring>& B, const BItem& it, const BInst& bi, uint32_t tid,
                                         unsigned char* smem) {
  const uint32_t L = it.L;
  PassArgs<Ring> A = batch_pass_args(B);
  A.logn = L;
  A.d0 = L - BLOG;
  A.logr = BLOG;
  A.logc = 0;
  A.tiles = 1u << A.d0;
  A.ninst = 1;
  A.final_store = 0;
  using T = typename Ring::T;
  const typename Ring::Params& rp = B.rp[L];
  // blocks it.arg .. it.arg + GROUPS - 1 of the (single) instance
  block_pass<Ring, BLOG, BT>(A, it.arg, tid, smem, rp, rp, rp, WsArr<T>{B.ws + bi.ws}, WsArr<T>{B.ws + bi.ws + (1ull << L)},
                             InstY<T, true>{B.y + bi.y});
}

template <class Ring, int BT>
__global__ void __launch_bounds__(BT) k_batched(BatchArgs<Ring> B) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_item, s_ok;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(B.head, 1u);
    __syncthreads();
    const uint32_t id = s_item;
    __syncthreads();
    if (id >= B.nitems) break;
    const BItem it = B.items[id];
    // A fresh, opaque copy of the thread index per item: index arithmetic then stays inside
    // the item's own code path instead of being hoisted out of the loop for every path.
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    if (it.type == IT_FULL) {
      switch (it.L) {
#define FCIRC_FULL(l) \
  case l: do_full<Ring, l, BT>(B, it, tid, smem); break;
        FCIRC_FULL(0) FCIRC_FULL(1) FCIRC_FULL(2) FCIRC_FULL(3) FCIRC_FULL(4) FCIRC_FULL(5) FCIRC_FULL(6)
        FCIRC_FULL(7) FCIRC_FULL(8) FCIRC_FULL(9) FCIRC_FULL(10) FCIRC_FULL(11) FCIRC_FULL(12)
#undef FCIRC_FULL
        case 13:
          if constexpr (BT >= 512) do_full<Ring, 13, BT>(B, it, tid, smem);
          break;
        default: break;
      }
    } else {
      const BInst bi = B.insts[it.inst];
      if (it.type == IT_SPLIT) {
        switch (it.L - bi.blog) {
#define FCIRC_SPLIT(r) \
  case r: do_split<Ring, r, BT>(B, it, bi, tid, smem); break;
          FCIRC_SPLIT(1) FCIRC_SPLIT(2) FCIRC_SPLIT(3) FCIRC_SPLIT(4) FCIRC_SPLIT(5) FCIRC_SPLIT(6)
#undef FCIRC_SPLIT
          default: break;
        }
        signal_done(&B.cnt[2 * bi.big]);
      } else if (it.type == IT_BLOCK) {
        // after a failed wait the item is skipped but still counted, so that its dependents
        // do not wait out their own bound as well
        if (wait_count(&B.cnt[2 * bi.big], bi.nsplit, B.status, &s_ok)) {
          switch (bi.blog) {
            case 10: do_block<Ring, 10, BT>(B, it, bi, tid, smem); break;
            case 11: do_block<Ring, 11, BT>(B, it, bi, tid, smem); break;
            case 12: do_block<Ring, 12, BT>(B, it, bi, tid, smem); break;
            case 13:
              if constexpr (BT >= 512) do_block<Ring, 13, BT>(B, it, bi, tid, smem);
              break;
            default: break;
          }
        }
        signal_done(&B.cnt[2 * bi.big + 1]);
      } else if (wait_count(&B.cnt[2 * bi.big + 1], bi.nblock, B.status, &s_ok)) {
        switch (it.L - bi.blog) {
#define FCIRC_MERGE(r) \
  case r: do_merge<Ring, r, BT>(B, it, bi, tid, smem); break;
          FCIRC_MERGE(1) FCIRC_MERGE(2) FCIRC_MERGE(3) FCIRC_MERGE(4) FCIRC_MERGE(5) FCIRC_MERGE(6)
#undef FCIRC_MERGE
          default: break;
        }
      }
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

__global__ void k_zero(uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// LDS bytes of each item kind, by workgroup size (host side).
template <class Ring, int BT, int... Ls>
constexpr size_t block_lds_of(int l, std::integer_sequence<int, Ls...>) {
  size_t out = 0;
  ((out = Ls == l ? block_lds_bytes<Ring, Ls, BT>() : out), ...);
  return out;
}
template <class Ring, int BT>
size_t item_lds(int blog_or_L) {  // FULL of size 2^L or BLOCK of 2^blog elements
  return block_lds_of<Ring, BT>(blog_or_L, std::make_integer_sequence<int, elog_of<BT>() + 1>{});
}

}  // namespace

bool batch_param_ok(fcirc_ring ring, int L, int bt, int blog) {
  if (bt != 256 && bt != 512) return false;
  if (ring != FCIRC_C64 && (ring < FCIRC_ZP_998244353 || ring > FCIRC_ZP_167772161)) return false;
  const int elog = bt == 512 ? 13 : 12;
  if (L < 0 || L > 16) return false;
  if (blog == 0) return L <= elog;
  return blog >= 10 && blog <= elog && L > blog && L - blog <= 6 && L >= elog;
}

// One cached batched launch: the device item queue and instance table built for one item
// list, and the two launches (counter reset, persistent kernel) with their arguments.
// The twiddle tables are not part of the entry: a later product with the same f may
// rebuild them with more levels (and free the old ones), so every run takes the tables the
// context holds at that moment.
struct BatchTables {
  const void* tw;
  const void* twi;
  const void* U;
};

struct BatchEntry {
  std::vector<uint64_t> key;
  void* dev = nullptr;  // items | insts | counters
  void* ws = nullptr;
  std::function<void(hipStream_t, const BatchTables&)> run;
  ~BatchEntry() {
    if (dev) (void)hipFree(dev);
    if (ws) (void)hipFree(ws);
  }
};

void release_batches(Ctx& c) {
  for (BatchEntry* g : c.batches) delete g;
  c.batches.clear();
}

namespace {

// At most this many item lists keep their queue and workspace; the least recently used
// one is dropped (after the device has finished with it) when another is added.
constexpr size_t MAX_BATCH_ENTRIES = 16;

fcirc_status evict_batches(Ctx& c) {
  if (c.batches.size() < MAX_BATCH_ENTRIES) return FCIRC_OK;
  if (hipDeviceSynchronize() != hipSuccess) return FCIRC_EDEVICE;
  while (c.batches.size() >= MAX_BATCH_ENTRIES) {
    delete c.batches.front();
    c.batches.erase(c.batches.begin());
  }
  return FCIRC_OK;
}

// Default form of a size: FULL when it fits the workgroup, else blocks of 2^12 elements.
int default_blog(int L, int bt) { return L <= (bt == 512 ? 13 : 12) ? 0 : 12; }

// Workgroup size of a launch: 512 threads when, over the sizes whose times were measured
// (or set) for both workgroup sizes, the coefficient-weighted time favours it.
int choose_bt(const Ctx& c, fcirc_ring ring, const fcirc_item* items, uint32_t count, const BatchForce* force) {
  if (force) return force->bt;
  std::map<int, double> coefs;
  for (uint32_t i = 0; i < count; ++i) coefs[(int)items[i].log2n] += (double)(1ull << items[i].log2n);
  double t[2] = {0.0, 0.0};
  for (const auto& kv : coefs) {
    auto it = c.batch_tuned.find(TuneKey{(int)ring, kv.first});
    if (it == c.batch_tuned.end() || it->second.ns[0] < 0.f || it->second.ns[1] < 0.f) continue;
    t[0] += kv.second * it->second.ns[0];
    t[1] += kv.second * it->second.ns[1];
  }
  return t[1] < t[0] ? 512 : 256;
}

// Block levels of size 2^L in a launch of bt threads (0: FULL).
int blog_for(const Ctx& c, fcirc_ring ring, int L, int bt, const BatchForce* force) {
  if (force && force->L == L && force->bt == bt) return force->blog;
  auto it = c.batch_tuned.find(TuneKey{(int)ring, L});
  if (it != c.batch_tuned.end()) {
    const int b = it->second.blog[bt == 512 ? 1 : 0];
    if (b >= 0 && batch_param_ok(ring, L, bt, b)) return b;
  }
  return default_blog(L, bt);
}

template <class Ring, int BT>
fcirc_status build_and_launch(Ctx& c, const std::vector<uint64_t>& key, fcirc_ring ring, const void* a_base,
                              const void* x_base, void* y_base, const fcirc_item* items, uint32_t count,
                              const BatchForce* force, const BatchTables& tabs, const typename Ring::Params* rp_by_L,
                              hipStream_t s) {
  using T = typename Ring::T;
  constexpr int TL = elog_of<BT>();
  // instances sorted by size, largest first
  std::vector<uint32_t> order(count);
  for (uint32_t i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t p, uint32_t q) { return items[p].log2n > items[q].log2n; });
  int blog_by_L[17];
  for (int L = 0; L <= 16; ++L) blog_by_L[L] = blog_for(c, ring, L, BT, force);
  std::vector<BInst> insts(count);
  uint64_t ws_elems = 0;
  uint32_t nbig = 0;
  size_t lds = 0;
  for (uint32_t k = 0; k < count; ++k) {
    const fcirc_item& it = items[order[k]];
    BInst b{it.a_off, it.x_off, it.y_off, 0, it.log2n, ~0u, 0, 0, 0, 0};
    const int blog = blog_by_L[it.log2n];
    if (blog > 0) {
      b.ws = ws_elems;
      ws_elems += 2ull << it.log2n;
      b.big = nbig++;
      b.blog = (uint32_t)blog;
      b.nsplit = 2u << (it.log2n - TL);
      const uint32_t groups = (uint32_t)BT >> (blog - EPT_LOG);
      b.nblock = (1u << (it.log2n - blog)) / groups;
      lds = std::max(lds, std::max(item_lds<Ring, BT>(blog), ((size_t)1 << TL) * sizeof(T)));
    } else {
      lds = std::max(lds, item_lds<Ring, BT>((int)it.log2n));
    }
    insts[k] = b;
  }
  // FULL items: consecutive instances of equal size, as many as one workgroup holds
  std::vector<BItem> full;
  for (uint32_t k = 0; k < count;) {
    if (insts[k].big != ~0u) {
      ++k;
      continue;
    }
    const uint32_t L = insts[k].L;
    const uint32_t per = L > 4 ? (uint32_t)BT >> (L - 4) : (uint32_t)BT;
    uint32_t m = 0;
    while (k + m < count && insts[k + m].L == L && m < per) ++m;
    full.push_back(BItem{IT_FULL, L, k, m});
    k += m;
  }
  // Large instances (largest first) in groups of about GROUP_WS_BYTES of split outputs. The
  // queue is pipelined over the groups: the SPLIT tiles of group g + 1, then the BLOCK
  // items of group g, then the MERGE tiles of group g - 1, with a share of the FULL items
  // after each step. A group's intermediates are then read back soon after they are
  // written, while they are still in the last-level cache, instead of after every large
  // instance has been split. Every item still waits only for items earlier in the queue.
  std::vector<std::pair<uint32_t, uint32_t>> groups;  // [first, last) instance ranges
  for (uint32_t k = 0; k < count;) {
    if (insts[k].big == ~0u) {
      ++k;
      continue;
    }
    uint32_t e = k;
    size_t bytes = 0;
    while (e < count && insts[e].big != ~0u && (e == k || bytes + (sizeof(T) << (insts[e].L + 1)) <= GROUP_WS_BYTES)) {
      bytes += sizeof(T) << (insts[e].L + 1);
      ++e;
    }
    groups.emplace_back(k, e);
    k = e;
  }
  const size_t ng = groups.size(), nsteps = ng + 2;
  std::vector<BItem> q;
  size_t fi = 0;
  for (size_t step = 0; step < nsteps; ++step) {
    if (step < ng)
      for (uint32_t k = groups[step].first; k < groups[step].second; ++k)
        for (uint32_t v = 0; v < insts[k].nsplit; ++v) q.push_back(BItem{IT_SPLIT, insts[k].L, k, v});
    if (step >= 1 && step - 1 < ng)
      for (uint32_t k = groups[step - 1].first; k < groups[step - 1].second; ++k) {
        const uint32_t gpb = (uint32_t)BT >> (insts[k].blog - EPT_LOG);
        for (uint32_t b = 0; b < insts[k].nblock; ++b) q.push_back(BItem{IT_BLOCK, insts[k].L, k, b * gpb});
      }
    if (step >= 2)
      for (uint32_t k = groups[step - 2].first; k < groups[step - 2].second; ++k)
        for (uint32_t v = 0; v < insts[k].nsplit / 2; ++v) q.push_back(BItem{IT_MERGE, insts[k].L, k, v});
    const size_t fe = full.size() * (step + 1) / nsteps;
    q.insert(q.end(), full.begin() + fi, full.begin() + fe);
    fi = fe;
  }

  BatchEntry* g = new BatchEntry;
  g->key = key;
  const size_t items_b = q.size() * sizeof(BItem), insts_b = insts.size() * sizeof(BInst);
  const uint32_t ncnt = 1 + 2 * nbig;  // head + counters
  const size_t off_insts = (items_b + 255) & ~(size_t)255, off_cnt = (off_insts + insts_b + 255) & ~(size_t)255;
  if (hipMalloc(&g->dev, off_cnt + ncnt * sizeof(uint32_t)) != hipSuccess ||
      (ws_elems && hipMalloc(&g->ws, ws_elems * sizeof(T)) != hipSuccess)) {
    (void)hipGetLastError();
    delete g;
    return FCIRC_ENOMEM;
  }
  char* dev = (char*)g->dev;
  if (hipMemcpy(dev, q.data(), items_b, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dev + off_insts, insts.data(), insts_b, hipMemcpyHostToDevice) != hipSuccess) {
    delete g;
    return FCIRC_EDEVICE;
  }
  BatchArgs<Ring> B{};
  B.a = (const T*)a_base;
  B.x = (const T*)x_base;
  B.y = (T*)y_base;
  B.ws = (T*)g->ws;
  B.items = (const BItem*)dev;
  B.insts = (const BInst*)(dev + off_insts);
  B.nitems = (uint32_t)q.size();
  B.head = (uint32_t*)(dev + off_cnt);
  B.cnt = B.head + 1;
  B.status = c.d_status;
  for (int L = 0; L <= 16; ++L) B.rp[L] = rp_by_L[L];
  auto kb = k_batched<Ring, BT>;
  allow_lds(kb, lds);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kb, BT, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  const uint32_t grid = (uint32_t)std::min<size_t>((size_t)per_cu * c.prop.multiProcessorCount, q.size());

  const uint32_t* head = B.head;
  g->run = [B, kb, grid, lds, head, ncnt](hipStream_t st, const BatchTables& t) {
    BatchArgs<Ring> Bt = B;
    Bt.tw = static_cast<typename Ring::Tw const*>(t.tw);
    Bt.twi = static_cast<typename Ring::Tw const*>(t.twi);
    Bt.U = static_cast<typename Ring::DeepW const*>(t.U);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, st, const_cast<uint32_t*>(head), ncnt);
    hipLaunchKernelGGL(kb, dim3(grid), dim3(BT), lds, st, Bt);
  };
  c.batches.push_back(g);
  return hip_status(launch(c, "fcirc_batched", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    if (e0_) (void)hipEventRecord(e0_, s);
    g->run(s, tabs);
    if (e1_) (void)hipEventRecord(e1_, s);
  }));
}

// Reuse the cached queue of this key, or build one for the workgroup size chosen.
template <class Ring>
fcirc_status launch_batched(Ctx& c, std::vector<uint64_t>& key, fcirc_ring ring, const void* a_base, const void* x_base,
                            void* y_base, const fcirc_item* items, uint32_t count, const BatchForce* force,
                            const BatchTables& tabs, const typename Ring::Params* rp_by_L, hipStream_t s) {
  // the parameters in force are part of the key: a queue built under others is not reused
  key.push_back(c.batch_gen);
  key.push_back(force ? ((uint64_t)force->L << 32 | (uint64_t)force->bt << 8 | (uint64_t)force->blog) : ~0ull);
  for (size_t i = 0; i < c.batches.size(); ++i)
    if (c.batches[i]->key == key) {
      BatchEntry* g = c.batches[i];
      c.batches.erase(c.batches.begin() + i);  // most recently used last
      c.batches.push_back(g);
      return hip_status(launch(c, "fcirc_batched", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
        if (e0_) (void)hipEventRecord(e0_, s);
        g->run(s, tabs);
        if (e1_) (void)hipEventRecord(e1_, s);
      }));
    }
  if (fcirc_status st = evict_batches(c); st != FCIRC_OK) return st;
  if (choose_bt(c, ring, items, count, force) == 512)
    return build_and_launch<Ring, 512>(c, key, ring, a_base, x_base, y_base, items, count, force, tabs, rp_by_L, s);
  return build_and_launch<Ring, 256>(c, key, ring, a_base, x_base, y_base, items, count, force, tabs, rp_by_L, s);
}

}  // namespace

fcirc_status batched_product(Ctx& c, const void* a_base, const void* x_base, void* y_base, const fcirc_item* items,
                             uint32_t count, const void* f, fcirc_ring ring, hipStream_t s, const BatchForce* force) {
  uint32_t maxL = 0;
  for (uint32_t i = 0; i < count; ++i) maxL = std::max(maxL, items[i].log2n);
  // key: ring, f, base pointers and the whole item list
  std::vector<uint64_t> key;
  key.reserve(10 + 4 * (size_t)count);
  key.push_back((uint64_t)ring);
  if (ring == FCIRC_C64) {
    uint64_t w[2];
    std::memcpy(w, f, 16);
    key.push_back(w[0]);
    key.push_back(w[1]);
  } else {
    key.push_back(*(const uint32_t*)f);
  }
  key.push_back((uint64_t)(uintptr_t)a_base);
  key.push_back((uint64_t)(uintptr_t)x_base);
  key.push_back((uint64_t)(uintptr_t)y_base);
  for (uint32_t i = 0; i < count; ++i) {
    key.push_back(items[i].a_off);
    key.push_back(items[i].x_off);
    key.push_back(items[i].y_off);
    key.push_back(items[i].log2n);
  }
  if (ring == FCIRC_C64) {
    const double* fc = (const double*)f;
    const C32Tables* T = nullptr;
    fcirc_status st = c32_tables(c, fc[0], fc[1], (int)std::max<uint32_t>(maxL, 1), s, &T);
    if (st != FCIRC_OK) return st;
    C32Params rp[17];
    for (int L = 0; L <= 16; ++L) rp[L] = C32Params{(float)std::ldexp(1.0, -L)};
    return launch_batched<C32>(c, key, ring, a_base, x_base, y_base, items, count, force,
                               BatchTables{T->tw, T->twi, T->dU}, rp, s);
  }
  const uint32_t p = zp_prime(ring), fv = *(const uint32_t*)f;
  const ZpTables* T = nullptr;
  fcirc_status st = zp_tables(c, p, fv, (int)std::max<uint32_t>(maxL, 1), &T);
  if (st != FCIRC_OK) return st;
  ZpParams rp[17];
  for (int L = 0; L <= 16; ++L) rp[L] = zp_params(p, L);
  return launch_batched<Zp>(c, key, ring, a_base, x_base, y_base, items, count, force, BatchTables{T->tw, T->twi, T->dU},
                            rp, s);
}

}  // namespace fcirc

using namespace fcirc;

namespace {

// FCIRC_CHECK_INPUTS over the union of the instances' input spans (instances may share
// or overlap inputs; gaps between them are not inputs and are not checked).
fcirc_status check_batched_inputs(Ctx& c, const void* a_base, const void* x_base, const fcirc_item* items,
                                  uint32_t count, uint32_t p, hipStream_t s) {
  InputCheck chk(c, p, s);
  std::vector<std::pair<uint64_t, uint64_t>> iv(count);
  for (int side = 0; side < 2; ++side) {
    for (uint32_t i = 0; i < count; ++i) {
      const uint64_t off = side ? items[i].x_off : items[i].a_off;
      iv[i] = {off, off + (1ull << items[i].log2n)};
    }
    std::sort(iv.begin(), iv.end());
    const uint32_t* base = (const uint32_t*)(side ? x_base : a_base);
    uint64_t lo = iv[0].first, hi = iv[0].second;
    for (size_t i = 1; i <= iv.size(); ++i) {
      if (i < iv.size() && iv[i].first <= hi) {
        hi = std::max(hi, iv[i].second);
        continue;
      }
      chk.span(base + lo, hi - lo);
      if (i < iv.size()) lo = iv[i].first, hi = iv[i].second;
    }
  }
  return chk.finish();
}

bool batch_ring(fcirc_ring ring) { return ring == FCIRC_C64 || (ring >= FCIRC_ZP_998244353 && ring <= FCIRC_ZP_167772161); }

}  // namespace

extern "C" fcirc_status fcirc_matvec_batched(fcirc_ctx* ctx, const void* a_base, const void* x_base, void* y_base,
                                             const fcirc_item* items, uint32_t count, const void* f, fcirc_ring ring,
                                             void* stream) {
  if (!ctx || !a_base || !x_base || !y_base || !items || !f) return FCIRC_EINVAL;
  if (!batch_ring(ring)) return FCIRC_EINVAL;
  if (count == 0) return FCIRC_OK;
  for (uint32_t i = 0; i < count; ++i)
    if (items[i].reserved != 0 || items[i].log2n > 16) return items[i].log2n > 16 ? FCIRC_ESIZE : FCIRC_EINVAL;
  if (ring != FCIRC_C64 && *(const uint32_t*)f >= zp_prime(ring)) return FCIRC_EINVAL;
  Ctx& c = ctx->c;
  if (hipSetDevice(c.device) != hipSuccess) return FCIRC_EDEVICE;
  hipStream_t s = (hipStream_t)stream;
  if (ring != FCIRC_C64 && c.check_inputs) {
    fcirc_status st = check_batched_inputs(c, a_base, x_base, items, count, zp_prime(ring), s);
    if (st != FCIRC_OK) return st;
  }
  return batched_product(c, a_base, x_base, y_base, items, count, f, ring, s);
}

extern "C" fcirc_status fcirc_set_batch_schedule(fcirc_ctx* ctx, fcirc_ring ring, uint64_t n, int workgroup,
                                                 int block_levels) {
  if (!ctx || !batch_ring(ring) || n == 0 || (n & (n - 1)) || n > (1u << 16)) return FCIRC_EINVAL;
  const int L = ilog2(n);
  Ctx& c = ctx->c;
  if (workgroup == -1) {
    c.batch_tuned.erase(TuneKey{(int)ring, L});
  } else {
    if (!batch_param_ok(ring, L, workgroup, block_levels)) return FCIRC_EINVAL;
    // counts as measured: this workgroup size fastest, the other not to be taken
    BatchTune t;
    const int w = workgroup == 512 ? 1 : 0;
    t.blog[w] = block_levels;
    t.ns[w] = 0.f;
    t.blog[1 - w] = default_blog(L, w ? 256 : 512);
    t.ns[1 - w] = 1e30f;
    c.batch_tuned[TuneKey{(int)ring, L}] = t;
  }
  ++c.batch_gen;
  return FCIRC_OK;
}

extern "C" int fcirc_get_batch_schedule(fcirc_ctx* ctx, fcirc_ring ring, uint64_t n, int* workgroup, int* block_levels) {
  if (!ctx || !batch_ring(ring) || n == 0 || (n & (n - 1)) || n > (1u << 16)) return -1;
  const int L = ilog2(n);
  fcirc_item it{0, 0, 0, (uint32_t)L, 0};
  const int bt = choose_bt(ctx->c, ring, &it, 1, nullptr);
  if (workgroup) *workgroup = bt;
  if (block_levels) *block_levels = blog_for(ctx->c, ring, L, bt, nullptr);
  return 0;
}
