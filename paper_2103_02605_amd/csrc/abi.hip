// C-ABI of libfcirc: argument validation, context management, dispatch.
// The operations are defined in include/fcirc.h; validation happens on the host before
// anything is enqueued, so an error return means nothing was written.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>

#include "host.hpp"

using namespace fcirc;

namespace fcirc {
// Schedules from a file written by fcirc_save_schedules (tune.hip; FCIRC_EINVAL, nothing
// changed, if the file is unreadable or malformed).
fcirc_status load_schedules(Ctx& c, const char* path);
}  // namespace fcirc


namespace {

bool is_pow2(uint64_t n) { return n && !(n & (n - 1)); }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

size_t elem_bytes(fcirc_ring r) {
  switch (r) {
    case FCIRC_C64: return 8;
    case FCIRC_GFP2: return 8;
    case FCIRC_R32: return 4;
    default: return 4;
  }
}

bool known_ring(int r) { return r >= FCIRC_ZP_998244353 && r <= FCIRC_GFP2; }

// FCIRC_CHECK_INPUTS for a Z/p or GF(p^2) call: every 32-bit word of each buffer (`words`
// of them) must lie in [0,p). Floating-point rings have no canonical form to check.
fcirc_status check_inputs(Ctx& c, fcirc_ring ring, std::initializer_list<const void*> bufs, uint64_t words,
                          hipStream_t s) {
  if (!c.check_inputs || ring == FCIRC_C64 || ring == FCIRC_R32) return FCIRC_OK;
  InputCheck chk(c, ring == FCIRC_GFP2 ? 0x7fffffffu : zp_prime(ring), s);
  for (const void* b : bufs) chk.span(b, words);
  return chk.finish();
}

uint64_t words_per_elem(fcirc_ring ring) { return ring == FCIRC_GFP2 ? 2 : 1; }

// Common checks of a product of `count` instances of size n. Returns FCIRC_OK and L.
fcirc_status check_product(fcirc_ctx* ctx, const void* a, const void* x, const void* y, uint64_t n, uint64_t count,
                           const void* f, fcirc_ring ring, int* L) {
  if (!ctx || !a || !x || !y || !f || !known_ring(ring)) return FCIRC_EINVAL;
  if (!is_pow2(n)) return FCIRC_ESIZE;
  const int l = ilog2(n);
  if (ring <= FCIRC_ZP_167772161) {
    const uint32_t p = zp_prime(ring);
    if (l > zp_two_adic(p)) return FCIRC_ESIZE;
    const uint32_t fv = *(const uint32_t*)f;
    if (fv >= p) return FCIRC_EINVAL;
    if (fv == 0) return FCIRC_ENOROOT;
  } else if (ring == FCIRC_GFP2) {
    if (l > 26) return FCIRC_ESIZE;
    const uint32_t* fv = (const uint32_t*)f;
    if (fv[0] > 0x7ffffffeu || fv[1] > 0x7ffffffeu) return FCIRC_EINVAL;
    if (fv[1] != 0 || (fv[0] != 1 && fv[0] != 0x7ffffffeu)) return FCIRC_ENOROOT;  // f = 1 or -1
  } else {
    if (l > 26) return FCIRC_ESIZE;
    if (ring == FCIRC_C64) {
      const double* fc = (const double*)f;
      if (fc[0] == 0.0 && fc[1] == 0.0) return FCIRC_ENOROOT;
    } else if (*(const double*)f == 0.0) {
      return FCIRC_ENOROOT;
    }
  }
  const size_t bytes = (size_t)n * count * elem_bytes(ring);
  if (overlaps(y, bytes, a, bytes) || overlaps(y, bytes, x, bytes)) return FCIRC_EINVAL;
  *L = l;
  return FCIRC_OK;
}

fcirc_status dispatch(fcirc_ctx* ctx, const void* a, const void* x, void* y, int L, uint32_t count, const void* f,
                      fcirc_ring ring, hipStream_t s, const FixedWs* fx = nullptr) {
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  if (ring <= FCIRC_ZP_167772161)
    return zp_matvec(ctx->c, (const uint32_t*)a, (const uint32_t*)x, (uint32_t*)y, L, count, zp_prime(ring),
                     *(const uint32_t*)f, s, fx);
  if (ring == FCIRC_C64) {
    const double* fc = (const double*)f;
    return c32_matvec(ctx->c, a, x, y, L, count, fc[0], fc[1], false, s, fx);
  }
  if (ring == FCIRC_GFP2) return gp2_matvec(ctx->c, a, x, y, L, count, ((const uint32_t*)f)[0] != 1, s, fx);
  return c32_matvec(ctx->c, a, x, y, L, count, *(const double*)f, 0.0, true, s, fx);
}

// Workspace of fcirc_matvec_noalloc: one array per GPU, alive until the process ends. In
// host code `scratch` names a host-side stand-in, not device memory; its device address is
// taken once per context (hipGetSymbolAddress, with the context's device current) in
// fcirc_create and kept in Ctx::scratch, which is what kernels receive.
static __device__ __align__(256) unsigned char scratch[FCIRC_NOALLOC_SCRATCH_BYTES];

}  // namespace

namespace fcirc {

// Sets *flag when a word of v[0, count) is >= bound. Global atomics only (vector memory).
__global__ __launch_bounds__(256) void k_input_check(const uint32_t* __restrict__ v, uint64_t count, uint32_t bound,
                                                     uint32_t* flag) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  bool bad = false;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < count; i += stride) bad |= v[i] >= bound;
  if (bad) atomicOr(flag, 1u);
}

InputCheck::InputCheck(Ctx& c, uint32_t bound, hipStream_t s) : c_(c), bound_(bound), s_(s) {
  if (c_.check_inputs) err_ = hipMemsetAsync(c_.d_status + 1, 0, sizeof(uint32_t), s_);
}

void InputCheck::span(const void* words, uint64_t count) {
  if (!c_.check_inputs || err_ != hipSuccess || count == 0) return;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((count + 255) / 256, 4096);
  const uint32_t* v = (const uint32_t*)words;
  uint32_t* flag = c_.d_status + 1;
  const uint32_t bound = bound_;
  err_ = launch(c_, "fcirc_input_check", s_, [&](hipEvent_t e0, hipEvent_t e1) {
    FCIRC_LAUNCH(e0, e1, k_input_check, dim3(grid), dim3(256), 0, s_, v, count, bound, flag);
  });
}

fcirc_status InputCheck::finish() {
  if (!c_.check_inputs) return FCIRC_OK;
  uint32_t bad = 0;
  if (err_ == hipSuccess) err_ = hipMemcpyAsync(&bad, c_.d_status + 1, sizeof bad, hipMemcpyDeviceToHost, s_);
  if (err_ == hipSuccess) err_ = hipStreamSynchronize(s_);
  if (err_ != hipSuccess) return hip_status(err_);
  return bad ? FCIRC_EINVAL : FCIRC_OK;
}

}  // namespace fcirc

extern "C" {

const char* fcirc_strerror(fcirc_status s) {
  switch (s) {
    case FCIRC_OK: return "ok";
    case FCIRC_EINVAL: return "invalid argument";
    case FCIRC_ESIZE: return "size not a power of two or above the ring's limit";
    case FCIRC_ENOROOT: return "f has no n-th root in the ring (or f is zero)";
    case FCIRC_ERANGE: return "a result coefficient is outside the exactly representable range";
    case FCIRC_ENOMEM: return "device memory allocation failed or exceeded the workspace limit";
    case FCIRC_EDEVICE: return "no usable gfx950 device, or a HIP call failed";
    case FCIRC_ESCHED: return "a batched launch gave up waiting for an earlier work item; its outputs are unspecified";
    case FCIRC_ENOPLAN: return "the twiddle tables of this (ring, f, n) are not resident and this call may not build them";
  }
  return "unknown status";
}

fcirc_status fcirc_create(fcirc_ctx** out, int dev) {
  if (!out) return FCIRC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || dev < 0 || dev >= ndev) {
    (void)hipGetLastError();
    return FCIRC_EDEVICE;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return FCIRC_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FCIRC_EDEVICE;
  if (hipSetDevice(dev) != hipSuccess) return FCIRC_EDEVICE;
  fcirc_ctx* ctx = new fcirc_ctx;
  ctx->c.device = dev;
  ctx->c.prop = prop;
  if (const char* lim = std::getenv("FCIRC_WORKSPACE_LIMIT")) ctx->c.ws_limit = (size_t)std::strtoull(lim, nullptr, 10);
  if (const char* dbg = std::getenv("FCIRC_DEBUG_SYNC")) ctx->c.debug_sync = dbg[0] == '1';
  if (const char* val = std::getenv("FCIRC_VALIDATE")) ctx->c.check_inputs = val[0] == '1';
  if (hipMalloc(&ctx->c.d_status, 2 * sizeof(uint32_t)) != hipSuccess ||
      hipMemset(ctx->c.d_status, 0, 2 * sizeof(uint32_t)) != hipSuccess) {
    delete ctx;
    return FCIRC_EDEVICE;
  }
  // this device's copy of the no-alloc workspace (the device is current)
  void* sp = nullptr;
  if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || sp == nullptr) {
    (void)hipGetLastError();
    (void)hipFree(ctx->c.d_status);
    delete ctx;
    return FCIRC_EDEVICE;
  }
  ctx->c.scratch = sp;
  if (const char* tf = std::getenv("FCIRC_TUNE_FILE")) {
    if (load_schedules(ctx->c, tf) != FCIRC_OK)
      std::fprintf(stderr, "libfcirc: FCIRC_TUNE_FILE=%s could not be read; default schedules kept\n", tf);
  }
  *out = ctx;
  return FCIRC_OK;
}

void fcirc_destroy(fcirc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->c.device);
  (void)hipDeviceSynchronize();
  for (auto& t : ctx->c.zp) {
    (void)hipFree(t.tw);
    (void)hipFree(t.twi);
    (void)hipFree(t.dU);
    for (int L = 0; L < 27; ++L) {
      if (t.ft[L]) (void)hipFree(t.ft[L]);
      if (t.fti[L]) (void)hipFree(t.fti[L]);
    }
  }
  for (auto& t : ctx->c.c32) {
    (void)hipFree(t.tw);
    (void)hipFree(t.twi);
    (void)hipFree(t.dU);
  }
  for (auto& t : ctx->c.gp2) {
    (void)hipFree(t.tw);
    (void)hipFree(t.twi);
    (void)hipFree(t.dU);
  }
  release_batches(ctx->c);
  if (ctx->c.ws) (void)hipFree(ctx->c.ws);
  if (ctx->c.ws2) (void)hipFree(ctx->c.ws2);
  if (ctx->c.d_status) (void)hipFree(ctx->c.d_status);
  delete ctx;
}

fcirc_status fcirc_matvec(fcirc_ctx* ctx, const void* a, const void* x, void* y, uint64_t n, const void* f,
                          fcirc_ring ring, void* stream) {
  int L = 0;
  fcirc_status st = check_product(ctx, a, x, y, n, 1, f, ring, &L);
  if (st != FCIRC_OK) return st;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  st = check_inputs(ctx->c, ring, {a, x}, n * words_per_elem(ring), (hipStream_t)stream);
  if (st != FCIRC_OK) return st;
  return dispatch(ctx, a, x, y, L, 1, f, ring, (hipStream_t)stream);
}

fcirc_status fcirc_matvec_noalloc(fcirc_ctx* ctx, const void* a, const void* x, void* y, uint64_t n, const void* f,
                                  fcirc_ring ring, void* stream) {
  int L = 0;
  fcirc_status st = check_product(ctx, a, x, y, n, 1, f, ring, &L);
  if (st != FCIRC_OK) return st;
  // the product's workspace: 2n elements (3n for real data) once it has top passes
  const uint64_t per = ring == FCIRC_R32 ? 3 * sizeof(float2) : 2 * elem_bytes(ring);
  if (L > 12 && n * per > FCIRC_NOALLOC_SCRATCH_BYTES) return FCIRC_ESIZE;
  if (!ctx->c.scratch) return FCIRC_EDEVICE;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  st = check_inputs(ctx->c, ring, {a, x}, n * words_per_elem(ring), (hipStream_t)stream);
  if (st != FCIRC_OK) return st;
  const FixedWs fx{ctx->c.scratch, FCIRC_NOALLOC_SCRATCH_BYTES};
  return dispatch(ctx, a, x, y, L, 1, f, ring, (hipStream_t)stream, &fx);
}

fcirc_status fcirc_matvec_many(fcirc_ctx* ctx, const void* a, const void* x, void* y, uint64_t n, uint32_t count,
                               const void* f, fcirc_ring ring, void* stream) {
  if (count == 0) return ctx && a && x && y && f ? FCIRC_OK : FCIRC_EINVAL;
  int L = 0;
  fcirc_status st = check_product(ctx, a, x, y, n, count, f, ring, &L);
  if (st != FCIRC_OK) return st;
  if ((uint64_t)count * (n >> 12 ? (n >> 12) : 1) * 2 > 0x7fffffffull) return FCIRC_ESIZE;  // grid limit
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  st = check_inputs(ctx->c, ring, {a, x}, n * count * words_per_elem(ring), (hipStream_t)stream);
  if (st != FCIRC_OK) return st;
  return dispatch(ctx, a, x, y, L, count, f, ring, (hipStream_t)stream);
}

// Shared validation of the embedded products: size limit of the cyclic length, f range.
static fcirc_status check_embed(fcirc_ctx* ctx, const void* a, const void* x, const void* y, uint64_t n, const void* f,
                                fcirc_ring ring) {
  if (!ctx || !a || !x || !y || !known_ring(ring) || ring == FCIRC_GFP2) return FCIRC_EINVAL;
  if (n == 0 || n > (1ull << 25)) return FCIRC_ESIZE;
  int L = 0;
  while ((1ull << L) < 2 * n - 1) ++L;
  if (ring <= FCIRC_ZP_167772161) {
    const uint32_t p = zp_prime(ring);
    if (L > zp_two_adic(p)) return FCIRC_ESIZE;
    if (f && *(const uint32_t*)f >= p) return FCIRC_EINVAL;
  } else if (L > 26) {
    return FCIRC_ESIZE;
  }
  const size_t bytes = (size_t)n * elem_bytes(ring);
  if (overlaps(y, bytes, a, bytes) || overlaps(y, bytes, x, bytes)) return FCIRC_EINVAL;
  return FCIRC_OK;
}

fcirc_status fcirc_matvec_any(fcirc_ctx* ctx, const void* a, const void* x, void* y, uint64_t n, const void* f,
                              fcirc_ring ring, void* stream) {
  if (!f) return FCIRC_EINVAL;
  fcirc_status st = check_embed(ctx, a, x, y, n, f, ring);
  if (st != FCIRC_OK) return st;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  st = check_inputs(ctx->c, ring, {a, x}, n, (hipStream_t)stream);
  if (st != FCIRC_OK) return st;
  int L = 0;
  if (is_pow2(n) && check_product(ctx, a, x, y, n, 1, f, ring, &L) == FCIRC_OK) {
    st = dispatch(ctx, a, x, y, L, 1, f, ring, (hipStream_t)stream);
    if (st != FCIRC_ENOROOT) return st;  // f without the needed root: embed instead
  }
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  return embed_product(ctx->c, ring, a, nullptr, f, x, y, n, (hipStream_t)stream);
}

fcirc_status fcirc_toeplitz_matvec(fcirc_ctx* ctx, const void* row, const void* col, const void* x, void* y, uint64_t n,
                                   fcirc_ring ring, void* stream) {
  if (!col) return FCIRC_EINVAL;
  fcirc_status st = check_embed(ctx, row, x, y, n, nullptr, ring);
  if (st != FCIRC_OK) return st;
  if (overlaps(y, (size_t)n * elem_bytes(ring), col, (size_t)n * elem_bytes(ring))) return FCIRC_EINVAL;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  st = check_inputs(ctx->c, ring, {row, col, x}, n, (hipStream_t)stream);
  if (st != FCIRC_OK) return st;
  return embed_product(ctx->c, ring, row, col, nullptr, x, y, n, (hipStream_t)stream);
}

fcirc_status fcirc_polymul_i64(fcirc_ctx* ctx, const int32_t* a, uint64_t na, const int32_t* b, uint64_t nb, int64_t* c,
                               void* stream) {
  if (!ctx || !a || !b || !c || na == 0 || nb == 0) return FCIRC_EINVAL;
  const uint64_t nc = na + nb - 1;
  if (nc > (1ull << 23)) return FCIRC_ESIZE;
  if (overlaps(c, nc * 8, a, na * 4) || overlaps(c, nc * 8, b, nb * 4)) return FCIRC_EINVAL;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  return polymul_i64(ctx->c, a, na, b, nb, c, (hipStream_t)stream);
}

fcirc_status fcirc_bigint_mul(fcirc_ctx* ctx, const uint16_t* a, uint64_t na, const uint16_t* b, uint64_t nb, uint16_t* c,
                              void* stream) {
  if (!ctx || !a || !b || !c || na == 0 || nb == 0) return FCIRC_EINVAL;
  const uint64_t nc = na + nb - 1;
  if (nc > (1ull << 23) || (na < nb ? na : nb) > (1ull << 20)) return FCIRC_ESIZE;
  if (overlaps(c, (nc + 1) * 2, a, na * 2) || overlaps(c, (nc + 1) * 2, b, nb * 2)) return FCIRC_EINVAL;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  return bigint_mul(ctx->c, a, na, b, nb, c, (hipStream_t)stream);
}

fcirc_status fcirc_fermat_matvec(fcirc_ctx* ctx, const uint32_t* a, const uint32_t* x, uint32_t* y, uint64_t n,
                                 uint32_t K, uint32_t f_shift, void* stream) {
  if (!ctx || !a || !x || !y) return FCIRC_EINVAL;
  if (K != 2048 && K != 4096 && K != 8192 && K != 16384) return FCIRC_EINVAL;
  if (f_shift >= 2 * K) return FCIRC_EINVAL;
  if (!is_pow2(n)) return FCIRC_ESIZE;
  const int L = ilog2(n);
  if (L >= 1 && (K & ((1u << (L - 1)) - 1)) != 0) return FCIRC_ESIZE;  // 2^(L-1) | K
  if (L >= 1 && (f_shift & ((1u << L) - 1)) != 0) return FCIRC_ENOROOT;
  const size_t bytes = (size_t)n * (K / 32 + 1) * 4;
  if (overlaps(y, bytes, a, bytes) || overlaps(y, bytes, x, bytes)) return FCIRC_EINVAL;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  return fermat_matvec(ctx->c, a, x, y, L, (int)(K / 2048), f_shift, (hipStream_t)stream);
}

fcirc_status fcirc_bigint_mul_fermat(fcirc_ctx* ctx, const uint16_t* a, uint64_t na, const uint16_t* b, uint64_t nb,
                                     uint16_t* c, void* stream) {
  if (!ctx || !a || !b || !c || na == 0 || nb == 0) return FCIRC_EINVAL;
  const uint64_t nc = na + nb - 1;
  if (nc > (1ull << 24)) return FCIRC_ESIZE;
  if (overlaps(c, (nc + 1) * 2, a, na * 2) || overlaps(c, (nc + 1) * 2, b, nb * 2)) return FCIRC_EINVAL;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  return fermat_bigint_mul(ctx->c, a, na, b, nb, c, (hipStream_t)stream);
}

fcirc_status fcirc_check(fcirc_ctx* ctx, void* stream) {
  if (!ctx) return FCIRC_EINVAL;
  if (hipSetDevice(ctx->c.device) != hipSuccess) return FCIRC_EDEVICE;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return hip_status(hipGetLastError());
  uint32_t st = 0;
  if (hipMemcpy(&st, ctx->c.d_status, sizeof st, hipMemcpyDeviceToHost) != hipSuccess) return FCIRC_EDEVICE;
  if (st) {
    if (hipMemset(ctx->c.d_status, 0, sizeof(uint32_t)) != hipSuccess) return FCIRC_EDEVICE;
    // a scheduling failure makes every output of its launch unspecified: report it first
    return (st & FCIRC_STATUS_SCHED) ? FCIRC_ESCHED : FCIRC_ERANGE;
  }
  return FCIRC_OK;
}

fcirc_status fcirc_set_checks(fcirc_ctx* ctx, int flags) {
  if (!ctx || (flags & ~(FCIRC_CHECK_INPUTS | FCIRC_CHECK_SYNC))) return FCIRC_EINVAL;
  ctx->c.check_inputs = (flags & FCIRC_CHECK_INPUTS) != 0;
  ctx->c.debug_sync = (flags & FCIRC_CHECK_SYNC) != 0;
  return FCIRC_OK;
}

fcirc_status fcirc_set_timing(fcirc_ctx* ctx, int enable) {
  if (!ctx) return FCIRC_EINVAL;
  ctx->c.timer.collect();
  ctx->c.timer.enabled = enable != 0;
  for (auto& v : ctx->c.timer.launches) v = 0;
  for (auto& v : ctx->c.timer.ms) v = 0.0;
  return FCIRC_OK;
}

int fcirc_stage_times(fcirc_ctx* ctx, const char** names, uint64_t* launches, double* ms, int max) {
  if (!ctx) return -1;
  ctx->c.timer.collect();
  const int n = (int)ctx->c.timer.names.size();
  for (int i = 0; i < n && i < max; ++i) {
    if (names) names[i] = ctx->c.timer.names[i].c_str();
    if (launches) launches[i] = ctx->c.timer.launches[i];
    if (ms) ms[i] = ctx->c.timer.ms[i];
  }
  return n;
}

fcirc_status fcirc_set_split(fcirc_ctx* ctx, int top_levels) {
  if (!ctx || top_levels < -1 || top_levels > 26) return FCIRC_EINVAL;
  ctx->c.forced_top = top_levels;
  return FCIRC_OK;
}

int fcirc_get_split(fcirc_ctx* ctx, uint64_t n, fcirc_ring ring) {
  if (!ctx || !is_pow2(n) || !known_ring(ring)) return -1;
  const Schedule S = schedule_for(ctx->c, ring, ilog2(n));
  return S.L - S.block_levels;
}

}  // extern "C"
