// Autotuner for the pass schedule of one (ring, n): how many top levels are streamed
// through HBM before the LDS-resident block pass, how large a top-pass tile is, and
// the top-pass flags (XCD-aware tile order; row and vector split jointly or in separate
// workgroups). Every candidate is timed with HIP
// events on the caller's stream over scratch buffers; the fastest is kept in the context.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "host.hpp"

using namespace fcirc;


namespace {

fcirc_status run_once(Ctx& c, fcirc_ring ring, int L, void* a, void* x, void* y, hipStream_t s) {
  if (ring <= FCIRC_ZP_167772161)
    return zp_matvec(c, (const uint32_t*)a, (const uint32_t*)x, (uint32_t*)y, L, 1, zp_prime(ring), 1u, s);
  if (ring == FCIRC_GFP2) return gp2_matvec(c, a, x, y, L, 1, 0, s);
  return c32_matvec(c, a, x, y, L, 1, 1.0, 0.0, ring == FCIRC_R32, s);
}

// Batched-launch parameters for instances of size 2^L: for each workgroup size, every valid
// form (one FULL item, or the three-pass form with blocks of 2^10 .. 2^13 elements) is timed
// on a scratch batch of max(1, 2^24 / 2^L) instances (at most 4096), and the fastest kept
// with its time per coefficient.
fcirc_status tune_batched(Ctx& c, fcirc_ring ring, int L, hipStream_t s) {
  const uint64_t n = 1ull << L;
  const uint32_t count = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(4096, (1ull << 24) >> L));
  const size_t eb = ring == FCIRC_C64 ? 8 : 4;
  const size_t bytes = (size_t)count * n * eb;
  void *a = nullptr, *x = nullptr, *y = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&x, bytes) != hipSuccess || hipMalloc(&y, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipFree(a);
    if (x) (void)hipFree(x);
    return FCIRC_ENOMEM;
  }
  fcirc_status st = FCIRC_OK;
  if (hipMemsetAsync(a, 0, bytes, s) != hipSuccess || hipMemsetAsync(x, 0, bytes, s) != hipSuccess) st = FCIRC_EDEVICE;
  std::vector<fcirc_item> items(count);
  for (uint32_t k = 0; k < count; ++k) items[k] = fcirc_item{k * n, k * n, k * n, (uint32_t)L, 0};
  const double f64[2] = {1.0, 0.0};
  const uint32_t f32 = 1;
  const void* f = ring == FCIRC_C64 ? (const void*)f64 : (const void*)&f32;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st == FCIRC_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = FCIRC_EDEVICE;
  BatchTune res;
  const int reps = 10;
  for (int w = 0; w < 2 && st == FCIRC_OK; ++w) {
    const int bt = w ? 512 : 256;
    for (int blog : {0, 10, 11, 12, 13}) {
      if (st != FCIRC_OK || !batch_param_ok(ring, L, bt, blog)) continue;
      const BatchForce F{L, bt, blog};
      for (int r = 0; r < 2 && st == FCIRC_OK; ++r) st = batched_product(c, a, x, y, items.data(), count, f, ring, s, &F);
      if (st != FCIRC_OK) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && st == FCIRC_OK; ++r) st = batched_product(c, a, x, y, items.data(), count, f, ring, s, &F);
      (void)hipEventRecord(e1, s);
      float ms = 0.f;
      if (st == FCIRC_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = FCIRC_EDEVICE;
      const float ns = (float)(ms * 1e6 / ((double)reps * count * n));
      if (st == FCIRC_OK && (res.ns[w] < 0.f || ns < res.ns[w])) {
        res.ns[w] = ns;
        res.blog[w] = blog;
      }
    }
  }
  if (st == FCIRC_OK) {
    c.batch_tuned[TuneKey{(int)ring, L}] = res;
    ++c.batch_gen;
    if (std::getenv("FCIRC_LOG"))
      std::fprintf(stderr, "fcirc_tune batched ring=%d L=%d: 256 threads blocks %d (%.4f ns/coef), 512 threads blocks %d (%.4f ns/coef)\n",
                   (int)ring, L, res.blog[0], res.ns[0], res.blog[1], res.ns[1]);
  }
  (void)hipStreamSynchronize(s);
  release_batches(c);  // the scratch batch's queues
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(a);
  (void)hipFree(x);
  (void)hipFree(y);
  return st;
}

// The device's architecture name (up to the first ':' feature suffix) and CU count.
void device_id(const Ctx& c, char* arch, size_t len, int* cus) {
  std::snprintf(arch, len, "%s", c.prop.gcnArchName);
  if (char* colon = std::strchr(arch, ':')) *colon = 0;
  *cus = c.prop.multiProcessorCount;
}

}  // namespace

namespace fcirc {

fcirc_status load_schedules(Ctx& c, const char* path) {
  std::FILE* f = std::fopen(path, "r");
  if (!f) return FCIRC_EINVAL;
  char arch[64];
  int cus = 0;
  device_id(c, arch, sizeof arch, &cus);
  std::map<TuneKey, TuneVal> got;
  std::map<TuneKey, BatchTune> gotb;
  char line[256];
  bool ok = true;
  while (ok && std::fgets(line, sizeof line, f)) {
    if (line[0] == '\n' || line[0] == '#') continue;
    char a[64];
    int u, ring, L, top, tile, flags;
    char tail;
    // batched-launch line: "<arch> <cus> batch <ring> <log2 n> <blocks 256> <ns 256> <blocks 512> <ns 512>"
    int b0, b1;
    float n0, n1;
    if (std::sscanf(line, "%63s %d batch %d %d %d %f %d %f %c", a, &u, &ring, &L, &b0, &n0, &b1, &n1, &tail) == 8) {
      const fcirc_ring r = (fcirc_ring)ring;
      if ((b0 != -1 && !batch_param_ok(r, L, 256, b0)) || (b1 != -1 && !batch_param_ok(r, L, 512, b1)) ||
          (b0 == -1 && b1 == -1) || !(n0 == n0) || !(n1 == n1)) {
        ok = false;
        break;
      }
      if (std::strcmp(a, arch) != 0 || u != cus) continue;
      BatchTune t;
      t.blog[0] = b0;
      t.blog[1] = b1;
      t.ns[0] = b0 == -1 ? -1.f : n0;
      t.ns[1] = b1 == -1 ? -1.f : n1;
      gotb[TuneKey{ring, L}] = t;
      continue;
    }
    if (std::sscanf(line, "%63s %d %d %d %d %d %d %c", a, &u, &ring, &L, &top, &tile, &flags, &tail) != 7) {
      ok = false;
      break;
    }
    const bool zp = ring >= FCIRC_ZP_998244353 && ring <= FCIRC_ZP_167772161;
    if (ring < FCIRC_ZP_998244353 || ring > FCIRC_GFP2 || L < 0 || L > 26 || top < -1 || top > 26 || tile < -1 ||
        tile > (zp ? 14 : 13) || flags < 0 || flags > 7) {
      ok = false;
      break;
    }
    if (std::strcmp(a, arch) != 0 || u != cus) continue;  // tuned on another device
    TuneVal v;
    v.top = top;
    v.tile_log = tile;
    v.flags = flags;
    got[TuneKey{ring, L}] = v;
  }
  if (std::ferror(f)) ok = false;
  std::fclose(f);
  if (!ok) return FCIRC_EINVAL;
  for (const auto& kv : got) c.tuned[kv.first] = kv.second;
  for (const auto& kv : gotb) c.batch_tuned[kv.first] = kv.second;
  if (!gotb.empty()) ++c.batch_gen;
  return FCIRC_OK;
}

}  // namespace fcirc

extern "C" {

fcirc_status fcirc_save_schedules(fcirc_ctx* ctx, const char* path) {
  if (!ctx || !path) return FCIRC_EINVAL;
  std::FILE* f = std::fopen(path, "w");
  if (!f) return FCIRC_EINVAL;
  char arch[64];
  int cus = 0;
  device_id(ctx->c, arch, sizeof arch, &cus);
  std::fprintf(f, "# arch cus ring log2n top_levels tile_log flags\n");
  for (const auto& kv : ctx->c.tuned)
    std::fprintf(f, "%s %d %d %d %d %d %d\n", arch, cus, kv.first.ring, kv.first.L, kv.second.top, kv.second.tile_log,
                 kv.second.flags);
  std::fprintf(f, "# arch cus batch ring log2n blocks_256 ns_per_coef_256 blocks_512 ns_per_coef_512 (blocks 0: one item)\n");
  for (const auto& kv : ctx->c.batch_tuned)
    std::fprintf(f, "%s %d batch %d %d %d %.6g %d %.6g\n", arch, cus, kv.first.ring, kv.first.L, kv.second.blog[0],
                 kv.second.ns[0], kv.second.blog[1], kv.second.ns[1]);
  const bool bad = std::ferror(f) != 0;
  return (std::fclose(f) != 0 || bad) ? FCIRC_EINVAL : FCIRC_OK;
}

fcirc_status fcirc_load_schedules(fcirc_ctx* ctx, const char* path) {
  if (!ctx || !path) return FCIRC_EINVAL;
  return load_schedules(ctx->c, path);
}

fcirc_status fcirc_set_schedule(fcirc_ctx* ctx, fcirc_ring ring, uint64_t n, int top_levels, int tile_log, int flags) {
  if (!ctx || n == 0 || (n & (n - 1)) || ring < FCIRC_ZP_998244353 || ring > FCIRC_GFP2) return FCIRC_EINVAL;
  if (top_levels < -1 || top_levels > 26 || tile_log < -1 || tile_log > (ring <= FCIRC_ZP_167772161 ? 14 : 13) || flags < 0 || flags > 7) return FCIRC_EINVAL;
  TuneVal v;
  v.top = top_levels;
  v.tile_log = tile_log;
  v.flags = flags;
  ctx->c.tuned[TuneKey{(int)ring, ilog2(n)}] = v;
  return FCIRC_OK;
}

fcirc_status fcirc_tune(fcirc_ctx* ctx, uint64_t n, fcirc_ring ring, void* stream) {
  if (!ctx || n == 0 || (n & (n - 1)) || ring < FCIRC_ZP_998244353 || ring > FCIRC_GFP2) return FCIRC_EINVAL;
  Ctx& c = ctx->c;
  if (hipSetDevice(c.device) != hipSuccess) return FCIRC_EDEVICE;
  const int L = ilog2(n);
  if (ring <= FCIRC_ZP_167772161 && L > zp_two_adic(zp_prime(ring))) return FCIRC_ESIZE;
  if (L > 26) return FCIRC_ESIZE;
  hipStream_t s = (hipStream_t)stream;
  const size_t eb = ring == FCIRC_C64 || ring == FCIRC_GFP2 ? 8 : 4;
  void *a = nullptr, *x = nullptr, *y = nullptr;
  if (hipMalloc(&a, n * eb) != hipSuccess || hipMalloc(&x, n * eb) != hipSuccess || hipMalloc(&y, n * eb) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipFree(a);
    if (x) (void)hipFree(x);
    return FCIRC_ENOMEM;
  }
  fcirc_status st = FCIRC_OK;
  if (hipMemsetAsync(a, 0, n * eb, s) != hipSuccess || hipMemsetAsync(x, 0, n * eb, s) != hipSuccess) st = FCIRC_EDEVICE;
  const bool zp = ring <= FCIRC_ZP_167772161;
  const int bmax = zp ? 13 : 12, bmin = 9;
  std::vector<TuneVal> cands;
  for (int bl = bmin; bl <= bmax; ++bl) {
    const int top = L - bl;
    if (top < 0) continue;
    if (top == 0) {
      TuneVal v;
      v.top = 0;
      v.flags = FCIRC_SCHED_XCD;
      cands.push_back(v);
      if (L >= 6 && L <= 12) {  // the several-wave small-product kernel
        v.flags = FCIRC_SCHED_XCD | FCIRC_SCHED_SMALL;
        cands.push_back(v);
      }
      continue;
    }
    for (int tl = 10; tl <= (zp ? 14 : 13); ++tl)
      for (int fl = 0; fl <= 3; ++fl) {
        TuneVal v;
        v.top = top;
        v.tile_log = tl;
        v.flags = fl;
        cands.push_back(v);
      }
  }
  if (cands.empty()) {
    TuneVal v;
    v.top = 0;
    cands.push_back(v);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (st == FCIRC_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) st = FCIRC_EDEVICE;
  const bool timing = c.timer.enabled;
  c.timer.enabled = false;
  const int forced = c.forced_top;
  c.forced_top = -1;
  const TuneKey key{(int)ring, L};
  float best = 1e30f;
  TuneVal bestv = cands[0];
  const int reps = n >= (1u << 20) ? 10 : 30;
  for (const TuneVal& v : cands) {
    if (st != FCIRC_OK) break;
    c.tuned[key] = v;
    for (int w = 0; w < 3 && st == FCIRC_OK; ++w) st = run_once(c, ring, L, a, x, y, s);
    if (st != FCIRC_OK) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == FCIRC_OK; ++r) st = run_once(c, ring, L, a, x, y, s);
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (st == FCIRC_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      st = FCIRC_EDEVICE;
    if (st == FCIRC_OK && ms < best) {
      best = ms;
      bestv = v;
    }
  }
  c.tuned[key] = bestv;
  c.timer.enabled = timing;
  c.forced_top = forced;
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(a);
  (void)hipFree(x);
  (void)hipFree(y);
  if (std::getenv("FCIRC_LOG"))
    std::fprintf(stderr, "fcirc_tune ring=%d L=%d: top=%d tile_log=%d flags=%d (%.2f us/call)\n", (int)ring, L, bestv.top,
                 bestv.tile_log, bestv.flags, 1000.0 * best / reps);
  if (st == FCIRC_OK && L <= 16 && (ring == FCIRC_C64 || ring <= FCIRC_ZP_167772161)) st = tune_batched(c, ring, L, s);
  return st;
}

int fcirc_get_schedule(fcirc_ctx* ctx, fcirc_ring ring, uint64_t n, int* top_levels, int* tile_log, int* flags) {
  if (!ctx || n == 0 || (n & (n - 1))) return -1;
  const Schedule S = schedule_for(ctx->c, ring, ilog2(n));
  if (top_levels) *top_levels = S.L - S.block_levels;
  if (tile_log) *tile_log = S.ntop ? S.top_r[0] + S.top_c[0] : -1;
  if (flags) *flags = S.flags;
  return S.ntop;
}

}  // extern "C"
