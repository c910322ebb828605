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
  char line[256];
  bool ok = true;
  while (ok && std::fgets(line, sizeof line, f)) {
    if (line[0] == '\n' || line[0] == '#') continue;
    char a[64];
    int u, ring, L, top, tile, flags;
    char tail;
    if (std::sscanf(line, "%63s %d %d %d %d %d %d %c", a, &u, &ring, &L, &top, &tile, &flags, &tail) != 7) {
      ok = false;
      break;
    }
    const bool zp = ring >= FCIRC_ZP_998244353 && ring <= FCIRC_ZP_167772161;
    if (ring < FCIRC_ZP_998244353 || ring > FCIRC_GFP2 || L < 0 || L > 26 || top < -1 || top > 26 || tile < -1 ||
        tile > (zp ? 14 : 13) || flags < 0 || flags > 3) {
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
  const bool bad = std::ferror(f) != 0;
  return (std::fclose(f) != 0 || bad) ? FCIRC_EINVAL : FCIRC_OK;
}

fcirc_status fcirc_load_schedules(fcirc_ctx* ctx, const char* path) {
  if (!ctx || !path) return FCIRC_EINVAL;
  return load_schedules(ctx->c, path);
}

fcirc_status fcirc_set_schedule(fcirc_ctx* ctx, fcirc_ring ring, uint64_t n, int top_levels, int tile_log, int flags) {
  if (!ctx || n == 0 || (n & (n - 1)) || ring < FCIRC_ZP_998244353 || ring > FCIRC_GFP2) return FCIRC_EINVAL;
  if (top_levels < -1 || top_levels > 26 || tile_log < -1 || tile_log > (ring <= FCIRC_ZP_167772161 ? 14 : 13) || flags < 0 || flags > 3) return FCIRC_EINVAL;
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
      cands.push_back(v);
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
