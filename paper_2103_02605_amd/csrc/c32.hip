// Complex (FP32 data) plans and products.
//
// Over the complex numbers Theorem 1's roots always exist. Taking principal square roots
// all the way down, the chain of roots of f is r_k = |f|^(1/2^k) e^(i arg(f) / 2^k), and
// the square root used at node b of depth d is
//     g_{d,b} = r_{d+1} * e^(i pi brev_d(b) / 2^d)
// (the second factor is rho_d^brev_d(b) with rho_d = e^(i pi / 2^d), a primitive
// 2^(d+1)-th root of unity; see zp.hip for why this satisfies Algorithm 1's recursion).
// The tables are computed in FP64 on the GPU and rounded once to FP32, so no FP32
// recurrence error accumulates across levels.
#include <hip/hip_runtime.h>

#include <cmath>

#include "host.hpp"

namespace fcirc {

__global__ void k_c32_tables(float2* tw, float2* twi, uint32_t nent, double lnabs, double arg_over_pi) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx == 0 || idx >= nent) {
    if (idx == 0) {
      tw[0] = make_float2(0.f, 0.f);
      twi[0] = make_float2(0.f, 0.f);
    }
    return;
  }
  const int d = 31 - __clz(idx);
  const uint32_t b = idx - (1u << d);
  const uint32_t br = d == 0 ? 0u : (__brev(b) >> (32 - d));
  const double scale = ldexp(1.0, -(d + 1));          // 1 / 2^(d+1)
  const double t = arg_over_pi * scale + ldexp((double)br, -d);
  double sn, cs;
  sincospi(t, &sn, &cs);
  const double mag = exp(lnabs * scale);
  tw[idx] = make_float2((float)(mag * cs), (float)(mag * sn));
  twi[idx] = make_float2((float)(cs / mag), (float)(-sn / mag));
}

Uniform16<C32> c32_uniform16() {
  // rho_j = e^(i pi / 2^j): tu = e^(i pi brev_j(g) / 2^j), tui its conjugate
  Uniform16<C32> U;
  for (int j = 0; j < 4; ++j)
    for (uint32_t g = 0; g < (1u << j); ++g) {
      const uint32_t e = j == 0 ? 0u : (__builtin_bitreverse32(g) >> (32 - j));
      const double ang = M_PI * (double)e / (double)(1u << j);
      U.tu[(1 << j) - 1 + g] = make_float2((float)std::cos(ang), (float)std::sin(ang));
      U.tui[(1 << j) - 1 + g] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
    }
  return U;
}

fcirc_status c32_tables(Ctx& c, double fre, double fim, int L, hipStream_t s, const C32Tables** out, bool build) {
  if (fre == 0.0 && fim == 0.0) return FCIRC_ENOROOT;
  for (auto& t : c.c32)
    if (t.fre == fre && t.fim == fim && t.levels >= L) {
      *out = &t;
      return FCIRC_OK;
    }
  if (!build) return FCIRC_ENOPLAN;
  const int levels = L < 16 ? 16 : L;
  const size_t ne = (size_t)1 << levels;
  C32Tables t;
  t.fre = fre;
  t.fim = fim;
  t.levels = levels;
  t.U = c32_uniform16();
  if (hipMalloc(&t.tw, ne * sizeof(float2)) != hipSuccess || hipMalloc(&t.twi, ne * sizeof(float2)) != hipSuccess) {
    (void)hipGetLastError();
    if (t.tw) (void)hipFree(t.tw);
    return FCIRC_ENOMEM;
  }
  const double lnabs = std::log(std::hypot(fre, fim));
  const double arg_over_pi = std::atan2(fim, fre) / M_PI;
  const uint32_t threads = 256, blocks = (uint32_t)((ne + threads - 1) / threads);
  hipLaunchKernelGGL(k_c32_tables, dim3(blocks), dim3(threads), 0, s, t.tw, t.twi, (uint32_t)ne, lnabs, arg_over_pi);
  if (hipGetLastError() != hipSuccess) return FCIRC_EDEVICE;
  if (hipMalloc(&t.dU, 30 * sizeof(float2)) != hipSuccess ||
      hipMemcpy(t.dU, t.U.tu, 15 * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.dU + 15, t.U.tui, 15 * sizeof(float2), hipMemcpyHostToDevice) != hipSuccess)
    return FCIRC_ENOMEM;
  for (auto& old : c.c32)
    if (old.fre == fre && old.fim == fim) {
      if (hipDeviceSynchronize() != hipSuccess) return FCIRC_EDEVICE;
      (void)hipFree(old.tw);
      (void)hipFree(old.twi);
      (void)hipFree(old.dU);
      old = t;
      *out = &old;
      return FCIRC_OK;
    }
  c.c32.push_back(t);
  *out = &c.c32.back();
  return FCIRC_OK;
}

fcirc_status c32_matvec(Ctx& c, const void* a, const void* x, void* y, int L, uint32_t count, double fre, double fim,
                        bool real_io, hipStream_t s, const FixedWs* fx) {
  const C32Tables* T = nullptr;
  fcirc_status st = c32_tables(c, fre, fim, L, s, &T, fx == nullptr);
  if (st != FCIRC_OK) return st;
  const Schedule S = schedule_for(c, real_io ? FCIRC_R32 : FCIRC_C64, L);
  void* wsp = nullptr;
  st = product_ws(c, fx, product_ws_elems(S, count, real_io) * sizeof(float2), &wsp);
  if (st != FCIRC_OK) return st;
  const C32Params rp{(float)std::ldexp(1.0, -L)};
  const C32Params rps[3] = {rp, rp, rp};
  const float2* tw[3] = {T->tw, T->tw, T->tw};
  const float2* twi[3] = {T->twi, T->twi, T->twi};
  const uint64_t n = (uint64_t)1 << L;
  float2* ws = (float2*)wsp;
  const float2* U[3] = {T->dU, T->dU, T->dU};
  hipError_t e;
  if (real_io) {
    e = run_product<C32>(c, S, count, rps, tw, twi, U, nullptr, nullptr, false, LdR32{(const float*)a, n}, LdR32{(const float*)x, n},
                         StR32{(float*)y, n}, nullptr, ws, s);
  } else {
    e = run_product<C32>(c, S, count, rps, tw, twi, U, nullptr, nullptr, false, LdPlain<float2>{(const float2*)a, n},
                         LdPlain<float2>{(const float2*)x, n}, StPlain<float2>{(float2*)y, n}, (float2*)y, ws, s);
  }
  return hip_status(e);
}

}  // namespace fcirc
