// The f-circulant product over GF(p^2) = Z/p[sqrt 3], p = 2^31 - 1: the ring section 3.1
// of Rosowski (arXiv 2103.02605) computes in, with the N-th roots of unity
// (2 + sqrt 3)^((p+1)/N). The same tile kernels run with the Gp2 ring policy.
#include <hip/hip_runtime.h>

#include <vector>

#include "host.hpp"

namespace fcirc {

namespace {

constexpr uint64_t GP = 0x7fffffffull;

struct E2 {  // host element a + b sqrt 3
  uint64_t a, b;
};
E2 e2mul(E2 u, E2 v) {
  const uint64_t ac = u.a * v.a % GP, bd = u.b * v.b % GP, ad = u.a * v.b % GP, bc = u.b * v.a % GP;
  return E2{(ac + 3 * bd) % GP, (ad + bc) % GP};
}
E2 e2pow(E2 u, uint64_t e) {
  E2 out{1, 0};
  while (e) {
    if (e & 1) out = e2mul(out, u);
    u = e2mul(u, u);
    e >>= 1;
  }
  return out;
}
// norm-one elements: the inverse is the conjugate
uint2 conj2(E2 u) { return make_uint2((uint32_t)u.a, (uint32_t)((GP - u.b) % GP)); }
uint2 to2(E2 u) { return make_uint2((uint32_t)u.a, (uint32_t)u.b); }
// rho_d = (2 + sqrt 3)^((p+1)/2^(d+1)), a primitive 2^(d+1)-th root of unity
E2 rho(int d) { return e2pow(E2{2, 1}, (GP + 1) >> (d + 1)); }
uint32_t brev2(uint32_t v, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1u) << (bits - 1 - i);
  return r;
}

fcirc_status gp2_tables(Ctx& c, int fneg, int L, const Gp2Tables** out, bool build) {
  for (auto& t : c.gp2)
    if (t.fneg == fneg && t.levels >= L) {
      *out = &t;
      return FCIRC_OK;
    }
  if (!build) return FCIRC_ENOPLAN;
  const int levels = L < 12 ? 12 : L;
  // g_{d,b} = r_{d+1} rho_d^brev_d(b): r_k = 1 for f = 1; for f = -1, r_k = rho_k (order
  // 2^(k+1)), so r_1^2 = -1 and r_(k+1)^2 = r_k.
  const size_t ne = (size_t)1 << levels;
  std::vector<uint2> tw(ne), twi(ne);
  tw[0] = twi[0] = make_uint2(0, 0);
  std::vector<E2> pw;
  for (int d = 0; d < levels; ++d) {
    const E2 rh = rho(d);
    const E2 r = fneg ? rho(d + 1) : E2{1, 0};
    const size_t m = (size_t)1 << d;
    pw.assign(m, E2{1, 0});
    for (size_t k = 1; k < m; ++k) pw[k] = e2mul(pw[k - 1], rh);
    for (size_t b = 0; b < m; ++b) {
      const E2 g = e2mul(r, pw[brev2((uint32_t)b, d)]);
      tw[m + b] = to2(g);
      twi[m + b] = conj2(g);
    }
  }
  uint2 u[30];
  for (int j = 0; j < 4; ++j) {
    const E2 rh = rho(j);
    for (uint32_t g = 0; g < (1u << j); ++g) {
      const E2 w = e2pow(rh, brev2(g, j));
      u[(1 << j) - 1 + g] = to2(w);
      u[15 + (1 << j) - 1 + g] = conj2(w);
    }
  }
  Gp2Tables t;
  t.fneg = fneg;
  t.levels = levels;
  if (hipMalloc(&t.tw, ne * sizeof(uint2)) != hipSuccess || hipMalloc(&t.twi, ne * sizeof(uint2)) != hipSuccess ||
      hipMalloc(&t.dU, sizeof u) != hipSuccess) {
    (void)hipGetLastError();
    if (t.tw) (void)hipFree(t.tw);
    if (t.twi) (void)hipFree(t.twi);
    return FCIRC_ENOMEM;
  }
  if (hipMemcpy(t.tw, tw.data(), ne * sizeof(uint2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.twi, twi.data(), ne * sizeof(uint2), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.dU, u, sizeof u, hipMemcpyHostToDevice) != hipSuccess)
    return FCIRC_EDEVICE;
  for (auto& old : c.gp2)
    if (old.fneg == fneg) {
      if (hipDeviceSynchronize() != hipSuccess) return FCIRC_EDEVICE;
      (void)hipFree(old.tw);
      (void)hipFree(old.twi);
      (void)hipFree(old.dU);
      old = t;
      *out = &old;
      return FCIRC_OK;
    }
  c.gp2.push_back(t);
  *out = &c.gp2.back();
  return FCIRC_OK;
}

}  // namespace

fcirc_status gp2_matvec(Ctx& c, const void* a, const void* x, void* y, int L, uint32_t count, int fneg, hipStream_t s,
                        const FixedWs* fx) {
  const Gp2Tables* T = nullptr;
  fcirc_status st = gp2_tables(c, fneg, L, &T, fx == nullptr);
  if (st != FCIRC_OK) return st;
  const Schedule S = schedule_for(c, FCIRC_GFP2, L);
  void* ws = nullptr;
  st = product_ws(c, fx, product_ws_elems(S, count, false) * sizeof(uint2), &ws);
  if (st != FCIRC_OK) return st;
  const Gp2Params rp{(uint32_t)((1ull << (31 - L)) % GP)};  // 1/n = 2^(31-L) since 2^31 = 1 mod p
  const Gp2Params rps[3] = {rp, rp, rp};
  const uint2* tw[3] = {T->tw, T->tw, T->tw};
  const uint2* twi[3] = {T->twi, T->twi, T->twi};
  const uint2* U[3] = {T->dU, T->dU, T->dU};
  const uint64_t n = (uint64_t)1 << L;
  return hip_status(run_product<Gp2>(c, S, count, rps, tw, twi, U, nullptr, nullptr, false, LdPlain<uint2>{(const uint2*)a, n},
                                     LdPlain<uint2>{(const uint2*)x, n}, StPlain<uint2>{(uint2*)y, n}, (uint2*)y,
                                     (uint2*)ws, s));
}

}  // namespace fcirc
