// Z/p plans and the Z/p f-circulant product.
//
// Theorem 1 (Rosowski, arXiv 2103.02605, section 2) needs an n-th root of f and an n-th
// root of unity. Section 3.1 precomputes the roots Algorithm 1 uses in linear time.
// Here the square root taken at node b of depth d is
//     g_{d,b} = r_{d+1} * rho_d^{brev_d(b)},
// where r_0 = f, r_{k+1}^2 = r_k is a fixed chain of square roots of f, rho_d is a
// primitive 2^(d+1)-th root of unity and brev_d reverses the low d bits. Then
// g_{d,b}^2 = g_{d-1,b/2} for even b and -g_{d-1,b/2} for odd b (rho_d^(2^d) = -1),
// which are exactly the values Algorithm 1 hands to the two children (+sqrt f and
// -sqrt f). The table does not depend on n beyond its number of levels, so one table per
// (p, f) serves every size. Merge twiddles are the inverses 1/g_{d,b}.
#include <hip/hip_runtime.h>

#include <cstring>

#include "host.hpp"

namespace fcirc {

namespace {

inline uint32_t mulmod(uint64_t a, uint64_t b, uint32_t p) { return (uint32_t)(a * b % p); }

uint32_t powmod(uint32_t b, uint64_t e, uint32_t p) {
  uint64_t r = 1, x = b % p;
  while (e) {
    if (e & 1) r = r * x % p;
    x = x * x % p;
    e >>= 1;
  }
  return (uint32_t)r;
}

uint32_t invmod(uint32_t v, uint32_t p) { return powmod(v, p - 2, p); }

// Smallest generator of (Z/p)^*.
uint32_t generator(uint32_t p) {
  uint32_t m = p - 1, f[32];
  int nf = 0;
  for (uint32_t d = 2; (uint64_t)d * d <= m; ++d)
    if (m % d == 0) {
      f[nf++] = d;
      while (m % d == 0) m /= d;
    }
  if (m > 1) f[nf++] = m;
  for (uint32_t g = 2;; ++g) {
    bool ok = true;
    for (int i = 0; i < nf && ok; ++i) ok = powmod(g, (p - 1) / f[i], p) != 1;
    if (ok) return g;
  }
}

// Square root of a quadratic residue v (Cipolla-free Tonelli-Shanks); v != 0.
uint32_t sqrtmod(uint32_t v, uint32_t p, uint32_t gen) {
  uint32_t q = p - 1;
  int s = 0;
  while ((q & 1) == 0) {
    q >>= 1;
    ++s;
  }
  uint32_t z = powmod(gen, q, p);  // a generator's q-th power has order exactly 2^s
  uint32_t m = (uint32_t)s, c = z, t = powmod(v, q, p), r = powmod(v, (q + 1) / 2, p);
  while (t != 1) {
    uint32_t i = 0, t2 = t;
    while (t2 != 1) {
      t2 = mulmod(t2, t2, p);
      ++i;
    }
    uint32_t b = c;
    for (uint32_t k = 0; k + i + 1 < m; ++k) b = mulmod(b, b, p);
    m = i;
    c = mulmod(b, b, p);
    t = mulmod(t, c, p);
    r = mulmod(r, b, p);
  }
  return r;
}

inline uint32_t brev(uint32_t b, int d) { return d == 0 ? 0 : (__builtin_bitreverse32(b) >> (32 - d)); }

inline ZpTw shoup_tw(uint32_t w, uint32_t p) { return ZpTw{w, (uint32_t)(((uint64_t)w << 32) / p)}; }

}  // namespace

uint32_t zp_prime(fcirc_ring r) {
  switch (r) {
    case FCIRC_ZP_998244353: return 998244353u;
    case FCIRC_ZP_469762049: return 469762049u;
    case FCIRC_ZP_167772161: return 167772161u;
    default: return 0;
  }
}

int zp_two_adic(uint32_t p) {
  int s = 0;
  uint32_t q = p - 1;
  while ((q & 1) == 0) {
    q >>= 1;
    ++s;
  }
  return s;
}

ZpParams zp_params(uint32_t p, int L) {
  ZpParams q;
  q.p = p;
  uint32_t inv = p;  // Newton iteration for p^-1 mod 2^32 (p odd)
  for (int i = 0; i < 5; ++i) inv *= 2u - p * inv;
  q.pinv = inv;
  q.npinv = 0u - inv;
  const uint32_t two32 = (uint32_t)(((uint64_t)1 << 32) % p);
  const uint32_t ninv = invmod(powmod(2, (uint64_t)L, p), p);
  q.leaf = shoup_tw(mulmod(two32, ninv, p), p);
  q.one = shoup_tw(1, p);
  q.two31 = (uint32_t)(((uint64_t)1 << 31) % p);
  q.r32 = shoup_tw(two32, p);
  return q;
}

// Uniform factors rho_j^brev_j(g) and their inverses, in Montgomery form (w 2^32 mod p):
// out[0..15) split and out[15..30) merge for the radix-16 items (j < 4), then the block
// factors of j < ZP_UB_LEVELS: out[30 .. 30 + ZP_UB) split, the next ZP_UB merge.
void zp_uniform_mont(uint32_t p, uint32_t* out) {
  // rho_j = gen^((p-1)/2^(j+1)), the same roots the tables are built from
  const uint32_t gen = generator(p);
  const uint32_t two32 = (uint32_t)(((uint64_t)1 << 32) % p);
  uint32_t* ub = out + 30;
  uint32_t* ubi = ub + ZP_UB;
  for (int j = 0; j < ZP_UB_LEVELS; ++j) {
    const uint32_t rho = powmod(gen, (uint64_t)(p - 1) >> (j + 1), p);
    for (uint32_t g = 0; g < (1u << j); ++g) {
      const uint32_t e = brev(g, j);
      const uint32_t w = powmod(rho, e, p), wi = invmod(w, p);
      ub[(1 << j) - 1 + g] = mulmod(w, two32, p);
      ubi[(1 << j) - 1 + g] = mulmod(wi, two32, p);
    }
  }
  for (int k = 0; k < 15; ++k) {
    out[k] = ub[k];
    out[15 + k] = ubi[k];
  }
}

fcirc_status zp_tables(Ctx& c, uint32_t p, uint32_t f, int L, const ZpTables** out, bool build) {
  const int e2 = zp_two_adic(p);
  if (L > e2) return FCIRC_ESIZE;
  if (f == 0 || f >= p) return FCIRC_ENOROOT;
  // Theorem 1 needs an n-th root of f; with 2^L | p - 1 it exists iff f^((p-1)/2^L) = 1.
  if (powmod(f, (uint64_t)(p - 1) >> L, p) != 1) return FCIRC_ENOROOT;
  for (auto& t : c.zp)
    if (t.p == p && t.f == f && t.levels >= L) {
      *out = &t;
      return FCIRC_OK;
    }
  if (!build) return FCIRC_ENOPLAN;
  // Build (or rebuild larger) with at least 12 levels so small sizes share one table.
  int levels = L < 12 ? 12 : L;
  while (levels > L && powmod(f, (uint64_t)(p - 1) >> levels, p) != 1) --levels;
  if (levels > e2) levels = e2;
  const uint32_t gen = generator(p);
  std::vector<uint32_t> r(levels + 1);
  r[0] = f;
  for (int k = 1; k <= levels; ++k) {
    if (f == 1)
      r[k] = 1;
    else if (f == p - 1)
      r[k] = powmod(gen, (uint64_t)(p - 1) >> (k + 1), p);  // gen^((p-1)/2^(k+1)): order 2^(k+1)
    else
      r[k] = sqrtmod(r[k - 1], p, gen);
  }
  for (int k = 1; k <= levels; ++k)
    if (mulmod(r[k], r[k], p) != r[k - 1]) return FCIRC_ENOROOT;
  const size_t ne = (size_t)1 << levels;
  std::vector<ZpTw> tw(ne), twi(ne);
  tw[0] = twi[0] = ZpTw{0, 0};
  std::vector<uint32_t> pw;
  for (int d = 0; d < levels; ++d) {
    const uint32_t rho = powmod(gen, (uint64_t)(p - 1) >> (d + 1), p);
    const size_t m = (size_t)1 << d;
    pw.assign(m, 1);
    for (size_t k = 1; k < m; ++k) pw[k] = mulmod(pw[k - 1], rho, p);
    const uint32_t rr = r[d + 1], rri = invmod(r[d + 1], p);
    for (size_t b = 0; b < m; ++b) {
      const uint32_t k = brev((uint32_t)b, d);
      const uint32_t g = mulmod(rr, pw[k], p);
      // rho^-k = -rho^(2^d - k) for k > 0
      const uint32_t pinvk = k == 0 ? 1u : (p - pw[m - k]) % p;
      const uint32_t gi = mulmod(rri, pinvk, p);
      tw[m + b] = shoup_tw(g, p);
      twi[m + b] = shoup_tw(gi, p);
    }
  }
  ZpTables t;
  t.p = p;
  t.f = f;
  t.levels = levels;
  if (hipMalloc(&t.tw, ne * sizeof(ZpTw)) != hipSuccess || hipMalloc(&t.twi, ne * sizeof(ZpTw)) != hipSuccess) {
    (void)hipGetLastError();
    if (t.tw) (void)hipFree(t.tw);
    return FCIRC_ENOMEM;
  }
  if (hipMemcpy(t.tw, tw.data(), ne * sizeof(ZpTw), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(t.twi, twi.data(), ne * sizeof(ZpTw), hipMemcpyHostToDevice) != hipSuccess)
    return FCIRC_EDEVICE;
  std::vector<uint32_t> um(30 + 2 * ZP_UB);
  zp_uniform_mont(p, um.data());
  const size_t ub_bytes = um.size() * sizeof(uint32_t);
  if (hipMalloc(&t.dU, ub_bytes) != hipSuccess || hipMemcpy(t.dU, um.data(), ub_bytes, hipMemcpyHostToDevice) != hipSuccess)
    return FCIRC_ENOMEM;
  // Replace a smaller table for the same (p, f) only after the device is idle.
  for (auto& old : c.zp)
    if (old.p == p && old.f == f) {
      if (hipDeviceSynchronize() != hipSuccess) return FCIRC_EDEVICE;
      (void)hipFree(old.tw);
      (void)hipFree(old.twi);
      (void)hipFree(old.dU);
      for (int l = 0; l < 27; ++l) {  // first-twiddle tables depend on (p, f, L) only
        t.ft[l] = old.ft[l];
        t.fti[l] = old.fti[l];
      }
      old = t;
      *out = &old;
      return FCIRC_OK;
    }
  c.zp.push_back(t);
  *out = &c.zp.back();
  return FCIRC_OK;
}

fcirc_status zp_first_tables(Ctx& c, const ZpTables* Tc, int L, const uint32_t** ft, const uint32_t** fti,
                             bool build) {
  ZpTables* T = const_cast<ZpTables*>(Tc);
  *ft = *fti = nullptr;
  if (L < 4 || L > 26) return FCIRC_OK;
  if (!T->ft[L] && !build) return FCIRC_ENOPLAN;
  if (!T->ft[L]) {
    // c_3 = g_{L-1, 8 b0} = r_L rho_{L-1}^{brev_dd(b0)} for the node b0 at depth dd = L - 4,
    // in Montgomery form; the kernels square it for the three levels above.
    const uint32_t p = T->p, f = T->f, gen = generator(p);
    const uint32_t two32 = (uint32_t)(((uint64_t)1 << 32) % p);
    const int dd = L - 4;
    std::vector<uint32_t> r(L + 1);
    r[0] = f;
    for (int k = 1; k <= L; ++k) {
      if (f == 1)
        r[k] = 1;
      else if (f == p - 1)
        r[k] = powmod(gen, (uint64_t)(p - 1) >> (k + 1), p);
      else
        r[k] = sqrtmod(r[k - 1], p, gen);
    }
    const size_t nb = (size_t)1 << dd;
    std::vector<uint32_t> h(nb), hi(nb), pw(nb), pwi(nb);
    const uint32_t rho = powmod(gen, (uint64_t)(p - 1) >> L, p), rhoi = invmod(rho, p);  // rho_{L-1}
    pw[0] = pwi[0] = 1;
    for (size_t k = 1; k < nb; ++k) {
      pw[k] = mulmod(pw[k - 1], rho, p);
      pwi[k] = mulmod(pwi[k - 1], rhoi, p);
    }
    const uint32_t rr = r[L], rri = invmod(rr, p);
    for (size_t b0 = 0; b0 < nb; ++b0) {
      const uint32_t k = brev((uint32_t)b0, dd);
      h[b0] = mulmod(mulmod(rr, pw[k], p), two32, p);
      hi[b0] = mulmod(mulmod(rri, pwi[k], p), two32, p);
    }
    uint32_t *d = nullptr, *di = nullptr;
    if (hipMalloc(&d, nb * sizeof(uint32_t)) != hipSuccess || hipMalloc(&di, nb * sizeof(uint32_t)) != hipSuccess) {
      (void)hipGetLastError();
      if (d) (void)hipFree(d);
      return FCIRC_ENOMEM;
    }
    if (hipMemcpy(d, h.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(di, hi.data(), nb * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
      return FCIRC_EDEVICE;
    T->ft[L] = d;
    T->fti[L] = di;
  }
  *ft = T->ft[L];
  *fti = T->fti[L];
  return FCIRC_OK;
}

fcirc_status zp_matvec(Ctx& c, const uint32_t* a, const uint32_t* x, uint32_t* y, int L, uint32_t count, uint32_t p,
                       uint32_t f, hipStream_t s, const FixedWs* fx) {
  const ZpTables* T = nullptr;
  fcirc_status st = zp_tables(c, p, f, L, &T, fx == nullptr);
  if (st != FCIRC_OK) return st;
  const int ring = p == 998244353u ? 0 : (p == 469762049u ? 1 : 2);
  const Schedule S = schedule_for(c, ring, L);
  void* ws = nullptr;
  st = product_ws(c, fx, product_ws_elems(S, count, false) * sizeof(uint32_t), &ws);
  if (st != FCIRC_OK) return st;
  const ZpParams rp = zp_params(p, L);
  const ZpParams rps[3] = {rp, rp, rp};
  const ZpTw* tw[3] = {T->tw, T->tw, T->tw};
  const ZpTw* twi[3] = {T->twi, T->twi, T->twi};
  const uint64_t n = (uint64_t)1 << L;
  const uint32_t* U[3] = {T->dU, T->dU, T->dU};
  const uint32_t *ft = nullptr, *fti = nullptr;
  st = zp_first_tables(c, T, L, &ft, &fti, fx == nullptr);
  if (st != FCIRC_OK) return st;
  const uint32_t* FT[3] = {ft, ft, ft};
  const uint32_t* FTI[3] = {fti, fti, fti};
  return hip_status(run_product<Zp>(c, S, count, rps, tw, twi, U, ft ? FT : nullptr, ft ? FTI : nullptr, false, LdPlain<uint32_t>{a, n},
                                    LdPlain<uint32_t>{x, n}, StPlain<uint32_t>{y, n}, y, (uint32_t*)ws, s));
}

}  // namespace fcirc
