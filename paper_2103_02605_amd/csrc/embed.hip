// Products of any size n through one cyclic product of power-of-two size N >= 2n - 1
// (Corollary 1 of Rosowski, arXiv 2103.02605, section 2, and the Toeplitz embedding the
// introduction recalls): the row is laid out as (t_0 .. t_(n-1), 0 .. 0, t_-(n-1) .. t_-1)
// and the vector as (x, 0 .. 0); the first n entries of the cyclic product are T x.
// An f-circulant row a is the Toeplitz matrix with t_k = a_k and t_-k = f a_(n-k).
#include <hip/hip_runtime.h>

#include "host.hpp"

namespace fcirc {

namespace {

__device__ __forceinline__ uint32_t mulmod_dev(uint32_t a, uint32_t b, uint32_t p) {
  return (uint32_t)(((uint64_t)a * b) % p);
}

// Wrapped entry m (1 <= m < n) of the embedded row: t_-m.
struct WrapZp {
  const uint32_t* r;
  const uint32_t* col;  // null: f-circulant
  uint32_t f, p;
  uint64_t n;
  __device__ __forceinline__ uint32_t operator()(uint64_t m) const { return col ? col[m] : mulmod_dev(f, r[n - m], p); }
};
struct WrapC64 {
  const float2* r;
  const float2* col;
  float2 f;
  uint64_t n;
  __device__ __forceinline__ float2 operator()(uint64_t m) const {
    if (col) return col[m];
    const float2 v = r[n - m];
    return make_float2(f.x * v.x - f.y * v.y, f.x * v.y + f.y * v.x);
  }
};
struct WrapR32 {
  const float* r;
  const float* col;
  float f;
  uint64_t n;
  __device__ __forceinline__ float operator()(uint64_t m) const { return col ? col[m] : f * r[n - m]; }
};

template <class T, class Wrap>
__global__ void k_embed(const T* __restrict__ r, const T* __restrict__ x, Wrap wrap, T* __restrict__ ap, T* __restrict__ xp,
                        uint64_t n, uint64_t N) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (uint64_t)gridDim.x * blockDim.x) {
    T a = T{}, v = T{};
    if (k < n) {
      a = r[k];
      v = x[k];
    } else if (k + n > N) {
      a = wrap(N - k);  // N - k in [1, n - 1]
    }
    ap[k] = a;
    xp[k] = v;
  }
}

template <class T, class Wrap>
fcirc_status run_embed(Ctx& c, fcirc_ring ring, const T* r, const T* x, Wrap wrap, void* y, uint64_t n, int L,
                       hipStream_t s) {
  const uint64_t N = 1ull << L;
  fcirc_status st = ws2_reserve(c, 3 * N * sizeof(T));
  if (st != FCIRC_OK) return st;
  T* ap = (T*)c.ws2;
  T* xp = ap + N;
  T* yp = xp + N;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((N + 255) / 256, 4096);
  auto kern = k_embed<T, Wrap>;
  hipError_t e = launch(c, "fcirc_embed", s, [&](hipEvent_t e0_, hipEvent_t e1_) {
    FCIRC_LAUNCH(e0_, e1_, kern, dim3(grid), dim3(256), 0, s, r, x, wrap, ap, xp, n, N);
  });
  if (e != hipSuccess) return hip_status(e);
  if (ring <= FCIRC_ZP_167772161)
    st = zp_matvec(c, (const uint32_t*)ap, (const uint32_t*)xp, (uint32_t*)yp, L, 1, zp_prime(ring), 1u, s);
  else
    st = c32_matvec(c, ap, xp, yp, L, 1, 1.0, 0.0, ring == FCIRC_R32, s);
  if (st != FCIRC_OK) return st;
  return hip_status(hipMemcpyAsync(y, yp, n * sizeof(T), hipMemcpyDeviceToDevice, s));
}

}  // namespace

// r: first row (t_0 .. t_(n-1)); col: first column (col[m] = t_-m, col[0] unused) or null
// for the f-circulant whose first row is r. Sizes and f are validated by the caller.
fcirc_status embed_product(Ctx& c, fcirc_ring ring, const void* r, const void* col, const void* f, const void* x, void* y,
                           uint64_t n, hipStream_t s) {
  int L = 0;
  while ((1ull << L) < 2 * n - 1) ++L;
  if (ring <= FCIRC_ZP_167772161) {
    const uint32_t p = zp_prime(ring);
    const WrapZp w{(const uint32_t*)r, (const uint32_t*)col, f ? *(const uint32_t*)f : 1u, p, n};
    return run_embed(c, ring, (const uint32_t*)r, (const uint32_t*)x, w, y, n, L, s);
  }
  if (ring == FCIRC_C64) {
    const double* fc = (const double*)f;
    const WrapC64 w{(const float2*)r, (const float2*)col, f ? make_float2((float)fc[0], (float)fc[1]) : make_float2(1.f, 0.f), n};
    return run_embed(c, ring, (const float2*)r, (const float2*)x, w, y, n, L, s);
  }
  const WrapR32 w{(const float*)r, (const float*)col, f ? (float)*(const double*)f : 1.f, n};
  return run_embed(c, ring, (const float*)r, (const float*)x, w, y, n, L, s);
}

}  // namespace fcirc
