/*
 * libfcirc -- FFT-free f-circulant matrix-vector products on AMD Instinct MI355X (gfx950).
 *
 * The product follows A. Rosowski, "On Fast Computation of a Circulant Matrix-Vector
 * Product" (arXiv 2103.02605):
 *   - Definition 2 (section 1.2): an n x n matrix is f-circulant when each row is the
 *     previous row shifted right by one place, the entry that wraps around to column 1
 *     being multiplied by f. Section 1.2 identifies such a matrix by its FIRST ROW a, so
 *     with 0-based indices A[i][j] = a[j-i] for j >= i and A[i][j] = f * a[n+j-i] for j < i.
 *   - Theorem 1 (section 2): for n a power of two, in a ring holding an n-th root of f,
 *     an n-th root of unity, 1/2 and 1/f, y = A x costs O(n log n) operations.
 *   - Algorithm 1 (section 2): split A into a sqrt(f)- and a (-sqrt f)-circulant product
 *     of half size, recurse down to scalars, merge the two halves back.
 *
 * All device work is asynchronous on the stream passed in (a hipStream_t, given here as
 * void*; NULL means the null stream). Every entry point validates its arguments on the
 * host first and returns an error without enqueueing anything when they are invalid.
 * The caller owns every data buffer. The context owns plans, twiddle tables, workspaces
 * and the work queues of batched launches, and frees them in fcirc_destroy.
 *
 * Threading: one context serves one host thread at a time (calls that share a context
 * must be serialised by the caller). The context's workspace is shared by its calls, so
 * calls on different streams with one context must not run concurrently on the device
 * (order the streams, or use one context per stream). Output buffers must not overlap
 * inputs.
 */
#ifndef FCIRC_H
#define FCIRC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcirc_ctx fcirc_ctx;

/* The ring R of Theorem 1. */
typedef enum {
  FCIRC_ZP_998244353 = 0, /* Z/p, p = 119*2^23 + 1: data uint32 in [0,p), n <= 2^23     */
  FCIRC_ZP_469762049 = 1, /* Z/p, p =   7*2^26 + 1: data uint32 in [0,p), n <= 2^26     */
  FCIRC_ZP_167772161 = 2, /* Z/p, p =   5*2^25 + 1: data uint32 in [0,p), n <= 2^25     */
  FCIRC_C64 = 3,          /* complex numbers: data interleaved complex64 (float re, im)   */
  FCIRC_R32 = 4,          /* real data float32; complex arithmetic inside; f real         */
  FCIRC_GFP2 = 5          /* the ring of section 3.1, Z/p[sqrt 3] = GF(p^2), p = 2^31 - 1:
                             data uint32 pairs (a, b) = a + b sqrt 3, both in [0,p);
                             roots of unity (2 + sqrt 3)^((p+1)/N); f = 1 or -1, n <= 2^26 */
} fcirc_ring;

typedef enum {
  FCIRC_OK = 0,
  FCIRC_EINVAL = 1,  /* null pointer, unknown ring, bad item list, overlapping buffers    */
  FCIRC_ESIZE = 2,   /* n not a power of two, n = 0, or n above the ring's limit          */
  FCIRC_ENOROOT = 3, /* f is zero or has no n-th root in the ring (Theorem 1's condition) */
  FCIRC_ERANGE = 4,  /* a product coefficient fell outside the exactly representable range
                        (reported by fcirc_check after the work has run)                  */
  FCIRC_ENOMEM = 5,  /* device allocation failed or exceeded FCIRC_WORKSPACE_LIMIT        */
  FCIRC_EDEVICE = 6, /* no usable gfx950 device, or a HIP call failed                     */
  FCIRC_ESCHED = 7,  /* fcirc_matvec_batched: a work item gave up waiting (bounded spin) for
                        the items it depends on; the outputs of that launch are unspecified
                        (reported by fcirc_check after the work has run)                  */
  FCIRC_ENOPLAN = 8  /* fcirc_matvec_noalloc: the twiddle tables of (ring, f, n) are not
                        resident in the context and may not be built by this call        */
} fcirc_status;

/* Create a context on HIP device `hip_device` (must be gfx950). */
fcirc_status fcirc_create(fcirc_ctx **ctx, int hip_device);
/* Synchronise the device and free everything the context owns. NULL is allowed. */
void fcirc_destroy(fcirc_ctx *ctx);
const char *fcirc_strerror(fcirc_status s);

/*
 * y = A(a, f) x: one f-circulant product of size n (Definition 2, Theorem 1, Algorithm 1).
 *   a : device, n elements, the FIRST ROW of A (section 1.2's row convention).
 *   x : device, n elements.  y : device, n elements (written; must not overlap a or x).
 *   f : host pointer to ONE ring element: uint32_t in [0,p) for Z/p, double[2] (re, im)
 *       for FCIRC_C64, double for FCIRC_R32, uint32_t[2] (a, b) for FCIRC_GFP2 (f must
 *       be 1 = (1, 0) or -1 = (p-1, 0) there).
 *   Z/p elements must be canonical (in [0,p)); outputs are canonical.
 * Errors: EINVAL (null pointer, f not canonical), ESIZE (n not a power of two, or n above
 * 2^23 / 2^26 / 2^25 for the three primes and 2^26 for the complex rings and GF(p^2)),
 * ENOROOT (f = 0 or f has no n-th root in Z/p; f other than 1 or -1 in GF(p^2)). Complex
 * rings accept any nonzero f; the accuracy statement (relative L2 error near 1e-6 for
 * n <= 2^16) is made for |f| = 1, and the tests also hold f = 2, 0.5i and 1.5 + 0.5i to
 * 1e-5 up to n = 2^15.
 */
fcirc_status fcirc_matvec(fcirc_ctx *ctx, const void *a, const void *x, void *y, uint64_t n,
                          const void *f, fcirc_ring ring, void *stream);

/*
 * fcirc_matvec for callers that cannot allocate device memory (code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid allocation). Same arguments, rings,
 * result and errors as fcirc_matvec, but the call allocates nothing: no hipMalloc/hipFree
 * and no allocating library routine.
 *   - Workspace: the product's intermediate rows (2n elements when n > 2^12) live in one
 *     static device array of FCIRC_NOALLOC_SCRATCH_BYTES per GPU, held by the library from
 *     its first use on that GPU until the process ends. n must fit: ESIZE above 2^22 for
 *     Z/p, 2^21 for FCIRC_C64 and FCIRC_GFP2, 2^20 for FCIRC_R32.
 *   - Plan: the twiddle tables of (ring, f, n) must already be resident in ctx; one earlier
 *     fcirc_matvec with the same ring, f and n on this context builds them (and keeps them
 *     until fcirc_destroy). Otherwise ENOPLAN, with nothing enqueued.
 *   - Every call on one GPU shares that GPU's array and leaves its contents behind (nothing
 *     in it needs to start at zero): calls that may overlap on one GPU, from any context or
 *     stream, race and give unspecified results; order them.
 *   - Per-kernel timing (fcirc_set_timing) creates events; leave it off for this call.
 */
#define FCIRC_NOALLOC_SCRATCH_BYTES (32u << 20)
fcirc_status fcirc_matvec_noalloc(fcirc_ctx *ctx, const void *a, const void *x, void *y, uint64_t n,
                                  const void *f, fcirc_ring ring, void *stream);

/*
 * `count` independent products of the same size n and the same f, stored back to back
 * (instance k at element offset k*n of a, x and y). Same rules as fcirc_matvec.
 * count = 0 enqueues nothing and returns FCIRC_OK (the pointers must still be non-null).
 */
fcirc_status fcirc_matvec_many(fcirc_ctx *ctx, const void *a, const void *x, void *y, uint64_t n,
                               uint32_t count, const void *f, fcirc_ring ring, void *stream);

/*
 * y = A(a, f) x for an f-circulant A of ANY size n >= 1 (Corollary 1, section 2).
 *   a, x, y, f : as for fcirc_matvec, with n elements each (n need not be a power of two).
 * A power-of-two n with an f that has the needed roots runs fcirc_matvec directly.
 * Otherwise the product is embedded in one cyclic product of size N, the smallest power
 * of two >= 2n-1 (for n not a power of two this is the corollary's N = 2^(d+1) with
 * 2^d > n): row (a_0 .. a_(n-1), 0 .. 0, f a_1 .. f a_(n-1)), vector (x, 0 .. 0); the
 * first n entries are y. Here f = 0 is allowed (the upper-triangular Toeplitz part).
 * The library holds 3N elements of workspace for the embedded operands.
 * Errors: EINVAL (null pointer, y overlapping a or x, Z/p f >= p), ESIZE (n = 0, or N
 * above the ring's limit: 2^23 / 2^26 / 2^25 for the three primes, 2^26 complex).
 */
fcirc_status fcirc_matvec_any(fcirc_ctx *ctx, const void *a, const void *x, void *y, uint64_t n,
                              const void *f, fcirc_ring ring, void *stream);

/*
 * y = T x for the n x n Toeplitz matrix T[i][j] = t_(j-i), any n >= 1 (the introduction
 * recalls that a Toeplitz product is a circulant product after embedding; Corollary 1
 * uses the same embedding).
 *   row : device, n elements, row[k] = t_k (the first row).
 *   col : device, n elements, col[k] = t_-k (the first column; col[0] is ignored).
 *   x, y : device, n elements each; y must not overlap row, col or x.
 * Embedded in one cyclic product of size N = smallest power of two >= 2n-1 with row
 * (t_0 .. t_(n-1), 0 .. 0, t_-(n-1) .. t_-1). Same rings, limits and errors as
 * fcirc_matvec_any (no f).
 */
fcirc_status fcirc_toeplitz_matvec(fcirc_ctx *ctx, const void *row, const void *col, const void *x, void *y,
                                   uint64_t n, fcirc_ring ring, void *stream);

/*
 * Exact product of two integer polynomials (section 3.1: a polynomial product is a
 * circulant product after filling up to a power of two).
 *   a : device int32[na], b : device int32[nb], coefficients of degree 0 first.
 *   c : device int64[na+nb-1], written with the exact coefficients.
 * The cyclic length N is the smallest power of two >= na+nb-1 (N <= 2^23). The product
 * is computed modulo 998244353, 469762049 and 167772161 and combined by the Chinese
 * remainder theorem. It is exact when every |c_k| < 998244353*469762049 (about 4.7e17);
 * a coefficient outside that range is written as 0 and makes fcirc_check return ERANGE.
 * EINVAL: null pointers, na = 0 or nb = 0, c overlapping a or b. ESIZE: N above 2^23.
 */
fcirc_status fcirc_polymul_i64(fcirc_ctx *ctx, const int32_t *a, uint64_t na, const int32_t *b,
                               uint64_t nb, int64_t *c, void *stream);

/*
 * Exact product of two non-negative integers given as little-endian 16-bit limbs
 * (section 3.2 applies Algorithm 1 to large integers).
 *   a : device uint16[na], b : device uint16[nb], c : device uint16[na+nb] (written).
 * Requires N = smallest power of two >= na+nb-1 to be <= 2^23 and min(na,nb) <= 2^20.
 * EINVAL: null pointers, na = 0 or nb = 0, c overlapping a or b; ESIZE otherwise.
 */
fcirc_status fcirc_bigint_mul(fcirc_ctx *ctx, const uint16_t *a, uint64_t na, const uint16_t *b,
                              uint64_t nb, uint16_t *c, void *stream);

/*
 * The f-circulant product over Z/(2^K + 1), the ring of section 3.2: there 2^K = -1, so
 * 2 is a root of unity of order 2K, f and every root Algorithm 1 uses are powers of two,
 * and multiplying by a root is a shift by a known count (the roots are never computed).
 *   K       : 2048, 4096, 8192 or 16384 bits.
 *   a, x, y : device arrays of n elements, each K/32 + 1 uint32 words: the K/32 words of
 *             the value (least significant first), then a top word that is 1 only for
 *             the value 2^K. Inputs must be canonical (value in [0, 2^K]; top word 0 or 1,
 *             and 1 only with all other words 0); y is canonical.
 *   f       : 2^f_shift, 0 <= f_shift < 2K (f_shift = 0: cyclic, f_shift = K: f = -1).
 *   n       : a power of two with 2^(L-1) | K (n <= 2^12 K / 2048, i.e. 2^12 .. 2^15).
 * Algorithm 1 needs a power-of-two square root at every node: 2^L must divide f_shift,
 * else ENOROOT. ESIZE: n not a power of two or too large for K. EINVAL: K not listed,
 * f_shift >= 2K, null pointers, overlapping buffers.
 */
fcirc_status fcirc_fermat_matvec(fcirc_ctx *ctx, const uint32_t *a, const uint32_t *x, uint32_t *y,
                                 uint64_t n, uint32_t K, uint32_t f_shift, void *stream);

/*
 * The same product as fcirc_bigint_mul, by the route section 3.2 describes: each factor is
 * cut into pieces that become coefficients over Z/(2^K + 1), one cyclic product of
 * fcirc_fermat_matvec's kind multiplies the two polynomials (pointwise products are full
 * K-bit products at the leaves), and the coefficients are added back with carries. K and
 * the number of pieces are chosen so that no coefficient reaches 2^K.
 *   a : device uint16[na], b : device uint16[nb], c : device uint16[na+nb] (written).
 * Requires na + nb - 1 <= 2^24; ESIZE if no parameter choice fits. EINVAL: null
 * pointers, na = 0 or nb = 0, c overlapping a or b.
 */
fcirc_status fcirc_bigint_mul_fermat(fcirc_ctx *ctx, const uint16_t *a, uint64_t na, const uint16_t *b,
                                     uint64_t nb, uint16_t *c, void *stream);

/*
 * Many independent products of different power-of-two sizes in one persistent launch.
 * items (host array of `count`) give each instance's element offsets into a_base,
 * x_base and y_base and its log2 size (0 <= log2n <= 16). All instances share ring
 * and f. The work queue is built and uploaded on first use of an item list and reused
 * when the same list (same pointers, offsets and sizes) comes again; each call then
 * enqueues two kernels (counter reset, persistent kernel). Calls with one item list
 * share its counters, so they must be ordered on the device (one stream, or streams that
 * wait for each other).
 * count = 0 enqueues nothing and returns FCIRC_OK (the pointers must still be non-null).
 * EINVAL: null pointers, a ring other than the three primes and C64, a nonzero reserved
 * field; ESIZE: log2n > 16.
 */
typedef struct {
  uint64_t a_off, x_off, y_off; /* element offsets */
  uint32_t log2n;
  uint32_t reserved;            /* must be 0 */
} fcirc_item;

fcirc_status fcirc_matvec_batched(fcirc_ctx *ctx, const void *a_base, const void *x_base,
                                  void *y_base, const fcirc_item *items, uint32_t count,
                                  const void *f, fcirc_ring ring, void *stream);

/*
 * Parameters of fcirc_matvec_batched for its instances of size n (a power of two <= 2^16)
 * over `ring` (the three primes or FCIRC_C64), as fcirc_tune sets them.
 *   workgroup    : 256 or 512 threads (16 elements per thread per stage); -1 drops the
 *                  setting of this size (back to the defaults).
 *   block_levels : 0 = each instance is one work item (split, leaf products and merge in
 *                  one workgroup; n <= 2^12 at 256 threads, n <= 2^13 at 512), or the levels
 *                  of the LDS-resident block of the three-pass form (10 .. 12 at 256 threads,
 *                  10 .. 13 at 512; n >= 2^12 resp. 2^13 and at most 6 levels above the block).
 * A launch uses 512 threads when the sizes in it whose times fcirc_tune measured (or that
 * this call set: the given workgroup size counts as the faster) favour it, weighted by
 * their coefficients; each size then takes its parameters for that workgroup size, and a
 * size without them the default (one item up to n = 2^12, resp. 2^13, else blocks of 2^12).
 * Defaults without any setting: 256 threads. EINVAL for other values.
 * fcirc_get_batch_schedule reports what a launch of instances of size n alone would use;
 * it returns 0, or -1 for invalid arguments.
 */
fcirc_status fcirc_set_batch_schedule(fcirc_ctx *ctx, fcirc_ring ring, uint64_t n, int workgroup,
                                      int block_levels);
int fcirc_get_batch_schedule(fcirc_ctx *ctx, fcirc_ring ring, uint64_t n, int *workgroup,
                             int *block_levels);

/*
 * Circulant layer over a batch with one shared row (f = 1; rings C64 or R32; 16 <= n <= 2^24):
 *   forward : y[b] = C(a) x[b] for b < batch (x, y: batch*n elements, row-major).
 *   backward: gx[b] = C(a)^H gy[b] and ga = sum_b C(gy[b]) conj(x[b]), i.e. the
 *             gradients of a real loss with upstream gradient gy (PyTorch's convention
 *             for complex tensors; the conjugates drop out for real data).
 * ga or gx may be NULL to skip that gradient.
 * EINVAL: null pointers (x is needed when ga is asked for), batch = 0, another ring;
 * ESIZE: n not a power of two in [16, 2^24].
 */
fcirc_status fcirc_matvec_fwd_shared(fcirc_ctx *ctx, const void *a, const void *x, void *y,
                                     uint64_t n, uint32_t batch, fcirc_ring ring, void *stream);
fcirc_status fcirc_matvec_backward(fcirc_ctx *ctx, const void *a, const void *x, const void *gy,
                                   void *ga, void *gx, uint64_t n, uint32_t batch,
                                   fcirc_ring ring, void *stream);

/* Synchronise `stream` and return (then clear) the sticky device status: ESCHED if a
 * batched launch gave up a dependency wait since the last check, else ERANGE if a CRT
 * result was out of range, else OK. */
fcirc_status fcirc_check(fcirc_ctx *ctx, void *stream);

/*
 * Debugging checks of a context; `flags` is a set of the bits below (0 turns all off).
 * Their defaults come from the environment at fcirc_create: FCIRC_VALIDATE=1 sets
 * FCIRC_CHECK_INPUTS, FCIRC_DEBUG_SYNC=1 sets FCIRC_CHECK_SYNC.
 *   FCIRC_CHECK_INPUTS: the Z/p and GF(p^2) products (fcirc_matvec, fcirc_matvec_many,
 *     fcirc_matvec_any, fcirc_toeplitz_matvec, fcirc_matvec_batched) take canonical inputs,
 *     every word in [0,p), and fcirc_fermat_matvec canonical elements (top word 0 or 1, and
 *     1 only with all other words 0); results are unspecified otherwise. With this bit, a
 *     kernel first checks every input of the call; the call then synchronises the stream
 *     and returns FCIRC_EINVAL, having written no output, when one is not canonical. Because
 *     it synchronises, it cannot be used while the stream is being captured into a graph.
 *   FCIRC_CHECK_SYNC: synchronise the stream after every kernel the library launches and
 *     return FCIRC_EDEVICE at the first failed one.
 * Returns FCIRC_EINVAL for a null context or unknown bits.
 */
#define FCIRC_CHECK_INPUTS 1
#define FCIRC_CHECK_SYNC 2
fcirc_status fcirc_set_checks(fcirc_ctx *ctx, int flags);

/*
 * Per-kernel timing with HIP events recorded on the caller's stream around each kernel
 * the library launches (for measurement; off by default). fcirc_stage_times
 * synchronises, then writes up to `max` entries: the kernel name, the number of launches
 * and the summed milliseconds since the last reset. Returns the number of kernel names.
 */
fcirc_status fcirc_set_timing(fcirc_ctx *ctx, int enable);
int fcirc_stage_times(fcirc_ctx *ctx, const char **names, uint64_t *launches, double *ms, int max);

/*
 * Tuning. fcirc_tune times the candidate split points and tile shapes for one
 * (ring, n) on scratch buffers and keeps the fastest for later calls with this context.
 * For the three primes and FCIRC_C64 with n <= 2^16 it also tunes fcirc_matvec_batched for
 * instances of size n (see fcirc_set_batch_schedule): on a scratch batch of
 * max(1, 2^24 / n) such instances (at most 4096) it times every valid form at both
 * workgroup sizes and keeps, per workgroup size, the fastest form and its time per
 * coefficient.
 * fcirc_set_split forces the number of top levels streamed through HBM before the
 * LDS-resident block (0 = single block kernel when it fits; -1 = back to automatic).
 * fcirc_get_split reports the split that fcirc_matvec would use for (ring, n).
 */
fcirc_status fcirc_tune(fcirc_ctx *ctx, uint64_t n, fcirc_ring ring, void *stream);
fcirc_status fcirc_set_split(fcirc_ctx *ctx, int top_levels);
int fcirc_get_split(fcirc_ctx *ctx, uint64_t n, fcirc_ring ring);
/*
 * Set the schedule for (ring, n) explicitly, as fcirc_tune would: top_levels (-1 default),
 * tile_log = log2 elements of a top-pass tile (-1 default, at most 14 for Z/p and 13 for the
 * complex rings), flags = a bitwise
 * OR of FCIRC_SCHED_* (0..7; the default is FCIRC_SCHED_XCD). fcirc_get_schedule reports
 * the schedule in use and returns the number of top passes.
 *   FCIRC_SCHED_XCD       top-pass tiles in XCD-aware order (neighbouring column tiles on
 *                         one XCD, so they share its L2)
 *   FCIRC_SCHED_SEPARATE  the split passes take the row and the vector in separate
 *                         workgroups (default: one workgroup splits the same tile of both)
 *   FCIRC_SCHED_SMALL     a product with no top pass and 2^6 <= n <= 2^12 runs as one
 *                         workgroup of several waves per instance (radix-4 register
 *                         stages, every twiddle in LDS) instead of the single-wave block
 *                         pass; ignored for other sizes
 */
#define FCIRC_SCHED_XCD 1
#define FCIRC_SCHED_SEPARATE 2
#define FCIRC_SCHED_SMALL 4
fcirc_status fcirc_set_schedule(fcirc_ctx *ctx, fcirc_ring ring, uint64_t n, int top_levels, int tile_log, int flags);
int fcirc_get_schedule(fcirc_ctx *ctx, fcirc_ring ring, uint64_t n, int *top_levels, int *tile_log, int *flags);

/*
 * Schedules chosen by fcirc_tune or fcirc_set_schedule kept in a text file, one line per
 * (ring, n): "<arch> <compute units> <ring> <log2 n> <top_levels> <tile_log> <flags>", and
 * the batched-launch parameters of fcirc_tune or fcirc_set_batch_schedule, one line per
 * (ring, n): "<arch> <compute units> batch <ring> <log2 n> <block_levels at 256 threads>
 * <ns per coefficient> <block_levels at 512 threads> <ns per coefficient>" (block levels
 * -1: not set).
 * fcirc_save_schedules writes every schedule the context holds (replacing the file).
 * fcirc_load_schedules reads such a file and takes the lines written for this device's
 * architecture and compute-unit count (other lines are skipped). A file that cannot be
 * read, or holds a malformed or out-of-range line, returns FCIRC_EINVAL and changes
 * nothing: the context keeps its schedules and defaults. fcirc_create loads the file named
 * by the environment variable FCIRC_TUNE_FILE, if set; when that fails it prints one
 * warning to stderr and keeps the defaults.
 */
fcirc_status fcirc_save_schedules(fcirc_ctx *ctx, const char *path);
fcirc_status fcirc_load_schedules(fcirc_ctx *ctx, const char *path);

#ifdef __cplusplus
}
#endif
#endif /* FCIRC_H */
