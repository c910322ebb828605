"""Python API of libfcirc over torch tensors (argument marshalling only).

Every computation runs in the HIP library; torch provides device memory and the stream
(the current torch stream of the tensors' device is passed to each call).

Conventions (Rosowski, arXiv 2103.02605):
* The f-circulant matrix A(a, f) is identified by its FIRST ROW a (section 1.2):
  A[i][j] = a[j-i] for j >= i and f * a[n+j-i] for j < i (Definition 2).
* ``matvec(a, x, f)`` returns y = A(a, f) x (Theorem 1, Algorithm 1).
* Z/p: pass ``p`` (998244353, 469762049 or 167772161) and int32/uint32 tensors with
  values in [0, p); complex64 tensors use the complex ring; float32 tensors the real one.
"""
from __future__ import annotations

import ctypes as C
import threading

import torch

from . import _lib as L

P1, P2, P3 = 998244353, 469762049, 167772161
RING_OF_PRIME = {P1: L.FCIRC_ZP_998244353, P2: L.FCIRC_ZP_469762049, P3: L.FCIRC_ZP_167772161}
P_GF = (1 << 31) - 1  # GF(p^2) = Z/p[sqrt 3] of section 3.1: tensors (..., 2) int32 holding (a, b)


class Context:
    """A libfcirc context on one HIP device (plans, workspaces, batched work queues).

    The library requires calls that share a context to be serialised, and their device
    work to be ordered (they share the context's workspace). enqueue() does both for the
    calls of this module: it holds a lock for the call, and makes the current stream wait
    for the stream of the context's previous call when the two differ."""

    def __init__(self, device: int = 0):
        self.device = device
        self.lock = threading.RLock()
        self._last_stream = None
        h = C.c_void_p()
        L.check(L.lib().fcirc_create(C.byref(h), device), "fcirc_create")
        self.handle = h

    def enqueue(self, stream: torch.cuda.Stream | None = None) -> "_Enqueue":
        """Hold the context for one call on `stream` (default: the current stream of the
        context's device); the with-statement yields that stream as the library's argument."""
        return _Enqueue(self, stream)

    def close(self):
        if self.handle:
            L.lib().fcirc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# The raw handle of a device's current stream, without building a Stream object (the
# common case needs only the handle; Stream objects are built when the stream changes).
_raw_current_stream = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _current_stream_handle(device: int) -> int:
    if _raw_current_stream is not None:
        return _raw_current_stream(device)
    return torch.cuda.current_stream(device).cuda_stream


class _Enqueue:
    """Context manager of Context.enqueue (a class: it runs on every call)."""
    __slots__ = ("ctx", "stream", "handle")

    def __init__(self, ctx: Context, stream):
        self.ctx, self.stream, self.handle = ctx, stream, None

    def __enter__(self) -> C.c_void_p:
        ctx = self.ctx
        ctx.lock.acquire()
        try:
            h = self.stream.cuda_stream if self.stream is not None else _current_stream_handle(ctx.device)
            last = ctx._last_stream
            if last is not None and last != h:
                cur = self.stream if self.stream is not None else torch.cuda.current_stream(ctx.device)
                cur.wait_stream(torch.cuda.ExternalStream(last, device=ctx.device))
        except BaseException:
            ctx.lock.release()
            raise
        self.handle = h
        return h  # ctypes passes an int as the stream's void*

    def __exit__(self, *exc):
        self.ctx._last_stream = self.handle  # raw handle of the stream of this call
        self.ctx.lock.release()
        return False


_contexts: dict[int, Context] = {}
_contexts_lock = threading.Lock()


def context(device=None) -> Context:
    if isinstance(device, int):  # a device index (Tensor.get_device(); -1 for host tensors)
        idx = max(device, 0)
    else:
        idx = torch.cuda.current_device() if device is None else torch.device(device).index or 0
    c = _contexts.get(idx)
    if c is not None:
        return c
    with _contexts_lock:
        if idx not in _contexts:
            _contexts[idx] = Context(idx)
        return _contexts[idx]


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()  # ctypes passes an int as void*


def _need(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ring_and_f(t: torch.Tensor, f, p):
    """(ring id, ctypes value of f) for a data tensor t."""
    if p == P_GF:
        if t.dtype != torch.int32 or t.shape[-1] != 2:
            raise TypeError("GF(p^2) data must be int32 tensors of shape (..., 2) holding (a, b) in [0, p)")
        fv = 1 if f is None else int(f) % P_GF
        return L.FCIRC_GFP2, (C.c_uint32 * 2)(fv, 0)
    if p is not None:
        if p not in RING_OF_PRIME:
            raise ValueError(f"unsupported prime {p}")
        if t.dtype not in (torch.int32, torch.uint32):
            raise TypeError("Z/p data must be int32 or uint32 tensors holding values in [0, p)")
        fv = int(f) % p if f is not None else 1
        return RING_OF_PRIME[p], C.c_uint32(fv)
    if t.dtype == torch.complex64:
        fc = complex(1.0 if f is None else f)
        return L.FCIRC_C64, (C.c_double * 2)(fc.real, fc.imag)
    if t.dtype == torch.float32:
        return L.FCIRC_R32, C.c_double(1.0 if f is None else float(f))
    raise TypeError(f"unsupported dtype {t.dtype}")


def matvec(a: torch.Tensor, x: torch.Tensor, f=None, p: int | None = None, out: torch.Tensor | None = None):
    """y = A(a, f) x for one product of power-of-two size n (Definition 2, Algorithm 1).

    p selects Z/p (int32/uint32 tensors of n residues) or, with p = 2^31 - 1, the ring of
    section 3.1 (int32 tensors of shape (n, 2), f = 1 or -1); otherwise complex64 or
    float32 tensors."""
    _need(a, "a")
    _need(x, "x")
    ring, fv = _ring_and_f(a, f, p)
    vdim = 2 if ring == L.FCIRC_GFP2 else 1
    if a.shape != x.shape or a.dim() != vdim or a.dtype != x.dtype:
        raise ValueError("a and x must be tensors of the same shape and dtype, one vector each")
    y = torch.empty_like(a) if out is None else out
    _need(y, "out")
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_matvec(ctx.handle, _ptr(a), _ptr(x), _ptr(y), a.shape[0], C.byref(fv), ring, s),
                "fcirc_matvec")
    return y


def matvec_any(a: torch.Tensor, x: torch.Tensor, f=None, p: int | None = None, out: torch.Tensor | None = None):
    """y = A(a, f) x for any size n >= 1 (Corollary 1's embedding when n is not a power of
    two, or when f lacks the roots the direct recursion needs)."""
    _need(a, "a")
    _need(x, "x")
    if a.shape != x.shape or a.dim() != 1 or a.dtype != x.dtype:
        raise ValueError("a and x must be 1-D tensors of the same shape and dtype")
    ring, fv = _ring_and_f(a, f, p)
    y = torch.empty_like(a) if out is None else out
    _need(y, "out")
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_matvec_any(ctx.handle, _ptr(a), _ptr(x), _ptr(y), a.numel(), C.byref(fv), ring, s),
                "fcirc_matvec_any")
    return y


def toeplitz_matvec(row: torch.Tensor, col: torch.Tensor, x: torch.Tensor, p: int | None = None,
                    out: torch.Tensor | None = None):
    """y = T x with T[i][j] = row[j - i] for j >= i and col[i - j] for j < i (col[0] unused)."""
    for t, name in ((row, "row"), (col, "col"), (x, "x")):
        _need(t, name)
    if not (row.shape == col.shape == x.shape) or row.dim() != 1 or not (row.dtype == col.dtype == x.dtype):
        raise ValueError("row, col and x must be 1-D tensors of the same shape and dtype")
    ring, _ = _ring_and_f(row, None, p)
    y = torch.empty_like(row) if out is None else out
    _need(y, "out")
    ctx = context(row.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_toeplitz_matvec(ctx.handle, _ptr(row), _ptr(col), _ptr(x), _ptr(y), row.numel(), ring,
                                              s), "fcirc_toeplitz_matvec")
    return y


def matvec_many(a: torch.Tensor, x: torch.Tensor, f=None, p: int | None = None, out: torch.Tensor | None = None):
    """Row k of the result is A(a[k], f) x[k]; a and x have shape (count, n) (or
    (count, n, 2) for the ring of section 3.1)."""
    _need(a, "a")
    _need(x, "x")
    ring, fv = _ring_and_f(a, f, p)
    vdim = 3 if ring == L.FCIRC_GFP2 else 2
    if a.shape != x.shape or a.dim() != vdim or a.dtype != x.dtype:
        raise ValueError("a and x must be tensors (count, n) of the same shape and dtype")
    y = torch.empty_like(a) if out is None else out
    if a.shape[0] == 0:  # an empty batch: nothing to compute (empty tensors have null pointers)
        return y
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_matvec_many(ctx.handle, _ptr(a), _ptr(x), _ptr(y), a.shape[1], a.shape[0], C.byref(fv),
                                          ring, s), "fcirc_matvec_many")
    return y


def polymul_i64(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None):
    """Exact int64 coefficients of the product of two int32 polynomials (section 3.1)."""
    _need(a, "a")
    _need(b, "b")
    if a.dtype != torch.int32 or b.dtype != torch.int32:
        raise TypeError("polymul_i64 takes int32 coefficient tensors")
    c = torch.empty(a.numel() + b.numel() - 1, dtype=torch.int64, device=a.device) if out is None else out
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_polymul_i64(ctx.handle, _ptr(a), a.numel(), _ptr(b), b.numel(), _ptr(c), s),
                "fcirc_polymul_i64")
    return c


def bigint_mul(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None):
    """Limbs (little-endian, 16-bit) of the product of two non-negative integers."""
    _need(a, "a")
    _need(b, "b")
    if a.dtype not in (torch.uint16, torch.int16) or b.dtype != a.dtype:
        raise TypeError("bigint_mul takes uint16 (or int16-viewed) limb tensors")
    c = torch.empty(a.numel() + b.numel(), dtype=a.dtype, device=a.device) if out is None else out
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_bigint_mul(ctx.handle, _ptr(a), a.numel(), _ptr(b), b.numel(), _ptr(c), s),
                "fcirc_bigint_mul")
    return c


def fermat_matvec(a: torch.Tensor, x: torch.Tensor, K: int, f_shift: int = 0, out: torch.Tensor | None = None):
    """y = A(a, 2^f_shift) x over Z/(2^K + 1) (section 3.2's ring; roots are shifts).

    a, x: int32/uint32 tensors of shape (n, K/32 + 1), one element per row: K/32 words of
    the value (least significant first), then the top word (1 only for the value 2^K)."""
    _need(a, "a")
    _need(x, "x")
    if a.dtype not in (torch.int32, torch.uint32) or a.dim() != 2 or a.shape != x.shape or a.dtype != x.dtype:
        raise ValueError("a and x must be (n, K/32 + 1) int32 tensors of the same shape")
    if a.shape[1] != K // 32 + 1:
        raise ValueError(f"elements of Z/(2^{K} + 1) take {K // 32 + 1} words")
    y = torch.empty_like(a) if out is None else out
    _need(y, "out")
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_fermat_matvec(ctx.handle, _ptr(a), _ptr(x), _ptr(y), a.shape[0], int(K), int(f_shift),
                                            s), "fcirc_fermat_matvec")
    return y


def bigint_mul_fermat(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None):
    """bigint_mul by section 3.2's route: one cyclic product over Z/(2^K + 1)."""
    _need(a, "a")
    _need(b, "b")
    if a.dtype not in (torch.int16, torch.uint16) or b.dtype != a.dtype:
        raise TypeError("bigint_mul_fermat takes uint16 (or int16-viewed) limb tensors")
    c = torch.empty(a.numel() + b.numel(), dtype=a.dtype, device=a.device) if out is None else out
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_bigint_mul_fermat(ctx.handle, _ptr(a), a.numel(), _ptr(b), b.numel(), _ptr(c), s),
                "fcirc_bigint_mul_fermat")
    return c


def check(device=None):
    """Synchronise the current stream and raise on a sticky device-side error (ERANGE)."""
    ctx = context(device)
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_check(ctx.handle, s), "fcirc_check")


CHECK_INPUTS = 1  # Z/p and GF(p^2) inputs must be canonical; EINVAL otherwise (synchronises)
CHECK_SYNC = 2    # synchronise after every kernel


def set_checks(flags: int, device=None):
    """Debugging checks of the device's context (defaults: FCIRC_VALIDATE, FCIRC_DEBUG_SYNC)."""
    ctx = context(device)
    with ctx.lock:
        L.check(L.lib().fcirc_set_checks(ctx.handle, int(flags)), "fcirc_set_checks")


def set_timing(enable: bool, device=None):
    ctx = context(device)
    with ctx.lock:
        L.check(L.lib().fcirc_set_timing(ctx.handle, int(bool(enable))), "fcirc_set_timing")


def stage_times(device=None) -> dict:
    """{kernel name: (launches, total ms)} since the last set_timing()."""
    ctx = context(device)
    with ctx.lock:
        n = L.lib().fcirc_stage_times(ctx.handle, None, None, None, 0)
        names = (C.c_char_p * max(n, 1))()
        launches = (C.c_uint64 * max(n, 1))()
        ms = (C.c_double * max(n, 1))()
        n = L.lib().fcirc_stage_times(ctx.handle, names, launches, ms, n)
    return {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(n)}


def set_split(top_levels: int, device=None):
    ctx = context(device)
    with ctx.lock:
        L.check(L.lib().fcirc_set_split(ctx.handle, int(top_levels)), "fcirc_set_split")


def get_split(n: int, ring: int, device=None) -> int:
    ctx = context(device)
    with ctx.lock:
        return int(L.lib().fcirc_get_split(ctx.handle, n, ring))


def tune(n: int, ring: int, device=None):
    ctx = context(device)
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_tune(ctx.handle, n, ring, s), "fcirc_tune")


SCHED_XCD = 1       # XCD-aware tile order in the top passes
SCHED_SEPARATE = 2  # split passes take the row and the vector in separate workgroups
SCHED_SMALL = 4     # 2^6..2^12 with no top pass: one several-wave workgroup per instance


def set_schedule(n: int, ring: int, top_levels: int = -1, tile_log: int = -1, flags: int = SCHED_XCD, device=None):
    """Fix the pass schedule for (ring, n): see fcirc_set_schedule in include/fcirc.h."""
    ctx = context(device)
    with ctx.lock:
        L.check(L.lib().fcirc_set_schedule(ctx.handle, ring, n, top_levels, tile_log, flags), "fcirc_set_schedule")


def save_schedules(path: str, device=None):
    """Write the device context's tuned/set schedules to a text file."""
    ctx = context(device)
    with ctx.lock:
        L.check(L.lib().fcirc_save_schedules(ctx.handle, str(path).encode()), "fcirc_save_schedules")


def load_schedules(path: str, device=None):
    """Take the schedules a file holds for this device (EINVAL and no change if malformed)."""
    ctx = context(device)
    with ctx.lock:
        L.check(L.lib().fcirc_load_schedules(ctx.handle, str(path).encode()), "fcirc_load_schedules")


def get_schedule(n: int, ring: int, device=None) -> dict:
    top, tile, flags = C.c_int(), C.c_int(), C.c_int()
    ctx = context(device)
    with ctx.lock:
        ntop = L.lib().fcirc_get_schedule(ctx.handle, ring, n, C.byref(top), C.byref(tile), C.byref(flags))
    return {"top_passes": ntop, "top_levels": top.value, "tile_log": tile.value, "flags": flags.value}


def set_batch_schedule(n: int, ring: int, workgroup: int, block_levels: int = 0, device=None):
    """Fix the batched launch's parameters for instances of size n: see
    fcirc_set_batch_schedule in include/fcirc.h (workgroup -1 drops the setting)."""
    ctx = context(device)
    with ctx.lock:
        L.check(L.lib().fcirc_set_batch_schedule(ctx.handle, ring, n, workgroup, block_levels),
                "fcirc_set_batch_schedule")


def get_batch_schedule(n: int, ring: int, device=None) -> dict:
    """What a batched launch of instances of size n alone uses: workgroup size and block
    levels (0: one work item per instance)."""
    wg, bl = C.c_int(), C.c_int()
    ctx = context(device)
    with ctx.lock:
        if L.lib().fcirc_get_batch_schedule(ctx.handle, ring, n, C.byref(wg), C.byref(bl)) != 0:
            raise ValueError("invalid ring or size for the batched launch")
    return {"workgroup": wg.value, "block_levels": bl.value}


# -------------------------------------------------------------------------------------
# Circulant layer (f = 1) with a hand-written backward: fcirc_matvec_fwd_shared and
# fcirc_matvec_backward. x has shape (batch, n) and a shape (n,), float32 or complex64.
# -------------------------------------------------------------------------------------

def _layer_ring(a: torch.Tensor):
    if a.dtype == torch.float32:
        return L.FCIRC_R32
    if a.dtype == torch.complex64:
        return L.FCIRC_C64
    raise TypeError("the circulant layer takes float32 or complex64 tensors")


def layer_forward(a: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """y[b] = C(a) x[b] for every row b (one shared defining row, f = 1)."""
    _need(a, "a")
    _need(x, "x")
    if x.dim() != 2 or a.dim() != 1 or x.shape[1] != a.shape[0] or x.dtype != a.dtype:
        raise ValueError("a must be (n,) and x (batch, n) of the same dtype")
    y = torch.empty_like(x)
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_matvec_fwd_shared(ctx.handle, _ptr(a), _ptr(x), _ptr(y), a.shape[0], x.shape[0],
                                                _layer_ring(a), s), "fcirc_matvec_fwd_shared")
    return y


def layer_backward(a: torch.Tensor, x: torch.Tensor, gy: torch.Tensor, need_a: bool = True, need_x: bool = True):
    """(grad_a, grad_x) of a real loss whose gradient with respect to y is gy."""
    _need(a, "a")
    _need(x, "x")
    _need(gy, "gy")
    ga = torch.empty_like(a) if need_a else None
    gx = torch.empty_like(x) if need_x else None
    ctx = context(a.get_device())
    with ctx.enqueue() as s:
        L.check(L.lib().fcirc_matvec_backward(ctx.handle, _ptr(a), _ptr(x), _ptr(gy),
                                              _ptr(ga) if ga is not None else None,
                                              _ptr(gx) if gx is not None else None,
                                              a.shape[0], x.shape[0], _layer_ring(a), s),
                "fcirc_matvec_backward")
    return ga, gx


class CirculantFn(torch.autograd.Function):
    """y = C(a) x row by row (f = 1) with the gradients computed by the library."""

    @staticmethod
    def forward(ctx, a, x):
        a = a.contiguous()
        x = x.contiguous()
        ctx.save_for_backward(a, x)
        return layer_forward(a, x)

    @staticmethod
    def backward(ctx, gy):
        a, x = ctx.saved_tensors
        ga, gx = layer_backward(a, x, gy.contiguous(), ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return ga, gx


def circulant(a: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Differentiable circulant layer: rows of x multiplied by the circulant with first row a."""
    return CirculantFn.apply(a, x)
