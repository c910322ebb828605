"""Reference gradients of the circulant layer y = C(a) x (test infrastructure only).

The layer is the f = 1 case of the product (Definition 2 with f = 1, a row-identified
circulant): y_i = sum_k a_k x_((i+k) mod n), applied to each row of a batch with one
shared a. Gradients follow PyTorch's conventions; for complex tensors the gradient of a
real loss is the conjugate Wirtinger one (grad = M^H g for y = M x).

Two independent references, both FP64 on the CPU:
* ``dense_autograd``: the dense matrix built by index gather, differentiated by torch.
* ``finite_differences``: central differences of the loss sum(g * y) for real data.
"""
from __future__ import annotations

import numpy as np
import torch


def _dense(a: torch.Tensor) -> torch.Tensor:
    n = a.shape[0]
    i = torch.arange(n)[:, None]
    j = torch.arange(n)[None, :]
    return a[(j - i) % n]  # f = 1: A[i][j] = a[(j - i) mod n]


def dense_forward(a, x):
    """y (batch, n) = x @ A^T for each row of x, FP64/complex128 on the CPU."""
    at = torch.as_tensor(np.asarray(a)).to(torch.complex128 if np.iscomplexobj(a) else torch.float64)
    xt = torch.as_tensor(np.asarray(x)).to(at.dtype)
    return (xt @ _dense(at).T).numpy()


def dense_autograd(a, x, g):
    """(y, grad_a, grad_x) of L = Re sum(conj(g) * y) via torch autograd on the dense matrix.

    For real inputs this is L = sum(g * y), so grad_a = dL/da and grad_x = dL/dx.
    """
    cplx = np.iscomplexobj(a) or np.iscomplexobj(x) or np.iscomplexobj(g)
    dt = torch.complex128 if cplx else torch.float64
    at = torch.as_tensor(np.asarray(a)).to(dt).clone().requires_grad_(True)
    xt = torch.as_tensor(np.asarray(x)).to(dt).clone().requires_grad_(True)
    gt = torch.as_tensor(np.asarray(g)).to(dt)
    y = xt @ _dense(at).T
    y.backward(gt)
    return y.detach().numpy(), at.grad.numpy(), xt.grad.numpy()


def layer_entries(a, x, g, idx):
    """Entries i in idx of y (every row), grad_x (every row) and grad_a, each by its O(n)
    sum (FP64/complex128), for sizes where the whole vectors are too costly on the CPU:
      y[b, i]      = sum_k a_k x_b[(i + k) mod n]               (Definition 2, f = 1)
      grad_x[b, i] = sum_k conj(a_k) g_b[(i - k) mod n]          (column i of C(a)^H)
                   = sum_k r_k g_b[(i + k) mod n], r_k = conj(a_((-k) mod n))
      grad_a[i]    = sum_b sum_j g_b[j] conj(x_b[(j + i) mod n]) (y_b[j] depends on a_i
                                                                  through x_b[(j + i) mod n])
    A cyclic shift by i is two contiguous pieces, so every sum is two dot products.
    Returns arrays of shape (batch, len(idx)), (len(idx),), (batch, len(idx))."""
    cplx = np.iscomplexobj(a) or np.iscomplexobj(x) or np.iscomplexobj(g)
    dt = np.complex128 if cplx else np.float64
    a = np.asarray(a, dtype=dt)
    x = np.atleast_2d(np.asarray(x, dtype=dt))
    g = np.atleast_2d(np.asarray(g, dtype=dt))
    n = a.shape[0]
    r = np.conj(np.concatenate([a[:1], a[:0:-1]]))  # r_k = conj(a_((-k) mod n))

    def shifted_dot(u, v, i):  # sum_k u_k v_((i + k) mod n)
        return np.dot(u[:n - i], v[i:]) + np.dot(u[n - i:], v[:i])

    y = np.array([[shifted_dot(a, xb, int(i)) for i in idx] for xb in x])
    gx = np.array([[shifted_dot(r, gb, int(i)) for i in idx] for gb in g])
    # sum_j g_j conj(x_(j+i)): np.vdot conjugates its first argument
    ga = np.array([sum(np.vdot(xb[int(i):], gb[:n - int(i)]) + np.vdot(xb[:int(i)], gb[n - int(i):])
                       for gb, xb in zip(g, x)) for i in idx])
    return y, ga, gx


def finite_differences(a, x, g, h: float = 1e-6):
    """Central differences of L = sum(g * y(a, x)) for real a (n,), x (batch, n)."""
    a = np.asarray(a, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)

    def loss(a_, x_):
        return float((g * dense_forward(a_, x_)).sum())

    ga = np.zeros_like(a)
    for k in range(a.shape[0]):
        e = np.zeros_like(a)
        e[k] = h
        ga[k] = (loss(a + e, x) - loss(a - e, x)) / (2 * h)
    gx = np.zeros_like(x)
    for idx in np.ndindex(*x.shape):
        e = np.zeros_like(x)
        e[idx] = h
        gx[idx] = (loss(a, x + e) - loss(a, x - e)) / (2 * h)
    return ga, gx


def grads_fft(a, x, g):
    """(y, grad_a, grad_x) of the layer through the f = 1 DFT identity (large n).

    Uses y_b = C(a) x_b, grad_x_b = C(a)^H g_b = C(conj(rev a)) g_b and
    grad_a = sum_b C(g_b) conj(x_b), each product computed by
    ``fcirc.cyclic_matvec_fft_c128``. The tests pin this against ``dense_autograd``.
    """
    from .fcirc import cyclic_matvec_fft_c128
    a = np.asarray(a)
    x = np.atleast_2d(np.asarray(x))
    g = np.atleast_2d(np.asarray(g))
    cplx = np.iscomplexobj(a) or np.iscomplexobj(x) or np.iscomplexobj(g)
    n = a.shape[0]
    rev_conj_a = np.conj(a[(-np.arange(n)) % n])
    y = np.stack([cyclic_matvec_fft_c128(a, xb) for xb in x])
    gx = np.stack([cyclic_matvec_fft_c128(rev_conj_a, gb) for gb in g])
    ga = sum(cyclic_matvec_fft_c128(gb, np.conj(xb)) for gb, xb in zip(g, x))
    if not cplx:
        return y.real, ga.real, gx.real
    return y, ga, gx
