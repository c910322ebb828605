"""Batched products of different sizes in one persistent launch (fcirc_matvec_batched).

Instances are packed back to back into three device buffers (rows, vectors, results);
the item list gives each instance's element offsets and log2 size. The library builds
the work queue the first time it sees an item list and keeps it, so a BatchPlan that is
run repeatedly (with new inputs loaded into the same buffers) costs two kernel launches
per run (counter reset, persistent kernel).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .fcirc import RING_OF_PRIME, context


class BatchPlan:
    """Device buffers and item list for a fixed batch shape."""

    def __init__(self, a_list, x_list, dtype=np.complex64, p: int | None = None, f=None, device=None):
        if len(a_list) != len(x_list) or not a_list:
            raise ValueError("a_list and x_list must be non-empty lists of equal length")
        self.sizes = [int(np.asarray(a).shape[0]) for a in a_list]
        for n, x in zip(self.sizes, x_list):
            if n & (n - 1) or np.asarray(x).shape[0] != n:
                raise ValueError("each instance needs power-of-two row and vector of equal length")
        self.p = p
        if p is not None:
            self.ring = RING_OF_PRIME[p]
            self.f = C.c_uint32(1 if f is None else int(f) % p)
            self.tdtype, self.ndtype = torch.int32, np.uint32
        else:
            fc = complex(1.0 if f is None else f)
            self.ring = L.FCIRC_C64
            self.f = (C.c_double * 2)(fc.real, fc.imag)
            self.tdtype, self.ndtype = torch.complex64, np.complex64
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        total = int(self.offsets[-1])
        dev = torch.device("cuda") if device is None else torch.device(device)
        self.a = torch.empty(total, dtype=self.tdtype, device=dev)
        self.x = torch.empty(total, dtype=self.tdtype, device=dev)
        self.y = torch.empty(total, dtype=self.tdtype, device=dev)
        items = (L.fcirc_item * len(self.sizes))()
        for k, n in enumerate(self.sizes):
            off = int(self.offsets[k])
            items[k].a_off = off
            items[k].x_off = off
            items[k].y_off = off
            items[k].log2n = n.bit_length() - 1
            items[k].reserved = 0
        self.items = items
        self.load(a_list, x_list)

    def _pack(self, arrs):
        flat = np.concatenate([np.asarray(v, dtype=self.ndtype) for v in arrs])
        if self.ndtype == np.uint32:
            flat = flat.view(np.int32)
        return torch.from_numpy(np.ascontiguousarray(flat))

    def load(self, a_list, x_list):
        """Copy new inputs (same sizes) into the plan's device buffers."""
        self.a.copy_(self._pack(a_list))
        self.x.copy_(self._pack(x_list))

    def run(self, stream=None, check: bool = False):
        """Enqueue the batch. With check=True, also wait for it and raise FcircError (ESCHED)
        if a work item gave up waiting for the items it depends on (see check())."""
        ctx = context(self.a.device)
        with ctx.enqueue(stream) as s:
            L.check(L.lib().fcirc_matvec_batched(ctx.handle, C.c_void_p(self.a.data_ptr()), C.c_void_p(self.x.data_ptr()),
                                                 C.c_void_p(self.y.data_ptr()), self.items, len(self.sizes),
                                                 C.byref(self.f), self.ring, s),
                    "fcirc_matvec_batched")
        if check:
            self.check(stream)
        return self.y

    def check(self, stream=None):
        """Synchronise and raise FcircError if the device status of the context reports a
        failure (ESCHED: a dependency wait of a batched launch gave up)."""
        ctx = context(self.a.device)
        with ctx.enqueue(stream) as s:
            L.check(L.lib().fcirc_check(ctx.handle, s), "fcirc_check")

    def outputs(self):
        """Per-instance results as host numpy arrays."""
        flat = self.y.cpu().numpy()
        if self.ndtype == np.uint32:
            flat = flat.view(np.uint32).astype(np.int64)
        return [flat[self.offsets[k]:self.offsets[k + 1]] for k in range(len(self.sizes))]


def matvec_batched_c64(a_list, x_list, f=None):
    plan = BatchPlan(a_list, x_list, dtype=np.complex64, f=f)
    plan.run(check=True)
    return plan.outputs()


def matvec_batched_modp(a_list, x_list, p: int, f=1):
    plan = BatchPlan(a_list, x_list, p=p, f=f)
    plan.run(check=True)
    return plan.outputs()
