"""Calls that share the device's context from several torch streams and host threads.

The library's calls share the context's workspace and require serialised, ordered use;
the Python binding orders a call after the previous call's stream and holds a lock for
each call. Products queued back to back on two streams, and products issued from two
host threads, must each equal the oracle's."""
import threading

import numpy as np
import pytest

from oracle import fcirc as O
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu
P = W.P1


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return fcirc


def dev(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr).view(np.int32)).cuda()


def test_two_streams_share_the_workspace(F):
    import torch
    n = 1 << 18
    cases = [W.modp_pair(n, P, seed=40 + k) for k in range(4)]
    want = [O.levels_matvec_modp(a, x, 1, P) for a, x in cases]
    ins = [(dev(a), dev(x)) for a, x in cases]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = []
    for k, (da, dx) in enumerate(ins):  # alternate streams, no synchronisation in between
        with torch.cuda.stream(streams[k % 2]):
            outs.append(F.matvec(da, dx, f=1, p=P))
    torch.cuda.synchronize()
    for k in range(4):
        got = outs[k].cpu().numpy().view(np.uint32).astype(np.int64)
        np.testing.assert_array_equal(got, want[k], err_msg=f"product {k}")


def test_two_host_threads(F):
    import torch
    n = 1 << 16
    cases = [W.modp_pair(n, P, seed=60 + k) for k in range(2)]
    want = [O.levels_matvec_modp(a, x, 1, P) for a, x in cases]
    ins = [(dev(a), dev(x)) for a, x in cases]
    errors = []

    def worker(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(20):
                    y = F.matvec(*ins[k], f=1, p=P)
                    s.synchronize()
                    got = y.cpu().numpy().view(np.uint32).astype(np.int64)
                    if not np.array_equal(got, want[k]):
                        errors.append(k)
                        return
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert errors == []
