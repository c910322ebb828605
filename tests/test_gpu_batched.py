"""GPU parity of the batched persistent launch (many products of different sizes in one
launch, its work queue reused for a repeated item list) against the CPU oracle."""
import numpy as np
import pytest

from oracle import fcirc as O
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def B():
    import torch
    from paper_2103_02605_amd import batched
    assert torch.cuda.is_available()
    return batched


def rel_l2(got, want):
    return np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)


def test_mixed_sizes_complex(B):
    import torch
    rng = np.random.default_rng(1)
    logs = [0, 1, 2, 3, 4, 5, 6, 9, 12, 13, 14, 15, 16] + list(rng.integers(0, 17, 40))
    a_list, x_list = [], []
    for k, L in enumerate(logs):
        a, x = W.complex_pair(1 << int(L), seed=1000 + k)
        a_list.append(a)
        x_list.append(x)
    ys = B.matvec_batched_c64(a_list, x_list)
    for k in range(len(logs)):
        want = O.cyclic_matvec_fft_c128(a_list[k].astype(np.complex128), x_list[k].astype(np.complex128))
        assert rel_l2(ys[k], want) <= TOL, (k, logs[k])


@pytest.mark.parametrize("f", [-1.0, np.exp(0.7j)])
def test_mixed_sizes_complex_f(B, f):
    """The batched launch with f != 1 (its twiddle tables are f's), sizes 2^0 .. 2^16."""
    rng = np.random.default_rng(7)
    logs = [0, 1, 4, 8, 12, 13, 16] + list(rng.integers(0, 17, 12))
    a_list, x_list = [], []
    for k, L in enumerate(logs):
        a, x = W.complex_pair(1 << int(L), seed=2000 + k)
        a_list.append(a)
        x_list.append(x)
    ys = B.matvec_batched_c64(a_list, x_list, f=f)
    for k in range(len(logs)):
        want = O.levels_matvec_c128(a_list[k].astype(np.complex128), x_list[k].astype(np.complex128), f)
        assert rel_l2(ys[k], want) <= TOL, (k, logs[k])


@pytest.mark.parametrize("p,f", [(W.P1, 1), (W.P2, W.P2 - 1), (W.P3, 1)])
def test_mixed_sizes_modp(B, p, f):
    rng = np.random.default_rng(p % 1000)
    logs = [0, 1, 3, 4, 7, 10, 12, 13, 16] + list(rng.integers(0, 15, 20))
    a_list, x_list = [], []
    for k, L in enumerate(logs):
        a, x = W.modp_pair(1 << int(L), p, seed=k)
        a_list.append(a)
        x_list.append(x)
    ys = B.matvec_batched_modp(a_list, x_list, p=p, f=f)
    for k, L in enumerate(logs):
        n = 1 << int(L)
        want = O.dense_matvec_modp(a_list[k], x_list[k], f, p) if n <= 2048 else O.levels_matvec_modp(a_list[k], x_list[k], f, p)
        np.testing.assert_array_equal(ys[k], want, err_msg=f"instance {k} n={n}")


def test_repeated_runs_with_eager_work_between(B):
    """Build the queue once, run it several times with other GPU work and synchronisations
    in between; every run must match the eager single-product results."""
    import torch
    from paper_2103_02605_amd import fcirc as F
    logs = [3, 8, 12, 13, 15, 16, 6, 6, 6, 11]
    inst = [W.complex_pair(1 << L, seed=50 + k) for k, L in enumerate(logs)]
    plan = B.BatchPlan([a for a, _ in inst], [x for _, x in inst], dtype=np.complex64)
    eager = [F.matvec(torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda()).cpu().numpy() for a, x in inst]
    for rep in range(4):
        plan.run()
        junk = torch.randn(1 << 20, device="cuda") * 3.0  # unrelated eager work
        torch.cuda.synchronize()
        ys = plan.outputs()
        for k in range(len(logs)):
            assert rel_l2(ys[k], eager[k]) <= 1e-6, (rep, k)
        del junk
    # new inputs in the same buffers, same queue: results follow the inputs
    new = [W.complex_pair(1 << L, seed=90 + k) for k, L in enumerate(logs)]
    plan.load([a for a, _ in new], [x for _, x in new])
    plan.run()
    ys = plan.outputs()
    for k in range(len(logs)):
        want = O.cyclic_matvec_fft_c128(new[k][0].astype(np.complex128), new[k][1].astype(np.complex128))
        assert rel_l2(ys[k], want) <= TOL


def test_c4_config_all_instances(B):
    """4096 complex64 instances, n = 2^e with e uniform on {6..16} (seed 6), every instance
    within 1e-5 relative L2 of the FP64 oracle."""
    e, a_list, x_list = W.batched_c64(4096, W.SEED_BATCHED)
    ys = B.matvec_batched_c64(a_list, x_list)
    worst = 0.0
    for k in range(len(a_list)):
        want = O.cyclic_matvec_fft_c128(a_list[k].astype(np.complex128), x_list[k].astype(np.complex128))
        worst = max(worst, rel_l2(ys[k], want))
    assert worst <= TOL, worst


def test_tables_rebuilt_between_runs(B):
    """A reused batched launch takes the twiddle tables the context holds at each run: a
    larger single product with the same f in between rebuilds them (the old ones are
    freed), and the next run of the same item list must still be exact."""
    import torch
    from paper_2103_02605_amd import fcirc as F
    p = W.P1
    f = pow(12345, 1 << 23, p)  # has 2^23-th roots; used by no other test
    logs = [5, 12, 13, 16, 16, 9]
    inst = [W.modp_pair(1 << L, p, seed=300 + k) for k, L in enumerate(logs)]
    want = [O.levels_matvec_modp(a, x, f, p) for a, x in inst]
    plan = B.BatchPlan([a for a, _ in inst], [x for _, x in inst], p=p, f=f)
    plan.run(check=True)
    for k, y in enumerate(plan.outputs()):
        np.testing.assert_array_equal(y, want[k], err_msg=f"first run, instance {k}")
    a, x = W.modp_pair(1 << 21, p, seed=301)
    F.matvec(torch.from_numpy(a.view(np.int32)).cuda(), torch.from_numpy(x.view(np.int32)).cuda(), f=f, p=p)
    plan.y.zero_()
    plan.run(check=True)
    for k, y in enumerate(plan.outputs()):
        np.testing.assert_array_equal(y, want[k], err_msg=f"run after the tables grew, instance {k}")
    # the same for the complex ring (tables computed on the GPU)
    fc = np.exp(0.37j)
    cinst = [W.complex_pair(1 << L, seed=400 + k) for k, L in enumerate(logs)]
    cwant = [O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128), fc) for a, x in cinst]
    cplan = B.BatchPlan([a for a, _ in cinst], [x for _, x in cinst], dtype=np.complex64, f=fc)
    cplan.run(check=True)
    a, x = W.complex_pair(1 << 21, seed=401)
    F.matvec(torch.from_numpy(a).cuda(), torch.from_numpy(x).cuda(), f=fc)
    cplan.y.zero_()
    cplan.run(check=True)
    for k, y in enumerate(cplan.outputs()):
        assert rel_l2(y, cwant[k]) <= TOL, k


def test_many_item_lists_bounded(B):
    """More distinct item lists than the context keeps: older queues are dropped and
    rebuilt on demand, results stay exact."""
    p = W.P3
    plans = []
    for k in range(20):
        logs = [4 + (k % 9), 13]
        inst = [W.modp_pair(1 << L, p, seed=500 + 10 * k + j) for j, L in enumerate(logs)]
        plans.append((B.BatchPlan([a for a, _ in inst], [x for _, x in inst], p=p, f=1), inst))
    for rep in range(2):
        for plan, inst in plans:
            plan.run(check=True)
            for j, y in enumerate(plan.outputs()):
                np.testing.assert_array_equal(y, O.levels_matvec_modp(inst[j][0], inst[j][1], 1, p))
