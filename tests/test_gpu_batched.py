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


def _ring_of(p):
    from paper_2103_02605_amd import _lib
    return {None: _lib.FCIRC_C64, W.P1: _lib.FCIRC_ZP_998244353}[p]


@pytest.mark.parametrize("p", [None, W.P1])
def test_every_batch_form(B, p):
    """Every form the tuner may pick (workgroup 256 or 512 threads; one item per instance or
    blocks of 2^10 .. 2^13 elements below 1 .. 6 top levels) gives the product: instances of
    2^13, 2^14 and 2^16 next to small ones, against the oracle."""
    from paper_2103_02605_amd import fcirc as F
    ring = _ring_of(p)
    small = [5, 9, 12]
    forms = []
    for bt in (256, 512):
        elog = 12 if bt == 256 else 13
        for L in (13, 14, 16):
            for blog in (0, 10, 11, 12, 13):
                full_ok = blog == 0 and L <= elog
                pass_ok = blog >= 10 and blog <= elog and L > blog and L - blog <= 6 and L >= elog
                if full_ok or pass_ok:
                    forms.append((bt, L, blog))
    inst = {}
    for L in small + [13, 14, 16]:
        if p is None:
            inst[L] = [W.complex_pair(1 << L, seed=700 + 10 * L + k) for k in range(2)]
        else:
            inst[L] = [W.modp_pair(1 << L, p, seed=700 + 10 * L + k) for k in range(2)]
    want = {}
    for L, pairs in inst.items():
        if p is None:
            want[L] = [O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128)) for a, x in pairs]
        else:
            want[L] = [O.levels_matvec_modp(a, x, 1, p) for a, x in pairs]
    try:
        for bt, L, blog in forms:
            for Ls in small:
                F.set_batch_schedule(1 << Ls, ring, bt, 0)
            F.set_batch_schedule(1 << L, ring, bt, blog)
            assert F.get_batch_schedule(1 << L, ring) == {"workgroup": bt, "block_levels": blog}
            sizes = small + [L]
            a_list = [a for Ls in sizes for a, _ in inst[Ls]]
            x_list = [x for Ls in sizes for _, x in inst[Ls]]
            if p is None:
                ys = B.matvec_batched_c64(a_list, x_list)
            else:
                ys = B.matvec_batched_modp(a_list, x_list, p=p, f=1)
            k = 0
            for Ls in sizes:
                for j in range(2):
                    if p is None:
                        assert rel_l2(ys[k], want[Ls][j]) <= TOL, (bt, L, blog, Ls, j)
                    else:
                        np.testing.assert_array_equal(ys[k], want[Ls][j], err_msg=f"{bt} {L} {blog} {Ls} {j}")
                    k += 1
    finally:
        for Ls in small + [13, 14, 16]:
            F.set_batch_schedule(1 << Ls, ring, -1)


def test_tuned_batch_parameters_saved_and_loaded(B, tmp_path):
    """fcirc_tune picks the batched launch's form per size; the schedule file keeps it and a
    load brings it back; a batch run with the tuned forms stays within the bar."""
    from paper_2103_02605_amd import fcirc as F
    from paper_2103_02605_amd import _lib
    ring = _lib.FCIRC_C64
    sizes = [10, 13, 15]
    try:
        for L in sizes:
            F.tune(1 << L, ring)
        tuned = {L: F.get_batch_schedule(1 << L, ring) for L in sizes}
        path = tmp_path / "sched.txt"
        F.save_schedules(path)
        text = path.read_text()
        assert " batch 3 13 " in text
        for L in sizes:
            F.set_batch_schedule(1 << L, ring, -1)
        F.load_schedules(path)
        assert {L: F.get_batch_schedule(1 << L, ring) for L in sizes} == tuned
        logs = [10, 13, 15, 13, 10, 15, 7]
        inst = [W.complex_pair(1 << L, seed=800 + k) for k, L in enumerate(logs)]
        ys = B.matvec_batched_c64([a for a, _ in inst], [x for _, x in inst])
        for k, (a, x) in enumerate(inst):
            want = O.levels_matvec_c128(a.astype(np.complex128), x.astype(np.complex128))
            assert rel_l2(ys[k], want) <= TOL, k
        # a malformed batch line is refused and changes nothing
        bad = tmp_path / "bad.txt"
        bad.write_text(text + "gfx950 256 batch 3 13 7 0.5 0 0.5\n")
        with pytest.raises(Exception):
            F.load_schedules(bad)
        assert {L: F.get_batch_schedule(1 << L, ring) for L in sizes} == tuned
    finally:
        for L in sizes:
            F.set_batch_schedule(1 << L, ring, -1)
