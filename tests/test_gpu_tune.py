"""GPU tests of the schedule file (save, load, refusal of malformed files) and of a tuned
schedule's parity."""
import numpy as np
import pytest

from oracle import fcirc as O
from paper_2103_02605_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def F():
    import torch
    from paper_2103_02605_amd import fcirc
    assert torch.cuda.is_available()
    return fcirc


def test_save_and_load_schedules(F, tmp_path):
    from paper_2103_02605_amd import _lib
    from paper_2103_02605_amd._lib import FcircError
    ring, n = _lib.FCIRC_ZP_998244353, 1 << 16
    path = tmp_path / "sched.txt"
    F.set_schedule(n, ring, 5, 11, F.SCHED_XCD)
    F.save_schedules(path)
    try:
        F.set_schedule(n, ring, -1, -1, F.SCHED_XCD)
        assert F.get_schedule(n, ring)["top_levels"] != 5
        F.load_schedules(path)
        s = F.get_schedule(n, ring)
        assert (s["top_levels"], s["tile_log"], s["flags"]) == (5, 11, F.SCHED_XCD)
        # a malformed file changes nothing
        bad = tmp_path / "bad.txt"
        good_lines = path.read_text().splitlines()
        bad.write_text("\n".join(good_lines + ["gfx950 256 0 17 6 11"]) + "\n")  # a field short
        F.set_schedule(n, ring, 7, 12, 0)
        with pytest.raises(FcircError, match="EINVAL"):
            F.load_schedules(bad)
        s = F.get_schedule(n, ring)
        assert (s["top_levels"], s["tile_log"], s["flags"]) == (7, 12, 0)
        bad.write_text("gfx950 256 0 16 99 11 1\n")  # top levels out of range
        with pytest.raises(FcircError, match="EINVAL"):
            F.load_schedules(bad)
        with pytest.raises(FcircError, match="EINVAL"):
            F.load_schedules(tmp_path / "missing.txt")
        # lines written for another device are skipped
        other = tmp_path / "other.txt"
        other.write_text("gfx942 304 0 16 3 11 1\n")
        F.load_schedules(other)
        assert F.get_schedule(n, ring)["top_levels"] == 7
        # the product under a loaded schedule is still exact
        F.load_schedules(path)
        a, x = W.modp_pair(n, W.P1, seed=16)
        import torch
        y = F.matvec(torch.from_numpy(a.view(np.int32)).cuda(), torch.from_numpy(x.view(np.int32)).cuda(), f=1, p=W.P1)
        np.testing.assert_array_equal(y.cpu().numpy().view(np.uint32).astype(np.int64), O.levels_matvec_modp(a, x, 1, W.P1))
    finally:
        F.set_schedule(n, ring, -1, -1, F.SCHED_XCD)
