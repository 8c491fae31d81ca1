"""Per-kernel timing restricted to one kernel name (trid_timing_select)."""

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def trid():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_03950_amd as trid

    trid.load_library()
    return trid


def _steps(trid, u, n, only, every=1):
    trid.timing_select(only, every)
    trid.timing_enable(True)
    for _ in range(n):
        trid.adi_step(u, s0=0.2, nsteps=1)
    kt = trid.timing_read()
    trid.timing_enable(False)
    trid.timing_select(None)
    return kt


def test_select_times_only_the_named_kernel(trid):
    u0 = torch.from_numpy(gen.adi3d_field((64, 48, 40), 2, seed=3)).cuda()
    ua, ub = u0.clone(), u0.clone()
    every = _steps(trid, ua, 3, None)
    assert set(every) == {"adi_stencil_x", "adi_y", "adi_z_update"}
    assert all(cnt == 3 for cnt, _ in every.values())
    only = _steps(trid, ub, 3, "adi_z_update")
    assert set(only) == {"adi_z_update"} and only["adi_z_update"][0] == 3
    assert only["adi_z_update"][1] > 0
    # the launches without events compute the same steps
    assert torch.equal(ua, ub)
    # every third launch of the name: the first, fourth and seventh of 7
    some = _steps(trid, ub, 7, "adi_y", 3)
    assert set(some) == {"adi_y"} and some["adi_y"][0] == 3
    _steps(trid, ua, 7, None)
    assert torch.equal(ua, ub)
    # every name, every second launch: steps 1, 3, 5 of 5
    half = _steps(trid, ub, 5, None, 2)
    assert set(half) == {"adi_stencil_x", "adi_y", "adi_z_update"}
    assert all(cnt == 3 for cnt, _ in half.values())
    _steps(trid, ua, 5, None)
    assert torch.equal(ua, ub)
    # a name no launch carries times nothing
    assert _steps(trid, ub, 1, "no_such_kernel") == {}
