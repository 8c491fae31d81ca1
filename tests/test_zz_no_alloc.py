"""The no-allocation ADI step (trid_adi_step_noalloc) against trid_adi_step (GPU).

Both run the same kernels; the no-allocation step keeps its d workspace in the
library's static device scratch.  Two calls in a row, the second on a smaller
mesh (the scratch keeps the first call's contents), each compared bitwise and
against the FP64 oracle at 1e-12 (FP32: 1e-5).
"""

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


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _field_err(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def test_noalloc_step_matches_adi_step_two_calls(trid, orc):
    # call 1: 3D FP64, constant s, 3 steps
    u1 = gen.adi3d_field((96, 80, 64), seed=11)
    ref1 = orc.adi_step(u1, s0=0.2, nsteps=3)
    a, b = _t(u1), _t(u1)
    trid.adi_step(a, s0=0.2, nsteps=3)
    trid.adi_step_noalloc(b, s0=0.2, nsteps=3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert _field_err(b.cpu().numpy(), ref1) <= 1e-12
    # call 2: a smaller 3D FP32 mesh with per-point s, 2 steps
    rng = np.random.default_rng(12)
    u2 = gen.adi3d_field((40, 24, 20), batch=2, seed=12, dtype=np.float32)
    s2 = (0.2 * rng.lognormal(0.0, 0.5, u2.shape)).astype(np.float32)
    ref2 = orc.adi_step(u2.astype(np.float64), s=s2.astype(np.float64), nsteps=2)
    a, b = _t(u2), _t(u2)
    ts = _t(s2)
    trid.adi_step(a, s=ts, nsteps=2)
    trid.adi_step_noalloc(b, s=ts, nsteps=2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert _field_err(b.cpu().numpy().astype(np.float64), ref2) <= 1e-5


def test_noalloc_2d_per_step_kernels(trid, orc):
    u = gen.adi3d_field((130, 70), batch=3, seed=13)  # lines longer than the resident loop takes
    ref = orc.adi_step(u, s0=0.15, nsteps=2)
    a, b = _t(u), _t(u)
    trid.adi_step(a, s0=0.15, nsteps=2, stream=True)
    trid.adi_step_noalloc(b, s0=0.15, nsteps=2, stream=True)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert _field_err(b.cpu().numpy(), ref) <= 1e-12


def test_noalloc_rejects_meshes_beyond_the_scratch(trid):
    u = torch.zeros((1, 256, 256, 256), dtype=torch.float64, device="cuda")  # 128 MiB of d
    with pytest.raises(trid.TridError) as ei:
        trid.adi_step_noalloc(u, s0=0.2, nsteps=1)
    assert ei.value.code == 4
    assert float(u.abs().max()) == 0.0  # untouched
