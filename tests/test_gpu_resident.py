"""GPU parity of the LDS-resident 2D ADI time loop against the CPU oracle.

2D meshes of at most 128 points per line run all time steps in one launch
with each mesh held in LDS.  Tolerances as for the streamed ADI step:
max|u - u_ref| / max|u_ref| <= 1e-12 (FP64), 1e-5 (FP32, oracle in FP64 on the
FP32-rounded inputs).
"""

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {np.float64: 1e-12, np.float32: 1e-5}


@pytest.fixture(scope="module")
def trid():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_03950_amd as trid

    trid.load_library()
    yield trid


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _field_err(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def _run(trid, tu, s, s0, steps, stream=False):
    """One adi_step call; returns the kernel names it launched."""
    trid.timing_enable(True)
    trid.adi_step(tu, s=s, s0=s0, nsteps=steps, stream=stream)
    names = set(trid.timing_read())
    trid.timing_enable(False)
    return names


# (nx, ny): 1 to 16 tiles per line; tiles of 8 (32, 64, 128), 10 (80), 12 (48,
# 96) and 14 rows (112, and 100 x 37 with padding); ragged tails, a single
# point per line, non-square meshes
SHAPES = [(32, 32), (64, 64), (48, 48), (80, 80), (96, 96), (112, 112), (128, 128), (100, 37), (13, 90),
          (60, 44), (5, 3), (1, 7), (128, 1)]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("perpoint", [False, True])
@pytest.mark.parametrize("nx,ny", SHAPES, ids=[str(s) for s in SHAPES])
def test_resident_matches_oracle(trid, orc, dt, perpoint, nx, ny):
    batch, steps = 3, 7
    u = gen.adi3d_field((nx, ny), batch, seed=nx + ny).astype(dt)
    s = None
    if perpoint:
        s = (0.2 * np.exp(0.5 * np.random.default_rng(nx * ny).standard_normal(u.shape))).astype(dt)
    ref = orc.adi_step(u, s=s, s0=0.25, nsteps=steps)
    tu = _t(u)
    names = _run(trid, tu, _t(s) if s is not None else None, 0.25, steps)
    # u, d (and s) must fit one workgroup's 160 KB of LDS, else the per-step kernels run
    fits = (3 if perpoint else 2) * nx * ny * np.dtype(dt).itemsize + 64 <= 160 * 1024
    if fits:
        assert names == {"adi2d_resident"}
    else:
        assert "adi2d_resident" not in names
    assert _field_err(tu.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_resident_agrees_with_streamed_steps(trid, dt):
    u = gen.adi3d_field((64, 64), 4, seed=5).astype(dt)
    a, b = _t(u), _t(u)
    assert _run(trid, a, None, 0.3, 20) == {"adi2d_resident"}
    assert "adi2d_resident" not in _run(trid, b, None, 0.3, 20, stream=True)
    assert _field_err(a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)) <= 2 * TOL[dt]


def test_resident_fourier_mode_decay(trid):
    """A product of sine modes is an eigenvector of every step: after n steps it
    is g^n times itself, g = 1 - 2 s (mu_x + mu_y) / ((1 + s mu_x)(1 + s mu_y))."""
    nx, ny, px, py, s, steps = 96, 64, 3, 2, 0.4, 120
    x = np.arange(1, nx + 1)
    y = np.arange(1, ny + 1)
    u0 = np.sin(np.pi * py * y / (ny + 1))[:, None] * np.sin(np.pi * px * x / (nx + 1))[None, :]
    mu = [4.0 * np.sin(np.pi * p / (2.0 * (n + 1))) ** 2 for p, n in ((px, nx), (py, ny))]
    g = 1.0 - 2.0 * s * sum(mu) / ((1.0 + s * mu[0]) * (1.0 + s * mu[1]))
    tu = _t(np.stack([u0, -u0]))
    assert _run(trid, tu, None, s, steps) == {"adi2d_resident"}
    ref = np.stack([u0, -u0]) * g ** steps
    assert float(np.max(np.abs(tu.cpu().numpy() - ref))) <= 1e-12


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_resident_paper_shape_sampled(trid, orc, dt):
    """1500 meshes of 64^2, 120 steps (the 2D application's shape): sampled
    meshes against the oracle run on those meshes alone."""
    batch, steps = 1500, 120
    u = gen.adi3d_field((64, 64), batch, seed=15).astype(dt)
    tu = _t(u)
    assert _run(trid, tu, None, 0.2, steps) == {"adi2d_resident"}
    out = tu.cpu().numpy().astype(np.float64)
    for m in (0, 1, 777, batch - 1):
        ref = orc.adi_step(u[m:m + 1], s0=0.2, nsteps=steps)
        assert _field_err(out[m:m + 1], ref) <= TOL[dt]


def test_resident_repeated_calls_and_zero_steps(trid, orc):
    u = gen.adi3d_field((40, 24), 2, seed=6)
    tu = _t(u)
    trid.adi_step(tu, s0=0.2, nsteps=0)
    assert np.array_equal(tu.cpu().numpy(), u)
    for _ in range(3):
        trid.adi_step(tu, s0=0.2, nsteps=2)
    ref = orc.adi_step(u, s0=0.2, nsteps=6)
    assert _field_err(tu.cpu().numpy(), ref) <= 1e-12
