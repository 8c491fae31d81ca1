"""GPU parity of the Hundsdorfer-Verwer SLV stand-in against the CPU oracle.

Each step is four predictor stencils and four batched s-form line solves
(x, y, x, y: the call structure of Alg. 4).  Tolerances as for the ADI step:
max|u - u_ref| / max|u_ref| <= 1e-12 (FP64), 1e-5 (FP32; oracle in FP64 on the
FP32-rounded inputs).
"""

import math

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = {np.float64: 1e-12, np.float32: 1e-5}
THETA = 0.5 + math.sqrt(3.0) / 6.0


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


# (nx, ny): the two SLV mesh sizes, one point per line, a single mesh row or
# column, lines past one tile with ragged tails and padded tiles (33: 5 tiles
# of 8 in 8 lanes), the largest resident line (128), and meshes that take the
# per-step kernels by default (x lines of 300 points; 128 x 128 FP64 is
# beyond one workgroup's LDS); 16 tiles per y line (x 128) with one pass or
# two passes of the workgroup over the lines; 100 x 56 FP64 (14-row tiles with
# a, b, c read from memory: the variant whose registers spill)
SHAPES = [(40, 20), (100, 50), (1, 1), (1, 9), (9, 1), (37, 13), (33, 70), (128, 40), (300, 7), (128, 128),
          (64, 128), (8, 128), (40, 128), (100, 56)]


def _kernels(trid, fn):
    trid.timing_enable(True)
    fn()
    names = set(trid.timing_read())
    trid.timing_enable(False)
    return names


@pytest.mark.parametrize("stream", [False, True], ids=["default", "stream"])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("nx,ny", SHAPES, ids=[str(s) for s in SHAPES])
def test_hv_matches_oracle(trid, orc, dt, nx, ny, stream):
    batch, steps, tau = 5, 4, 0.25
    u, a, b, c = (v.astype(dt) for v in gen.hv_slv((nx, ny), batch, seed=nx * 7 + ny))
    ref = orc.hv_step(u.astype(np.float64), a.astype(np.float64), b.astype(np.float64),
                      c.astype(np.float64), tau, THETA, steps)
    tu = _t(u)
    names = _kernels(trid, lambda: trid.hv_step(tu, _t(a), _t(b), _t(c), tau, THETA, steps, stream=stream))
    torch.cuda.synchronize()
    err = _field_err(tu.cpu().numpy().astype(np.float64), ref)
    print("hv %dx%d x%d %s steps=%d stream=%d err=%.2e %s" % (nx, ny, batch, np.dtype(dt).name, steps, stream, err,
                                                            sorted(names)))
    assert err <= TOL[dt]
    resident = not stream and nx <= 128 and ny <= 128 and nx * ny * np.dtype(dt).itemsize * 3 < 150 * 1024
    assert ("hv_resident" in names) == resident


@pytest.mark.parametrize("stream", [False, True], ids=["default", "stream"])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("nx,ny", [(100, 50), (40, 20)], ids=["100x50", "40x20"])
def test_hv_slv_batch_sampled(trid, orc, stream, dt, nx, ny):
    """The SLV meshes at batch 3000 (the largest SLV configuration), in the launch
    configuration the bench times: the oracle recomputes a sample of the meshes,
    which are independent."""
    batch, steps, tau = 3000, 3, 0.25
    u, a, b, c = (v.astype(dt) for v in gen.hv_slv((nx, ny), batch))
    tu = _t(u)
    trid.hv_step(tu, _t(a), _t(b), _t(c), tau, THETA, steps, stream=stream)
    out = tu.cpu().numpy().astype(np.float64)
    pick = np.array([0, 1, 1499, 2998, 2999])
    ref = orc.hv_step(*(v[pick].astype(np.float64) for v in (u, a, b, c)), tau, THETA, steps)
    err = _field_err(out[pick], ref)
    print("hv sampled %dx%d %s stream=%d err=%.2e" % (nx, ny, np.dtype(dt).name, stream, err))
    assert err <= TOL[dt]


def test_hv_resident_matches_streamed_over_many_steps(trid):
    """Both paths over 60 steps on the 40 x 20 meshes (FP64): the same steps up to rounding."""
    u, a, b, c = (_t(v) for v in gen.hv_slv((40, 20), 300))
    u1 = u.clone()
    trid.hv_step(u, a, b, c, 0.25, THETA, 60)
    trid.hv_step(u1, a, b, c, 0.25, THETA, 60, stream=True)
    torch.cuda.synchronize()
    err = float((u - u1).abs().max() / u1.abs().max())
    print("resident vs streamed, 60 steps: %.2e" % err)
    assert err <= 1e-12


@pytest.mark.parametrize("stream", [False, True], ids=["default", "stream"])
def test_hv_zero_steps_and_zero_dt(trid, stream):
    u, a, b, c = (_t(v) for v in gen.hv_slv((12, 6), 2))
    u0 = u.clone()
    trid.hv_step(u, a, b, c, 0.3, THETA, 0, stream=stream)
    assert torch.equal(u, u0)
    trid.hv_step(u, a, b, c, 0.0, THETA, 3, stream=stream)  # tau = 0: every predictor and solve is the identity
    torch.cuda.synchronize()
    assert torch.equal(u, u0)


@pytest.mark.parametrize("stream", [False, True], ids=["default", "stream"])
def test_hv_repeated_calls_compose(trid, stream):
    """Two calls of k steps equal one call of 2k (the work arrays are rebuilt each call)."""
    u, a, b, c = (_t(v) for v in gen.hv_slv((40, 20), 4))
    u1 = u.clone()
    trid.hv_step(u, a, b, c, 0.25, THETA, 3, stream=stream)
    trid.hv_step(u, a, b, c, 0.25, THETA, 3, stream=stream)
    trid.hv_step(u1, a, b, c, 0.25, THETA, 6, stream=stream)
    torch.cuda.synchronize()
    assert torch.equal(u, u1)


def test_hv_rejects_bad_arguments(trid):
    u, a, b, c = (_t(v) for v in gen.hv_slv((8, 4), 1))
    with pytest.raises(trid.TridError):
        trid.hv_step(u, a, b, c, -0.1, THETA, 1)
    with pytest.raises(trid.TridError):
        trid.hv_step(u, a, b, c, 0.1, 0.0, 1)
    with pytest.raises(trid.TridError):
        trid.hv_step(u, a, b, c, float("nan"), THETA, 1)
    with pytest.raises(trid.TridError):
        trid.hv_step(u, a, b, c, 0.1, THETA, -1)
    with pytest.raises(ValueError):
        trid.hv_step(u[0], a[0], b[0], c[0], 0.1, THETA, 1)  # 1D is not a 2D mesh batch
    with pytest.raises(ValueError):
        trid.hv_step(u, a.float(), b, c, 0.1, THETA, 1)
