"""GPU parity of the FP32 + FP64-refinement solves against the FP64 oracle.

The FP32 coefficients are the matrix of record: the oracle solves with their
exact FP64 promotions.  Each case also reports the plain FP32 error (the
oracle's binary32 Thomas) and requires the refined error to be far below it.
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


def _line_err(x, ref, axis):
    ax = x.ndim - 1 - axis
    num = np.max(np.abs(np.moveaxis(x - ref, ax, -1)), axis=-1)
    den = np.max(np.abs(np.moveaxis(ref, ax, -1)), axis=-1)
    return float(np.max(num / np.maximum(den, 1e-300)))


GEOMS = [((33, 41, 10), 2, 0), ((33, 41, 10), 2, 1), ((33, 41, 10), 2, 2), ((1000, 3), 2, 0),
         ((5, 700), 1, 1), ((256, 64), 1, 0), ((64, 256), 1, 1), ((3,), 4, 0), ((1,), 4, 0),
         # x lines staged up to 4096 rows, beyond that strided 16-row tiles up to the 8192-row
         # limit (a ragged last tile at 7001 rows); y lines of 32-row tiles at the limit
         ((4096, 2), 1, 0), ((4097, 2), 1, 0), ((7001, 3), 1, 0), ((8192, 2), 1, 0), ((3, 8192), 1, 1),
         # x lines of 2^k 16-row tiles (the register-lean staged kernel), ragged last tiles and blocks
         ((1017, 5), 1, 0), ((120, 9), 2, 0), ((512, 3), 3, 0),
         # strided lines of >= 512 rows (the register-lean kernel, 512-thread blocks): a ragged
         # last block of 1024-row lines, z lines of 34 tiles
         ((37, 1024), 1, 1), ((7, 5, 530), 1, 2),
         # 798 blocks of 512-row y lines: the grouped block order's trailing partial round
         ((600, 512), 21, 1),
         # y and z lines of 1, 2 and 3 rows
         ((6, 1), 2, 1), ((70, 2), 2, 1), ((4, 3, 3), 2, 2)]


@pytest.mark.parametrize("d64", [True, False])
@pytest.mark.parametrize("geom", GEOMS, ids=[str(g) for g in GEOMS])
def test_refine_arrays(trid, orc, geom, d64):
    dims, batch, axis = geom
    a, b, c, d = gen.dd_mesh(dims, batch, seed=7 + axis)
    a32, b32, c32 = (v.astype(np.float32) for v in (a, b, c))
    d = d if d64 else d.astype(np.float32)
    ref = orc.gtsv(a32, b32, c32, d, axis)
    plain = orc.gtsv_f32(a32, b32, c32, d, axis).astype(np.float64)
    x = torch.empty(d.shape, dtype=torch.float64, device="cuda")
    trid.gtsv_refine(_t(a32), _t(b32), _t(c32), _t(d), x, axis)
    err = _line_err(x.cpu().numpy(), ref, axis)
    err32 = _line_err(plain, ref, axis)
    assert err <= 1e-5
    assert err <= 1e-9 and err < err32 / 100, (err, err32)


@pytest.mark.parametrize("d64", [True, False])
@pytest.mark.parametrize("geom", GEOMS, ids=[str(g) for g in GEOMS])
def test_refine_s(trid, orc, geom, d64):
    dims, batch, axis = geom
    s32, d32 = gen.adi2d_varcoef((1, 1), 1)  # seeds the recipe; shapes below
    rng = np.random.default_rng(3 + axis)
    shape = gen.mesh_shape(dims, batch)
    s32 = (0.1 * np.exp(0.5 * rng.standard_normal(shape))).astype(np.float32)
    d = rng.standard_normal(shape)
    d = d if d64 else d.astype(np.float32)
    ref = orc.gtsv_s(s32.astype(np.float64), d, axis)
    a, b, c = orc.implicit_coefs(s32.astype(np.float64))
    plain = orc.gtsv_f32(a, b, c, d, axis).astype(np.float64)
    x = torch.empty(shape, dtype=torch.float64, device="cuda")
    trid.gtsv_s_refine(_t(s32), _t(d), x, axis)
    err = _line_err(x.cpu().numpy(), ref, axis)
    err32 = _line_err(plain, ref, axis)
    assert err <= 1e-5
    assert err <= 1e-9 and err < err32 / 100, (err, err32)


def test_refine_2d_xy_64x1024sq_sample(trid, orc):
    """The 2D workload's x-then-y refinement at reduced batch (4 of 64 meshes), FP64 intermediate."""
    s32, d32 = gen.adi2d_varcoef((1024, 1024), 4, seed=2)
    ref = orc.adi_xy(s32.astype(np.float64), d32.astype(np.float64))
    ts, td = _t(s32), _t(d32)
    mid = torch.empty(s32.shape, dtype=torch.float64, device="cuda")
    out = torch.empty_like(mid)
    trid.gtsv_s_refine(ts, td, mid, 0)
    trid.gtsv_s_refine(ts, mid, out, 1)
    err = float(np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref)))
    assert err <= 1e-9, err


def test_refine_rejects_aliasing(trid):
    d = torch.zeros((2, 8), dtype=torch.float64, device="cuda")
    s = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(trid.TridError):
        trid.gtsv_s_refine(s, d, d, 0)
