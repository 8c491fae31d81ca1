"""GPU parity against the oracle at the full sizes of the workloads, in the
launch configurations the benchmark times.

- 64 meshes of 1024 x 1024 (per-point s, x then y solves of a given right-hand
  side), plain FP64 and plain FP32: the GPU solves the whole batch; the oracle
  solves four sampled meshes (first, two inner, last), which are independent of
  the others.  Per-line relative error along the y lines of the output.
- The uneven batch of 20,000 systems (lengths log-uniform in [32, 8192]), plain
  FP64 and plain FP32, every system against the oracle.
- The 256^3 ADI step (s = 0.2) in FP32 on the rounded U(0, 1) field.

Tolerances: FP64 <= 1e-12 and FP32 <= 1e-5 relative, against the FP64 oracle
run on the same (FP32-rounded where the GPU computes in FP32) inputs.
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
    return trid


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _line_err(x, ref, axis):
    ax = x.ndim - 1 - axis
    num = np.max(np.abs(np.moveaxis(x - ref, ax, -1)), axis=-1)
    den = np.max(np.abs(np.moveaxis(ref, ax, -1)), axis=-1)
    return float(np.max(num / np.maximum(den, 1e-300)))


def _sys_err(x, ref, off):
    num = np.maximum.reduceat(np.abs(x - ref), off[:-1])
    den = np.maximum.reduceat(np.abs(ref), off[:-1])
    return float(np.max(num / np.maximum(den, 1e-300)))


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_2d_64x1024sq_x_then_y_sampled_meshes(trid, orc, dt):
    s32, d32 = gen.adi2d_varcoef()  # the full batch: 64 meshes of 1024 x 1024
    assert s32.shape == (64, 1024, 1024)
    ts, td = _t(s32.astype(dt)), _t(d32.astype(dt))
    trid.gtsv_s(ts, td, 0)
    trid.gtsv_s(ts, td, 1)
    sample = [0, 21, 42, 63]
    got = td[sample].cpu().numpy().astype(np.float64)
    ref = orc.adi_xy(s32[sample].astype(np.float64), d32[sample].astype(np.float64))
    err = _line_err(got, ref, 1)
    print("64 x 1024^2 x-then-y %s: per-line error %.3g" % (np.dtype(dt).name, err))
    assert err <= TOL[dt], err


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_varlen_20000_systems_plain(trid, orc, dt):
    a32, b32, c32, d64, off = gen.varlen_batch()
    d_in = d64.astype(dt).astype(np.float64)
    ref = orc.gtsv_varlen(a32, b32, c32, d_in, off)
    a, b, c = (_t(v.astype(dt)) for v in (a32, b32, c32))
    d = _t(d64.astype(dt))
    x = torch.empty_like(d)
    p = trid.PREC_F64 if dt == np.float64 else trid.PREC_F32
    trid.gtsv_varlen(p, a, b, c, d, x, off)
    err = _sys_err(x.cpu().numpy().astype(np.float64), ref, off)
    print("20,000 uneven systems %s: per-system error %.3g" % (np.dtype(dt).name, err))
    assert err <= TOL[dt], err


def test_adi3d_256cubed_fp32_one_step_matches_oracle(trid, orc):
    u32 = gen.adi3d_field((256, 256, 256), seed=1, dtype=np.float32)
    ref = orc.adi_step(u32.astype(np.float64), s0=0.2, nsteps=1)
    tu = _t(u32)
    trid.adi_step(tu, s0=0.2, nsteps=1, graph=True)
    got = tu.cpu().numpy().astype(np.float64)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    print("256^3 FP32 ADI step: field error %.3g" % err)
    assert err <= TOL[np.float32], err
