"""GPU parity of contiguous lines longer than one workgroup (the chunked solve).

Lines of more than 8192 rows along axis 0 are cut into 2048-row chunks coupled
through a reduced system of two rows per chunk (the tiling of Section III-B
one level up).  Tolerances as for the other line solves (relative error per
line, infinity norm): FP64 <= 1e-12, FP32 <= 1e-5 against the FP64 oracle on
the same FP32-rounded inputs; the near-singular case derives its own bound
from the condition number.
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


def _err(x, ref):
    """Max over lines (last axis) of the relative infinity-norm error."""
    num = np.max(np.abs(x - ref), axis=-1)
    den = np.max(np.abs(ref), axis=-1)
    return float(np.max(num / np.maximum(den, 1e-300)))


# (n, lines): a last chunk of one row, exact chunks, ragged tails, many chunks
LONG = [(8193, 2), (10240, 1), (20000, 3), (100001, 2), (1 << 20, 1)]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("n,lines", LONG, ids=[str(g) for g in LONG])
def test_long_arrays_match_oracle(trid, orc, dt, n, lines):
    a, b, c, d = (v.astype(dt) for v in gen.dd_lines(lines, n, seed=n % 1000))
    # the first row's a and the last row's c are outside the system: make them
    # nonzero so that a solve that used them would fail
    a[:, 0] = 0.75
    c[:, -1] = -0.5
    ref = orc.gtsv(a, b, c, d, 0)
    ta, tb, tc, td = (_t(v) for v in (a, b, c, d))
    trid.gtsv(ta, tb, tc, td, 0)
    assert _err(td.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("mode", ["const", "s"])
def test_long_generated_rows_match_oracle(trid, orc, dt, mode):
    rng = np.random.default_rng(77)
    n, lines = 50000, 2
    d = rng.standard_normal((lines, n)).astype(dt)
    td = _t(d)
    if mode == "const":
        ref = orc.gtsv_const(-0.4, 1.5, -0.6, d, 0)
        trid.gtsv_const(-0.4, 1.5, -0.6, td, 0)
    else:
        s = (0.1 * np.exp(rng.standard_normal((lines, n)))).astype(dt)
        ref = orc.gtsv_s(s, d, 0)
        trid.gtsv_s(_t(s), td, 0)
    assert _err(td.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


def test_long_lines_of_a_2d_mesh(trid, orc):
    # dims [9000, 3], batch 2: six contiguous long lines
    a, b, c, d = gen.dd_mesh((9000, 3), 2, seed=9)
    ref = orc.gtsv(a, b, c, d, 0)
    ta, tb, tc, td = (_t(v) for v in (a, b, c, d))
    trid.gtsv(ta, tb, tc, td, 0)
    assert _err(td.cpu().numpy(), ref) <= 1e-12


def test_long_maximum_length(trid, orc):
    n = 8388608  # TRID_MAX_LONG_LINE: 4096 chunks, a reduced line of 8192 rows
    a, b, c, d = gen.dd_lines(1, n, seed=3)
    ref = orc.gtsv(a, b, c, d, 0)
    ta, tb, tc, td = (_t(v) for v in (a, b, c, d))
    trid.gtsv(ta, tb, tc, td, 0)
    assert _err(td.cpu().numpy(), ref) <= 1e-12


def test_long_strongly_coupled_chunks(trid, orc):
    """Rows (-1, 2 + 1e-5, -1): a unit at one row still reaches about 1e-3 of
    itself 2048 rows away, so every coupling term of the reduced rows matters.
    The infinity-norm condition number is about (b + 2) / (b - 2) = 4e5; both
    solutions are within a small multiple of kappa * u of the exact one, so the
    bound is 20 * kappa * 2^-53 (about 1e-9), far below the 1e-3 a dropped
    coupling term would leave."""
    n, eps = 30000, 1e-5
    rng = np.random.default_rng(12)
    d = rng.uniform(0.0, 1.0, (2, n))
    td = _t(d)
    ref = orc.gtsv_const(-1.0, 2.0 + eps, -1.0, d, 0)
    trid.gtsv_const(-1.0, 2.0 + eps, -1.0, td, 0)
    kappa = (4.0 + eps) / eps
    assert _err(td.cpu().numpy(), ref) <= 20 * kappa * 2.0**-53


def test_long_lines_run_in_place_repeatedly(trid, orc):
    """Two calls in a row on the same handle (workspace reuse), the second on
    a shorter and a longer batch than the first."""
    for n, lines in [(40000, 3), (12000, 1), (70000, 4)]:
        a, b, c, d = gen.dd_lines(lines, n, seed=lines)
        ref = orc.gtsv(a, b, c, d, 0)
        ta, tb, tc, td = (_t(v) for v in (a, b, c, d))
        trid.gtsv(ta, tb, tc, td, 0)
        assert _err(td.cpu().numpy(), ref) <= 1e-12
