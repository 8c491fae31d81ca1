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


# ------------------------------------------ refinement and adjoint, long lines --

LONG_REF = [(8193, 2), (100001, 1), (1 << 20, 1)]


@pytest.mark.parametrize("form", ["arrays", "s"])
@pytest.mark.parametrize("d64", [True, False])
@pytest.mark.parametrize("n,lines", LONG_REF, ids=[str(g) for g in LONG_REF])
def test_long_refine_matches_oracle(trid, orc, form, d64, n, lines):
    """FP32 chunked solves + one FP64 residual sweep: error <= 1e-9 and far below plain FP32."""
    a, b, c, d = gen.dd_lines(lines, n, seed=n % 997)
    d = d if d64 else d.astype(np.float32)
    if form == "s":  # the matrix of record: rows (-s, 1 + 2 s, -s) of the FP32 s, in FP64
        s32 = (0.1 * np.exp(0.5 * np.random.default_rng(n).standard_normal((lines, n)))).astype(np.float32)
        ref = orc.gtsv_s(s32.astype(np.float64), d, 0)
        plain = orc.gtsv_f32(*orc.implicit_coefs(s32.astype(np.float64)), d, 0).astype(np.float64)
    else:
        a32, b32, c32 = (v.astype(np.float32) for v in (a, b, c))
        ref = orc.gtsv(a32, b32, c32, d, 0)
        plain = orc.gtsv_f32(a32, b32, c32, d, 0).astype(np.float64)
    x = torch.empty((lines, n), dtype=torch.float64, device="cuda")
    if form == "s":
        trid.gtsv_s_refine(_t(s32), _t(d), x, 0)
    else:
        trid.gtsv_refine(_t(a32), _t(b32), _t(c32), _t(d), x, 0)
    err, err32 = _err(x.cpu().numpy(), ref), _err(plain, ref)
    print("long refine %s n=%d: %.3g (plain FP32 %.3g)" % (form, n, err, err32))
    assert err <= 1e-9 and err < err32 / 100, (err, err32)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("n,lines", [(20000, 2), (100001, 1)], ids=["20000x2", "100001x1"])
def test_long_adjoints_match_oracle(trid, orc, dt, n, lines):
    """Transposed chunked solve + gradients; coefficient gradients within the
    line tolerance carried through the product with x."""
    a, b, c, d = (v.astype(dt) for v in gen.dd_lines(lines, n, seed=n % 991))
    x = orc.gtsv(a, b, c, d, 0).astype(dt)
    gy = np.random.default_rng(n).standard_normal((lines, n)).astype(dt)
    lam, ga, gb, gc = orc.gtsv_adjoint(a, b, c, x, gy, 0)
    tg = _t(gy)
    tga, tgb, tgc = (torch.empty_like(tg) for _ in range(3))
    trid.gtsv_adjoint(_t(a), _t(b), _t(c), _t(x), tg, 0, tga, tgb, tgc)
    assert _err(tg.cpu().numpy().astype(np.float64), lam) <= TOL[dt]
    scale = float(np.max(np.abs(lam)) * np.max(np.abs(x)))
    eps = float(np.finfo(dt).eps)
    for got, want in ((tga, ga), (tgb, gb), (tgc, gc)):
        err = float(np.max(np.abs(got.cpu().numpy() - want)) / np.max(np.abs(want)))
        assert err <= TOL[dt] * scale / np.max(np.abs(want)) + 8 * eps, err
    # s form: gs accumulates lambda_i (x_{i-1} - 2 x_i + x_{i+1})
    s = (0.2 * np.random.default_rng(n + 1).lognormal(0.0, 0.5, (lines, n))).astype(dt)
    sa, sb, sc = orc.implicit_coefs(s)
    lam_s, gas, gbs, gcs = orc.gtsv_adjoint(sa, sb, sc, x, gy, 0)
    gs0 = np.random.default_rng(n + 2).standard_normal((lines, n)).astype(dt)
    gs_ref = gs0 + (-gas + 2.0 * gbs - gcs)
    tg, tgs = _t(gy), _t(gs0)
    trid.gtsv_s_adjoint(_t(s), _t(x), tg, tgs, 0)
    assert _err(tg.cpu().numpy().astype(np.float64), lam_s) <= TOL[dt]
    err = float(np.max(np.abs(tgs.cpu().numpy() - gs_ref)) / np.max(np.abs(gs_ref)))
    bound = TOL[dt] * 4 * float(np.max(np.abs(lam_s)) * np.max(np.abs(x))) / np.max(np.abs(gs_ref)) + 8 * eps
    assert err <= bound, err


# ------------------------------------------ uneven batch with long systems --

def _sys_err(x, ref, off):
    num = np.maximum.reduceat(np.abs(x - ref), off[:-1])
    den = np.maximum.reduceat(np.abs(ref), off[:-1])
    return float(np.max(num / np.maximum(den, 1e-300)))


@pytest.mark.parametrize("prec", ["f64", "f32", "refine"])
def test_varlen_with_systems_beyond_one_workgroup(trid, orc, monkeypatch, prec):
    """Systems of 10^4..10^6 rows among short ones: the long ones take the
    chunked solve after the persistent launch (every plan; the tuner reports them)."""
    rng = np.random.default_rng(150)
    short = np.clip(np.rint(np.exp(rng.uniform(np.log(32), np.log(8192), 300))), 32, 8192).astype(np.int64)
    lens = np.concatenate([short, [10000, 150001, 1000000, 8193]])
    rng.shuffle(lens)
    a32, b32, c32, d64, off = gen.varlen_batch_lengths(lens, seed=151)
    p = {"f64": trid.PREC_F64, "f32": trid.PREC_F32, "refine": trid.PREC_F32_REFINE64}[prec]
    d_in = d64.astype(np.float32).astype(np.float64) if prec == "f32" else d64
    ref = orc.gtsv_varlen(a32, b32, c32, d_in, off)
    if prec == "f64":
        a, b, c, d = (_t(v.astype(np.float64)) for v in (a32, b32, c32, d64))
    elif prec == "f32":
        a, b, c, d = (_t(v.astype(np.float32)) for v in (a32, b32, c32, d64))
    else:
        a, b, c, d = _t(a32), _t(b32), _t(c32), _t(d64)
    x = torch.empty_like(d)
    monkeypatch.setenv("TRID_AUTOTUNE", "1")
    trid.gtsv_varlen(p, a, b, c, d, x, off)
    rep = trid.autotune_report()
    assert rep and all(q["long"] == 4 for q in rep)
    tol = {"f64": 1e-12, "f32": 1e-5, "refine": 1e-9}[prec]
    err = _sys_err(x.cpu().numpy().astype(np.float64), ref, off)
    print("uneven batch with long systems %s: %.3g" % (prec, err))
    assert err <= tol, err
    # replays of the captured launch (counter reset, long systems included)
    x2 = torch.zeros_like(x)
    trid.gtsv_varlen(p, a, b, c, d, x2, off)
    assert torch.equal(x, x2)


def test_varlen_only_long_systems(trid, orc):
    a32, b32, c32, d64, off = gen.varlen_batch_lengths([50000, 9000], seed=152)
    ref = orc.gtsv_varlen(a32, b32, c32, d64, off)
    a, b, c, d = (_t(v.astype(np.float64)) for v in (a32, b32, c32, d64))
    trid.gtsv_varlen(trid.PREC_F64, a, b, c, d, d, off)  # in place
    assert _sys_err(d.cpu().numpy(), ref, off) <= 1e-12
