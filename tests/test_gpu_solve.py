"""GPU parity of the batched line solves and the ADI step against the CPU oracle.

Tolerances (relative error per line in the infinity norm, max over lines):
FP64 <= 1e-12; FP32 <= 1e-5 against the FP64 oracle run on the same
FP32-rounded inputs.  ADI fields use max|u - u_ref| / max|u_ref|.
"""

import math

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
    trid.set_tile(0, 0)


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _line_err(x, ref, axis):
    ax = x.ndim - 1 - axis
    num = np.max(np.abs(np.moveaxis(x - ref, ax, -1)), axis=-1)
    den = np.max(np.abs(np.moveaxis(ref, ax, -1)), axis=-1)
    return float(np.max(num / np.maximum(den, 1e-300)))


def _field_err(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def _product_tol(tol, lam, x, grad, k):
    """Bound on max|error of grad| / max|grad| for grad_i = lambda_i * (k terms
    of x), with x an exact input: |d(grad_i)| <= k max|x| |d(lambda_i)| <=
    k max|x| tol max|lambda|, plus a few roundings of the product and sum."""
    eps = float(np.finfo(x.dtype).eps)
    return tol * k * float(np.max(np.abs(lam)) * np.max(np.abs(x)) / np.max(np.abs(grad))) + 8 * eps


# ------------------------------------------- 1024 systems of 256 rows, FP64 --

@pytest.mark.parametrize("layout", ["x", "y"])
def test_1024_systems_n256_fp64(trid, orc, layout):
    a, b, c, d = gen.dd_lines(1024, 256, seed=0)
    if layout == "x":  # dims [256, 1024], axis 0: each system contiguous
        arrs = [v[None] for v in (a, b, c, d)]
        axis = 0
    else:  # dims [1024, 256], axis 1: systems interleaved
        arrs = [np.ascontiguousarray(v.T)[None] for v in (a, b, c, d)]
        axis = 1
    ref = orc.gtsv(*arrs, axis)
    ta, tb, tc, td = (_t(v) for v in arrs)
    trid.gtsv(ta, tb, tc, td, axis)
    assert _line_err(td.cpu().numpy(), ref, axis) <= 1e-12


@pytest.mark.parametrize("layout", ["x", "y"])
def test_1024_systems_graph_replays_match_eager(trid, orc, layout):
    """The batched solve captured in a torch CUDA graph (the library launches on
    the capturing stream) and replayed three times, with eager work between the
    replays: every replay equals the eager call bitwise and the oracle to 1e-12."""
    a, b, c, d = gen.dd_lines(1024, 256, seed=0)
    arrs = [v[None] if layout == "x" else np.ascontiguousarray(v.T)[None] for v in (a, b, c, d)]
    axis = 0 if layout == "x" else 1
    ref = orc.gtsv(*arrs, axis)
    ta, tb, tc, td0 = (_t(v) for v in arrs)
    eager = td0.clone()
    trid.gtsv(ta, tb, tc, eager, axis)
    td = td0.clone()
    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        warm = td0.clone()
        trid.gtsv(ta, tb, tc, warm, axis)
        with torch.cuda.graph(g, stream=cap):
            trid.gtsv(ta, tb, tc, td, axis)
    torch.cuda.current_stream().wait_stream(cap)
    for _ in range(3):
        td.copy_(td0)
        g.replay()
        other = td0.clone()
        trid.gtsv(ta, tb, tc, other, axis)  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(td, eager)
        assert _line_err(td.cpu().numpy(), ref, axis) <= 1e-12


# ------------------------------------------------------ geometry / plan sweep --

GEOMS = [
    ((5, 6, 7), 2, 0), ((5, 6, 7), 2, 1), ((5, 6, 7), 2, 2),
    ((257, 3), 2, 0), ((3, 300), 1, 1), ((70, 33), 3, 1),
    ((1,), 9, 0), ((2,), 9, 0), ((3,), 9, 0),
    ((64, 1000), 1, 1), ((1000, 5), 1, 0), ((9, 10, 129), 1, 2),
    ((130, 1, 17), 2, 1),
    # y and z lines shorter than a tile: 1, 2 and 3 rows
    ((6, 1), 2, 1), ((6, 2), 2, 1), ((5, 3), 3, 1), ((4, 3, 1), 2, 2), ((4, 3, 2), 2, 2), ((70, 2, 3), 1, 2),
]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("geom", GEOMS, ids=[str(g) for g in GEOMS])
def test_arrays_any_axis(trid, orc, dt, geom):
    dims, batch, axis = geom
    a, b, c, d = (v.astype(dt) for v in gen.dd_mesh(dims, batch, seed=sum(dims) + axis))
    ref = orc.gtsv(a, b, c, d, axis)
    ta, tb, tc, td = (_t(v) for v in (a, b, c, d))
    trid.gtsv(ta, tb, tc, td, axis)
    assert _line_err(td.cpu().numpy().astype(np.float64), ref, axis) <= TOL[dt]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("mode", ["const", "s"])
@pytest.mark.parametrize("geom", [((33, 41, 10), 2, 0), ((33, 41, 10), 2, 1), ((33, 41, 10), 2, 2),
                                  ((300, 7), 1, 0), ((7, 300), 1, 1), ((9, 1100), 1, 1), ((6, 4, 1500), 1, 2),
                                  # 512-row y lines in 672 blocks: the grouped block order's trailing
                                  # partial round
                                  ((1000, 512), 21, 1),
                                  # y and z lines of 1, 2 and 3 rows
                                  ((6, 1), 2, 1), ((70, 2), 2, 1), ((5, 3), 3, 1), ((4, 3, 1), 2, 2),
                                  ((65, 3, 2), 2, 2), ((9, 4, 3), 1, 2)])
def test_generated_coefficients(trid, orc, dt, mode, geom):
    dims, batch, axis = geom
    rng = np.random.default_rng(5)
    shape = gen.mesh_shape(dims, batch)
    d = rng.standard_normal(shape).astype(dt)
    td = _t(d)
    if mode == "const":
        ref = orc.gtsv_const(-0.3, 1.6, -0.3, d, axis)
        trid.gtsv_const(-0.3, 1.6, -0.3, td, axis)
    else:
        s = (0.1 * np.exp(0.5 * rng.standard_normal(shape))).astype(dt)
        ref = orc.gtsv_s(s, d, axis)
        trid.gtsv_s(_t(s), td, axis)
    assert _line_err(td.cpu().numpy().astype(np.float64), ref, axis) <= TOL[dt]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("mode", ["arrays", "s"])
def test_x_lines_large_grid(trid, orc, dt, mode):
    """65,536 x lines of 200 rows: a grid of many thousand blocks (arrays loaded
    one at a time), against the small grids of the other cases (all at once)."""
    a, b, c, d = (v.astype(dt) for v in gen.dd_lines(65536, 200, seed=12))
    td = _t(d[None])
    if mode == "arrays":
        ref = orc.gtsv(a[None], b[None], c[None], d[None], 0)
        trid.gtsv(_t(a[None]), _t(b[None]), _t(c[None]), td, 0)
    else:
        s = (0.5 * b).astype(dt)
        ref = orc.gtsv_s(s[None], d[None], 0)
        trid.gtsv_s(_t(s[None]), td, 0)
    assert _line_err(td.cpu().numpy().astype(np.float64), ref, 0) <= TOL[dt]


@pytest.mark.parametrize("n", [8192, 5001, 4096, 3000])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("mode", ["arrays", "s", "const"])
@pytest.mark.parametrize("axis", [0, 1])
def test_lines_of_maximum_length(trid, orc, dt, mode, axis, n):
    """Lines of TRID_MAX_LINE = 8192 rows, the longest one workgroup holds, and
    of 5001, 4096 and 3000 rows, along x (staged with 16- or 32-row tiles where
    the LDS holds the line; FP64 8192-row lines with each lane loading its own
    8-row tile) and y (strided, 3 lines)."""
    m = 3
    a, b, c, d = (v.astype(dt) for v in gen.dd_lines(m, n, seed=81))
    if axis == 1:  # dims [3, 8192]: the 3 lines interleaved
        a, b, c, d = (np.ascontiguousarray(v.T) for v in (a, b, c, d))
    a, b, c, d = (v[None] for v in (a, b, c, d))
    td = _t(d)
    if mode == "arrays":
        ref = orc.gtsv(a, b, c, d, axis)
        trid.gtsv(_t(a), _t(b), _t(c), td, axis)
    elif mode == "s":
        s = (0.5 * b).astype(dt)
        ref = orc.gtsv_s(s, d, axis)
        trid.gtsv_s(_t(s), td, axis)
    else:
        ref = orc.gtsv_const(-0.3, 1.7, -0.4, d, axis)
        trid.gtsv_const(-0.3, 1.7, -0.4, td, axis)
    assert _line_err(td.cpu().numpy().astype(np.float64), ref, axis) <= TOL[dt]


PLANS = [(8, 1), (8, 2), (8, 16), (8, 64), (16, 1), (16, 8), (16, 32), (32, 1), (32, 4), (32, 8)]


@pytest.mark.parametrize("plan", PLANS, ids=[str(p) for p in PLANS])
@pytest.mark.parametrize("axis", [0, 1])
def test_forced_tile_plans_agree(trid, orc, plan, axis):
    dims = (77, 75) if axis == 0 else (75, 77)
    a, b, c, d = gen.dd_mesh(dims, 3, seed=plan[0] + plan[1])
    ref = orc.gtsv(a, b, c, d, axis)
    trid.set_tile(*plan)
    try:
        ta, tb, tc, td = (_t(v) for v in (a, b, c, d))
        trid.gtsv(ta, tb, tc, td, axis)
    finally:
        trid.set_tile(0, 0)
    assert _line_err(td.cpu().numpy(), ref, axis) <= 1e-12


# ------------------------------------------------------------------------ ADI --

@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("perpoint", [False, True])
@pytest.mark.parametrize("graph", [False, True])
def test_adi3d_small_matches_oracle(trid, orc, dt, perpoint, graph):
    dims, batch, steps = (40, 33, 29), 2, 3
    u = gen.adi3d_field(dims, batch, seed=3).astype(dt)
    s = None
    if perpoint:
        s = (0.2 * np.random.default_rng(4).lognormal(0.0, 0.5, u.shape)).astype(dt)
        ref = orc.adi_step(u, s=s, nsteps=steps)
    else:
        ref = orc.adi_step(u, s0=0.2, nsteps=steps)
    tu = _t(u)
    trid.adi_step(tu, s=_t(s) if s is not None else None, s0=0.2, nsteps=steps, graph=graph)
    if graph:  # replay the captured graph once more and compare with one more oracle step
        trid.adi_step(tu, s=_t(s) if s is not None else None, s0=0.2, nsteps=steps, graph=graph)
        ref = orc.adi_step(ref, s=s, s0=0.2, nsteps=steps)
    assert _field_err(tu.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("perpoint", [False, True])
@pytest.mark.parametrize("stream", [False, True], ids=["resident", "streamed"])
def test_adi2d_small_matches_oracle(trid, orc, dt, perpoint, stream):
    dims, batch, steps = (61, 45), 3, 4
    u = gen.adi3d_field(dims, batch, seed=8).astype(dt)
    s = (0.1 * np.exp(0.5 * np.random.default_rng(9).standard_normal(u.shape))).astype(dt) if perpoint else None
    ref = orc.adi_step(u, s=s, s0=0.3, nsteps=steps)
    tu = _t(u)
    trid.adi_step(tu, s=_t(s) if s is not None else None, s0=0.3, nsteps=steps, stream=stream)
    assert _field_err(tu.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


def _mu(p, n):
    return 4.0 * math.sin(math.pi * p / (2.0 * (n + 1))) ** 2


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_adi3d_256cubed_fourier_decay(trid, dt):
    """Full-size (256^3, bench launch configuration) check against the closed form."""
    dims, modes, s, steps = (256, 256, 256), (3, 5, 2), 0.2, 10
    u0 = gen.fourier_mode_3d(dims, modes)
    mus = [_mu(p, n) for p, n in zip(modes, dims)]
    g = 1.0 - 2.0 * s * sum(mus) / math.prod(1.0 + s * m for m in mus)
    tu = _t(u0.astype(dt))
    trid.adi_step(tu, s0=s, nsteps=steps, graph=True)
    err = float(np.max(np.abs(tu.cpu().numpy().astype(np.float64) - g ** steps * u0)))
    assert err <= (1e-12 if dt == np.float64 else 2e-6), err


def test_adi3d_256cubed_one_step_matches_oracle(trid, orc):
    u = gen.adi3d_field((256, 256, 256), seed=1)
    ref = orc.adi_step(u, s0=0.2, nsteps=1)
    tu = _t(u)
    trid.adi_step(tu, s0=0.2, nsteps=1, graph=True)
    assert _field_err(tu.cpu().numpy(), ref) <= 1e-12


# ------------------------------------------------------------------- adjoints --

@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("geom", [((33, 41, 10), 2, 0), ((33, 41, 10), 2, 1), ((33, 41, 10), 2, 2),
                                  ((260,), 5, 0),
                                  # lines of 1, 2 and 3 rows on every axis
                                  ((1,), 7, 0), ((2,), 7, 0), ((6, 1), 2, 1), ((5, 2), 3, 1), ((4, 3, 3), 2, 2)])
def test_arrays_adjoint_matches_oracle(trid, orc, dt, geom):
    dims, batch, axis = geom
    a, b, c, d = (v.astype(dt) for v in gen.dd_mesh(dims, batch, seed=12))
    x = orc.gtsv(a, b, c, d, axis).astype(dt)
    gy = np.random.default_rng(13).standard_normal(d.shape).astype(dt)
    lam, ga, gb, gc = orc.gtsv_adjoint(a, b, c, x, gy, axis)
    tg = _t(gy)
    tga, tgb, tgc = (torch.empty_like(tg) for _ in range(3))
    trid.gtsv_adjoint(_t(a), _t(b), _t(c), _t(x), tg, axis, tga, tgb, tgc)
    assert _line_err(tg.cpu().numpy().astype(np.float64), lam, axis) <= TOL[dt]
    # each gradient is -lambda_i times a neighbour of x (x exact, an input): the
    # line tolerance on lambda carries over scaled by max|lambda| max|x| / max|grad|
    for got, want in ((tga, ga), (tgb, gb), (tgc, gc)):
        g = got.cpu().numpy()
        if not np.any(want):  # one-row lines: a and c hold only the ignored entries, gradient 0
            assert not np.any(g)
            continue
        err = float(np.max(np.abs(g - want)) / np.max(np.abs(want)))
        assert err <= _product_tol(TOL[dt], lam, x, want, 1), err


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("dims", [(31, 29, 27), (4, 2, 3), (2, 3, 1)], ids=str)
def test_s_adjoint_matches_oracle(trid, orc, dt, axis, dims):
    batch = 2
    rng = np.random.default_rng(20 + axis)
    shape = gen.mesh_shape(dims, batch)
    s = (0.2 * rng.lognormal(0.0, 0.5, shape)).astype(dt)
    x = rng.standard_normal(shape).astype(dt)
    gy = rng.standard_normal(shape).astype(dt)
    gs0 = rng.standard_normal(shape).astype(dt)
    a, b, c = orc.implicit_coefs(s)
    lam, ga, gb, gc = orc.gtsv_adjoint(a, b, c, x, gy, axis)
    gs_ref = gs0 + (-ga + 2.0 * gb - gc)
    tg, tgs = _t(gy), _t(gs0)
    trid.gtsv_s_adjoint(_t(s), _t(x), tg, tgs, axis)
    assert _line_err(tg.cpu().numpy().astype(np.float64), lam, axis) <= TOL[dt]
    # gs += lambda_i (x_{i-1} - 2 x_i + x_{i+1}): |second difference| <= 4 max|x|
    err = float(np.max(np.abs(tgs.cpu().numpy() - gs_ref)) / np.max(np.abs(gs_ref)))
    assert err <= _product_tol(TOL[dt], lam, x, gs_ref, 4), err


# staged x solves: every reduced-solve form (DPP row shifts for P = 1..16 tiles
# per line, LDS PCR for 32 and for P not a power of two), both tile sizes
STAGED_P = [8, 16, 24, 32, 64, 100, 128, 256]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("M", [8, 16])
@pytest.mark.parametrize("n", STAGED_P)
def test_staged_x_every_reduced_form(trid, orc, dt, M, n):
    lines = 37  # ragged last block for every L
    a, b, c, d = (v.astype(dt) for v in gen.dd_mesh((n,), lines, seed=n + M))
    ref = orc.gtsv(a, b, c, d, 0)
    s = (0.2 * np.random.default_rng(n).lognormal(0.0, 0.5, d.shape)).astype(dt)
    ref_s = orc.gtsv_s(s, d, 0)
    trid.set_tile(M, 0)
    try:
        td = _t(d)
        trid.gtsv(_t(a), _t(b), _t(c), td, 0)
        ts = _t(d)
        trid.gtsv_s(_t(s), ts, 0)
        u = gen.adi3d_field((n, 6, 5), 2, seed=n).astype(dt)
        sp = (0.2 * np.random.default_rng(n + 1).lognormal(0.0, 0.5, u.shape)).astype(dt)
        ref_u = orc.adi_step(u, s=sp, nsteps=2)
        tu = _t(u)
        trid.adi_step(tu, s=_t(sp), nsteps=2)
    finally:
        trid.set_tile(0, 0)
    assert _line_err(td.cpu().numpy().astype(np.float64), ref, 0) <= TOL[dt]
    assert _line_err(ts.cpu().numpy().astype(np.float64), ref_s, 0) <= TOL[dt]
    assert _field_err(tu.cpu().numpy().astype(np.float64), ref_u) <= TOL[dt]


# fused stencil + x solves: whole lines per wavefront (P = nx / 8 tiles not a
# power of two: Table 3's 48..112-point meshes, a two-lines-per-wavefront
# length), the 16-byte staged per-point kernel (nx = 8 P, also rows spanning
# two wavefronts at 512 FP64), the constant-row kernels; per-point and
# constant s, ragged last blocks, and planes of whole blocks (slab order)
RHS_LANES = [((80, 7, 5), 2), ((96, 5, 3), 3), ((112, 3, 4), 2), ((48, 9, 2), 2), ((200, 4, 3), 1),
             ((80, 11), 3), ((512, 3, 2), 2), ((32, 9, 5), 3), ((64, 7), 5), ((128, 5, 3), 1), ((256, 3, 3), 1),
             ((80, 40, 3), 2), ((96, 32, 4), 1)]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("perpoint", [False, True])
@pytest.mark.parametrize("dims,batch", RHS_LANES, ids=[str(g) for g in RHS_LANES])
def test_rhs_x_whole_lines_per_wavefront(trid, orc, dt, perpoint, dims, batch):
    u = gen.adi3d_field(dims, batch, seed=dims[0]).astype(dt)
    s = (0.2 * np.random.default_rng(dims[1]).lognormal(0.0, 0.5, u.shape)).astype(dt) if perpoint else None
    ref = orc.adi_step(u, s=s, s0=0.2, nsteps=2)
    tu = _t(u)
    trid.adi_step(tu, s=_t(s) if s is not None else None, s0=0.2, nsteps=2, stream=True)
    assert _field_err(tu.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("perpoint", [False, True])
def test_adi_step_on_unaligned_views(trid, orc, dt, perpoint):
    """Arrays one element past a 16-byte boundary: the 16-byte staged kernels
    decline them and the general kernels run (same results)."""
    dims, batch = (64, 12, 5), 2
    u = gen.adi3d_field(dims, batch, seed=21).astype(dt)
    s = (0.2 * np.random.default_rng(22).lognormal(0.0, 0.5, u.shape)).astype(dt) if perpoint else None
    ref = orc.adi_step(u, s=s, s0=0.2, nsteps=2)

    def unaligned(a):
        buf = torch.zeros(a.size + 1, dtype=_t(a).dtype, device="cuda")
        v = buf[1:].view(a.shape)
        v.copy_(_t(a))
        return v

    tu = unaligned(u)
    assert tu.data_ptr() % 16 != 0
    trid.adi_step(tu, s=unaligned(s) if s is not None else None, s0=0.2, nsteps=2, stream=True)
    assert _field_err(tu.cpu().numpy().astype(np.float64), ref) <= TOL[dt]


# x lines take the LDS-staged transposed solve: line lengths across the tile
# sizes and the one-line-per-block limit, line counts with a ragged last block
S_ADJ_X = [(1, 7), (2, 5), (8, 33), (9, 70), (33, 9), (64, 21), (100, 10), (128, 19), (255, 13), (256, 40),
           (1000, 3), (2048, 2), (2100, 3)]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("n,lines", S_ADJ_X, ids=[str(g) for g in S_ADJ_X])
def test_s_adjoint_x_lines(trid, orc, dt, n, lines):
    rng = np.random.default_rng(n + lines)
    shape = gen.mesh_shape((n,), lines)
    s = (0.2 * rng.lognormal(0.0, 0.5, shape)).astype(dt)
    x = rng.standard_normal(shape).astype(dt)
    gy = rng.standard_normal(shape).astype(dt)
    gs0 = rng.standard_normal(shape).astype(dt)
    a, b, c = orc.implicit_coefs(s)
    lam, ga, gb, gc = orc.gtsv_adjoint(a, b, c, x, gy, 0)
    gs_ref = gs0 + (-ga + 2.0 * gb - gc)
    tg, tgs = _t(gy), _t(gs0)
    trid.gtsv_s_adjoint(_t(s), _t(x), tg, tgs, 0)
    assert _line_err(tg.cpu().numpy().astype(np.float64), lam, 0) <= TOL[dt]
    err = float(np.max(np.abs(tgs.cpu().numpy() - gs_ref)) / max(np.max(np.abs(gs_ref)), 1e-30))
    assert err <= _product_tol(TOL[dt], lam, x, gs_ref, 4), err


# ------------------------------------------------ constant-row fast path ----

CONST_GEOMS = [((64, 96, 32), 2, 0), ((64, 96, 32), 2, 1), ((64, 96, 32), 2, 2),
               ((256, 3), 5, 0), ((100, 256), 1, 1), ((70, 3, 128), 1, 2), ((32,), 7, 0),
               ((80, 7), 3, 0), ((96, 5, 3), 2, 0), ((48, 9), 4, 0), ((112, 3), 5, 0), ((160, 3), 2, 0),
               # strided lines whose count per outer index is not a multiple of 64: blocks run on
               # across outer indices
               ((80, 80, 9), 2, 1), ((80, 80, 9), 2, 2), ((96, 40, 7), 1, 1), ((33, 41, 10), 2, 1),
               ((33, 41, 10), 2, 2)]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("geom", CONST_GEOMS, ids=[str(g) for g in CONST_GEOMS])
def test_const_fast_path_matches_oracle(trid, orc, dt, geom):
    dims, batch, axis = geom
    d = np.random.default_rng(31).standard_normal(gen.mesh_shape(dims, batch)).astype(dt)
    ref = orc.gtsv_const(-0.2, 1.4, -0.2, d, axis)
    td = _t(d)
    trid.gtsv_const(-0.2, 1.4, -0.2, td, axis)
    assert _line_err(td.cpu().numpy().astype(np.float64), ref, axis) <= TOL[dt]


@pytest.mark.parametrize("dt", [np.float64, np.float32])
@pytest.mark.parametrize("dims,batch", [((64, 96, 32), 2), ((256, 40, 24), 1), ((128, 70), 3),
                                         ((32, 3, 5), 2), ((64, 5, 7), 3), ((64, 1, 9), 1), ((32, 2), 5),
                                         ((80, 80, 80), 1), ((96, 24, 40), 2)])
def test_adi_const_fast_path_matches_oracle(trid, orc, dt, dims, batch):
    u = gen.adi3d_field(dims, batch, seed=4).astype(dt)
    ref = orc.adi_step(u, s0=0.2, nsteps=3)
    tu = _t(u)
    trid.adi_step(tu, s0=0.2, nsteps=3, stream=True)  # the per-step kernels, also in 2D
    assert _field_err(tu.cpu().numpy().astype(np.float64), ref) <= TOL[dt]
