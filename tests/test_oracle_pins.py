"""Pins of the CPU oracle against things other than itself (CPU only).

Each test fixes the oracle to an independent fact: a library dense solver, exact
rational arithmetic, a manufactured solution built by multiplication (not by
solving), the closed-form decay of a discrete Fourier mode under the ADI step,
algebraic invariants, or finite differences.  The paper (arxiv 2201.03950)
prints no worked numerical example, so no value here comes from it.
"""

import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from workloads import gen

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _dense(a, b, c):
    """Dense matrix of one line (eq. (2)): sub-diagonal a[1:], diagonal b, super-diagonal c[:-1]."""
    n = len(b)
    A = np.diag(np.asarray(b, dtype=np.float64))
    if n > 1:
        A += np.diag(np.asarray(a[1:], dtype=np.float64), -1)
        A += np.diag(np.asarray(c[:-1], dtype=np.float64), 1)
    return A


def _banded_matvec(a, b, c, x, axis):
    """y = A x along ``axis`` of a mesh array, by multiplication (never by solving)."""
    ax = x.ndim - 1 - axis  # numpy axis of the mesh axis
    xm = np.moveaxis(x, ax, -1)
    am, bm, cm = (np.moveaxis(v, ax, -1) for v in (a, b, c))
    y = bm * xm
    y[..., 1:] += am[..., 1:] * xm[..., :-1]
    y[..., :-1] += cm[..., :-1] * xm[..., 1:]
    return np.moveaxis(y, -1, ax)


def _rel_line_err(x, ref, axis):
    ax = x.ndim - 1 - axis
    num = np.max(np.abs(np.moveaxis(x - ref, ax, -1)), axis=-1)
    den = np.max(np.abs(np.moveaxis(ref, ax, -1)), axis=-1)
    return float(np.max(num / np.maximum(den, 1e-300)))


# ----------------------------------------------------------------------------- Alg. 1

@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 16, 33, 64])
def test_thomas_matches_dense_lu(orc, n):
    a, b, c, d = gen.dd_lines(6, n, seed=100 + n)
    x = orc.gtsv(a, b, c, d, 0)
    for k in range(6):
        ref = np.linalg.solve(_dense(a[k], b[k], c[k]), d[k])
        assert np.max(np.abs(x[k] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [2, 5, 64])
def test_thomas_matches_solve_banded(orc, n):
    a, b, c, d = gen.dd_lines(4, n, seed=7)
    x = orc.gtsv(a, b, c, d, 0)
    for k in range(4):
        ab = np.zeros((3, n))
        ab[0, 1:] = c[k, :-1]
        ab[1] = b[k]
        ab[2, :-1] = a[k, 1:]
        ref = scipy.linalg.solve_banded((1, 1), ab, d[k])
        assert np.max(np.abs(x[k] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def _exact_solve(rows, rhs):
    """Gauss-Jordan elimination over the rationals (brute force, exact)."""
    n = len(rhs)
    M = [list(r) + [v] for r, v in zip(rows, rhs)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_thomas_matches_exact_rational(orc, n):
    rng = np.random.default_rng(n)
    a = [Fraction(int(v), 4) for v in rng.integers(-4, 5, n)]
    c = [Fraction(int(v), 4) for v in rng.integers(-4, 5, n)]
    b = [abs(a[i]) + abs(c[i]) + Fraction(int(rng.integers(1, 5)), 2) for i in range(n)]
    d = [Fraction(int(v), 3) for v in rng.integers(-9, 10, n)]
    rows = []
    for i in range(n):
        r = [Fraction(0)] * n
        r[i] = b[i]
        if i > 0:
            r[i - 1] = a[i]
        if i < n - 1:
            r[i + 1] = c[i]
        rows.append(r)
    exact = np.array([float(v) for v in _exact_solve(rows, d)])
    fa, fb, fc, fd = (np.array([[float(v) for v in arr]]) for arr in (a, b, c, d))
    x = orc.gtsv(fa, fb, fc, fd, 0)[0]
    assert np.max(np.abs(x - exact)) <= 4e-15 * max(1.0, np.max(np.abs(exact)))


def test_manufactured_solution_and_residual(orc):
    n = 256
    a, b, c, _ = gen.dd_lines(64, n, seed=11)
    rng = np.random.default_rng(12)
    xt = rng.standard_normal((64, n))
    d = _banded_matvec(a, b, c, xt, 0)
    x = orc.gtsv(a, b, c, d, 0)
    eps = np.finfo(np.float64).eps
    # kappa_inf <= (max row sum)/(min dominance margin) <= 5/1 for this distribution
    assert _rel_line_err(x, xt, 0) <= n * 6 * eps
    res = np.max(np.abs(d - _banded_matvec(a, b, c, x, 0)))
    assert res <= 8 * eps * 5 * np.max(np.abs(x))


def test_first_sub_and_last_super_are_ignored(orc):
    a, b, c, d = gen.dd_lines(5, 17, seed=3)
    x0 = orc.gtsv(a, b, c, d, 0)
    a2, c2 = a.copy(), c.copy()
    a2[:, 0] = 1e30
    c2[:, -1] = np.nan
    x1 = orc.gtsv(a2, b, c2, d, 0)
    assert np.array_equal(x0, x1)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mesh_lines_match_dense_per_line(orc, axis):
    dims, batch = (5, 6, 7), 2
    a, b, c, d = gen.dd_mesh(dims, batch, seed=21 + axis)
    x = orc.gtsv(a, b, c, d, axis)
    ax = 3 - axis
    am, bm, cm, dm, xm = (np.moveaxis(v, ax, -1).reshape(-1, dims[axis]) for v in (a, b, c, d, x))
    for k in range(am.shape[0]):
        ref = np.linalg.solve(_dense(am[k], bm[k], cm[k]), dm[k])
        assert np.max(np.abs(xm[k] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_fp32_thomas_error_within_bound(orc):
    n = 256
    a, b, c, d = (v.astype(np.float32) for v in gen.dd_lines(64, n, seed=1))
    x32 = orc.gtsv_f32(a, b, c, d, 0)
    x64 = orc.gtsv(a, b, c, d, 0)
    err = _rel_line_err(x32.astype(np.float64), x64, 0)
    eps32 = float(np.finfo(np.float32).eps)
    assert 0.0 < err <= n * 6 * eps32


# ----------------------------------------------------------------------------- Alg. 2, eq. (7)

@pytest.mark.parametrize("n", [1, 2, 3, 8, 31, 64, 100])
def test_pcr_matches_thomas_and_zeroes_offdiagonals(orc, n):
    a, b, c, d = gen.dd_lines(1, n, seed=40 + n)
    x, ap, cp = orc.pcr_line(a[0], b[0], c[0], d[0])
    ref = np.linalg.solve(_dense(a[0], b[0], c[0]), d[0])
    assert np.max(np.abs(x - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
    assert np.all(ap == 0.0) and np.all(cp == 0.0)


@pytest.mark.parametrize("n,m", [(1, 3), (5, 3), (64, 4), (65, 4), (256, 16), (250, 16), (1000, 32), (37, 8)])
def test_tiled_modified_thomas_matches_dense(orc, n, m):
    a, b, c, d = gen.dd_lines(1, n, seed=n * 7 + m)
    x = orc.tiled_thomas_line(a[0], b[0], c[0], d[0], m)
    ref = np.linalg.solve(_dense(a[0], b[0], c[0]), d[0])
    assert np.max(np.abs(x - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


# ----------------------------------------------------------------------------- varlen

def test_varlen_matches_dense(orc):
    a, b, c, d, off = gen.varlen_batch(nsys=40, lmin=1, lmax=90, seed=9)
    x = orc.gtsv_varlen(a, b, c, d, off)
    for k in range(40):
        s, e = off[k], off[k + 1]
        ref = np.linalg.solve(_dense(a[s:e], b[s:e], c[s:e]), d[s:e])
        assert np.max(np.abs(x[s:e] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


# ----------------------------------------------------------------------------- Alg. 3 (ADI)

def _mu(p, n):
    return 4.0 * math.sin(math.pi * p / (2.0 * (n + 1))) ** 2


@pytest.mark.parametrize("modes", [(1, 1, 1), (1, 2, 3), (5, 1, 4)])
def test_adi3d_fourier_mode_decays_in_closed_form(orc, modes):
    dims, s, steps = (12, 10, 9), 0.2, 4
    u0 = gen.fourier_mode_3d(dims, modes)
    mus = [_mu(p, n) for p, n in zip(modes, dims)]
    g = 1.0 - 2.0 * s * sum(mus) / math.prod(1.0 + s * m for m in mus)
    u = orc.adi_step(u0, s0=s, nsteps=steps)
    assert np.max(np.abs(u - g ** steps * u0)) <= 1e-13


@pytest.mark.parametrize("modes", [(1, 1), (3, 2), (7, 5)])
def test_adi2d_fourier_mode_decays_in_closed_form(orc, modes):
    dims, s, steps = (16, 11), 0.35, 3
    u0 = gen.fourier_mode_3d(dims, modes)
    mus = [_mu(p, n) for p, n in zip(modes, dims)]
    g = 1.0 - 2.0 * s * sum(mus) / math.prod(1.0 + s * m for m in mus)
    u = orc.adi_step(u0, s0=s, nsteps=steps)
    assert np.max(np.abs(u - g ** steps * u0)) <= 1e-13


def test_xy_solve_of_a_mode_in_closed_form(orc):
    dims, s, modes = (20, 13), 0.3, (4, 6)
    d = gen.fourier_mode_3d(dims, modes)
    out = orc.adi_xy(np.full(d.shape, s), d)
    fac = 1.0 / math.prod(1.0 + s * _mu(p, n) for p, n in zip(modes, dims))
    assert np.max(np.abs(out - fac * d)) <= 1e-14


def test_adi_zero_diffusion_is_identity(orc):
    u = gen.adi3d_field((9, 8, 7), batch=2, seed=5)
    assert np.array_equal(orc.adi_step(u, s0=0.0, nsteps=3), u)


def test_adi_is_linear(orc):
    u = gen.adi3d_field((9, 8, 7), seed=5)
    v = gen.adi3d_field((9, 8, 7), seed=6)
    s = 0.1 + gen.adi3d_field((9, 8, 7), seed=7)
    lhs = orc.adi_step(2.5 * u - 1.5 * v, s=s)
    rhs = 2.5 * orc.adi_step(u, s=s) - 1.5 * orc.adi_step(v, s=s)
    assert np.max(np.abs(lhs - rhs)) <= 1e-13


def test_adi_axis_permutation_symmetry_on_a_cube(orc):
    u = gen.adi3d_field((10, 10, 10), seed=8)
    ref = orc.adi_step(u, s0=0.2, nsteps=2)
    ut = np.ascontiguousarray(np.transpose(u, (0, 3, 2, 1)))  # swap x and z
    out = orc.adi_step(ut, s0=0.2, nsteps=2)
    assert np.max(np.abs(np.transpose(out, (0, 3, 2, 1)) - ref)) <= 1e-13


def test_xy_solve_recovers_manufactured_field_with_variable_s(orc):
    s32, _ = gen.adi2d_varcoef((24, 19), batch=3, seed=5)
    s = s32.astype(np.float64)
    v = np.random.default_rng(6).standard_normal(s.shape)
    a, b, c = -s, 1.0 + 2.0 * s, -s
    d = _banded_matvec(a, b, c, _banded_matvec(a, b, c, v, 1), 0)  # d = X (Y v)
    out = orc.adi_xy(s, d)  # Y^{-1} X^{-1} d
    assert np.max(np.abs(out - v)) <= 1e-13


def test_laplacian_symmetric_and_mode_eigenvalue(orc):
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal((2, 1, 6, 7, 8))
    assert abs(np.sum(orc.laplacian(u) * v) - np.sum(u * orc.laplacian(v))) <= 1e-12
    dims, modes = (8, 7, 6), (2, 3, 1)
    m = gen.fourier_mode_3d(dims, modes)
    lam = -sum(_mu(p, n) for p, n in zip(modes, dims))
    assert np.max(np.abs(orc.laplacian(m) - lam * m)) <= 1e-14


# ----------------------------------------------------------------------------- adjoints

@pytest.mark.parametrize("axis", [0, 1, 2])
def test_adjoint_dot_product(orc, axis):
    a, b, c, d = gen.dd_mesh((6, 5, 7), 2, seed=50 + axis)
    g = np.random.default_rng(axis).standard_normal(d.shape)
    x = orc.gtsv(a, b, c, d, axis)
    lam, _, _, _ = orc.gtsv_adjoint(a, b, c, x, g, axis)
    assert abs(np.sum(x * g) - np.sum(d * lam)) <= 1e-13 * np.sum(np.abs(x * g))


def test_adjoint_coefficient_gradients_match_finite_differences(orc):
    n = 9
    a, b, c, d = gen.dd_lines(1, n, seed=77)
    g = np.random.default_rng(78).standard_normal((1, n))

    def loss(aa, bb, cc, dd):
        return float(np.sum(orc.gtsv(aa, bb, cc, dd, 0) * g))

    x = orc.gtsv(a, b, c, d, 0)
    lam, ga, gb, gc = orc.gtsv_adjoint(a, b, c, x, g, 0)
    for name, arr, grad in (("a", a, ga), ("b", b, gb), ("c", c, gc), ("d", d, lam)):
        for i in range(n):
            h = 1e-6 * max(1.0, abs(arr[0, i]))
            p, m = arr.copy(), arr.copy()
            p[0, i] += h
            m[0, i] -= h
            args_p = {"a": a, "b": b, "c": c, "d": d}
            args_m = dict(args_p)
            args_p[name], args_m[name] = p, m
            fd = (loss(**{k + k: v for k, v in args_p.items()}) -
                  loss(**{k + k: v for k, v in args_m.items()})) / (2 * h)
            assert abs(fd - grad[0, i]) <= 1e-7 * max(1.0, abs(fd)), (name, i)
    assert ga[0, 0] == 0.0 and gc[0, -1] == 0.0


@pytest.mark.parametrize("dims", [(6, 5, 4), (7, 6)])
def test_adi_gradients_match_finite_differences(orc, dims):
    kappa, u0, kstar = (v.astype(np.float64) for v in gen.diffusion3d(dims, seed=4, target_seed=104))
    s0, steps = 0.2, 3
    s = s0 * kappa
    target = orc.adi_step(u0, s=s0 * kstar, nsteps=steps)

    def loss(uu, ss):
        uT = orc.adi_step(uu, s=ss, nsteps=steps)
        return float(np.sum((uT - target) ** 2))

    L, du0, ds = orc.adi_forward_backward(u0, s, target, steps)
    assert abs(L - loss(u0, s)) <= 1e-12 * max(1.0, L)
    rng = np.random.default_rng(5)
    flat = rng.choice(u0.size, size=12, replace=False)
    for f in flat:
        for arr, grad, is_s in ((u0, du0, False), (s, ds, True)):
            idx = np.unravel_index(f, arr.shape)
            h = 1e-6 * max(1.0, abs(arr[idx]))
            p, m = arr.copy(), arr.copy()
            p[idx] += h
            m[idx] -= h
            fd = ((loss(u0, p) - loss(u0, m)) if is_s else (loss(p, s) - loss(m, s))) / (2 * h)
            assert abs(fd - grad[idx]) <= 1e-6 * max(1e-3, abs(fd)), (is_s, idx, fd, grad[idx])


def test_symmetric_constant_transposed_solve_equals_forward(orc):
    d = np.random.default_rng(2).standard_normal((2, 6, 7, 8))
    a, b, c = orc.implicit_coefs(0.3, d.shape)
    x = orc.gtsv(a, b, c, d, 1)
    lam, _, _, _ = orc.gtsv_adjoint(a, b, c, np.zeros_like(d), d, 1)
    assert np.max(np.abs(lam - x)) <= 1e-15


# ------------------------------------------- Hundsdorfer-Verwer (SLV stand-in) --

HV_THETA = 0.5 + math.sqrt(3.0) / 6.0


def _hv_amplification(z1, z2, theta):
    """One HV step on an eigenvector of both one-dimensional operators (z_k = dt lambda_k):
    the scheme's stages applied to scalars."""
    y0 = 1.0 + z1 + z2
    y1 = (y0 - theta * z1) / (1.0 - theta * z1)
    y2 = (y1 - theta * z2) / (1.0 - theta * z2)
    w0 = y0 + 0.5 * (z1 + z2) * (y2 - 1.0)
    w1 = (w0 - theta * z1 * y2) / (1.0 - theta * z1)
    return (w1 - theta * z2 * y2) / (1.0 - theta * z2)


@pytest.mark.parametrize("theta", [HV_THETA, 1.0])
def test_hv_fourier_mode_amplification(orc, theta):
    """c = 0, constant a, b: a product of sine modes is an eigenvector of a D_xx
    (eigenvalue -a mu_p) and b D_yy, so n steps multiply it by R(z1, z2)^n."""
    nx, ny, p, q, a, b, dt, steps = 23, 17, 3, 2, 0.7, 1.3, 0.4, 6
    x = np.arange(1, nx + 1)
    y = np.arange(1, ny + 1)
    u0 = np.sin(np.pi * q * y / (ny + 1))[:, None] * np.sin(np.pi * p * x / (nx + 1))[None, :]
    mu = lambda k, n: 4.0 * math.sin(math.pi * k / (2.0 * (n + 1))) ** 2
    R = _hv_amplification(-dt * a * mu(p, nx), -dt * b * mu(q, ny), theta)
    out = orc.hv_step(u0[None], a, b, 0.0, dt, theta, steps)
    assert np.max(np.abs(out[0] - R ** steps * u0)) <= 1e-13


def test_hv_matches_dense_operators(orc):
    """Per-point a, b, c on tiny meshes: the scheme written with dense matrices
    (the three difference operators assembled entry by entry) and dense solves."""
    nx, ny, batch, dt, theta = 5, 4, 2, 0.3, HV_THETA
    rng = np.random.default_rng(17)
    u = rng.standard_normal((batch, ny, nx))
    a = rng.uniform(0.2, 1.0, (batch, ny, nx))
    b = rng.uniform(0.2, 1.0, (batch, ny, nx))
    c = rng.uniform(-0.3, 0.3, (batch, ny, nx))
    N = nx * ny
    Dxx, Dyy, Dxy = np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, N))
    idx = lambda i, j: j * nx + i
    for j in range(ny):
        for i in range(nx):
            r = idx(i, j)
            Dxx[r, r] = Dyy[r, r] = -2.0
            for di in (-1, 1):
                if 0 <= i + di < nx:
                    Dxx[r, idx(i + di, j)] = 1.0
            for dj in (-1, 1):
                if 0 <= j + dj < ny:
                    Dyy[r, idx(i, j + dj)] = 1.0
            for di in (-1, 1):
                for dj in (-1, 1):
                    if 0 <= i + di < nx and 0 <= j + dj < ny:
                        Dxy[r, idx(i + di, j + dj)] = di * dj / 4.0
    out = orc.hv_step(u, a, b, c, dt, theta, 2)
    I = np.eye(N)
    for m in range(batch):
        A0, A1, A2 = (np.diag(v[m].ravel()) @ D for v, D in ((c, Dxy), (a, Dxx), (b, Dyy)))
        F = A0 + A1 + A2
        U = u[m].ravel()
        for _ in range(2):
            Y0 = U + dt * F @ U
            Y1 = np.linalg.solve(I - theta * dt * A1, Y0 - theta * dt * A1 @ U)
            Y2 = np.linalg.solve(I - theta * dt * A2, Y1 - theta * dt * A2 @ U)
            W0 = Y0 + 0.5 * dt * (F @ Y2 - F @ U)
            W1 = np.linalg.solve(I - theta * dt * A1, W0 - theta * dt * A1 @ Y2)
            U = np.linalg.solve(I - theta * dt * A2, W1 - theta * dt * A2 @ Y2)
        assert np.max(np.abs(out[m].ravel() - U)) <= 1e-13 * max(1.0, np.max(np.abs(U)))


def test_hv_is_second_order_against_the_exact_flow(orc):
    """Independent of the scheme's formulas: the semi-discrete system u' = F u
    (F assembled densely, mixed term included) has the exact solution
    expm(T F) u0; the HV scheme is second order in time, so halving dt divides
    the error at T by about 4."""
    nx, ny, T = 6, 5, 0.8
    rng = np.random.default_rng(23)
    u = rng.standard_normal((1, ny, nx))
    a = rng.uniform(0.2, 0.6, (1, ny, nx))
    b = rng.uniform(0.2, 0.6, (1, ny, nx))
    c = rng.uniform(-0.2, 0.2, (1, ny, nx))
    N = nx * ny
    F = np.zeros((N, N))
    for j in range(ny):
        for i in range(nx):
            r = j * nx + i
            F[r, r] = -2.0 * (a[0, j, i] + b[0, j, i])
            for di, dj, w in ((-1, 0, a), (1, 0, a), (0, -1, b), (0, 1, b)):
                if 0 <= i + di < nx and 0 <= j + dj < ny:
                    F[r, (j + dj) * nx + i + di] += w[0, j, i]
            for di in (-1, 1):
                for dj in (-1, 1):
                    if 0 <= i + di < nx and 0 <= j + dj < ny:
                        F[r, (j + dj) * nx + i + di] += c[0, j, i] * di * dj / 4.0
    exact = scipy.linalg.expm(T * F) @ u.ravel()
    errs = []
    for steps in (8, 16, 32):
        out = orc.hv_step(u, a, b, c, T / steps, HV_THETA, steps)
        errs.append(np.max(np.abs(out.ravel() - exact)))
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.3 <= e1 / e2 <= 4.7, errs


def test_hv_zero_step_is_identity(orc):
    u = np.random.default_rng(3).standard_normal((2, 6, 7))
    assert np.array_equal(orc.hv_step(u, 0.5, 0.5, 0.1, 0.0, HV_THETA, 3), u)
