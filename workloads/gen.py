"""Seeded input generators for the synthetic workloads.

Layout convention for every mesh array: numpy C order with shape
``(batch, nz, ny, nx)`` in 3D, ``(batch, ny, nx)`` in 2D and ``(batch, nx)``
in 1D, so ``x`` is the contiguous (column-major, x-fastest) axis that the
paper's multi-dimensional setting assumes (Section II-B).  ``dims`` passed to
the solvers is ``[nx, ny, nz]`` (fastest first).

Workloads (sizes are parameters so the tests can run the same recipe small):

* ``dd_lines``      -- many independent diagonally dominant systems:
                       a, c ~ U(-1, 1), b = |a| + |c| + U(1, 2), d ~ N(0, 1);
                       the sub-diagonal of each line's first row and the
                       super-diagonal of its last row are zero (eq. (1)).
* ``adi3d_field``   -- initial field u0 ~ U(0, 1) on an nx*ny*nz mesh.
* ``adi2d_varcoef`` -- per-point diffusion numbers s = 0.1*exp(N(0, 0.25)),
                       (0.25 is the variance), and a right-hand side ~ N(0, 1),
                       both rounded to float32.
* ``varlen_batch``  -- systems with lengths log-uniform in [lmin, lmax], packed
                       back to back, coefficients drawn as in ``dd_lines`` and
                       rounded to float32; right-hand side kept in float64.
* ``diffusion3d``   -- kappa ~ lognormal(0, 0.5) per cell, u0 ~ U(0, 1), and a
                       second kappa* from its own seed for the target field.
* ``hv_slv``        -- batched 2D meshes for the SLV-like mixed-derivative
                       model: u0 ~ U(0, 1); a, b ~ U(0.1, 1); c = 2 rho sqrt(a b)
                       with rho ~ U(-0.9, 0.9), so c^2 < 4ab at every point
                       (the operator stays elliptic).

No function here performs any step of the solver; draws happen in a fixed order
so that a given seed always yields the same arrays.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "mesh_shape",
    "dd_lines",
    "dd_mesh",
    "adi3d_field",
    "adi2d_varcoef",
    "varlen_lengths",
    "varlen_batch",
    "diffusion3d",
    "fourier_mode_3d",
    "hv_slv",
    "SEEDS",
]

# Seed of each named workload; the target field of the differentiable run has its own.
SEEDS = {"lines": 0, "adi3d": 1, "adi2d": 2, "varlen": 3, "diffusion3d": 4, "diffusion3d_target": 104, "hv": 5}


def mesh_shape(dims, batch):
    """numpy shape of a mesh with ``dims`` = [nx, (ny, (nz))] and ``batch`` meshes."""
    return (int(batch),) + tuple(int(n) for n in reversed(list(dims)))


def dd_lines(nsys, n, seed=SEEDS["lines"], dtype=np.float64):
    """``nsys`` systems of length ``n`` as (nsys, n) arrays (line-contiguous).

    Draw order: a, c, b increment, d, each as a full (nsys, n) array.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, (nsys, n))
    c = rng.uniform(-1.0, 1.0, (nsys, n))
    inc = rng.uniform(1.0, 2.0, (nsys, n))
    d = rng.standard_normal((nsys, n))
    a[:, 0] = 0.0
    c[:, -1] = 0.0
    b = np.abs(a) + np.abs(c) + inc
    return tuple(np.ascontiguousarray(v, dtype=dtype) for v in (a, b, c, d))


def dd_mesh(dims, batch, seed=0, dtype=np.float64):
    """Per-point diagonally dominant coefficients on a mesh (any solve axis).

    The first-row sub-diagonal and last-row super-diagonal are *not* zeroed:
    they depend on the solve axis, and the solvers ignore them by contract.
    """
    rng = np.random.default_rng(seed)
    shape = mesh_shape(dims, batch)
    a = rng.uniform(-1.0, 1.0, shape)
    c = rng.uniform(-1.0, 1.0, shape)
    inc = rng.uniform(1.0, 2.0, shape)
    d = rng.standard_normal(shape)
    b = np.abs(a) + np.abs(c) + inc
    return tuple(np.ascontiguousarray(v, dtype=dtype) for v in (a, b, c, d))


def adi3d_field(dims=(256, 256, 256), batch=1, seed=SEEDS["adi3d"], dtype=np.float64):
    """Initial field u0 ~ U(0, 1); a float32 run uses the rounded copy."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, mesh_shape(dims, batch))
    return np.ascontiguousarray(u, dtype=dtype)


def adi2d_varcoef(dims=(1024, 1024), batch=64, seed=SEEDS["adi2d"]):
    """(s, d) float32 arrays: s = 0.1*exp(0.5*z1), d = z2, z ~ N(0, 1), drawn s first."""
    rng = np.random.default_rng(seed)
    shape = mesh_shape(dims, batch)
    s = (0.1 * np.exp(0.5 * rng.standard_normal(shape, dtype=np.float32))).astype(np.float32)
    d = rng.standard_normal(shape, dtype=np.float32)
    return np.ascontiguousarray(s), np.ascontiguousarray(d)


def varlen_lengths(nsys, lmin=32, lmax=8192, seed=SEEDS["varlen"]):
    """Lengths L = clamp(round(exp(U(ln lmin, ln lmax))), lmin, lmax), in draw order."""
    rng = np.random.default_rng(seed)
    lens = np.rint(np.exp(rng.uniform(math.log(lmin), math.log(lmax), nsys)))
    return np.clip(lens, lmin, lmax).astype(np.int64), rng


def varlen_batch(nsys=20000, lmin=32, lmax=8192, seed=SEEDS["varlen"]):
    """Packed uneven batch: returns (a32, b32, c32, d64, offsets int64[nsys+1]).

    The coefficients are drawn in float64 as in ``dd_lines`` and rounded to
    float32 (these rounded values are the matrix of record); d stays float64.
    """
    lens, rng = varlen_lengths(nsys, lmin, lmax, seed)
    return _varlen_pack(lens, rng)


def varlen_batch_lengths(lengths, seed):
    """Packed batch of systems with the given lengths (in that order), drawn as
    ``varlen_batch`` draws them."""
    return _varlen_pack(np.asarray(lengths, dtype=np.int64), np.random.default_rng(seed))


def _varlen_pack(lens, rng):
    nsys = len(lens)
    offsets = np.zeros(nsys + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    total = int(offsets[-1])
    a = rng.uniform(-1.0, 1.0, total)
    c = rng.uniform(-1.0, 1.0, total)
    inc = rng.uniform(1.0, 2.0, total)
    d = rng.standard_normal(total)
    a[offsets[:-1]] = 0.0
    c[offsets[1:] - 1] = 0.0
    b = np.abs(a) + np.abs(c) + inc
    return (a.astype(np.float32), b.astype(np.float32), c.astype(np.float32),
            np.ascontiguousarray(d), offsets)


def diffusion3d(dims=(128, 128, 128), batch=1, seed=SEEDS["diffusion3d"],
                target_seed=SEEDS["diffusion3d_target"], dtype=np.float32):
    """(kappa, u0, kappa_star) for the differentiable run; kappa drawn before u0."""
    shape = mesh_shape(dims, batch)
    rng = np.random.default_rng(seed)
    kappa = rng.lognormal(0.0, 0.5, shape)
    u0 = rng.uniform(0.0, 1.0, shape)
    kstar = np.random.default_rng(target_seed).lognormal(0.0, 0.5, shape)
    return tuple(np.ascontiguousarray(v, dtype=dtype) for v in (kappa, u0, kstar))


def hv_slv(dims=(100, 50), batch=300, seed=SEEDS["hv"], dtype=np.float64):
    """(u0, a, b, c) for the SLV-like model; drawn u0, a, b, rho in that order."""
    shape = mesh_shape(dims, batch)
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(0.0, 1.0, shape)
    a = rng.uniform(0.1, 1.0, shape)
    b = rng.uniform(0.1, 1.0, shape)
    rho = rng.uniform(-0.9, 0.9, shape)
    c = 2.0 * rho * np.sqrt(a * b)
    return tuple(np.ascontiguousarray(v, dtype=dtype) for v in (u0, a, b, c))


def fourier_mode_3d(dims, modes):
    """Separable sine mode prod_axis sin(pi*p*(i+1)/(n+1)); zero on the ghost layer.

    This is the field whose decay under one ADI step has a closed form; it is an
    input, built here, not a result.
    """
    fields = []
    for n, p in zip(dims, modes):
        i = np.arange(n, dtype=np.float64)
        fields.append(np.sin(math.pi * p * (i + 1) / (n + 1)))
    out = fields[0]
    for f in fields[1:]:
        out = np.multiply.outer(f, out)
    return np.ascontiguousarray(out[None, ...])
