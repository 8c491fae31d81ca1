"""Python face of the CPU oracle (``trid_oracle.c``), built with gcc and loaded by ctypes.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module; the HIP library and its
Python binding never do.

Every array is a numpy mesh in the layout of ``workloads.gen``: shape
``(batch, [nz,] [ny,] nx)``, C order, so x is contiguous.  ``axis`` counts from
x: 0 = x, 1 = y, 2 = z.  Functions return new arrays; inputs are not modified.

Paper references (arxiv 2201.03950): the problem is eqs. (1)-(2); ``gtsv`` is
Alg. 1 (Thomas) applied to every line of one axis (Section II-B); ``pcr_line``
is Alg. 2; ``tiled_thomas_line`` is the tiled modified Thomas of eq. (7)
(Section III-B); ``adi_step`` is Alg. 3 (Section IV-A) in the Douglas delta
form; ``gtsv_adjoint`` and ``adi_step_adjoint`` are the reverse-mode
derivatives of the same computations (not in the paper).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trid_oracle.c")
_LIB = os.path.join(_HERE, "libtrid_oracle.so")

_lib = None


def build(force=False):
    """Compile the oracle library with gcc (plain -O2, IEEE arithmetic, OpenMP over lines)."""
    stale = os.path.exists(_LIB) and os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L = ctypes.c_long
        I = ctypes.c_int
        D = ctypes.c_double
        LP = ctypes.POINTER(ctypes.c_long)
        sig = {
            "orc_num_threads": ([], I),
            "orc_set_num_threads": ([I], None),
            "orc_gtsv": ([P, P, P, P, I, LP, I, L], I),
            "orc_gtsv_f32": ([P, P, P, P, I, LP, I, L], I),
            "orc_gtsv_varlen": ([P, P, P, P, LP, L], I),
            "orc_pcr_line": ([L, P, P, P, P], I),
            "orc_tiled_thomas_line": ([L, P, P, P, P, L], I),
            "orc_laplacian": ([P, P, I, LP, L], I),
            "orc_adi_step": ([P, P, D, I, LP, L, I], I),
            "orc_gtsv_adjoint": ([P, P, P, P, P, P, P, P, I, LP, I, L], I),
            "orc_adi_step_adjoint": ([P, P, P, P, I, LP, L], I),
            "orc_hv_step": ([P, P, P, P, D, D, LP, L, I], I),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(x):
    return x.ctypes.data_as(ctypes.c_void_p)


def _geom(arr):
    """(ndim, dims array, batch) of a mesh array of shape (batch, ..., nx)."""
    if arr.ndim < 2 or arr.ndim > 4:
        raise ValueError("mesh arrays have shape (batch, [nz,] [ny,] nx)")
    dims = (ctypes.c_long * (arr.ndim - 1))(*reversed(arr.shape[1:]))
    return arr.ndim - 1, dims, arr.shape[0]


def _check(rc, name):
    if rc != 0:
        raise ValueError("oracle %s rejected its arguments" % name)


def num_threads():
    return _load().orc_num_threads()


def set_num_threads(n):
    _load().orc_set_num_threads(int(n))


def gtsv(a, b, c, d, axis):
    """Solve every line of ``axis`` (Alg. 1); a at each line's first row and c at its last are ignored."""
    lib = _load()
    a, b, c = _f64(a), _f64(b), _f64(c)
    x = _f64(d).copy()
    ndim, dims, batch = _geom(x)
    _check(lib.orc_gtsv(_ptr(a), _ptr(b), _ptr(c), _ptr(x), ndim, dims, axis, batch), "gtsv")
    return x


def gtsv_f32(a, b, c, d, axis):
    """Alg. 1 with every operation in binary32 (only to report an unrefined FP32 error)."""
    lib = _load()
    a, b, c = (np.ascontiguousarray(v, dtype=np.float32) for v in (a, b, c))
    x = np.ascontiguousarray(d, dtype=np.float32).copy()
    ndim, dims, batch = _geom(x)
    _check(lib.orc_gtsv_f32(_ptr(a), _ptr(b), _ptr(c), _ptr(x), ndim, dims, axis, batch), "gtsv_f32")
    return x


def implicit_coefs(s, shape=None):
    """Rows of the implicit ADI operator along any axis: a = c = -s, b = 1 + 2 s (Alg. 3)."""
    s = np.asarray(s, dtype=np.float64)
    if shape is not None:
        s = np.broadcast_to(s, shape)
    a = np.ascontiguousarray(-s)
    return a, np.ascontiguousarray(1.0 + 2.0 * s), a.copy()


def gtsv_s(s, d, axis):
    """Line solves with a = c = -s, b = 1 + 2 s (s per point, or a scalar)."""
    a, b, c = implicit_coefs(s, np.shape(d))
    return gtsv(a, b, c, d, axis)


def gtsv_const(a0, b0, c0, d, axis):
    """Line solves with the same (a0, b0, c0) on every row."""
    shape = np.shape(d)
    return gtsv(np.full(shape, a0), np.full(shape, b0), np.full(shape, c0), d, axis)


def gtsv_varlen(a, b, c, d, offsets):
    """Packed systems: system k occupies [offsets[k], offsets[k+1])."""
    lib = _load()
    a, b, c = _f64(a), _f64(b), _f64(c)
    x = _f64(d).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_long))
    _check(lib.orc_gtsv_varlen(_ptr(a), _ptr(b), _ptr(c), _ptr(x), offp, len(off) - 1), "gtsv_varlen")
    return x


def pcr_line(a, b, c, d):
    """Alg. 2 on one line; returns (x, a_P, c_P), the level-P off-diagonals being exact zeros."""
    lib = _load()
    a, b, c, d = (_f64(v).copy() for v in (a, b, c, d))
    _check(lib.orc_pcr_line(len(d), _ptr(a), _ptr(b), _ptr(c), _ptr(d)), "pcr_line")
    return d, a, c


def tiled_thomas_line(a, b, c, d, m):
    """Tiled modified Thomas (eq. (7)) with tiles of ``m`` rows and a Thomas reduced solve."""
    lib = _load()
    a, b, c = _f64(a), _f64(b), _f64(c)
    x = _f64(d).copy()
    _check(lib.orc_tiled_thomas_line(len(x), _ptr(a), _ptr(b), _ptr(c), _ptr(x), int(m)),
           "tiled_thomas_line")
    return x


def laplacian(u):
    """(L u) with zero ghosts: 7-point in 3D, 5-point in 2D, 3-point in 1D."""
    lib = _load()
    u = _f64(u)
    out = np.empty_like(u)
    ndim, dims, batch = _geom(u)
    _check(lib.orc_laplacian(_ptr(u), _ptr(out), ndim, dims, batch), "laplacian")
    return out


def adi_step(u, s=None, s0=0.0, nsteps=1):
    """``nsteps`` ADI steps (Alg. 3): d = 2 s L u; solve along x, y(, z); u += d."""
    lib = _load()
    x = _f64(u).copy()
    sp = None
    if s is not None:
        sp = _f64(np.broadcast_to(s, x.shape))
    ndim, dims, batch = _geom(x)
    _check(lib.orc_adi_step(_ptr(x), _ptr(sp) if sp is not None else None, float(s0), ndim, dims,
                            batch, int(nsteps)), "adi_step")
    return x


def hv_step(u, a, b, c, dt, theta, nsteps=1):
    """``nsteps`` Hundsdorfer-Verwer steps of u_t = a u_xx + b u_yy + c u_xy on 2D
    meshes (batch, ny, nx), zero ghosts: the synthetic stand-in for the call
    structure of Alg. 4 (predictor stencils alternating with x and y solves)."""
    lib = _load()
    x = _f64(u).copy()
    a, b, c = (_f64(np.broadcast_to(v, x.shape)) for v in (a, b, c))
    ndim, dims, batch = _geom(x)
    if ndim != 2:
        raise ValueError("hv_step takes 2D meshes")
    _check(lib.orc_hv_step(_ptr(x), _ptr(a), _ptr(b), _ptr(c), float(dt), float(theta), dims, batch,
                           int(nsteps)), "hv_step")
    return x


def adi_xy(s, d):
    """x-solve then y-solve of a given 2D right-hand side, rows (-s, 1 + 2 s, -s)."""
    return gtsv_s(s, gtsv_s(s, d, 0), 1)


def gtsv_adjoint(a, b, c, x, g, axis):
    """Adjoint of x = A^{-1} d along ``axis``: returns (dL/dd, dL/da, dL/db, dL/dc) given g = dL/dx."""
    lib = _load()
    a, b, c, x = _f64(a), _f64(b), _f64(c), _f64(x)
    lam = _f64(g).copy()
    ga, gb, gc = np.empty_like(lam), np.empty_like(lam), np.empty_like(lam)
    ndim, dims, batch = _geom(lam)
    _check(lib.orc_gtsv_adjoint(_ptr(a), _ptr(b), _ptr(c), _ptr(x), _ptr(lam), _ptr(ga), _ptr(gb),
                                _ptr(gc), ndim, dims, axis, batch), "gtsv_adjoint")
    return lam, ga, gb, gc


def adi_step_adjoint(u_t, s, ubar, sbar=None):
    """One ADI step backwards from the checkpoint u_t: returns (dL/du_t, sbar + dL/ds of this step)."""
    lib = _load()
    u_t = _f64(u_t)
    s = _f64(np.broadcast_to(s, u_t.shape))
    ub = _f64(ubar).copy()
    sb = np.zeros_like(u_t) if sbar is None else _f64(sbar).copy()
    ndim, dims, batch = _geom(u_t)
    _check(lib.orc_adi_step_adjoint(_ptr(u_t), _ptr(s), _ptr(ub), _ptr(sb), ndim, dims, batch),
           "adi_step_adjoint")
    return ub, sb


def adi_forward_backward(u0, s, u_target, nsteps):
    """Loss sum((u_T - u_target)^2) and its gradients (dL/du0, dL/ds) by per-step checkpoints."""
    ckpt = [_f64(u0)]
    for _ in range(nsteps):
        ckpt.append(adi_step(ckpt[-1], s=s, nsteps=1))
    diff = ckpt[-1] - _f64(u_target)
    loss = float(np.sum(diff * diff))
    ubar = 2.0 * diff
    sbar = np.zeros_like(ckpt[0])
    for t in range(nsteps - 1, -1, -1):
        ubar, sbar = adi_step_adjoint(ckpt[t], s, ubar, sbar)
    return loss, ubar, sbar
