"""ctypes binding of ``libtrid.so`` (the C ABI of ``include/trid.h``).

Argument marshalling only: every function takes torch tensors already on the
GPU, checks dtype / device / contiguity, and passes raw device pointers, the
mesh extents and the current HIP stream to the library.  There is no other
code path: if the library is missing or no GPU is present, calls raise.

Mesh tensors have shape ``(batch, [nz,] [ny,] nx)`` (C order, x contiguous);
``axis`` counts from x (0 = x, 1 = y, 2 = z).
"""

from __future__ import annotations

import ctypes
import os
import threading

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtrid.so")

TRID_F32, TRID_F64 = 0, 1
PREC_F64, PREC_F32, PREC_F32_REFINE64 = 0, 1, 2
TRID_ADI_GRAPH = 1
TRID_ADI_STREAM = 2
ERRORS = {1: "TRID_ERR_ARG", 2: "TRID_ERR_ALLOC", 3: "TRID_ERR_HIP", 4: "TRID_ERR_UNSUPPORTED"}

# exported symbol -> (argtypes, restype); mirrors include/trid.h
_H = ctypes.c_void_p
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
_I64P = ctypes.POINTER(ctypes.c_int64)
SIGNATURES = {
    "trid_create": ([ctypes.POINTER(_H)], _I),
    "trid_destroy": ([_H], _I),
    "trid_set_stream": ([_H, _P], _I),
    "trid_last_error": ([_H], ctypes.c_char_p),
    "trid_version": ([], _I),
    "trid_set_tile": ([_H, _I, _I], _I),
    "trid_timing_enable": ([_H, _I], _I),
    "trid_timing_read": ([_H, ctypes.c_char_p, _I64], _I),
    "trid_timing_select": ([_H, ctypes.c_char_p, _I], _I),
    "trid_gtsv_batched": ([_H, _I, _P, _P, _P, _P, _I, _I64P, _I, _I64], _I),
    "trid_gtsv_batched_const": ([_H, _I, _D, _D, _D, _P, _I, _I64P, _I, _I64], _I),
    "trid_gtsv_batched_s": ([_H, _I, _P, _P, _I, _I64P, _I, _I64], _I),
    "trid_gtsv_batched_refine": ([_H, _I, _P, _P, _P, _P, _P, _I, _I64P, _I, _I64], _I),
    "trid_gtsv_batched_s_refine": ([_H, _I, _P, _P, _P, _I, _I64P, _I, _I64], _I),
    "trid_gtsv_varlen": ([_H, _I, _P, _P, _P, _P, _P, _I64P, _I64], _I),
    "trid_gtsv_varlen_dev": ([_H, _I, _P, _P, _P, _P, _P, _P, _I64], _I),
    "trid_adi_step": ([_H, _I, _P, _P, _D, _I, _I64P, _I64, _I, ctypes.c_uint], _I),
    "trid_adi_step_noalloc": ([_H, _I, _P, _P, _D, _I, _I64P, _I64, _I, ctypes.c_uint], _I),
    "trid_gtsv_batched_adjoint": ([_H, _I, _P, _P, _P, _P, _P, _P, _P, _P, _I, _I64P, _I, _I64], _I),
    "trid_gtsv_batched_s_adjoint": ([_H, _I, _P, _P, _P, _P, _I, _I64P, _I, _I64], _I),
    "trid_model_gtsv": ([_H, _I, _I, _I, _I64P, _I, _I64, ctypes.POINTER(ctypes.c_double), ctypes.c_char_p,
                         ctypes.c_size_t], _I),
    "trid_autotune_report": ([_H, ctypes.c_char_p, ctypes.c_size_t], _I),
    "trid_cache_report": ([_H, ctypes.c_char_p, ctypes.c_size_t], _I),
    "trid_model_adi": ([_H, _I, _I, _I64P, _I64, _I, _I, ctypes.c_uint, ctypes.POINTER(ctypes.c_double),
                        ctypes.c_char_p, ctypes.c_size_t], _I),
    "trid_model_hv": ([_H, _I, _I64P, _I64, _I, ctypes.c_uint, ctypes.POINTER(ctypes.c_double), ctypes.c_char_p,
                       ctypes.c_size_t], _I),
    "trid_resident_layout": ([_H, _I, _I64, _I64, _I, _I, _I, _I64P, _I], _I),
    "trid_hv_step": ([_H, _I, _P, _P, _P, _P, _D, _D, _I64P, _I64, _I, ctypes.c_uint], _I),
    "trid_adi_step_adjoint": ([_H, _I, _P, _P, _D, _P, _P, _I, _I64P, _I64], _I),
    "trid_adi_step_keep": ([_H, _I, _P, _P, _I, _I64P, _I64, _P, _P, _P], _I),
    "trid_adi_step_adjoint_kept": ([_H, _I, _P, _P, _P, _P, _P, _P, _P, _I, _I64P, _I64], _I),
    "trid_plan_load": ([_H, ctypes.c_char_p], _I),
    "trid_plan_save": ([_H, ctypes.c_char_p], _I),
}

_lib = None
_tls = threading.local()


class TridError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "TRID_ERR"), code, msg))
        self.code = code


def load_library(path=LIB_PATH):
    """Load libtrid.so and declare every exported signature (no GPU needed)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("libtrid.so not built (run __graft_entry__.build()): %s" % path)
        # torch ships its own HIP runtime; loaded first, it also serves libtrid's
        # dependency, so both use one runtime (loading libtrid first would bring
        # in a second copy that sees no device once torch has initialised its own)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def handle():
    """This thread's library handle (created on first use)."""
    h = getattr(_tls, "h", None)
    if h is None:
        lib = load_library()
        hp = _H()
        rc = lib.trid_create(ctypes.byref(hp))
        if rc != 0:
            raise TridError(rc, lib.trid_last_error(None).decode())
        _tls.h = hp
        h = hp
    return h


def _check(rc, h):
    if rc != 0:
        raise TridError(rc, load_library().trid_last_error(h).decode())


def _dtype_code(t):
    import torch

    if t.dtype == torch.float64:
        return TRID_F64
    if t.dtype == torch.float32:
        return TRID_F32
    raise TypeError("tensors must be float32 or float64, got %s" % t.dtype)


def _dev(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("tensors must be on the GPU")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _mesh(t):
    if t.dim() < 2 or t.dim() > 4:
        raise ValueError("mesh tensors have shape (batch, [nz,] [ny,] nx)")
    dims = (ctypes.c_int64 * (t.dim() - 1))(*reversed(t.shape[1:]))
    return t.dim() - 1, dims, t.shape[0]


def _same(ref, *ts):
    for t in ts:
        if t is not None and (t.shape != ref.shape or t.dtype != ref.dtype):
            raise ValueError("all mesh tensors must share shape and dtype")


def _prep(h):
    import torch

    lib = load_library()
    _check(lib.trid_set_stream(h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), h)
    return lib


def set_tile(M=0, L=0):
    """Force the tile plan of later solves on this thread (0, 0 = automatic)."""
    h = handle()
    _check(load_library().trid_set_tile(h, int(M), int(L)), h)


def timing_enable(on=True):
    """Bracket this thread's later launches with HIP events (clears totals)."""
    h = handle()
    _check(load_library().trid_timing_enable(h, 1 if on else 0), h)


def timing_select(name=None, every=1):
    """Time only launches named ``name`` (None: every name), every ``every``-th of each; clears totals."""
    h = handle()
    _check(load_library().trid_timing_select(h, name.encode() if name else None, int(every)), h)


def timing_read():
    """{kernel name: (launch count, total ms)} accumulated since timing_enable."""
    import json

    h = handle()
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load_library().trid_timing_read(h, buf, len(buf)), h)
    return {k: (int(v[0]), float(v[1])) for k, v in json.loads(buf.value.decode()).items()}


TRID_FORM_ARRAYS = 0
TRID_FORM_S = 1


def model_gtsv(dtype, form, dims, axis, batch=1):
    """Predicted kernel microseconds and plan of the batched solve ``gtsv`` (form
    TRID_FORM_ARRAYS) or ``gtsv_s`` (TRID_FORM_S) would launch on meshes of
    ``dims`` = [nx, (ny, (nz))]; host computation only."""
    import json

    import torch

    h = handle()
    lib = load_library()
    code = {torch.float64: TRID_F64, torch.float32: TRID_F32}[dtype]
    d = (ctypes.c_int64 * len(dims))(*dims)
    us = ctypes.c_double()
    buf = ctypes.create_string_buffer(1024)
    _check(lib.trid_model_gtsv(h, code, int(form), len(dims), d, int(axis), int(batch), ctypes.byref(us), buf,
                               len(buf)), h)
    return us.value, json.loads(buf.value.decode())


def model_adi(dtype, dims, batch=1, per_point_s=False, nsteps=1, stream=False):
    """Predicted kernel microseconds of ``adi_step`` on ``batch`` meshes of
    ``dims`` = [nx, ny, (nz)] over ``nsteps`` steps, with the per-kernel split;
    host computation only."""
    import json

    import torch

    h = handle()
    lib = load_library()
    code = {torch.float64: TRID_F64, torch.float32: TRID_F32}[dtype]
    d = (ctypes.c_int64 * len(dims))(*dims)
    us = ctypes.c_double()
    buf = ctypes.create_string_buffer(4096)
    _check(lib.trid_model_adi(h, code, len(dims), d, int(batch), int(bool(per_point_s)), int(nsteps),
                              TRID_ADI_STREAM if stream else 0, ctypes.byref(us), buf, len(buf)), h)
    return us.value, json.loads(buf.value.decode())


def model_hv(dtype, dims, batch=1, nsteps=1, stream=False):
    """Predicted kernel microseconds of ``hv_step`` on ``batch`` meshes of
    ``dims`` = [nx, ny] over ``nsteps`` steps, with the per-kernel split."""
    import json

    import torch

    h = handle()
    lib = load_library()
    code = {torch.float64: TRID_F64, torch.float32: TRID_F32}[dtype]
    d = (ctypes.c_int64 * 2)(*dims)
    us = ctypes.c_double()
    buf = ctypes.create_string_buffer(4096)
    _check(lib.trid_model_hv(h, code, d, int(batch), int(nsteps), TRID_ADI_STREAM if stream else 0,
                             ctypes.byref(us), buf, len(buf)), h)
    return us.value, json.loads(buf.value.decode())


def autotune_report():
    """The most recent uneven-batch autotuning run: per plan the model's
    prediction and the measured time (-1 where the plan was not timed)."""
    import json

    h = handle()
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load_library().trid_autotune_report(h, buf, len(buf)), h)
    return json.loads(buf.value.decode())


def cache_report():
    """Sizes and capacities of this thread's handle caches (captured graphs,
    uneven-batch schedules)."""
    import json

    h = handle()
    buf = ctypes.create_string_buffer(1024)
    _check(load_library().trid_cache_report(h, buf, len(buf)), h)
    return json.loads(buf.value.decode())


def gtsv(a, b, c, d, axis):
    """Solve all lines of ``axis`` in place on d (eqs. (1)-(2), Alg. 1 / eq. (7))."""
    _dev(a, b, c, d)
    _same(d, a, b, c)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(d)
    _check(lib.trid_gtsv_batched(h, _dtype_code(d), a.data_ptr(), b.data_ptr(), c.data_ptr(),
                                 d.data_ptr(), nd, dims, int(axis), batch), h)
    return d


def gtsv_const(a, b, c, d, axis):
    """Solve with the same (a, b, c) on every row, in place on d."""
    _dev(d)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(d)
    _check(lib.trid_gtsv_batched_const(h, _dtype_code(d), float(a), float(b), float(c),
                                       d.data_ptr(), nd, dims, int(axis), batch), h)
    return d


def gtsv_s(s, d, axis):
    """Solve with rows (-s, 1 + 2 s, -s) from a per-point s, in place on d."""
    _dev(s, d)
    _same(d, s)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(d)
    _check(lib.trid_gtsv_batched_s(h, _dtype_code(d), s.data_ptr(), d.data_ptr(), nd, dims,
                                   int(axis), batch), h)
    return d


def gtsv_refine(a, b, c, d, x, axis):
    """FP32 solve + one FP64 refinement: x (float64) = A(a, b, c float32)^{-1} d."""
    import torch

    _dev(a, b, c, d, x)
    _same(a, b, c)
    if a.dtype != torch.float32 or x.dtype != torch.float64 or x.shape != d.shape:
        raise ValueError("refine: a, b, c float32, x float64 of d's shape")
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(d)
    _check(lib.trid_gtsv_batched_refine(h, _dtype_code(d), a.data_ptr(), b.data_ptr(),
                                        c.data_ptr(), d.data_ptr(), x.data_ptr(), nd, dims,
                                        int(axis), batch), h)
    return x


def gtsv_s_refine(s, d, x, axis):
    """FP32 solve + one FP64 refinement with rows (-s, 1 + 2 s, -s), s float32."""
    import torch

    _dev(s, d, x)
    if s.dtype != torch.float32 or x.dtype != torch.float64 or x.shape != d.shape:
        raise ValueError("refine: s float32, x float64 of d's shape")
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(d)
    _check(lib.trid_gtsv_batched_s_refine(h, _dtype_code(d), s.data_ptr(), d.data_ptr(),
                                          x.data_ptr(), nd, dims, int(axis), batch), h)
    return x


def gtsv_varlen(prec, a, b, c, d, x, offsets):
    """Packed uneven batch in one persistent launch; ``offsets`` is a host int64 sequence."""
    import numpy as np

    _dev(a, b, c, d, x)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    h = handle()
    lib = _prep(h)
    _check(lib.trid_gtsv_varlen(h, int(prec), a.data_ptr(), b.data_ptr(), c.data_ptr(),
                                d.data_ptr(), x.data_ptr(),
                                off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                len(off) - 1), h)
    return x


def gtsv_varlen_dev(prec, a, b, c, d, x, offsets):
    """As gtsv_varlen with ``offsets`` an int64 tensor on the GPU (nsys + 1 entries)."""
    import torch

    _dev(a, b, c, d, x, offsets)
    if offsets.dtype != torch.int64 or offsets.dim() != 1 or offsets.numel() < 2:
        raise ValueError("offsets: a 1-D int64 tensor of nsys + 1 entries")
    h = handle()
    lib = _prep(h)
    _check(lib.trid_gtsv_varlen_dev(h, int(prec), a.data_ptr(), b.data_ptr(), c.data_ptr(),
                                    d.data_ptr(), x.data_ptr(), offsets.data_ptr(), offsets.numel() - 1), h)
    return x


def adi_step(u, s=None, s0=0.0, nsteps=1, graph=False, stream=False):
    """``nsteps`` ADI steps (Alg. 3) in place on u; s per point (tensor) or constant s0.

    Small 2D meshes run all steps in one LDS-resident launch unless ``stream``."""
    _dev(u, s)
    _same(u, s)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(u)
    _check(lib.trid_adi_step(h, _dtype_code(u), u.data_ptr(), s.data_ptr() if s is not None else None,
                             float(s0), nd, dims, batch, int(nsteps),
                             (TRID_ADI_GRAPH if graph else 0) | (TRID_ADI_STREAM if stream else 0)), h)
    return u


def adi_step_noalloc(u, s=None, s0=0.0, nsteps=1, stream=False):
    """As adi_step, with the workspace in the library's static device scratch
    (no device allocation; meshes up to TRID_NOALLOC_SCRATCH_BYTES of d)."""
    _dev(u, s)
    _same(u, s)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(u)
    _check(lib.trid_adi_step_noalloc(h, _dtype_code(u), u.data_ptr(), s.data_ptr() if s is not None else None,
                                     float(s0), nd, dims, batch, int(nsteps),
                                     TRID_ADI_STREAM if stream else 0), h)
    return u


def hv_step(u, a, b, c, dt, theta, nsteps=1, stream=False):
    """``nsteps`` Hundsdorfer-Verwer ADI steps of u_t = a u_xx + b u_yy + c u_xy in place
    on the 2D meshes u (batch, ny, nx); a, b, c per point, same shape and dtype.

    Small meshes run all steps in one LDS-resident launch unless ``stream``."""
    _dev(u, a, b, c)
    _same(u, a, b, c)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(u)
    if nd != 2:
        raise ValueError("hv_step takes 2D meshes (batch, ny, nx)")
    _check(lib.trid_hv_step(h, _dtype_code(u), u.data_ptr(), a.data_ptr(), b.data_ptr(), c.data_ptr(),
                            float(dt), float(theta), dims, batch, int(nsteps),
                            TRID_ADI_STREAM if stream else 0), h)
    return u


def gtsv_adjoint(a, b, c, x, g, axis, ga, gb, gc):
    """Reverse mode of the arrays solve: g (in dL/dx, out dL/dd); ga, gb, gc written."""
    _dev(a, b, c, x, g, ga, gb, gc)
    _same(g, a, b, c, x, ga, gb, gc)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(g)
    _check(lib.trid_gtsv_batched_adjoint(h, _dtype_code(g), a.data_ptr(), b.data_ptr(),
                                         c.data_ptr(), x.data_ptr(), g.data_ptr(), ga.data_ptr(),
                                         gb.data_ptr(), gc.data_ptr(), nd, dims, int(axis), batch), h)
    return g, ga, gb, gc


def gtsv_s_adjoint(s, x, g, gs, axis):
    """Reverse mode of the s-form solve: g (in dL/dx, out dL/dd); gs accumulated."""
    _dev(s, x, g, gs)
    _same(g, s, x, gs)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(g)
    _check(lib.trid_gtsv_batched_s_adjoint(h, _dtype_code(g), s.data_ptr(), x.data_ptr(),
                                           g.data_ptr(), gs.data_ptr(), nd, dims, int(axis),
                                           batch), h)
    return g, gs


def adi_step_adjoint(u_t, s, u_bar, s_bar, s0=0.0):
    """One ADI step in reverse from checkpoint u_t: u_bar := dL/du_t, s_bar += dL/ds.

    s is a per-point tensor, or None for the constant s0 (then s_bar receives the
    per-point derivative at s = s0; its sum is dL/ds0).  s_bar may be None."""
    _dev(u_t, s, u_bar, s_bar)
    _same(u_t, s, u_bar, s_bar)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(u_t)
    _check(lib.trid_adi_step_adjoint(h, _dtype_code(u_t), u_t.data_ptr(),
                                     s.data_ptr() if s is not None else None, float(s0), u_bar.data_ptr(),
                                     s_bar.data_ptr() if s_bar is not None else None, nd, dims, batch), h)
    return u_bar, s_bar


def adi_step_keep(u, s, w1, w2, w3=None):
    """One ADI step in place on u (per-point s) that keeps its intermediates in
    w1, w2 and (3D) w3 for adi_step_adjoint_kept."""
    _dev(u, s, w1, w2, w3)
    _same(u, s, w1, w2, w3)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(u)
    _check(lib.trid_adi_step_keep(h, _dtype_code(u), u.data_ptr(), s.data_ptr(), nd, dims, batch,
                                  w1.data_ptr(), w2.data_ptr(), w3.data_ptr() if w3 is not None else None), h)
    return u


def adi_step_adjoint_kept(u_t, s, w1, w2, w3, u_bar, s_bar):
    """Reverse of a kept step: u_bar := dL/du_t, s_bar += dL/ds (no recomputation)."""
    _dev(u_t, s, w1, w2, w3, u_bar, s_bar)
    _same(u_t, s, w1, w2, w3, u_bar, s_bar)
    h = handle()
    lib = _prep(h)
    nd, dims, batch = _mesh(u_t)
    _check(lib.trid_adi_step_adjoint_kept(h, _dtype_code(u_t), u_t.data_ptr(), s.data_ptr(), w1.data_ptr(),
                                          w2.data_ptr(), w3.data_ptr() if w3 is not None else None,
                                          u_bar.data_ptr(), s_bar.data_ptr(), nd, dims, batch), h)
    return u_bar, s_bar


def plan_load(path):
    h = handle()
    _check(load_library().trid_plan_load(h, str(path).encode()), h)


def plan_save(path):
    h = handle()
    _check(load_library().trid_plan_save(h, str(path).encode()), h)
