"""The C ABI without a GPU: the library loads, exports every declared symbol, and
validates arguments on the host before any HIP call (CPU only)."""

import ctypes
import os
import re

import pytest

from paper_2201_03950_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "trid.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(trid_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2201_03950_amd import build

        build.build()
    return B.load_library()


@pytest.fixture()
def h(lib):
    hp = ctypes.c_void_p()
    assert lib.trid_create(ctypes.byref(hp)) == 0
    yield hp
    assert lib.trid_destroy(hp) == 0


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.SIGNATURES), set(names) ^ set(B.SIGNATURES)


def test_version_and_create_null(lib):
    assert lib.trid_version() >= 10000
    assert lib.trid_create(None) == 1
    assert b"NULL" in lib.trid_last_error(None)
    assert lib.trid_destroy(None) == 0


def _dims(*v):
    return (ctypes.c_int64 * len(v))(*v)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
U = ctypes.c_void_p(0x3000)  # a distinct fake array (entry points that reject aliasing)


@pytest.mark.parametrize(
    "ndim,dims,axis,batch,dt",
    [
        (0, (4,), 0, 1, 1),
        (4, (4, 4, 4, 4), 0, 1, 1),
        (2, (4, 4), 2, 1, 1),
        (2, (4, 4), -1, 1, 1),
        (2, (4, 0), 0, 1, 1),
        (2, (4, 4), 0, 0, 1),
        (2, (4, 4), 0, 1, 7),
    ],
)
def test_gtsv_rejects_bad_geometry(lib, h, ndim, dims, axis, batch, dt):
    rc = lib.trid_gtsv_batched(h, dt, FAKE, FAKE, FAKE, FAKE, ndim, _dims(*dims), axis, batch)
    assert rc == 1
    assert lib.trid_last_error(h) != b""


def test_null_pointers_rejected(lib, h):
    d = _dims(8, 8)
    assert lib.trid_gtsv_batched(h, 1, None, FAKE, FAKE, FAKE, 2, d, 0, 1) == 1
    assert lib.trid_gtsv_batched_const(h, 1, -1.0, 4.0, -1.0, None, 2, d, 0, 1) == 1
    assert lib.trid_gtsv_batched_s(h, 1, None, FAKE, 2, d, 0, 1) == 1
    assert lib.trid_gtsv_batched(h, 1, FAKE, FAKE, FAKE, FAKE, 2, None, 0, 1) == 1
    assert lib.trid_adi_step(h, 1, None, None, 0.2, 3, _dims(8, 8, 8), 1, 1, 0) == 1
    assert lib.trid_gtsv_batched_adjoint(h, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, 2, d, 0, 1) == 1
    assert lib.trid_gtsv_batched_s_adjoint(h, 1, FAKE, FAKE, None, FAKE, 2, d, 0, 1) == 1
    assert lib.trid_gtsv_batched(None, 1, FAKE, FAKE, FAKE, FAKE, 2, d, 0, 1) == 1


def test_line_longer_than_limit_is_unsupported(lib, h):
    # strided lines (axis > 0) stay within one workgroup
    rc = lib.trid_gtsv_batched(h, 1, FAKE, FAKE, FAKE, FAKE, 2, _dims(4, 8193), 1, 1)
    assert rc == 4
    assert b"TRID_MAX_LINE" in lib.trid_last_error(h)
    # contiguous lines take the chunked solve up to TRID_MAX_LONG_LINE
    rc = lib.trid_gtsv_batched_s(h, 1, FAKE, FAKE, 1, _dims(8388609), 0, 1)
    assert rc == 4
    assert b"TRID_MAX_LONG_LINE" in lib.trid_last_error(h)
    # the refinement and adjoint solves take the chunked solve for contiguous
    # lines too, and keep strided lines within one workgroup
    rc = lib.trid_gtsv_batched_refine(h, 1, FAKE, FAKE, FAKE, FAKE, ctypes.c_void_p(0x2000), 1, _dims(8388609), 0, 1)
    assert rc == 4
    assert b"TRID_MAX_LONG_LINE" in lib.trid_last_error(h)
    rc = lib.trid_gtsv_batched_refine(h, 1, FAKE, FAKE, FAKE, FAKE, ctypes.c_void_p(0x2000), 2, _dims(3, 8193), 1, 1)
    assert rc == 4
    rc = lib.trid_gtsv_batched_s_adjoint(h, 1, FAKE, FAKE, FAKE, FAKE, 2, _dims(3, 8193), 1, 1)
    assert rc == 4
    assert b"TRID_MAX_LINE" in lib.trid_last_error(h)


def test_adi_argument_checks(lib, h):
    assert lib.trid_adi_step(h, 1, FAKE, None, 0.2, 1, _dims(8), 1, 1, 0) == 1  # ADI needs 2D/3D
    assert lib.trid_adi_step(h, 1, FAKE, None, 0.2, 3, _dims(8, 8, 8), 1, -1, 0) == 1
    assert lib.trid_adi_step(h, 1, FAKE, None, 0.2, 3, _dims(8, 8, 8), 1, 1, 8) == 1  # unknown flag
    assert lib.trid_adi_step(h, 1, FAKE, None, 0.2, 3, _dims(8, 8, 8), 1, 0, 0) == 0  # no steps: no-op
    assert lib.trid_adi_step(h, 1, FAKE, None, 0.2, 2, _dims(8, 8), 1, 0, 3) == 0  # graph | stream: valid flags
    assert lib.trid_adi_step(h, 1, FAKE, None, 0.2, 2, _dims(8, 8), 1, 0, 4) == 1  # unknown flag


def test_set_tile_validation(lib, h):
    assert lib.trid_set_tile(h, 7, 0) == 1
    assert lib.trid_set_tile(h, 8, 3) == 1
    assert lib.trid_set_tile(h, 16, 32) == 0
    assert lib.trid_set_tile(h, 0, 0) == 0
    assert lib.trid_set_tile(None, 0, 0) == 1


def test_timing_select_validation(lib, h):
    assert lib.trid_timing_select(None, b"adi_y", 1) == 1
    assert lib.trid_timing_select(h, b"x" * 201, 1) == 1
    assert lib.trid_timing_select(h, b"adi_y", 0) == 1
    assert lib.trid_timing_select(h, b"adi_z_update", 4) == 0
    assert lib.trid_timing_select(h, None, 0) == 1
    assert lib.trid_timing_select(h, None, 3) == 0
    assert lib.trid_timing_select(h, b"", 1) == 0


def test_set_stream_and_error_text(lib, h):
    assert lib.trid_set_stream(h, None) == 0
    assert lib.trid_set_stream(None, None) == 1
    assert lib.trid_gtsv_batched(h, 1, FAKE, FAKE, FAKE, FAKE, 5, _dims(1), 0, 1) == 1
    assert b"ndim" in lib.trid_last_error(h)


def test_varlen_argument_checks(lib, h):
    off = (ctypes.c_int64 * 4)(0, 3, 3, 7)  # a zero-length system
    assert lib.trid_gtsv_varlen(h, 0, FAKE, FAKE, FAKE, FAKE, FAKE, off, 3) == 1
    off = (ctypes.c_int64 * 3)(1, 3, 7)  # offsets[0] != 0
    assert lib.trid_gtsv_varlen(h, 0, FAKE, FAKE, FAKE, FAKE, FAKE, off, 2) == 1
    off = (ctypes.c_int64 * 2)(0, 8388609)  # longer than TRID_MAX_LONG_LINE
    assert lib.trid_gtsv_varlen(h, 0, FAKE, FAKE, FAKE, FAKE, FAKE, off, 1) == 4
    off = (ctypes.c_int64 * 2)(0, 10)
    assert lib.trid_gtsv_varlen(h, 9, FAKE, FAKE, FAKE, FAKE, FAKE, off, 1) == 1  # bad precision
    assert lib.trid_gtsv_varlen(h, 2, FAKE, FAKE, FAKE, FAKE, FAKE, off, 1) == 1  # x aliases d (refine)
    assert lib.trid_gtsv_varlen(h, 0, FAKE, FAKE, FAKE, FAKE, FAKE, None, 1) == 1
    # device offsets: checked before the offsets are read
    assert lib.trid_gtsv_varlen_dev(h, 0, FAKE, FAKE, FAKE, FAKE, FAKE, None, 1) == 1
    assert lib.trid_gtsv_varlen_dev(h, 0, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 0) == 1  # nsys
    assert lib.trid_gtsv_varlen_dev(h, 9, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 1) == 1  # precision
    assert lib.trid_gtsv_varlen_dev(h, 0, None, FAKE, FAKE, FAKE, FAKE, FAKE, 1) == 1
    assert lib.trid_gtsv_varlen_dev(None, 0, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 1) == 1


def test_cache_report(lib, h):
    """A new handle holds no captured graphs or schedules; the caps are positive."""
    import json

    buf = ctypes.create_string_buffer(512)
    assert lib.trid_cache_report(h, buf, len(buf)) == 0
    rep = json.loads(buf.value.decode())
    assert rep["adi_graphs"] == rep["varlen_schedules"] == rep["varlen_graphs"] == 0
    assert min(rep["adi_graph_cap"], rep["varlen_schedule_cap"], rep["varlen_graph_cap"]) > 0
    assert lib.trid_cache_report(h, buf, 8) == 1  # too small
    assert lib.trid_cache_report(h, None, 64) == 1
    assert lib.trid_cache_report(None, buf, len(buf)) == 1


def test_refine_and_adjoint_argument_checks(lib, h):
    d = _dims(8, 8)
    assert lib.trid_gtsv_batched_refine(h, 1, FAKE, FAKE, FAKE, FAKE, FAKE, 2, d, 0, 1) == 1  # x aliases d
    assert lib.trid_gtsv_batched_s_refine(h, 5, FAKE, FAKE, ctypes.c_void_p(0x2000), 2, d, 0, 1) == 1
    assert lib.trid_adi_step_adjoint(h, 1, None, FAKE, 0.2, FAKE, FAKE, 3, _dims(8, 8, 8), 1) == 1  # no u_t
    assert lib.trid_adi_step_adjoint(h, 1, FAKE, FAKE, 0.2, None, FAKE, 3, _dims(8, 8, 8), 1) == 1  # no u_bar
    assert lib.trid_adi_step_adjoint(h, 1, FAKE, FAKE, 0.2, FAKE, FAKE, 1, _dims(8), 1) == 1
    # constant s (s NULL) needs a finite s0
    assert lib.trid_adi_step_adjoint(h, 1, FAKE, None, float("nan"), FAKE, FAKE, 3, _dims(8, 8, 8), 1) == 1
    assert lib.trid_adi_step_adjoint(h, 1, FAKE, None, float("inf"), FAKE, None, 3, _dims(8, 8, 8), 1) == 1
    assert b"s0" in lib.trid_last_error(h)
    assert lib.trid_adi_step_adjoint(h, 7, FAKE, None, 0.2, FAKE, None, 3, _dims(8, 8, 8), 1) == 1  # dtype
    assert lib.trid_adi_step_keep(h, 1, FAKE, FAKE, 3, _dims(8, 8, 8), 1, FAKE, FAKE, None) == 1  # 3D needs w3
    assert lib.trid_adi_step_keep(h, 1, FAKE, None, 3, _dims(8, 8, 8), 1, FAKE, FAKE, FAKE) == 1
    assert lib.trid_adi_step_keep(h, 1, FAKE, FAKE, 1, _dims(8), 1, FAKE, FAKE, None) == 1
    assert lib.trid_adi_step_adjoint_kept(h, 1, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, 3, _dims(8, 8, 8), 1) == 1
    assert lib.trid_plan_load(h, None) == 1
    assert lib.trid_plan_load(h, b"/nonexistent/plans.json") == 1


def test_hv_argument_checks(lib, h):
    d = _dims(8, 4)
    th = 0.5 + 3 ** 0.5 / 6
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, 0.1, th, d, 2, 0, 0) == 0  # no steps: no-op
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, None, 0.1, th, d, 2, 1, 0) == 1
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, -0.1, th, d, 2, 1, 0) == 1
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, float("inf"), th, d, 2, 1, 0) == 1
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, 0.1, 0.0, d, 2, 1, 0) == 1
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, 0.1, float("nan"), d, 2, 1, 0) == 1
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, 0.1, th, d, 2, -1, 0) == 1
    assert lib.trid_hv_step(h, 7, U, FAKE, FAKE, FAKE, 0.1, th, d, 2, 1, 0) == 1
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, 0.1, th, d, 0, 1, 0) == 1  # empty batch
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, 0.1, th, _dims(9000, 4), 1, 1, 0) == 4
    assert lib.trid_hv_step(None, 1, U, FAKE, FAKE, FAKE, 0.1, th, d, 2, 1, 0) == 1
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, 0.1, th, d, 2, 1, 1) == 1  # graph flag: not for HV
    other = ctypes.c_void_p(0x2000)
    assert lib.trid_hv_step(h, 1, FAKE, FAKE, other, other, 0.1, th, d, 2, 1, 0) == 1  # u aliases a
    assert b"alias" in lib.trid_last_error(h)


def test_model_and_report_argument_checks(lib, h):
    us = ctypes.c_double()
    buf = ctypes.create_string_buffer(64)
    assert lib.trid_model_gtsv(h, 1, 1, 3, _dims(64, 64, 64), 2, 1, ctypes.byref(us), buf, len(buf)) == 0
    assert us.value > 0 and buf.value.startswith(b"{")
    assert lib.trid_model_gtsv(h, 1, 1, 3, _dims(64, 64, 64), 2, 1, None, None, 0) == 1  # no output
    assert lib.trid_model_gtsv(h, 1, 5, 3, _dims(64, 64, 64), 2, 1, ctypes.byref(us), None, 0) == 1  # form
    assert lib.trid_model_gtsv(h, 9, 1, 3, _dims(64, 64, 64), 2, 1, ctypes.byref(us), None, 0) == 1  # dtype
    assert lib.trid_model_gtsv(None, 1, 1, 1, _dims(64), 0, 1, ctypes.byref(us), None, 0) == 1
    assert lib.trid_autotune_report(h, buf, len(buf)) == 0 and buf.value == b"[]"
    assert lib.trid_autotune_report(h, buf, 2) == 1  # too small for "[]"
    assert lib.trid_autotune_report(h, None, 64) == 1


def test_noalloc_step_argument_checks(lib, h):
    """Checked on the host before any HIP call: the graph flag (a graph would
    allocate) and meshes whose d exceeds the static scratch (64 MiB)."""
    assert lib.trid_adi_step_noalloc(h, 1, FAKE, None, 0.2, 3, _dims(8, 8, 8), 1, 1, 1) == 1  # graph flag
    assert lib.trid_adi_step_noalloc(h, 1, None, None, 0.2, 3, _dims(8, 8, 8), 1, 1, 0) == 1
    assert lib.trid_adi_step_noalloc(h, 1, FAKE, None, 0.2, 1, _dims(8), 1, 1, 0) == 1
    assert lib.trid_adi_step_noalloc(h, 1, FAKE, None, 0.2, 3, _dims(8, 8, 8), 1, 0, 0) == 0  # no steps
    assert lib.trid_adi_step_noalloc(h, 1, FAKE, None, 0.2, 3, _dims(256, 256, 129), 1, 1, 0) == 4
    assert b"scratch" in lib.trid_last_error(h)
    assert lib.trid_adi_step_noalloc(h, 0, FAKE, None, 0.2, 3, _dims(256, 256, 257), 1, 1, 0) == 4  # FP32
    assert lib.trid_adi_step_noalloc(None, 1, FAKE, None, 0.2, 3, _dims(8, 8, 8), 1, 1, 0) == 1


def test_forced_allocation_failure(lib, h, monkeypatch):
    """TRID_FAIL_ALLOC makes every workspace allocation fail before any HIP call."""
    monkeypatch.setenv("TRID_FAIL_ALLOC", "1")
    assert lib.trid_adi_step(h, 1, FAKE, None, 0.2, 3, _dims(8, 8, 8), 1, 1, 0) == 2
    assert b"TRID_FAIL_ALLOC" in lib.trid_last_error(h)
    # contiguous lines beyond TRID_MAX_LINE need the chunked solve's workspace
    assert lib.trid_gtsv_batched_s(h, 1, FAKE, FAKE, 1, _dims(9000), 0, 1) == 2
    assert lib.trid_hv_step(h, 1, U, FAKE, FAKE, FAKE, 0.1, 0.8, _dims(8, 4), 1, 1, 2) == 2  # per-step path (its workspace)


def test_plan_cache_environment(lib, tmp_path, monkeypatch):
    """TRID_PLAN_CACHE: a new handle loads the file; a handle with plans writes it back."""
    cache = tmp_path / "plans.json"
    cache.write_text('{\n "plans": {\n  "varlen/abc/0": {"M": 16, "NT": 512}\n }\n}\n')
    monkeypatch.setenv("TRID_PLAN_CACHE", str(cache))
    hp = ctypes.c_void_p()
    assert lib.trid_create(ctypes.byref(hp)) == 0
    out = tmp_path / "saved.json"
    assert lib.trid_plan_save(hp, str(out).encode()) == 0
    assert '"varlen/abc/0": {"M": 16, "NT": 512' in out.read_text()
    cache.unlink()
    assert lib.trid_destroy(hp) == 0
    assert '"varlen/abc/0"' in cache.read_text()  # written back on destroy
