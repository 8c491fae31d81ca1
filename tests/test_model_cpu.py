"""The performance model's host entry (no GPU): predictions for the batched
line solves follow the plan the library would launch and respond to the
quantities the model is built from (bytes, tile plan, precision)."""

import pytest

torch = pytest.importorskip("torch")

import paper_2201_03950_amd as trid  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _library():
    import os

    from paper_2201_03950_amd import _binding

    if not os.path.exists(_binding.LIB_PATH):
        from paper_2201_03950_amd import build

        build.build()
    _binding.load_library()


@pytest.fixture(autouse=True)
def _auto_plan(_library):
    trid.set_tile(0, 0)
    yield
    trid.set_tile(0, 0)


def test_prediction_and_plan_fields():
    us, plan = trid.model_gtsv(torch.float64, trid.TRID_FORM_S, [256, 256, 256], 2, 1)
    assert us > 0 and plan["us"] == pytest.approx(us, rel=1e-3)
    for k in ("kernel", "M", "L", "P", "threads", "nblocks", "bytes", "t_bytes_us", "t_lat_us"):
        assert k in plan
    assert plan["bytes"] == 3 * 8 * 256 ** 3  # s, d in, x out
    assert plan["kernel"] == "strided" and plan["P"] * plan["M"] >= 256


def test_prediction_grows_with_the_bytes():
    small, _ = trid.model_gtsv(torch.float64, trid.TRID_FORM_S, [256, 256, 64], 2, 1)
    large, _ = trid.model_gtsv(torch.float64, trid.TRID_FORM_S, [256, 256, 256], 2, 4)
    arrays, _ = trid.model_gtsv(torch.float64, trid.TRID_FORM_ARRAYS, [256, 256, 256], 2, 4)
    f32, _ = trid.model_gtsv(torch.float32, trid.TRID_FORM_S, [256, 256, 256], 2, 4)
    assert small < large < arrays
    assert f32 < large


def test_prediction_follows_the_forced_tile_plan():
    _, auto = trid.model_gtsv(torch.float32, trid.TRID_FORM_S, [1024, 1024], 1, 1)
    trid.set_tile(32, 0)
    _, forced = trid.model_gtsv(torch.float32, trid.TRID_FORM_S, [1024, 1024], 1, 1)
    assert forced["M"] == 32 and forced["M"] != auto["M"]


def test_model_rejects_what_the_solver_rejects():
    with pytest.raises(trid.TridError):
        trid.model_gtsv(torch.float64, 7, [256], 0, 1)
    with pytest.raises(trid.TridError):
        trid.model_gtsv(torch.float64, trid.TRID_FORM_S, [9000], 0, 1)  # beyond one workgroup's line
    with pytest.raises(trid.TridError):
        trid.model_gtsv(torch.float64, trid.TRID_FORM_S, [64, 64], 2, 1)  # no such axis


def test_autotune_report_is_empty_before_tuning():
    import threading

    out = {}
    th = threading.Thread(target=lambda: out.update(rep=trid.autotune_report()))  # a fresh handle
    th.start()
    th.join()
    assert out["rep"] == []


def _cpp_params(struct_fn):
    """The constants of lines_params() / varlen_params() as written in perf_model.cpp."""
    import os
    import re

    src = open(os.path.join(os.path.dirname(trid.__file__), "csrc", "perf_model.cpp")).read()
    body = src[src.index(struct_fn):]
    body = body[:body.index("};")]
    return [float(v) for v in re.findall(r"/\*\w+\*/\s*([-0-9.eE]+)", body)]


def test_calibration_mirror_matches_the_library():
    """The refit script's mirror of the line model reproduces the library's predictions
    with the library's constants (so a refit's constants mean the same thing)."""
    from paper_2201_03950_amd import model_calibrate as mc

    p = _cpp_params("const LinesParams &lines_params()")
    assert len(p) == len(mc.LINE_NAMES)
    cases = [(torch.float64, trid.TRID_FORM_S, [256, 256, 256], 2, 1), (torch.float32, trid.TRID_FORM_ARRAYS,
             [1024], 0, 512), (torch.float64, trid.TRID_FORM_ARRAYS, [64, 2048], 1, 4),
             (torch.float32, trid.TRID_FORM_S, [4096], 0, 64)]
    for dt, form, dims, axis, batch in cases:
        us, plan = trid.model_gtsv(dt, form, dims, axis, batch)
        rec = {"plan": plan, "dtype": str(dt)[6:], "dims": dims, "axis": axis, "form": form}
        assert mc._pred_lines(p, rec) == pytest.approx(us, rel=1e-3)
    assert len(_cpp_params("const VarlenParams &varlen_params()")) == len(mc.VARLEN_NAMES)


def test_calibration_fit_runs_on_a_recorded_sweep(tmp_path, capsys):
    """The refit path of the calibration script on a small synthetic record set
    (measurements = the library's own predictions, so the fit must recover
    accuracy close to 1)."""
    import json

    import numpy as np

    from paper_2201_03950_amd import model_calibrate as mc

    rng = np.random.default_rng(0)
    recs = []
    for dt in (torch.float64, torch.float32):
        for form in (trid.TRID_FORM_S, trid.TRID_FORM_ARRAYS):
            for axis, dims in ((0, [256]), (1, [256, 256]), (2, [64, 64, 128])):
                for batch in (4, 64):
                    us, plan = trid.model_gtsv(dt, form, dims, axis, batch)
                    recs.append({"kind": "lines", "dtype": str(dt)[6:], "form": form, "axis": axis, "n": dims[-1],
                                 "size": batch * int(np.prod(dims)), "dims": dims, "batch": batch, "force_M": 0,
                                 "meas_us": us, "pred_us": us, "plan": plan})
    pv = _cpp_params("const VarlenParams &varlen_params()")
    for mix in mc.CAL_MIXES + ("held_a", "held_b"):
        lens = [int(v) for v in rng.integers(32, 2048, 300)]
        for prec in (0, 1):
            plans = []
            for M, NT in ((8, 1024), (16, 512), (32, 256)):
                q = {"M": M, "NT": NT, "reduced": "pcr", "split": 0, "blocks": 256, "blocks_small": 0}
                q["meas_us"] = mc._pred_varlen(pv, prec, mc._varlen_launches(lens, q))
                plans.append(q)
            recs.append({"kind": "varlen", "mix": mix, "prec": prec, "plans": plans, "lens": lens})
    path = tmp_path / "sweep.jsonl"
    path.write_text("".join(json.dumps(r) + "\n" for r in recs))
    mc.fit(str(path))
    out = capsys.readouterr().out
    assert "LinesParams" in out and "VarlenParams" in out
    accs = [float(x) for x in __import__("re").findall(r"'mean': ([0-9.]+)", out)]
    assert len(accs) == 4 and min(accs) > 0.9


ADI_CASES = [("adi", [256, 256, 256], 1, False, True), ("adi", [128, 128, 128], 2, True, True),
             ("adi", [80, 80, 80], 72, False, True), ("adi", [1024, 1024], 4, True, True),
             ("adi", [64, 64], 3000, False, False), ("adi", [200, 200], 10, False, False),
             ("hv", [100, 50], 3000, False, False), ("hv", [100, 50], 300, False, True),
             ("hv", [300, 200], 4, False, False)]


def _adi_model(dt, kind, dims, batch, pp, stream, steps):
    if kind == "adi":
        return trid.model_adi(dt, dims, batch, pp, steps, stream)
    return trid.model_hv(dt, dims, batch, steps, stream)


def test_adi_calibration_mirror_matches_the_library():
    """The calibration script's mirror of the ADI / HV terms reproduces the
    library's predictions with the library's constants."""
    from paper_2201_03950_amd import model_calibrate as mc

    p = _cpp_params("const AdiParams &adi_params()")
    assert len(p) == len(mc.ADI_NAMES)
    lp = _cpp_params("const LinesParams &lines_params()")
    assert (mc.LINES_T0_US, mc.LINES_BW_GBS) == (lp[0], lp[1])
    for dt in (torch.float64, torch.float32):
        for kind, dims, batch, pp, stream in ADI_CASES:
            us, js = _adi_model(dt, kind, dims, batch, pp, stream, 10)
            assert js["us"] == pytest.approx(us, rel=1e-4)
            rec = {"dtype": str(dt)[6:], "steps": 10, "terms": js["kernels"]}
            assert mc._pred_adi(p, rec) == pytest.approx(us, rel=1e-3)


def test_adi_model_follows_the_call_structure():
    # 3D: the three per-step kernels, launched once per step, under the timer's names
    us1, js1 = trid.model_adi(torch.float64, [256, 256, 256], 1, False, 1)
    us4, js4 = trid.model_adi(torch.float64, [256, 256, 256], 1, False, 4)
    assert [k["name"] for k in js1["kernels"]] == ["adi_stencil_x", "adi_y", "adi_z_update"]
    assert us4 == pytest.approx(4 * us1, rel=1e-6)
    assert all(k["launches"] == 4 for k in js4["kernels"])
    # the stencil + x kernel moves 2 words per point with constant s, 3 with per-point s
    assert js1["kernels"][0]["bytes"] == 2 * 8 * 256 ** 3
    _, jp = trid.model_adi(torch.float64, [256, 256, 256], 1, True, 1)
    assert jp["kernels"][0]["bytes"] == 3 * 8 * 256 ** 3
    # 2D meshes that fit one workgroup's LDS: one resident launch unless forced per step
    _, jr = trid.model_adi(torch.float32, [64, 64], 3000, False, 120)
    _, js = trid.model_adi(torch.float32, [64, 64], 3000, False, 120, stream=True)
    assert [k["name"] for k in jr["kernels"]] == ["adi2d_resident"]
    assert [k["name"] for k in js["kernels"]] == ["adi_stencil_x", "adi_y_update"]
    _, jh = trid.model_hv(torch.float64, [100, 50], 3000, 50, stream=True)
    assert [k["name"] for k in jh["kernels"]] == ["hv_pred", "gtsv_staged", "gtsv_strided"]
    assert [k["launches"] for k in jh["kernels"]] == [200, 100, 100]


def test_adi_model_argument_checks():
    import ctypes

    from paper_2201_03950_amd import _binding as B

    ERR_ARG = 1
    lib = B.load_library()
    h = B.handle()
    dims = (ctypes.c_int64 * 3)(32, 32, 32)
    us = ctypes.c_double()
    buf = ctypes.create_string_buffer(4096)
    ok = lib.trid_model_adi(h, B.TRID_F64, 3, dims, 2, 0, 5, 0, ctypes.byref(us), buf, len(buf))
    assert ok == 0 and us.value > 0
    assert lib.trid_model_adi(h, 7, 3, dims, 2, 0, 5, 0, ctypes.byref(us), buf, len(buf)) == ERR_ARG
    assert lib.trid_model_adi(h, B.TRID_F64, 4, dims, 2, 0, 5, 0, ctypes.byref(us), buf, len(buf)) == ERR_ARG
    assert lib.trid_model_adi(h, B.TRID_F64, 3, dims, 2, 0, -1, 0, ctypes.byref(us), buf, len(buf)) == ERR_ARG
    assert lib.trid_model_adi(h, B.TRID_F64, 3, dims, 2, 0, 5, 1 << 9, ctypes.byref(us), buf,
                              len(buf)) == ERR_ARG
    assert lib.trid_model_adi(h, B.TRID_F64, 3, dims, 2, 0, 5, 0, None, buf, len(buf)) == ERR_ARG
    assert lib.trid_model_adi(h, B.TRID_F64, 3, dims, 2, 0, 5, 0, ctypes.byref(us), buf, 16) == ERR_ARG
    assert lib.trid_model_adi(h, B.TRID_F64, 3, dims, 2, 0, 5, 0, ctypes.byref(us), None, 0) == 0
    d2 = (ctypes.c_int64 * 2)(100, 50)
    assert lib.trid_model_hv(h, B.TRID_F32, d2, 30, 5, 0, ctypes.byref(us), buf, len(buf)) == 0
    assert lib.trid_model_hv(h, B.TRID_F32, d2, 0, 5, 0, ctypes.byref(us), buf, len(buf)) != 0
