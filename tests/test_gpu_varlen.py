"""GPU parity of the uneven-batch persistent solver against the oracle.

Per-system relative infinity-norm error, max over systems: FP64 <= 1e-12; FP32
<= 1e-5; FP32 + FP64 refinement <= 1e-9 (and <= 1e-5, the stated bound).
"""

import os

import numpy as np
import pytest

from workloads import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def trid():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_03950_amd as trid

    trid.load_library()
    return trid


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _sys_err(x, ref, off):
    num = np.maximum.reduceat(np.abs(x - ref), off[:-1])
    den = np.maximum.reduceat(np.abs(ref), off[:-1])
    return float(np.max(num / np.maximum(den, 1e-300)))


def _run(trid, prec, a32, b32, c32, d64):
    if prec == trid.PREC_F64:
        a, b, c, d = (_t(v.astype(np.float64)) for v in (a32, b32, c32, d64))
        x = torch.empty_like(d)
    elif prec == trid.PREC_F32:
        a, b, c, d = (_t(v.astype(np.float32)) for v in (a32, b32, c32, d64))
        x = torch.empty_like(d)
    else:
        a, b, c, d = _t(a32), _t(b32), _t(c32), _t(d64)
        x = torch.empty_like(d)
    return a, b, c, d, x


CASES = [(300, 1, 300), (200, 32, 8192), (2000, 32, 1024), (5, 8000, 8192)]


@pytest.mark.parametrize("prec", ["f64", "f32", "refine"])
@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_varlen_matches_oracle(trid, orc, prec, case):
    nsys, lmin, lmax = case
    a32, b32, c32, d64, off = gen.varlen_batch(nsys, lmin, lmax, seed=nsys + lmin)
    p = {"f64": trid.PREC_F64, "f32": trid.PREC_F32, "refine": trid.PREC_F32_REFINE64}[prec]
    d_in = d64.astype(np.float32).astype(np.float64) if prec == "f32" else d64
    ref = orc.gtsv_varlen(a32, b32, c32, d_in, off)
    a, b, c, d, x = _run(trid, p, a32, b32, c32, d64)
    trid.gtsv_varlen(p, a, b, c, d, x, off)
    err = _sys_err(x.cpu().numpy().astype(np.float64), ref, off)
    tol = {"f64": 1e-12, "f32": 1e-5, "refine": 1e-9}[prec]
    assert err <= tol, err
    # a second call replays the captured launch; the work counter must have reset
    x2 = torch.zeros_like(x)
    trid.gtsv_varlen(p, a, b, c, d, x2, off)
    x3 = torch.zeros_like(x)
    trid.gtsv_varlen(p, a, b, c, d, x3, off)
    assert torch.equal(x2, x3) and torch.equal(x, x2)


def test_varlen_20000_systems_refine_full(trid, orc):
    """The uneven workload at full size: 20,000 systems, lengths log-uniform in [32, 8192]."""
    a32, b32, c32, d64, off = gen.varlen_batch()
    ref = orc.gtsv_varlen(a32, b32, c32, d64, off)
    a, b, c, d, x = _run(trid, trid.PREC_F32_REFINE64, a32, b32, c32, d64)
    trid.gtsv_varlen(trid.PREC_F32_REFINE64, a, b, c, d, x, off)
    err = _sys_err(x.cpu().numpy(), ref, off)
    assert err <= 1e-9, err


def test_varlen_in_place_f64(trid, orc):
    a32, b32, c32, d64, off = gen.varlen_batch(100, 1, 500, seed=9)
    ref = orc.gtsv_varlen(a32, b32, c32, d64, off)
    a, b, c, d, _ = _run(trid, trid.PREC_F64, a32, b32, c32, d64)
    trid.gtsv_varlen(trid.PREC_F64, a, b, c, d, d, off)
    assert _sys_err(d.cpu().numpy(), ref, off) <= 1e-12


def test_varlen_autotune_and_plan_cache(trid, orc, tmp_path, monkeypatch):
    a32, b32, c32, d64, off = gen.varlen_batch(3000, 32, 2048, seed=77)
    ref = orc.gtsv_varlen(a32, b32, c32, d64, off)
    monkeypatch.setenv("TRID_AUTOTUNE", "1")
    a, b, c, d, x = _run(trid, trid.PREC_F32_REFINE64, a32, b32, c32, d64)
    trid.gtsv_varlen(trid.PREC_F32_REFINE64, a, b, c, d, x, off)
    assert _sys_err(x.cpu().numpy(), ref, off) <= 1e-9
    path = tmp_path / "plans.json"
    trid.plan_save(str(path))
    text = path.read_text()
    assert '"arch"' in text and "varlen/p2/n3000" in text
    trid.plan_load(str(path))
    with pytest.raises(trid.TridError):
        trid.plan_load(str(tmp_path / "missing.json"))


FORCED = {
    # systems above 2048 rows in 1024-thread blocks, the rest in 256-thread blocks (two launches)
    "split": '"%s": {"M": 8, "NT": 1024},\n  "%s/small": {"M": 8, "NT": 256}',
    # reduced systems solved by Thomas on one thread per system (Thomas-Thomas)
    "thomas16": '"%s": {"M": 16, "NT": 512, "reduced": "thomas"}',
    "thomas32": '"%s": {"M": 32, "NT": 256, "reduced": "thomas"}',
    # wavefront-level items: 8-row FP64 tiles, 16 wavefronts per workgroup
    "wave8": '"%s": {"M": 8, "NT": 1024, "reduced": "wave"}',
    "wave16": '"%s": {"M": 16, "NT": 512, "reduced": "wave"}',
}


@pytest.mark.parametrize("prec,plan", [("f64", "split"), ("f32", "split"), ("refine", "split"),
                                       ("f64", "thomas16"), ("f64", "thomas32"), ("f32", "thomas16"),
                                       ("f32", "thomas32"), ("f64", "wave8"), ("f64", "wave16"),
                                       ("f32", "wave16"), ("refine", "wave16")])
def test_varlen_forced_plan_matches_oracle(trid, orc, tmp_path, monkeypatch, prec, plan):
    """A plan forced through the plan cache of a fresh handle."""
    import json
    import threading

    a32, b32, c32, d64, off = gen.varlen_batch(1500, 32, 8192, seed=41)
    p = {"f64": trid.PREC_F64, "f32": trid.PREC_F32, "refine": trid.PREC_F32_REFINE64}[prec]
    d_in = d64.astype(np.float32).astype(np.float64) if prec == "f32" else d64
    ref = orc.gtsv_varlen(a32, b32, c32, d_in, off)
    a, b, c, d, x = _run(trid, p, a32, b32, c32, d64)
    monkeypatch.setenv("TRID_AUTOTUNE", "1")
    trid.gtsv_varlen(p, a, b, c, d, x, off)  # autotuned on this thread's handle: learn the plan key
    monkeypatch.delenv("TRID_AUTOTUNE")
    saved = tmp_path / "tuned.json"
    trid.plan_save(str(saved))
    key = next(k for k in json.loads(saved.read_text())["plans"] if k.startswith("varlen/") and "/small" not in k)
    forced = tmp_path / "forced.json"
    entry = FORCED[plan] % ((key, key) if plan == "split" else key)
    forced.write_text('{\n "plans": {\n  %s\n }\n}\n' % entry)
    out = {}

    def worker():  # a new thread gets a new library handle (empty schedule cache)
        try:
            trid.plan_load(str(forced))
            xs = [torch.zeros_like(x) for _ in range(2)]
            for xi in xs:
                trid.gtsv_varlen(p, a, b, c, d, xi, off)
            torch.cuda.synchronize()
            out["x"] = xs
        except Exception as e:  # re-raised on the test thread
            out["err"] = e

    th = threading.Thread(target=worker)
    th.start()
    th.join()
    if "err" in out:
        raise out["err"]
    x1, x2 = out["x"]
    tol = {"f64": 1e-12, "f32": 1e-5, "refine": 1e-9}[prec]
    assert _sys_err(x1.cpu().numpy().astype(np.float64), ref, off) <= tol
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("top", [0, 2])
def test_varlen_autotune_pruned_by_the_model(trid, orc, monkeypatch, top):
    """TRID_AUTOTUNE_TOP=k times only the model's best k plans (0: all); the
    report lists every plan best-predicted first, and the chosen plan solves."""
    a32, b32, c32, d64, off = gen.varlen_batch(2500 + top, 32, 4096, seed=90 + top)  # a fresh schedule key
    ref = orc.gtsv_varlen(a32, b32, c32, d64.astype(np.float64), off)
    monkeypatch.setenv("TRID_AUTOTUNE", "1")
    monkeypatch.setenv("TRID_AUTOTUNE_TOP", str(top))
    a, b, c, d, x = _run(trid, trid.PREC_F64, a32, b32, c32, d64)
    trid.gtsv_varlen(trid.PREC_F64, a, b, c, d, x, off)
    rep = trid.autotune_report()
    preds = [q["pred_us"] for q in rep]
    assert len(rep) >= 2 and preds == sorted(preds) and all(p > 0 for p in preds)
    timed = [q for q in rep if q["meas_us"] >= 0]
    assert len(timed) == (len(rep) if top == 0 else min(top, len(rep)))
    assert timed == rep[:len(timed)]
    assert _sys_err(x.cpu().numpy(), ref, off) <= 1e-12
    # the calibration script's mirror of the wavefront-plan model (its packing
    # included) reproduces the library's predictions with the library's constants
    import re

    from paper_2201_03950_amd import model_calibrate as mc

    src = open(os.path.join(os.path.dirname(trid.__file__), "csrc", "perf_model.cpp")).read()
    body = src[src.index("const VarlenWaveParams &varlen_wave_params()"):]
    pw = [float(v) for v in re.findall(r"/\*\w+\*/\s*([-0-9.eE]+)", body[:body.index("};")])]
    assert len(pw) == len(mc.VARLEN_WAVE_NAMES)
    lens = np.diff(off)
    waves = [q for q in rep if q["reduced"] == "wave"]
    assert waves
    for q in waves:
        st = mc._wave_stats(lens, q["M"], mc._wave_nw(0, q["M"]))
        assert mc._pred_varlen_wave(pw, 0, st, q["M"], q["blocks"]) == pytest.approx(q["pred_us"], rel=1e-3)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_varlen_autotune_in_place(trid, orc, monkeypatch, prec):
    """With autotuning, the candidate timings must not run on an in-place call's
    own output: x = d still returns A^{-1} d."""
    a32, b32, c32, d64, off = gen.varlen_batch(1200, 32, 4096, seed=131 if prec == "f64" else 132)
    p = trid.PREC_F64 if prec == "f64" else trid.PREC_F32
    d_in = d64.astype(np.float32).astype(np.float64) if prec == "f32" else d64
    ref = orc.gtsv_varlen(a32, b32, c32, d_in, off)
    a, b, c, d, _ = _run(trid, p, a32, b32, c32, d64)
    monkeypatch.setenv("TRID_AUTOTUNE", "1")
    monkeypatch.setenv("TRID_AUTOTUNE_TOP", "3")
    trid.gtsv_varlen(p, a, b, c, d, d, off)
    assert any(q["meas_us"] >= 0 for q in trid.autotune_report())  # the call did tune
    tol = 1e-12 if prec == "f64" else 1e-5
    assert _sys_err(d.cpu().numpy().astype(np.float64), ref, off) <= tol


@pytest.mark.parametrize("prec", ["f64", "refine"])
def test_varlen_device_offsets(trid, orc, prec):
    """Offsets in device memory give the same result as the host offsets (same schedule)."""
    a32, b32, c32, d64, off = gen.varlen_batch(700, 1, 3000, seed=133)
    p = trid.PREC_F64 if prec == "f64" else trid.PREC_F32_REFINE64
    ref = orc.gtsv_varlen(a32, b32, c32, d64, off)
    a, b, c, d, x = _run(trid, p, a32, b32, c32, d64)
    trid.gtsv_varlen(p, a, b, c, d, x, off)
    x2 = torch.zeros_like(x)
    trid.gtsv_varlen_dev(p, a, b, c, d, x2, _t(off))
    assert torch.equal(x, x2)
    assert _sys_err(x2.cpu().numpy(), ref, off) <= (1e-12 if prec == "f64" else 1e-9)


def test_varlen_two_streams_share_one_schedule(trid, orc):
    """Calls of one handle on two streams share the schedule's work counter; the
    stream switch orders them, so both solves are complete."""
    a32, b32, c32, d64, off = gen.varlen_batch(4000, 32, 8192, seed=134)
    ref = orc.gtsv_varlen(a32, b32, c32, d64, off)
    a, b, c, d, x = _run(trid, trid.PREC_F64, a32, b32, c32, d64)
    xs = [torch.zeros_like(x) for _ in range(4)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for k, xk in enumerate(xs):
        with torch.cuda.stream(streams[k % 2]):
            trid.gtsv_varlen(trid.PREC_F64, a, b, c, d, xk, off)
    torch.cuda.synchronize()
    for xk in xs:
        assert _sys_err(xk.cpu().numpy(), ref, off) <= 1e-12
