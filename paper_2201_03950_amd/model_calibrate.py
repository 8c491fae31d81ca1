"""Calibration of the performance model's constants (csrc/perf_model.cpp).

    python -m paper_2201_03950_amd.model_calibrate sweep OUT.jsonl   # on the GPU
    python -m paper_2201_03950_amd.model_calibrate fit OUT.jsonl     # on any host

``sweep`` measures kernel durations (dispatch-stamped events) of the batched
line solves over both forms (s and coefficient arrays), FP64 and FP32, x/y/z
lines of 32..8192 rows, 2^16..2^24 rows per call, automatic and forced tile
plans, together with each launch's plan (``model_gtsv``); and every plan of the
uneven-batch autotuner on six length mixes (``autotune_report`` with
TRID_AUTOTUNE_TOP=0).  ``fit`` fits the constants by least squares on
log(predicted / measured): the line-solve constants on a seeded random half of
the line configurations, the uneven-batch constants on three of the mixes,
and reports the accuracy (1 - |pred - meas| / meas) on the other half and on
the other three mixes, as the paper does for its own model.  It prints the
constants in the order of LinesParams and VarlenParams.
"""

from __future__ import annotations

import json
import math
import os
import sys

LINE_NAMES = ["t0_us", "bw_gbs", "seg_half", "staged_eff", "xs_eff", "arr_eff", "lat_us", "row_ns", "f64_factor",
              "lvl_ns", "lvl_wave_ns", "issue_row_ns", "issue_lvl_ns"]
VARLEN_NAMES = ["t0_us", "bw_gbs", "lat_us", "cu_gbs", "row_ns", "f64_factor", "lvl_ns", "thomas_ns"]
CAL_MIXES = ("loguni_32_8192_x20000", "uni_32_512_x100000", "bimodal_64_4096_x20000")


def _mixes():
    import numpy as np

    from workloads import gen

    rng = np.random.default_rng(77)
    m = {"loguni_32_8192_x20000": gen.varlen_lengths(20000, 32, 8192, seed=3)[0]}
    m["uni_32_512_x100000"] = rng.integers(32, 513, 100000)
    m["uni_2048_8192_x2000"] = rng.integers(2048, 8193, 2000)
    m["bimodal_64_4096_x20000"] = np.where(rng.random(20000) < 0.9, 64, 4096)
    m["loguni_32_8192_x500"] = gen.varlen_lengths(500, 32, 8192, seed=9)[0]
    m["loguni_16_2048_x50000"] = np.clip(np.rint(np.exp(rng.uniform(np.log(16), np.log(2048), 50000))), 16, 2048)
    return m


def sweep(path):
    import numpy as np
    import torch

    import paper_2201_03950_amd as trid

    trid.load_library()
    out = open(path, "w")

    def geom(axis, n, size):
        if axis == 0:
            return [n], size // n
        if axis == 1:
            w = min(256, max(1, size // n))
            return [w, n], max(1, size // (w * n))
        return ([64, 64, n], size // (4096 * n)) if size >= 4096 * n else (None, 0)

    for dt in (torch.float64, torch.float32):
        for form in (trid.TRID_FORM_S, trid.TRID_FORM_ARRAYS):
            for axis in (0, 1, 2):
                for n in (32, 64, 128, 256, 512, 1024, 2048, 4096, 8192):
                    for size in (1 << 16, 1 << 20, 1 << 24):
                        dims, batch = geom(axis, n, size)
                        if dims is None or batch < 1:
                            continue
                        shape = [batch] + list(reversed(dims))
                        d = torch.randn(shape, dtype=dt, device="cuda")
                        if form == trid.TRID_FORM_S:
                            s = 0.1 + 0.2 * torch.rand(shape, dtype=dt, device="cuda")
                            call = lambda: trid.gtsv_s(s, d, axis)  # noqa: E731
                        else:
                            a = torch.rand(shape, dtype=dt, device="cuda") - 0.5
                            c = torch.rand(shape, dtype=dt, device="cuda") - 0.5
                            b = a.abs() + c.abs() + 1.0
                            call = lambda: trid.gtsv(a, b, c, d, axis)  # noqa: E731
                        for M in (0, 8, 16, 32):
                            trid.set_tile(M, 0)
                            try:
                                pred, plan = trid.model_gtsv(dt, form, dims, axis, batch)
                            except trid.TridError:
                                continue
                            trid.timing_enable(True)  # warm up with timing on, then restart
                            call()
                            torch.cuda.synchronize()
                            trid.timing_enable(True)
                            for _ in range(3 if size >= (1 << 24) else 10):
                                call()
                            (k, ms), = trid.timing_read().values()
                            trid.timing_enable(False)
                            out.write(json.dumps({"kind": "lines", "dtype": str(dt)[6:], "form": form, "axis": axis,
                                                  "n": n, "size": size, "dims": dims, "batch": batch, "force_M": M,
                                                  "meas_us": ms / k * 1e3, "pred_us": pred, "plan": plan}) + "\n")
                        trid.set_tile(0, 0)
                        torch.cuda.empty_cache()
            print("lines %s form %d done" % (dt, form), flush=True)
    os.environ["TRID_AUTOTUNE"] = "1"
    os.environ["TRID_AUTOTUNE_TOP"] = "0"
    for name, lens in _mixes().items():
        lens = np.asarray(lens, dtype=np.int64)
        off = np.zeros(len(lens) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        rows = int(off[-1])
        for prec in (0, 1, 2):
            cd = torch.float64 if prec == 0 else torch.float32
            a = torch.rand(rows, dtype=cd, device="cuda") - 0.5
            c = torch.rand(rows, dtype=cd, device="cuda") - 0.5
            b = a.abs() + c.abs() + 1.0
            d = torch.randn(rows, dtype=torch.float32 if prec == 1 else torch.float64, device="cuda")
            x = torch.empty_like(d)
            trid.gtsv_varlen(prec, a, b, c, d, x, off)
            torch.cuda.synchronize()
            out.write(json.dumps({"kind": "varlen", "mix": name, "prec": prec, "plans": trid.autotune_report(),
                                  "lens": lens.tolist()}) + "\n")
            del a, b, c, d, x
            torch.cuda.empty_cache()
        print("uneven batch %s done" % name, flush=True)
    out.close()


def _log2c(v):
    n = 0
    while (1 << n) < v:
        n += 1
    return n


def _pred_lines(p, r):
    """Mirror of model_lines (perf_model.cpp) on a recorded plan."""
    t0, bw, sh, se, xe, ae, lat, row, fx, lvl, lvlw, ri, li = p
    pl = r["plan"]
    w = 8 if r["dtype"] == "float64" else 4
    d = r["dims"]
    inner = 1 if r["axis"] == 0 else (d[0] if r["axis"] == 1 else d[0] * d[1])
    if pl["kernel"] == "staged":
        eff = se
    elif inner == 1:
        eff = xe
    else:
        seg = min(pl["L"], inner) * w
        eff = seg / (seg + sh)
    if r["form"] == 0:
        eff *= ae
    tb = pl["bytes"] / (bw * eff * 1e3)
    f = fx if w == 8 else 1.0
    lev = _log2c(pl["P"])
    dpp = pl["kernel"] == "staged" and pl["P"] <= 16
    chain = lat + (pl["M"] * row * f + lev * (lvl + (0.0 if dpp else lvlw * pl["threads"] / 256.0))) * 1e-3
    issue = pl["nblocks"] * math.ceil(pl["threads"] / 64.0) / 1024.0 * (pl["M"] * ri * f + lev * li) * 1e-3
    return t0 + max(tb, chain, issue)


def _pack(lens, M, NT):
    """Mirror of varlen_pack: (longest system's tiles, rows) per work item."""
    items, used, pmax, rows = [], 0, 0, 0
    for n in sorted(lens, reverse=True):
        P = (n + M - 1) // M
        if used + P > NT:
            items.append((pmax, rows))
            used, pmax, rows = 0, 0, 0
        used += P
        pmax = max(pmax, P)
        rows += n
    items.append((pmax, rows))
    return items


def _varlen_launches(lens, q):
    def feats(items, M, blocks, thomas):
        red = [pm if thomas else _log2c(pm) for pm, _ in items]
        return {"n": len(items), "rows": sum(r for _, r in items), "red": sum(red), "M": M, "thomas": thomas,
                "b": max(1, min(blocks, len(items))), "rmax": max(r for _, r in items), "redmax": max(red)}

    thomas = q["reduced"] == "thomas"
    if not q["split"]:
        return [feats(_pack(lens, q["M"], q["NT"]), q["M"], q["blocks"], thomas)]
    cap = 8 * 256
    lng = [n for n in lens if n > cap]
    shr = [n for n in lens if n <= cap]
    out = []
    if lng:
        out.append(feats(_pack(lng, q["M"], q["NT"]), q["M"], q["blocks"], thomas))
    if shr:
        out.append(feats(_pack(shr, 8, 256), 8, q["blocks_small"], False))
    return out


def _pred_varlen(p, prec, launches):
    """Mirror of model_varlen (perf_model.cpp), summed over a plan's launches."""
    t0, bw, lat, cub, row, fx, lvl, th = p
    bpr = {0: 40.0, 1: 20.0, 2: 28.0}[prec]
    f = 1.0 if prec == 1 else fx
    tot = 0.0
    for L in launches:
        rc = th if L["thomas"] else lvl
        s = L["n"] * lat + L["rows"] * bpr / (cub * 1e3) + (L["n"] * L["M"] * row * f + L["red"] * rc) * 1e-3
        mx = lat + L["rmax"] * bpr / (cub * 1e3) + (L["M"] * row * f + L["redmax"] * rc) * 1e-3
        tot += t0 + max(L["rows"] * bpr / (bw * 1e3), s / L["b"], mx)
    return tot


def _accuracy(pairs):
    import numpy as np

    e = np.array([abs(p - m) / m for p, m in pairs])
    return {"n": int(len(e)), "mean": round(1 - float(e.mean()), 3), "within_15pct": round(float((e <= 0.15).mean()), 3),
            "within_25pct": round(float((e <= 0.25).mean()), 3)}


def fit(path):
    import numpy as np
    from scipy.optimize import least_squares

    recs = [json.loads(line) for line in open(path)]
    lines = [r for r in recs if r["kind"] == "lines"]
    keys = sorted({(r["dtype"], r["form"], r["axis"], r["n"], r["size"]) for r in lines})
    rng = np.random.default_rng(2026)
    cal_keys = {k for k in keys if rng.random() < 0.5}
    key = lambda r: (r["dtype"], r["form"], r["axis"], r["n"], r["size"])  # noqa: E731
    cal = [r for r in lines if key(r) in cal_keys]
    val = [r for r in lines if key(r) not in cal_keys]
    p0 = [2.5, 7000, 16, 0.9, 0.3, 0.75, 3.0, 100, 1.5, 100, 50, 50, 50]
    lb = [0, 1000, 0, 0.05, 0.02, 0.1, 0, 0, 1, 0, 0, 0, 0]
    ub = [20, 8000, 4096, 1.0, 1.0, 1.0, 50, 5000, 4, 5000, 5000, 5000, 5000]
    f = least_squares(lambda p: np.array([math.log(_pred_lines(p, r) / r["meas_us"]) for r in cal]), p0,
                      bounds=(lb, ub))
    pl = f.x
    print("LinesParams", {k: round(float(v), 4) for k, v in zip(LINE_NAMES, pl)})
    print("  calibration", _accuracy([(_pred_lines(pl, r), r["meas_us"]) for r in cal]))
    print("  validation ", _accuracy([(_pred_lines(pl, r), r["meas_us"]) for r in val]))

    var = [(r, q, _varlen_launches(r["lens"], q)) for r in recs if r["kind"] == "varlen" for q in r["plans"]]
    vcal = [x for x in var if x[0]["mix"] in CAL_MIXES]
    vval = [x for x in var if x[0]["mix"] not in CAL_MIXES]
    lb = [0, 500, 0, 0.5, 0, 1, 0, 0]
    ub = [50, 8000, 100, 2000, 5000, 6, 20000, 20000]
    best = None
    for _ in range(30):  # multi-start: the max() terms make the fit multimodal
        q0 = [rng.uniform(1, 20), rng.uniform(1000, 7000), rng.uniform(0, 30), rng.uniform(5, 500),
              rng.uniform(10, 500), rng.uniform(1, 4), rng.uniform(10, 3000), rng.uniform(10, 500)]
        f = least_squares(lambda p: np.array([math.log(_pred_varlen(p, x[0]["prec"], x[2]) / x[1]["meas_us"])
                                              for x in vcal]), q0, bounds=(lb, ub))
        if best is None or f.cost < best.cost:
            best = f
    pv = best.x
    print("VarlenParams", {k: round(float(v), 4) for k, v in zip(VARLEN_NAMES, pv)})
    print("  calibration", _accuracy([(_pred_varlen(pv, x[0]["prec"], x[2]), x[1]["meas_us"]) for x in vcal]))
    print("  validation ", _accuracy([(_pred_varlen(pv, x[0]["prec"], x[2]), x[1]["meas_us"]) for x in vval]))


if __name__ == "__main__":
    if len(sys.argv) != 3 or sys.argv[1] not in ("sweep", "fit"):
        sys.exit(__doc__)
    sweep(sys.argv[2]) if sys.argv[1] == "sweep" else fit(sys.argv[2])
