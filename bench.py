#!/usr/bin/env python3
"""Benchmark of the batched tridiagonal line solves on one MI355X.

One step = one ADI heat-diffusion step (Alg. 3 of arxiv 2201.03950) on a
256 x 256 x 256 FP64 mesh with s = 0.2: the fused stencil + x-line solve, the
y-line solve and the fused z-line solve + update (3 x 65,536 tridiagonal
solves of length 256).  Inputs are seeded synthetic fields already resident in
HBM.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extra] [--no-cpu]

value        tridiagonal solves per second over the K timed steps
roofline     the dominant kernel's algorithmic bytes / its mean duration (HIP
             events recorded by the library on the launch stream during the
             timed steps) against the 8 TB/s HBM peak
cpu_baseline the CPU oracle (plain C, OpenMP over lines) on a bounded sample
extra        the other workloads: 1024 x 256 systems (x and y layouts, and a
             262,144-system bandwidth variant), the FP32 ADI step, the 2D
             64 x 1024^2 x-then-y solves, uneven batches and gradients
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "tridiag solves/s + HBM GB/s (% peak); 256^3 ADI step ms; fwd+bwd/fwd ratio"
PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_adi3d_256_f64.json")


# Algorithmic words moved per row (each array read once / written once):
# coefficient arrays a, b, c, d in and x out = 5; per-point s: s, d, x = 3;
# constant rows: d in, x out = 2.
ALG_WORDS = {"arrays": 5, "s": 3, "const": 2}


def alg_bytes(mode, word_bytes, rows):
    """Bytes a batched solve must move: the bandwidth convention of the paper's Table 1."""
    return ALG_WORDS[mode] * word_bytes * rows


# Sources the three kernels of the ADI step are built from (the constant-row
# solves, their staging and epilogues, the tile sweep).  A stored counter
# measurement stays valid while none of these change.
TIMED_EVERY = 4  # the timed steps stamp the kernels of every 4th step
ADI_KERNEL_SOURCES = ("tile.hpp", "lines.hpp", "const_lines.hpp", "k_const.hip", "dispatch.hpp")


def kernel_source_hash():
    """Hash of the ADI step's kernel sources; a stored counter measurement is valid only for this hash."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2201_03950_amd", "csrc")
    for name in ADI_KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None if stale."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else float(k["hbm_bytes_per_launch"])


def log(msg):
    """Progress line on stderr (stdout carries only the JSON result)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def sync():
    import torch

    torch.cuda.synchronize()


def time_calls(fn, reps, warm=2):
    """Mean wall seconds per call of fn() over `reps` calls (synchronised)."""
    for _ in range(warm):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    sync()
    return (time.perf_counter() - t0) / reps


def timed_calls(trid, fn, reps, warm=2):
    """(mean wall seconds per call, per-kernel timings) of `reps` calls of fn()
    with the library's kernel timer on; the `warm` calls before them run with
    the timer off (the first launches after an allocation or a free can take
    several times the steady-state time)."""
    for _ in range(warm):
        fn()
    sync()
    trid.timing_enable(True)
    t = time_calls(fn, reps, warm=0)
    kt = trid.timing_read()
    trid.timing_enable(False)
    return t, kt


def adi_main(trid, steps, warmup):
    import torch

    from workloads import gen

    dims = (256, 256, 256)
    pts = dims[0] * dims[1] * dims[2]
    u = torch.from_numpy(gen.adi3d_field(dims, seed=1)).cuda()
    for _ in range(warmup):
        trid.adi_step(u, s0=0.2, nsteps=1)
    sync()
    # the timed steps stamp the kernels of every TIMED_EVERY-th step with HIP
    # events from their dispatch (events on every launch cost about 15 us per
    # step); one more warm-up step on that launch path, then the accumulators
    # restart
    trid.timing_select(None, TIMED_EVERY)
    trid.timing_enable(True)
    trid.adi_step(u, s0=0.2, nsteps=1)
    sync()
    trid.timing_select(None, TIMED_EVERY)
    t0 = time.perf_counter()
    for _ in range(steps):
        trid.adi_step(u, s0=0.2, nsteps=1)
    sync()
    elapsed = time.perf_counter() - t0
    kt = trid.timing_read()
    trid.timing_enable(False)
    trid.timing_select(None)
    # same steps replayed as one captured graph per step (production path)
    for _ in range(2):
        trid.adi_step(u, s0=0.2, nsteps=1, graph=True)
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        trid.adi_step(u, s0=0.2, nsteps=1, graph=True)
    sync()
    elapsed_graph = time.perf_counter() - t0
    w = 8
    words = {"adi_stencil_x": 2, "adi_y": 2, "adi_z_update": 3}

    def rate(name, cnt, ms):
        avg = ms / cnt
        b = words[name] * w * pts
        return {"mean_ms": round(avg, 5), "launches": cnt, "alg_bytes": b,
                "gbs": round(b / (avg * 1e-3) / 1e9, 1),
                "frac": round(b / (avg * 1e-3) / 1e9 / PEAK_GBS, 4)}

    kernels = {name: rate(name, cnt, ms) for name, (cnt, ms) in kt.items()}
    dom = max(kernels, key=lambda k: kernels[k]["mean_ms"])
    dominant = dict(kernels[dom], kernel=dom)
    # correctness of the timed configuration: a discrete sine mode decays by the
    # closed-form factor G per step (Alg. 3 with rows (-s, 1 + 2 s, -s))
    import math

    modes, s0, nchk = (3, 5, 2), 0.2, 10
    mus = [4.0 * math.sin(math.pi * p / (2.0 * (n + 1))) ** 2 for p, n in zip(modes, dims)]
    g = 1.0 - 2.0 * s0 * sum(mus) / math.prod(1.0 + s0 * m for m in mus)
    uf = torch.from_numpy(gen.fourier_mode_3d(dims, modes)).cuda()
    want = uf * g ** nchk
    for _ in range(nchk):
        trid.adi_step(uf, s0=s0, nsteps=1, graph=True)
    sync()
    fourier_err = float((uf - want).abs().max() / want.abs().max())
    return {"elapsed": elapsed, "elapsed_graph": elapsed_graph, "kernels": kernels, "dominant": dominant,
            "solves_per_step": 3 * dims[1] * dims[2], "pts": pts, "fourier_err_10steps": fourier_err}


def extra_workloads(trid):
    import numpy as np
    import torch

    from workloads import gen

    out = {}
    # -- FP32 256^3 ADI step (right after the FP64 one, on fresh allocations)
    u = torch.from_numpy(gen.adi3d_field((256, 256, 256), seed=1, dtype=np.float32)).cuda()
    for _ in range(5):  # fresh allocations: first touches stay out of the timing
        trid.adi_step(u, s0=0.2, nsteps=1)
    sync()
    t, kt = timed_calls(trid, lambda: trid.adi_step(u, s0=0.2, nsteps=1), 10)
    pts = 256 ** 3
    words = {"adi_stencil_x": 2, "adi_y": 2, "adi_z_update": 3}
    out["adi3d_256_f32"] = {"ms_per_step": round(t * 1e3, 4), "kernels": {
        k: {"mean_ms": round(ms / cnt, 5),
            "frac": round(words[k] * 4 * pts / (ms / cnt * 1e-3) / 1e9 / PEAK_GBS, 4)}
        for k, (cnt, ms) in kt.items()}}
    del u
    # -- 1024 systems of 256 rows, FP64, coefficient arrays (x and y layouts)
    a, b, c, d = gen.dd_lines(1024, 256, seed=0)
    for lay in ("x", "y"):
        arr = [v[None] if lay == "x" else np.ascontiguousarray(v.T)[None] for v in (a, b, c, d)]
        ta, tb, tc, td0 = (torch.from_numpy(v).cuda() for v in arr)
        td = td0.clone()
        axis = 0 if lay == "x" else 1
        t = time_calls(lambda: trid.gtsv(ta, tb, tc, td, axis), 1000, warm=20)
        trid.timing_enable(True)  # the kernel itself (the wall time per call is launch-bound)
        time_calls(lambda: trid.gtsv(ta, tb, tc, td, axis), 200, warm=0)
        (cnt, ms), = trid.timing_read().values()
        trid.timing_enable(False)
        kus = ms / cnt * 1e3
        # the same call captured 100 times in one graph (torch's capture of the
        # library's launches on the current stream), replayed: no launch overhead
        gph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            trid.gtsv(ta, tb, tc, td, axis)  # workspace and plans exist before capture
            with torch.cuda.graph(gph, stream=cap):
                for _ in range(100):
                    trid.gtsv(ta, tb, tc, td, axis)
        torch.cuda.current_stream().wait_stream(cap)
        tg = time_calls(gph.replay, 20, warm=2) / 100
        out["sys1024x256_f64_%s" % lay] = {"us_per_call": round(t * 1e6, 2),
                                          "us_per_call_graph": round(tg * 1e6, 2),
                                          "solves_per_s_graph": round(1024 / tg, 1),
                                          "solves_per_s": round(1024 / t, 1),
                                          "kernel_us": round(kus, 2),
                                          "solves_per_s_kernel": round(1024 / (kus * 1e-6), 1),
                                          "gbs_kernel": round(alg_bytes("arrays", 8, 1024 * 256) / (kus * 1e-6) / 1e9, 1)}
    # -- bandwidth variant: 262,144 systems of 256 rows (2.7 GB moved per call)
    nsys = 262144
    rng_a, rng_b, rng_c, rng_d = gen.dd_lines(nsys, 256, seed=10)
    for lay in ("x", "y"):
        arr = [v[None] if lay == "x" else np.ascontiguousarray(v.T)[None]
               for v in (rng_a, rng_b, rng_c, rng_d)]
        ta, tb, tc, td = (torch.from_numpy(v).cuda() for v in arr)
        del arr
        axis = 0 if lay == "x" else 1
        t, kt = timed_calls(trid, lambda: trid.gtsv(ta, tb, tc, td, axis), 10)
        name, (cnt, ms) = next(iter(kt.items()))
        kern = ms / cnt * 1e-3
        byts = alg_bytes("arrays", 8, nsys * 256)
        log("bandwidth variant %s layout done" % lay)
        out["sys262144x256_f64_%s" % lay] = {
            "ms_per_call": round(t * 1e3, 4), "kernel": name, "kernel_ms": round(kern * 1e3, 4),
            "solves_per_s": round(nsys / kern, 1), "gbs": round(byts / kern / 1e9, 1),
            "frac": round(byts / kern / 1e9 / PEAK_GBS, 4)}
        del ta, tb, tc, td
        torch.cuda.empty_cache()
    for name, fn in EXTRA_LEGS.items():
        log("extra: " + name)
        try:
            out.update(fn(trid))
        except Exception as exc:  # keep the main line even if one extra fails
            out[name + "_error"] = repr(exc)
        torch.cuda.empty_cache()
    return out


def kernel_split(trid, fn, reps=5):
    """Mean kernel microseconds per launch name over `reps` calls of fn (timing on)."""
    trid.timing_enable(True)
    for _ in range(reps):
        fn()
    kt = trid.timing_read()
    trid.timing_enable(False)
    return {k: round(ms / cnt * 1e3, 2) for k, (cnt, ms) in kt.items()}


def _err_vs(ref, x):
    """max |x - ref| / max |ref| (torch tensors, compared in FP64)."""
    ref, x = ref.double(), x.double()
    return float((x - ref).abs().max() / ref.abs().max())


def _apply_rows(s, v, axis):
    """Rows (-s, 1 + 2 s, -s) along mesh axis `axis` (0 = x, the last tensor dim),
    zero outside the line: the operator whose solve is timed, applied to check a
    residual (FP64)."""
    import torch

    dim = v.dim() - 1 - axis
    n = v.shape[dim]
    lo = torch.zeros_like(v)
    hi = torch.zeros_like(v)
    lo.narrow(dim, 1, n - 1).copy_(v.narrow(dim, 0, n - 1))   # v_{i-1}
    hi.narrow(dim, 0, n - 1).copy_(v.narrow(dim, 1, n - 1))   # v_{i+1}
    return (1 + 2 * s) * v - s * (lo + hi)


def extra_2d(trid):
    """64 meshes of 1024^2: x then y solves with per-point s; FP64, FP32, FP32 + FP64 refinement.

    Errors: FP64 by its residual (the x-then-y result v must satisfy X (Y v) = d),
    FP32 and FP32 + refinement against the FP64 result."""
    import torch

    from workloads import gen

    out = {}
    s32, d32 = gen.adi2d_varcoef((1024, 1024), 64, seed=2)
    pts = 64 * 1024 * 1024
    res = {}
    x64 = None
    for tag, dt in (("f64", torch.float64), ("f32", torch.float32)):
        ts = torch.from_numpy(s32).cuda().to(dt)
        d0 = torch.from_numpy(d32).cuda().to(dt)
        td = d0.clone()

        def xy():
            td.copy_(d0)
            trid.gtsv_s(ts, td, 0)
            trid.gtsv_s(ts, td, 1)

        t = time_calls(xy, 5, warm=1)  # td holds the last x-then-y result
        if tag == "f64":
            x64 = td[:2].clone()
            r = _apply_rows(ts[:2], _apply_rows(ts[:2], x64, 1), 0)
            err = {"rel_residual": _err_vs(d0[:2], r)}
        else:
            err = {"err_vs_f64": _err_vs(x64, td[:2])}
        t -= time_calls(lambda: td.copy_(d0), 5, warm=1)  # the reset copy is not solver time
        wb = 8 if dt == torch.float64 else 4
        byts = 2 * alg_bytes("s", wb, pts)
        split = kernel_split(trid, xy)
        res[tag] = {"ms": round(t * 1e3, 4), "gbs": round(byts / t / 1e9, 1),
                    "frac": round(byts / t / 1e9 / PEAK_GBS, 4), **err,
                    "kernel_us": split,
                    "kernel_gbs": {k: round(alg_bytes("s", wb, pts) / (v * 1e-6) / 1e9, 1) for k, v in split.items()}}
        del ts, d0, td
        torch.cuda.empty_cache()
    ts = torch.from_numpy(s32).cuda()
    td = torch.from_numpy(d32).cuda()
    mid = torch.empty(s32.shape, dtype=torch.float64, device="cuda")
    xo = torch.empty_like(mid)

    def xy_ref():
        trid.gtsv_s_refine(ts, td, mid, 0)
        trid.gtsv_s_refine(ts, mid, xo, 1)

    t = time_calls(xy_ref, 5, warm=1)
    byts = (4 + 4 + 8) * pts + (4 + 8 + 8) * pts  # x: s32, d32 -> x64; y: s32, x64 -> out64
    split = kernel_split(trid, xy_ref)
    res["f32_refine64"] = {"ms": round(t * 1e3, 4), "gbs": round(byts / t / 1e9, 1),
                           "frac": round(byts / t / 1e9 / PEAK_GBS, 4),
                           "err_vs_f64": _err_vs(x64, xo[:2]), "kernel_us": split}
    res["refine_time_vs_f64"] = round(res["f32_refine64"]["ms"] / res["f64"]["ms"], 3)
    out["adi2d_64x1024sq_xy"] = res
    return out


def extra_long(trid):
    """64 contiguous lines of 2^20 rows (FP64): the chunked solve for lines longer
    than one workgroup holds.  Coefficient arrays and per-point s; the error is
    the relative residual of the first two lines."""
    import torch

    from workloads import gen

    nl, n = 64, 1 << 20
    a, b, c, d = gen.dd_lines(nl, n, seed=21)
    ta, tb, tc, d0 = (torch.from_numpy(v).cuda() for v in (a, b, c, d))
    del a, b, c, d
    td = d0.clone()
    out = {}
    for mode in ("arrays", "s"):
        def call():
            if mode == "arrays":
                trid.gtsv(ta, tb, tc, td, 0)
            else:
                trid.gtsv_s(tb, td, 0)

        td.copy_(d0)
        call()
        x = td[:2].double()
        if mode == "arrays":
            ax = tb[:2] * x
            ax[:, 1:] += ta[:2, 1:] * x[:, :-1]
            ax[:, :-1] += tc[:2, :-1] * x[:, 1:]
        else:
            ax = _apply_rows(tb[:2], x, 0)
        resid = _err_vs(d0[:2], ax)
        t, kt = timed_calls(trid, call, 10)
        cnt, ms = kt["gtsv_long"]
        kern = ms / cnt * 1e-3
        byts = alg_bytes(mode, 8, nl * n)
        out[mode] = {"ms_per_call": round(t * 1e3, 4), "ms_events": round(kern * 1e3, 4),
                     "rows_per_s": round(nl * n / kern, 1), "gbs_alg": round(byts / kern / 1e9, 1),
                     "frac_alg": round(byts / kern / 1e9 / PEAK_GBS, 4), "rel_residual": resid}
    return {"long_64x1M_f64": out}


# Words per point and time step that the calls of Alg. 3 access (coefficients
# generated, not stored): the right-hand side reads u and writes d, each line
# solve reads and writes d, the update reads u and d and writes u.
ALG3_WORDS = {2: 2 + 2 + 2 + 3, 3: 2 + 2 + 2 + 2 + 3}


def extra_small_batched(trid):
    """Batched small meshes at the 2D and 3D application shapes: 2D meshes of
    32^2..128^2, 1500 and 3000 meshes, 120 steps; 3D meshes of 32^3..96^3, 24 and
    72 meshes, 100 steps; s = 0.2.  2D runs the LDS-resident time loop (one
    launch) and, for comparison, the per-step kernels.  Bandwidths count the mesh
    words every call of Alg. 3 accesses (the convention of the paper's
    application tables), so the resident loop's figure exceeds what HBM moves."""
    import numpy as np
    import torch

    out = {}
    rng = np.random.default_rng(33)
    for dt, tag in ((torch.float32, "f32"), (torch.float64, "f64")):
        w = 4 if dt == torch.float32 else 8
        for n in (32, 48, 64, 80, 96, 112, 128):
            for batch in (1500, 3000):
                steps = 120
                u0 = torch.from_numpy(rng.uniform(0.0, 1.0, (batch, n, n))).to(dt).cuda()
                u = u0.clone()
                res = {}
                for mode in ("resident", "streamed"):
                    stream = mode == "streamed"
                    t, kt = timed_calls(trid, lambda: trid.adi_step(u, s0=0.2, nsteps=steps, stream=stream), 2, warm=1)
                    if mode == "resident" and "adi2d_resident" not in kt:
                        continue  # does not fit one workgroup's LDS
                    pts = batch * n * n * steps
                    r = {"ms": round(t * 1e3, 3), "mpoint_steps_per_s": round(pts / t / 1e6, 1),
                         "alg3_gbs": round(ALG3_WORDS[2] * w * pts / t / 1e9, 1)}
                    if stream:
                        words = {"adi_stencil_x": 2, "adi_y_update": 3}
                        r["kernel_gbs"] = {k: round(words[k] * w * batch * n * n / (ms / cnt * 1e-3) / 1e9, 1)
                                           for k, (cnt, ms) in kt.items() if k in words}
                    res[mode] = r
                if "resident" in res:
                    res["speedup_resident"] = round(res["streamed"]["ms"] / res["resident"]["ms"], 2)
                out["2d_%s_%d^2_x%d" % (tag, n, batch)] = res
                del u0, u
        for n in (32, 48, 64, 80, 96):
            for batch in (24, 72):
                out["3d_%s_%d^3_x%d" % (tag, n, batch)] = small3d_case(trid, dt, n, batch, 100, rng)
        log("small batched meshes %s done" % tag)
    return {"adi_small_batched": out}


def small3d_case(trid, dt, n, batch, steps, rng):
    """One 3D batched-mesh case: graph-replayed time of `steps` steps and the
    per-kernel split of one eager call (bandwidths count each kernel's
    algorithmic words: stencil + x 2, y 2, z + update 3)."""
    import torch

    w = 4 if dt == torch.float32 else 8
    u = torch.from_numpy(rng.uniform(0.0, 1.0, (batch, n, n, n))).to(dt).cuda()
    t = time_calls(lambda: trid.adi_step(u, s0=0.2, nsteps=steps, graph=True), 2, warm=1)
    pts = batch * n ** 3 * steps
    trid.timing_enable(True)  # events cost launch time: a call of its own
    trid.adi_step(u, s0=0.2, nsteps=steps)
    kt = trid.timing_read()
    trid.timing_enable(False)
    words = {"adi_stencil_x": 2, "adi_y": 2, "adi_z_update": 3}
    res = {"ms": round(t * 1e3, 3), "mpoint_steps_per_s": round(pts / t / 1e6, 1),
           "alg3_gbs": round(ALG3_WORDS[3] * w * pts / t / 1e9, 1),
           "kernel_us": {k: round(ms / cnt * 1e3, 2) for k, (cnt, ms) in kt.items() if k in words},
           "kernel_gbs": {k: round(words[k] * w * batch * n ** 3 / (ms / cnt * 1e-3) / 1e9, 1)
                          for k, (cnt, ms) in kt.items() if k in words}}
    del u
    return res


def extra_small3d(n):
    """Leg factory: n^3 meshes x 72 (Table 3's largest 3D batch), FP64 and FP32,
    20 steps, s = 0.2 -- one shape per leg so that a profile of the leg covers it alone."""
    def leg(trid):
        import numpy as np
        import torch

        rng = np.random.default_rng(n)
        return {"adi3d_%dcubed_x72" % n: {tag: small3d_case(trid, dt, n, 72, 20, rng)
                                          for dt, tag in ((torch.float64, "f64"), (torch.float32, "f32"))}}
    return leg


# Mesh words per point and HV step that the stand-in's kernels must move: the
# four predictors read u, r, z and the coefficients they use and write r, z or
# u (6 + 4 + 6 + 4 words); the four s-form solves read d and s and write x
# (3 words each).
HV_WORDS = {"hv_pred": 20, "solves": 12}


def extra_hv(trid):
    """The SLV-like Hundsdorfer-Verwer stand-in (Alg. 4's call structure) at the
    SLV mesh sizes 40 x 20 and 100 x 50 with 30, 300 and 3000 meshes, 50 steps
    per call, FP64 and FP32: the LDS-resident loop (one launch per call) and the
    per-step kernels.  gbs_32w counts HV_WORDS per point and step (what the
    per-step kernels move), so the resident figure exceeds what HBM moves."""
    import math

    import torch

    from workloads import gen

    theta = 0.5 + math.sqrt(3.0) / 6.0
    out = {}
    for dt, tag in ((torch.float64, "f64"), (torch.float32, "f32")):
        w = 8 if dt == torch.float64 else 4
        for nx, ny in ((40, 20), (100, 50)):
            for batch in (30, 300, 3000):
                steps = 50
                u, a, b, c = (torch.from_numpy(v).to(dt).cuda() for v in gen.hv_slv((nx, ny), batch))
                pts = batch * nx * ny
                words = HV_WORDS["hv_pred"] + HV_WORDS["solves"]
                res = {}
                for mode in ("resident", "streamed"):
                    stream = mode == "streamed"
                    t = time_calls(lambda: trid.hv_step(u, a, b, c, 0.25, theta, steps, stream=stream), 2, warm=1)
                    trid.timing_enable(True)  # kernel times from a call of its own (events cost launch time)
                    trid.hv_step(u, a, b, c, 0.25, theta, steps, stream=stream)
                    kt = trid.timing_read()
                    trid.timing_enable(False)
                    res[mode] = {"ms_per_step": round(t / steps * 1e3, 4),
                                 "mpoint_steps_per_s": round(pts * steps / t / 1e6, 1),
                                 "gbs_32w": round(words * w * pts * steps / t / 1e9, 1),
                                 "kernel_ms_per_step": {k: round(ms / steps, 4) for k, (cnt, ms) in kt.items()}}
                if "hv_resident" in res["resident"]["kernel_ms_per_step"]:
                    res["speedup_resident"] = round(res["streamed"]["ms_per_step"] / res["resident"]["ms_per_step"], 2)
                else:
                    del res["resident"]  # does not fit one workgroup's LDS
                out["%s_%dx%d_x%d" % (tag, nx, ny, batch)] = res
                del u, a, b, c
        log("hv stand-in %s done" % tag)
    return {"hv_slv": out}


def extra_perf_model(trid):
    """Validation of the performance model on configurations outside its
    calibration sweep: line lengths that are not powers of two (96 .. 3072),
    both forms, x/y/z lines, FP64 and FP32, 2^20 and 2^23 rows per call, the
    library's own tile plans; and three uneven-batch length mixes that were not
    fitted, every plan timed.  Accuracy = 1 - |predicted - measured| / measured
    (the paper's measure for its model), and for the autotuner the measured time
    of the best of the model's top 3 plans over the best plan's."""
    import numpy as np
    import torch

    from paper_2201_03950_amd.model_calibrate import kernel_median_us
    from workloads import gen

    errs, worst = [], []
    for dt in (torch.float64, torch.float32):
        for form in (trid.TRID_FORM_S, trid.TRID_FORM_ARRAYS):
            for axis in (0, 1, 2):
                for n in (96, 192, 384, 768, 1536, 3072):
                    for size in (1 << 20, 1 << 23):
                        if axis == 0:
                            dims = [n]
                        elif axis == 1:
                            dims = [256, n]
                        else:
                            dims = [64, 64, n]
                        batch = size // int(np.prod(dims))
                        if batch < 1:
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
                        pred, _ = trid.model_gtsv(dt, form, dims, axis, batch)
                        # steady-state kernel time: the median of individually timed calls
                        # after warm-up calls (the first launches on freshly allocated
                        # arrays can take several times as long)
                        meas = kernel_median_us(trid, call)
                        e = abs(pred - meas) / meas
                        errs.append(e)
                        worst.append((e, "%s form%d axis%d n%d rows%d pred %.1f meas %.1f" % (
                            str(dt)[6:], form, axis, n, size, pred, meas)))
                        del d
        torch.cuda.empty_cache()
    errs = np.array(errs)
    worst.sort(reverse=True)
    res = {"lines": {"configs": int(len(errs)), "mean_accuracy": round(1 - float(errs.mean()), 3),
                     "median_accuracy": round(1 - float(np.median(errs)), 3),
                     "within_15pct": round(float((errs <= 0.15).mean()), 3),
                     "within_25pct": round(float((errs <= 0.25).mean()), 3),
                     "worst": [w for _, w in worst[:5]]}}
    log("model validation: line solves done")
    # uneven batches outside the fit: every plan timed (TRID_AUTOTUNE_TOP=0)
    os.environ["TRID_AUTOTUNE"] = "1"
    os.environ["TRID_AUTOTUNE_TOP"] = "0"
    rng = np.random.default_rng(77)
    rng.integers(32, 513, 100000)  # the calibration mixes' draws come first in this stream
    mixes = {"uni_2048_8192_x2000": rng.integers(2048, 8193, 2000),
             "loguni_32_8192_x500": gen.varlen_lengths(500, 32, 8192, seed=9)[0],
             "loguni_16_2048_x50000": None}
    rng.random(20000)
    mixes["loguni_16_2048_x50000"] = np.clip(np.rint(np.exp(rng.uniform(np.log(16), np.log(2048), 50000))), 16,
                                             2048)
    verrs, prune = [], {}
    for name, lens in mixes.items():
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
            sync()
            rep = trid.autotune_report()
            for q in rep:
                verrs.append(abs(q["pred_us"] - q["meas_us"]) / q["meas_us"])
            best = min(q["meas_us"] for q in rep)
            prune["%s_prec%d" % (name, prec)] = round(min(q["meas_us"] for q in rep[:3]) / best, 3)
            del a, b, c, d, x
            torch.cuda.empty_cache()
    os.environ.pop("TRID_AUTOTUNE_TOP")
    os.environ.pop("TRID_AUTOTUNE")
    verrs = np.array(verrs)
    res["varlen"] = {"plans": int(len(verrs)), "mean_accuracy": round(1 - float(verrs.mean()), 3),
                     "within_25pct": round(float((verrs <= 0.25).mean()), 3),
                     "top3_best_over_best": prune}
    log("model validation: uneven batches done")
    res["adi"] = adi_model_validation(trid)
    log("model validation: ADI and HV calls done")
    return {"perf_model": res}


# Shapes none of which is in the ADI calibration sweep (model_calibrate.adi_cases).
ADI_HELDOUT = [("adi", [40, 40, 40], 60, False, True), ("adi", [40, 40, 40], 60, True, True),
               ("adi", [56, 56, 56], 30, False, True), ("adi", [72, 72, 72], 16, True, True),
               ("adi", [144, 144, 144], 4, False, True), ("adi", [144, 144, 144], 4, True, True),
               ("adi", [200, 200, 200], 1, False, True), ("adi", [72, 72], 800, True, True),
               ("adi", [200, 200], 150, False, True), ("adi", [400, 400], 40, True, True),
               ("adi", [56, 56], 1000, False, False), ("adi", [72, 72], 2000, False, False),
               ("adi", [88, 88], 1200, False, False), ("hv", [50, 30], 1000, False, False),
               ("hv", [50, 30], 1000, False, True), ("hv", [80, 40], 2000, False, False),
               ("hv", [80, 40], 2000, False, True), ("hv", [120, 60], 500, False, True)]


def adi_model_validation(trid):
    """The performance model's predictions of whole ADI and Hundsdorfer-Verwer
    calls (trid_model_adi / trid_model_hv: all kernels of the call) against the
    measured kernel times, on held-out shapes, FP64 and FP32, 10 steps."""
    import numpy as np
    import torch

    rng = np.random.default_rng(11)
    errs, rows = [], []
    for dt in (torch.float64, torch.float32):
        for kind, dims, batch, pp, stream in ADI_HELDOUT:
            shape = [batch] + list(reversed(dims))
            u = torch.from_numpy(rng.uniform(0.0, 1.0, shape)).to(dt).cuda()
            steps = 10
            if kind == "adi":
                s = (0.1 + 0.2 * torch.rand(shape, dtype=dt, device="cuda")) if pp else None
                call = lambda: trid.adi_step(u, s=s, s0=0.2, nsteps=steps, stream=stream)  # noqa: E731
                pred, _ = trid.model_adi(dt, dims, batch, pp, steps, stream)
            else:
                a = 0.1 + 0.9 * torch.rand(shape, dtype=dt, device="cuda")
                b = 0.1 + 0.9 * torch.rand(shape, dtype=dt, device="cuda")
                c = 0.5 * torch.sqrt(a * b) * (2 * torch.rand(shape, dtype=dt, device="cuda") - 1)
                call = lambda: trid.hv_step(u, a, b, c, 0.25, 0.7887, steps, stream=stream)  # noqa: E731
                pred, _ = trid.model_hv(dt, dims, batch, steps, stream)
            trid.timing_enable(True)
            call()
            sync()
            trid.timing_enable(True)
            call()
            meas = sum(ms for _, ms in trid.timing_read().values()) * 1e3
            trid.timing_enable(False)
            e = abs(pred - meas) / meas
            errs.append(e)
            rows.append("%s %s %s x%d%s%s pred %.0f meas %.0f us" % (
                kind, str(dt)[6:], "x".join(map(str, dims)), batch, " s(x)" if pp else "",
                " per-step" if stream else "", pred, meas))
            del u
            torch.cuda.empty_cache()
    errs = np.array(errs)
    order = np.argsort(-errs)
    return {"calls": int(len(errs)), "mean_accuracy": round(1 - float(errs.mean()), 3),
            "median_accuracy": round(1 - float(np.median(errs)), 3),
            "within_15pct": round(float((errs <= 0.15).mean()), 3),
            "within_25pct": round(float((errs <= 0.25).mean()), 3),
            "worst": [rows[i] for i in order[:5]]}


def extra_varlen(trid):
    """20,000 systems with lengths log-uniform in [32, 8192] in one persistent launch.

    The FP32 + FP64-refinement result is compared with the FP64 result per
    system (max and median of the per-system relative inf-norm error)."""
    import json
    import tempfile

    import numpy as np
    import torch

    from workloads import gen

    a32, b32, c32, d64, off = gen.varlen_batch()
    rows = int(off[-1])
    # Each precision's kernel time is the median of 11 individually timed
    # (synchronised) calls after 10 warm-up calls: the first launches after a
    # precision's autotuned call (which frees the losing plans' schedules) run
    # slower, and the dispatch-stamped events of back-to-back launches of this
    # persistent kernel have read up to 1.5x the trace's kernel durations.
    # wall_ms is the mean wall time per call of 20 back-to-back calls, each a
    # replay of the captured launch (timer off).
    from paper_2201_03950_amd.model_calibrate import kernel_median_us

    def kernel_and_wall(call):
        kern = kernel_median_us(trid, call, reps=11, warm=10) * 1e-6
        return kern, time_calls(call, 20, warm=2)
    # fresh device allocations for the arrays (torch's cached blocks of the
    # earlier workloads released first): the work items read them at scattered
    # positions, and placements inside reused blocks measured up to 18% slower
    torch.cuda.empty_cache()
    os.environ["TRID_AUTOTUNE"] = "1"  # the first call times every tile plan on this batch
    res = {"systems": int(len(off) - 1), "rows": rows}
    ta, tb, tc, td = (torch.from_numpy(v).cuda() for v in (a32, b32, c32, d64))
    a64, b64, c64 = (v.double() for v in (ta, tb, tc))
    x64 = torch.empty_like(td)
    tune = {}
    trid.gtsv_varlen(trid.PREC_F64, a64, b64, c64, td, x64, off)  # the autotuned first call
    tune["f64"] = trid.autotune_report()
    kern, wall = kernel_and_wall(lambda: trid.gtsv_varlen(trid.PREC_F64, a64, b64, c64, td, x64, off))
    byts = alg_bytes("arrays", 8, rows)
    res["f64"] = {"ms": round(kern * 1e3, 4), "solves_per_s": round((len(off) - 1) / kern, 1),
                  "gbs": round(byts / kern / 1e9, 1), "frac": round(byts / kern / 1e9 / PEAK_GBS, 4),
                  "wall_ms": round(wall * 1e3, 4)}
    # plain FP32 (d rounded to FP32)
    td32 = td.float()
    x32 = torch.empty_like(td32)
    trid.gtsv_varlen(trid.PREC_F32, ta, tb, tc, td32, x32, off)
    tune["f32"] = trid.autotune_report()
    kern, wall = kernel_and_wall(lambda: trid.gtsv_varlen(trid.PREC_F32, ta, tb, tc, td32, x32, off))
    byts = alg_bytes("arrays", 4, rows)
    res["f32"] = {"ms": round(kern * 1e3, 4), "solves_per_s": round((len(off) - 1) / kern, 1),
                  "gbs": round(byts / kern / 1e9, 1), "frac": round(byts / kern / 1e9 / PEAK_GBS, 4),
                  "wall_ms": round(wall * 1e3, 4)}
    x = torch.empty_like(td)
    trid.gtsv_varlen(trid.PREC_F32_REFINE64, ta, tb, tc, td, x, off)
    tune["f32_refine64"] = trid.autotune_report()
    kern, wall = kernel_and_wall(lambda: trid.gtsv_varlen(trid.PREC_F32_REFINE64, ta, tb, tc, td, x, off))
    ref = x64.cpu().numpy()
    num = np.maximum.reduceat(np.abs(x.cpu().numpy() - ref), off[:-1])
    den = np.maximum.reduceat(np.abs(ref), off[:-1])
    e = num / den
    byts = 28 * rows
    res["f32_refine64"] = {"ms": round(kern * 1e3, 4), "solves_per_s": round((len(off) - 1) / kern, 1),
                           "gbs": round(byts / kern / 1e9, 1), "frac": round(byts / kern / 1e9 / PEAK_GBS, 4),
                           "err_vs_f64_max": float(e.max()), "err_vs_f64_median": float(np.median(e)),
                           "time_vs_f64": round(kern * 1e3 / res["f64"]["ms"], 3), "wall_ms": round(wall * 1e3, 4)}
    res["autotune"] = tune
    with tempfile.TemporaryDirectory() as tmp:  # the autotuned plans
        path = os.path.join(tmp, "plans.json")
        trid.plan_save(path)
        with open(path) as f:
            plans = json.load(f)["plans"]
    res["plans"] = {k.split("/")[1] + ("/small" if k.endswith("/small") else ""): v
                    for k, v in plans.items() if k.startswith("varlen/")}
    return {"varlen_20000": res}


def extra_gradient(trid):
    """Differentiable 3D ADI, 128^3, 20 steps, s = 0.2 kappa: forward vs forward+backward.

    Two reverse-pass modes: intermediates kept by the forward steps (default),
    or one checkpoint per step with the step recomputed in the reverse pass."""
    import numpy as np
    import torch

    from paper_2201_03950_amd import _binding as B
    from paper_2201_03950_amd import autograd
    from workloads import gen

    kappa, u0, kstar = gen.diffusion3d((128, 128, 128))
    steps, s0 = 20, 0.2
    tk, tu, tks = (torch.from_numpy(v).cuda() for v in (kappa, u0, kstar))
    with torch.no_grad():
        target = autograd.adi(tu, s0 * tks, steps, False)

    def fwd():
        with torch.no_grad():
            uT = autograd.adi(tu, s0 * tk, steps, False)
            return torch.sum((uT.double() - target.double()) ** 2)

    def fwd_bwd(keep, dt=torch.float32):
        k = tk.detach().to(dt).clone().requires_grad_(True)  # fresh leaves every call
        u = tu.detach().to(dt).clone().requires_grad_(True)
        uT = autograd.adi(u, s0 * k, steps, keep)
        loss = torch.sum((uT.double() - target.double()) ** 2)
        loss.backward()
        return k.grad, u.grad

    tf = time_calls(fwd, 3, warm=1)
    trid.timing_enable(True)
    fwd()
    fwd_kernels = {k: round(ms / c * 1e3, 2) for k, (c, ms) in trid.timing_read().items()}  # us per launch
    trid.timing_enable(False)
    tb_keep = time_calls(lambda: fwd_bwd(True), 3, warm=1)
    tb_rec = time_calls(lambda: fwd_bwd(False), 3, warm=1)
    # the kept-mode kernels, launched from this thread (autograd runs its
    # backward on a worker thread, whose handle is not the one timed here)
    s_pp = (s0 * tk).contiguous()
    u = tu.clone()
    saved = []
    trid.timing_enable(True)
    for _ in range(steps):
        ws = [torch.empty_like(u) for _ in range(3)]
        saved.append((u.clone(), ws))
        B.adi_step_keep(u, s_pp, *ws)
    ubar, sbar = torch.ones_like(u), torch.zeros_like(s_pp)
    for ck, ws in reversed(saved):
        B.adi_step_adjoint_kept(ck, s_pp, ws[0], ws[1], ws[2], ubar, sbar)
    kept_kernels = {k: [c, round(ms / c * 1e3, 2)] for k, (c, ms) in trid.timing_read().items()}
    trid.timing_enable(False)
    del saved
    u64 = tu.double()
    k64 = tk.double()
    tf64 = time_calls(lambda: autograd.adi(u64, s0 * k64, steps, False), 3, warm=1)
    # gradient error of the FP32 run: normwise against the FP64 GPU gradient of
    # the same loss (the FP64 path is itself checked against the oracle's
    # adjoint and finite differences in the tests)
    gk32, gu32 = fwd_bwd(True)
    gk64, gu64 = fwd_bwd(True, torch.float64)

    def nrel(a, b):
        return float((a.double() - b).norm() / b.norm())

    grad_err = {"dL_dkappa": nrel(gk32, gk64), "dL_du0": nrel(gu32, gu64)}
    return {"diff_adi3d_128_20steps": {"fwd_ms_f32": round(tf * 1e3, 3), "fwd_bwd_ms_f32": round(tb_keep * 1e3, 3),
                                       "fwd_bwd_over_fwd": round(tb_keep / tf, 3),
                                       "fwd_bwd_ms_f32_recompute": round(tb_rec * 1e3, 3),
                                       "fwd_bwd_over_fwd_recompute": round(tb_rec / tf, 3),
                                       "fwd_ms_f64": round(tf64 * 1e3, 3),
                                       "grad_err_f32_vs_f64": grad_err,
                                       "fwd_kernel_us": fwd_kernels, "kept_kernels_count_us": kept_kernels}}


def pmc_copy_calibration():
    """A plain device copy of known size (2 x 536,870,912 bytes moved), for counter scaling.

    The source is larger than every cache level (8 x 4 MB L2, 256 MB MALL) and a
    64 MB write in between evicts the L2s, so the copy's reads all miss."""
    import torch

    src = torch.ones(COPY_ELEMS, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    evict = torch.zeros(1 << 23, dtype=torch.float64, device="cuda")
    sync()
    dst.copy_(src)
    sync()
    del src, dst, evict


COPY_ELEMS = 1 << 26  # 512 MiB of float64


def pmc_read(d, counter):
    """Per-kernel-name list of a counter's per-dispatch values (bytes) from a rocprofv3 --pmc run."""
    import csv
    import glob

    per = {}
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
    return per


def pmc_copy_scale(per):
    """Known bytes of the calibration copy over what the counter reports for it
    (the largest device-to-device copy dispatch of the run)."""
    vals = [x for k, v in per.items() if "copyBuffer" in k for x in v]
    return COPY_ELEMS * 8.0 / max(vals)


def pmc_table(fetch_dir, write_dir):
    """Markdown table: launches and copy-scaled FETCH / WRITE bytes per launch of
    every library kernel in two rocprofv3 --pmc runs."""
    fetch, write = pmc_read(fetch_dir, "FETCH_SIZE"), pmc_read(write_dir, "WRITE_SIZE")
    kf, kw = pmc_copy_scale(fetch), pmc_copy_scale(write)
    print("| kernel | launches | FETCH (MB/launch) | WRITE (MB/launch) | total (MB/launch) |")
    print("|---|---|---|---|---|")
    for k in sorted(fetch):
        if "trid::" not in k:
            continue
        f = sum(fetch[k]) / len(fetch[k]) * kf
        wv = write.get(k, [0.0])
        w = sum(wv) / len(wv) * kw
        name = k.replace("(anonymous namespace)::", "").split("(")[0].replace("trid::", "").replace("void ", "")
        print("| `%s` | %d | %.2f | %.2f | %.2f |" % (name, len(fetch[k]),
                                                     f / 1e6, w / 1e6, (f + w) / 1e6))
    print("copy calibration factors: fetch %.4f, write %.4f" % (kf, kw))


def ingest_pmc(fetch_dir, write_dir):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) into HBM bytes per launch.

    Each counter is scaled by the ratio of the known bytes of the calibration copy
    (COPY_ELEMS float64 read and written once) to what the counter reports for it.
    Writes TRAFFIC_FILE (tagged with the current source hash) and prints a table.
    """
    fetch, write = pmc_read(fetch_dir, "FETCH_SIZE"), pmc_read(write_dir, "WRITE_SIZE")
    known = COPY_ELEMS * 8.0
    kf, kw = pmc_copy_scale(fetch), pmc_copy_scale(write)
    names = {"StgRhs": "adi_stencil_x", "EpiAdd": "adi_z_update", "EpiStore": "adi_y"}
    rec = {"source_hash": kernel_source_hash(), "copy_scale_fetch": kf, "copy_scale_write": kw,
           "copy_bytes": known, "kernels": {}}
    rows = []
    for k in sorted(fetch):
        if "trid::" not in k:
            continue
        tag = next((v for key, v in names.items() if key in k), k.split("(")[0])
        f = sum(fetch[k]) / len(fetch[k]) * kf
        w = sum(write.get(k, [0.0])) / max(1, len(write.get(k, []))) * kw
        rec["kernels"][tag] = {"fetch_bytes_per_launch": f, "write_bytes_per_launch": w,
                               "hbm_bytes_per_launch": f + w, "name": k.split("(")[0]}
        rows.append((tag, f, w))
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print("| kernel | FETCH (MB/launch) | WRITE (MB/launch) | total (MB) |")
    print("|---|---|---|---|")
    for tag, f, w in rows:
        print("| %s | %.1f | %.1f | %.1f |" % (tag, f / 1e6, w / 1e6, (f + w) / 1e6))
    print("copy calibration factors: fetch %.4f, write %.4f" % (kf, kw))


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo), and the
    CPUs this process may run on."""
    model, logical = "unknown", 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                if line.startswith("processor"):
                    logical += 1
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 0
    return {"model": model, "logical_cpus": logical, "usable_cpus": usable}


def cpu_baseline(budget_s=12.0, max_steps=60):
    """The oracle (never tuned) on the same 256^3 FP64 workload, a bounded number of steps."""
    from oracle import oracle
    from workloads import gen

    oracle.build()
    u = gen.adi3d_field((256, 256, 256), seed=1)
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps and (time.perf_counter() - t0) < budget_s:
        u = oracle.adi_step(u, s0=0.2, nsteps=1)
        steps += 1
    el = time.perf_counter() - t0
    cores = oracle.num_threads()
    # the same oracle on one host thread, one step
    oracle.set_num_threads(1)
    t1 = time.perf_counter()
    oracle.adi_step(u, s0=0.2, nsteps=1)
    el1 = time.perf_counter() - t1
    oracle.set_num_threads(cores)
    return {"value": round(3 * 65536 * steps / el, 1), "unit": "solves/s",
            "cores": cores, "kind": "oracle", "host": host_cpu(),
            "sample": "%d ADI step(s) of the 256^3 FP64 workload (s=0.2), %.1f s wall" % (steps, el),
            "value_1_thread": round(3 * 65536 / el1, 1)}


# The other workloads, each a function of the loaded binding returning {name: result}.
EXTRA_LEGS = {"adi2d_64x1024sq_xy": extra_2d, "varlen_20000": extra_varlen,
              "diff_adi3d_128_20steps": extra_gradient, "long_64x1M_f64": extra_long,
              "adi_small_batched": extra_small_batched, "hv_slv": extra_hv, "perf_model": extra_perf_model,
              "adi3d_80cubed_x72": extra_small3d(80), "adi3d_96cubed_x72": extra_small3d(96)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--pmc-copy", action="store_true",
                    help="run a plain copy of known size first (counter calibration)")
    ap.add_argument("--ingest-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the HBM-traffic summary from two rocprofv3 --pmc runs and exit")
    ap.add_argument("--only", choices=sorted(EXTRA_LEGS),
                    help="run one of the other workloads alone, print its JSON and exit (for profiling)")
    ap.add_argument("--pmc-table", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print copy-scaled HBM bytes per launch of every library kernel of two "
                         "rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    args = ap.parse_args()
    if args.ingest_pmc:
        ingest_pmc(*args.ingest_pmc)
        return
    if args.pmc_table:
        pmc_table(*args.pmc_table)
        return
    if args.gpus != 1:
        print("bench.py: only one GPU is measured; --gpus %d is not supported "
              "(sharding over several GPUs is a design, not built or run)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2201_03950_amd as trid

    trid.load_library()
    torch.cuda.init()
    if args.pmc_copy:
        pmc_copy_calibration()
    if args.only:
        print(json.dumps(EXTRA_LEGS[args.only](trid)))
        return
    log("main workload: 256^3 FP64 ADI, %d warmup + %d timed steps" % (args.warmup, args.steps))
    main_run = adi_main(trid, args.steps, args.warmup)
    log("main done: %.3f ms/step" % (main_run["elapsed"] / args.steps * 1e3))
    ms = main_run["elapsed"] / args.steps * 1e3
    value = main_run["solves_per_step"] * args.steps / main_run["elapsed"]
    kern = main_run["kernels"]
    dk = main_run["dominant"]
    dom = dk["kernel"]
    roofline = {"bound": "hbm", "achieved": dk["gbs"], "peak": PEAK_GBS, "unit": "GB/s",
                "frac": dk["frac"], "traffic": stored_traffic(dom), "kernel": dom,
                "launches": dk["launches"], "mean_ms": dk["mean_ms"]}
    extra = {"adi3d_256_f64": {"ms_per_step_graph": round(main_run["elapsed_graph"] / args.steps * 1e3, 4),
                               "kernels": kern, "kernels_sampled_every": TIMED_EVERY,
                               "fourier_err_10steps": main_run["fourier_err_10steps"]}}
    if not args.no_extra:
        log("extra workloads")
        extra.update(extra_workloads(trid))
    if not args.no_cpu:
        log("cpu baseline (oracle)")
    cpu = None if args.no_cpu else cpu_baseline()
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "adi3d_256x256x256_f64_const_s0.2", "mesh": [256, 256, 256], "batch": 1,
                   "solves_per_step": main_run["solves_per_step"], "kernels_per_step": 3},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
