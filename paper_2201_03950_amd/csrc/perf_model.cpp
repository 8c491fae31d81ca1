// perf_model.cpp -- predictive performance model (host only).
//
// A launch is modelled as its fixed cost plus the largest of three terms, as
// the memory stream and the per-tile sweeps overlap across resident
// workgroups:
//   bandwidth: the bytes the launch must move over the streaming bandwidth of
//              its access pattern;
//   chain:     one workgroup's critical path (M tile rows, the reduced-solve
//              levels, each LDS level slower with more wavefronts);
//   issue:     the grid's wavefronts over the chip's SIMD slots times each
//              wavefront's instruction time.
// The constants were fitted to kernel durations measured on one MI355X: for the
// line solves, a seeded random half of a sweep over both forms, FP64 and FP32,
// x/y/z lines of 32..8192 rows, 2^16..2^24 rows per call, automatic and forced
// tile plans; for the uneven batch, every plan of three length mixes.  The
// other half of the line sweep and three other mixes are the validation set.
#include "perf_model.hpp"

#include "resident.hpp"

#include <algorithm>
#include <cmath>

namespace trid {

namespace {

constexpr int kCUs = 256;
constexpr int kThreadsPerCU = 2048;      // 32 wavefronts of 64
constexpr double kLdsPerCU = 160 * 1024;
constexpr int kVgprPerSimdLane = 512;

int log2_ceil(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Workgroups of `threads` threads and `shmem` LDS bytes resident per CU, with
// the registers of a tile of M rows of w-byte words estimated as three words
// per row plus a fixed share.
int per_cu(int threads, double shmem, int M, int w) {
    const int vgpr = std::min(256, 24 + 3 * M * w / 4);
    const int waves_simd = std::max(1, kVgprPerSimdLane / vgpr);
    int n = std::max(1, kThreadsPerCU / std::max(threads, 64));
    n = std::min(n, std::max(1, (4 * waves_simd * 64) / std::max(threads, 64)));
    if (shmem > 0) n = std::min(n, std::max(1, (int)(kLdsPerCU / shmem)));
    return n;
}

}  // namespace

// Fitted (log-ratio least squares) to a calibration half of the sweep; the
// other half of the sweep is the validation set.
const LinesParams &lines_params() {
    static const LinesParams p{
        /*t0_us*/ 2.40,        /*bw_gbs*/ 6661.0,   /*seg_half*/ 17.5,     /*staged_eff*/ 0.986,
        /*xs_eff*/ 0.333,      /*arr_eff*/ 0.705,   /*lat_us*/ 0.0,        /*row_ns*/ 256.8,
        /*f64_factor*/ 1.053,  /*lvl_ns*/ 71.4,     /*lvl_wave_ns*/ 436.9, /*issue_row_ns*/ 140.5,
        /*issue_lvl_ns*/ 13.07,
    };
    return p;
}

const VarlenParams &varlen_params() {
    static const VarlenParams p{
        /*t0_us*/ 15.31,  /*bw_gbs*/ 3084.0,   /*lat_us*/ 3.663,  /*cu_gbs*/ 2000.0,
        /*row_ns*/ 321.6, /*f64_factor*/ 3.501, /*lvl_ns*/ 1236.9, /*thomas_ns*/ 103.7,
    };
    return p;
}

// Fitted on the wavefront plans of the same three calibration mixes, with
// t0 held within 2..6 us and the FP64 and refinement row factors at least 1.
const VarlenWaveParams &varlen_wave_params() {
    static const VarlenWaveParams p{
        /*t0_us*/ 6.0,     /*bw_gbs*/ 3493.40,    /*lat_us*/ 4.0953, /*cu_gbs*/ 362.45,
        /*row_ns*/ 538.09, /*f64_factor*/ 1.045, /*lvl_ns*/ 331.99, /*ref_factor*/ 1.0037,
    };
    return p;
}

// Fitted like LinesParams: on the calibration shapes of model_calibrate.py's
// ADI sweep (the other shapes are its validation set).
const AdiParams &adi_params() {
    static const AdiParams p{
        /*sx_eff*/ 1.0,      /*sx_blk_us*/ 5.534, /*cs_eff*/ 0.9303, /*cs_blk_us*/ 3.688, /*res_io_ns*/ 5296.7,
        /*res_ns*/ 62.56,    /*res_f64*/ 1.938,   /*hv_ns*/ 852.8,    /*pred_eff*/ 0.882,
    };
    return p;
}

ModelTerms model_lines(const LineReq &r, const LinePlan &pl) {
    const LinesParams &p = lines_params();
    const int w = r.f64 ? 8 : 4;
    int words = 3;  // s form: s, d in, x out
    if (r.mode == Mode::Arrays || r.mode == Mode::ArraysT) words = 5;
    if (r.mode == Mode::Const) words = 2;
    if (r.out == Out::Add) words += 1;
    ModelTerms t;
    const double rows = (double)r.n * (double)r.inner * (double)r.outer;
    t.bytes = words * (double)w * rows;
    double eff;
    if (pl.staged) {
        eff = p.staged_eff;
    } else if (r.inner == 1) {
        eff = p.xs_eff;
    } else {
        const double seg = (double)std::min<i64>(pl.L, r.inner) * w;  // contiguous bytes per tile row
        eff = seg / (seg + p.seg_half);
    }
    if (r.mode == Mode::Arrays || r.mode == Mode::ArraysT) eff *= p.arr_eff;
    t.t_bytes = t.bytes / (p.bw_gbs * eff * 1e3);
    t.per_cu = per_cu(pl.threads(), (double)pl.shmem, pl.M, w);
    t.rounds = std::ceil((double)pl.nblocks / (double)(kCUs * t.per_cu));
    const double f = r.f64 ? p.f64_factor : 1.0;
    const int lev = log2_ceil(pl.P);
    const bool dpp = pl.staged && pl.P <= 16;  // reduced solve by lane moves, no LDS levels
    const double chain =
        p.lat_us + (pl.M * p.row_ns * f + lev * (p.lvl_ns + (dpp ? 0.0 : p.lvl_wave_ns * pl.threads() / 256.0))) * 1e-3;
    const double waves = (double)pl.nblocks * std::ceil(pl.threads() / 64.0);
    const double issue = waves / (4.0 * kCUs) * (pl.M * p.issue_row_ns * f + lev * p.issue_lvl_ns) * 1e-3;
    t.t_lat = std::max(chain, issue);
    t.us = p.t0_us + std::max(t.t_bytes, t.t_lat);
    return t;
}

// Wavefront variants: a work item is a workgroup's wavefront slots; its cost
// is one workgroup's stream of the item's rows plus the tile sweep and the
// in-wavefront reduced solve (six lane-move PCR levels, lvl_ns / 4 each, as
// they need no barrier), plus one level for the exchange of a long system.
static ModelTerms model_varlen_wave(const int64_t *off, const std::vector<int> &ids, int prec, const VarlenVariant &v,
                                    int blocks) {
    const VarlenWaveParams &p = varlen_wave_params();
    const int NW = varlen_wave_NW(prec, v.M);
    std::vector<int> order, tstart, wdesc;
    varlen_wave_pack(off, ids, v.M, NW, &order, &tstart, &wdesc);
    ModelTerms t;
    const double per_row = prec == 0 ? 40.0 : (prec == 1 ? 20.0 : 28.0);
    const double f = prec == 0 ? p.f64_factor : (prec == 1 ? 1.0 : p.ref_factor);
    const size_t nitems = wdesc.size() / 4 / NW;
    double sum = 0, rows = 0, mx = 0;
    for (size_t i = 0; i < nitems; ++i) {
        double irows = 0;
        bool lng = false;
        for (int w = 0; w < NW; ++w) {
            const int *dsc = &wdesc[(i * NW + w) * 4];
            if (dsc[3] > 0) {
                lng = true;
                if ((dsc[2] & 0xff) == w) irows += (double)(off[order[dsc[0]] + 1] - off[order[dsc[0]]]);
            } else {
                for (int j = 0; j < dsc[1]; ++j) irows += (double)(off[order[dsc[0] + j] + 1] - off[order[dsc[0] + j]]);
            }
        }
        const double red = (6 * p.lvl_ns / 4 + (lng ? p.lvl_ns : 0.0)) * (prec == 2 ? 2 : 1);
        const double c = p.lat_us + irows * per_row / (p.cu_gbs * 1e3) + (v.M * p.row_ns * f + red) * 1e-3;
        sum += c;
        rows += irows;
        mx = std::max(mx, c);
    }
    t.bytes = per_row * rows;
    t.t_bytes = t.bytes / (p.bw_gbs * 1e3);
    const int b = std::max(1, std::min(blocks, (int)nitems));
    t.per_cu = std::max(1, blocks / kCUs);
    t.rounds = (double)nitems / b;
    t.t_lat = std::max(sum / b, mx);
    t.us = p.t0_us + std::max(t.t_bytes, t.t_lat);
    return t;
}

ModelTerms model_varlen(const int64_t *off, std::vector<int> ids, int prec, const VarlenVariant &v, int blocks) {
    if (v.wave) return model_varlen_wave(off, ids, prec, v, blocks);
    const VarlenParams &p = varlen_params();
    std::vector<int> tstart, item_begin, item_pmax;
    varlen_pack(off, &ids, v, &tstart, &item_begin, &item_pmax);
    ModelTerms t;
    const double per_row = prec == 0 ? 40.0 : (prec == 1 ? 20.0 : 28.0);  // a, b, c, d in, x out
    const double f = prec == 1 ? 1.0 : p.f64_factor;
    // the longest item is bounded by the largest rows and reduced-solve cost
    // of any item (the packing puts the longest systems first)
    double sum = 0, rows = 0, rmax = 0, redmax = 0;
    for (size_t i = 0; i < item_pmax.size(); ++i) {
        double irows = 0;
        for (int k = item_begin[i]; k < item_begin[i + 1]; ++k) irows += (double)(off[ids[k] + 1] - off[ids[k]]);
        const int pm = item_pmax[i];
        const double red = v.thomas ? pm * p.thomas_ns : log2_ceil(pm) * p.lvl_ns;
        sum += p.lat_us + irows * per_row / (p.cu_gbs * 1e3) + (v.M * p.row_ns * f + red) * 1e-3;
        rows += irows;
        rmax = std::max(rmax, irows);
        redmax = std::max(redmax, red);
    }
    const double mx = p.lat_us + rmax * per_row / (p.cu_gbs * 1e3) + (v.M * p.row_ns * f + redmax) * 1e-3;
    t.bytes = per_row * rows;
    t.t_bytes = t.bytes / (p.bw_gbs * 1e3);
    const int b = std::max(1, std::min(blocks, (int)item_pmax.size()));
    t.per_cu = std::max(1, blocks / kCUs);
    t.rounds = (double)item_pmax.size() / b;
    t.t_lat = std::max(sum / b, mx);
    t.us = p.t0_us + std::max(t.t_bytes, t.t_lat);
    return t;
}

// ------------------------------------------------------------ ADI / HV --

namespace {

// A bandwidth-or-latency kernel: t0 + max(bytes at bw * eff, rounds * blk).
KernelPred stream_kernel(const char *name, const char *cls, double bytes, i64 nblocks, int threads, double shmem,
                         int M, int w, double eff, double blk_us, int launches) {
    const LinesParams &lp = lines_params();
    KernelPred k;
    k.name = name;
    k.cls = cls;
    k.launches = launches;
    k.bytes = bytes;
    const int pc = per_cu(threads, shmem, M, w);
    k.rounds = std::ceil((double)nblocks / (double)(kCUs * pc));
    k.us = launches * (lp.t0_us + std::max(bytes / (lp.bw_gbs * eff * 1e3), k.rounds * blk_us));
    return k;
}

KernelPred line_kernel(const char *name, const LineReq &q, int launches, std::string *err, bool *ok) {
    const AdiParams &ap = adi_params();
    const int w = q.f64 ? 8 : 4;
    const int cm = const_lines_M(q);
    if (cm) {  // k_strided_const: 64 lines x P tiles per workgroup
        const int P = (int)(q.n / cm);
        int words = 2 + (q.out == Out::Add ? 1 : 0);
        const double rows = (double)q.n * (double)q.inner * (double)q.outer;
        const i64 nb = (q.inner * q.outer + 63) / 64;
        return stream_kernel(name, "const_lines", words * w * rows, nb, 64 * P, 2.0 * 8 * 64 * w, cm, w, ap.cs_eff,
                             ap.cs_blk_us, launches);
    }
    LinePlan pl;
    KernelPred k;
    k.name = name;
    k.cls = "lines";
    k.launches = launches;
    if (!plan_lines(q, &pl, err)) {
        *ok = false;
        return k;
    }
    const ModelTerms t = model_lines(q, pl);
    k.us = launches * t.us;
    k.bytes = t.bytes;
    k.rounds = t.rounds;
    return k;
}

}  // namespace

bool model_adi(const AdiReq &r, int nsteps, bool stream, std::vector<KernelPred> *ks, std::string *err) {
    const AdiParams &ap = adi_params();
    const int w = r.f64 ? 8 : 4;
    ks->clear();
    if (r.ndim == 2 && !stream) {
        ResidentReq rr;
        rr.f64 = r.f64;
        rr.u = const_cast<void *>(r.u);
        rr.s = r.s;
        rr.nx = r.nx;
        rr.ny = r.ny;
        rr.batch = r.batch;
        rr.nsteps = nsteps;
        int64_t lay[10];
        if (resident_fits(rr) && resident_layout(rr, 0, lay)) {
            const int threads = (int)lay[8];
            const double bytes = (double)lay[9];
            const int pc = std::max(1, std::min(kThreadsPerCU / threads, (int)(kLdsPerCU / bytes)));
            KernelPred k;
            k.name = "adi2d_resident";
            k.cls = "resident";
            k.launches = 1;
            k.bytes = (2.0 + (r.s ? 1.0 : 0.0)) * w * (double)(r.nx * r.ny * r.batch);
            k.rounds = std::ceil((double)r.batch / (double)(kCUs * pc));
            k.units = (double)(r.nx * r.ny) / threads;
            const double ns = ap.res_io_ns + nsteps * ap.res_ns * (r.f64 ? ap.res_f64 : 1.0);
            k.us = lines_params().t0_us + k.rounds * k.units * ns * 1e-3;
            ks->push_back(k);
            return true;
        }
    }
    const double pts = (double)(r.nx * r.ny * r.nz * r.batch);
    // stencil + x
    const int cmx = const_rhs_M(r);
    if (cmx) {
        int threads, L;
        size_t shm;
        i64 nb;
        const_rhs_geometry(r, cmx, &threads, &L, &shm, &nb);
        ks->push_back(stream_kernel("adi_stencil_x", "stencil_x", 2.0 * w * pts, nb, threads, (double)shm, cmx, w,
                                    ap.sx_eff, ap.sx_blk_us, nsteps));
    } else {
        LinePlan px;
        if (!plan_rhs_x(r, &px, err)) return false;
        ks->push_back(stream_kernel("adi_stencil_x", "stencil_x", (r.s ? 3.0 : 2.0) * w * pts, px.nblocks,
                                    px.threads(), (double)px.shmem, px.M, w, ap.sx_eff, ap.sx_blk_us, nsteps));
    }
    LineReq ry;
    ry.f64 = r.f64;
    ry.mode = r.s ? Mode::S : Mode::Const;
    ry.ca = -r.s0;
    ry.cb = 1.0 + 2.0 * r.s0;
    ry.cc = -r.s0;
    ry.s = r.s;
    ry.d = r.d;
    ry.x = r.ndim == 2 ? const_cast<void *>(r.u) : r.d;
    ry.inner = r.nx;
    ry.n = r.ny;
    ry.outer = r.nz * r.batch;
    ry.out = r.ndim == 2 ? Out::Add : Out::Store;
    ry.force_M = r.force_M;
    ry.force_L = r.force_L;
    bool ok = true;
    ks->push_back(line_kernel(r.ndim == 3 ? "adi_y" : "adi_y_update", ry, nsteps, err, &ok));
    if (r.ndim == 3) {
        LineReq rz = ry;
        rz.inner = r.nx * r.ny;
        rz.n = r.nz;
        rz.outer = r.batch;
        rz.out = Out::Add;
        rz.x = const_cast<void *>(r.u);
        ks->push_back(line_kernel("adi_z_update", rz, nsteps, err, &ok));
    }
    return ok;
}

bool model_hv(bool f64, i64 nx, i64 ny, i64 batch, int nsteps, bool stream, std::vector<KernelPred> *ks,
              std::string *err) {
    const AdiParams &ap = adi_params();
    const int w = f64 ? 8 : 4;
    ks->clear();
    // 16-byte aligned non-NULL stand-ins for the requests' arrays (the plans depend on alignment only)
    alignas(16) static char one[16] = {0};
    if (!stream) {
        ResidentReq rr;
        rr.f64 = f64;
        rr.u = one;
        rr.nx = nx;
        rr.ny = ny;
        rr.batch = batch;
        rr.nsteps = nsteps;
        rr.hv = true;
        rr.a = rr.b = rr.c = one;
        int64_t lay[10];
        if (resident_fits(rr) && resident_layout(rr, 0, lay)) {
            const int threads = (int)lay[8];
            const double bytes = (double)lay[9];
            const int pc = std::max(1, std::min(kThreadsPerCU / threads, (int)(kLdsPerCU / bytes)));
            KernelPred k;
            k.name = "hv_resident";
            k.cls = "hv_resident";
            k.launches = 1;
            k.bytes = 5.0 * w * (double)(nx * ny * batch);  // u in and out, a, b, c once
            k.rounds = std::ceil((double)batch / (double)(kCUs * pc));
            k.units = (double)(nx * ny) / threads;
            const double ns = ap.res_io_ns + nsteps * ap.hv_ns * (f64 ? ap.res_f64 : 1.0);
            k.us = lines_params().t0_us + k.rounds * k.units * ns * 1e-3;
            ks->push_back(k);
            return true;
        }
    }
    const double pts = (double)(nx * ny * batch);
    const i64 nb = (i64)std::ceil(pts / 256.0);
    // predictors: 6 + 4 + 6 + 4 words per point and step; the coefficient fill once per call
    ks->push_back(stream_kernel("hv_pred", "hv_pred", 5.0 * w * pts, nb, 256, 0.0, 8, w, ap.pred_eff, 0.0,
                                4 * nsteps));
    ks->back().us += stream_kernel("", "", 4.0 * w * pts, nb, 256, 0.0, 8, w, ap.pred_eff, 0.0, 1).us;
    bool ok = true;
    for (int axis = 0; axis < 2; ++axis) {
        LineReq q;
        q.f64 = f64;
        q.mode = Mode::S;
        q.s = one;
        q.d = one;
        q.x = one;
        q.out = Out::Store;
        q.inner = axis == 0 ? 1 : nx;
        q.n = axis == 0 ? nx : ny;
        q.outer = axis == 0 ? ny * batch : batch;
        ks->push_back(line_kernel(axis == 0 ? "gtsv_staged" : "gtsv_strided", q, 2 * nsteps, err, &ok));
    }
    return ok;
}

}  // namespace trid
