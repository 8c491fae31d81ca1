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
    const VarlenParams &p = varlen_params();
    const int NW = varlen_wave_NW(prec, v.M);
    std::vector<int> order, tstart, wdesc;
    varlen_wave_pack(off, ids, v.M, NW, &order, &tstart, &wdesc);
    ModelTerms t;
    const double per_row = prec == 0 ? 40.0 : (prec == 1 ? 20.0 : 28.0);
    const double f = prec == 1 ? 1.0 : p.f64_factor;
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

}  // namespace trid
