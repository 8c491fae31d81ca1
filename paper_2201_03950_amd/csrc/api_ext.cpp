// api_ext.cpp -- extern "C" entry points beyond the plain solves: tile-plan
// control and timing, refinement, line-solve and ADI-step adjoints, the uneven
// batch (schedule cache, autotuner, graph replay) and the plan cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "../../include/trid.h"
#include "dispatch.hpp"
#include "ext.hpp"
#include "hv.hpp"
#include "long_ext.hpp"
#include "long_lines.hpp"
#include "perf_model.hpp"
#include "refine.hpp"
#include "resident.hpp"
#include "varlen.hpp"

namespace trid {

LaunchEvents &launch_events() {
    thread_local LaunchEvents ev;
    return ev;
}

}  // namespace trid

namespace trid {

void ExtState::release() {
    timer.release();
    if (ws2) hipFree(ws2);
    ws2 = nullptr;
    ws2_bytes = 0;
    varlen.clear([](const std::string &, VarlenSchedule *sc) {
        varlen_free(sc);
        delete sc;
    });
    if (capture_stream) hipStreamDestroy(capture_stream);
    capture_stream = nullptr;
}

int handle_workspace2(trid_handle_t h, size_t bytes, void **ptr) {
    if (alloc_failure_forced())
        return handle_fail(h, TRID_ERR_ALLOC, "workspace allocation failed (TRID_FAIL_ALLOC)");
    ExtState &x = handle_ext(h);
    if (x.ws2_bytes < bytes) {
        if (x.ws2) {
            hipError_t e = hipStreamSynchronize(handle_stream(h));
            if (e != hipSuccess) return handle_hip_fail(h, e, "hipStreamSynchronize");
            hipFree(x.ws2);
            x.ws2 = nullptr;
            x.ws2_bytes = 0;
        }
        hipError_t e = hipMalloc(&x.ws2, bytes);
        if (e != hipSuccess) {
            x.ws2 = nullptr;
            return handle_fail(h, TRID_ERR_ALLOC, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
        }
        x.ws2_bytes = bytes;
    }
    *ptr = x.ws2;
    return TRID_OK;
}

}  // namespace trid

extern "C" {

int trid_set_tile(trid_handle_t h, int M, int L) {
    if (!h) return TRID_ERR_ARG;
    if (M != 0 && M != 8 && M != 16 && M != 32)
        return trid::handle_fail(h, TRID_ERR_ARG, "tile rows must be 0, 8, 16 or 32");
    if (L < 0 || L > 1024 || (L & (L - 1)) != 0)
        return trid::handle_fail(h, TRID_ERR_ARG, "lines per block must be 0 or a power of two <= 1024");
    trid::ExtState &x = trid::handle_ext(h);
    x.force_M = M;
    x.force_L = L;
    return TRID_OK;
}

int trid_timing_enable(trid_handle_t h, int on) {
    if (!h) return TRID_ERR_ARG;
    trid::ExtState &x = trid::handle_ext(h);
    hipError_t e = x.timer.flush();
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "timing flush");
    x.timer.acc.clear();
    x.timer.on = on != 0;
    return TRID_OK;
}

int trid_timing_select(trid_handle_t h, const char *name, int every) {
    if (!h) return TRID_ERR_ARG;
    if (name && strlen(name) > 200) return trid::handle_fail(h, TRID_ERR_ARG, "kernel name too long");
    if (every < 1) return trid::handle_fail(h, TRID_ERR_ARG, "every must be >= 1");
    trid::ExtState &x = trid::handle_ext(h);
    hipError_t e = x.timer.flush();
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "timing flush");
    x.timer.acc.clear();
    x.timer.only = name ? name : "";
    x.timer.every = every;
    x.timer.seen.clear();
    return TRID_OK;
}

int trid_timing_read(trid_handle_t h, char *buf, int64_t len) {
    if (!h || !buf || len < 3) return h ? trid::handle_fail(h, TRID_ERR_ARG, "bad buffer") : TRID_ERR_ARG;
    trid::ExtState &x = trid::handle_ext(h);
    hipError_t e = x.timer.flush();
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "timing flush");
    std::string out = "{";
    bool first = true;
    for (auto &kv : x.timer.acc) {
        char tmp[256];
        snprintf(tmp, sizeof tmp, "%s\"%s\": [%ld, %.6f]", first ? "" : ", ", kv.first.c_str(),
                 kv.second.first, kv.second.second);
        out += tmp;
        first = false;
    }
    out += "}";
    if ((int64_t)out.size() + 1 > len) return trid::handle_fail(h, TRID_ERR_ARG, "buffer too small");
    memcpy(buf, out.c_str(), out.size() + 1);
    return TRID_OK;
}

// Contiguous lines longer than TRID_MAX_LINE: the transposed solve through the
// chunked solve, with the transposed rows in the handle's workspace.
static int run_long_adjoint(trid_handle_t h, const trid::LongAdjReq &q) {
    void *ws = nullptr;
    int rc = trid::handle_workspace2(h, trid::long_adjoint_workspace(q.f64, q.n, q.lines), &ws);
    if (rc) return rc;
    hipStream_t st = trid::handle_stream(h);
    std::string msg;
    hipError_t e = trid::handle_ext(h).timer.time_recorded(
        "adjoint_long", st, [&] { return trid::launch_long_adjoint(q, ws, st, &msg); });
    if (e != hipSuccess) {
        if (!msg.empty()) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
        return trid::handle_hip_fail(h, e, "long-line adjoint launch");
    }
    return TRID_OK;
}

// Contiguous lines longer than TRID_MAX_LINE: the refinement as passes around
// the chunked FP32 solve, with x32 and the residual in the handle's workspace.
static int run_long_refine(trid_handle_t h, const trid::LongRefineReq &q) {
    void *ws = nullptr;
    int rc = trid::handle_workspace2(h, trid::long_refine_workspace(q.n, q.lines), &ws);
    if (rc) return rc;
    hipStream_t st = trid::handle_stream(h);
    std::string msg;
    hipError_t e = trid::handle_ext(h).timer.time_recorded(
        "refine_long", st, [&] { return trid::launch_long_refine(q, ws, st, &msg); });
    if (e != hipSuccess) {
        if (!msg.empty()) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
        return trid::handle_hip_fail(h, e, "long-line refinement launch");
    }
    return TRID_OK;
}

int trid_gtsv_batched_adjoint(trid_handle_t h, trid_dtype_t dt, const void *a, const void *b,
                              const void *c, const void *x, void *g, void *ga, void *gb, void *gc,
                              int ndim, const int64_t *dims, int axis, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (!a || !b || !c || !x || !g || !ga || !gb || !gc)
        return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    trid::LineReq r;
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer, true);
    if (rc) return rc;
    if (r.n > TRID_MAX_LINE) {
        trid::LongAdjReq q;
        q.f64 = dt == TRID_F64;
        q.a = a;
        q.b = b;
        q.c = c;
        q.x = x;
        q.g = g;
        q.ga = ga;
        q.gb = gb;
        q.gc = gc;
        q.n = r.n;
        q.lines = r.outer;
        return run_long_adjoint(h, q);
    }
    r.f64 = dt == TRID_F64;
    r.mode = trid::Mode::ArraysT;
    r.out = trid::Out::AdjArrays;
    r.a = a;
    r.b = b;
    r.c = c;
    r.xf = x;
    r.g = g;
    r.ga = ga;
    r.gb = gb;
    r.gc = gc;
    return trid::handle_run_lines(h, r);
}

int trid_gtsv_batched_s_adjoint(trid_handle_t h, trid_dtype_t dt, const void *s, const void *x,
                                void *g, void *gs, int ndim, const int64_t *dims, int axis,
                                int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (!s || !x || !g || !gs) return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    trid::LineReq r;
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer, true);
    if (rc) return rc;
    if (r.n > TRID_MAX_LINE) {
        trid::LongAdjReq q;
        q.f64 = dt == TRID_F64;
        q.s = s;
        q.x = x;
        q.g = g;
        q.gs = gs;
        q.n = r.n;
        q.lines = r.outer;
        return run_long_adjoint(h, q);
    }
    r.f64 = dt == TRID_F64;
    r.mode = trid::Mode::ST;
    r.out = trid::Out::AdjS;
    r.s = s;
    r.xf = x;
    r.g = g;
    r.gs = gs;
    return trid::handle_run_lines(h, r);
}

static int run_refine(trid_handle_t h, trid::RefineReq &r, const char *what) {
    trid::ExtState &x = trid::handle_ext(h);
    if (x.force_M == 16 || x.force_M == 32) r.force_M = x.force_M;
    if (x.force_L) r.force_L = x.force_L;
    trid::RefPlan pl;
    std::string msg;
    if (!trid::plan_refine(r, &pl, &msg)) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
    hipStream_t st = trid::handle_stream(h);
    hipError_t e = x.timer.time(pl.staged ? "refine_staged" : "refine_strided", st,
                                [&] { return trid::launch_refine(r, pl, st); });
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, what);
    return TRID_OK;
}

int trid_gtsv_batched_refine(trid_handle_t h, trid_dtype_t d_dt, const float *a, const float *b,
                             const float *c, const void *d, double *x, int ndim, const int64_t *dims,
                             int axis, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (d_dt != TRID_F32 && d_dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype of d");
    if (!a || !b || !c || !d || !x) return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    if ((const void *)x == d) return trid::handle_fail(h, TRID_ERR_ARG, "x may not alias d");
    trid::RefineReq r;
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer, true);
    if (rc) return rc;
    if (r.n > TRID_MAX_LINE) {
        trid::LongRefineReq q;
        q.a = a;
        q.b = b;
        q.c = c;
        q.d = d;
        q.d_f64 = d_dt == TRID_F64;
        q.x = x;
        q.n = r.n;
        q.lines = r.outer;
        return run_long_refine(h, q);
    }
    r.smode = false;
    r.d_f64 = d_dt == TRID_F64;
    r.src.a = a;
    r.src.b = b;
    r.src.c = c;
    r.d = d;
    r.x = x;
    return run_refine(h, r, "refine launch");
}

int trid_gtsv_batched_s_refine(trid_handle_t h, trid_dtype_t d_dt, const float *s, const void *d, double *x,
                               int ndim, const int64_t *dims, int axis, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (d_dt != TRID_F32 && d_dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype of d");
    if (!s || !d || !x) return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    if ((const void *)x == d) return trid::handle_fail(h, TRID_ERR_ARG, "x may not alias d");
    trid::RefineReq r;
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer, true);
    if (rc) return rc;
    if (r.n > TRID_MAX_LINE) {
        trid::LongRefineReq q;
        q.s = s;
        q.d = d;
        q.d_f64 = d_dt == TRID_F64;
        q.x = x;
        q.n = r.n;
        q.lines = r.outer;
        return run_long_refine(h, q);
    }
    r.smode = true;
    r.d_f64 = d_dt == TRID_F64;
    r.src.s = s;
    r.d = d;
    r.x = x;
    return run_refine(h, r, "refine launch");
}

namespace {

// Plan-cache key of an uneven batch: precision, count and a log2 histogram of lengths.
std::string varlen_plan_key(const int64_t *off, int64_t nsys, int prec) {
    int hist[64] = {0};
    for (int64_t k = 0; k < nsys; ++k) {
        int64_t len = off[k + 1] - off[k];
        int b = 0;
        while ((int64_t)1 << (b + 1) <= len) ++b;
        ++hist[b];
    }
    std::ostringstream os;
    os << "varlen/p" << prec << "/n" << nsys << "/h";
    bool first = true;
    for (int b = 0; b < 64; ++b)
        if (hist[b]) {
            os << (first ? "" : ",") << b << ":" << hist[b];
            first = false;
        }
    return os.str();
}

// Exact identity of an offsets array (FNV-1a) for the schedule cache.
std::string varlen_sched_key(const int64_t *off, int64_t nsys, int prec) {
    uint64_t h = 1469598103934665603ull;
    for (int64_t k = 0; k <= nsys; ++k) {
        uint64_t v = (uint64_t)off[k];
        for (int byte = 0; byte < 8; ++byte) {
            h ^= (v >> (8 * byte)) & 0xff;
            h *= 1099511628211ull;
        }
    }
    char buf[64];
    snprintf(buf, sizeof buf, "%d/%lld/%016llx", prec, (long long)nsys, (unsigned long long)h);
    return buf;
}

bool autotune_requested() {
    const char *v = std::getenv("TRID_AUTOTUNE");
    return v && v[0] == '1';
}

// Plans the autotuner times: the best TRID_AUTOTUNE_TOP by the model (default
// 3; 0 times every plan).
size_t autotune_top() {
    const char *v = std::getenv("TRID_AUTOTUNE_TOP");
    if (!v || !*v) return 3;
    const long n = std::strtol(v, nullptr, 10);
    return n <= 0 ? (size_t)-1 : (size_t)n;
}

// Predicted time of an uneven-batch plan: one launch, or for a split plan the
// launch of the long systems with v followed by the short ones with `small`
// (the partition of varlen_build).
double predict_varlen_plan(const int64_t *off, int64_t nsys, int prec, const trid::VarlenVariant &v, bool split,
                           const trid::VarlenVariant &small) {
    // the systems of the persistent launch (the longer ones take the chunked
    // solve under every plan)
    std::vector<int> all, lng, shr;
    for (int64_t k = 0; k < nsys; ++k)
        if (off[k + 1] - off[k] <= trid::kVarlenMaxTiled) all.push_back((int)k);
    if (all.empty()) return 0.0;
    if (!split) return trid::model_varlen(off, all, prec, v, trid::varlen_blocks(prec, v)).us;
    const int64_t cap = (int64_t)small.M * small.NT;
    for (int k : all) (off[k + 1] - off[k] > cap ? lng : shr).push_back(k);
    double us = 0;
    if (!lng.empty()) us += trid::model_varlen(off, lng, prec, v, trid::varlen_blocks(prec, v)).us;
    if (!shr.empty()) us += trid::model_varlen(off, shr, prec, small, trid::varlen_blocks(prec, small)).us;
    return us;
}

// Time one schedule: one warm-up and three timed launches on stream st.
hipError_t time_schedule(const trid::VarlenSchedule &sc, const void *a, const void *b, const void *c,
                         const void *d, void *x, hipStream_t st, float *us) {
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return e;
    }
    e = trid::varlen_launch(sc, a, b, c, d, x, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int i = 0; i < 3 && e == hipSuccess; ++i) e = trid::varlen_launch(sc, a, b, c, d, x, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    *us = ms * 1000.f / 3.f;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return e;
}

}  // namespace

int trid_gtsv_varlen(trid_handle_t h, trid_prec_t prec, const void *a, const void *b, const void *c,
                     const void *d, void *x, const int64_t *off, int64_t nsys) {
    if (!h) return TRID_ERR_ARG;
    if (prec != TRID_PREC_F64 && prec != TRID_PREC_F32 && prec != TRID_PREC_F32_REFINE64)
        return trid::handle_fail(h, TRID_ERR_ARG, "bad precision");
    if (!a || !b || !c || !d || !x || !off) return trid::handle_fail(h, TRID_ERR_ARG, "NULL pointer");
    if (nsys < 1 || nsys > ((int64_t)1 << 30)) return trid::handle_fail(h, TRID_ERR_ARG, "nsys out of range");
    if (prec == TRID_PREC_F32_REFINE64 && d == x) return trid::handle_fail(h, TRID_ERR_ARG, "x may not alias d");
    if (off[0] != 0) return trid::handle_fail(h, TRID_ERR_ARG, "offsets[0] must be 0");
    int64_t maxlen = 0, nlong = 0;  // longest system of the persistent launch; systems of the chunked solve
    for (int64_t k = 0; k < nsys; ++k) {
        const int64_t len = off[k + 1] - off[k];
        if (len < 1) return trid::handle_fail(h, TRID_ERR_ARG, "every system needs at least one row");
        if (len > TRID_MAX_LONG_LINE)
            return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, "system longer than TRID_MAX_LONG_LINE");
        if (len > trid::kVarlenMaxTiled)
            ++nlong;
        else
            maxlen = std::max(maxlen, len);
    }
    trid::ExtState &xs = trid::handle_ext(h);
    hipStream_t st = trid::handle_stream(h);
    const int p = (int)prec;
    const std::string skey = varlen_sched_key(off, nsys, p);
    trid::VarlenSchedule **found = xs.varlen.find(skey);
    if (!found) {
        const std::string pkey = varlen_plan_key(off, nsys, p);
        std::vector<trid::VarlenVariant> cands;
        for (const auto &v : trid::varlen_variants(p))
            if (trid::varlen_variant_fits(v, maxlen)) cands.push_back(v);
        if (cands.empty()) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, "no tile plan fits the longest system");
        // split plans: systems longer than a 256-thread block of 8-row tiles
        // holds run with a big-block variant, the rest with 256-thread blocks
        // (several per CU)
        const trid::VarlenVariant small{8, 256};
        struct Plan {
            trid::VarlenVariant v;
            bool split;
        };
        std::vector<Plan> plans;
        for (const auto &v : cands) plans.push_back({v, false});
        if (maxlen > (int64_t)small.M * small.NT)
            for (const auto &v : cands)
                if (v.NT > small.NT && !v.wave) plans.push_back({v, true});
        auto tuned = xs.tuned.find(pkey);
        auto tuned_small = xs.tuned.find(pkey + "/small");
        const bool tune = autotune_requested() && plans.size() > 1;
        trid::VarlenSchedule *best = nullptr;
        if (tune) {
            // Candidates are timed on this call's inputs.  Each timing runs the
            // solve several times; when x is d (an in-place solve), a repeated
            // run would solve again with its own output, so the timed runs then
            // write a workspace array instead, and the real solve follows once.
            void *xt = x;
            if (x == d) {
                const size_t bytes = (size_t)off[nsys] * (p == 1 ? sizeof(float) : sizeof(double));
                int rc = trid::handle_workspace2(h, bytes, &xt);
                if (rc) return rc;
            }
            bool best_split = false;
            // rank the plans by the model, time the best few
            std::vector<double> pred(plans.size());
            std::vector<size_t> rank(plans.size());
            for (size_t i = 0; i < plans.size(); ++i) {
                pred[i] = predict_varlen_plan(off, nsys, p, plans[i].v, plans[i].split, small);
                rank[i] = i;
            }
            std::stable_sort(rank.begin(), rank.end(), [&](size_t x, size_t y) { return pred[x] < pred[y]; });
            const size_t ntime = std::min(plans.size(), autotune_top());
            xs.last_tune.clear();
            for (size_t i : rank) {
                trid::TuneRecord tr;
                tr.M = plans[i].v.M;
                tr.NT = plans[i].v.NT;
                tr.thomas = plans[i].v.thomas;
                tr.wave = plans[i].v.wave;
                tr.split = plans[i].split ? 1 : 0;
                tr.blocks = trid::varlen_blocks(p, plans[i].v);
                tr.blocks_small = plans[i].split ? trid::varlen_blocks(p, small) : 0;
                tr.pred_us = pred[i];
                tr.nlong = (int)nlong;
                xs.last_tune.push_back(tr);
            }
            for (size_t ri = 0; ri < ntime; ++ri) {
                const auto &pl = plans[rank[ri]];
                auto *sc = new trid::VarlenSchedule();
                hipError_t e = trid::varlen_build(off, nsys, p, pl.v, sc, pl.split ? &small : nullptr);
                float us = 0.f;
                if (e == hipSuccess) e = time_schedule(*sc, a, b, c, d, xt, st, &us);
                if (e != hipSuccess) {
                    trid::varlen_free(sc);
                    delete sc;
                    if (best) {
                        trid::varlen_free(best);
                        delete best;
                    }
                    return trid::handle_hip_fail(h, e, "uneven batch: autotune");
                }
                sc->tuned_us = us;
                xs.last_tune[ri].meas_us = us;
                if (!best || us < best->tuned_us) {
                    if (best) {
                        trid::varlen_free(best);
                        delete best;
                    }
                    best = sc;
                    best_split = pl.split;
                } else {
                    trid::varlen_free(sc);
                    delete sc;
                }
            }
            xs.tuned[pkey] = {best->M, best->NT, best->thomas, best->wave};
            if (best_split)
                xs.tuned[pkey + "/small"] = {small.M, small.NT, small.thomas};
            else
                xs.tuned.erase(pkey + "/small");
        } else {
            trid::VarlenVariant v = cands.front();
            if (tuned != xs.tuned.end())
                for (const auto &c2 : cands)
                    if (c2.M == tuned->second.M && c2.NT == tuned->second.NT && c2.thomas == tuned->second.thomas &&
                        c2.wave == tuned->second.wave)
                        v = c2;
            const bool split = tuned_small != xs.tuned.end() && tuned_small->second.M == small.M &&
                               tuned_small->second.NT == small.NT && maxlen > (int64_t)small.M * small.NT;
            best = new trid::VarlenSchedule();
            hipError_t e = trid::varlen_build(off, nsys, p, v, best, split ? &small : nullptr);
            if (e != hipSuccess) {
                trid::varlen_free(best);
                delete best;
                return trid::handle_hip_fail(h, e, "uneven batch: schedule");
            }
        }
        // an evicted schedule may still be in use by work on the stream
        found = xs.varlen.insert(skey, best, [&](const std::string &, trid::VarlenSchedule *old) {
            (void)hipStreamSynchronize(st);
            trid::varlen_free(old);
            delete old;
        });
    }
    trid::VarlenSchedule &sc = **found;
    // With the kernel timer on, a schedule of one persistent launch runs
    // directly, so that its dispatch stamps the kernel's own start and end
    // (events around a graph launch would also count the launch latency).
    if (xs.timer.on && sc.nitems > 0 && !sc.next && sc.long_off.empty()) {
        hipError_t e = xs.timer.time("varlen", st, [&] { return trid::varlen_launch(sc, a, b, c, d, x, st); });
        if (e != hipSuccess) return trid::handle_hip_fail(h, e, "uneven batch: launch");
        return TRID_OK;
    }
    // one persistent launch, replayed from a captured graph per (pointers, stream)
    const trid::VarlenSchedule::GraphKey gkey = std::make_tuple(a, b, c, d, x, st);
    hipGraphExec_t *git = sc.graphs.find(gkey);
    hipError_t e;
    if (!git) {
        if (!xs.capture_stream) {
            e = hipStreamCreateWithFlags(&xs.capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                xs.capture_stream = nullptr;
                return trid::handle_hip_fail(h, e, "hipStreamCreate");
            }
        }
        e = hipStreamBeginCapture(xs.capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return trid::handle_hip_fail(h, e, "hipStreamBeginCapture");
        hipError_t el = trid::varlen_launch(sc, a, b, c, d, x, xs.capture_stream);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(xs.capture_stream, &graph);
        if (el != hipSuccess || e != hipSuccess) {
            if (graph) hipGraphDestroy(graph);
            return trid::handle_hip_fail(h, el != hipSuccess ? el : e, "uneven batch: capture");
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return trid::handle_hip_fail(h, e, "hipGraphInstantiate");
        git = sc.graphs.insert(gkey, exec, [](const trid::VarlenSchedule::GraphKey &k, hipGraphExec_t g) {
            trid::destroy_graph_exec(g, std::get<5>(k));
        });
    }
    e = xs.timer.time_recorded("varlen", st, [&] { return hipGraphLaunch(*git, st); });
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "uneven batch: launch");
    return TRID_OK;
}

int trid_gtsv_varlen_dev(trid_handle_t h, trid_prec_t prec, const void *a, const void *b, const void *c,
                         const void *d, void *x, const int64_t *offsets_dev, int64_t nsys) {
    if (!h) return TRID_ERR_ARG;
    if (!offsets_dev) return trid::handle_fail(h, TRID_ERR_ARG, "NULL pointer");
    if (nsys < 1 || nsys > ((int64_t)1 << 30)) return trid::handle_fail(h, TRID_ERR_ARG, "nsys out of range");
    if (prec != TRID_PREC_F64 && prec != TRID_PREC_F32 && prec != TRID_PREC_F32_REFINE64)
        return trid::handle_fail(h, TRID_ERR_ARG, "bad precision");
    if (!a || !b || !c || !d || !x) return trid::handle_fail(h, TRID_ERR_ARG, "NULL pointer");
    // the schedule is built and looked up on the host: read the offsets after
    // the work already enqueued on the stream (which may have written them)
    std::vector<int64_t> off((size_t)nsys + 1);
    hipStream_t st = trid::handle_stream(h);
    hipError_t e = hipMemcpyAsync(off.data(), offsets_dev, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "uneven batch: reading the offsets");
    return trid_gtsv_varlen(h, prec, a, b, c, d, x, off.data(), nsys);
}

int trid_cache_report(trid_handle_t h, char *buf, size_t len) {
    if (!h) return TRID_ERR_ARG;
    if (!buf || len < 2) return trid::handle_fail(h, TRID_ERR_ARG, "buffer too small");
    trid::ExtState &xs = trid::handle_ext(h);
    size_t vgraphs = 0;
    xs.varlen.for_each([&](const std::string &, trid::VarlenSchedule *sc) { vgraphs += sc->graphs.size(); });
    char out[320];
    const int nw = snprintf(out, sizeof out,
                            "{\"adi_graphs\": %zu, \"adi_graph_cap\": %zu, \"varlen_schedules\": %zu, "
                            "\"varlen_schedule_cap\": %zu, \"varlen_graphs\": %zu, \"varlen_graph_cap\": %zu}",
                            trid::handle_adi_graphs(h), trid::handle_adi_graph_cap(), xs.varlen.size(), xs.varlen.cap,
                            vgraphs, trid::VarlenSchedule().graphs.cap);
    if (nw < 0 || (size_t)nw + 1 > len) return trid::handle_fail(h, TRID_ERR_ARG, "buffer too small");
    std::memcpy(buf, out, (size_t)nw + 1);
    return TRID_OK;
}

}  // extern "C"

namespace {

struct AdiGeom {
    bool f64;
    int ndim;
    trid::i64 inner[3], n[3], outer[3];
    trid::i64 nx, ny, nz, batch;
    size_t bytes;  // one mesh-sized array
};

// Shared argument checks of the per-point-s ADI entry points beyond the plain step.
int adi_geom(trid_handle_t h, trid_dtype_t dt, int ndim, const int64_t *dims, int64_t batch, AdiGeom *g) {
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (ndim != 2 && ndim != 3) return trid::handle_fail(h, TRID_ERR_ARG, "ADI needs ndim 2 or 3");
    for (int ax = 0; ax < ndim; ++ax) {
        int rc = trid::handle_check_mesh(h, ndim, dims, ax, batch, &g->inner[ax], &g->n[ax], &g->outer[ax]);
        if (rc) return rc;
    }
    g->f64 = dt == TRID_F64;
    g->ndim = ndim;
    g->nx = dims[0];
    g->ny = dims[1];
    g->nz = ndim == 3 ? dims[2] : 1;
    g->batch = batch;
    g->bytes = (size_t)(g->nx * g->ny * g->nz * batch) * (g->f64 ? 8 : 4);
    return TRID_OK;
}

// Forward pieces of one step with per-point s: W1 = X^{-1} (2 s L u) and the
// line solves after it.  keep_u: NULL -> W[k+1] = A_k^{-1} W[k] for every axis
// (the recompute of the reverse pass); non-NULL -> the last solve also does
// u += W[ndim] (the step itself, intermediates kept).
int adi_forward_parts(trid_handle_t h, const AdiGeom &g, const void *u, const void *s, void *const W[4],
                      void *keep_u, const char *names[3]) {
    trid::ExtState &x = trid::handle_ext(h);
    hipStream_t st = trid::handle_stream(h);
    std::string msg;
    trid::AdiReq ar;
    ar.f64 = g.f64;
    ar.ndim = g.ndim;
    ar.u = u;
    ar.s = s;
    ar.d = W[1];
    ar.nx = g.nx;
    ar.ny = g.ny;
    ar.nz = g.nz;
    ar.batch = g.batch;
    trid::LinePlan pl;
    if (!trid::plan_rhs_x(ar, &pl, &msg)) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
    hipError_t e = x.timer.time(names[0], st, [&] { return trid::launch_rhs_x(ar, pl, st); });
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI: stencil + x launch");
    for (int k = 1; k < g.ndim; ++k) {
        trid::LineReq r;
        r.f64 = g.f64;
        r.mode = trid::Mode::S;
        r.s = s;
        r.d = W[k];
        const bool last = k == g.ndim - 1;
        if (keep_u && last) {
            r.out = trid::Out::AddKeep;
            r.x = keep_u;
            r.x2 = W[k + 1];
        } else {
            r.out = trid::Out::Store;
            r.x = W[k + 1];
        }
        r.inner = g.inner[k];
        r.n = g.n[k];
        r.outer = g.outer[k];
        if (!trid::plan_lines(r, &pl, &msg)) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
        e = x.timer.time(names[k], st, [&] { return trid::launch_lines(r, pl, st); });
        if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI: line-solve launch");
    }
    return TRID_OK;
}

// Reverse sweep of one step given its intermediates W[1..ndim] and scratch W[4]:
// lambda = A_k^{-T} lambda (z, y, x), sbar += lambda * second difference of
// W[k+1], then the stencil adjoint into u_bar and s_bar.
int adi_reverse(trid_handle_t h, const AdiGeom &g, const void *u_t, const void *s, void *const W[5], void *u_bar,
                void *s_bar) {
    trid::ExtState &x = trid::handle_ext(h);
    hipStream_t st = trid::handle_stream(h);
    std::string msg;
    trid::LinePlan pl;
    hipError_t e;
    for (int k = g.ndim - 1; k >= 0; --k) {
        trid::LineReq r;
        r.f64 = g.f64;
        r.mode = trid::Mode::ST;
        r.out = trid::Out::AdjS;
        r.s = s;
        r.xf = W[k + 1];
        r.d = (k == g.ndim - 1) ? u_bar : W[4];
        r.g = W[4];
        r.gs = s_bar;
        r.inner = g.inner[k];
        r.n = g.n[k];
        r.outer = g.outer[k];
        if (!trid::plan_lines(r, &pl, &msg)) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
        e = x.timer.time("adj_solve", st, [&] { return trid::launch_lines(r, pl, st); });
        if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI adjoint: transposed solve launch");
    }
    // lambda is now dLoss/d(rhs): stencil adjoint into u_bar and s_bar
    trid::StencilAdjReq sa;
    sa.f64 = g.f64;
    sa.ndim = g.ndim;
    sa.u = u_t;
    sa.s = s;
    sa.rbar = W[4];
    sa.ubar = u_bar;
    sa.sbar = s_bar;
    sa.nx = g.nx;
    sa.ny = g.ny;
    sa.nz = g.nz;
    sa.batch = g.batch;
    e = x.timer.time("adj_stencil", st, [&] { return trid::launch_stencil_adjoint(sa, st); });
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI adjoint: stencil adjoint launch");
    return TRID_OK;
}

}  // namespace

extern "C" {

int trid_hv_step(trid_handle_t h, trid_dtype_t dt, void *u, const void *a, const void *b, const void *c,
                 double tau, double theta, const int64_t *dims, int64_t batch, int nsteps, unsigned flags) {
    if (!h) return TRID_ERR_ARG;
    if (flags & ~(unsigned)TRID_ADI_STREAM) return trid::handle_fail(h, TRID_ERR_ARG, "unknown flag");
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (!u || !a || !b || !c) return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    if (u == a || u == b || u == c) return trid::handle_fail(h, TRID_ERR_ARG, "u may not alias a, b or c");
    if (nsteps < 0) return trid::handle_fail(h, TRID_ERR_ARG, "nsteps must be >= 0");
    if (!(tau >= 0.0) || !(theta > 0.0) || tau > 1e300 || theta > 1e300)
        return trid::handle_fail(h, TRID_ERR_ARG, "dt must be >= 0 and theta > 0, both finite");
    int64_t inner, n, outer;
    for (int ax = 0; ax < 2; ++ax) {
        int rc = trid::handle_check_mesh(h, 2, dims, ax, batch, &inner, &n, &outer);
        if (rc) return rc;
    }
    if (nsteps == 0) return TRID_OK;
    const bool f64 = dt == TRID_F64;
    const int64_t nx = dims[0], ny = dims[1], pts = nx * ny * batch;
    trid::ExtState &xs = trid::handle_ext(h);
    hipStream_t st = trid::handle_stream(h);
    if (!(flags & TRID_ADI_STREAM)) {  // all steps in one launch, each mesh resident in LDS
        trid::ResidentReq rq;
        rq.f64 = f64;
        rq.u = u;
        rq.nx = nx;
        rq.ny = ny;
        rq.batch = batch;
        rq.nsteps = nsteps;
        rq.hv = true;
        rq.a = a;
        rq.b = b;
        rq.c = c;
        rq.dt = tau;
        rq.theta = theta;
        if (trid::resident_fits(rq)) {
            hipError_t e = xs.timer.time("hv_resident", st, [&] { return trid::launch_resident(rq, st); });
            return e == hipSuccess ? TRID_OK : trid::handle_hip_fail(h, e, "resident HV launch");
        }
    }
    const size_t slot = ((size_t)pts * (f64 ? 8 : 4) + 255) & ~(size_t)255;
    void *ws = nullptr;
    int rc = trid::handle_workspace2(h, 4 * slot, &ws);
    if (rc) return rc;
    char *wb = static_cast<char *>(ws);
    trid::HvReq q;
    q.f64 = f64;
    q.u = u;
    q.r = wb;
    q.z = wb + slot;
    q.sa = wb + 2 * slot;
    q.sb = wb + 3 * slot;
    q.a = a;
    q.b = b;
    q.c = c;
    q.nx = nx;
    q.ny = ny;
    q.batch = batch;
    q.dt = tau;
    q.theta = theta;
    auto pred = [&](int which) {
        hipError_t e = xs.timer.time("hv_pred", st, [&] { return trid::launch_hv_pred(q, which, st); });
        return e == hipSuccess ? TRID_OK : trid::handle_hip_fail(h, e, "predictor launch");
    };
    // the implicit rows (-s, 1 + 2 s, -s): s = theta dt a along x, theta dt b along y
    auto solve = [&](void *d, int axis) {
        trid::LineReq r;
        r.f64 = f64;
        r.mode = trid::Mode::S;
        r.out = trid::Out::Store;
        r.s = axis == 0 ? q.sa : q.sb;
        r.d = d;
        r.x = d;
        r.inner = axis == 0 ? 1 : nx;
        r.n = axis == 0 ? nx : ny;
        r.outer = axis == 0 ? ny * batch : batch;
        return trid::handle_run_lines(h, r);
    };
    if ((rc = pred(4))) return rc;
    for (int it = 0; it < nsteps; ++it) {
        if ((rc = pred(0)) || (rc = solve(q.r, 0)) || (rc = pred(1)) || (rc = solve(q.r, 1)) ||
            (rc = pred(2)) || (rc = solve(q.z, 0)) || (rc = pred(3)) || (rc = solve(u, 1)))
            return rc;
    }
    return TRID_OK;
}

int trid_adi_step_adjoint(trid_handle_t h, trid_dtype_t dt, const void *u_t, const void *s, double s0, void *u_bar,
                          void *s_bar, int ndim, const int64_t *dims, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (!u_t || !u_bar) return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    if (!s && !(std::fabs(s0) <= 1e300)) return trid::handle_fail(h, TRID_ERR_ARG, "s0 must be finite");
    AdiGeom g;
    int rc = adi_geom(h, dt, ndim, dims, batch, &g);
    if (rc) return rc;
    const size_t slot = (g.bytes + 255) & ~(size_t)255;
    // W[1..3]: forward outputs, W[4]: lambda, then the constant s (s NULL) and
    // the discarded s gradient (s_bar NULL)
    const int nslots = 4 + (s ? 0 : 1) + (s_bar ? 0 : 1);
    void *ws = nullptr;
    rc = trid::handle_workspace2(h, nslots * slot, &ws);
    if (rc) return rc;
    char *wb = static_cast<char *>(ws);
    void *W[5] = {nullptr, wb, wb + slot, wb + 2 * slot, wb + 3 * slot};
    int next = 4;
    if (!s) {
        // the constant diffusion number as a per-point array: the reverse pass
        // then returns dL/ds_i at s = s0 for every point (their sum is dL/ds0)
        void *sc = wb + (next++) * slot;
        const trid::i64 pts = g.nx * g.ny * g.nz * g.batch;
        hipError_t e = trid::handle_ext(h).timer.time("adj_fill_s", trid::handle_stream(h), [&] {
            return trid::launch_fill(sc, g.f64, s0, pts, trid::handle_stream(h));
        });
        if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI adjoint: fill launch");
        s = sc;
    }
    if (!s_bar) s_bar = wb + (next++) * slot;
    // recompute the forward step from the checkpoint: W1 = X^-1 (2 s L u_t), W[k+1] = A_k^-1 W[k]
    const char *names[3] = {"adj_rhs_x", "adj_fwd_solve", "adj_fwd_solve"};
    rc = adi_forward_parts(h, g, u_t, s, W, nullptr, names);
    if (rc) return rc;
    return adi_reverse(h, g, u_t, s, W, u_bar, s_bar);
}

int trid_adi_step_keep(trid_handle_t h, trid_dtype_t dt, void *u, const void *s, int ndim, const int64_t *dims,
                       int64_t batch, void *w1, void *w2, void *w3) {
    if (!h) return TRID_ERR_ARG;
    if (!u || !s || !w1 || !w2 || (ndim == 3 && !w3)) return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    AdiGeom g;
    int rc = adi_geom(h, dt, ndim, dims, batch, &g);
    if (rc) return rc;
    if (w1 == u || w2 == u || w1 == w2 || (ndim == 3 && (w3 == u || w3 == w1 || w3 == w2)))
        return trid::handle_fail(h, TRID_ERR_ARG, "u, w1, w2 and w3 must be distinct arrays");
    void *W[4] = {nullptr, w1, w2, w3};
    const char *names[3] = {"keep_rhs_x", "keep_y", "keep_z"};
    return adi_forward_parts(h, g, u, s, W, u, names);
}

int trid_adi_step_adjoint_kept(trid_handle_t h, trid_dtype_t dt, const void *u_t, const void *s, const void *w1,
                               const void *w2, const void *w3, void *u_bar, void *s_bar, int ndim,
                               const int64_t *dims, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (!u_t || !s || !w1 || !w2 || (ndim == 3 && !w3) || !u_bar || !s_bar)
        return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    AdiGeom g;
    int rc = adi_geom(h, dt, ndim, dims, batch, &g);
    if (rc) return rc;
    void *ws = nullptr;
    rc = trid::handle_workspace2(h, g.bytes, &ws);  // lambda only
    if (rc) return rc;
    void *W[5] = {nullptr, const_cast<void *>(w1), const_cast<void *>(w2), const_cast<void *>(w3), ws};
    return adi_reverse(h, g, u_t, s, W, u_bar, s_bar);
}

int trid_model_gtsv(trid_handle_t h, trid_dtype_t dt, int form, int ndim, const int64_t *dims, int axis,
                    int64_t batch, double *us, char *json, size_t len) {
    if (!h) return TRID_ERR_ARG;
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (form != TRID_FORM_ARRAYS && form != TRID_FORM_S) return trid::handle_fail(h, TRID_ERR_ARG, "bad form");
    if (!us) return trid::handle_fail(h, TRID_ERR_ARG, "us is NULL");
    trid::LineReq r;
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer);
    if (rc) return rc;
    r.f64 = dt == TRID_F64;
    r.mode = form == TRID_FORM_S ? trid::Mode::S : trid::Mode::Arrays;
    r.out = trid::Out::Store;
    trid::handle_ext(h).apply_overrides(&r);
    trid::LinePlan pl;
    std::string msg;
    if (!trid::plan_lines(r, &pl, &msg)) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
    const trid::ModelTerms t = trid::model_lines(r, pl);
    *us = t.us;
    if (json && len) {
        snprintf(json, len,
                 "{\"kernel\": \"%s\", \"M\": %d, \"L\": %d, \"P\": %d, \"threads\": %d, \"nblocks\": %lld, "
                 "\"shmem\": %zu, \"bytes\": %.0f, \"t_bytes_us\": %.3f, \"t_lat_us\": %.3f, \"rounds\": %.0f, "
                 "\"per_cu\": %d, \"us\": %.3f}",
                 pl.staged ? "staged" : "strided", pl.M, pl.L, pl.P, pl.threads(), (long long)pl.nblocks, pl.shmem,
                 t.bytes, t.t_bytes, t.t_lat, t.rounds, t.per_cu, t.us);
    }
    return TRID_OK;
}

namespace {

int model_report(trid_handle_t h, const std::vector<trid::KernelPred> &ks, double *us, char *json, size_t len) {
    double total = 0;
    for (const auto &k : ks) total += k.us;
    *us = total;
    if (json && len) {
        std::ostringstream o;
        char item[320];
        snprintf(item, sizeof item, "{\"us\": %.3f, \"kernels\": [", total);
        o << item;
        for (size_t i = 0; i < ks.size(); ++i) {
            snprintf(item, sizeof item,
                     "%s{\"name\": \"%s\", \"class\": \"%s\", \"us\": %.3f, \"launches\": %d, "
                     "\"bytes\": %.0f, \"rounds\": %.0f, \"units\": %.3f}",
                     i ? ", " : "", ks[i].name.c_str(), ks[i].cls.c_str(), ks[i].us, ks[i].launches, ks[i].bytes,
                     ks[i].rounds, ks[i].units);
            o << item;
        }
        o << "]}";
        const std::string txt = o.str();
        if (txt.size() + 1 > len) return trid::handle_fail(h, TRID_ERR_ARG, "json buffer too small");
        memcpy(json, txt.c_str(), txt.size() + 1);
    }
    return TRID_OK;
}

}  // namespace

int trid_model_adi(trid_handle_t h, trid_dtype_t dt, int ndim, const int64_t *dims, int64_t batch, int per_point_s,
                   int nsteps, unsigned flags, double *us, char *json, size_t len) {
    if (!h) return TRID_ERR_ARG;
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (ndim != 2 && ndim != 3) return trid::handle_fail(h, TRID_ERR_ARG, "ADI needs ndim 2 or 3");
    if (!us) return trid::handle_fail(h, TRID_ERR_ARG, "us is NULL");
    if (nsteps < 0) return trid::handle_fail(h, TRID_ERR_ARG, "nsteps must be >= 0");
    if (flags & ~(TRID_ADI_GRAPH | TRID_ADI_STREAM)) return trid::handle_fail(h, TRID_ERR_ARG, "unknown flags");
    int64_t inner, n, outer;
    for (int ax = 0; ax < ndim; ++ax) {
        int rc = trid::handle_check_mesh(h, ndim, dims, ax, batch, &inner, &n, &outer, false);
        if (rc) return rc;
    }
    // 16-byte aligned stand-ins: the plans depend on the arrays' alignment only
    alignas(16) static const double pad[2] = {0, 0};
    trid::AdiReq r;
    r.f64 = dt == TRID_F64;
    r.ndim = ndim;
    r.u = pad;
    r.d = const_cast<double *>(pad);
    r.s = per_point_s ? pad : nullptr;
    r.s0 = 0.2;
    r.nx = dims[0];
    r.ny = dims[1];
    r.nz = ndim == 3 ? dims[2] : 1;
    r.batch = batch;
    trid::handle_ext(h).apply_adi_overrides(&r);
    std::vector<trid::KernelPred> ks;
    std::string msg;
    if (!trid::model_adi(r, nsteps, (flags & TRID_ADI_STREAM) != 0, &ks, &msg))
        return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
    return model_report(h, ks, us, json, len);
}

int trid_model_hv(trid_handle_t h, trid_dtype_t dt, const int64_t *dims, int64_t batch, int nsteps, unsigned flags,
                  double *us, char *json, size_t len) {
    if (!h) return TRID_ERR_ARG;
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (!us) return trid::handle_fail(h, TRID_ERR_ARG, "us is NULL");
    if (nsteps < 0) return trid::handle_fail(h, TRID_ERR_ARG, "nsteps must be >= 0");
    if (flags & ~(TRID_ADI_GRAPH | TRID_ADI_STREAM)) return trid::handle_fail(h, TRID_ERR_ARG, "unknown flags");
    int64_t inner, n, outer;
    for (int ax = 0; ax < 2; ++ax) {
        int rc = trid::handle_check_mesh(h, 2, dims, ax, batch, &inner, &n, &outer, false);
        if (rc) return rc;
    }
    std::vector<trid::KernelPred> ks;
    std::string msg;
    if (!trid::model_hv(dt == TRID_F64, dims[0], dims[1], batch, nsteps, (flags & TRID_ADI_STREAM) != 0, &ks, &msg))
        return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
    return model_report(h, ks, us, json, len);
}

int trid_resident_layout(trid_handle_t h, trid_dtype_t dt, int64_t nx, int64_t ny, int hv, int per_point_s,
                         int force_M, int64_t *out, int len) {
    if (!h) return TRID_ERR_ARG;
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (!out || len < 10) return trid::handle_fail(h, TRID_ERR_ARG, "out needs 10 entries");
    if (force_M != 0 && force_M != 8 && force_M != 10 && force_M != 12 && force_M != 14)
        return trid::handle_fail(h, TRID_ERR_ARG, "tile rows must be 0, 8, 10, 12 or 14");
    trid::ResidentReq r;
    r.f64 = dt == TRID_F64;
    r.nx = nx;
    r.ny = ny;
    r.hv = hv != 0;
    static const char one = 0;  // a non-NULL marker: the layout depends on whether s varies per point
    r.s = (per_point_s && !r.hv) ? &one : nullptr;
    if (!trid::resident_layout(r, force_M, out))
        return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, "no resident layout for this mesh and tile size");
    return TRID_OK;
}

int trid_autotune_report(trid_handle_t h, char *buf, size_t len) {
    if (!h) return TRID_ERR_ARG;
    if (!buf || len < 3) return trid::handle_fail(h, TRID_ERR_ARG, "buffer too small");
    const auto &rec = trid::handle_ext(h).last_tune;
    std::ostringstream o;
    o << "[";
    char item[256];
    for (size_t i = 0; i < rec.size(); ++i) {
        snprintf(item, sizeof item,
                 "%s{\"M\": %d, \"NT\": %d, \"reduced\": \"%s\", \"split\": %d, \"blocks\": %d, "
                 "\"blocks_small\": %d, \"long\": %d, \"pred_us\": %.3f, \"meas_us\": %.3f}",
                 i ? ", " : "", rec[i].M, rec[i].NT, rec[i].wave ? "wave" : (rec[i].thomas ? "thomas" : "pcr"),
                 rec[i].split, rec[i].blocks, rec[i].blocks_small, rec[i].nlong, rec[i].pred_us, rec[i].meas_us);
        o << item;
    }
    o << "]";
    const std::string out = o.str();
    if (out.size() + 1 > len) return trid::handle_fail(h, TRID_ERR_ARG, "buffer too small");
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return TRID_OK;
}

static std::string device_arch() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

int trid_plan_save(trid_handle_t h, const char *path) {
    if (!h) return TRID_ERR_ARG;
    if (!path) return trid::handle_fail(h, TRID_ERR_ARG, "path is NULL");
    std::ofstream f(path);
    if (!f) return trid::handle_fail(h, TRID_ERR_ARG, std::string("cannot write ") + path);
    trid::ExtState &x = trid::handle_ext(h);
    f << "{\n \"arch\": \"" << device_arch() << "\",\n \"plans\": {\n";
    size_t i = 0;
    for (auto &kv : x.tuned) {
        f << "  \"" << kv.first << "\": {\"M\": " << kv.second.M << ", \"NT\": " << kv.second.NT
          << ", \"reduced\": \"" << (kv.second.wave ? "wave" : (kv.second.thomas ? "thomas" : "pcr")) << "\"}"
          << (++i < x.tuned.size() ? "," : "") << "\n";
    }
    f << " }\n}\n";
    return f.good() ? TRID_OK : trid::handle_fail(h, TRID_ERR_ARG, "write failed");
}

int trid_plan_load(trid_handle_t h, const char *path) {
    if (!h) return TRID_ERR_ARG;
    if (!path) return trid::handle_fail(h, TRID_ERR_ARG, "path is NULL");
    std::ifstream f(path);
    if (!f) return trid::handle_fail(h, TRID_ERR_ARG, std::string("cannot read ") + path);
    trid::ExtState &x = trid::handle_ext(h);
    std::string line;
    while (std::getline(f, line)) {
        const size_t mpos = line.find("\"M\":"), npos = line.find("\"NT\":");
        const size_t q0 = line.find('"'), q1 = q0 == std::string::npos ? q0 : line.find('"', q0 + 1);
        if (mpos == std::string::npos || npos == std::string::npos || q1 == std::string::npos) continue;
        const std::string key = line.substr(q0 + 1, q1 - q0 - 1);
        const int M = std::atoi(line.c_str() + mpos + 4), NT = std::atoi(line.c_str() + npos + 5);
        // "reduced": "thomas" selects the Thomas reduced solve, "wave" the
        // wavefront-level kernels (absent: PCR across the work item)
        const int thomas = line.find("\"thomas\"") != std::string::npos ? 1 : 0;
        const int wave = line.find("\"wave\"") != std::string::npos ? 1 : 0;
        if (key.rfind("varlen/", 0) != 0 || M <= 0 || NT <= 0) continue;  // unknown keys are ignored
        x.tuned[key] = {M, NT, thomas, wave};
    }
    return TRID_OK;
}

}  // extern "C"
