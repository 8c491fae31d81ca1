// api_ext.cpp -- extern "C" entry points beyond the plain solves: tile-plan
// control, line-solve adjoints, and the entry points not yet available on this
// build (which return TRID_ERR_UNSUPPORTED).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/trid.h"
#include "dispatch.hpp"
#include "ext.hpp"
#include "refine.hpp"

namespace trid {

void ExtState::release() {
    timer.release();
    if (ws2) hipFree(ws2);
    ws2 = nullptr;
    ws2_bytes = 0;
}

int handle_workspace2(trid_handle_t h, size_t bytes, void **ptr) {
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

int trid_gtsv_batched_adjoint(trid_handle_t h, trid_dtype_t dt, const void *a, const void *b,
                              const void *c, const void *x, void *g, void *ga, void *gb, void *gc,
                              int ndim, const int64_t *dims, int axis, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (!a || !b || !c || !x || !g || !ga || !gb || !gc)
        return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    trid::LineReq r;
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer);
    if (rc) return rc;
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
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer);
    if (rc) return rc;
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
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer);
    if (rc) return rc;
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
    int rc = trid::handle_check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer);
    if (rc) return rc;
    r.smode = true;
    r.d_f64 = d_dt == TRID_F64;
    r.src.s = s;
    r.d = d;
    r.x = x;
    return run_refine(h, r, "refine launch");
}

int trid_gtsv_varlen(trid_handle_t h, trid_prec_t, const void *, const void *, const void *,
                     const void *, void *, const int64_t *, int64_t) {
    return h ? trid::handle_fail(h, TRID_ERR_UNSUPPORTED, "varlen: not in this build") : TRID_ERR_ARG;
}

int trid_adi_step_adjoint(trid_handle_t h, trid_dtype_t dt, const void *u_t, const void *s, void *u_bar,
                          void *s_bar, int ndim, const int64_t *dims, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (dt != TRID_F32 && dt != TRID_F64) return trid::handle_fail(h, TRID_ERR_ARG, "bad dtype");
    if (!u_t || !s || !u_bar || !s_bar) return trid::handle_fail(h, TRID_ERR_ARG, "NULL data pointer");
    if (ndim != 2 && ndim != 3) return trid::handle_fail(h, TRID_ERR_ARG, "ADI needs ndim 2 or 3");
    trid::i64 inner[3], n[3], outer[3];
    for (int ax = 0; ax < ndim; ++ax) {
        int rc = trid::handle_check_mesh(h, ndim, dims, ax, batch, &inner[ax], &n[ax], &outer[ax]);
        if (rc) return rc;
    }
    const bool f64 = dt == TRID_F64;
    const trid::i64 nx = dims[0], ny = dims[1], nz = ndim == 3 ? dims[2] : 1;
    const size_t bytes = (size_t)(nx * ny * nz * batch) * (f64 ? 8 : 4);
    const size_t slot = (bytes + 255) & ~(size_t)255;
    void *ws = nullptr;
    int rc = trid::handle_workspace2(h, 4 * slot, &ws);
    if (rc) return rc;
    char *wb = static_cast<char *>(ws);
    void *W[5] = {nullptr, wb, wb + slot, wb + 2 * slot, wb + 3 * slot};  // W[1..3]: forward outputs, W[4]: lambda
    trid::ExtState &x = trid::handle_ext(h);
    hipStream_t st = trid::handle_stream(h);
    std::string msg;
    // recompute the forward step from the checkpoint: W1 = X^-1 (2 s L u_t), W[k+1] = A_k^-1 W[k]
    trid::AdiReq ar;
    ar.f64 = f64;
    ar.ndim = ndim;
    ar.u = u_t;
    ar.s = s;
    ar.d = W[1];
    ar.nx = nx;
    ar.ny = ny;
    ar.nz = nz;
    ar.batch = batch;
    trid::LinePlan pl;
    if (!trid::plan_rhs_x(ar, &pl, &msg)) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
    hipError_t e = x.timer.time("adj_rhs_x", st, [&] { return trid::launch_rhs_x(ar, pl, st); });
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI adjoint: stencil + x launch");
    for (int k = 1; k < ndim; ++k) {
        trid::LineReq r;
        r.f64 = f64;
        r.mode = trid::Mode::S;
        r.out = trid::Out::Store;
        r.s = s;
        r.d = W[k];
        r.x = W[k + 1];
        r.inner = inner[k];
        r.n = n[k];
        r.outer = outer[k];
        if (!trid::plan_lines(r, &pl, &msg)) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
        e = x.timer.time("adj_fwd_solve", st, [&] { return trid::launch_lines(r, pl, st); });
        if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI adjoint: forward solve launch");
    }
    // reverse sweep: lambda = A_k^-T lambda, sbar += lambda * (second difference of A_k's output)
    for (int k = ndim - 1; k >= 0; --k) {
        trid::LineReq r;
        r.f64 = f64;
        r.mode = trid::Mode::ST;
        r.out = trid::Out::AdjS;
        r.s = s;
        r.xf = W[k + 1];
        r.d = (k == ndim - 1) ? u_bar : W[4];
        r.g = W[4];
        r.gs = s_bar;
        r.inner = inner[k];
        r.n = n[k];
        r.outer = outer[k];
        if (!trid::plan_lines(r, &pl, &msg)) return trid::handle_fail(h, TRID_ERR_UNSUPPORTED, msg);
        e = x.timer.time("adj_solve", st, [&] { return trid::launch_lines(r, pl, st); });
        if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI adjoint: transposed solve launch");
    }
    // lambda is now dLoss/d(rhs): stencil adjoint into u_bar and s_bar
    trid::StencilAdjReq sa;
    sa.f64 = f64;
    sa.ndim = ndim;
    sa.u = u_t;
    sa.s = s;
    sa.rbar = W[4];
    sa.ubar = u_bar;
    sa.sbar = s_bar;
    sa.nx = nx;
    sa.ny = ny;
    sa.nz = nz;
    sa.batch = batch;
    e = x.timer.time("adj_stencil", st, [&] { return trid::launch_stencil_adjoint(sa, st); });
    if (e != hipSuccess) return trid::handle_hip_fail(h, e, "ADI adjoint: stencil adjoint launch");
    return TRID_OK;
}

int trid_plan_load(trid_handle_t h, const char *) {
    return h ? trid::handle_fail(h, TRID_ERR_UNSUPPORTED, "plan cache: not in this build") : TRID_ERR_ARG;
}

int trid_plan_save(trid_handle_t h, const char *) {
    return h ? trid::handle_fail(h, TRID_ERR_UNSUPPORTED, "plan cache: not in this build") : TRID_ERR_ARG;
}

}  // extern "C"
