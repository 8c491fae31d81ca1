// long_ext.hpp -- refinement and adjoint solves on contiguous lines longer
// than one workgroup holds: pointwise passes (k_long_ext.hip) around the
// chunked solve (k_long.hip).
#pragma once

#include <string>

#include "dispatch.hpp"

namespace trid {

hipError_t launch_to_f32(const void *d, bool d_f64, float *o, i64 N, hipStream_t s);
hipError_t launch_residual32(const float *a, const float *b, const float *c, const float *sv, const void *d,
                             bool d_f64, const float *x, float *r, i64 n, i64 N, hipStream_t s);
hipError_t launch_sum64(const float *x, const float *dx, double *o, i64 N, hipStream_t s);
hipError_t launch_transpose_rows(bool f64, const void *a, const void *b, const void *c, const void *sv, void *at,
                                 void *bt, void *ct, i64 n, i64 N, hipStream_t s);
hipError_t launch_adj_grads(bool f64, const void *lam, const void *x, void *ga, void *gb, void *gc, void *gs, i64 n,
                            i64 N, hipStream_t s);

// FP32 bulk solve + one FP64 refinement sweep of `lines` contiguous lines of n
// rows: FP32 rows from a, b, c (s == NULL) or s; d (FP64 or FP32) read only;
// x (FP64) written.
struct LongRefineReq {
    const float *a = nullptr, *b = nullptr, *c = nullptr, *s = nullptr;
    const void *d = nullptr;
    bool d_f64 = true;
    double *x = nullptr;
    i64 n = 0, lines = 0;
};
size_t long_refine_workspace(i64 n, i64 lines);
hipError_t launch_long_refine(const LongRefineReq &r, void *ws, hipStream_t s, std::string *err);

// Adjoint of `lines` contiguous lines of n rows (arrays form, or s form when
// s != NULL): g IN/OUT (dL/dx in, lambda = A^{-T} g out); arrays form writes
// ga, gb, gc, s form accumulates into gs.
struct LongAdjReq {
    bool f64 = true;
    const void *a = nullptr, *b = nullptr, *c = nullptr, *s = nullptr, *x = nullptr;
    void *g = nullptr, *ga = nullptr, *gb = nullptr, *gc = nullptr, *gs = nullptr;
    i64 n = 0, lines = 0;
};
size_t long_adjoint_workspace(bool f64, i64 n, i64 lines);
hipError_t launch_long_adjoint(const LongAdjReq &r, void *ws, hipStream_t s, std::string *err);

}  // namespace trid
