// k_long_ext.hip -- pointwise passes that let the refinement and adjoint solves
// run on contiguous lines longer than one workgroup holds, around the chunked
// solve of k_long.hip (Section III-B's tiling one level up).
//
// Refinement (FP32 bulk + one FP64 residual sweep), as separate passes:
//   d32 = fp32(d);  x32 = solve32(A, d32);  r32 = fp32(d - A x32) with the
//   residual in FP64;  dx = solve32(A, r32);  x = x32 + dx in FP64.
// Adjoint: the rows of A^T (sub c_{i-1}, diagonal b_i, super a_{i+1}) are
// written out, lambda = A^{-T} g by the chunked solve, then the coefficient
// gradients pointwise.
// Lines are contiguous: `nlines` lines of n rows, row i of line l at l n + i.
#include <algorithm>

#include "dispatch.hpp"
#include "long_ext.hpp"
#include "tile.hpp"

namespace trid {

namespace {

constexpr int kB = 256;

__device__ __forceinline__ i64 gid() { return (i64)blockIdx.x * kB + threadIdx.x; }

template <typename TD>
__global__ __launch_bounds__(kB) void k_to_f32(const TD *__restrict__ d, float *__restrict__ o, i64 N) {
    const i64 step = (i64)gridDim.x * kB;
    for (i64 i = gid(); i < N; i += step) o[i] = (float)d[i];
}

// Row i of a line as FP64 promotions of the FP32 coefficients (ignored a_0 and
// c_{n-1} are 0): arrays form from a, b, c; s form a = c = -s, b = 1 + 2 s.
struct RowsF32 {
    const float *a, *b, *c, *s;
    __device__ __forceinline__ void row(i64 i, bool first, bool last, double &ra, double &rb, double &rc) const {
        if (s) {
            const double sv = (double)s[i];
            ra = first ? 0.0 : -sv;
            rb = 1.0 + 2.0 * sv;
            rc = last ? 0.0 : -sv;
        } else {
            ra = first ? 0.0 : (double)a[i];
            rb = (double)b[i];
            rc = last ? 0.0 : (double)c[i];
        }
    }
};

template <typename TD>
__global__ __launch_bounds__(kB) void k_residual32(RowsF32 rows, const TD *__restrict__ d, const float *__restrict__ x,
                                                   float *__restrict__ r, i64 n, i64 N) {
    const i64 step = (i64)gridDim.x * kB;
    for (i64 i = gid(); i < N; i += step) {
        const i64 k = i % n;
        const bool first = k == 0, last = k == n - 1;
        double ra, rb, rc;
        rows.row(i, first, last, ra, rb, rc);
        const double xm = first ? 0.0 : (double)x[i - 1];
        const double xp = last ? 0.0 : (double)x[i + 1];
        r[i] = (float)((double)d[i] - (ra * xm + rb * (double)x[i] + rc * xp));
    }
}

__global__ __launch_bounds__(kB) void k_sum64(const float *__restrict__ x, const float *__restrict__ dx,
                                              double *__restrict__ o, i64 N) {
    const i64 step = (i64)gridDim.x * kB;
    for (i64 i = gid(); i < N; i += step) o[i] = (double)x[i] + (double)dx[i];
}

// Rows of A^T: at_i = c_{i-1}, bt_i = b_i, ct_i = a_{i+1} (arrays form; the s
// form's A^T has at_i = -s_{i-1}, bt_i = 1 + 2 s_i, ct_i = -s_{i+1}).
template <typename T>
__global__ __launch_bounds__(kB) void k_transpose_rows(const T *__restrict__ a, const T *__restrict__ b,
                                                       const T *__restrict__ c, const T *__restrict__ s,
                                                       T *__restrict__ at, T *__restrict__ bt, T *__restrict__ ct,
                                                       i64 n, i64 N) {
    const i64 step = (i64)gridDim.x * kB;
    for (i64 i = gid(); i < N; i += step) {
        const i64 k = i % n;
        if (s) {
            at[i] = k > 0 ? -s[i - 1] : T(0);
            bt[i] = T(1) + T(2) * s[i];
            ct[i] = k < n - 1 ? -s[i + 1] : T(0);
        } else {
            at[i] = k > 0 ? c[i - 1] : T(0);
            bt[i] = b[i];
            ct[i] = k < n - 1 ? a[i + 1] : T(0);
        }
    }
}

// Coefficient gradients from lambda and the forward solution x: arrays form
// writes ga = -lambda_i x_{i-1}, gb = -lambda_i x_i, gc = -lambda_i x_{i+1} (0
// for the ignored a_0, c_{n-1}); s form accumulates gs += lambda_i (x_{i-1} -
// 2 x_i + x_{i+1}).
template <typename T>
__global__ __launch_bounds__(kB) void k_adj_grads(const T *__restrict__ lam, const T *__restrict__ x,
                                                  T *__restrict__ ga, T *__restrict__ gb, T *__restrict__ gc,
                                                  T *__restrict__ gs, i64 n, i64 N) {
    const i64 step = (i64)gridDim.x * kB;
    for (i64 i = gid(); i < N; i += step) {
        const i64 k = i % n;
        const T l = lam[i];
        const T xm = k > 0 ? x[i - 1] : T(0), xc = x[i], xp = k < n - 1 ? x[i + 1] : T(0);
        if (gs) {
            gs[i] += l * (xm - T(2) * xc + xp);
        } else {
            ga[i] = -l * xm;
            gb[i] = -l * xc;
            gc[i] = -l * xp;
        }
    }
}

unsigned grid_of(i64 N) { return (unsigned)std::max<i64>(1, std::min<i64>((N + kB - 1) / kB, 1 << 16)); }

}  // namespace

hipError_t launch_to_f32(const void *d, bool d_f64, float *o, i64 N, hipStream_t s) {
    if (d_f64)
        launch(k_to_f32<double>, dim3(grid_of(N)), dim3(kB), 0, s, static_cast<const double *>(d), o, N);
    else
        launch(k_to_f32<float>, dim3(grid_of(N)), dim3(kB), 0, s, static_cast<const float *>(d), o, N);
    return hipGetLastError();
}

hipError_t launch_residual32(const float *a, const float *b, const float *c, const float *sv, const void *d,
                             bool d_f64, const float *x, float *r, i64 n, i64 N, hipStream_t s) {
    RowsF32 rows{a, b, c, sv};
    if (d_f64)
        launch(k_residual32<double>, dim3(grid_of(N)), dim3(kB), 0, s, rows, static_cast<const double *>(d), x, r,
               n, N);
    else
        launch(k_residual32<float>, dim3(grid_of(N)), dim3(kB), 0, s, rows, static_cast<const float *>(d), x, r, n,
               N);
    return hipGetLastError();
}

hipError_t launch_sum64(const float *x, const float *dx, double *o, i64 N, hipStream_t s) {
    launch(k_sum64, dim3(grid_of(N)), dim3(kB), 0, s, x, dx, o, N);
    return hipGetLastError();
}

hipError_t launch_transpose_rows(bool f64, const void *a, const void *b, const void *c, const void *sv, void *at,
                                 void *bt, void *ct, i64 n, i64 N, hipStream_t s) {
    if (f64)
        launch(k_transpose_rows<double>, dim3(grid_of(N)), dim3(kB), 0, s, static_cast<const double *>(a),
               static_cast<const double *>(b), static_cast<const double *>(c), static_cast<const double *>(sv),
               static_cast<double *>(at), static_cast<double *>(bt), static_cast<double *>(ct), n, N);
    else
        launch(k_transpose_rows<float>, dim3(grid_of(N)), dim3(kB), 0, s, static_cast<const float *>(a),
               static_cast<const float *>(b), static_cast<const float *>(c), static_cast<const float *>(sv),
               static_cast<float *>(at), static_cast<float *>(bt), static_cast<float *>(ct), n, N);
    return hipGetLastError();
}

hipError_t launch_adj_grads(bool f64, const void *lam, const void *x, void *ga, void *gb, void *gc, void *gs, i64 n,
                            i64 N, hipStream_t s) {
    if (f64)
        launch(k_adj_grads<double>, dim3(grid_of(N)), dim3(kB), 0, s, static_cast<const double *>(lam),
               static_cast<const double *>(x), static_cast<double *>(ga), static_cast<double *>(gb),
               static_cast<double *>(gc), static_cast<double *>(gs), n, N);
    else
        launch(k_adj_grads<float>, dim3(grid_of(N)), dim3(kB), 0, s, static_cast<const float *>(lam),
               static_cast<const float *>(x), static_cast<float *>(ga), static_cast<float *>(gb),
               static_cast<float *>(gc), static_cast<float *>(gs), n, N);
    return hipGetLastError();
}

}  // namespace trid

// ------------------------------------------------------------ host passes --

#include "long_lines.hpp"

namespace trid {

namespace {

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

LineReq long_req(bool f64, i64 n, i64 lines) {
    LineReq q;
    q.f64 = f64;
    q.out = Out::Store;
    q.inner = 1;
    q.n = n;
    q.outer = lines;
    return q;
}

}  // namespace

size_t long_refine_workspace(i64 n, i64 lines) {
    const LineReq q = long_req(false, n, lines);
    return 2 * up256((size_t)(n * lines) * sizeof(float)) + long_lines_workspace(q);
}

hipError_t launch_long_refine(const LongRefineReq &r, void *ws, hipStream_t s, std::string *err) {
    const i64 N = r.n * r.lines;
    char *wb = static_cast<char *>(ws);
    float *x32 = reinterpret_cast<float *>(wb);
    float *r32 = reinterpret_cast<float *>(wb + up256((size_t)N * sizeof(float)));
    void *lws = wb + 2 * up256((size_t)N * sizeof(float));
    LineReq q = long_req(false, r.n, r.lines);
    if (r.s) {
        q.mode = Mode::S;
        q.s = r.s;
    } else {
        q.mode = Mode::Arrays;
        q.a = r.a;
        q.b = r.b;
        q.c = r.c;
    }
    // x32 = solve32(A, fp32(d))
    const void *d32 = r.d;
    if (r.d_f64) {
        hipError_t e = launch_to_f32(r.d, true, r32, N, s);
        if (e != hipSuccess) return e;
        d32 = r32;
    }
    q.d = d32;
    q.x = x32;
    hipError_t e = launch_long_lines(q, lws, s, err);
    if (e != hipSuccess) return e;
    // r = d - A x32 in FP64, rounded to FP32; dx = solve32(A, r) in place; x = x32 + dx
    e = launch_residual32(r.a, r.b, r.c, r.s, r.d, r.d_f64, x32, r32, r.n, N, s);
    if (e != hipSuccess) return e;
    q.d = r32;
    q.x = r32;
    e = launch_long_lines(q, lws, s, err);
    if (e != hipSuccess) return e;
    return launch_sum64(x32, r32, r.x, N, s);
}

size_t long_adjoint_workspace(bool f64, i64 n, i64 lines) {
    const LineReq q = long_req(f64, n, lines);
    return 3 * up256((size_t)(n * lines) * (f64 ? 8 : 4)) + long_lines_workspace(q);
}

hipError_t launch_long_adjoint(const LongAdjReq &r, void *ws, hipStream_t s, std::string *err) {
    const i64 N = r.n * r.lines;
    const size_t slot = up256((size_t)N * (r.f64 ? 8 : 4));
    char *wb = static_cast<char *>(ws);
    void *at = wb, *bt = wb + slot, *ct = wb + 2 * slot, *lws = wb + 3 * slot;
    hipError_t e = launch_transpose_rows(r.f64, r.a, r.b, r.c, r.s, at, bt, ct, r.n, N, s);
    if (e != hipSuccess) return e;
    LineReq q = long_req(r.f64, r.n, r.lines);
    q.mode = Mode::Arrays;
    q.a = at;
    q.b = bt;
    q.c = ct;
    q.d = r.g;
    q.x = r.g;
    e = launch_long_lines(q, lws, s, err);
    if (e != hipSuccess) return e;
    return launch_adj_grads(r.f64, r.g, r.x, r.ga, r.gb, r.gc, r.s ? r.gs : nullptr, r.n, N, s);
}

}  // namespace trid
