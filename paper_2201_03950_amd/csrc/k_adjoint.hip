// k_adjoint.hip -- reverse mode of the ADI step's explicit right-hand side (Alg. 3).
// Forward: d = 2 s (L u) with L the 7-point (3D) / 5-point (2D) Laplacian and
// zero values outside the mesh.  Given rbar = dLoss/dd:
//   sbar += 2 rbar (L u)
//   ubar += 2 L (s rbar)        (L is symmetric)
// One thread per mesh point, one block per chunk of an x line (so the line's
// y/z position is one scalar division per block); neighbours are read through
// the caches with branch-free loads, blocks in XCD-contiguous order.  The transposed line solves of the step's
// reverse pass are the adjoint epilogues of the line-solve kernels (lines.hpp).
#include <algorithm>

#include "dispatch.hpp"
#include "tile.hpp"

namespace trid {

template <typename T, int NDIM>
__global__ __launch_bounds__(256) void k_stencil_adjoint(const T *__restrict__ u, const T *__restrict__ s,
                                                         const T *__restrict__ rbar, T *__restrict__ ubar,
                                                         T *__restrict__ sbar, int nx, int ny, int nz, int cpl) {
    // XCD-contiguous block order: the neighbour lines and planes a block reads
    // were read by the blocks just before it on the same XCD (its L2)
    const i64 b = xcd_block_id();
    const i64 line = b / cpl;  // uniform: scalar unit
    const int i = (int)(b - line * cpl) * (int)blockDim.x + (int)threadIdx.x;
    const int j = (int)(line % ny);
    const int k = (int)((line / ny) % nz);
    const bool v = i < nx;
    const i64 q = line * nx + (v ? i : nx - 1);  // idle lanes stand in for the line's last point
    const i64 sy = nx, sz = (i64)nx * ny;
    const T uq = u[q], rq = rbar[q];
    const T wq = s[q] * rq;
    // neighbours (zero outside the mesh), all loads issued before any use
    const bool ok[6] = {v && i > 0, v && i < nx - 1, j > 0, j < ny - 1, NDIM == 3 && k > 0,
                        NDIM == 3 && k < nz - 1};
    const i64 off[6] = {-1, 1, -sy, sy, -sz, sz};
    T un[6], sn[6], rn[6];
#pragma unroll
    for (int m = 0; m < (NDIM == 3 ? 6 : 4); ++m) {
        un[m] = load_if(u, q + off[m], ok[m], q);
        sn[m] = load_if(s, q + off[m], ok[m], q);
        rn[m] = load_if(rbar, q + off[m], ok[m], q);
    }
    const T sb = sbar[q], ub = ubar[q];
    T lu = -T(2 * NDIM) * uq;
    T lw = -T(2 * NDIM) * wq;
#pragma unroll
    for (int m = 0; m < (NDIM == 3 ? 6 : 4); ++m) {
        lu += un[m];
        lw += sn[m] * rn[m];
    }
    if (v) {
        sbar[q] = sb + T(2) * rq * lu;
        ubar[q] = ub + T(2) * lw;
    }
}

namespace {

template <typename T, int NDIM>
hipError_t go(const StencilAdjReq &r, hipStream_t st) {
    const i64 lines = r.ny * r.nz * r.batch;
    const int bd = (int)std::min<i64>(256, (r.nx + 63) / 64 * 64);
    const int cpl = (int)((r.nx + bd - 1) / bd);
    const i64 nb = lines * cpl;
    if (nb >= ((i64)1 << 31)) return hipErrorInvalidValue;
    launch((k_stencil_adjoint<T, NDIM>), dim3((unsigned)nb), dim3(bd), 0, st,
                       static_cast<const T *>(r.u), static_cast<const T *>(r.s), static_cast<const T *>(r.rbar),
                       static_cast<T *>(r.ubar), static_cast<T *>(r.sbar), (int)r.nx, (int)r.ny, (int)r.nz, cpl);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stencil_adjoint(const StencilAdjReq &r, hipStream_t st) {
    if (r.f64) return r.ndim == 3 ? go<double, 3>(r, st) : go<double, 2>(r, st);
    return r.ndim == 3 ? go<float, 3>(r, st) : go<float, 2>(r, st);
}

// p[0..n) = v (grid-stride loop).
template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *__restrict__ p, T v, i64 n) {
    const i64 step = (i64)gridDim.x * 256;
    for (i64 k = (i64)blockIdx.x * 256 + threadIdx.x; k < n; k += step) p[k] = v;
}

hipError_t launch_fill(void *p, bool f64, double v, i64 n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<i64>((n + 255) / 256, 1 << 16);
    if (f64)
        launch(k_fill<double>, dim3(nb), dim3(256), 0, st, static_cast<double *>(p), v, n);
    else
        launch(k_fill<float>, dim3(nb), dim3(256), 0, st, static_cast<float *>(p), (float)v, n);
    return hipGetLastError();
}

}  // namespace trid
