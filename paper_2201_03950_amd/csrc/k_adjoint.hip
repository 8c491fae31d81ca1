// k_adjoint.hip -- reverse mode of the ADI right-hand side (Alg. 3, line 2).
// Forward: d = 2 s (L u) with L the 7-point (3D) / 5-point (2D) Laplacian and
// zero values outside the mesh.  Given rbar = dLoss/dd:
//   sbar += 2 rbar (L u)
//   ubar += 2 L (s rbar)        (L is symmetric)
// One thread per mesh point; neighbours are read through the caches.  The
// transposed line solves of the step's reverse pass are the adjoint epilogues of
// the line-solve kernels (lines.hpp).
#include "dispatch.hpp"
#include "tile.hpp"

namespace trid {

template <typename T, int NDIM>
__global__ __launch_bounds__(256) void k_stencil_adjoint(const T *__restrict__ u, const T *__restrict__ s,
                                                         const T *__restrict__ rbar, T *__restrict__ ubar,
                                                         T *__restrict__ sbar, int nx, int ny, int nz, i64 total) {
    const i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const i64 line = q / nx;
    const int i = (int)(q - line * nx);
    const int j = (int)(line % ny);
    const int k = (int)((line / ny) % nz);
    const i64 sy = nx, sz = (i64)nx * ny;
    const T sr = s[q] * rbar[q];
    T lu = -T(2 * NDIM) * u[q];
    T lw = -T(2 * NDIM) * sr;
    auto nb = [&](i64 o) {
        lu += u[o];
        lw += s[o] * rbar[o];
    };
    if (i > 0) nb(q - 1);
    if (i < nx - 1) nb(q + 1);
    if (j > 0) nb(q - sy);
    if (j < ny - 1) nb(q + sy);
    if (NDIM == 3) {
        if (k > 0) nb(q - sz);
        if (k < nz - 1) nb(q + sz);
    }
    sbar[q] += T(2) * rbar[q] * lu;
    ubar[q] += T(2) * lw;
}

namespace {

template <typename T, int NDIM>
hipError_t go(const StencilAdjReq &r, hipStream_t st) {
    const i64 total = r.nx * r.ny * r.nz * r.batch;
    const unsigned nb = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL((k_stencil_adjoint<T, NDIM>), dim3(nb), dim3(256), 0, st, static_cast<const T *>(r.u),
                       static_cast<const T *>(r.s), static_cast<const T *>(r.rbar), static_cast<T *>(r.ubar),
                       static_cast<T *>(r.sbar), (int)r.nx, (int)r.ny, (int)r.nz, total);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_stencil_adjoint(const StencilAdjReq &r, hipStream_t st) {
    if (r.f64) return r.ndim == 3 ? go<double, 3>(r, st) : go<double, 2>(r, st);
    return r.ndim == 3 ? go<float, 3>(r, st) : go<float, 2>(r, st);
}

}  // namespace trid
