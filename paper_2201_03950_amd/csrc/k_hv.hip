// k_hv.hip -- predictor stencils of the synthetic SLV stand-in (Alg. 4's call
// structure: explicit predictors alternating with x- and y-line solves).
//
// The model is u_t = F(u) = a u_xx + b u_yy + c u_xy on 2D meshes (per-point
// a, b, c, unit spacing, zero ghosts), integrated by the Hundsdorfer-Verwer
// ADI scheme with parameter theta.  With F1 = a D_xx, F2 = b D_yy and
// F0 = c D_xy (D_xy: the 4-point cross stencil / 4), one step is
//   pred0: r = U + dt F(U) - theta dt F1(U),  z = U + dt/2 F(U)
//   x solve (s = theta dt a) of r           -> Y1
//   pred1: r = Y1 - theta dt F2(U)
//   y solve (s = theta dt b) of r           -> Y2
//   pred2: z = z + dt/2 F(Y2) - theta dt F1(Y2)
//   x solve of z                             -> W1
//   pred3: u = W1 - theta dt F2(Y2)
//   y solve of u                             -> U_next
// Every predictor is one pass over the mesh; the solves are the batched s-form
// line solves of the library.
#include "dispatch.hpp"
#include "hv.hpp"
#include "tile.hpp"

namespace trid {

namespace {

struct HvGeom {
    int nx, ny;
    i64 total;
    double dt, theta;
};

// The 3 x 3 neighbourhood of point p = (i, j) of its mesh, zero outside
// (branch-free: every load comes from an in-bounds index).
template <typename T>
struct Nbh {
    T c, w, e, s, n, sw, se, nw, ne;
    __device__ __forceinline__ void load(const T *__restrict__ u, i64 p, int i, int j, int nx, int ny) {
        const bool hw = i > 0, he = i < nx - 1, hs = j > 0, hn = j < ny - 1;
        c = u[p];
        w = load_if(u, p - 1, hw, p);
        e = load_if(u, p + 1, he, p);
        s = load_if(u, p - nx, hs, p);
        n = load_if(u, p + nx, hn, p);
        sw = load_if(u, p - 1 - nx, hw && hs, p);
        se = load_if(u, p + 1 - nx, he && hs, p);
        nw = load_if(u, p - 1 + nx, hw && hn, p);
        ne = load_if(u, p + 1 + nx, he && hn, p);
    }
    __device__ __forceinline__ T dxx() const { return w - T(2) * c + e; }
    __device__ __forceinline__ T dyy() const { return s - T(2) * c + n; }
    __device__ __forceinline__ T dxy() const { return (ne - se - nw + sw) * T(0.25); }
};

// which: 0..3 = pred0..pred3; 4 = the solve coefficients sa = theta dt a, sb = theta dt b.
template <typename T, int WHICH>
__global__ __launch_bounds__(256) void k_hv_pred(HvGeom g, T *__restrict__ u, T *__restrict__ r,
                                                 T *__restrict__ z, const T *__restrict__ a,
                                                 const T *__restrict__ b, const T *__restrict__ c,
                                                 T *__restrict__ sa, T *__restrict__ sb) {
    // XCD-contiguous block order: the rows above and below a block's points were
    // read by the neighbouring blocks on the same XCD (its L2)
    const i64 p = xcd_block_id() * blockDim.x + threadIdx.x;
    if (p >= g.total) return;
    const T dt = (T)g.dt, th = (T)g.theta;
    if constexpr (WHICH == 4) {
        sa[p] = th * dt * a[p];
        sb[p] = th * dt * b[p];
        return;
    }
    const i64 row = p / g.nx;
    const int i = (int)(p - row * g.nx), j = (int)(row % g.ny);
    Nbh<T> v;
    if constexpr (WHICH == 0) {  // stencils of U
        v.load(u, p, i, j, g.nx, g.ny);
        const T f1 = a[p] * v.dxx(), f = c[p] * v.dxy() + f1 + b[p] * v.dyy();
        r[p] = v.c + dt * f - th * dt * f1;
        z[p] = v.c + T(0.5) * dt * f;
    } else if constexpr (WHICH == 1) {  // r holds Y1; stencil of U along y
        v.load(u, p, i, j, g.nx, g.ny);
        r[p] = r[p] - th * dt * b[p] * v.dyy();
    } else if constexpr (WHICH == 2) {  // r holds Y2
        v.load(r, p, i, j, g.nx, g.ny);
        const T f1 = a[p] * v.dxx(), f = c[p] * v.dxy() + f1 + b[p] * v.dyy();
        z[p] = z[p] + T(0.5) * dt * f - th * dt * f1;
    } else {  // z holds W1, r holds Y2
        v.load(r, p, i, j, g.nx, g.ny);
        u[p] = z[p] - th * dt * b[p] * v.dyy();
    }
}

template <typename T, int WHICH>
hipError_t go(const HvReq &q, hipStream_t s) {
    HvGeom g;
    g.nx = (int)q.nx;
    g.ny = (int)q.ny;
    g.total = q.nx * q.ny * q.batch;
    g.dt = q.dt;
    g.theta = q.theta;
    const i64 nb = (g.total + 255) / 256;
    launch((k_hv_pred<T, WHICH>), dim3((unsigned)nb), dim3(256), 0, s, g, static_cast<T *>(q.u),
           static_cast<T *>(q.r), static_cast<T *>(q.z), static_cast<const T *>(q.a), static_cast<const T *>(q.b),
           static_cast<const T *>(q.c), static_cast<T *>(q.sa), static_cast<T *>(q.sb));
    return hipGetLastError();
}

template <typename T>
hipError_t go_t(const HvReq &q, int which, hipStream_t s) {
    switch (which) {
        case 0: return go<T, 0>(q, s);
        case 1: return go<T, 1>(q, s);
        case 2: return go<T, 2>(q, s);
        case 3: return go<T, 3>(q, s);
        default: return go<T, 4>(q, s);
    }
}

}  // namespace

hipError_t launch_hv_pred(const HvReq &q, int which, hipStream_t s) {
    if (q.nx * q.ny * q.batch >= ((i64)1 << 31) * 256) return hipErrorInvalidValue;
    return q.f64 ? go_t<double>(q, which, s) : go_t<float>(q, which, s);
}

}  // namespace trid
