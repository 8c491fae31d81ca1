// k_resident.hip -- the 2D ADI time loop (Alg. 3) with each mesh resident in
// one workgroup's LDS.
//
// The streamed step moves every mesh through HBM twice per time step.  For the
// small batched meshes of the 2D application (up to 128 x 128 points per mesh,
// thousands of meshes) a mesh fits in LDS, so one workgroup loads it once, runs
// all the time steps on chip and stores it once -- the GPU counterpart of
// keeping the RHS, x-solve and y-solve pipeline on chip and unrolling the time
// loop (Section V, 2D ADI).  Per step:
//   phase A (x lines): thread (y, p) owns tile p of row y, forms d = 2 s L u
//     for its M points from the u array, solves along x (eq. (7) tile sweep,
//     reduced solve by PCR over DPP row shifts, Alg. 2) and stores d;
//   phase B (y lines): thread (x, q) owns tile q of column x, solves d along y
//     and adds the result to u.
// Lines are cut into P tiles of M rows (M = 8, 10, 12 or 14, chosen so that the
// tiles cover the line with the least padding) with P a power of two <= 16
// (rows beyond the mesh are identity rows), so a line's tiles are P adjacent
// lanes.
// LDS holds u, d (and s when it varies per point) with a host-chosen row pitch
// and per-tile skews that spread both phases' accesses over the banks.
// The same layout, tiles and reduced solves serve k_hv_resident, the
// Hundsdorfer-Verwer steps of the SLV stand-in (Alg. 4's call structure).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "resident.hpp"
#include "tile.hpp"

namespace trid {

namespace {

constexpr int kTileRows[4] = {8, 10, 12, 14};
constexpr int kMaxLine = 128;    // 16 tiles of 8 rows
constexpr size_t kLdsBytes = 160 * 1024;

// Threads per workgroup at most: 1024 for 8-row tiles, 512 for longer tiles
// (their registers).
constexpr int max_threads(int M) { return M <= 8 ? 1024 : 512; }

struct ResGeom {
    int nx, ny;
    int m;          // rows per tile
    int px, py;     // tiles per x line and per y line (powers of two)
    int ldx, skw;   // row pitch, extra offset per block of m rows (elements)
    int tp;         // 1: one pad element after every m points of a row
    int region;     // elements per array (multiple of 4)
    int nsteps;
    int cl;         // HV: 2 = a, b, c staged in LDS as three more arrays; 1 = b only
};

// LDS position of point (y, x); M is the tile size (g.m), a constant in kernels.
template <int M>
__host__ __device__ __forceinline__ int res_at(const ResGeom &g, int y, int x) {
    return y * g.ldx + (y / M) * g.skw + x + (g.tp ? (x / M) : 0);
}
__host__ __forceinline__ int res_at_h(const ResGeom &g, int y, int x) {
    return y * g.ldx + (y / g.m) * g.skw + x + (g.tp ? (x / g.m) : 0);
}

// Rows (-s, 1 + 2 s, -s) of one tile along a line of n points starting at
// line position i0; rows past the line's end are identity rows.
template <typename T>
struct SRows {
    const T *sv;
    int i0, n;
    __device__ __forceinline__ void operator()(int k, T &a, T &b, T &c) const {
        const int i = i0 + k;
        const bool v = i < n;
        const T s = sv[k];
        a = (v && i > 0) ? -s : T(0);
        b = v ? T(1) + T(2) * s : T(1);
        c = (v && i < n - 1) ? -s : T(0);
    }
};

// Reduced solve of a line's P tiles in adjacent lanes (P a power of two <= 16).
template <typename T, int M>
__device__ __forceinline__ void dpp_reduced(const TileState<T, M> &ts, int P, int p, T &f, T &lv) {
    switch (P) {
        case 1: reduced_pcr_dpp<T, M, 1>(ts, p, f, lv); return;
        case 2: reduced_pcr_dpp<T, M, 2>(ts, p, f, lv); return;
        case 4: reduced_pcr_dpp<T, M, 4>(ts, p, f, lv); return;
        case 8: reduced_pcr_dpp<T, M, 8>(ts, p, f, lv); return;
        default: reduced_pcr_dpp<T, M, 16>(ts, p, f, lv); return;
    }
}

// Constant rows (s the same at every point): the tile sweep of eq. (7) and the
// PCR of the reduced system (Alg. 2) involve the right-hand side only
// linearly, with multipliers that depend on the tile's position in its line
// alone.  They are computed once per tile position and kept in LDS; a time
// step then applies them to the right-hand side:
//   dp_1 = rr_1 d_1,  dp_k = rr_k d_k - ar_k dp_{k-1}      (forward)
//   dp_k -= cf_k dp_{k+1}                                  (backward, k = M-3..1)
//   fd = d_0 - c0 dp_1;  g = rg fd - far ld_{p-1} - fcr ld_p   (reduced row)
//   g = pr_j g - par_j g_{p-S} - pcr_j g_{p+S}             (PCR level j, S = 2^j)
//   lv = ld - la f - lc f_{p+1};  u_k = dp_k - ap_k f - cp_k lv.
// Field f of tile position p sits at tab[f * P + p]; only the multipliers a
// step uses are kept (M = 8, P = 8: 45 fields).
template <int M>
struct CF {
    static constexpr int rr = -1;              // rr_k, k = 1..M-1
    static constexpr int ar = rr + M - 2;      // ar_k, k = 2..M-1
    static constexpr int cf = ar + M - 1;      // cf_k, k = 1..M-3
    static constexpr int ap = cf + M - 3;      // ap_k, k = 1..M-2
    static constexpr int cp = ap + M - 2;      // cp_k, k = 1..M-2
    static constexpr int c0 = cp + M - 1, rg = c0 + 1, far = c0 + 2, fcr = c0 + 3, la = c0 + 4, lc = c0 + 5;
    static constexpr int lev = c0 + 6;  // level j: pr, par, pcr at lev + 3 j
    static constexpr int fields(int P) {
        int n = lev;
        for (int s = 1; s < P; s <<= 1) n += 3;
        return n;
    }
};
static_assert(CF<8>::rr + 1 == 0 && CF<8>::ar + 2 == 7 && CF<8>::cf + 1 == 13 && CF<8>::ap + 1 == 18 &&
                  CF<8>::cp + 1 == 24 && CF<8>::c0 == 30 && CF<8>::fields(8) == 45,
              "factor table fields are packed");

template <int S, int P, typename T>
__device__ __forceinline__ T lower_masked(T v, int p) {
    const T x = row_from_lower<S>(v);
    return p >= S ? x : T(0);
}
template <int S, int P, typename T>
__device__ __forceinline__ T upper_masked(T v, int p) {
    const T x = row_from_upper<S>(v);
    return p + S < P ? x : T(0);
}

template <typename T, int M, int P, int S = 1, int J = 0>
__device__ __forceinline__ void cf_levels_setup(T *tab, int p, bool wr, T a, T c) {
    if constexpr (S < P) {
        const T am = lower_masked<S, P>(a, p), cm = lower_masked<S, P>(c, p);
        const T an = upper_masked<S, P>(a, p), cn = upper_masked<S, P>(c, p);
        const T r = T(1) / (T(1) - a * cm - c * an);
        if (wr) {
            tab[(CF<M>::lev + 3 * J) * P + p] = r;
            tab[(CF<M>::lev + 3 * J + 1) * P + p] = r * a;
            tab[(CF<M>::lev + 3 * J + 2) * P + p] = r * c;
        }
        cf_levels_setup<T, M, P, 2 * S, J + 1>(tab, p, wr, -r * (a * am), -r * (c * cn));
    }
}

// Factors of tile p of a line of n points with rows (-s, 1 + 2 s, -s); every
// lane of a wavefront calls it (lanes >= P repeat tile positions), lanes < P
// store them.
template <typename T, int M, int P>
__device__ __forceinline__ void cf_setup(T s, int n, int lane, T *tab) {
    const int p = lane % P;
    const bool wr = lane < P;
    T a[M], b[M], c[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int i = p * M + k;
        const bool v = i < n;
        a[k] = (v && i > 0) ? -s : T(0);
        b[k] = v ? T(1) + T(2) * s : T(1);
        c[k] = (v && i < n - 1) ? -s : T(0);
    }
    T ap[M], cp[M], rr[M], ar[M], cf[M];
#pragma unroll
    for (int k = 0; k < M; ++k) rr[k] = ar[k] = cf[k] = ap[k] = cp[k] = T(0);
    rr[1] = T(1) / b[1];
    ap[1] = a[1] * rr[1];
    cp[1] = c[1] * rr[1];
#pragma unroll
    for (int k = 2; k < M; ++k) {
        const T r = T(1) / (b[k] - a[k] * cp[k - 1]);
        rr[k] = r;
        ar[k] = r * a[k];
        ap[k] = -r * a[k] * ap[k - 1];
        cp[k] = r * c[k];
    }
    const T la = ap[M - 1], lc = cp[M - 1];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {
        cf[k] = cp[k];
        ap[k] -= cp[k] * ap[k + 1];
        cp[k] = -cp[k] * cp[k + 1];
    }
    const T fa = a[0], fb = b[0] - c[0] * ap[1], fc = -c[0] * cp[1];
    const T pa = lower_masked<1, P>(la, p), pc = lower_masked<1, P>(lc, p);
    const T rg = T(1) / (fb - fa * pc - fc * la);
    if (wr) {
#pragma unroll
        for (int k = 1; k < M; ++k) tab[(CF<M>::rr + k) * P + p] = rr[k];
#pragma unroll
        for (int k = 2; k < M; ++k) tab[(CF<M>::ar + k) * P + p] = ar[k];
#pragma unroll
        for (int k = 1; k <= M - 3; ++k) tab[(CF<M>::cf + k) * P + p] = cf[k];
#pragma unroll
        for (int k = 1; k <= M - 2; ++k) {
            tab[(CF<M>::ap + k) * P + p] = ap[k];
            tab[(CF<M>::cp + k) * P + p] = cp[k];
        }
        tab[CF<M>::c0 * P + p] = c[0];
        tab[CF<M>::rg * P + p] = rg;
        tab[CF<M>::far * P + p] = fa * rg;
        tab[CF<M>::fcr * P + p] = fc * rg;
        tab[CF<M>::la * P + p] = la;
        tab[CF<M>::lc * P + p] = lc;
    }
    cf_levels_setup<T, M, P>(tab, p, wr, -fa * pa * rg, -fc * lc * rg);
}

template <typename T, int M>
__device__ __forceinline__ void cf_setup_p(T s, int n, int P, int lane, T *tab) {
    switch (P) {
        case 1: cf_setup<T, M, 1>(s, n, lane, tab); return;
        case 2: cf_setup<T, M, 2>(s, n, lane, tab); return;
        case 4: cf_setup<T, M, 4>(s, n, lane, tab); return;
        case 8: cf_setup<T, M, 8>(s, n, lane, tab); return;
        default: cf_setup<T, M, 16>(s, n, lane, tab); return;
    }
}

template <typename T, int M, int P, int S = 1, int J = 0>
__device__ __forceinline__ void cf_levels(const T *tab, int p, T &g) {
    if constexpr (S < P) {
        const T gm = lower_masked<S, P>(g, p), gn = upper_masked<S, P>(g, p);
        g = tab[(CF<M>::lev + 3 * J) * P + p] * g - tab[(CF<M>::lev + 3 * J + 1) * P + p] * gm -
            tab[(CF<M>::lev + 3 * J + 2) * P + p] * gn;
        cf_levels<T, M, P, 2 * S, J + 1>(tab, p, g);
    }
}

template <typename T, int M, int P>
__device__ __forceinline__ void cf_solve(const T *tab, int p, const T (&rd)[M], T (&u)[M]) {
    auto F = [&](int f) { return tab[f * P + p]; };
    T dp[M];
    dp[0] = T(0);
    dp[1] = F(CF<M>::rr + 1) * rd[1];
#pragma unroll
    for (int k = 2; k < M; ++k) dp[k] = F(CF<M>::rr + k) * rd[k] - F(CF<M>::ar + k) * dp[k - 1];
    const T ld = dp[M - 1];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) dp[k] -= F(CF<M>::cf + k) * dp[k + 1];
    const T fd = rd[0] - F(CF<M>::c0) * dp[1];
    const T pd = lower_masked<1, P>(ld, p);
    T g = F(CF<M>::rg) * fd - F(CF<M>::far) * pd - F(CF<M>::fcr) * ld;
    cf_levels<T, M, P>(tab, p, g);
    const T f = g;
    const T fn = upper_masked<1, P>(f, p);
    const T lv = ld - F(CF<M>::la) * f - F(CF<M>::lc) * fn;
    u[0] = f;
    u[M - 1] = lv;
#pragma unroll
    for (int k = 1; k < M - 1; ++k) u[k] = dp[k] - F(CF<M>::ap + k) * f - F(CF<M>::cp + k) * lv;
}

template <typename T, int M>
__device__ __forceinline__ void cf_solve_p(const T *tab, int P, int p, const T (&rd)[M], T (&u)[M]) {
    switch (P) {
        case 1: cf_solve<T, M, 1>(tab, p, rd, u); return;
        case 2: cf_solve<T, M, 2>(tab, p, rd, u); return;
        case 4: cf_solve<T, M, 4>(tab, p, rd, u); return;
        case 8: cf_solve<T, M, 8>(tab, p, rd, u); return;
        default: cf_solve<T, M, 16>(tab, p, rd, u); return;
    }
}

template <typename T, bool PS, int kRM>
__global__ __launch_bounds__(max_threads(kRM)) void k_adi2d_resident(ResGeom g, T *__restrict__ u_all,
                                                                    const T *__restrict__ s_all, T s0) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *U = reinterpret_cast<T *>(smem_raw);
    T *D = U + g.region;
    T *S = D + g.region;  // per-point s: its values; constant s: the factor tables
    T *tabA = S, *tabB = S + CF<kRM>::fields(g.px) * g.px;
    const int nt = blockDim.x, t = threadIdx.x;
    const int nx = g.nx, ny = g.ny, npts = nx * ny;
    T *um = u_all + (i64)blockIdx.x * npts;
    const T *sm = PS ? s_all + (i64)blockIdx.x * npts : nullptr;
    for (int e = t; e < npts; e += nt) {
        const int y = e / nx, x = e - y * nx;
        U[res_at<kRM>(g, y, x)] = um[e];
        if (PS) S[res_at<kRM>(g, y, x)] = sm[e];
    }
    if (!PS && t < 64) {  // one wavefront tabulates both line directions
        cf_setup_p<T, kRM>(s0, nx, g.px, t, tabA);
        cf_setup_p<T, kRM>(s0, ny, g.py, t, tabB);
    }
    __syncthreads();
    const int la = nt / g.px, lb = nt / g.py;  // lines per pass
    for (int it = 0; it < g.nsteps; ++it) {
        // ---- phase A: d = 2 s L u, then the x-line solve of d
        for (int yb = 0; yb < ny; yb += la) {
            const int y = yb + t / g.px, p = t % g.px, x0 = p * kRM;
            const bool live = y < ny;
            const int ya = live ? y : 0;  // dead lanes address row 0
            const int xc = x0 < nx ? x0 : 0;  // tiles past the line's end address column 0
            const int base = res_at<kRM>(g, ya, xc);
            const int dn = res_at<kRM>(g, ya + 1, xc) - base, ds = base - res_at<kRM>(g, ya > 0 ? ya - 1 : 0, xc);
            const bool hn = live && y + 1 < ny, hs = live && y > 0;
            // guarded LDS reads fall back to the tile's own first point (a point
            // of the mesh), so no lane addresses outside the array
            T uc[kRM + 2];  // u of the tile's points and their x neighbours
            uc[0] = load_if(U, base - 1 - g.tp, live && x0 > 0 && x0 < nx, base);
#pragma unroll
            for (int k = 0; k < kRM; ++k) uc[k + 1] = load_if(U, base + k, live && x0 + k < nx, base);
            uc[kRM + 1] = load_if(U, base + kRM + g.tp, live && x0 + kRM < nx, base);
            T rd[kRM], sv[kRM];
#pragma unroll
            for (int k = 0; k < kRM; ++k) {
                const bool v = live && x0 + k < nx;
                const T un = load_if(U, base + dn + k, v && hn, base);
                const T us = load_if(U, base - ds + k, v && hs, base);
                sv[k] = PS ? load_if(S, base + k, v, base) : s0;
                const T lap = un + us + uc[k] + uc[k + 2] - T(4) * uc[k + 1];
                rd[k] = v ? T(2) * sv[k] * lap : T(0);
            }
            T xs[kRM];
            if constexpr (PS) {
                TileState<T, kRM> ts;
                tile_eliminate_fn<T, kRM>(SRows<T>{sv, x0, live ? nx : 0}, rd, ts);
                T f, lv;
                dpp_reduced<T, kRM>(ts, g.px, p, f, lv);
                tile_backsub<T, kRM>(ts, f, lv, xs);
            } else {
                cf_solve_p<T, kRM>(tabA, g.px, p, rd, xs);
            }
#pragma unroll
            for (int k = 0; k < kRM; ++k)
                if (live && x0 + k < nx) D[base + k] = xs[k];
        }
        __syncthreads();
        // ---- phase B: the y-line solve of d, then u += d
        for (int xb = 0; xb < nx; xb += lb) {
            const int x = xb + t / g.py, q = t % g.py, y0 = q * kRM;
            const bool live = x < nx;
            const int xa = live ? x : 0;
            T rd[kRM], sv[kRM];
            int off[kRM];
#pragma unroll
            for (int k = 0; k < kRM; ++k) {
                const int y = y0 + k;
                const bool v = live && y < ny;
                off[k] = res_at<kRM>(g, v ? y : 0, xa);
                rd[k] = load_if(D, off[k], v, off[k]);
                sv[k] = PS ? load_if(S, off[k], v, off[k]) : s0;
            }
            T xs[kRM];
            if constexpr (PS) {
                TileState<T, kRM> ts;
                tile_eliminate_fn<T, kRM>(SRows<T>{sv, y0, live ? ny : 0}, rd, ts);
                T f, lv;
                dpp_reduced<T, kRM>(ts, g.py, q, f, lv);
                tile_backsub<T, kRM>(ts, f, lv, xs);
            } else {
                cf_solve_p<T, kRM>(tabB, g.py, q, rd, xs);
            }
#pragma unroll
            for (int k = 0; k < kRM; ++k)
                if (live && y0 + k < ny) U[off[k]] += xs[k];
        }
        __syncthreads();
    }
    for (int e = t; e < npts; e += nt) {
        const int y = e / nx, x = e - y * nx;
        um[e] = U[res_at<kRM>(g, y, x)];
    }
}

// The Hundsdorfer-Verwer steps of the SLV stand-in (u_t = a u_xx + b u_yy +
// c u_xy, Alg. 4's call structure) with the mesh resident in LDS: U, R, Z
// (three arrays, same layout as above); a, b, c are read from memory where a
// phase needs them (read-only; they stay in the caches between steps).  Each
// predictor is fused into the line solve that follows it:
//   A (x lines): from U: Z = U + dt/2 F(U), R = X^-1 (U + dt F(U) - th dt F1(U))
//   B (y lines): R = Y^-1 (R - th dt F2(U))                       (R = Y2)
//   C (x lines): from R: Z = X^-1 (Z + dt/2 F(Y2) - th dt F1(Y2))  (Z = W1)
//   D (y lines): U = Y^-1 (Z - th dt F2(Y2))
// with X, Y the rows (-th dt a, 1 + 2 th dt a, -th dt a) and the same with b.
// A thread reads the stencil neighbourhood of its tile and writes only its
// own tile's points, so one barrier after each phase orders the phases.
template <typename T>
struct HvCoef {
    const T *a, *b, *c;
    T dt, theta;
};

// CL = 2: a, b, c staged in LDS (CA, CB, CC, same layout as U) instead of read
// from memory in every phase; CL = 1: b only (it is read in all four phases).
template <typename T, int kRM, int STAGE, int CL>
__device__ __forceinline__ void hv_x_phase(const ResGeom &g, const HvCoef<T> &cf, i64 mb, const T *src, T *R, T *Z,
                                           const T *CA, const T *CB, const T *CC) {
    const int nt = blockDim.x, t = threadIdx.x;
    const int nx = g.nx, ny = g.ny, la = nt / g.px;
    const T dt = cf.dt, tdt = cf.theta * cf.dt, hdt = T(0.5) * cf.dt;
    for (int yb = 0; yb < ny; yb += la) {
        const int y = yb + t / g.px, p = t % g.px, x0 = p * kRM;
        const bool live = y < ny;
        const int ya = live ? y : 0;
        // tiles past the line's end (identity tiles) address column 0, so every
        // address, also of a guarded read's fallback, is a point of the mesh
        const int xc = x0 < nx ? x0 : 0;
        const int base = res_at<kRM>(g, ya, xc);
        const int dn = res_at<kRM>(g, ya + 1, xc) - base, ds = base - res_at<kRM>(g, ya > 0 ? ya - 1 : 0, xc);
        const bool hn = live && y + 1 < ny, hs = live && y > 0;
        const bool hw = live && x0 > 0 && x0 < nx, he = live && x0 + kRM < nx;
        // rows y-1, y, y+1 over x0-1 .. x0+M (zero outside the mesh); guarded
        // reads fall back to the tile's own first point
        T vs[kRM + 2], vc[kRM + 2], vn[kRM + 2];
        vs[0] = load_if(src, base - ds - 1 - g.tp, hs && hw, base);
        vc[0] = load_if(src, base - 1 - g.tp, hw, base);
        vn[0] = load_if(src, base + dn - 1 - g.tp, hn && hw, base);
#pragma unroll
        for (int k = 0; k < kRM; ++k) {
            const bool v = live && x0 + k < nx;
            vs[k + 1] = load_if(src, base - ds + k, v && hs, base);
            vc[k + 1] = load_if(src, base + k, v, base);
            vn[k + 1] = load_if(src, base + dn + k, v && hn, base);
        }
        vs[kRM + 1] = load_if(src, base - ds + kRM + g.tp, hs && he, base);
        vc[kRM + 1] = load_if(src, base + kRM + g.tp, he, base);
        vn[kRM + 1] = load_if(src, base + dn + kRM + g.tp, hn && he, base);
        const i64 e0 = mb + (i64)ya * nx + x0;
        T rd[kRM], sv[kRM];
#pragma unroll
        for (int k = 0; k < kRM; ++k) {
            const bool v = live && x0 + k < nx;
            T ak, bk, ck;
            if constexpr (CL == 2) {
                ak = load_if(CA, base + k, v, base);
                ck = load_if(CC, base + k, v, base);
            } else {
                ak = load_if(cf.a, e0 + k, v, mb);
                ck = load_if(cf.c, e0 + k, v, mb);
            }
            if constexpr (CL >= 1) {
                bk = load_if(CB, base + k, v, base);
            } else {
                bk = load_if(cf.b, e0 + k, v, mb);
            }
            const T f1 = ak * (vc[k] - T(2) * vc[k + 1] + vc[k + 2]);
            const T f = ck * ((vn[k + 2] - vs[k + 2] - vn[k] + vs[k]) * T(0.25)) + f1 +
                        bk * (vs[k + 1] - T(2) * vc[k + 1] + vn[k + 1]);
            sv[k] = tdt * ak;
            if constexpr (STAGE == 0) {
                if (v) Z[base + k] = vc[k + 1] + hdt * f;
                rd[k] = v ? vc[k + 1] + dt * f - tdt * f1 : T(0);
            } else {
                rd[k] = v ? Z[base + k] + hdt * f - tdt * f1 : T(0);
            }
        }
        TileState<T, kRM> ts;
        tile_eliminate_fn<T, kRM>(SRows<T>{sv, x0, live ? nx : 0}, rd, ts);
        T f, lv, xs[kRM];
        dpp_reduced<T, kRM>(ts, g.px, p, f, lv);
        tile_backsub<T, kRM>(ts, f, lv, xs);
        T *dst = STAGE == 0 ? R : Z;
#pragma unroll
        for (int k = 0; k < kRM; ++k)
            if (live && x0 + k < nx) dst[base + k] = xs[k];
    }
}

template <typename T, int kRM, int STAGE, int CL>
__device__ __forceinline__ void hv_y_phase(const ResGeom &g, const HvCoef<T> &cf, i64 mb, const T *src,
                                           const T *own, T *dst, const T *CB) {
    const int nt = blockDim.x, t = threadIdx.x;
    const int nx = g.nx, ny = g.ny, lb = nt / g.py;
    const T tdt = cf.theta * cf.dt;
    for (int xb = 0; xb < nx; xb += lb) {
        const int x = xb + t / g.py, q = t % g.py, y0 = q * kRM;
        const bool live = x < nx;
        const int xa = live ? x : 0;
        T col[kRM + 2], rd[kRM], sv[kRM];
        int off[kRM];
        {
            const bool v = live && y0 > 0 && y0 < ny;  // the point above a tile inside the line
            const int o = res_at<kRM>(g, v ? y0 - 1 : 0, xa);
            col[0] = load_if(src, o, v, o);
        }
#pragma unroll
        for (int k = 0; k < kRM; ++k) {
            const int y = y0 + k;
            const bool v = live && y < ny;
            off[k] = res_at<kRM>(g, v ? y : 0, xa);
            col[k + 1] = load_if(src, off[k], v, off[k]);
        }
        {
            const bool v = live && y0 + kRM < ny;
            const int o = res_at<kRM>(g, v ? y0 + kRM : 0, xa);
            col[kRM + 1] = load_if(src, o, v, o);
        }
#pragma unroll
        for (int k = 0; k < kRM; ++k) {
            const int y = y0 + k;
            const bool v = live && y < ny;
            const T bk = CL >= 1 ? load_if(CB, off[k], v, off[k]) : load_if(cf.b, mb + (i64)y * nx + xa, v, mb);
            const T ok = load_if(own, off[k], v, off[k]);
            sv[k] = tdt * bk;
            rd[k] = v ? ok - tdt * bk * (col[k] - T(2) * col[k + 1] + col[k + 2]) : T(0);
        }
        TileState<T, kRM> ts;
        tile_eliminate_fn<T, kRM>(SRows<T>{sv, y0, live ? ny : 0}, rd, ts);
        T f, lv, xs[kRM];
        dpp_reduced<T, kRM>(ts, g.py, q, f, lv);
        tile_backsub<T, kRM>(ts, f, lv, xs);
#pragma unroll
        for (int k = 0; k < kRM; ++k)
            if (live && y0 + k < ny) dst[off[k]] = xs[k];
    }
}

// 512 threads at most for every tile size: a tile's three stencil rows and
// coefficients need up to 256 VGPRs (FP64, 14-row tiles).
constexpr int kHvMaxThreads = 512;

template <typename T, int kRM, int CL>
__global__ __launch_bounds__(kHvMaxThreads) void k_hv_resident(ResGeom g, HvCoef<T> cf, T *__restrict__ u_all) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *U = reinterpret_cast<T *>(smem_raw);
    T *R = U + g.region;
    T *Z = R + g.region;
    T *CB = Z + g.region, *CA = CB + g.region, *CC = CA + g.region;  // CL >= 1: CB; CL = 2: all
    const int nt = blockDim.x, t = threadIdx.x;
    const int nx = g.nx, npts = nx * g.ny;
    const i64 mb = (i64)blockIdx.x * npts;
    T *um = u_all + mb;
    for (int e = t; e < npts; e += nt) {
        const int y = e / nx, x = e - y * nx;
        const int o = res_at<kRM>(g, y, x);
        U[o] = um[e];
        if constexpr (CL >= 1) CB[o] = cf.b[mb + e];
        if constexpr (CL == 2) {
            CA[o] = cf.a[mb + e];
            CC[o] = cf.c[mb + e];
        }
    }
    __syncthreads();
    for (int it = 0; it < g.nsteps; ++it) {
        hv_x_phase<T, kRM, 0, CL>(g, cf, mb, U, R, Z, CA, CB, CC);
        __syncthreads();
        hv_y_phase<T, kRM, 0, CL>(g, cf, mb, U, R, R, CB);
        __syncthreads();
        hv_x_phase<T, kRM, 1, CL>(g, cf, mb, R, R, Z, CA, CB, CC);
        __syncthreads();
        hv_y_phase<T, kRM, 1, CL>(g, cf, mb, R, Z, U, CB);
        __syncthreads();
    }
    for (int e = t; e < npts; e += nt) {
        const int y = e / nx, x = e - y * nx;
        um[e] = U[res_at<kRM>(g, y, x)];
    }
}

int pow2_ceil(int v) {
    int p = 1;
    while (p < v) p *= 2;
    return p;
}

int tiles_of(i64 n, int M) { return pow2_ceil((int)((n + M - 1) / M)); }

// Threads per workgroup: one per tile of a pass over the lines; 1024 (8-row
// tiles only) when a direction has at least 2048 tiles (measured: 128^2 gains,
// 96^2 and 64^2 do not).
int threads_of(const ResGeom &g, bool hv = false) {
    const int need = std::max(g.ny * g.px, g.nx * g.py);
    const int cap = (need >= 2048 && !hv) ? max_threads(g.m) : 512;
    return std::max(64, std::min(cap, pow2_ceil(need)));
}

// Largest number of dwords one bank (32 banks of 4 bytes) serves for one
// wavefront's access (lanes touch distinct points), over the tile rows k, for
// both phases.
int bank_conflicts(const ResGeom &g, int w) {
    const int lanes = std::min(64, threads_of(g));
    int worst = 0;
    for (int phase = 0; phase < 2; ++phase) {
        const int P = phase == 0 ? g.px : g.py;
        for (int k = 0; k < g.m; ++k) {
            int cnt[32] = {0};
            for (int l = 0; l < lanes; ++l) {
                const int line = l / P, tile = l % P;
                const int y = phase == 0 ? line : tile * g.m + k;
                const int x = phase == 0 ? tile * g.m + k : line;
                if (y >= g.ny || x >= g.nx) continue;
                const int a = res_at_h(g, y, x) * w / 4;
                for (int dw = 0; dw < w / 4; ++dw) worst = std::max(worst, ++cnt[(a + dw) % 32]);
            }
        }
    }
    return worst;
}

int cf_fields(int M, int P) {
    switch (M) {
        case 8: return CF<8>::fields(P);
        case 10: return CF<10>::fields(P);
        case 12: return CF<12>::fields(P);
        default: return CF<14>::fields(P);
    }
}

// Layout search for tile size M.
bool search_layout_m(const ResidentReq &r, int M, int narr, ResGeom *out, size_t *bytes) {
    const int w = r.f64 ? 8 : 4;
    const int px = tiles_of(r.nx, M), py = tiles_of(r.ny, M);
    if (px > 16 || py > 16) return false;
    const size_t tabs =  // constant s: the factor tables
        (r.s || r.hv) ? 0 : (size_t)(cf_fields(M, px) * px + cf_fields(M, py) * py) * w;
    // preference: two workgroups per CU where LDS allows it, then the fewest
    // bank conflicts, then the least LDS
    ResGeom best{};
    size_t best_bytes = 0;
    int best_conf = 1 << 30, best_occ = 0;
    for (int tp = 1; tp >= 0; --tp) {
        ResGeom g{};
        g.nx = (int)r.nx;
        g.ny = (int)r.ny;
        g.m = M;
        g.px = px;
        g.py = py;
        g.tp = tp;
        g.nsteps = r.nsteps;
        const int rowlen = g.nx + (tp ? (g.nx - 1) / M + 1 : 0);
        for (int ldx = rowlen; ldx < rowlen + 32; ++ldx) {
            for (int skw = 0; skw < 32; ++skw) {
                g.ldx = ldx;
                g.skw = skw;
                g.region = (res_at_h(g, g.ny - 1, g.nx - 1) + 1 + 3) & ~3;
                const size_t b = (size_t)narr * g.region * w + tabs;
                if (b > kLdsBytes) continue;
                const int occ = (int)std::min<size_t>(2, kLdsBytes / b);
                const int conf = bank_conflicts(g, w);
                if (occ > best_occ || (occ == best_occ && (conf < best_conf ||
                                                           (conf == best_conf && b < best_bytes)))) {
                    best = g;
                    best_occ = occ;
                    best_conf = conf;
                    best_bytes = b;
                }
            }
        }
    }
    if (best_conf == (1 << 30)) return false;
    *out = best;
    *bytes = best_bytes;
    return true;
}

// Tile size: the least padded tile rows over both directions (ties: the
// smaller tile), among those whose layout fits.  Measured at 1500 meshes x
// 120 steps, this pick was the fastest of the four sizes for 48^2 (12 rows),
// 80^2 (10), 96^2 (12) and 112^2 (14), FP32 and FP64.
bool search_layout(const ResidentReq &r, ResGeom *out, size_t *bytes) {
    int order[4] = {0, 1, 2, 3};
    auto padded = [&](int M) {
        return (i64)tiles_of(r.nx, M) * M * r.ny + (i64)tiles_of(r.ny, M) * M * r.nx;
    };
    std::stable_sort(order, order + 4, [&](int a, int b) { return padded(kTileRows[a]) < padded(kTileRows[b]); });

    // arrays: u, d (, s); HV: u, r, z, and a, b, c too where they fit
    for (int i : order) {
        if (r.hv && search_layout_m(r, kTileRows[i], 6, out, bytes)) {
            out->cl = 2;
            return true;
        }
        if (r.hv && search_layout_m(r, kTileRows[i], 4, out, bytes)) {
            out->cl = 1;
            return true;
        }
        if (search_layout_m(r, kTileRows[i], (r.s || r.hv) ? 3 : 2, out, bytes)) {
            out->cl = 0;
            return true;
        }
    }
    return false;
}

// The layout for a forced tile size (0: the automatic choice); no caching.
bool search_layout_forced(const ResidentReq &r, int M, ResGeom *out, size_t *bytes) {
    if (!M) return search_layout(r, out, bytes);
    if (r.hv && search_layout_m(r, M, 6, out, bytes)) {
        out->cl = 2;
        return true;
    }
    if (r.hv && search_layout_m(r, M, 4, out, bytes)) {
        out->cl = 1;
        return true;
    }
    if (search_layout_m(r, M, (r.s || r.hv) ? 3 : 2, out, bytes)) {
        out->cl = 0;
        return true;
    }
    return false;
}

// Layouts are searched once per (nx, ny, precision, s form, HV or ADI) and kept.
bool plan_resident(const ResidentReq &r, ResGeom *out, size_t *bytes) {
    if (r.nx < 1 || r.ny < 1 || r.nx > kMaxLine || r.ny > kMaxLine) return false;
    static std::mutex mu;
    static std::map<std::tuple<int, int, bool, bool, bool>, std::pair<ResGeom, size_t>> cache;
    const auto key = std::make_tuple((int)r.nx, (int)r.ny, r.f64, r.s != nullptr, r.hv);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it == cache.end()) {
        ResGeom g;
        size_t b = 0;
        if (!search_layout(r, &g, &b)) b = 0;
        it = cache.emplace(key, std::make_pair(g, b)).first;
    }
    if (!it->second.second) return false;
    *out = it->second.first;
    out->nsteps = r.nsteps;
    *bytes = it->second.second;
    return true;
}

template <typename T, bool PS, int M>
hipError_t go(const ResidentReq &r, const ResGeom &g, size_t bytes, hipStream_t s) {
    auto kern = k_adi2d_resident<T, PS, M>;
    if (bytes > 64 * 1024) {
        static bool raised = false;  // one attribute call per instantiation
        if (!raised) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)kLdsBytes);
            if (e != hipSuccess) return e;
            raised = true;
        }
    }
    launch(kern, dim3((unsigned)r.batch), dim3(threads_of(g)), bytes, s, g, static_cast<T *>(r.u),
           static_cast<const T *>(r.s), (T)r.s0);
    return hipGetLastError();
}

template <typename T, int M, int CL>
hipError_t go_hv(const ResidentReq &r, const ResGeom &g, size_t bytes, hipStream_t s) {
    auto kern = k_hv_resident<T, M, CL>;
    if (bytes > 64 * 1024) {
        static bool raised = false;
        if (!raised) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)kLdsBytes);
            if (e != hipSuccess) return e;
            raised = true;
        }
    }
    HvCoef<T> cf{static_cast<const T *>(r.a), static_cast<const T *>(r.b), static_cast<const T *>(r.c), (T)r.dt,
                 (T)r.theta};
    launch(kern, dim3((unsigned)r.batch), dim3(threads_of(g, true)), bytes, s, g, cf, static_cast<T *>(r.u));
    return hipGetLastError();
}

template <int M>
hipError_t go_t(const ResidentReq &r, const ResGeom &g, size_t bytes, hipStream_t s) {
    if (r.hv) {
        if (g.cl == 2) return r.f64 ? go_hv<double, M, 2>(r, g, bytes, s) : go_hv<float, M, 2>(r, g, bytes, s);
        if (g.cl == 1) return r.f64 ? go_hv<double, M, 1>(r, g, bytes, s) : go_hv<float, M, 1>(r, g, bytes, s);
        return r.f64 ? go_hv<double, M, 0>(r, g, bytes, s) : go_hv<float, M, 0>(r, g, bytes, s);
    }
    if (r.f64) return r.s ? go<double, true, M>(r, g, bytes, s) : go<double, false, M>(r, g, bytes, s);
    return r.s ? go<float, true, M>(r, g, bytes, s) : go<float, false, M>(r, g, bytes, s);
}

}  // namespace

bool resident_layout(const ResidentReq &r, int force_M, int64_t out[10]) {
    if (r.nx < 1 || r.ny < 1 || r.nx > kMaxLine || r.ny > kMaxLine) return false;
    if (force_M != 0 && force_M != 8 && force_M != 10 && force_M != 12 && force_M != 14) return false;
    ResGeom g;
    size_t bytes = 0;
    if (!search_layout_forced(r, force_M, &g, &bytes)) return false;
    const int64_t v[10] = {g.m, g.px, g.py, g.ldx, g.skw, g.tp, g.region, g.cl, threads_of(g, r.hv), (int64_t)bytes};
    for (int i = 0; i < 10; ++i) out[i] = v[i];
    return true;
}

bool resident_fits(const ResidentReq &r) {
    ResGeom g;
    size_t b;
    return r.batch >= 1 && r.batch < ((i64)1 << 31) && plan_resident(r, &g, &b);
}

hipError_t launch_resident(const ResidentReq &r, hipStream_t s) {
    ResGeom g;
    size_t bytes;
    if (r.batch < 1 || r.batch >= ((i64)1 << 31) || !plan_resident(r, &g, &bytes)) return hipErrorInvalidValue;
    switch (g.m) {
        case 8: return go_t<8>(r, g, bytes, s);
        case 10: return go_t<10>(r, g, bytes, s);
        case 12: return go_t<12>(r, g, bytes, s);
        default: return go_t<14>(r, g, bytes, s);
    }
}

}  // namespace trid
