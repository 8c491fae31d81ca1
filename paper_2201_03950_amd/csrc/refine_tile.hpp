// refine_tile.hpp -- device part of the FP32 solve + FP64 refinement of one tile
// (shared by the batched and the uneven-batch kernels).
#pragma once

#include "tile.hpp"

namespace trid {

// FP32 coefficients of one tile, loaded once and reused by both solves.
template <int M, bool SM>
struct RefCoef;

template <int M>
struct RefCoef<M, true> {  // rows (-s, 1 + 2 s, -s)
    float s[M];
    int g0, n;
    __device__ __forceinline__ void row32(int k, float &a, float &b, float &c) const {
        const int g = g0 + k;
        const bool v = g < n;
        a = (v && g > 0) ? -s[k] : 0.f;
        b = v ? 1.f + 2.f * s[k] : 1.f;
        c = (v && g < n - 1) ? -s[k] : 0.f;
    }
    __device__ __forceinline__ void row64(int k, double &a, double &b, double &c) const {
        const int g = g0 + k;
        const bool v = g < n;
        const double sv = (double)s[k];
        a = (v && g > 0) ? -sv : 0.0;
        b = v ? 1.0 + 2.0 * sv : 1.0;
        c = (v && g < n - 1) ? -sv : 0.0;
    }
};

template <int M>
struct RefCoef<M, false> {  // per-point a, b, c
    float a[M], b[M], c[M];
    int g0, n;
    __device__ __forceinline__ void row32(int k, float &ra, float &rb, float &rc) const {
        const int g = g0 + k;
        const bool v = g < n;
        ra = (v && g > 0) ? a[k] : 0.f;
        rb = v ? b[k] : 1.f;
        rc = (v && g < n - 1) ? c[k] : 0.f;
    }
    __device__ __forceinline__ void row64(int k, double &ra, double &rb, double &rc) const {
        float fa, fb, fc;
        row32(k, fa, fb, fc);
        ra = fa;
        rb = fb;
        rc = fc;
    }
};

// Both solves and the residual for one tile; returns x = x32 + dx in `out`.
// red: 6 S floats of PCR scratch; xb: 2 S doubles for the tile-boundary exchange.
template <int M, bool SM>
__device__ __forceinline__ void refine_tile(const RefCoef<M, SM> &cf, const double (&dd)[M],
                                            float *__restrict__ red, double *__restrict__ xb, int S,
                                            int P, int p, int slot, int pstride, double (&out)[M],
                                            int Pu = 0) {
    auto rows = [&](int k, float &a, float &b, float &c) { cf.row32(k, a, b, c); };
    float rd[M];
#pragma unroll
    for (int k = 0; k < M; ++k) rd[k] = (float)dd[k];
    float x32[M];
    // the tile factor of the first solve serves the correction solve too
    // (16-row tiles; 32-row tiles sweep again, their factor would not fit
    // in registers beside the rows)
    constexpr bool kKeep = M <= 16;
    TileFactor<float, kKeep ? M : 3> fct;
    float dp[kKeep ? M : 3];
    if constexpr (!kKeep) {
        TileState<float, M> ts;
        tile_eliminate_fn<float, M>(rows, rd, ts);
        float f, lv;
        if (Pu)
            reduced_pcr<float, M>(ts, red, S, P, p, slot, pstride, f, lv, Pu);
        else
            reduced_solve<float, M>(ts, red, S, P, p, slot, pstride, f, lv);
        tile_backsub<float, M>(ts, f, lv, x32);
    } else {
        TileEnds<float> ts;
        tile_factor_fn<float, M>(rows, rd, fct, dp, ts);
        float f, lv;
        if (Pu)  // lines of different lengths share the block (uneven batch)
            reduced_pcr<float, M>(ts, red, S, P, p, slot, pstride, f, lv, Pu);
        else
            reduced_solve<float, M>(ts, red, S, P, p, slot, pstride, f, lv);
        tile_factor_backsub<float, M>(fct, dp, f, lv, x32);
    }
    // neighbours of the tile's first and last rows for the residual
    xb[slot] = x32[0];
    xb[S + slot] = x32[M - 1];
    __syncthreads();
    const double xprev = (p > 0) ? xb[S + slot - pstride] : 0.0;
    const double xnext = (p + 1 < P) ? xb[slot + pstride] : 0.0;
    // r = d - A x32 in FP64 (A: FP64 promotion of the FP32 rows)
#pragma unroll
    for (int k = 0; k < M; ++k) {
        double a, b, c;
        cf.row64(k, a, b, c);
        const double xm = k > 0 ? (double)x32[k - 1] : xprev;
        const double xp = k < M - 1 ? (double)x32[k + 1] : xnext;
        rd[k] = (float)(dd[k] - (a * xm + b * (double)x32[k] + c * xp));
    }
    float dx[M];
    if constexpr (!kKeep) {
        TileState<float, M> ts;
        tile_eliminate_fn<float, M>(rows, rd, ts);
        float f, lv;
        if (Pu)
            reduced_pcr<float, M>(ts, red, S, P, p, slot, pstride, f, lv, Pu);
        else
            reduced_solve<float, M>(ts, red, S, P, p, slot, pstride, f, lv);
        tile_backsub<float, M>(ts, f, lv, dx);
    } else {
        TileEnds<float> ts;
        tile_factor_rhs<float, M>(fct, rd, dp, ts);
        float f, lv;
        if (Pu)  // lines of different lengths share the block (uneven batch)
            reduced_pcr<float, M>(ts, red, S, P, p, slot, pstride, f, lv, Pu);
        else
            reduced_solve<float, M>(ts, red, S, P, p, slot, pstride, f, lv);
        tile_factor_backsub<float, M>(fct, dp, f, lv, dx);
    }
#pragma unroll
    for (int k = 0; k < M; ++k) out[k] = (double)x32[k] + (double)dx[k];
}

}  // namespace trid
