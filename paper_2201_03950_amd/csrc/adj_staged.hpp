// adj_staged.hpp -- transposed solve of the s operator along contiguous (x)
// lines, staged through LDS.  The reverse pass of one ADI step solves
// A^T lambda = g with A = rows (-s, 1 + 2 s, -s), i.e. rows
// (-s_{g-1}, 1 + 2 s_g, -s_{g+1}), and accumulates the gradient of s:
//   sbar_g += lambda_g (x_{g-1} - 2 x_g + x_{g+1})        (x: the forward solution)
// The strided kernel would read x lines with one line per lane (no
// coalescing); here every array moves through LDS with coalesced accesses, as
// the forward x solve does (Section III-A).  s and g are loaded together, x and
// sbar while the solve runs; one LDS region serves the four arrays in turn.
#pragma once

#include "lines.hpp"

namespace trid {

template <typename T, int M>
__global__ __launch_bounds__(256) void k_staged_adj_s(StagedGeom gm, const T *__restrict__ s,
                                                      const T *grhs, const T *__restrict__ xf, T *g,
                                                      T *__restrict__ gs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    const int L = gm.L, P = gm.P, n = gm.n, ls = gm.ls;
    T *red = sh + L * ls;  // reduced-solve scratch (6 L P elements)
    const int t = threadIdx.x, p = t % P, l = t / P;
    const i64 o0 = xcd_block_id() * L;
    const int nl = (int)((gm.nlines - o0) < (i64)L ? (gm.nlines - o0) : (i64)L);
    const bool act = l < nl;
    const int pos = l * ls + p * (M + 1);
    const i64 off = o0 * n;
    const int cnt = nl * n;
    // grhs may alias g (in-place adjoint): it is read completely here, before
    // anything is written
    T vs[M], vd[M];
    stage_load<T, M>(vs, s + off, cnt);
    stage_load<T, M>(vd, grhs + off, cnt);
    // staged value of row g0 + k of this thread's line, k = -1 .. M (0 outside the line)
    auto window = [&](T(&w)[M + 2]) {
#pragma unroll
        for (int k = -1; k <= M; ++k) {
            const int gg = p * M + k;
            const int q = k < 0 ? pos - 2 : (k == M ? pos + M + 1 : pos + k);
            const bool ok = act && gg >= 0 && gg < n;
            const T v = sh[ok ? q : pos];
            w[k + 1] = ok ? v : T(0);
        }
    };
    // transposed rows come from the s window on demand (fewer live registers
    // than materialised sub/diag/super arrays)
    T sv[M + 2], rd[M];
    stage_put<T, M>(sh, vs, cnt, n, ls);
    __syncthreads();
    window(sv);
    __syncthreads();
    stage_put<T, M>(sh, vd, cnt, n, ls);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const T v = sh[pos + k];
        rd[k] = (act && p * M + k < n) ? v : T(0);
    }
    // x and sbar are only needed after the solve: their loads fly during it
    T vx[M], vg[M];
    stage_load<T, M>(vx, xf + off, cnt);
    stage_load<T, M>(vg, gs + off, cnt);
    T lam[M];
    {
        auto rows = [&](int k, T &a, T &b, T &c) {
            const int gg = p * M + k;
            a = (gg > 0) ? -sv[k] : T(0);
            b = T(1) + T(2) * sv[k + 1];
            c = (gg < n - 1) ? -sv[k + 2] : T(0);
        };
        TileState<T, M> ts;
        tile_eliminate_fn<T, M>(rows, rd, ts);
        T f, lv;
        reduced_solve<T, M>(ts, red, L * P, P, p, t, 1, f, lv);
        tile_backsub<T, M>(ts, f, lv, lam);
    }
    __syncthreads();  // every thread has taken its rhs
    stage_put<T, M>(sh, vx, cnt, n, ls);
    __syncthreads();
    T gsd[M];
    {
        T xv[M + 2];
        window(xv);
#pragma unroll
        for (int k = 0; k < M; ++k) gsd[k] = lam[k] * (xv[k] - T(2) * xv[k + 1] + xv[k + 2]);
    }
    __syncthreads();
    stage_put<T, M>(sh, vg, cnt, n, ls);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < M; ++k) sh[pos + k] += gsd[k];  // own slots; padding slots are never copied out
    __syncthreads();
    stage_out<T, M>(gs + off, sh, cnt, n, ls);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < M; ++k) sh[pos + k] = lam[k];
    __syncthreads();
    stage_out<T, M>(g + off, sh, cnt, n, ls);
}

}  // namespace trid
