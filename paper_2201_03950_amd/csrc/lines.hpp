// lines.hpp -- the two line-solve kernel templates and their row sources / epilogues.
//
//  k_strided : lines with element stride >= 1 that is the fastest mesh extent
//              product (y and z lines, Section II-B).  Lanes map to adjacent
//              lines, so every row load/store of a wavefront is one contiguous
//              run of memory (the GPU counterpart of the paper's XY / XZ plane
//              buffering, Section III-A).  Thread t owns tile p = t / L of line
//              l = t % L; tiles of a line sit in different wavefronts.
//  k_staged  : contiguous lines (x lines).  The block's L lines are one
//              contiguous range of memory; it is loaded with coalesced accesses
//              into LDS (padded per tile against bank conflicts), each thread
//              reads its tile from LDS, and results leave through LDS again --
//              the LDS form of the paper's x-line transpose (Section III-A).
//              Thread t owns tile p = t % P of line l = t / P, so the tiles of
//              a line are adjacent lanes of one wavefront.
//
// Row sources produce (sub, diag, super, rhs) of the rows of a tile; the
// epilogue consumes the solution.  Both are small structs passed by value.
#pragma once

#include "tile.hpp"

namespace trid {

struct StridedGeom {
    i64 inner;  // line stride = number of lines per outer index
    i64 nib;    // blocks along inner = ceil(inner / L)
    int n;      // line length
    int L;      // lines per block
    int P;      // tiles per line
    unsigned lines = 0;  // inner * outer (k_strided_const: lines numbered across outer indices)
};

// ------------------------------------------------------------------ sources --
// load<M>(base, st, g0, n, act, ra, rb, rc, rd): rows g0..g0+M-1 of the line at
// element offset `base` with stride `st`.  Inactive threads and rows >= n get
// identity rows.

template <typename T>
struct SrcArrays {  // per-point a, b, c arrays; rhs from d
    const T *a, *b, *c, *d;
    template <int M>
    __device__ __forceinline__ void load(i64 base, i64 st, int g0, int n, bool act, T (&ra)[M],
                                         T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            const i64 off = base + (i64)g * st;
            ra[k] = load_if(a, off, v && g > 0, base);
            const T bv = load_if(b, off, v, base);
            rb[k] = v ? bv : T(1);
            rc[k] = load_if(c, off, v && g < n - 1, base);
            rd[k] = load_if(d, off, v, base);
        }
    }
};

template <typename T>
struct SrcConst {  // the same (a, b, c) on every row, generated in-kernel
    T a, b, c;
    const T *d;
    template <int M>
    __device__ __forceinline__ void load(i64 base, i64 st, int g0, int n, bool act, T (&ra)[M],
                                         T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            ra[k] = (v && g > 0) ? a : T(0);
            rb[k] = v ? b : T(1);
            rc[k] = (v && g < n - 1) ? c : T(0);
            rd[k] = load_if(d, base + (i64)g * st, v, base);
        }
    }
};

template <typename T>
struct SrcS {  // rows (-s, 1 + 2 s, -s) from a per-point s array
    const T *s, *d;
    template <int M>
    __device__ __forceinline__ void load(i64 base, i64 st, int g0, int n, bool act, T (&ra)[M],
                                         T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            const i64 off = base + (i64)g * st;
            const T sv = load_if(s, off, v, base);
            ra[k] = (g > 0) ? -sv : T(0);
            rb[k] = T(1) + T(2) * sv;
            rc[k] = (g < n - 1) ? -sv : T(0);
            rd[k] = load_if(d, off, v, base);
        }
    }
};

// Transposed rows (for adjoint solves): row g of A^T has sub-diagonal c_{g-1},
// diagonal b_g and super-diagonal a_{g+1}.
template <typename T>
struct SrcArraysT {
    const T *a, *b, *c, *d;
    template <int M>
    __device__ __forceinline__ void load(i64 base, i64 st, int g0, int n, bool act, T (&ra)[M],
                                         T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            const i64 off = base + (i64)g * st;
            ra[k] = load_if(c, off - st, v && g > 0, base);
            const T bv = load_if(b, off, v, base);
            rb[k] = v ? bv : T(1);
            rc[k] = load_if(a, off + st, v && g < n - 1, base);
            rd[k] = load_if(d, off, v, base);
        }
    }
};

template <typename T>
struct SrcST {  // transposed rows of the s operator: (-s_{g-1}, 1 + 2 s_g, -s_{g+1})
    const T *s, *d;
    template <int M>
    __device__ __forceinline__ void load(i64 base, i64 st, int g0, int n, bool act, T (&ra)[M],
                                         T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
        T sv[M + 2];
#pragma unroll
        for (int k = 0; k < M + 2; ++k) {
            const int g = g0 + k - 1;
            sv[k] = load_if(s, base + (i64)g * st, act && g >= 0 && g < n, base);
        }
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            ra[k] = (g > 0) ? -sv[k] : T(0);
            rb[k] = T(1) + T(2) * sv[k + 1];
            rc[k] = (g < n - 1) ? -sv[k + 2] : T(0);
            rd[k] = load_if(d, base + (i64)g * st, v, base);
        }
    }
};

// ---------------------------------------------------------------- epilogues --
// prefetch<M>(...) runs with the loads (before any barrier) so that operands of
// the epilogue are in flight together with the rows; store<M>(...) writes.

template <typename T>
struct EpiStore {  // x = solution
    static constexpr bool kWide = false;  // keeps no extra words per row
    T *x;
    // all M rows valid, 32-bit row offsets from `off` (used by the constant-row kernels)
    template <int M>
    __device__ __forceinline__ void store_rows(i64 off, unsigned st, bool act, const T (&u)[M]) const {
        if (!act) return;
        T *px = x + off;
#pragma unroll
        for (int k = 0; k < M; ++k) px[k * st] = u[k];
    }
    template <int M>
    struct Pre {};
    template <int M>
    __device__ __forceinline__ void prefetch(Pre<M> &, i64, i64, int, int, bool) const {}
    template <int M>
    __device__ __forceinline__ void store(const Pre<M> &, i64 base, i64 st, int g0, int n, bool act,
                                          const T (&u)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            if (act && g < n) x[base + (i64)g * st] = u[k];
        }
    }
};

template <typename T>
struct EpiAdd {  // u += solution (the update of Alg. 3, fused into the last solve)
    static constexpr bool kWide = true;  // keeps the M prefetched values of u
    T *u;
    // all M rows valid; u is read only now (not prefetched) and in groups of 8
    // rows (the empty asm keeps the compiler from hoisting every load), which
    // keeps VGPRs low enough for two blocks per CU
    template <int M>
    __device__ __forceinline__ void store_rows(i64 off, unsigned st, bool act, const T (&x)[M]) const {
        if (!act) return;
        T *pu = u + off;
        constexpr int G = M < 8 ? M : 8;
#pragma unroll
        for (int c = 0; c < M; c += G) {
            T v[G];
#pragma unroll
            for (int k = 0; k < G; ++k) v[k] = pu[(c + k) * st];
#pragma unroll
            for (int k = 0; k < G; ++k) pu[(c + k) * st] = v[k] + x[c + k];
            asm volatile("" ::: "memory");
        }
    }
    template <int M>
    struct Pre {
        T v[M];
    };
    template <int M>
    __device__ __forceinline__ void prefetch(Pre<M> &pre, i64 base, i64 st, int g0, int n,
                                             bool act) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            pre.v[k] = load_if(u, base + (i64)g * st, act && g < n, base);
        }
    }
    template <int M>
    __device__ __forceinline__ void store(const Pre<M> &pre, i64 base, i64 st, int g0, int n,
                                          bool act, const T (&x)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            if (act && g < n) u[base + (i64)g * st] = pre.v[k] + x[k];
        }
    }
};

// u += solution and w = solution: the update of Alg. 3 for a step whose
// intermediates are kept for the reverse pass (w is the step's increment).
template <typename T>
struct EpiAddKeep {
    static constexpr bool kWide = true;  // keeps the M prefetched values of u
    T *u;
    T *w;
    template <int M>
    struct Pre {
        T v[M];
    };
    template <int M>
    __device__ __forceinline__ void prefetch(Pre<M> &pre, i64 base, i64 st, int g0, int n,
                                             bool act) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            pre.v[k] = load_if(u, base + (i64)g * st, act && g < n, base);
        }
    }
    template <int M>
    __device__ __forceinline__ void store(const Pre<M> &pre, i64 base, i64 st, int g0, int n,
                                          bool act, const T (&x)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            if (act && g < n) {
                const i64 off = base + (i64)g * st;
                u[off] = pre.v[k] + x[k];
                w[off] = x[k];
            }
        }
    }
};

// Adjoint epilogue, arrays form: lambda -> g; ga = -lambda x_{g-1}, gb = -lambda x_g,
// gc = -lambda x_{g+1} (0 at the ignored a_0 / c_{N-1}).
template <typename T>
struct EpiAdjArrays {
    static constexpr bool kWide = true;  // keeps the forward solution and its neighbours
    const T *x;
    T *g, *ga, *gb, *gc;
    template <int M>
    struct Pre {
        T xv[M + 2];
    };
    template <int M>
    __device__ __forceinline__ void prefetch(Pre<M> &pre, i64 base, i64 st, int g0, int n,
                                             bool act) const {
#pragma unroll
        for (int k = 0; k < M + 2; ++k) {
            const int gg = g0 + k - 1;
            pre.xv[k] = load_if(x, base + (i64)gg * st, act && gg >= 0 && gg < n, base);
        }
    }
    template <int M>
    __device__ __forceinline__ void store(const Pre<M> &pre, i64 base, i64 st, int g0, int n,
                                          bool act, const T (&lam)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int gg = g0 + k;
            if (act && gg < n) {
                const i64 off = base + (i64)gg * st;
                g[off] = lam[k];
                ga[off] = -lam[k] * pre.xv[k];
                gb[off] = -lam[k] * pre.xv[k + 1];
                gc[off] = -lam[k] * pre.xv[k + 2];
            }
        }
    }
};

// Adjoint epilogue, s form: lambda -> g; gs += lambda (x_{g-1} - 2 x_g + x_{g+1}).
template <typename T>
struct EpiAdjS {
    static constexpr bool kWide = true;  // keeps the forward solution and its neighbours
    const T *x;
    T *g, *gs;
    template <int M>
    struct Pre {
        T xv[M + 2];
        T sv[M];
    };
    template <int M>
    __device__ __forceinline__ void prefetch(Pre<M> &pre, i64 base, i64 st, int g0, int n,
                                             bool act) const {
#pragma unroll
        for (int k = 0; k < M + 2; ++k) {
            const int gg = g0 + k - 1;
            pre.xv[k] = load_if(x, base + (i64)gg * st, act && gg >= 0 && gg < n, base);
        }
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int gg = g0 + k;
            pre.sv[k] = load_if(gs, base + (i64)gg * st, act && gg < n, base);
        }
    }
    template <int M>
    __device__ __forceinline__ void store(const Pre<M> &pre, i64 base, i64 st, int g0, int n,
                                          bool act, const T (&lam)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int gg = g0 + k;
            if (act && gg < n) {
                const i64 off = base + (i64)gg * st;
                g[off] = lam[k];
                gs[off] = pre.sv[k] + lam[k] * (pre.xv[k] - T(2) * pre.xv[k + 1] + pre.xv[k + 2]);
            }
        }
    }
};

// ------------------------------------------------------------------ kernels --

template <typename T, int M, int MAXT, class Src, class Epi>
__global__ __launch_bounds__(MAXT) void k_strided(StridedGeom gm, Src src, Epi epi) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    const int L = gm.L, P = gm.P;
    const int t = threadIdx.x, l = t % L, p = t / L;
    const i64 blk = xcd_block_id();
    const i64 ib = blk % gm.nib, ob = blk / gm.nib;
    const i64 ii = ib * L + l;
    const bool act = ii < gm.inner;
    const i64 st = gm.inner;
    const i64 base = ob * (i64)gm.n * st + (act ? ii : 0);
    const int g0 = p * M;
    T ra[M], rb[M], rc[M], rd[M];
    src.template load<M>(base, st, g0, gm.n, act, ra, rb, rc, rd);
    typename Epi::template Pre<M> pre;
    epi.template prefetch<M>(pre, base, st, g0, gm.n, act);
    // keep the scheduler from sinking loads into the elimination: every load
    // of the tile is issued before the first arithmetic waits on one
    asm volatile("" ::: "memory");
    T u[M];
    tile_solve<T, M>(ra, rb, rc, rd, sh, L * P, P, p, t, L, u);
    epi.template store<M>(pre, base, st, g0, gm.n, act, u);
}

// Register-lean strided solve of rows (-s, 1 + 2 s, -s): a thread keeps only
// its tile's s and d (2 M words) in registers -- no per-row elimination state --
// so blocks of up to 1024 threads cover more adjacent lines, and every row
// access of a wavefront reads a longer contiguous segment.  The boundary
// equations come from tile_ends_fn (two streaming sweeps), the reduced system
// is solved as in k_strided, and the interior rows 1..M-2 are then solved by
// Thomas (Alg. 1) with the tile's end values known, in place in the s and d
// registers.  Rows are addressed by 32-bit offsets from the line's first
// element (the host checks that a line spans less than 2^31 elements), so a
// row's address costs no 64-bit register pair.
// OUT: 0 x = solution; 1 x += solution; 2 x += solution and x2 = solution.
template <typename T, int M, int MAXT, int OUT>
__global__ __launch_bounds__(MAXT) void k_strided_lean(StridedGeom gm, const T *__restrict__ s,
                                                       const T *__restrict__ d, T *__restrict__ x,
                                                       T *__restrict__ x2) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    const int L = gm.L, P = gm.P, n = gm.n;
    const int t = threadIdx.x, l = t % L, p = t / L;
    const i64 blk = xcd_group_block_id<16>();
    const i64 ib = blk % gm.nib, ob = blk / gm.nib;
    const i64 ii = ib * L + l;
    const bool act = ii < gm.inner;
    const unsigned st = (unsigned)gm.inner;
    const i64 base = ob * (i64)n * (i64)gm.inner + (act ? ii : 0);
    const T *sp = s + base;
    const T *dp = d + base;
    const int g0 = p * M;
    T sv[M], dv[M], uo[OUT ? M : 1];
#pragma unroll
    for (int k = 0; k < M; ++k) {  // rows past the line load its first row (values unused)
        const int g = g0 + k;
        const unsigned o = (act && g < n) ? (unsigned)g * st : 0u;
        sv[k] = sp[o];
        dv[k] = dp[o];
        if constexpr (OUT != 0) uo[k] = x[base + o];
    }
    asm volatile("" ::: "memory");  // every load of the tile is issued before the first use
    // rows past the line become identity rows (s = d = 0), whose solution is 0
    // exactly, so the last row's c (coupling to them) and the first row's a
    // (only in fa, whose coupling the reduced solve drops for the first tile)
    // need no masks: every row is (-s, 1 + 2 s, -s)
#pragma unroll
    for (int k = 0; k < M; ++k)
        if (!(act && g0 + k < n)) sv[k] = dv[k] = T(0);
    auto rows = [&](int k, T &a, T &b, T &c) {
        const T sk = sv[k];
        a = -sk;
        b = T(1) + T(2) * sk;
        c = -sk;
    };
    // each sweep regenerates the rows from s: the empty asm makes s look
    // rewritten, so the compiler does not keep every row's (a, b, c) live
    auto fence = [&] {
#pragma unroll
        for (int k = 0; k < M; ++k) asm volatile("" : "+v"(sv[k]));
    };
    TileEnds<T> e;
    tile_ends_fn<T, M>(rows, dv, e, fence);
    fence();
    T f, lv;
    reduced_solve<T, M>(e, sh, L * P, P, p, t, L, f, lv);
    // interior rows with u_0 = f and u_{M-1} = lv known: c* into sv, d* into dv
    T cprev = T(0), dprev = T(0);
#pragma unroll
    for (int k = 1; k < M - 1; ++k) {
        T a, b, c;
        rows(k, a, b, c);
        T rhs = dv[k];
        if (k == 1) {
            rhs -= a * f;
            a = T(0);
        }
        if (k == M - 2) {
            rhs -= c * lv;
            c = T(0);
        }
        const T r = fast_rcp(b - a * cprev);
        cprev = c * r;
        dprev = (rhs - a * dprev) * r;
        sv[k] = cprev;
        dv[k] = dprev;
    }
    dv[0] = f;
    dv[M - 1] = lv;
#pragma unroll
    for (int k = M - 3; k >= 1; --k) dv[k] -= sv[k] * dv[k + 1];
    T *xp = x + base;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int g = g0 + k;
        if (act && g < n) {
            const unsigned o = (unsigned)g * st;
            if constexpr (OUT == 0) {
                xp[o] = dv[k];
            } else {
                xp[o] = uo[k] + dv[k];
                if constexpr (OUT == 2) x2[base + o] = dv[k];
            }
        }
    }
}

// ------------------------------------------------------------ staged kernel --

struct StagedGeom {
    i64 nlines;  // number of contiguous lines
    int n;       // line length
    int L;       // lines per block
    int P;       // tiles per line
    int ls;      // LDS elements per staged line (>= P * (M + 1))
};

// LDS position of element i of staged line ll (tiles padded to M+1 elements).
template <int M>
__device__ __forceinline__ int staged_pos(int ll, int i, int ls) {
    return ll * ls + (i / M) * (M + 1) + (i % M);
}

// Cooperative coalesced copy of `cnt` contiguous elements from global `src`
// into staged positions of region `dst` (line length n).  cnt <= blockDim * M
// (a block holds at most P * M >= n rows per line and L * P threads), so each
// thread handles at most M elements, in two halves that may be split apart:
//   stage_load: the thread's M elements into registers (all loads in flight
//               together; branch-free, idle slots read element cnt - 1),
//   stage_put : those registers into their staged LDS positions.
template <typename T, int M>
__device__ __forceinline__ void stage_load(T (&v)[M], const T *__restrict__ src, int cnt) {
    const int nt = blockDim.x;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int e = threadIdx.x + k * nt;
        v[k] = load_if(src, e, e < cnt, cnt - 1);
    }
}

template <typename T, int M>
__device__ __forceinline__ void stage_put(T *__restrict__ dst, const T (&v)[M], int cnt, int n, int ls) {
    const int nt = blockDim.x;
    int ll = threadIdx.x / n, i = threadIdx.x % n;
    const int dl = nt / n, di = nt % n;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int e = threadIdx.x + k * nt;
        if (e < cnt) dst[staged_pos<M>(ll, i, ls)] = v[k];
        ll += dl;
        i += di;
        if (i >= n) {
            i -= n;
            ++ll;
        }
    }
}

template <typename T, int M>
__device__ __forceinline__ void stage_in(T *__restrict__ dst, const T *__restrict__ src, int cnt,
                                         int n, int ls) {
    T v[M];
    stage_load<T, M>(v, src, cnt);
    stage_put<T, M>(dst, v, cnt, n, ls);
}

template <typename T, int M>
__device__ __forceinline__ void stage_out(T *__restrict__ dst, const T *__restrict__ src, int cnt,
                                          int n, int ls) {
    const int nt = blockDim.x;
    int ll = threadIdx.x / n, i = threadIdx.x % n;
    const int dl = nt / n, di = nt % n;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int e = threadIdx.x + k * nt;
        if (e < cnt) dst[e] = src[staged_pos<M>(ll, i, ls)];
        ll += dl;
        i += di;
        if (i >= n) {
            i -= n;
            ++ll;
        }
    }
}

// Staged sources stage their arrays one at a time through ONE LDS region of
// L * ls elements (so a block's LDS does not grow with the number of arrays):
//   stage<M>(r, sh, o0, nl, n, ls, scratch): fill the region with array r of
//       lines [o0, o0 + nl) (coalesced); scratch is the reduced-solve LDS area,
//       free during staging;
//   take<M>(r, sh, pos, g0, n, act, ra, rb, rc, rd): move this thread's tile
//       of array r from LDS into the raw rows.
// The kernel runs stage(r), barrier, take(r), barrier for r = 0..kRegions-1.

template <typename T>
struct StgArrays {
    static constexpr int kRegions = 4;
    const T *a, *b, *c, *d;
    template <int M>
    __device__ __forceinline__ void stage(int r, T *__restrict__ sh, i64 o0, int nl, int n, int ls,
                                          void *) const {
        const T *src = r == 0 ? a : (r == 1 ? b : (r == 2 ? c : d));
        stage_in<T, M>(sh, src + o0 * n, nl * n, n, ls);
    }
    template <int M>
    __device__ __forceinline__ void take(int r, const T *__restrict__ sh, int pos, int g0, int n, bool act,
                                         T (&ra)[M], T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            const T val = sh[pos + k];  // own tile slot: always inside the region
            if (r == 0) ra[k] = (v && g > 0) ? val : T(0);
            if (r == 1) rb[k] = v ? val : T(1);
            if (r == 2) rc[k] = (v && g < n - 1) ? val : T(0);
            if (r == 3) rd[k] = v ? val : T(0);
        }
    }
};

template <typename T>
struct StgConst {
    static constexpr int kRegions = 1;
    T a, b, c;
    const T *d;
    template <int M>
    __device__ __forceinline__ void stage(int, T *__restrict__ sh, i64 o0, int nl, int n, int ls,
                                          void *) const {
        stage_in<T, M>(sh, d + o0 * n, nl * n, n, ls);
    }
    template <int M>
    __device__ __forceinline__ void take(int, const T *__restrict__ sh, int pos, int g0, int n, bool act,
                                         T (&ra)[M], T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            ra[k] = (v && g > 0) ? a : T(0);
            rb[k] = v ? b : T(1);
            rc[k] = (v && g < n - 1) ? c : T(0);
            const T val = sh[pos + k];
            rd[k] = v ? val : T(0);
        }
    }
};

template <typename T>
struct StgS {
    static constexpr int kRegions = 2;
    const T *s, *d;
    template <int M>
    __device__ __forceinline__ void stage(int r, T *__restrict__ sh, i64 o0, int nl, int n, int ls,
                                          void *) const {
        stage_in<T, M>(sh, (r == 0 ? s : d) + o0 * n, nl * n, n, ls);
    }
    template <int M>
    __device__ __forceinline__ void take(int r, const T *__restrict__ sh, int pos, int g0, int n, bool act,
                                         T (&ra)[M], T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            if (r == 0) {
                const T val = sh[pos + k];
                const T sv = v ? val : T(0);
                ra[k] = (g > 0) ? -sv : T(0);
                rb[k] = T(1) + T(2) * sv;
                rc[k] = (g < n - 1) ? -sv : T(0);
            } else {
                const T val = sh[pos + k];
                rd[k] = v ? val : T(0);
            }
        }
    }
};

// Staged epilogue: results are in LDS region 0 (rhs region for StgConst, the a
// region otherwise -- it is no longer read); copy them out coalesced.
template <typename T>
struct StgOut {
    T *x;
    template <int M>
    __device__ __forceinline__ void out(const T *__restrict__ sh, i64 o0, int nl, int n,
                                        int ls) const {
        stage_out<T, M>(x + o0 * n, sh, nl * n, n, ls);
    }
};

template <typename T, int M, int MAXT, class Src, class Out>
__global__ __launch_bounds__(MAXT) void k_staged(StagedGeom gm, Src src, Out out) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    const int L = gm.L, P = gm.P, n = gm.n, ls = gm.ls;
    const int S = L * P;
    T *red = sh + L * ls;  // reduced-solve scratch (6 S elements)
    const int t = threadIdx.x, p = t % P, l = t / P;
    const i64 o0 = xcd_block_id() * L;
    const int nl = (int)((gm.nlines - o0) < (i64)L ? (gm.nlines - o0) : (i64)L);
    const bool act = l < nl;
    const int pos = l * ls + p * (M + 1);
    T ra[M], rb[M], rc[M], rd[M];
#pragma unroll
    for (int r = 0; r < Src::kRegions; ++r) {
        if (r > 0) __syncthreads();  // every thread has taken region r - 1
        src.template stage<M>(r, sh, o0, nl, n, ls, red);
        __syncthreads();
        src.template take<M>(r, sh, pos, p * M, n, act, ra, rb, rc, rd);
    }
    T u[M];
    tile_solve<T, M>(ra, rb, rc, rd, red, S, P, p, t, 1, u);
    // take() reads only this thread's own slots, so they can hold its results
    // right away (no other thread reads them before the barrier below)
#pragma unroll
    for (int k = 0; k < M; ++k) sh[pos + k] = u[k];
    __syncthreads();
    out.template out<M>(sh, o0, nl, n, ls);
}

}  // namespace trid
