// k_refine.hip -- FP32 bulk solve with one FP64 residual and refinement sweep,
// fused while each tile stays in registers:
//   x32 = solve32(A32, fp32(d));  r = d - A x32 (FP64);  dx = solve32(A32, fp32(r));
//   x = x32 + dx (FP64).
// A is the matrix of record given by FP32 coefficients (a, b, c arrays, or s with
// rows (-s, 1 + 2 s, -s)); its FP64 rows are exact promotions of them.  The
// solves are the tiled modified Thomas of eq. (7) with the PCR reduced solve
// (Section III-B), as in the plain kernels.  Not in the paper: the precision
// scheme is an addition of this library.
#include <algorithm>
#include <type_traits>

#include "dispatch.hpp"
#include "lines.hpp"
#include "refine.hpp"
#include "refine_tile.hpp"

namespace trid {

// ------------------------------------------------------------- strided --

template <typename TD, int M, bool SM, int MAXT>
__global__ __launch_bounds__(MAXT) void k_refine_strided(StridedGeom gm, RefPtrs src, const TD *__restrict__ d,
                                                         double *__restrict__ x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = gm.L, P = gm.P, S = L * P;
    double *xb = reinterpret_cast<double *>(smem_raw);
    float *red = reinterpret_cast<float *>(xb + 2 * S);
    const int t = threadIdx.x, l = t % L, p = t / L;
    const i64 blk = xcd_block_id();
    const i64 ib = blk % gm.nib, ob = blk / gm.nib;
    const i64 ii = ib * L + l;
    const bool act = ii < gm.inner;
    const i64 st = gm.inner;
    const i64 base = ob * (i64)gm.n * st + (act ? ii : 0);
    const int g0 = p * M, n = gm.n;
    RefCoef<M, SM> cf;
    cf.g0 = g0;
    cf.n = act ? n : 0;  // inactive lanes see identity rows only
    double dd[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int g = g0 + k;
        const bool v = act && g < n;
        const i64 off = base + (i64)g * st;  // base itself is in bounds for every lane
        if constexpr (SM) {
            cf.s[k] = load_if(src.s, off, v, base);
        } else {
            cf.a[k] = load_if(src.a, off, v, base);
            cf.b[k] = v ? load_if(src.b, off, v, base) : 1.f;
            cf.c[k] = load_if(src.c, off, v, base);
        }
        dd[k] = (double)load_if(d, off, v, base);
    }
    double out[M];
    refine_tile<M, SM>(cf, dd, red, xb, S, P, p, t, L, out);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int g = g0 + k;
        if (act && g < n) x[base + (i64)g * st] = out[k];
    }
}

// --------------------------------------------------------- strided, lean --
// Rows (-s, 1 + 2 s, -s) from FP32 s on strided lines, with a thread's
// registers holding only its tile's s, its right-hand side and one more tile
// of values: each FP32 solve finds the tile's boundary equations by two
// streaming sweeps (tile_ends_fn), the reduced system as the other kernels
// do, and the interior by Thomas (Alg. 1) with the tile's end values known.
// d is read from HBM once: its FP32 rounding d32 goes to LDS, and for FP64 d
// so does the tail fp32(d - d32), so the residual takes d as d32 + tail (48
// significant bits, a relative error of at most 2^-48 in d).  The tail waits
// in the thread's x32 slots during the first solve and moves to the
// registers of the Thomas multipliers once that solve is done.
// Rows past the line are identity rows (s = d = 0, solution 0).  32-bit row
// offsets from the line's first element (the host checks that a line spans
// less than 2^31 elements).
template <typename TD, int M, int MAXT>
__global__ __launch_bounds__(MAXT) void k_refine_lean(StridedGeom gm, const float *__restrict__ s,
                                                      const TD *__restrict__ d, double *__restrict__ x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = gm.L, P = gm.P, S = L * P, n = gm.n;
    float *red = reinterpret_cast<float *>(smem_raw);  // 6 S: reduced-solve scratch
    float *xs = red + 6 * S;                           // S (M + 1): every tile's x32 (padded)
    float *dh = xs + S * (M + 1);                      // M S: d32, row k of tile t at k S + t
    const int t = threadIdx.x, l = t % L, p = t / L;
    const i64 blk = xcd_group_block_id<16>();
    const i64 ib = blk % gm.nib, ob = blk / gm.nib;
    const i64 ii = ib * L + l;
    const bool act = ii < gm.inner;
    const unsigned st = (unsigned)gm.inner;
    const i64 base = ob * (i64)n * (i64)gm.inner + (act ? ii : 0);
    const float *sp = s + base;
    const TD *dp = d + base;
    const int g0 = p * M;
    float sv[M], w[M], cs[M];
    TD dk[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int g = g0 + k;
        const unsigned o = (act && g < n) ? (unsigned)g * st : 0u;
        sv[k] = sp[o];
        dk[k] = dp[o];
    }
    asm volatile("" ::: "memory");
    // x32 goes to LDS (tile t at t (M + 1)) after the first solve: the residual
    // reads the tile's rows and the adjacent tiles' boundary rows (tiles p -+ 1
    // of the line are threads t -+ L) from there; until then the slots hold
    // the tail of d
    float *xm = xs + t * (M + 1);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const bool v = act && g0 + k < n;
        w[k] = v ? (float)dk[k] : 0.f;
        if constexpr (sizeof(TD) == 8) xm[k] = v ? (float)((double)dk[k] - (double)w[k]) : 0.f;
        if (!v) sv[k] = 0.f;
        dh[k * S + t] = w[k];
    }
    auto rows = [&](int k, float &a, float &b, float &c) {
        const float sk = sv[k];
        a = -sk;
        b = 1.f + 2.f * sk;
        c = -sk;
    };
    auto fence = [&] {
#pragma unroll
        for (int k = 0; k < M; ++k) asm volatile("" : "+v"(sv[k]));
    };
    // one FP32 solve of the right-hand side in w, in place
    auto solve32 = [&]() {
        TileEnds<float> e;
        tile_ends_fn<float, M>(rows, w, e, fence);
        fence();
        float f, lv;
        reduced_solve<float, M>(e, red, S, P, p, t, L, f, lv);
        float cprev = 0.f, dprev = 0.f;
#pragma unroll
        for (int k = 1; k < M - 1; ++k) {
            float a, b, c;
            rows(k, a, b, c);
            float rhs = w[k];
            if (k == 1) {
                rhs -= a * f;
                a = 0.f;
            }
            if (k == M - 2) {
                rhs -= c * lv;
                c = 0.f;
            }
            const float r = fast_rcp(b - a * cprev);
            cprev = c * r;
            dprev = (rhs - a * dprev) * r;
            cs[k] = cprev;
            w[k] = dprev;
        }
        w[0] = f;
        w[M - 1] = lv;
#pragma unroll
        for (int k = M - 3; k >= 1; --k) w[k] -= cs[k] * w[k + 1];
        fence();
    };
    solve32();
#pragma unroll
    for (int k = 0; k < M; ++k) {
        cs[k] = sizeof(TD) == 8 ? xm[k] : 0.f;  // the tail of d
        xm[k] = w[k];
    }
    __syncthreads();
    const double xprev = (p > 0) ? (double)xs[(t - L) * (M + 1) + M - 1] : 0.0;
    const double xnext = (p + 1 < P) ? (double)xs[(t + L) * (M + 1)] : 0.0;
    // r = d - A x32 in FP64
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const bool v = act && g0 + k < n;
        const double dd = (double)dh[k * S + t] + (double)cs[k];
        const double sk = (double)sv[k];
        const double um = k > 0 ? (double)xm[k - 1] : xprev;
        const double up = k < M - 1 ? (double)xm[k + 1] : xnext;
        const double r = dd - (-sk * um + (1.0 + 2.0 * sk) * (double)xm[k] - sk * up);
        w[k] = v ? (float)r : 0.f;
    }
    solve32();
    double *xo = x + base;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int g = g0 + k;
        if (act && g < n) xo[(unsigned)g * st] = (double)xm[k] + (double)w[k];
    }
}

// -------------------------------------------------------------- staged --
// x lines: the block's coefficient arrays and d are staged into LDS (tiles
// padded to M + 1 elements); the FP64 result leaves through the same LDS area.

template <typename TD, int M, bool SM>
__global__ __launch_bounds__(256) void k_refine_staged(StagedGeom gm, RefPtrs src, const TD *__restrict__ d,
                                                       double *__restrict__ x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = gm.L, P = gm.P, n = gm.n, ls = gm.ls, S = L * P;
    const int reg = L * ls;
    constexpr int NC = SM ? 1 : 3;
    float *cst = reinterpret_cast<float *>(smem_raw);  // NC coefficient regions
    // d region, 16-byte aligned (the planner reserves the padding)
    const size_t doff = ((size_t)NC * reg * sizeof(float) + 15) & ~(size_t)15;
    TD *dst = reinterpret_cast<TD *>(smem_raw + doff);
    unsigned char *after = reinterpret_cast<unsigned char *>(dst + reg);
    after += (16 - (reinterpret_cast<uintptr_t>(after) & 15)) & 15;
    double *xb = reinterpret_cast<double *>(after);
    float *red = reinterpret_cast<float *>(xb + 2 * S);
    const int t = threadIdx.x, p = t % P, l = t / P;
    const i64 o0 = xcd_block_id() * L;
    const int nl = (int)((gm.nlines - o0) < (i64)L ? (gm.nlines - o0) : (i64)L);
    const i64 off = o0 * n;
    const int cnt = nl * n;
    if constexpr (SM) {
        stage_in<float, M>(cst, src.s + off, cnt, n, ls);
    } else {
        stage_in<float, M>(cst, src.a + off, cnt, n, ls);
        stage_in<float, M>(cst + reg, src.b + off, cnt, n, ls);
        stage_in<float, M>(cst + 2 * reg, src.c + off, cnt, n, ls);
    }
    stage_in<TD, M>(dst, d + off, cnt, n, ls);
    __syncthreads();
    const bool act = l < nl;
    const int pos = l * ls + p * (M + 1);
    RefCoef<M, SM> cf;
    cf.g0 = p * M;
    cf.n = act ? n : 0;
    double dd[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const bool v = act && p * M + k < n;
        if constexpr (SM) {
            cf.s[k] = v ? cst[pos + k] : 0.f;
        } else {
            cf.a[k] = v ? cst[pos + k] : 0.f;
            cf.b[k] = v ? cst[reg + pos + k] : 1.f;
            cf.c[k] = v ? cst[2 * reg + pos + k] : 0.f;
        }
        dd[k] = v ? (double)dst[pos + k] : 0.0;
    }
    double out[M];
    refine_tile<M, SM>(cf, dd, red, xb, S, P, p, t, 1, out);
    // the staged inputs are dead (every thread passed refine_tile's barriers):
    // reuse the area, viewed as doubles at the same staged positions
    double *ost = reinterpret_cast<double *>(smem_raw);
#pragma unroll
    for (int k = 0; k < M; ++k) ost[pos + k] = out[k];
    __syncthreads();
    stage_out<double, M>(x + off, ost, cnt, n, ls);
}

// The two streaming sweeps of tile_ends_fn with the forward sweep's pivot
// reciprocals rf[k] = 1 / (b_k - a_k cp_{k-1}), k = 1..M-1, kept: they depend on
// the matrix only, so the interior sweep of the same solve (whose pivots are
// the same) and every later solve with the same matrix reuse them (HAVE: rf
// holds them already).
template <typename T, int M, bool HAVE, class Rows, class Fence>
__device__ __forceinline__ void tile_ends_rf(const Rows &rows, const T (&rd)[M], T (&rf)[M], TileEnds<T> &e,
                                             Fence &&fence) {
    static_assert(M >= 3, "tiles need at least three rows");
    T a, b, c;
    rows(1, a, b, c);
    T r;
    if constexpr (HAVE) {
        r = rf[1];
    } else {
        r = fast_rcp(b);
        rf[1] = r;
    }
    T ap = a * r, cp = c * r, dp = rd[1] * r;
#pragma unroll
    for (int k = 2; k < M; ++k) {
        rows(k, a, b, c);
        if constexpr (HAVE) {
            r = rf[k];
        } else {
            r = fast_rcp(b - a * cp);
            rf[k] = r;
        }
        ap = -r * a * ap;
        cp = r * c;
        dp = r * (rd[k] - a * dp);
    }
    e.la = ap;
    e.lc = cp;
    e.ld = dp;
    fence();
    rows(M - 2, a, b, c);
    r = fast_rcp(b);
    T al = -a * r, be = -c * r, ga = rd[M - 2] * r;
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {
        rows(k, a, b, c);
        r = fast_rcp(b + c * al);
        be = -c * be * r;
        ga = (rd[k] - c * ga) * r;
        al = -a * r;
    }
    rows(0, a, b, c);
    e.fa = a;
    e.fb = b + c * al;
    e.fc = c * be;
    e.fd = rd[0] - c * ga;
}

// ---------------------------------------------------- staged, lean --
// x lines of per-point s and FP32 d whose P tiles (a power of two up to 64)
// sit in adjacent lanes of one wavefront: the block's s and d are staged into LDS,
// and each thread keeps only its tile's s, the FP32 solution and the
// residual.  Each FP32 solve finds the tile's boundary equations by two
// streaming sweeps (tile_ends_rf: the forward sweep's pivot reciprocals are
// kept for the interior sweep and the second solve), the reduced system by
// lane moves (no LDS, no barrier), and the interior by Thomas (Alg. 1) with
// both end values known.
// The neighbours of a tile's end rows for the FP64 residual come from the
// adjacent lanes; d is read again from its staged slots.  Rows past the line
// are identity rows (s = d = 0, solution 0).
template <typename TD, int M>
__global__ __launch_bounds__(256, 3) void k_refine_staged_lean(StagedGeom gm, const float *__restrict__ s,
                                                            const TD *__restrict__ d, double *__restrict__ x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int L = gm.L, P = gm.P, n = gm.n, ls = gm.ls;
    const int reg = L * ls;
    float *cst = reinterpret_cast<float *>(smem_raw);  // staged s
    const size_t doff = ((size_t)reg * sizeof(float) + 15) & ~(size_t)15;
    TD *dst = reinterpret_cast<TD *>(smem_raw + doff);  // staged d
    const int t = threadIdx.x, p = t % P, l = t / P;
    const i64 o0 = xcd_block_id() * L;
    const int nl = (int)((gm.nlines - o0) < (i64)L ? (gm.nlines - o0) : (i64)L);
    const i64 off = o0 * n;
    const int cnt = nl * n;
    stage_in<float, M>(cst, s + off, cnt, n, ls);
    stage_in<TD, M>(dst, d + off, cnt, n, ls);
    __syncthreads();
    const bool act = l < nl;
    // threads of lines past the block's last line (l < L always) take their
    // own unstaged slots and mask what they read there
    const int pos = l * ls + p * (M + 1);
    const int g0 = p * M;
    float sv[M], w[M], rf[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const bool v = act && g0 + k < n;
        const float sk = cst[pos + k];
        const TD dk = dst[pos + k];
        sv[k] = v ? sk : 0.f;
        w[k] = v ? (float)dk : 0.f;
    }
    auto rows = [&](int k, float &a, float &b, float &c) {
        const float sk = sv[k];
        a = -sk;
        b = 1.f + 2.f * sk;
        c = -sk;
    };
    auto fence = [&] {
#pragma unroll
        for (int k = 0; k < M; ++k) asm volatile("" : "+v"(sv[k]));
    };
    // one FP32 solve of the right-hand side in v, in place; the first keeps
    // the forward pivots' reciprocals in rf, the second (same matrix) reuses
    // them.  The interior sweep (both end values known) has the same pivots
    // b_k - a_k cp_{k-1} for k = 1..M-2, and its c' = c_k rf[k].
    auto solve32 = [&](float (&v)[M], auto have) {
        TileEnds<float> e;
        tile_ends_rf<float, M, decltype(have)::value>(rows, v, rf, e, fence);
        fence();
        float f, lv;
        reduced_solve<float, M>(e, nullptr, 0, P, p, t, 1, f, lv);
        float dprev = 0.f;
#pragma unroll
        for (int k = 1; k < M - 1; ++k) {
            float a, b, c;
            rows(k, a, b, c);
            float rhs = v[k];
            if (k == 1) {
                rhs -= a * f;
                a = 0.f;
            }
            if (k == M - 2) rhs -= c * lv;
            dprev = (rhs - a * dprev) * rf[k];
            v[k] = dprev;
        }
        v[0] = f;
        v[M - 1] = lv;
#pragma unroll
        for (int k = M - 3; k >= 1; --k) {
            float a, b, c;
            rows(k, a, b, c);
            v[k] -= c * rf[k] * v[k + 1];
        }
        fence();
    };
    solve32(w, std::false_type{});
    // x32 goes to the thread's own staged-s slots (s is in registers now; no
    // other thread reads them); the neighbours of the tile's end rows come
    // from the adjacent lanes (0 outside the line)
    float *xm = cst + pos;
    double xprev = (double)lane_up(w[M - 1], 1), xnext = (double)lane_down(w[0], 1);
    if (p == 0) xprev = 0.0;
    if (p + 1 >= P) xnext = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) xm[k] = w[k];
    // r = d - A x32 in FP64, into w
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const bool v = act && g0 + k < n;
        const double dk = (double)dst[pos + k];
        const double sk = (double)sv[k];
        const double um = k > 0 ? (double)xm[k - 1] : xprev;
        const double up = k < M - 1 ? (double)xm[k + 1] : xnext;
        const double rk = dk - (-sk * um + (1.0 + 2.0 * sk) * (double)xm[k] - sk * up);
        w[k] = v ? (float)rk : 0.f;
    }
    solve32(w, std::true_type{});
    float xo[M];
#pragma unroll
    for (int k = 0; k < M; ++k) xo[k] = xm[k];
    // every thread has read its staged inputs: the area takes the FP64 result
    // at the same staged positions
    __syncthreads();
    double *ost = reinterpret_cast<double *>(smem_raw);
    if (act) {
#pragma unroll
        for (int k = 0; k < M; ++k) ost[pos + k] = (double)xo[k] + (double)w[k];
    }
    __syncthreads();
    stage_out<double, M>(x + off, ost, cnt, n, ls);
}

// ---------------------------------------------------------------- host --

namespace {

i64 cdiv(i64 a, i64 b) { return (a + b - 1) / b; }

int pow2_floor(i64 v) {
    int p = 1;
    while ((i64)p * 2 <= v) p *= 2;
    return p;
}

int pow2_ceil(i64 v) {
    int p = 1;
    while ((i64)p < v) p *= 2;
    return p;
}

// Block size bound from the per-thread register footprint (FP32 tile state,
// FP32 coefficients, FP64 right-hand side).
constexpr int refine_strided_maxt(int M, bool sm) {
    return M <= 16 ? 512 : 256;
}

template <typename TD, int M, bool SM>
hipError_t go_strided(const RefineReq &r, const RefPlan &pl, hipStream_t s) {
    StridedGeom g;
    g.inner = r.inner;
    g.nib = cdiv(r.inner, pl.L);
    g.n = (int)r.n;
    g.L = pl.L;
    g.P = pl.P;
    constexpr int MAXT = refine_strided_maxt(M, SM);
    launch((k_refine_strided<TD, M, SM, MAXT>), dim3((unsigned)pl.nblocks), dim3(pl.L * pl.P),
                       pl.shmem, s, g, r.src, static_cast<const TD *>(r.d), r.x);
    return hipGetLastError();
}

template <typename TD, int M, bool SM>
hipError_t go_staged(const RefineReq &r, const RefPlan &pl, hipStream_t s) {
    StagedGeom g;
    g.nlines = r.outer;
    g.n = (int)r.n;
    g.L = pl.L;
    g.P = pl.P;
    g.ls = pl.ls;
    launch((k_refine_staged<TD, M, SM>), dim3((unsigned)pl.nblocks), dim3(pl.L * pl.P),
                       pl.shmem, s, g, r.src, static_cast<const TD *>(r.d), r.x);
    return hipGetLastError();
}

template <typename TD>
hipError_t go_lean(const RefineReq &r, const RefPlan &pl, hipStream_t s) {
    StridedGeom g;
    g.inner = r.inner;
    g.nib = cdiv(r.inner, pl.L);
    g.n = (int)r.n;
    g.L = pl.L;
    g.P = pl.P;
    auto kern = k_refine_lean<TD, 16, 1024>;
    if (pl.shmem > 64 * 1024) {
        static bool raised = false;  // one attribute call per instantiation
        if (!raised) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               160 * 1024);
            if (e != hipSuccess) return e;
            raised = true;
        }
    }
    launch(kern, dim3((unsigned)pl.nblocks), dim3(pl.L * pl.P), pl.shmem, s, g, r.src.s,
           static_cast<const TD *>(r.d), r.x);
    return hipGetLastError();
}

template <typename TD>
hipError_t go_staged_lean(const RefineReq &r, const RefPlan &pl, hipStream_t s) {
    StagedGeom g;
    g.nlines = r.outer;
    g.n = (int)r.n;
    g.L = pl.L;
    g.P = pl.P;
    g.ls = pl.ls;
    launch((k_refine_staged_lean<TD, 16>), dim3((unsigned)pl.nblocks), dim3(pl.L * pl.P), pl.shmem, s, g,
           r.src.s, static_cast<const TD *>(r.d), r.x);
    return hipGetLastError();
}

template <typename TD, bool SM>
hipError_t go_m(const RefineReq &r, const RefPlan &pl, hipStream_t s) {
    if constexpr (SM) {
        if (pl.lean && !pl.staged) return go_lean<TD>(r, pl, s);
        if constexpr (std::is_same<TD, float>::value)
            if (pl.lean) return go_staged_lean<TD>(r, pl, s);
    }
    if (pl.staged) return pl.M == 32 ? go_staged<TD, 32, SM>(r, pl, s) : go_staged<TD, 16, SM>(r, pl, s);
    return pl.M == 32 ? go_strided<TD, 32, SM>(r, pl, s) : go_strided<TD, 16, SM>(r, pl, s);
}

constexpr size_t kMaxShmem = 64 * 1024;

}  // namespace

bool plan_refine(const RefineReq &r, RefPlan *pl, std::string *err) {
    RefPlan p;
    const bool sm = r.smode;
    // strided lines of per-point s of at least 512 rows: the register-lean
    // kernel, 16-row tiles, as many adjacent lines as 512 threads hold (two
    // workgroups per CU, so one's loads overlap the other's solves; 1024
    // threads for lines of more than 512 tiles)
    if (sm && r.inner > 1 && r.n >= 512 && r.n * r.inner < ((i64)1 << 31) && (!r.force_M || r.force_M == 16)) {
        const i64 P = cdiv(r.n, 16);
        if (P <= 1024) {
            int L = r.force_L ? r.force_L : pow2_floor(std::max<i64>(1, 512 / P));
            if (!r.force_L) {
                if (r.inner < L) L = std::max(1, pow2_ceil(r.inner));
                while (L > 4 && cdiv(r.inner, L) * r.outer < 512) L /= 2;
            }
            if ((i64)L * P <= 1024) {
                p.M = 16;
                p.P = (int)P;
                p.L = L;
                p.lean = true;
                p.shmem = (size_t)(6 + 17 + 16) * L * P * sizeof(float);
                p.nblocks = cdiv(r.inner, L) * r.outer;
                if (p.nblocks < (i64)1 << 31) {
                    *pl = p;
                    return true;
                }
            }
        }
    }
    // x lines of per-point s and FP32 d with P = n / 16 tiles a power of two up
    // to 64: the register-lean staged kernel (a line's tiles in adjacent lanes
    // of one wavefront), one wavefront per workgroup (no barrier waits on other
    // wavefronts; 168 VGPRs, 12 workgroups per CU; measured 8% faster than four
    // wavefronts on 1024-row lines)
    if (sm && r.inner == 1 && !r.d_f64 && (!r.force_M || r.force_M == 16)) {
        const i64 P = cdiv(r.n, 16);
        if (P <= 64 && (P & (P - 1)) == 0) {
            const int ls = (int)P * 17;
            int L = r.force_L ? r.force_L : 64 / (int)P;
            L = std::max(1, std::min(L, pow2_ceil(r.outer)));
            const size_t dw = r.d_f64 ? 8 : 4;
            auto bytes = [&](int LL) {
                const size_t reg = (size_t)LL * ls;
                return std::max(((reg * 4 + 15) & ~(size_t)15) + reg * dw, reg * 8) + 16;
            };
            if ((i64)L * P <= 256 && bytes(L) <= kMaxShmem && cdiv(r.outer, L) < (i64)1 << 31) {
                p.M = 16;
                p.P = (int)P;
                p.L = L;
                p.ls = ls;
                p.staged = true;
                p.lean = true;
                p.shmem = bytes(L);
                p.nblocks = cdiv(r.outer, L);
                *pl = p;
                return true;
            }
        }
    }
    // 16-row tiles up to 256 tiles per line (measured on 1024-row lines: 34%
    // faster than 32-row tiles through LDS, 3% on strided lines)
    int M = r.force_M ? r.force_M : 16;
    if (M != 16 && M != 32) M = 16;
    i64 P = cdiv(r.n, M);
    if (P > 256 && M == 16) {
        M = 32;
        P = cdiv(r.n, M);
    }
    p.M = M;
    p.P = (int)P;
    const size_t dw = r.d_f64 ? 8 : 4;
    if (r.inner == 1 && P <= 256) {
        const int ls = (int)P * (M + 1);
        const int nc = sm ? 1 : 3;
        auto bytes = [&](int L) {
            size_t in = (size_t)L * ls * (4 * nc + dw) + 16;  // + alignment of the d region
            in = std::max(in, (size_t)L * ls * 8) + 16;
            return in + 2 * (size_t)L * P * 8 + 6 * (size_t)L * P * 4;
        };
        int L = r.force_L ? r.force_L : std::max(1, 256 / (int)P);
        L = std::max(1, std::min(L, pow2_ceil(r.outer)));
        while (L > 1 && bytes(L) > kMaxShmem) L /= 2;
        if (bytes(L) <= kMaxShmem && (i64)L * P <= 256) {
            p.staged = true;
            p.L = L;
            p.ls = ls;
            p.shmem = bytes(L);
            p.nblocks = cdiv(r.outer, L);
            *pl = p;
            return true;
        }
    }
    // x lines that did not stage: 16-row tiles whenever a 512-thread block
    // holds the line (measured 1.35x faster than 32-row tiles on 8192-row lines)
    if (r.inner == 1 && !r.force_M && M == 32 && cdiv(r.n, 16) <= refine_strided_maxt(16, sm)) {
        M = 16;
        P = cdiv(r.n, 16);
        p.M = M;
        p.P = (int)P;
    }
    const int maxt = refine_strided_maxt(M, sm);
    if (P > maxt) {
        *err = "line too long for the refinement kernels";
        return false;
    }
    int L = r.force_L ? r.force_L : std::min(64, pow2_floor(maxt / P));
    if (!r.force_L && r.inner < L) L = std::max(1, pow2_ceil(r.inner));
    if ((i64)L * P > maxt) {
        *err = "refinement plan exceeds the block size";
        return false;
    }
    p.staged = false;
    p.L = L;
    p.shmem = 2 * (size_t)L * P * 8 + 6 * (size_t)L * P * 4;
    p.nblocks = cdiv(r.inner, L) * r.outer;
    if (p.nblocks >= (i64)1 << 31) {
        *err = "too many blocks";
        return false;
    }
    *pl = p;
    return true;
}

hipError_t launch_refine(const RefineReq &r, const RefPlan &pl, hipStream_t s) {
    if (r.d_f64) return r.smode ? go_m<double, true>(r, pl, s) : go_m<double, false>(r, pl, s);
    return r.smode ? go_m<float, true>(r, pl, s) : go_m<float, false>(r, pl, s);
}

}  // namespace trid
