// k_adi.hip -- the explicit-stencil right-hand side of the ADI step (Alg. 3)
// fused with the step's x-line solve (Alg. 3): u is read once, the RHS
// d = 2 s L u is formed while staging the block's x lines into LDS, the rows
// (-s, 1 + 2 s, -s) are generated in-kernel (Section IV-A: coefficient
// generation fused into the solver), and only d is written.
//
// The block's L x lines are consecutive lines of the mesh, so their y
// neighbours are the lines themselves plus one line on each side: the window
// of lines o0 - 1 .. o0 + L is copied into LDS with 16-byte loads, and the x
// and y neighbours of every point are read from there.  Only the two z
// neighbours (3D) and s come from global memory, once per point each.
//
// Lines of P tiles, P not a power of two and at most 64, are laid out so that
// none straddles two wavefronts (64 / P lines per wavefront); their reduced
// systems are then solved by lane moves with no barrier.
#include <algorithm>

#include "const_lines.hpp"
#include "dispatch.hpp"
#include "lines.hpp"

namespace trid {

struct RhsGeom {
    i64 nlines;  // x lines of all meshes = ny * nz * batch
    int n;       // x line length
    int L, P, ls;
    int ny, nz;  // lines of one mesh = ny * nz (nz = 1 in 2D)
    int uoff;    // LDS element offset of the u window
    int soff;    // LDS element offset of the staged s (per-point s)
    int roff;    // LDS element offset of the reduced-solve scratch (first: line flags)
};

// Contiguous copy of cnt elements global -> LDS by the whole block, 16-byte
// vectors when both sides are aligned.  The first K * blockDim vectors go in
// one unrolled batch (all loads issued before the first LDS store); any rest
// follows in a plain loop.
template <typename T, int K>
__device__ __forceinline__ void copy_to_lds(T *__restrict__ dst, const T *__restrict__ src, int cnt) {
    constexpr int V = 16 / sizeof(T);
    using VT = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
    const int nt = blockDim.x, t = threadIdx.x;
    const bool vec = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0;
    int done = 0;
    if (vec) {
        const int nv = cnt / V;
        const VT *s4 = reinterpret_cast<const VT *>(src);
        VT *d4 = reinterpret_cast<VT *>(dst);
        if (nv > 0) {
            VT v[K];
#pragma unroll
            for (int k = 0; k < K; ++k) v[k] = load_if(s4, t + k * nt, t + k * nt < nv, nv - 1);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (t + k * nt < nv) d4[t + k * nt] = v[k];
        }
        for (int e = K * nt + t; e < nv; e += nt) d4[e] = s4[e];
        done = nv * V;
    }
    for (int e = done + t; e < cnt; e += nt) dst[e] = src[e];
}

// Staged elements back to global memory in index order (cnt <= blockDim * M):
// all of a thread's LDS reads go out before its stores (idle slots read slot 0).
template <typename T, int M>
__device__ __forceinline__ void stage_out_all(T *__restrict__ dst, const T *__restrict__ src, int cnt, int n,
                                              int ls) {
    const int nt = blockDim.x;
    int ll = threadIdx.x / n, i = threadIdx.x % n;
    const int dl = nt / n, di = nt % n;
    T v[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int e = threadIdx.x + k * nt;
        v[k] = src[e < cnt ? staged_pos<M>(ll, i, ls) : 0];
        ll += dl;
        i += di;
        if (i >= n) {
            i -= n;
            ++ll;
        }
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int e = threadIdx.x + k * nt;
        if (e < cnt) dst[e] = v[k];
    }
}

template <typename T, int M, bool PP, int NDIM, bool WV>
__global__ __launch_bounds__(256) void k_rhs_x(RhsGeom g, const T *__restrict__ u, const T *__restrict__ s,
                                               T s0, T *__restrict__ x) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);  // staged RHS, then the solution
    T *uw = sh + g.uoff;                      // u window
    T *ss = sh + g.soff;                      // staged s (per-point s)
    T *red = sh + g.roff;
    int *flags = reinterpret_cast<int *>(red);
    const int L = g.L, P = g.P, n = g.n, ls = g.ls;
    const int t = threadIdx.x, nt = blockDim.x;
    // thread -> (line l, tile p): P consecutive threads per line; with WV,
    // 64 / P lines per wavefront and the wavefront's last 64 % P lanes idle
    int p, l;
    bool lane_ok = true;
    if (WV) {
        const int G = 64 / P, j = t & 63;
        p = j % P;
        l = (t >> 6) * G + j / P;
        lane_ok = j < G * P;
    } else {
        p = t % P;
        l = t / P;
    }
    const i64 o0 = xcd_block_id() * L;
    const int nl = (int)((g.nlines - o0) < (i64)L ? (g.nlines - o0) : (i64)L);
    const bool act = lane_ok && l < nl;
    const int pos = (act ? l : 0) * ls + p * (M + 1);

    const i64 off = o0 * n;
    const i64 sz = (i64)g.ny * n;
    const i64 total = g.nlines * n;
    const int cnt = nl * n;
    // z neighbours and s of the thread's points go out first (they need no
    // LDS): a z neighbour is loaded whenever it is inside the array and masked
    // by the line flags below, so every load of the block is in flight at once
    T zl[M], zr[M], sv[M];
    int lls[M], is[M];
    {
        int ll = t / n, i = t % n;
        const int dl = nt / n, di = nt % n;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            lls[k] = ll;
            is[k] = i;
            const int e = t + k * nt;
            const bool v = e < cnt;
            const i64 q = off + e;
            const i64 qs = off + (v ? e : cnt - 1);  // in-bounds stand-in for idle lanes
            if (NDIM == 3) {
                zl[k] = load_if(u, q - sz, v && q >= sz, qs);
                zr[k] = load_if(u, q + sz, v && q + sz < total, qs);
            }
            if (PP) sv[k] = load_if(s, q, v, qs);
            ll += dl;
            i += di;
            if (i >= n) {
                i -= n;
                ++ll;
            }
        }
    }
    // window row r holds line o0 - 1 + r; rows outside the line range stay unread
    // (a line's y-1 / y+1 neighbour exists only inside its own plane)
    {
        const i64 w0 = o0 > 0 ? o0 - 1 : 0;
        const i64 w1 = (o0 + nl + 1) < g.nlines ? (o0 + nl + 1) : g.nlines;
        copy_to_lds<T, (2 * M * sizeof(T) + 15) / 16 + 1>(uw + (w0 - (o0 - 1)) * n, u + w0 * n, (int)(w1 - w0) * n);
    }
    // neighbour-existence flags of the block's lines: bit0 y-1, bit1 y+1, bit2 z-1, bit3 z+1
    for (int ll = t; ll < nl; ll += nt) {
        const i64 o = o0 + ll;
        const int j = (int)(o % g.ny);
        const int k = (int)((o / g.ny) % g.nz);
        flags[ll] = (j > 0 ? 1 : 0) | (j < g.ny - 1 ? 2 : 0) | (k > 0 ? 4 : 0) | (k < g.nz - 1 ? 8 : 0);
    }
    __syncthreads();

    // RHS of every point: x, y neighbours from the window.  Every read is
    // issued (idle slots and missing neighbours read in-window slots) and the
    // unused values are selected away, so the reads overlap.
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int ll = lls[k], i = is[k];
        const bool v = t + k * nt < cnt;
        const int f = flags[v ? ll : 0];
        const int b = v ? (ll + 1) * n + i : n;  // b - n >= 0, b + n < (L + 2) n
        const T c = uw[b], wm = uw[b - 1], wp = uw[b + 1], ym = uw[b - n], yp = uw[b + n];
        T acc = T(0);
        if (NDIM == 3) {
            acc += (f & 4) ? zl[k] : T(0);
            acc += (f & 8) ? zr[k] : T(0);
        }
        acc += (v && i > 0) ? wm : T(0);
        acc += (v && i < n - 1) ? wp : T(0);
        acc += (f & 1) ? ym : T(0);
        acc += (f & 2) ? yp : T(0);
        const T sk = PP ? sv[k] : s0;
        const T dk = T(2) * sk * (acc - T(2 * NDIM) * c);
        if (v) {
            const int q = staged_pos<M>(ll, i, ls);
            sh[q] = dk;
            if (PP) ss[q] = sk;
        }
    }
    __syncthreads();
    T ra[M], rb[M], rc[M], rd[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const int gi = p * M + k;
        const bool v = act && gi < n;
        const T dk = sh[pos + k];  // own tile slots: always inside the regions
        const T sl = PP ? ss[pos + k] : s0;
        rd[k] = v ? dk : T(0);
        const T sk = v ? sl : T(0);
        ra[k] = (gi > 0) ? -sk : T(0);
        rb[k] = T(1) + T(2) * sk;
        rc[k] = (gi < n - 1) ? -sk : T(0);
    }
    T uu[M];
    if (WV) {
        TileState<T, M> ts;
        tile_eliminate<T, M>(ra, rb, rc, rd, ts);
        T f, lv;
        reduced_pcr_lanes<T>(ts, p, P, f, lv);
        tile_backsub<T, M>(ts, f, lv, uu);
    } else {
        tile_solve<T, M>(ra, rb, rc, rd, red, L * P, P, p, t, 1, uu);
    }
    // each thread overwrites only the slots it read itself (no other thread
    // reads them before the barrier below)
    if (act) {
#pragma unroll
        for (int k = 0; k < M; ++k) sh[pos + k] = uu[k];
    }
    __syncthreads();
    stage_out_all<T, M>(x + off, sh, cnt, n, ls);
}

// Per-point s with lines of exactly P tiles of 8 rows (P a power of two up to
// 64, or 6, 10, 12, 14 with whole lines per wavefront): the stencil part L u
// is staged by the register-window source of the constant-row kernels (y
// neighbours from the thread's own previous and next line, x neighbours by
// lane moves, z neighbours and the rows by 16-byte loads, no LDS window), s
// is read by each thread for its own tile with 16-byte loads, and the rows
// (-s, 1 + 2 s, -s) and d = 2 s L u are formed in registers.  One barrier
// before the solve, one before the 16-byte stores of the result.
template <typename T, int M, int P, int NDIM>
__global__ __launch_bounds__(256) void k_rhs_pp(ConstStagedGeom g, CStgRhs<T, NDIM> src, const T *__restrict__ s,
                                                T *__restrict__ out) {
    using VT = typename Vec<T>::type;
    constexpr int V = Vec<T>::n;
    static_assert(M % V == 0 && M >= 3, "tiles of whole 16-byte vectors");
    constexpr bool LANES = (P & (P - 1)) != 0;
    static_assert(P <= 64, "a line's tiles stay in one wavefront");
    constexpr int n = P * M;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    const int L = g.L, t = threadIdx.x;
    int p, l;
    bool lane_ok = true;
    if constexpr (LANES) {
        constexpr int G = 64 / P;
        const int j = t & 63;
        p = j % P;
        l = (t >> 6) * G + j / P;
        lane_ok = j < G * P;
    } else {
        p = t % P;
        l = t / P;
    }
    const i64 o0 = staged_block_origin(g, xcd_block_id());
    const int nl = (int)((g.nlines - o0) < (i64)L ? (g.nlines - o0) : (i64)L);
    const bool act = lane_ok && l < nl;
    // s of the thread's own tile (idle threads read the block's first tile)
    VT sv4[M / V];
    {
        const VT *s4 = reinterpret_cast<const VT *>(s + (o0 + (act ? l : 0)) * n + (act ? p * M : 0));
#pragma unroll
        for (int q = 0; q < M / V; ++q) sv4[q] = s4[q];
    }
    src.template stage<M, n, LANES>(sh, g, o0, nl, nullptr);
    __syncthreads();
    const int pos = (act ? l : 0) * g.ls + p * (M + 1);
    T sk[M], rd[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const T sv = vget<T>(sv4[k / V], k % V);
        const T lu = sh[pos + k];
        sk[k] = act ? sv : T(0);
        rd[k] = act ? T(2) * sv * lu : T(0);
    }
    auto rows = [&](int k, T &a, T &b, T &c) {
        const int gi = p * M + k;
        a = gi > 0 ? -sk[k] : T(0);
        b = T(1) + T(2) * sk[k];
        c = gi < n - 1 ? -sk[k] : T(0);
    };
    TileState<T, M> ts;
    tile_eliminate_fn<T, M>(rows, rd, ts);
    T f, lv;
    if constexpr (LANES)
        reduced_pcr_lanes<T>(ts, p, P, f, lv);
    else if constexpr (P <= 16)
        reduced_pcr_dpp<T, M, P>(ts, p, f, lv);
    else
        reduced_pcr_wave<T, M, P>(ts, p, f, lv);
    T uu[M];
    tile_backsub<T, M>(ts, f, lv, uu);
    if (act) {
#pragma unroll
        for (int k = 0; k < M; ++k) sh[pos + k] = uu[k];
    }
    __syncthreads();
    const int nc = nl * n / V;
    VT *dst = reinterpret_cast<VT *>(out + o0 * n);
#pragma unroll
    for (int k = 0; k < M / V; ++k) {
        const int ch = t + k * 256;
        if (ch < nc) {
            const int e = ch * V, ll = e / n, i = e - ll * n;
            const T *sp = sh + ll * g.ls + (i / M) * (M + 1) + (i % M);
            VT v;
            T *vp = reinterpret_cast<T *>(&v);
#pragma unroll
            for (int q = 0; q < V; ++q) vp[q] = sp[q];
            dst[ch] = v;
        }
    }
}

namespace {

constexpr int kMaxThreads = 256;
constexpr int kPpM = 8;  // tile rows of k_rhs_pp

i64 cdiv(i64 a, i64 b) { return (a + b - 1) / b; }

// Lines per block of k_rhs_pp: 256 / P, or 4 (64 / P) whole lines per
// wavefront, within the lines the staging source's thread groups cover (each
// group of C = n / VB threads stages LG = M / VB lines, VB = one or two
// 16-byte vectors).  0 when the source cannot stage them.
int pp_lines(int n, int P, int w) {
    const int V = 16 / w;
    const int VB = (n / V > 64 ? 2 : 1) * V;
    const int C = n / VB, LG = kPpM / VB;
    if (C < 1 || C > 256 || LG < 1) return 0;
    const int staged = (256 / C) * LG;
    const bool lanes = (P & (P - 1)) != 0;
    const int L = lanes ? std::min(4 * (64 / P), staged) : 256 / P;
    return L <= staged ? L : 0;
}

bool pp_supported_P(i64 P) {
    switch (P) {
        case 4: case 6: case 8: case 10: case 12: case 14: case 16: case 32: case 64: return true;
        default: return false;
    }
}

template <typename T, int P, int NDIM>
hipError_t go_pp(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    ConstStagedGeom g;
    g.nlines = r.ny * r.nz * r.batch;
    g.n = (int)r.nx;
    g.L = pl.L;
    g.ls = pl.ls;
    CStgRhs<T, NDIM> src{static_cast<const T *>(r.u), T(1), (int)r.ny, NDIM == 3 ? (int)r.nz : 1};
    src.block_order(g);
    launch(k_rhs_pp<T, kPpM, P, NDIM>, dim3((unsigned)pl.nblocks), dim3(256), pl.shmem, s, g, src,
           static_cast<const T *>(r.s), static_cast<T *>(r.d));
    return hipGetLastError();
}

template <typename T, int NDIM>
hipError_t go_pp_p(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    switch (pl.P) {
        case 4: return go_pp<T, 4, NDIM>(r, pl, s);
        case 6: return go_pp<T, 6, NDIM>(r, pl, s);
        case 8: return go_pp<T, 8, NDIM>(r, pl, s);
        case 10: return go_pp<T, 10, NDIM>(r, pl, s);
        case 12: return go_pp<T, 12, NDIM>(r, pl, s);
        case 14: return go_pp<T, 14, NDIM>(r, pl, s);
        case 16: return go_pp<T, 16, NDIM>(r, pl, s);
        case 32: return go_pp<T, 32, NDIM>(r, pl, s);
        case 64: return go_pp<T, 64, NDIM>(r, pl, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t go_pp_t(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    return r.ndim == 3 ? go_pp_p<T, 3>(r, pl, s) : go_pp_p<T, 2>(r, pl, s);
}

bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// k_rhs_pp takes per-point s, lines of exactly P tiles of 8 rows with a
// supported P, 16-byte aligned arrays and 32-bit byte offsets (the staging
// source's addressing).
bool plan_pp(const AdiReq &r, LinePlan *pl) {
    const int w = r.f64 ? 8 : 4;
    if (!r.s || (r.force_M && r.force_M != kPpM) || r.nx % kPpM) return false;
    if (r.nx * r.ny * r.nz * r.batch * w >= ((i64)1 << 32)) return false;
    if (!aligned16(r.u) || !aligned16(r.s) || !aligned16(r.d)) return false;
    const i64 P = r.nx / kPpM;
    if (!pp_supported_P(P)) return false;
    const bool lanes = (P & (P - 1)) != 0;
    int L = pp_lines((int)r.nx, (int)P, w);
    if (!L) return false;
    if (lanes && r.force_L > 0 && r.force_L < L) L = r.force_L;  // fewer whole lines per wavefront
    LinePlan p;
    p.M = kPpM;
    p.P = (int)P;
    p.L = L;
    p.staged = true;
    p.vec = true;
    p.lanes = lanes;
    p.ls = (int)P * (kPpM + 1);
    p.shmem = (size_t)L * p.ls * w;
    p.nblocks = cdiv(r.ny * r.nz * r.batch, L);
    if (p.nblocks >= (i64)1 << 31) return false;
    *pl = p;
    return true;
}
constexpr size_t kMaxShmem = 160 * 1024;

// LDS layout (elements): [staged RHS L*ls][u window (L+2)*n][staged s L*ls,
// per-point s only][reduced scratch: 6*L*P unless the lines' reduced systems
// are solved by lane moves, and at least L ints of flags], regions 16-byte
// aligned.
size_t rhs_layout(int L, int P, int ls, int n, bool pp, bool lanes, int w, int *uoff, int *soff, int *roff) {
    const int q = 16 / w;
    auto up = [&](i64 v) { return (v + q - 1) / q * q; };
    const i64 u0 = up((i64)L * ls);
    const i64 s0 = up(u0 + (i64)(L + 2) * n);
    const i64 r0 = pp ? up(s0 + (i64)L * ls) : s0;
    const i64 red = std::max(lanes ? (i64)0 : (i64)6 * L * P, cdiv((i64)L * 4, w));
    if (uoff) *uoff = (int)u0;
    if (soff) *soff = (int)s0;
    if (roff) *roff = (int)r0;
    return (size_t)(r0 + red) * w;
}

template <typename T, int M, bool PP, int NDIM, bool WV>
hipError_t go(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    RhsGeom g;
    g.nlines = r.ny * r.nz * r.batch;
    g.n = (int)r.nx;
    g.L = pl.L;
    g.P = pl.P;
    g.ls = pl.ls;
    g.ny = (int)r.ny;
    g.nz = (int)r.nz;
    rhs_layout(pl.L, pl.P, pl.ls, g.n, PP, WV, (int)sizeof(T), &g.uoff, &g.soff, &g.roff);
    auto kern = k_rhs_x<T, M, PP, NDIM, WV>;
    if (pl.shmem > 64 * 1024) {
        static bool raised = false;  // one attribute call per instantiation
        if (!raised) {
            hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)kMaxShmem);
            if (e != hipSuccess) return e;
            raised = true;
        }
    }
    launch(kern, dim3((unsigned)pl.nblocks), dim3(pl.threads()), pl.shmem, s, g,
                       static_cast<const T *>(r.u), static_cast<const T *>(r.s), (T)r.s0,
                       static_cast<T *>(r.d));
    return hipGetLastError();
}

template <typename T, int M, bool WV>
hipError_t go_m(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    const bool pp = r.s != nullptr;
    if (r.ndim == 3) return pp ? go<T, M, true, 3, WV>(r, pl, s) : go<T, M, false, 3, WV>(r, pl, s);
    return pp ? go<T, M, true, 2, WV>(r, pl, s) : go<T, M, false, 2, WV>(r, pl, s);
}

template <typename T>
hipError_t go_t(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    switch (pl.M) {
        case 8: return pl.lanes ? go_m<T, 8, true>(r, pl, s) : go_m<T, 8, false>(r, pl, s);
        case 16: return pl.lanes ? go_m<T, 16, true>(r, pl, s) : go_m<T, 16, false>(r, pl, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool plan_rhs_x(const AdiReq &r, LinePlan *pl, std::string *err) {
    if (plan_pp(r, pl)) return true;
    const int w = r.f64 ? 8 : 4;
    LinePlan p;
    // 8-row tiles: the block then holds few enough lines that several blocks
    // share a CU (measured faster than 16 rows in both precisions)
    int M = r.force_M ? r.force_M : (cdiv(r.nx, 8) <= kMaxThreads ? 8 : 16);
    if (M != 8 && M != 16) {
        *err = "fused stencil + x solve supports tiles of 8 or 16 rows";
        return false;
    }
    const i64 P = cdiv(r.nx, M);
    if (P > kMaxThreads) {
        *err = "x lines too long for the fused stencil + x solve";
        return false;
    }
    const int ls = (int)P * (M + 1);
    // lines of P tiles, P not a power of two, at most 64: whole lines per
    // wavefront (reduced systems by lane moves); otherwise P threads per line
    const bool lanes = P <= 64 && (P & (P - 1)) != 0;
    const int Lmax = lanes ? (kMaxThreads / 64) * (64 / (int)P) : kMaxThreads / (int)P;
    int L = r.force_L ? r.force_L : std::max(1, Lmax);
    const bool pp = r.s != nullptr;
    auto bytes = [&](int LL) {
        return rhs_layout(LL, (int)P, ls, (int)r.nx, pp, lanes, w, nullptr, nullptr, nullptr);
    };
    while (bytes(L) > kMaxShmem && L > 1) L /= 2;
    if (bytes(L) > kMaxShmem || L > Lmax) {
        *err = "fused stencil + x solve does not fit in LDS";
        return false;
    }
    p.M = M;
    p.P = (int)P;
    p.L = L;
    p.staged = true;
    p.lanes = lanes;
    p.ls = ls;
    p.shmem = bytes(L);
    p.nblocks = cdiv(r.ny * r.nz * r.batch, L);
    if (p.nblocks >= (i64)1 << 31) {
        *err = "too many blocks";
        return false;
    }
    *pl = p;
    return true;
}

hipError_t launch_rhs_x(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    if (pl.vec) return r.f64 ? go_pp_t<double>(r, pl, s) : go_pp_t<float>(r, pl, s);
    return r.f64 ? go_t<double>(r, pl, s) : go_t<float>(r, pl, s);
}

}  // namespace trid
