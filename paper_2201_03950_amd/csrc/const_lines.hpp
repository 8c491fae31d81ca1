// const_lines.hpp -- line solves whose rows are the same (a, b, c) everywhere
// (the in-kernel coefficient generation of Section IV-A; Alg. 3 with a
// constant diffusion number).
//
// With constant rows every coefficient of the tiled modified Thomas sweep
// (eq. (7)) and of the reduced system is the same for every line: only the
// right-hand side differs.  The host therefore runs the coefficient part of the
// elimination once, in FP64, and passes it as kernel arguments:
//   - per tile row k: the forward multipliers, the backward factors and the
//     back-substitution factors of eq. (7);
//   - the reduced system over the P tiles' first unknowns, already inverted:
//     f = W1 * fd + W2 * ld, where fd / ld are the tiles' first-row and
//     last-row right-hand sides.  P <= 8 so the inverse is a tiny dense matrix.
// Per point the kernel then does about five FMAs, and each block needs a single
// LDS exchange (all tiles' fd, ld) with one barrier.
//
// Requirements (checked by the planner): n = P * M exactly, P <= 8.
#pragma once

#include "lines.hpp"

namespace trid {

constexpr int kConstMaxM = 32;
constexpr int kConstMaxP = 8;

template <typename T>
struct ConstTab {
    T rr[kConstMaxM];   // forward reciprocal of row k (k >= 1)
    T am[kConstMaxM];   // rr[k] * a (k >= 2)
    T cpf[kConstMaxM];  // forward super-diagonal factor c'_k (k = 1..M-2)
    T apb[kConstMaxM];  // back-substitution factor of u_0 (k = 1..M-2)
    T cpb[kConstMaxM];  // back-substitution factor of u_{M-1} (k = 1..M-2)
    // f_p = sum_q w1[p][q] fd_q + w2[p][q] ld_q; row kConstMaxP is an all-zero
    // row so that "row p + 1" of the last tile reads zeros
    T w1[(kConstMaxP + 1) * kConstMaxP];
    T w2[(kConstMaxP + 1) * kConstMaxP];
    T c;   // super-diagonal (first-row elimination)
    T la;  // last row: coefficient of the tile's first unknown
    T lc;  // last row: coefficient of the next tile's first unknown (0 for the last tile)
    int P;
};

// Host: fill the tables for rows (a, b, c), tiles of M rows, P = n / M tiles.
// Returns false if the reduced system is singular.
template <typename T>
bool make_const_tab(double a, double b, double c, int M, int P, ConstTab<T> *t);

// Forward / backward sweep of one tile (eq. (7)) with tabulated coefficients.
// x holds the tile's right-hand sides on entry and d'_k on return (x[0] keeps
// the raw first row's rhs); returns fd and ld, the reduced rows' rhs.
template <typename T, int M, class Tab>
__device__ __forceinline__ void const_tile_sweep(const Tab &tb, T (&x)[M], T &fd, T &ld) {
    x[1] = tb.rr[1] * x[1];
#pragma unroll
    for (int k = 2; k < M; ++k) x[k] = tb.rr[k] * x[k] - tb.am[k] * x[k - 1];
    ld = x[M - 1];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) x[k] -= tb.cpf[k] * x[k + 1];
    fd = x[0] - tb.c * x[1];
}

// Back substitution once f (tile's first unknown) and fn (next tile's) are known.
template <typename T, int M>
__device__ __forceinline__ void const_tile_backsub(const ConstTab<T> &tb, T f, T fn, bool last,
                                                   T (&x)[M]) {
    const T lv = x[M - 1] - tb.la * f - (last ? T(0) : tb.lc) * fn;
    x[0] = f;
    x[M - 1] = lv;
#pragma unroll
    for (int k = 1; k < M - 1; ++k) x[k] = x[k] - tb.apb[k] * f - tb.cpb[k] * lv;
}

// ---------------------------------------------------------------- strided --
// y / z lines: 64 lanes = 64 adjacent lines, wavefront w = tile w (uniform, so
// every table read is a scalar load).  Block = 64 lines x P tiles.  Lines are
// numbered across outer indices (line j: outer j / inner, inner j % inner), so
// when inner is not a multiple of 64 a block runs on past the last line of one
// outer index into the next instead of leaving lanes idle (the planner keeps
// inner * outer below 2^31).

template <typename T, int M, class Epi>
__global__ __launch_bounds__(64 * kConstMaxP) void k_strided_const(StridedGeom gm, ConstTab<T> tb,
                                                                  const T *__restrict__ d, Epi epi) {
    __shared__ T sfd[kConstMaxP * 64], sld[kConstMaxP * 64];
    const int l = threadIdx.x & 63;
    const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int P = tb.P;
    // the block's first line is split by one scalar division; a lane moves on
    // by at most one outer index when inner >= 64
    const unsigned in = (unsigned)gm.inner;
    const unsigned j0 = (unsigned)xcd_block_id() * 64u;
    const unsigned ob0 = j0 / in, ii0 = j0 - ob0 * in;
    const bool act = j0 + (unsigned)l < gm.lines;
    unsigned ob = ob0, ii = ii0 + (unsigned)l;
    if (in >= 64u) {
        if (ii >= in) {
            ii -= in;
            ++ob;
        }
    } else {
        ob += ii / in;
        ii %= in;
    }
    if (!act) ob = ii = 0u;
    const i64 st = gm.inner;
    const i64 base = (i64)ob * (i64)gm.n * st + ii;
    const int g0 = p * M;
    // rows of one tile lie within one slab of n * inner < 2^31 elements (planner):
    // 32-bit offsets from the tile's first row
    const unsigned sst = (unsigned)st;
    const T *dp = d + base + (i64)g0 * st;
    T x[M];
#pragma unroll
    for (int k = 0; k < M; ++k) x[k] = act ? dp[k * sst] : T(0);
    T fd, ld;
    const_tile_sweep<T, M>(tb, x, fd, ld);
    sfd[p * 64 + l] = fd;
    sld[p * 64 + l] = ld;
    __syncthreads();
    T f = T(0), fn = T(0);
    const T *w1 = tb.w1 + p * kConstMaxP, *w2 = tb.w2 + p * kConstMaxP;
#pragma unroll
    for (int q = 0; q < kConstMaxP; ++q) {
        if (q < P) {
            const T vf = sfd[q * 64 + l], vl = sld[q * 64 + l];
            f += w1[q] * vf + w2[q] * vl;
            fn += w1[q + kConstMaxP] * vf + w2[q + kConstMaxP] * vl;  // row p+1 (zero past the end)
        }
    }
    const_tile_backsub<T, M>(tb, f, fn, p == P - 1, x);
    epi.template store_rows<M>(base + (i64)g0 * st, sst, act, x);
}

// ----------------------------------------------------------------- staged --
// x lines: L lines x P tiles per block, thread t -> tile p = t % P of line
// l = t / P.  A source stages the block's right-hand sides into LDS (tiles
// padded to M + 1 elements, against bank conflicts); results leave through the
// same region with 16-byte stores.

struct ConstStagedGeom {
    i64 nlines;
    int n, L, ls;
    // Block order of the 3D stencil sources (Y = 0: block b takes lines
    // b L ..).  With Y = ny / L blocks per plane, each mesh's planes are taken
    // in slabs of zc planes, and inside a slab the blocks of one y range run
    // through the slab's planes one after another: a block's z-neighbour rows
    // are the rows the previous and next block stage, and its y-neighbour rows
    // those of the blocks zc places away, so the L2 of the XCD that runs a
    // contiguous range of blocks serves them instead of HBM.
    int Y = 0, ny = 1, nz = 1, zc = 1;
};

// First line of logical block b (see ConstStagedGeom).
__device__ __forceinline__ i64 staged_block_origin(const ConstStagedGeom &g, i64 b) {
    if (g.Y == 0) return b * g.L;
    const i64 per_mesh = (i64)g.Y * g.nz;
    const i64 m = b / per_mesh;
    const int bm = (int)(b - m * per_mesh);
    const int slab = bm / (g.Y * g.zc);
    const int r = bm - slab * g.Y * g.zc;
    const int z0 = slab * g.zc;
    const int zc = g.nz - z0 < g.zc ? g.nz - z0 : g.zc;
    const int yb = r / zc, z = z0 + (r - yb * zc);
    return (m * g.nz + z) * (i64)g.ny + (i64)yb * g.L;
}

// Vector width (elements per 16-byte access).
template <typename T>
struct Vec;
template <>
struct Vec<double> {
    using type = double2;
    static constexpr int n = 2;
};
template <>
struct Vec<float> {
    using type = float4;
    static constexpr int n = 4;
};

template <typename T>
__device__ __forceinline__ T vget(const typename Vec<T>::type &v, int j);
template <>
__device__ __forceinline__ double vget<double>(const double2 &v, int j) {
    return j == 0 ? v.x : v.y;
}
template <>
__device__ __forceinline__ float vget<float>(const float4 &v, int j) {
    return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

// Plain right-hand side: copy d's block into LDS with 16-byte loads.
template <typename T>
struct CStgCopy {
    const T *d;
    void block_order(ConstStagedGeom &) const {}  // independent lines: natural order
    template <int M, int N, bool GUARD = false>
    __device__ __forceinline__ void stage(T *__restrict__ sh, const ConstStagedGeom &g, i64 o0, int nl,
                                          int *) const {
        using VT = typename Vec<T>::type;
        constexpr int V = Vec<T>::n;
        constexpr int n = N;
        const int nc = nl * n / V, nt = blockDim.x;
        const VT *src = reinterpret_cast<const VT *>(d + o0 * n);
        VT v[M / V];
#pragma unroll
        for (int k = 0; k < M / V; ++k) {
            const int ch = threadIdx.x + k * nt;
            v[k] = load_if(src, ch, ch < nc, nc - 1);
        }
#pragma unroll
        for (int k = 0; k < M / V; ++k) {
            const int ch = threadIdx.x + k * nt;
            if (ch < nc) {
                const int e = ch * V, ll = e / n, i = e - ll * n;
                T *dst = sh + ll * g.ls + (i / M) * (M + 1) + (i % M);
#pragma unroll
                for (int j = 0; j < V; ++j) dst[j] = vget<T>(v[k], j);
            }
        }
    }
};

// Right-hand side of the ADI step, d = 2 s0 (sum of neighbours - 2 NDIM u),
// zero outside the mesh, computed while staging.  Thread t owns VB consecutive
// x elements (one or two 16-byte vectors: VB is chosen so that a line row
// spans at most one wavefront, C = N / VB <= 64 lanes) of LG = M / VB
// consecutive lines, so
//   - the y neighbours of its lines are its own previous / next line (a
//     sliding window in registers; only the two halo lines are extra loads),
//   - the x neighbours across its VB elements come from the adjacent lanes
//     (DPP wave shifts); when a line row fills whole wavefronts, the first
//     and last lanes of a row are the line ends and no other load is needed,
//   - the z neighbours are coalesced vector loads.
// Offsets are 32-bit byte offsets from the array start (the planner keeps the
// array below 4 GB), so loads use a scalar base and one VGPR offset.  The
// planner guarantees N = P * M, blockDim = 256 = L * P, and 256 / C thread
// groups of LG lines cover the block's L lines.
template <typename T>
__device__ __forceinline__ T wave_from_lower_lane(T v) {  // lane i <- lane i - 1 (lane 0: 0)
    return dpp_move<0x138>(v);
}
template <typename T>
__device__ __forceinline__ T wave_from_upper_lane(T v) {  // lane i <- lane i + 1 (lane 63: 0)
    return dpp_move<0x130>(v);
}

template <typename T, int NV>
struct Cols {  // VB = NV * V consecutive elements of one line row
    typename Vec<T>::type v[NV];
    __device__ __forceinline__ T operator[](int e) const { return vget<T>(v[e / Vec<T>::n], e % Vec<T>::n); }
};

template <typename T, int NDIM>
struct CStgRhs {
    const T *u;
    T s2;  // 2 s0
    int ny, nz;
    // Host: slab block order (ConstStagedGeom) for 3D meshes whose planes hold
    // whole blocks; slabs of up to 64 planes.
    void block_order(ConstStagedGeom &g) const {
        if (NDIM != 3 || nz < 2 || ny % g.L) return;
        g.Y = ny / g.L;
        g.ny = ny;
        g.nz = nz;
        g.zc = nz < 64 ? nz : 64;
    }
    template <int M, int N, bool GUARD = false>
    __device__ __forceinline__ void stage(T *__restrict__ sh, const ConstStagedGeom &g, i64 o0, int nl,
                                          int *) const {
        using VT = typename Vec<T>::type;
        constexpr int V = Vec<T>::n;
        constexpr int NV = (N / V > 64) ? 2 : 1;  // 16-byte vectors per thread and row
        constexpr int VB = NV * V;                // elements per thread and row
        constexpr int C = N / VB;                 // threads per line row
        constexpr bool kEdges = !(C <= 64 && 64 % C == 0);  // rows straddle wavefronts
        constexpr int LG = M / VB;                // lines per thread
        static_assert(M % VB == 0 && N % VB == 0, "a thread's elements stay in one tile");
        const int t = threadIdx.x, c = t % C, grp = t / C;
        const int lane = t & 63;
        const int lfirst = grp * LG;  // first block line of this thread
        // (j, k) of the block's first line: one uniform division per block
        const unsigned o0u = (unsigned)o0;
        const unsigned plane0 = __builtin_amdgcn_readfirstlane(o0u / (unsigned)ny);
        int j = (int)(o0u - plane0 * (unsigned)ny) + lfirst, k = (int)(plane0 % (unsigned)nz);
        while (j >= ny) {
            j -= ny;
            k = (k + 1 == nz) ? 0 : k + 1;
        }
        const bool live0 = lfirst < nl;
        // neighbour existence of the thread's lines (no loads involved)
        bool jp[LG], jn[LG], kp[LG], kn[LG];
        {
            int jj = j, kk = k;
#pragma unroll
            for (int r = 0; r < LG; ++r) {
                jp[r] = jj > 0;
                jn[r] = jj < ny - 1;
                kp[r] = kk > 0;
                kn[r] = kk < nz - 1;
                if (++jj == ny) {  // the next line starts a new plane
                    jj = 0;
                    kk = (kk + 1 == nz) ? 0 : kk + 1;
                }
            }
        }
        // byte offsets: this thread's column in the block's first line, the
        // block's last line (in bounds for every lane: idle lanes read it)
        constexpr unsigned W = sizeof(T), RB = N * sizeof(T);
        const unsigned col0 = (o0u * N + (unsigned)(c * VB)) * W;
        const unsigned safe = col0 + (unsigned)(nl - 1) * RB;
        const unsigned zb = (unsigned)ny * RB;
        const char *ub = reinterpret_cast<const char *>(u);
        auto rowld = [&](Cols<T, NV> &dst, unsigned off, bool ok) {
            const unsigned o = ok ? off : safe;
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const VT v = *reinterpret_cast<const VT *>(ub + (o + q * 16u));
                dst.v[q] = ok ? v : VT{};
            }
        };
        auto eld = [&](unsigned off, bool ok) -> T {
            const T v = *reinterpret_cast<const T *>(ub + (ok ? off : safe));
            return ok ? v : T(0);
        };
        // sliding window over lines lfirst-1 .. lfirst+LG (y neighbours).  The
        // rows go in chunks of CH: all loads of a chunk are issued before any of
        // its arithmetic.
        Cols<T, NV> cur, prev;
        rowld(cur, col0 + (unsigned)lfirst * RB, live0);
        rowld(prev, col0 + (unsigned)lfirst * RB - RB, live0 && jp[0]);
        constexpr int CH = (LG * NV <= 4) ? LG : (4 / NV > 0 ? 4 / NV : 1);
#pragma unroll
        for (int c0 = 0; c0 < LG; c0 += CH) {
            Cols<T, NV> nx[CH], zm[CH], zp[CH];
            T el[CH], er[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int ll = lfirst + c0 + i;
                const bool live = ll < nl;
                const unsigned off = col0 + (unsigned)ll * RB;
                // the next line (y+1 neighbour, or the next plane's first line)
                rowld(nx[i], off + RB, live && (ll + 1 < nl || o0 + nl < g.nlines));
                if (NDIM == 3) {
                    rowld(zm[i], off - zb, live && kp[c0 + i]);
                    rowld(zp[i], off + zb, live && kn[c0 + i]);
                }
                if (kEdges) {
                    el[i] = eld(off - W, live && lane == 0 && c > 0);
                    er[i] = eld(off + VB * W, live && lane == 63 && c < C - 1);
                }
            }
            asm volatile("" ::: "memory");  // the chunk's loads stay above its arithmetic
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const int r = c0 + i, ll = lfirst + r;
                // x neighbours of the thread's first and last element
                T left = wave_from_lower_lane<T>(cur[VB - 1]);
                T right = wave_from_upper_lane<T>(cur[0]);
                if (kEdges) {
                    if (lane == 0) left = el[i];
                    if (lane == 63) right = er[i];
                }
                if (c == 0) left = T(0);
                if (c == C - 1) right = T(0);
                // ll < L when the thread groups tile the block's L lines exactly
                // (rows past nl are written but never read, so the store needs no
                // branch); GUARD: groups past the block's L lines store nothing
                T *dst = sh + ll * g.ls + ((c * VB) / M) * (M + 1) + ((c * VB) % M);
                if (!GUARD || ll < g.L) {
#pragma unroll
                    for (int e = 0; e < VB; ++e) {
                        T acc = (jn[r] ? nx[i][e] : T(0)) + (jp[r] ? prev[e] : T(0));
                        if (NDIM == 3) acc += zm[i][e] + zp[i][e];
                        const T xl = e == 0 ? left : cur[e - 1];
                        const T xr = e == VB - 1 ? right : cur[e + 1];
                        dst[e] = s2 * (acc + xl + xr - T(2 * NDIM) * cur[e]);
                    }
                }
                prev = cur;
                cur = nx[i];
            }
        }
    }
};

// ------------------------------------------------------ staged, DPP PCR --
// x lines with P = n / M a power of two <= 16: the P tiles of a line are P
// adjacent lanes inside one 16-lane DPP row, so the reduced system over the
// tiles' first unknowns is solved by PCR (Alg. 2) with row shifts of the
// wavefront (no LDS, no barrier).  Its coefficients do not depend on the line
// and come tabulated per (level, tile); only right-hand sides move.

constexpr int kDppMaxP = 16;
constexpr int kDppLevels = 4;

template <typename T>
struct PcrTab {
    T rr[kConstMaxM], am[kConstMaxM], cpf[kConstMaxM], apb[kConstMaxM], cpb[kConstMaxM];
    T c, la, lc;
    // G row of tile p: gd = rg fd - gA ld_{p-1} - gC ld_p (normalised, b = 1)
    T rg[kDppMaxP], gA[kDppMaxP], gC[kDppMaxP];
    // PCR level j (stride 2^j): d = pr d - pa d_{p-s} - pc d_{p+s}
    T pr[kDppLevels][kDppMaxP], pa[kDppLevels][kDppMaxP], pc[kDppLevels][kDppMaxP];
};

template <typename T>
bool make_pcr_tab(double a, double b, double c, int M, int P, PcrTab<T> *t);

template <typename T, int P, int S>
struct PcrLevels {
    __device__ __forceinline__ static void run(const PcrTab<T> &tb, int p, T &d) {
        if constexpr (S < P) {
            constexpr int j = (S == 1) ? 0 : (S == 2) ? 1 : (S == 4) ? 2 : 3;
            T dm = row_from_lower<S>(d);
            T dn = row_from_upper<S>(d);
            if (P < 16) {  // rows hold several lines: mask neighbours of other lines
                dm = (p >= S) ? dm : T(0);
                dn = (p + S < P) ? dn : T(0);
            }
            d = tb.pr[j][p] * d - tb.pa[j][p] * dm - tb.pc[j][p] * dn;
            PcrLevels<T, P, 2 * S>::run(tb, p, d);
        }
    }
};

template <typename T, int M, int P, class Src>
__global__ __launch_bounds__(256) void k_staged_dpp(ConstStagedGeom g, PcrTab<T> tb, Src src,
                                                    T *__restrict__ out) {
    static_assert(P >= 1 && P <= 16 && (P & (P - 1)) == 0, "P must be a power of two <= 16");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    constexpr int n = P * M;  // the planner only sends lines of exactly P tiles
    const int L = g.L;
    int *flags = reinterpret_cast<int *>(sh + L * g.ls);
    const int t = threadIdx.x, p = t % P, l = t / P;
    const i64 o0 = staged_block_origin(g, xcd_block_id());
    const int nl = (int)((g.nlines - o0) < (i64)L ? (g.nlines - o0) : (i64)L);
    src.template stage<M, n>(sh, g, o0, nl, flags);
    __syncthreads();
    const bool act = l < nl;
    const int pos = l * g.ls + p * (M + 1);
    T x[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const T val = sh[pos + k];  // own tile slot: always inside the region
        x[k] = act ? val : T(0);
    }
    T fd, ld;
    const_tile_sweep<T, M>(tb, x, fd, ld);
    T ldp = row_from_lower<1>(ld);
    if (P < 16) ldp = (p >= 1) ? ldp : T(0);
    T d = tb.rg[p] * fd - tb.gA[p] * ldp - tb.gC[p] * ld;
    PcrLevels<T, P, 1>::run(tb, p, d);
    const T f = d;
    T fn = row_from_upper<1>(f);
    if (P < 16) fn = (p + 1 < P) ? fn : T(0);
    const T lv = x[M - 1] - tb.la * f - ((p == P - 1) ? T(0) : tb.lc) * fn;
    x[0] = f;
    x[M - 1] = lv;
#pragma unroll
    for (int k = 1; k < M - 1; ++k) x[k] = x[k] - tb.apb[k] * f - tb.cpb[k] * lv;
#pragma unroll
    for (int k = 0; k < M; ++k) sh[pos + k] = x[k];
    __syncthreads();
    using VT = typename Vec<T>::type;
    constexpr int V = Vec<T>::n;
    const int nc = nl * n / V;
    VT *dst = reinterpret_cast<VT *>(out + o0 * n);
#pragma unroll
    for (int k = 0; k < M / V; ++k) {
        const int ch = t + k * (int)blockDim.x;
        if (ch < nc) {
            const int e = ch * V, ll = e / n, i = e - ll * n;
            const T *sp = sh + ll * g.ls + (i / M) * (M + 1) + (i % M);
            VT v;
            T *vp = reinterpret_cast<T *>(&v);
#pragma unroll
            for (int j = 0; j < V; ++j) vp[j] = sp[j];
            dst[ch] = v;
        }
    }
}

// ---------------------------------------------------- staged, lane PCR --
// x lines of P = n / M tiles, P in {3, 5, 6, 7} (Table 3's 48- to 112-point
// lines): 64 / P whole lines per wavefront, the wavefront's last 64 % P lanes
// idle, and the reduced system solved by PCR (Alg. 2) with lane moves through
// the LDS crossbar and the same tabulated coefficients -- no barrier.  256
// threads, L <= 4 (64 / P) lines per block (the planner also keeps L within
// the lines the source's thread groups stage).
template <typename T, int M, int P, class Src>
__global__ __launch_bounds__(256) void k_staged_lanes(ConstStagedGeom g, PcrTab<T> tb, Src src,
                                                      T *__restrict__ out) {
    static_assert(P >= 3 && P <= 7 && (P & (P - 1)) != 0, "lane layout for P in {3, 5, 6, 7}");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sh = reinterpret_cast<T *>(smem_raw);
    constexpr int n = P * M;
    constexpr int G = 64 / P;
    const int L = g.L;
    int *flags = reinterpret_cast<int *>(sh + L * g.ls);
    const int t = threadIdx.x, j = t & 63;
    const int p = j % P, l = (t >> 6) * G + j / P;
    const i64 o0 = staged_block_origin(g, xcd_block_id());
    const int nl = (int)((g.nlines - o0) < (i64)L ? (g.nlines - o0) : (i64)L);
    src.template stage<M, n, true>(sh, g, o0, nl, flags);
    __syncthreads();
    const bool act = j < G * P && l < nl;
    const int pos = (act ? l : 0) * g.ls + p * (M + 1);
    T x[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const T val = sh[pos + k];
        x[k] = act ? val : T(0);
    }
    T fd, ld;
    const_tile_sweep<T, M>(tb, x, fd, ld);
    T ldp = lane_up(ld, 1);
    if (p == 0) ldp = T(0);
    T d = tb.rg[p] * fd - tb.gA[p] * ldp - tb.gC[p] * ld;
#pragma unroll
    for (int lev = 0, S = 1; S < P; ++lev, S <<= 1) {
        T dm = lane_up(d, S), dn = lane_down(d, S);
        if (p < S) dm = T(0);
        if (p + S >= P) dn = T(0);
        d = tb.pr[lev][p] * d - tb.pa[lev][p] * dm - tb.pc[lev][p] * dn;
    }
    const T f = d;
    T fn = lane_down(f, 1);
    if (p + 1 >= P) fn = T(0);
    const T lv = x[M - 1] - tb.la * f - ((p == P - 1) ? T(0) : tb.lc) * fn;
    x[0] = f;
    x[M - 1] = lv;
#pragma unroll
    for (int k = 1; k < M - 1; ++k) x[k] = x[k] - tb.apb[k] * f - tb.cpb[k] * lv;
    if (act) {
#pragma unroll
        for (int k = 0; k < M; ++k) sh[pos + k] = x[k];
    }
    __syncthreads();
    using VT = typename Vec<T>::type;
    constexpr int V = Vec<T>::n;
    const int nc = nl * n / V;
    VT *dst = reinterpret_cast<VT *>(out + o0 * n);
#pragma unroll
    for (int k = 0; k < M / V; ++k) {
        const int ch = t + k * (int)blockDim.x;
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

}  // namespace trid
