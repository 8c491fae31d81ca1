// tile.hpp -- device building blocks of the batched tridiagonal line solver (gfx950).
//
// Every line of N rows is cut into P tiles of M consecutive rows; one thread
// owns one tile.  Per tile, the "modified Thomas" sweep of eq. (7)
// (arxiv 2201.03950, Section III-B, larger-systems solve) expresses each
// interior unknown through the tile's first and last unknowns, keeping the
// tile in registers, so every array is read once and written once.  The 2P
// first/last unknowns of a line form a tridiagonal reduced system; one local
// elimination step turns it into a P-row system over the tiles' first unknowns,
// which the P threads of the line solve with PCR (Alg. 2) through LDS -- the
// Thomas-PCR hybrid of Section III-B.  A final substitution recovers the rows.
//
// Rows beyond the end of a line are identity rows (a = c = d = 0, b = 1), which
// leave the solution of the real rows unchanged.  a at row 0 and c at row N-1
// are never read (eq. (1)).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trid {

using i64 = int64_t;

// Workgroup id remapped so that each of the 8 XCDs (each with its own L2)
// receives one contiguous range of logical blocks: hardware dispatches
// workgroup w to XCD w % 8.  Neighbouring logical blocks (which share stencil
// halo lines) then run on the same XCD and hit the same L2.
__device__ __forceinline__ i64 xcd_block_id() {
    const unsigned G = gridDim.x, w = blockIdx.x;
    const unsigned q = G >> 3, r = G & 7u, x = w & 7u, idx = w >> 3;
    return (x < r) ? (i64)x * (q + 1) + idx : (i64)r * (q + 1) + (i64)(x - r) * q + idx;
}

// Block order for strided lines of many rows, whose consecutive blocks read
// adjacent segments of the same rows: groups of K consecutive blocks run on
// one XCD (blocks whose segments share cache lines share its L2), and
// consecutive groups go to consecutive XCDs, so the blocks dispatched
// together cover whole rows and each DRAM page is read by many of them at
// about the same time (the trailing partial round of 8 K blocks keeps its
// order).  Hardware dispatch sends block i to XCD i mod 8.
template <unsigned K>
__device__ __forceinline__ i64 xcd_group_block_id() {
    const unsigned G = gridDim.x, b = blockIdx.x, W = 8u * K;
    if (b >= G / W * W) return b;
    const unsigned x = b & 7u, r = b >> 3;
    return (i64)(r / K) * W + x * K + r % K;
}

// Reciprocal for the elimination pivots.  FP32: the hardware reciprocal
// (about 1 ulp), well inside the FP32 tolerance.  FP64: the hardware estimate
// refined by two Newton-Raphson steps r <- r + r (1 - x r), each of which
// roughly squares the relative error, giving a result within an ulp or two.
// Pivots of the diagonally dominant systems solved here are far from zero,
// infinity and the denormal range, so the scaling steps of a full IEEE divide
// are not needed.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Guarded load without a branch: every lane loads (a lane with !ok from the
// in-bounds index `safe`) and the value is selected afterwards.  A load inside
// a divergent branch makes the compiler wait for it where the branches join,
// which serialises a thread's loads; in this form they stay in flight together.
template <typename U, typename I>
__device__ __forceinline__ U load_if(const U *p, I i, bool ok, I safe) {
    const U v = p[ok ? i : safe];
    return ok ? v : U{};
}

// DPP lane moves (row shifts within 16-lane rows, wave shifts by one lane);
// lanes whose source is outside the row / wavefront receive 0.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <int S, typename T>
__device__ __forceinline__ T row_from_lower(T v) {  // value of tile p - S
    return dpp_move<0x110 + S>(v);
}
template <int S, typename T>
__device__ __forceinline__ T row_from_upper(T v) {  // value of tile p + S
    return dpp_move<0x100 + S>(v);
}

// The tile's two boundary equations (eq. (7)), all the reduced solve needs:
//   first row: fa*l_{p-1} + fb*f_p + fc*l_p = fd   (f_p, l_p: tile's first/last unknown)
//   last row:  la*f_p + l_p + lc*f_{p+1} = ld
template <typename T>
struct TileEnds {
    T fa, fb, fc, fd;
    T la, lc, ld;
};

// Result of the per-tile sweep: the boundary equations and the interior
//   ap[k]*f_p + u_k + cp[k]*l_p = dp[k], k = 1..M-2
template <typename T, int M>
struct TileState : TileEnds<T> {
    T ap[M], cp[M], dp[M];
};

// Forward then backward sweep of the modified Thomas algorithm on one tile.
// Inputs are the raw rows (sub, diag, super, rhs) of the tile's M rows.
template <typename T, int M>
__device__ __forceinline__ void tile_eliminate(const T (&ra)[M], const T (&rb)[M], const T (&rc)[M],
                                               const T (&rd)[M], TileState<T, M> &s) {
    static_assert(M >= 3, "tiles need at least three rows");
    const T r1 = fast_rcp(rb[1]);
    s.ap[1] = ra[1] * r1;
    s.cp[1] = rc[1] * r1;
    s.dp[1] = rd[1] * r1;
#pragma unroll
    for (int k = 2; k < M; ++k) {
        const T r = fast_rcp(rb[k] - ra[k] * s.cp[k - 1]);
        s.ap[k] = -r * ra[k] * s.ap[k - 1];
        s.cp[k] = r * rc[k];
        s.dp[k] = r * (rd[k] - ra[k] * s.dp[k - 1]);
    }
    s.la = s.ap[M - 1];
    s.lc = s.cp[M - 1];
    s.ld = s.dp[M - 1];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {
        s.dp[k] -= s.cp[k] * s.dp[k + 1];
        s.ap[k] -= s.cp[k] * s.ap[k + 1];
        s.cp[k] = -s.cp[k] * s.cp[k + 1];
    }
    s.fa = ra[0];
    s.fb = rb[0] - rc[0] * s.ap[1];
    s.fc = -rc[0] * s.cp[1];
    s.fd = rd[0] - rc[0] * s.dp[1];
}

// Same sweep with rows produced on demand by rows(k, a, b, c) (so a caller that
// solves twice need not keep the rows in registers); rd holds the rhs.
template <typename T, int M, class Rows>
__device__ __forceinline__ void tile_eliminate_fn(const Rows &rows, const T (&rd)[M], TileState<T, M> &s) {
    static_assert(M >= 3, "tiles need at least three rows");
    T a, b, c;
    rows(1, a, b, c);
    const T r1 = fast_rcp(b);
    s.ap[1] = a * r1;
    s.cp[1] = c * r1;
    s.dp[1] = rd[1] * r1;
#pragma unroll
    for (int k = 2; k < M; ++k) {
        rows(k, a, b, c);
        const T r = fast_rcp(b - a * s.cp[k - 1]);
        s.ap[k] = -r * a * s.ap[k - 1];
        s.cp[k] = r * c;
        s.dp[k] = r * (rd[k] - a * s.dp[k - 1]);
    }
    s.la = s.ap[M - 1];
    s.lc = s.cp[M - 1];
    s.ld = s.dp[M - 1];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {
        s.dp[k] -= s.cp[k] * s.dp[k + 1];
        s.ap[k] -= s.cp[k] * s.ap[k + 1];
        s.cp[k] = -s.cp[k] * s.cp[k + 1];
    }
    rows(0, a, b, c);
    s.fa = a;
    s.fb = b - c * s.ap[1];
    s.fc = -c * s.cp[1];
    s.fd = rd[0] - c * s.dp[1];
}

// The coefficient part of the tile sweep of eq. (7), kept so that a second
// right-hand side with the same rows (the correction solve of the mixed-
// precision refinement) needs no pivots again: only the right-hand-side
// recurrences and the back substitution.
//   forward  : d'_1 = r_1 d_1, d'_k = r_k d_k - m_k d'_{k-1}   (m_k = r_k a_k)
//   backward : d'_k -= cf_k d'_{k+1}, k = M-3 .. 1             (cf_k = r_k c_k)
//   first row: fd = d_0 - c0 d'_1
// The back-substitution factors follow from (m, cf) by one product each.
template <typename T, int M>
struct TileFactor {
    T r[M], m[M], cf[M];
    T fa, fb, fc, c0, la, lc;
};

// Full sweep of rows(k, a, b, c) with right-hand side rd: the factor, the
// interior right-hand sides dp (d'_k, k = 1 .. M-2, after both sweeps) and the
// tile's end relations.
template <typename T, int M, class Rows>
__device__ __forceinline__ void tile_factor_fn(const Rows &rows, const T (&rd)[M], TileFactor<T, M> &fc,
                                               T (&dp)[M], TileEnds<T> &e) {
    static_assert(M >= 3, "tiles need at least three rows");
    T a, b, c;
    rows(1, a, b, c);
    fc.r[1] = fast_rcp(b);
    fc.m[1] = a * fc.r[1];  // the forward u_0 factor of row 1
    fc.cf[1] = c * fc.r[1];
    dp[1] = rd[1] * fc.r[1];
    T ap = fc.m[1];
#pragma unroll
    for (int k = 2; k < M; ++k) {
        rows(k, a, b, c);
        const T r = fast_rcp(b - a * fc.cf[k - 1]);
        fc.r[k] = r;
        fc.m[k] = r * a;
        fc.cf[k] = r * c;
        ap = -fc.m[k] * ap;
        dp[k] = r * rd[k] - fc.m[k] * dp[k - 1];
    }
    e.la = fc.la = ap;
    e.lc = fc.lc = fc.cf[M - 1];
    e.ld = dp[M - 1];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) dp[k] -= fc.cf[k] * dp[k + 1];
    // first-row factors: final u_0 and u_{M-1} coefficients of row 1
    T apf[M], cpf = fc.cf[M - 2];
    apf[1] = fc.m[1];
#pragma unroll
    for (int k = 2; k < M - 1; ++k) apf[k] = -fc.m[k] * apf[k - 1];
    T apF = apf[M - 2];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {
        apF = apf[k] - fc.cf[k] * apF;
        cpf = -fc.cf[k] * cpf;
    }
    rows(0, a, b, c);
    fc.c0 = c;
    e.fa = fc.fa = a;
    e.fb = fc.fb = b - c * apF;
    e.fc = fc.fc = -c * cpf;
    e.fd = rd[0] - c * dp[1];
}

// A further right-hand side rd through a kept factor: dp and the end relations.
template <typename T, int M>
__device__ __forceinline__ void tile_factor_rhs(const TileFactor<T, M> &fc, const T (&rd)[M], T (&dp)[M],
                                                TileEnds<T> &e) {
    dp[1] = fc.r[1] * rd[1];
#pragma unroll
    for (int k = 2; k < M; ++k) dp[k] = fc.r[k] * rd[k] - fc.m[k] * dp[k - 1];
    e.la = fc.la;
    e.lc = fc.lc;
    e.ld = dp[M - 1];
#pragma unroll
    for (int k = M - 3; k >= 1; --k) dp[k] -= fc.cf[k] * dp[k + 1];
    e.fa = fc.fa;
    e.fb = fc.fb;
    e.fc = fc.fc;
    e.fd = rd[0] - fc.c0 * dp[1];
}

// Back substitution (eq. (7)) through a factor: u_k = d'_k - ap_k u_0 - cp_k
// u_{M-1}, the final factors ap_k, cp_k rebuilt from (m, cf).
template <typename T, int M>
__device__ __forceinline__ void tile_factor_backsub(const TileFactor<T, M> &fc, const T (&dp)[M], T f, T lv,
                                                    T (&u)[M]) {
    T apf[M];
    apf[1] = fc.m[1];
#pragma unroll
    for (int k = 2; k < M - 1; ++k) apf[k] = -fc.m[k] * apf[k - 1];
    u[0] = f;
    u[M - 1] = lv;
    T apF = apf[M - 2], cpF = fc.cf[M - 2];
    u[M - 2] = dp[M - 2] - apF * f - cpF * lv;
#pragma unroll
    for (int k = M - 3; k >= 1; --k) {
        apF = apf[k] - fc.cf[k] * apF;
        cpF = -fc.cf[k] * cpF;
        u[k] = dp[k] - apF * f - cpF * lv;
    }
}

// Reduced solve of one line across its P tiles.
//   sh      : LDS scratch of 6*S elements, S = number of threads of the block
//   slot    : this thread's slot in [0, S)
//   pstride : slot distance between tiles p and p+1 of the same line
// Every thread of the block must call this (it contains barriers).  P is the
// number of tiles of this thread's line; Pu >= P is a bound uniform over the
// block (it sets the number of PCR levels and barriers; lines of different
// lengths may share a block).  Returns f (tile's first unknown) and lv (its last).
template <typename T, int M>
__device__ __forceinline__ void reduced_pcr(const TileEnds<T> &ts, T *__restrict__ sh, int S,
                                            int P, int p, int slot, int pstride, T &f, T &lv,
                                            int Pu = 0) {
    if (Pu < P) Pu = P;
    T *b0a = sh, *b0c = sh + S, *b0d = sh + 2 * S;
    T *b1a = sh + 3 * S, *b1c = sh + 4 * S, *b1d = sh + 5 * S;
    // 1. each tile publishes its last row (through buffer 1, first used by level 2)
    b1a[slot] = ts.la;
    b1c[slot] = ts.lc;
    b1d[slot] = ts.ld;
    __syncthreads();
    T pa = T(0), pc = T(0), pd = T(0);
    if (p > 0) {
        pa = b1a[slot - pstride];
        pc = b1c[slot - pstride];
        pd = b1d[slot - pstride];
    }
    // 2. eliminate l_{p-1} (previous tile's last row) and l_p (own last row)
    //    from the first row: a P-row tridiagonal system over f_0..f_{P-1}
    const T gsub = -ts.fa * pa;
    const T gdia = ts.fb - ts.fa * pc - ts.fc * ts.la;
    const T gsup = -ts.fc * ts.lc;
    const T grhs = ts.fd - ts.fa * pd - ts.fc * ts.ld;
    const T rg = fast_rcp(gdia);
    T a = gsub * rg, c = gsup * rg, d = grhs * rg;
    // 3. PCR (Alg. 2) over the P rows, double-buffered: one barrier per level
    int lev = 0;
    for (int s = 1; s < Pu; s <<= 1, ++lev) {
        T *ba = (lev & 1) ? b1a : b0a;
        T *bc = (lev & 1) ? b1c : b0c;
        T *bd = (lev & 1) ? b1d : b0d;
        ba[slot] = a;
        bc[slot] = c;
        bd[slot] = d;
        __syncthreads();
        T am = T(0), cm = T(0), dm = T(0), an = T(0), cn = T(0), dn = T(0);
        if (p - s >= 0) {
            const int q = slot - s * pstride;
            am = ba[q];
            cm = bc[q];
            dm = bd[q];
        }
        if (p + s < P) {
            const int q = slot + s * pstride;
            an = ba[q];
            cn = bc[q];
            dn = bd[q];
        }
        const T r = fast_rcp(T(1) - a * cm - c * an);
        const T na = -r * (a * am);
        const T nc = -r * (c * cn);
        const T nd = r * (d - a * dm - c * dn);
        a = na;
        c = nc;
        d = nd;
    }
    f = d;
    // 4. last unknown of the tile from its last row; needs f_{p+1}
    T fn = T(0);
    if (Pu > 1) {
        T *bx = (lev & 1) ? b1d : b0d;  // last read at level lev-2: free
        bx[slot] = f;
        __syncthreads();
        if (p + 1 < P) fn = bx[slot + pstride];
    }
    lv = ts.ld - ts.la * f - ts.lc * fn;
}

// Reduced solve of one line with its P tiles in P adjacent lanes of one
// 16-lane DPP row (P a power of two <= 16, lines aligned to P-lane groups):
// the same elimination and PCR (Alg. 2) as reduced_pcr, with every neighbour
// value moved by a DPP row shift instead of LDS -- no barrier, no scratch.
template <typename T, int M, int P, int S>
struct DppPcr {
    __device__ __forceinline__ static void run(int p, T &a, T &c, T &d) {
        if constexpr (S < P) {
            T am = row_from_lower<S>(a), cm = row_from_lower<S>(c), dm = row_from_lower<S>(d);
            T an = row_from_upper<S>(a), cn = row_from_upper<S>(c), dn = row_from_upper<S>(d);
            if (p < S) am = cm = dm = T(0);  // the row also holds other lines
            if (p + S >= P) an = cn = dn = T(0);
            const T r = fast_rcp(T(1) - a * cm - c * an);
            const T na = -r * (a * am);
            const T nc = -r * (c * cn);
            d = r * (d - a * dm - c * dn);
            a = na;
            c = nc;
            DppPcr<T, M, P, 2 * S>::run(p, a, c, d);
        }
    }
};

template <typename T, int M, int P>
__device__ __forceinline__ void reduced_pcr_dpp(const TileEnds<T> &ts, int p, T &f, T &lv) {
    T pa = row_from_lower<1>(ts.la), pc = row_from_lower<1>(ts.lc), pd = row_from_lower<1>(ts.ld);
    if (p == 0) pa = pc = pd = T(0);
    const T gsub = -ts.fa * pa;
    const T gdia = ts.fb - ts.fa * pc - ts.fc * ts.la;
    const T gsup = -ts.fc * ts.lc;
    const T grhs = ts.fd - ts.fa * pd - ts.fc * ts.ld;
    const T rg = fast_rcp(gdia);
    T a = gsub * rg, c = gsup * rg, d = grhs * rg;
    DppPcr<T, M, P, 1>::run(p, a, c, d);
    f = d;
    T fn = row_from_upper<1>(f);
    if (p + 1 >= P) fn = T(0);
    lv = ts.ld - ts.la * f - ts.lc * fn;
}

// Same reduced solve for a line of 32 or 64 tiles in adjacent lanes of one
// wavefront: neighbours at any stride come through the LDS crossbar
// (ds_bpermute) within the wavefront -- no LDS storage, no barrier.
template <typename T>
__device__ __forceinline__ T lane_up(T v, int s) {  // value of lane - s
    return __shfl_up(v, (unsigned)s, 64);
}
template <typename T>
__device__ __forceinline__ T lane_down(T v, int s) {  // value of lane + s
    return __shfl_down(v, (unsigned)s, 64);
}

template <typename T, int M, int P>
__device__ __forceinline__ void reduced_pcr_wave(const TileEnds<T> &ts, int p, T &f, T &lv) {
    T pa = lane_up(ts.la, 1), pc = lane_up(ts.lc, 1), pd = lane_up(ts.ld, 1);
    if (p == 0) pa = pc = pd = T(0);
    const T gsub = -ts.fa * pa;
    const T gdia = ts.fb - ts.fa * pc - ts.fc * ts.la;
    const T gsup = -ts.fc * ts.lc;
    const T grhs = ts.fd - ts.fa * pd - ts.fc * ts.ld;
    const T rg = fast_rcp(gdia);
    T a = gsub * rg, c = gsup * rg, d = grhs * rg;
#pragma unroll
    for (int S = 1; S < P; S <<= 1) {
        T am = lane_up(a, S), cm = lane_up(c, S), dm = lane_up(d, S);
        T an = lane_down(a, S), cn = lane_down(c, S), dn = lane_down(d, S);
        if (p < S) am = cm = dm = T(0);
        if (p + S >= P) an = cn = dn = T(0);
        const T r = fast_rcp(T(1) - a * cm - c * an);
        const T na = -r * (a * am);
        const T nc = -r * (c * cn);
        d = r * (d - a * dm - c * dn);
        a = na;
        c = nc;
    }
    f = d;
    T fn = lane_down(f, 1);
    if (p + 1 >= P) fn = T(0);
    lv = ts.ld - ts.la * f - ts.lc * fn;
}

// The same reduced solve with P (any value up to 64) known only at run time:
// the line's tiles sit in P adjacent lanes of one wavefront (callers lay lines
// out so that none straddles two wavefronts), the lane moves go through the
// LDS crossbar, and no barrier or LDS storage is involved.
template <typename T>
__device__ __forceinline__ void reduced_pcr_lanes(const TileEnds<T> &ts, int p, int P, T &f, T &lv) {
    T pa = lane_up(ts.la, 1), pc = lane_up(ts.lc, 1), pd = lane_up(ts.ld, 1);
    if (p == 0) pa = pc = pd = T(0);
    const T gsub = -ts.fa * pa;
    const T gdia = ts.fb - ts.fa * pc - ts.fc * ts.la;
    const T gsup = -ts.fc * ts.lc;
    const T grhs = ts.fd - ts.fa * pd - ts.fc * ts.ld;
    const T rg = fast_rcp(gdia);
    T a = gsub * rg, c = gsup * rg, d = grhs * rg;
    for (int S = 1; S < P; S <<= 1) {
        T am = lane_up(a, S), cm = lane_up(c, S), dm = lane_up(d, S);
        T an = lane_down(a, S), cn = lane_down(c, S), dn = lane_down(d, S);
        if (p < S) am = cm = dm = T(0);
        if (p + S >= P) an = cn = dn = T(0);
        const T r = fast_rcp(T(1) - a * cm - c * an);
        const T na = -r * (a * am);
        const T nc = -r * (c * cn);
        d = r * (d - a * dm - c * dn);
        a = na;
        c = nc;
    }
    f = d;
    T fn = lane_down(f, 1);
    if (p + 1 >= P) fn = T(0);
    lv = ts.ld - ts.la * f - ts.lc * fn;
}

// Reduced solve dispatch (a uniform choice: P is the same for the whole
// launch).  With the line's tiles in adjacent lanes (pstride 1, slot = line *
// P + p): DPP row shifts for P a power of two <= 16, wavefront lane moves for
// P = 32 or 64 (a line never straddles two wavefronts); reduced_pcr otherwise.
// Callers must not rely on a barrier inside (the lane forms have none).
template <typename T, int M>
__device__ __forceinline__ void reduced_solve(const TileEnds<T> &ts, T *__restrict__ sh, int S, int P,
                                              int p, int slot, int pstride, T &f, T &lv) {
    if (pstride == 1) {
        switch (P) {
            case 1: reduced_pcr_dpp<T, M, 1>(ts, p, f, lv); return;
            case 2: reduced_pcr_dpp<T, M, 2>(ts, p, f, lv); return;
            case 4: reduced_pcr_dpp<T, M, 4>(ts, p, f, lv); return;
            case 8: reduced_pcr_dpp<T, M, 8>(ts, p, f, lv); return;
            case 16: reduced_pcr_dpp<T, M, 16>(ts, p, f, lv); return;
            case 32: reduced_pcr_wave<T, M, 32>(ts, p, f, lv); return;
            case 64: reduced_pcr_wave<T, M, 64>(ts, p, f, lv); return;
            default: break;
        }
    }
    reduced_pcr<T, M>(ts, sh, S, P, p, slot, pstride, f, lv);
}

// The boundary equations alone, by two streaming sweeps that keep O(1) state
// (the register-lean form of the tile sweep): forward elimination gives the
// last row's relation to u_0 (as in tile_eliminate); a sweep from the tile's
// end writes u_k = al_k u_{k-1} + be_k u_{M-1} + ga_k for k = M-2..1, which
// put into row 0 gives the first row's relation.  rows(k, a, b, c) produces
// row k; rd holds the right-hand side; between the sweeps fence() runs (a
// caller that regenerates rows from a few registers uses it to keep the
// compiler from holding every row's (a, b, c) in registers for the second).
template <typename T, int M, class Rows, class Fence>
__device__ __forceinline__ void tile_ends_fn(const Rows &rows, const T (&rd)[M], TileEnds<T> &e, Fence &&fence) {
    static_assert(M >= 3, "tiles need at least three rows");
    T a, b, c;
    rows(1, a, b, c);
    T r = fast_rcp(b);
    T ap = a * r, cp = c * r, dp = rd[1] * r;
#pragma unroll
    for (int k = 2; k < M; ++k) {
        rows(k, a, b, c);
        r = fast_rcp(b - a * cp);
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

// Back substitution (eq. (7)): the tile's M unknowns.
template <typename T, int M>
__device__ __forceinline__ void tile_backsub(const TileState<T, M> &ts, T f, T lv, T (&u)[M]) {
    u[0] = f;
    u[M - 1] = lv;
#pragma unroll
    for (int k = 1; k < M - 1; ++k) u[k] = ts.dp[k] - ts.ap[k] * f - ts.cp[k] * lv;
}

// Full line-tile solve of raw rows into u (all threads of the block must call).
template <typename T, int M>
__device__ __forceinline__ void tile_solve(const T (&ra)[M], const T (&rb)[M], const T (&rc)[M],
                                           const T (&rd)[M], T *__restrict__ sh, int S, int P,
                                           int p, int slot, int pstride, T (&u)[M]) {
    TileState<T, M> ts;
    tile_eliminate<T, M>(ra, rb, rc, rd, ts);
    T f, lv;
    reduced_solve<T, M>(ts, sh, S, P, p, slot, pstride, f, lv);
    tile_backsub<T, M>(ts, f, lv, u);
}

}  // namespace trid
