// k_varlen_wave.hip -- uneven batches with wavefront-level work: one
// persistent launch in which every wavefront stages, solves and stores its own
// 64 tiles without block barriers, and a system longer than one wavefront is
// coupled across its wavefronts through one small exchange per work item.
//
// Tiling (arxiv 2201.03950, Section III-B): every system is cut into tiles of
// M rows, one per lane; each lane runs the modified Thomas sweep of eq. (7) on
// its tile, which leaves per tile a first-row and a last-row equation over the
// tiles' first and last unknowns f_p, l_p:
//     fa_p l_{p-1} + fb_p f_p + fc_p l_p = fd_p,   la_p f_p + l_p + lc_p f_{p+1} = ld_p.
// Eliminating l gives the reduced tridiagonal system over f (Thomas-PCR
// hybrid), solved by PCR (Alg. 2) with lane moves inside the wavefront.
//
// Short systems (at most 64 tiles) lie wholly in one wavefront, several per
// wavefront: the reduced system is solved by PCR segmented by system.
//
// A long system spans k consecutive wavefronts of one workgroup (64 tiles
// each).  In wavefront w, the chain of its tiles 1..63 is solved by PCR for
// three right-hand sides at once, with the wavefront's own boundary unknowns
// F_w = f_0 (its first tile's first unknown) and L_w = l_63 (its last tile's
// last unknown) as parameters:  f_p = y_p + v_p F_w + w_p L_w.  Substituting
// into tile 0's first-row and tile 63's last-row equations gives two rows per
// wavefront -- the Schur complement of the reduced system onto (F_w, L_w),
// tridiagonal in the order F_0, L_0, F_1, L_1, ... (the tiling idea of eq. (7)
// applied once more, to the wavefronts' groups of tiles).  The 2k rows go
// through LDS (one workgroup barrier), every wavefront of the system solves
// them by Thomas (Alg. 1), and recovers its f, l and rows locally.
//
// Precisions: FP64, FP32, and FP32 solves with one FP64 residual and
// refinement sweep (FP32 a, b, c; FP64 d and x), whose correction solve needs
// a second exchange.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <numeric>
#include <vector>

#include "dispatch.hpp"
#include "tile.hpp"
#include "varlen.hpp"

namespace trid {

namespace {

constexpr int WL = 64;  // lanes per wavefront

struct VlwArgs {
    const void *a, *b, *c, *d;
    void *x;
    const int4 *rec;     // systems in packing order: {first row (low, high 32 bits), rows, first lane}
    const int4 *wdesc;   // [nitems * NW]: {first, count, w0 | item has a long system << 8, k}
    int *counter;        // [0]: next item, [1]: finished workgroups
    int nitems;
};

// Orders this wavefront's LDS accesses before and after it (the lanes of a
// wavefront execute together and LDS serves a wavefront's requests in order,
// so no workgroup barrier is needed for wavefront-private regions).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ T up1(T v) {
    return __shfl_up(v, 1u, WL);
}
template <typename T>
__device__ __forceinline__ T dn1(T v) {
    return __shfl_down(v, 1u, WL);
}

// Lane's place in the work item: system, tile index p within the system, tile
// count P, row count n, first element of the system.
struct LanePlace {
    int sys = -1, p = 0, P = 1, n = 0;
    i64 sbase = 0;
    bool act = false;
};

// A work item's wavefront slot and, for a segment of a long system, that
// system's record; fetched one item ahead (after the previous item's barrier)
// so the dependent loads overlap that item's tail.
struct VlwSlot {
    int4 dsc = {0, 0, 0, 0};
    int4 lr = {0, 0, 0, 0};
};

template <int NW>
__device__ __forceinline__ VlwSlot vlw_fetch(const VlwArgs &g, int item, int w) {
    VlwSlot s;
    if (item < g.nitems) {
        s.dsc = g.wdesc[(i64)item * NW + w];
        if (s.dsc.w > 0) s.lr = g.rec[s.dsc.x];
    }
    return s;
}

__device__ __forceinline__ i64 rec_base(int4 r) { return (i64)(((unsigned long long)(unsigned)r.y << 32) | (unsigned)r.x); }

// Lane assignment of wavefront slot dsc = {first, count, w0 | flag << 8, k}
// (wavefront w of the workgroup).  Short wavefronts: the lanes find their
// system from the systems' first lanes through a wavefront-private map in LDS.
template <int M>
__device__ __forceinline__ LanePlace vlw_place(const VlwArgs &g, const VlwSlot &sl, int w, int lane, int *map) {
    LanePlace L;
    const int4 dsc = sl.dsc;
    if (dsc.y <= 0) return L;  // empty slot: identity tiles
    if (dsc.w > 0) {           // a segment of a long system
        L.sys = dsc.x;
        L.sbase = rec_base(sl.lr);
        L.n = sl.lr.z;
        L.P = (L.n + M - 1) / M;
        L.p = (w - (dsc.z & 0xff)) * WL + lane;
    } else {
        map[lane] = -1;
        wave_sync();
        if (lane < dsc.y) map[g.rec[dsc.x + lane].w] = lane;
        wave_sync();
        const int j = map[lane];
        const unsigned long long starts = __ballot(j >= 0);
        const unsigned long long below = starts & (lane == WL - 1 ? ~0ull : ((2ull << lane) - 1ull));
        if (below) {
            const int st = 63 - __builtin_clzll(below);
            const int4 r = g.rec[dsc.x + map[st]];
            L.sys = dsc.x + map[st];
            L.sbase = rec_base(r);
            L.n = r.z;
            L.P = (L.n + M - 1) / M;
            L.p = lane - st;
        }
        wave_sync();  // map is rewritten by the next item
    }
    L.act = L.sys >= 0 && L.p < L.P;
    if (!L.act) {
        L.p = 0;
        L.P = 1;
    }
    return L;
}

// Publish the lane's tile range (first element, valid rows) for the staging passes.
template <int M>
__device__ __forceinline__ void vlw_ranges(const LanePlace &L, int lane, i64 *s_base, int *s_cnt) {
    const int cnt = L.act ? L.n - L.p * M : 0;
    s_base[lane] = L.act ? L.sbase + (i64)L.p * M : 0;
    s_cnt[lane] = cnt < 0 ? 0 : (cnt > M ? M : cnt);
    wave_sync();
}

// Coalesced load of the wavefront's 64 tiles of one packed array: element
// e = lane + 64 i is row e % M of tile e / M (consecutive lanes read
// consecutive rows of a tile).  Rows past a tile's count load element 0
// instead; their values are never used (the row masks of the solve replace
// them), so no select follows the load -- a select on the loaded value would
// make the compiler wait for each load before issuing the next.
template <typename E, int M>
__device__ __forceinline__ void vlw_load(E (&v)[M], const E *__restrict__ src, const i64 *s_base, const int *s_cnt,
                                         int lane) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int e = lane + WL * i;
        const int tau = e / M, k = e % M;
        v[i] = src[k < s_cnt[tau] ? s_base[tau] + k : (i64)0];
    }
}

// Tile tau's row k lands at tau (M + 1) + k of the wavefront's staging region.
template <typename E, int M>
__device__ __forceinline__ void vlw_put(E *__restrict__ st, const E (&v)[M], int lane) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int e = lane + WL * i;
        st[(e / M) * (M + 1) + e % M] = v[i];
    }
}

template <typename E, int M>
__device__ __forceinline__ void vlw_store(E *__restrict__ dst, const E *__restrict__ st, const i64 *s_base,
                                          const int *s_cnt, int lane) {
#pragma unroll 4
    for (int i = 0; i < M; ++i) {
        const int e = lane + WL * i;
        const int tau = e / M, k = e % M;
        if (k < s_cnt[tau]) dst[s_base[tau] + k] = st[tau * (M + 1) + k];
    }
}

// The tile sweep of eq. (7) run on the tile's two halves side by side (two
// independent dependency chains per lane instead of one twice as long), the
// halves then joined into the whole tile's boundary equations: eliminating
// the two unknowns where they meet, l_A (last of the upper half) and f_B
// (first of the lower half), is the tiles' own reduction applied to a pair of
// half-tiles.  Both are kept as functions of the tile's f and l:
//     f_B = bt + bf f + bl l,   l_A = dt + df f + dl l.
template <typename T, int M>
struct HalfTiles : TileEnds<T> {
    TileState<T, M / 2> A, B;
    T bt, bf, bl, dt, df, dl;
};

template <typename T, int M>
__device__ __forceinline__ void half_eliminate(const T (&ra)[M], const T (&rb)[M], const T (&rc)[M],
                                               const T (&rd)[M], HalfTiles<T, M> &s) {
    constexpr int H = M / 2;
    using Half = const T(&)[H];
    tile_eliminate<T, H>(reinterpret_cast<Half>(ra[0]), reinterpret_cast<Half>(rb[0]),
                         reinterpret_cast<Half>(rc[0]), reinterpret_cast<Half>(rd[0]), s.A);
    tile_eliminate<T, H>(reinterpret_cast<Half>(ra[H]), reinterpret_cast<Half>(rb[H]),
                         reinterpret_cast<Half>(rc[H]), reinterpret_cast<Half>(rd[H]), s.B);
    const TileState<T, H> &A = s.A, &B = s.B;
    // B's first row fa_B l_A + fb_B f_B + fc_B l = fd_B with A's last row l_A = ld_A - la_A f - lc_A f_B
    const T rg = fast_rcp(B.fb - B.fa * A.lc);
    s.bt = (B.fd - B.fa * A.ld) * rg;
    s.bf = B.fa * A.la * rg;
    s.bl = -B.fc * rg;
    s.dt = A.ld - A.lc * s.bt;
    s.df = -A.la - A.lc * s.bf;
    s.dl = -A.lc * s.bl;
    // the tile's first row is A's with l_A substituted, its last row B's with f_B substituted
    s.fa = A.fa;
    s.fb = A.fb + A.fc * s.df;
    s.fc = A.fc * s.dl;
    s.fd = A.fd - A.fc * s.dt;
    const T rn = fast_rcp(T(1) + B.la * s.bl);
    s.la = B.la * s.bf * rn;
    s.lc = B.lc * rn;
    s.ld = (B.ld - B.la * s.bt) * rn;
}

template <typename T, int M>
__device__ __forceinline__ void half_backsub(const HalfTiles<T, M> &s, T f, T lv, T (&u)[M]) {
    constexpr int H = M / 2;
    const T fB = s.bt + s.bf * f + s.bl * lv;
    const T lA = s.dt + s.df * f + s.dl * lv;
    tile_backsub<T, H>(s.A, f, lA, reinterpret_cast<T(&)[H]>(u[0]));
    tile_backsub<T, H>(s.B, fB, lv, reinterpret_cast<T(&)[H]>(u[H]));
}

// One PCR level (Alg. 2) across lanes: neighbours at distance S within the
// lane's segment [lane - q, lane - q + Q).
template <typename T>
__device__ __forceinline__ void pcr_level(int S, int q, int Q, T &a, T &c, T &d) {
    T am = __shfl_up(a, (unsigned)S, WL), cm = __shfl_up(c, (unsigned)S, WL), dm = __shfl_up(d, (unsigned)S, WL);
    T an = __shfl_down(a, (unsigned)S, WL), cn = __shfl_down(c, (unsigned)S, WL), dn = __shfl_down(d, (unsigned)S, WL);
    if (q < S) am = cm = dm = T(0);
    if (q + S >= Q) an = cn = dn = T(0);
    const T r = fast_rcp(T(1) - a * cm - c * an);
    const T na = -r * (a * am);
    const T nc = -r * (c * cn);
    d = r * (d - a * dm - c * dn);
    a = na;
    c = nc;
}

// The same level for three right-hand sides sharing the matrix.
template <typename T>
__device__ __forceinline__ void pcr_level3(int S, int q, int Q, T &a, T &c, T &d0, T &d1, T &d2) {
    T am = __shfl_up(a, (unsigned)S, WL), cm = __shfl_up(c, (unsigned)S, WL);
    T an = __shfl_down(a, (unsigned)S, WL), cn = __shfl_down(c, (unsigned)S, WL);
    T m0 = __shfl_up(d0, (unsigned)S, WL), m1 = __shfl_up(d1, (unsigned)S, WL), m2 = __shfl_up(d2, (unsigned)S, WL);
    T n0 = __shfl_down(d0, (unsigned)S, WL), n1 = __shfl_down(d1, (unsigned)S, WL), n2 = __shfl_down(d2, (unsigned)S, WL);
    if (q < S) am = cm = m0 = m1 = m2 = T(0);
    if (q + S >= Q) an = cn = n0 = n1 = n2 = T(0);
    const T r = fast_rcp(T(1) - a * cm - c * an);
    const T na = -r * (a * am);
    const T nc = -r * (c * cn);
    d0 = r * (d0 - a * m0 - c * n0);
    d1 = r * (d1 - a * m1 - c * n1);
    d2 = r * (d2 - a * m2 - c * n2);
    a = na;
    c = nc;
}

// Reduced solve of the short systems of a wavefront: f (tile's first unknown)
// and lv (its last) from the tile sweep's state.
template <typename T, int M>
__device__ __forceinline__ void vlw_short(const TileEnds<T> &ts, const LanePlace &L, T &f, T &lv) {
    T pa = up1(ts.la), pc = up1(ts.lc), pd = up1(ts.ld);
    if (L.p == 0) pa = pc = pd = T(0);
    const T gsub = -ts.fa * pa;
    const T gdia = ts.fb - ts.fa * pc - ts.fc * ts.la;
    const T gsup = -ts.fc * ts.lc;
    const T grhs = ts.fd - ts.fa * pd - ts.fc * ts.ld;
    const T rg = fast_rcp(gdia);
    T a = gsub * rg, c = gsup * rg, d = grhs * rg;
#pragma unroll
    for (int S = 1; S < WL; S <<= 1) pcr_level(S, L.p, L.P, a, c, d);
    f = d;
    T fn = dn1(f);
    if (L.p + 1 >= L.P) fn = T(0);
    lv = ts.ld - ts.la * f - ts.lc * fn;
}

// First half of a long system's reduced solve in one wavefront: the chain of
// tiles 1..63 for three right-hand sides (y, v, w), and the wavefront's two
// Schur rows (lane 0: the F row, lane 63: the L row) as (sub, dia, sup, rhs)
// into xrow[0..3] (F row) and xrow[4..7] (L row) of the exchange buffer.
template <typename T, int M>
__device__ __forceinline__ void vlw_long_chain(const TileEnds<T> &ts, int lane, T &y, T &v, T &w,
                                               T *__restrict__ xrow) {
    const T pa = up1(ts.la), pc = up1(ts.lc), pd = up1(ts.ld);
    T gsub = T(0), gdia = T(1), gsup = T(0), grhs = T(0), vr = T(0), wr = T(0);
    if (lane >= 1) {
        gsub = -ts.fa * pa;
        gdia = ts.fb - ts.fa * pc;
        grhs = ts.fd - ts.fa * pd;
        if (lane < WL - 1) {  // l_p eliminated by the tile's own last row
            gdia -= ts.fc * ts.la;
            gsup = -ts.fc * ts.lc;
            grhs -= ts.fc * ts.ld;
        } else {  // lane 63 keeps l_63 = L_w: its coefficient moves to the w right-hand side
            wr = -ts.fc;
        }
        if (lane == 1) {  // the coefficient of f_0 = F_w moves to the v right-hand side
            vr = -gsub;
            gsub = T(0);
        }
    }
    const T rg = fast_rcp(gdia);
    T a = gsub * rg, c = gsup * rg;
    y = grhs * rg;
    v = vr * rg;
    w = wr * rg;
    const int q = lane >= 1 ? lane - 1 : 0, Q = lane >= 1 ? WL - 1 : 1;
#pragma unroll
    for (int S = 1; S < WL; S <<= 1) pcr_level3(S, q, Q, a, c, y, v, w);
    const T y1 = dn1(y), v1 = dn1(v), w1 = dn1(w);
    if (lane == 0) {  // fa l_{-1} + fb F + fc l_0 = fd with l_0 = ld - la F - lc f_1
        const T fl = ts.fc * ts.lc;
        xrow[0] = ts.fa;
        xrow[1] = ts.fb - ts.fc * ts.la - fl * v1;
        xrow[2] = -fl * w1;
        xrow[3] = ts.fd - ts.fc * ts.ld + fl * y1;
    }
    if (lane == WL - 1) {  // la f_63 + L + lc F_{w+1} = ld with f_63 = y + v F + w L
        xrow[4] = ts.la * v;
        xrow[5] = T(1) + ts.la * w;
        xrow[6] = ts.lc;
        xrow[7] = ts.ld - ts.la * y;
    }
}

// Second half, after the workgroup barrier: the system's 2k Schur rows are
// solved by PCR (Alg. 2) across the wavefront's first 2k lanes (lane j holds
// row j; they stay diagonally dominant, as Schur complements of a diagonally
// dominant matrix), every wavefront of the system redundantly; then the
// wavefront's F, L and, for a refinement residual, the last unknown of the
// previous wavefront (Lp) and the first of the next (Fn).
template <typename T, int NW>
__device__ __forceinline__ void vlw_schur_solve(const T *__restrict__ xb, int w0, int k, int w, int lane, T &F,
                                                T &Lw, T &Lp, T &Fn) {
    const int R = 2 * k;
    const bool ok = lane < R;
    const T *row = xb + (2 * w0 + (ok ? lane : 0)) * 4;
    const T sub = ok ? row[0] : T(0), dia = ok ? row[1] : T(1), sup = ok ? row[2] : T(0), rhs = ok ? row[3] : T(0);
    const T rg = fast_rcp(dia);
    T a = sub * rg, c = sup * rg, d = rhs * rg;
    const int q = ok ? lane : 0, Q = ok ? R : 1;
#pragma unroll
    for (int S = 1; S < 2 * NW; S <<= 1) pcr_level(S, q, Q, a, c, d);
    const int i = 2 * (w - w0);
    F = __shfl(d, i, WL);
    Lw = __shfl(d, i + 1, WL);
    const T lp = __shfl(d, i > 0 ? i - 1 : 0, WL), fn = __shfl(d, i + 2 < R ? i + 2 : 0, WL);
    Lp = i > 0 ? lp : T(0);
    Fn = i + 2 < R ? fn : T(0);
}

// Dynamic LDS: per wavefront a staging region of 64 (M + 1) elements of E,
// tile ranges (i64 + int per lane) and the lane map (int per lane); then the
// exchange buffers: `nx` sets of 2 parities x 2 NW rows x 4 values of T.
template <int M, int NW, typename E, typename T>
struct VlwLds {
    static constexpr size_t stage = (size_t)WL * (M + 1) * sizeof(E);
    static constexpr size_t per_wave = (stage + 15) / 16 * 16 + WL * (8 + 4 + 4);
    static size_t bytes(int nx) { return per_wave * NW + (size_t)nx * 2 * 2 * NW * 4 * sizeof(T) + 16; }
};

// Last workgroup out resets the work counters (vector atomics only).
__device__ __forceinline__ void vlw_finish(int *counter) {
    if (threadIdx.x == 0) {
        __threadfence();
        const int done = atomicAdd(&counter[1], 1);
        if (done == (int)gridDim.x - 1) {
            atomicExch(&counter[0], 0);
            atomicExch(&counter[1], 0);
        }
    }
}

// PIPE: 0 loads and stages one array at a time; 1 issues the next array's
// loads before the current one is staged; 2 issues all four arrays' loads
// before the first is staged (the most loads in flight; the raw tiles then
// occupy no more registers than the elimination that follows).
// WPE: wavefronts per SIMD the register allocation must allow (two
// workgroups of 8 wavefronts per CU need 4).
template <typename T, int M, int NW, int PIPE, int WPE = 1>
__global__ __launch_bounds__(WL *NW, WPE) void k_vlw_plain(VlwArgs g) {
    using Lds = VlwLds<M, NW, T, T>;
    __shared__ int s_next[2];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x & (WL - 1), w = threadIdx.x / WL;
    unsigned char *wr = smem_raw + Lds::per_wave * w;
    T *st = reinterpret_cast<T *>(wr);
    i64 *s_base = reinterpret_cast<i64 *>(wr + (Lds::stage + 15) / 16 * 16);
    int *s_cnt = reinterpret_cast<int *>(s_base + WL);
    int *map = s_cnt + WL;
    T *xbuf = reinterpret_cast<T *>(smem_raw + Lds::per_wave * NW);  // [2 parities][2 NW rows][4]
    const T *arr[4] = {static_cast<const T *>(g.a), static_cast<const T *>(g.b), static_cast<const T *>(g.c),
                       static_cast<const T *>(g.d)};
    T *x = static_cast<T *>(g.x);
    if (threadIdx.x == 0) s_next[0] = atomicAdd(&g.counter[0], 1);
    __syncthreads();
    int item = s_next[0];
    VlwSlot nxt = vlw_fetch<NW>(g, item, w);
    for (int it = 0; item < g.nitems; ++it) {
        const int par = it & 1;
        if (threadIdx.x == 0) s_next[par ^ 1] = atomicAdd(&g.counter[0], 1);
        const VlwSlot sl = nxt;
        const int4 dsc = sl.dsc;
        const bool has_long = (dsc.z >> 8) != 0;
        const LanePlace L = vlw_place<M>(g, sl, w, lane, map);
        vlw_ranges<M>(L, lane, s_base, s_cnt);
        T ra[M], rb[M], rc[M], rd[M];
        if constexpr (PIPE == 2) {
            T v[4][M];
#pragma unroll
            for (int r = 0; r < 4; ++r) vlw_load<T, M>(v[r], arr[r], s_base, s_cnt, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                vlw_put<T, M>(st, v[r], lane);
                wave_sync();
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const int row = L.p * M + k;
                    const bool ok = L.act && row < L.n;
                    const T val = st[lane * (M + 1) + k];
                    if (r == 0) ra[k] = (ok && row > 0) ? val : T(0);
                    if (r == 1) rb[k] = ok ? val : T(1);
                    if (r == 2) rc[k] = (ok && row < L.n - 1) ? val : T(0);
                    if (r == 3) rd[k] = ok ? val : T(0);
                }
                wave_sync();
            }
        } else {
            T vn[M];
            vlw_load<T, M>(vn, arr[0], s_base, s_cnt, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T vc[M];
                if (!PIPE && r > 0) vlw_load<T, M>(vn, arr[r], s_base, s_cnt, lane);
#pragma unroll
                for (int k = 0; k < M; ++k) vc[k] = vn[k];
                if (PIPE && r < 3) vlw_load<T, M>(vn, arr[r + 1], s_base, s_cnt, lane);
                vlw_put<T, M>(st, vc, lane);
                wave_sync();
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const int row = L.p * M + k;
                    const bool ok = L.act && row < L.n;
                    const T val = st[lane * (M + 1) + k];
                    if (r == 0) ra[k] = (ok && row > 0) ? val : T(0);
                    if (r == 1) rb[k] = ok ? val : T(1);
                    if (r == 2) rc[k] = (ok && row < L.n - 1) ? val : T(0);
                    if (r == 3) rd[k] = ok ? val : T(0);
                }
                wave_sync();
            }
        }
        HalfTiles<T, M> ts;
        half_eliminate<T, M>(ra, rb, rc, rd, ts);
        T f, lv;
        T y = T(0), v = T(0), wv = T(0);
        T *xb = xbuf + par * (2 * NW * 4);
        if (dsc.w > 0) {
            vlw_long_chain<T, M>(ts, lane, y, v, wv, xb + 2 * w * 4);
        } else {
            vlw_short<T, M>(ts, L, f, lv);
        }
        if (has_long) {  // the Schur rows and the next item's index are visible
            __syncthreads();
            item = s_next[par ^ 1];
            nxt = vlw_fetch<NW>(g, item, w);
        }
        if (dsc.w > 0) {
            T F, Lw, Lp, Fn;
            vlw_schur_solve<T, NW>(xb, dsc.z & 0xff, dsc.w, w, lane, F, Lw, Lp, Fn);
            f = lane == 0 ? F : y + v * F + wv * Lw;
            const T fn = dn1(f);
            lv = lane == WL - 1 ? Lw : ts.ld - ts.la * f - ts.lc * fn;
        }
        T u[M];
        half_backsub<T, M>(ts, f, lv, u);
#pragma unroll
        for (int k = 0; k < M; ++k) st[lane * (M + 1) + k] = u[k];
        wave_sync();
        vlw_store<T, M>(x, st, s_base, s_cnt, lane);
        wave_sync();
        if (!has_long) {  // the next item's index is visible
            __syncthreads();
            item = s_next[par ^ 1];
            nxt = vlw_fetch<NW>(g, item, w);
        }
    }
    vlw_finish(g.counter);
}

// FP32 solves + one FP64 residual and refinement sweep: a, b, c float, d and x double.
template <int M, int NW>
__global__ __launch_bounds__(WL *NW) void k_vlw_refine(VlwArgs g) {
    using Lds = VlwLds<M, NW, double, float>;
    __shared__ int s_next[2];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x & (WL - 1), w = threadIdx.x / WL;
    unsigned char *wr = smem_raw + Lds::per_wave * w;
    double *st = reinterpret_cast<double *>(wr);
    float *stf = reinterpret_cast<float *>(wr);
    i64 *s_base = reinterpret_cast<i64 *>(wr + (Lds::stage + 15) / 16 * 16);
    int *s_cnt = reinterpret_cast<int *>(s_base + WL);
    int *map = s_cnt + WL;
    float *xbuf = reinterpret_cast<float *>(smem_raw + Lds::per_wave * NW);  // [2 passes][2 parities][2 NW][4]
    const float *arr[3] = {static_cast<const float *>(g.a), static_cast<const float *>(g.b),
                           static_cast<const float *>(g.c)};
    const double *dg = static_cast<const double *>(g.d);
    double *x = static_cast<double *>(g.x);
    if (threadIdx.x == 0) s_next[0] = atomicAdd(&g.counter[0], 1);
    __syncthreads();
    int item = s_next[0];
    VlwSlot nxt = vlw_fetch<NW>(g, item, w);
    for (int it = 0; item < g.nitems; ++it) {
        const int par = it & 1;
        if (threadIdx.x == 0) s_next[par ^ 1] = atomicAdd(&g.counter[0], 1);
        const VlwSlot sl = nxt;
        const int4 dsc = sl.dsc;
        const bool has_long = (dsc.z >> 8) != 0;
        const bool lng = dsc.w > 0;
        const LanePlace L = vlw_place<M>(g, sl, w, lane, map);
        vlw_ranges<M>(L, lane, s_base, s_cnt);
        float ra[M], rb[M], rc[M];
        double dd[M];
        {
            // every array's loads of the item in flight before the first is staged
            float vn[3][M];
            double vd[M];
#pragma unroll
            for (int r = 0; r < 3; ++r) vlw_load<float, M>(vn[r], arr[r], s_base, s_cnt, lane);
            vlw_load<double, M>(vd, dg, s_base, s_cnt, lane);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                vlw_put<float, M>(stf, vn[r], lane);
                wave_sync();
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    const int row = L.p * M + k;
                    const bool ok = L.act && row < L.n;
                    const float val = stf[lane * (M + 1) + k];
                    if (r == 0) ra[k] = (ok && row > 0) ? val : 0.f;
                    if (r == 1) rb[k] = ok ? val : 1.f;
                    if (r == 2) rc[k] = (ok && row < L.n - 1) ? val : 0.f;
                }
                wave_sync();
            }
            vlw_put<double, M>(st, vd, lane);
            wave_sync();
#pragma unroll
            for (int k = 0; k < M; ++k) dd[k] = (L.act && L.p * M + k < L.n) ? st[lane * (M + 1) + k] : 0.0;
            wave_sync();
        }
        // two FP32 solves; the second has the FP64 residual as right-hand side
        // and reuses the first one's tile factor (no pivots again)
        float x32[M];
        float rhs[M];
#pragma unroll
        for (int k = 0; k < M; ++k) rhs[k] = (float)dd[k];
        TileFactor<float, M> fct;
        float dp[M];
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            TileEnds<float> ts;
            if (pass == 0) {
                auto rows = [&](int k, float &a, float &b, float &c) {
                    a = ra[k];
                    b = rb[k];
                    c = rc[k];
                };
                tile_factor_fn<float, M>(rows, rhs, fct, dp, ts);
            } else {
                tile_factor_rhs<float, M>(fct, rhs, dp, ts);
            }
            float f, lv, y = 0.f, v = 0.f, wv = 0.f;
            float *xb = xbuf + (pass * 2 + par) * (2 * NW * 4);
            if (lng)
                vlw_long_chain<float, M>(ts, lane, y, v, wv, xb + 2 * w * 4);
            else
                vlw_short<float, M>(ts, L, f, lv);
            if (has_long) {
                __syncthreads();
                if (pass == 1) {  // the next item's index is visible
                    item = s_next[par ^ 1];
                    nxt = vlw_fetch<NW>(g, item, w);
                }
            }
            float Lp = 0.f, Fn = 0.f;
            if (lng) {
                float F, Lw;
                vlw_schur_solve<float, NW>(xb, dsc.z & 0xff, dsc.w, w, lane, F, Lw, Lp, Fn);
                f = lane == 0 ? F : y + v * F + wv * Lw;
                const float fn = dn1(f);
                lv = lane == WL - 1 ? Lw : ts.ld - ts.la * f - ts.lc * fn;
            }
            float u[M];
            tile_factor_backsub<float, M>(fct, dp, f, lv, u);
            if (pass == 0) {
                // r = d - A x32 in FP64; the neighbours of the tile's first and
                // last rows come from the adjacent lanes, or across wavefronts
                // of a long system from the Schur solution
                double xprev = (double)up1(u[M - 1]), xnext = (double)dn1(u[0]);
                if (L.p == 0) xprev = 0.0;
                if (L.p + 1 >= L.P) xnext = 0.0;
                if (lng && lane == 0) xprev = (double)Lp;
                if (lng && lane == WL - 1) xnext = (double)Fn;
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    x32[k] = u[k];
                    const double xm = k > 0 ? (double)u[k - 1] : xprev;
                    const double xp = k < M - 1 ? (double)u[k + 1] : xnext;
                    rhs[k] = (float)(dd[k] - ((double)ra[k] * xm + (double)rb[k] * (double)u[k] + (double)rc[k] * xp));
                }
            } else {
#pragma unroll
                for (int k = 0; k < M; ++k) dd[k] = (double)x32[k] + (double)u[k];
            }
        }
#pragma unroll
        for (int k = 0; k < M; ++k) st[lane * (M + 1) + k] = dd[k];
        wave_sync();
        vlw_store<double, M>(x, st, s_base, s_cnt, lane);
        wave_sync();
        if (!has_long) {
            __syncthreads();
            item = s_next[par ^ 1];
            nxt = vlw_fetch<NW>(g, item, w);
        }
    }
    vlw_finish(g.counter);
}

// Calls f(kernel, threads, dynamic LDS bytes) for the compiled wavefront variant.
template <class F>
auto with_wave_kernel(int prec, int M, int NW, F &&f) -> decltype(f(k_vlw_refine<16, 8>, 512, size_t(0))) {
    if (prec == 2) return f(k_vlw_refine<16, 8>, 512, VlwLds<16, 8, double, float>::bytes(2));
    if (prec == 0 && M == 8)  // 16 wavefronts, 4 per SIMD: 128 VGPRs (40 bytes per lane spilled)
        return f(k_vlw_plain<double, 8, 16, 1>, 1024, VlwLds<8, 16, double, double>::bytes(1));
    if (prec == 0) return f(k_vlw_plain<double, 16, 8, 2>, 512, VlwLds<16, 8, double, double>::bytes(1));
    if (M == 32) return f(k_vlw_plain<float, 32, 4, 1>, 256, VlwLds<32, 4, float, float>::bytes(1));
    return f(k_vlw_plain<float, 16, 8, 2, 4>, 512, VlwLds<16, 8, float, float>::bytes(1));
}

template <class K>
int wave_occupancy(K kernel, int nt, size_t lds) {
    hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    return per_cu * cus;
}

}  // namespace

// Wavefront variants: M rows per tile, NW wavefronts per workgroup (the
// longest system is 64 NW tiles).
int varlen_wave_NW(int prec, int M) { return (prec == 1 && M == 32) ? 4 : ((prec == 0 && M == 8) ? 16 : 8); }

void varlen_wave_pack(const int64_t *off, std::vector<int> ids, int M, int NW, std::vector<int> *order,
                      std::vector<int> *tstart, std::vector<int> *wdesc) {
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int i, int j) { return off[i + 1] - off[i] > off[j + 1] - off[j]; });
    order->clear();
    tstart->clear();
    wdesc->clear();
    auto tiles = [&](int s) { return (int)((off[s + 1] - off[s] + M - 1) / M); };
    // long systems: k consecutive wavefronts of one work item (next fit)
    std::vector<std::array<int, 4>> slots;  // {first, count, w0, k} per wavefront slot
    int used = NW;                          // wavefronts used in the current item
    size_t i = 0;
    for (; i < ids.size() && tiles(ids[i]) > WL; ++i) {
        const int k = (tiles(ids[i]) + WL - 1) / WL;
        if (used + k > NW) {
            for (; used < NW && !slots.empty(); ++used) slots.push_back({0, 0, 0, 0});
            used = 0;
        }
        const int first = (int)order->size();
        order->push_back(ids[i]);
        tstart->push_back(0);
        for (int j = 0; j < k; ++j) slots.push_back({first, 1, used, k});
        used += k;
    }
    // short systems: packed into wavefronts of 64 lanes (next fit, longest
    // first), filling the free slots of the items above, then new items
    std::vector<size_t> free_slots;
    for (size_t s = 0; s < slots.size(); ++s)
        if (slots[s][1] == 0) free_slots.push_back(s);
    for (; used < NW && !slots.empty(); ++used) {
        free_slots.push_back(slots.size());
        slots.push_back({0, 0, 0, 0});
    }
    size_t fi = 0;
    while (i < ids.size()) {
        const int first = (int)order->size();
        int lanes = 0, cnt = 0;
        for (; i < ids.size() && lanes + tiles(ids[i]) <= WL; ++i, ++cnt) {
            order->push_back(ids[i]);
            tstart->push_back(lanes);
            lanes += tiles(ids[i]);
        }
        const std::array<int, 4> s{first, cnt, 0, 0};
        if (fi < free_slots.size()) {
            slots[free_slots[fi++]] = s;
        } else {
            slots.push_back(s);
        }
    }
    while (slots.size() % NW) slots.push_back({0, 0, 0, 0});
    // flag every slot of an item that holds a long system (its workgroup
    // exchanges Schur rows): w0 | 1 << 8
    for (size_t it = 0; it < slots.size(); it += NW) {
        bool lng = false;
        for (int j = 0; j < NW; ++j) lng |= slots[it + j][3] > 0;
        if (lng)
            for (int j = 0; j < NW; ++j) slots[it + j][2] |= 1 << 8;
    }
    wdesc->reserve(slots.size() * 4);
    for (const auto &s : slots) wdesc->insert(wdesc->end(), s.begin(), s.end());
}

int varlen_wave_blocks(int prec, int M) {
    return with_wave_kernel(prec, M, varlen_wave_NW(prec, M),
                            [&](auto k, int nt, size_t lds) { return wave_occupancy(k, nt, lds); });
}

hipError_t varlen_wave_build(const int64_t *off, std::vector<int> ids, int prec, const VarlenVariant &v,
                             VarlenSchedule *sc) {
    const int NW = varlen_wave_NW(prec, v.M);
    std::vector<int> order, tstart, wdesc;
    varlen_wave_pack(off, ids, v.M, NW, &order, &tstart, &wdesc);
    // per system in packing order: first row (two 32-bit halves), rows, first lane
    std::vector<int> rec(order.size() * 4);
    for (size_t i = 0; i < order.size(); ++i) {
        const unsigned long long b = (unsigned long long)off[order[i]];
        rec[4 * i] = (int)(unsigned)(b & 0xffffffffull);
        rec[4 * i + 1] = (int)(unsigned)(b >> 32);
        rec[4 * i + 2] = (int)(off[order[i] + 1] - off[order[i]]);
        rec[4 * i + 3] = tstart[i];
    }
    sc->prec = prec;
    sc->M = v.M;
    sc->NT = WL * NW;
    sc->thomas = 0;
    sc->wave = 1;
    sc->nsys = (i64)ids.size();
    sc->nitems = (int)(wdesc.size() / 4 / NW);
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t b_rec = sizeof(int) * rec.size(), b_wd = sizeof(int) * wdesc.size();
    const size_t total = up(b_rec) + up(b_wd) + 256;
    hipError_t e = hipMalloc(&sc->dev, total);
    if (e != hipSuccess) {
        sc->dev = nullptr;
        return e;
    }
    char *p = static_cast<char *>(sc->dev);
    sc->rec = reinterpret_cast<int *>(p);
    p += up(b_rec);
    sc->wdesc = reinterpret_cast<int *>(p);
    p += up(b_wd);
    sc->counter = reinterpret_cast<int *>(p);
    if ((e = hipMemcpy(sc->rec, rec.data(), b_rec, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(sc->wdesc, wdesc.data(), b_wd, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemset(sc->counter, 0, 2 * sizeof(int))) != hipSuccess) return e;
    sc->nblocks = std::max(1, std::min(varlen_wave_blocks(prec, v.M), sc->nitems));
    return hipSuccess;
}

hipError_t varlen_wave_launch(const VarlenSchedule &sc, const void *a, const void *b, const void *c, const void *d,
                              void *x, hipStream_t s) {
    VlwArgs g;
    g.a = a;
    g.b = b;
    g.c = c;
    g.d = d;
    g.x = x;
    g.rec = reinterpret_cast<const int4 *>(sc.rec);
    g.wdesc = reinterpret_cast<const int4 *>(sc.wdesc);
    g.counter = sc.counter;
    g.nitems = sc.nitems;
    return with_wave_kernel(sc.prec, sc.M, varlen_wave_NW(sc.prec, sc.M), [&](auto k, int nt, size_t lds) {
        hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        launch(k, dim3((unsigned)sc.nblocks), dim3(nt), lds, s, g);
        return hipGetLastError();
    });
}

}  // namespace trid
