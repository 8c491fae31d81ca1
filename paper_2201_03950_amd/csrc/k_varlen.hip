// k_varlen.hip -- uneven batches: systems of different lengths packed back to
// back, solved by ONE persistent launch.
//
// Schedule (host, once per offsets content and tile plan): systems are sorted
// longest first and packed greedily into work items of at most NT tiles (one
// thread per tile of M rows, eq. (7) of arxiv 2201.03950, Section III-B); an
// item's systems occupy consecutive threads.  The persistent blocks pull items
// from a device counter; the last block to finish resets the counter, so every
// launch (and every replay of a captured graph) starts from zero without a
// memset.  Within an item each system's reduced system is solved by PCR over
// its own tiles; the number of PCR levels is the item's maximum (uniform), and
// shorter systems simply see no neighbours at the extra levels.
//
// Precisions: FP64, FP32, and FP32 bulk + one FP64 refinement sweep (FP32
// coefficients, FP64 right-hand side and solution).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "dispatch.hpp"
#include "long_ext.hpp"
#include "long_lines.hpp"
#include "refine_tile.hpp"
#include "varlen.hpp"

namespace trid {

struct VarlenArgs {
    const void *a, *b, *c, *d;
    void *x;
    const i64 *off;         // [nsys + 1]
    const int *order;       // systems in item order
    const int *tstart;      // first thread of each system within its item (order positions)
    const int *item_begin;  // [nitems + 1] range into order
    const int *item_pmax;   // [nitems] largest tile count in the item
    int *counter;           // [0]: next item, [1]: finished blocks
    int nitems;
};

// Block-local assignment of threads to (system, tile) for one work item, and
// per-tile row ranges published in LDS for the staging passes:
//   s_base[t]: element offset of tile t's first row, s_cnt[t]: its valid rows.
// Returns, per thread: system id (or -1), tile p, tile count P, row count n.
template <int M, int NT>
__device__ __forceinline__ void varlen_assign(const VarlenArgs &g, int item, short *s_sys, short *s_p,
                                             i64 *s_base, int *s_cnt, int &sys, int &p, int &P, int &n) {
    const int t = threadIdx.x;
    const int ib = g.item_begin[item], ie = g.item_begin[item + 1];
    s_sys[t] = -1;
    __syncthreads();
    for (int j = t; j < ie - ib; j += NT) {
        const int sy = g.order[ib + j];
        const int len = (int)(g.off[sy + 1] - g.off[sy]);
        const int Pj = (len + M - 1) / M;
        const int t0 = g.tstart[ib + j];
        for (int q = 0; q < Pj; ++q) {
            s_sys[t0 + q] = (short)j;
            s_p[t0 + q] = (short)q;
        }
    }
    __syncthreads();
    const int j = s_sys[t];
    i64 base = 0;
    if (j >= 0) {
        sys = g.order[ib + j];
        base = g.off[sys];
        n = (int)(g.off[sys + 1] - base);
        P = (n + M - 1) / M;
        p = s_p[t];
    } else {
        sys = -1;
        n = 0;
        P = 1;
        p = 0;
    }
    const int cnt = n - p * M;
    s_base[t] = base + (i64)p * M;
    s_cnt[t] = cnt < 0 ? 0 : (cnt > M ? M : cnt);
    __syncthreads();
}

// Staging of one packed array, in two halves so that the loads of the next
// array can be in flight while this one moves through LDS:
//   varlen_load : consecutive lanes take consecutive (tile, row) positions, i.e.
//                 consecutive elements of the same system; rows past a tile's
//                 count load element 0 instead (branch-free) and are zeroed;
//   varlen_put  : tile t's row k lands at t * (M + 1) + k (every slot is
//                 written; slots past a tile's count hold 0 and are never used).
template <typename E, int M, int NT>
__device__ __forceinline__ void varlen_load(E (&v)[M], const E *__restrict__ src, const i64 *s_base,
                                            const int *s_cnt) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int e = threadIdx.x + i * NT;
        const int tau = e / M, k = e % M;
        v[i] = load_if(src, s_base[tau] + k, k < s_cnt[tau], (i64)0);
    }
}

template <typename E, int M, int NT>
__device__ __forceinline__ void varlen_put(E *__restrict__ reg, const E (&v)[M]) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const int e = threadIdx.x + i * NT;
        reg[(e / M) * (M + 1) + e % M] = v[i];
    }
}

template <typename E, int M, int NT>
__device__ __forceinline__ void varlen_stage_out(E *__restrict__ dst, const E *__restrict__ reg,
                                                 const i64 *s_base, const int *s_cnt) {
#pragma unroll 4
    for (int i = 0; i < M; ++i) {
        const int e = threadIdx.x + i * NT;
        const int tau = e / M, k = e % M;
        if (k < s_cnt[tau]) dst[s_base[tau] + k] = reg[tau * (M + 1) + k];
    }
}

// Last block out resets the work counters (vector atomics only).
__device__ __forceinline__ void varlen_finish(int *counter) {
    if (threadIdx.x == 0) {
        __threadfence();
        const int done = atomicAdd(&counter[1], 1);
        if (done == (int)gridDim.x - 1) {
            atomicExch(&counter[0], 0);
            atomicExch(&counter[1], 0);
        }
    }
}

// Dynamic LDS of the uneven-batch kernels: staging region of NT (M + 1)
// elements of `Big` bytes (which also holds the solver scratch), then tile
// ranges, then `red_bytes` more.
template <int M, int NT>
constexpr size_t varlen_lds_bytes(size_t big, size_t red_bytes) {
    static_assert(M + 1 >= 6, "the staging region holds the reduced solve's 6 NT elements");
    return ((size_t)NT * (M + 1) * big + 15) / 16 * 16 + (size_t)NT * (8 + 4) + red_bytes;
}

// Reduced solve by Thomas (Alg. 1): the Thomas-Thomas hybrid of Section III-B.
// Each tile forms its row of the reduced system over the tiles' first unknowns
// (the same local elimination as the PCR form), then the first thread of each
// system runs Thomas over the system's P rows in LDS.  sh: 4 S elements; every
// thread of the block calls it (three barriers).
template <typename T, int M>
__device__ __forceinline__ void reduced_thomas(const TileState<T, M> &ts, T *__restrict__ sh, int S, int P, int p,
                                               int slot, T &f, T &lv) {
    T *ga = sh, *gb = sh + S, *gc = sh + 2 * S, *gd = sh + 3 * S;
    ga[slot] = ts.la;  // the tiles' last rows first
    gb[slot] = ts.lc;
    gc[slot] = ts.ld;
    __syncthreads();
    T pa = T(0), pc = T(0), pd = T(0);
    if (p > 0) {
        pa = ga[slot - 1];
        pc = gb[slot - 1];
        pd = gc[slot - 1];
    }
    __syncthreads();
    ga[slot] = -ts.fa * pa;
    gb[slot] = ts.fb - ts.fa * pc - ts.fc * ts.la;
    gc[slot] = -ts.fc * ts.lc;
    gd[slot] = ts.fd - ts.fa * pd - ts.fc * ts.ld;
    __syncthreads();
    if (p == 0) {  // Alg. 1 over rows slot .. slot + P - 1; c* kept in gc, x written to gd
        T cp = gc[slot] / gb[slot], dp = gd[slot] / gb[slot];
        gc[slot] = cp;
        gd[slot] = dp;
        for (int i = 1; i < P; ++i) {
            const T a = ga[slot + i];
            const T r = T(1) / (gb[slot + i] - a * cp);
            cp = r * gc[slot + i];
            dp = r * (gd[slot + i] - a * dp);
            gc[slot + i] = cp;
            gd[slot + i] = dp;
        }
        T x = dp;
        for (int i = P - 2; i >= 0; --i) {
            x = gd[slot + i] - gc[slot + i] * x;
            gd[slot + i] = x;
        }
    }
    __syncthreads();
    f = gd[slot];
    const T fn = (p + 1 < P) ? gd[slot + 1] : T(0);
    lv = ts.ld - ts.la * f - ts.lc * fn;
}

template <typename T, int M, int NT, bool THOMAS>
__global__ __launch_bounds__(NT) void k_varlen_plain(VarlenArgs g) {
    __shared__ int s_item;
    __shared__ short s_sys[NT], s_p[NT];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *reg = reinterpret_cast<T *>(smem_raw);
    i64 *s_base = reinterpret_cast<i64 *>(smem_raw + ((size_t)NT * (M + 1) * sizeof(T) + 15) / 16 * 16);
    int *s_cnt = reinterpret_cast<int *>(s_base + NT);
    // the reduced solve's scratch (6 NT elements) reuses the staging region:
    // the rows are in registers by then, and the solution goes back only after
    // a barrier
    T *red = reg;
    const T *arr[4] = {static_cast<const T *>(g.a), static_cast<const T *>(g.b), static_cast<const T *>(g.c),
                       static_cast<const T *>(g.d)};
    T *x = static_cast<T *>(g.x);
    const int t = threadIdx.x;
    const int pos = t * (M + 1);
    for (;;) {
        if (t == 0) s_item = atomicAdd(&g.counter[0], 1);
        __syncthreads();
        const int item = s_item;
        if (item >= g.nitems) break;
        int sys, p, P, n;
        varlen_assign<M, NT>(g, item, s_sys, s_p, s_base, s_cnt, sys, p, P, n);
        const bool act = sys >= 0;
        T ra[M], rb[M], rc[M], rd[M];
        // the next array's loads are issued before this one is staged where
        // registers allow it: small tiles, and 512-thread blocks (one block
        // per CU in any case, so up to 256 VGPRs cost no occupancy) of the PCR
        // variant; otherwise one array at a time
        constexpr bool pipe = M * sizeof(T) <= 64 || (NT >= 512 && M * sizeof(T) <= 128 && !THOMAS);
        T vn[M];
        varlen_load<T, M, NT>(vn, arr[0], s_base, s_cnt);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T vc[M];
            if (!pipe && r > 0) varlen_load<T, M, NT>(vn, arr[r], s_base, s_cnt);
#pragma unroll
            for (int k = 0; k < M; ++k) vc[k] = vn[k];
            if (pipe && r < 3) varlen_load<T, M, NT>(vn, arr[r + 1], s_base, s_cnt);
            varlen_put<T, M, NT>(reg, vc);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int row = p * M + k;
                const bool v = act && row < n;
                const T val = reg[pos + k];
                if (r == 0) ra[k] = (v && row > 0) ? val : T(0);
                if (r == 1) rb[k] = v ? val : T(1);
                if (r == 2) rc[k] = (v && row < n - 1) ? val : T(0);
                if (r == 3) rd[k] = v ? val : T(0);
            }
            __syncthreads();
        }
        TileState<T, M> ts;
        tile_eliminate<T, M>(ra, rb, rc, rd, ts);
        T f, lv;
        if constexpr (THOMAS)
            reduced_thomas<T, M>(ts, red, NT, P, p, t, f, lv);
        else
            reduced_pcr<T, M>(ts, red, NT, P, p, t, 1, f, lv, g.item_pmax[item]);
        T u[M];
        tile_backsub<T, M>(ts, f, lv, u);
        __syncthreads();  // the reduced solve's last reads of the shared region are done
#pragma unroll
        for (int k = 0; k < M; ++k) reg[pos + k] = u[k];
        __syncthreads();
        varlen_stage_out<T, M, NT>(x, reg, s_base, s_cnt);
        __syncthreads();  // s_item, s_sys, the staging region and red are reused by the next item
    }
    varlen_finish(g.counter);
}

template <int M, int NT>
__global__ __launch_bounds__(NT) void k_varlen_refine(VarlenArgs g) {
    __shared__ int s_item;
    __shared__ short s_sys[NT], s_p[NT];
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *reg = reinterpret_cast<double *>(smem_raw);
    float *regf = reinterpret_cast<float *>(smem_raw);
    i64 *s_base = reinterpret_cast<i64 *>(smem_raw + ((size_t)NT * (M + 1) * 8 + 15) / 16 * 16);
    int *s_cnt = reinterpret_cast<int *>(s_base + NT);
    // refinement scratch (2 NT doubles + 6 NT floats) inside the staging region,
    // used only between the barriers around refine_tile
    double *xb = reg;
    float *red = reinterpret_cast<float *>(xb + 2 * NT);
    const float *arr[3] = {static_cast<const float *>(g.a), static_cast<const float *>(g.b),
                           static_cast<const float *>(g.c)};
    const double *d = static_cast<const double *>(g.d);
    double *x = static_cast<double *>(g.x);
    const int t = threadIdx.x;
    const int pos = t * (M + 1);
    for (;;) {
        if (t == 0) s_item = atomicAdd(&g.counter[0], 1);
        __syncthreads();
        const int item = s_item;
        if (item >= g.nitems) break;
        int sys, p, P, n;
        varlen_assign<M, NT>(g, item, s_sys, s_p, s_base, s_cnt, sys, p, P, n);
        const bool act = sys >= 0;
        RefCoef<M, false> cf;
        cf.g0 = p * M;
        cf.n = act ? n : 0;
        float v[M];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            varlen_load<float, M, NT>(v, arr[r], s_base, s_cnt);
            varlen_put<float, M, NT>(regf, v);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const bool ok = act && p * M + k < n;
                const float val = regf[pos + k];
                if (r == 0) cf.a[k] = ok ? val : 0.f;
                if (r == 1) cf.b[k] = ok ? val : 1.f;
                if (r == 2) cf.c[k] = ok ? val : 0.f;
            }
            __syncthreads();
        }
        {
            double vd[M];
            varlen_load<double, M, NT>(vd, d, s_base, s_cnt);
            varlen_put<double, M, NT>(reg, vd);
        }
        __syncthreads();
        double dd[M];
#pragma unroll
        for (int k = 0; k < M; ++k) dd[k] = (act && p * M + k < n) ? reg[pos + k] : 0.0;
        double out[M];
        __syncthreads();  // every thread has read its d: the region becomes scratch
        refine_tile<M, false>(cf, dd, red, xb, NT, P, p, t, 1, out, g.item_pmax[item]);
        __syncthreads();  // scratch reads done: the region takes the solution
#pragma unroll
        for (int k = 0; k < M; ++k) reg[pos + k] = out[k];
        __syncthreads();
        varlen_stage_out<double, M, NT>(x, reg, s_base, s_cnt);
        __syncthreads();
    }
    varlen_finish(g.counter);
}

// ------------------------------------------------------------------- host --

namespace {

template <class K>
int occupancy_blocks(K kernel, int nt, size_t lds) {
    hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    return per_cu * cus;
}

template <typename K>
hipError_t launch_persistent(K kernel, int nt, size_t lds, const VarlenSchedule &sc, const VarlenArgs &g,
                             hipStream_t s) {
    launch(kernel, dim3((unsigned)sc.nblocks), dim3(nt), lds, s, g);
    return hipGetLastError();
}

}  // namespace

// The (M, NT) variants compiled for each precision.
// The first variant whose tiles hold the longest system is the default plan.
const std::vector<VarlenVariant> &varlen_variants(int prec) {
    static const std::vector<VarlenVariant> f64 = {{16, 512, 0, 1}, {8, 1024, 0, 1}, {8, 1024}, {16, 512},
                                                   {32, 256}, {8, 256}, {16, 512, 1}, {32, 256, 1}};
    static const std::vector<VarlenVariant> f32 = {{16, 512, 0, 1}, {32, 256, 0, 1}, {8, 1024}, {16, 512}, {32, 256},
                                                   {8, 256}, {16, 512, 1}, {32, 256, 1}};
    static const std::vector<VarlenVariant> ref = {{16, 512, 0, 1}, {8, 1024}, {16, 512}, {32, 256}, {8, 256}};
    return prec == 0 ? f64 : (prec == 1 ? f32 : ref);
}

namespace {

// Calls f(kernel, threads, dynamic LDS bytes) for the compiled variant (prec, M, NT).
template <class F>
auto with_kernel(int prec, int M, int NT, int thomas, F &&f) -> decltype(f(k_varlen_refine<16, 512>, 512, size_t(0))) {
    if (thomas && prec == 0) {
        if (M == 16) return f(k_varlen_plain<double, 16, 512, true>, 512, varlen_lds_bytes<16, 512>(8, 0));
        return f(k_varlen_plain<double, 32, 256, true>, 256, varlen_lds_bytes<32, 256>(8, 0));
    }
    if (thomas && prec == 1) {
        if (M == 16) return f(k_varlen_plain<float, 16, 512, true>, 512, varlen_lds_bytes<16, 512>(4, 0));
        return f(k_varlen_plain<float, 32, 256, true>, 256, varlen_lds_bytes<32, 256>(4, 0));
    }
    if (prec == 2) {
        if (M == 8 && NT == 1024)
            return f(k_varlen_refine<8, 1024>, 1024, varlen_lds_bytes<8, 1024>(8, 0));
        if (M == 16 && NT == 512)
            return f(k_varlen_refine<16, 512>, 512, varlen_lds_bytes<16, 512>(8, 0));
        if (M == 8 && NT == 256)
            return f(k_varlen_refine<8, 256>, 256, varlen_lds_bytes<8, 256>(8, 0));
        return f(k_varlen_refine<32, 256>, 256, varlen_lds_bytes<32, 256>(8, 0));
    }
    if (prec == 0) {
        if (M == 16 && NT == 512)
            return f(k_varlen_plain<double, 16, 512, false>, 512, varlen_lds_bytes<16, 512>(8, 0));
        if (M == 8 && NT == 1024)
            return f(k_varlen_plain<double, 8, 1024, false>, 1024, varlen_lds_bytes<8, 1024>(8, 0));
        if (M == 8 && NT == 256)
            return f(k_varlen_plain<double, 8, 256, false>, 256, varlen_lds_bytes<8, 256>(8, 0));
        return f(k_varlen_plain<double, 32, 256, false>, 256, varlen_lds_bytes<32, 256>(8, 0));
    }
    if (M == 16 && NT == 512)
        return f(k_varlen_plain<float, 16, 512, false>, 512, varlen_lds_bytes<16, 512>(4, 0));
    if (M == 8 && NT == 1024)
        return f(k_varlen_plain<float, 8, 1024, false>, 1024, varlen_lds_bytes<8, 1024>(4, 0));
    if (M == 8 && NT == 256)
        return f(k_varlen_plain<float, 8, 256, false>, 256, varlen_lds_bytes<8, 256>(4, 0));
    return f(k_varlen_plain<float, 32, 256, false>, 256, varlen_lds_bytes<32, 256>(4, 0));
}

}  // namespace

int varlen_blocks(int prec, const VarlenVariant &v) {
    if (v.wave) return varlen_wave_blocks(prec, v.M);
    return with_kernel(prec, v.M, v.NT, v.thomas, [&](auto k, int nt, size_t lds) { return occupancy_blocks(k, nt, lds); });
}

bool varlen_variant_fits(const VarlenVariant &v, i64 maxlen) { return (maxlen + v.M - 1) / v.M <= v.NT; }

void varlen_pack(const int64_t *offsets_host, std::vector<int> *ids, const VarlenVariant &v, std::vector<int> *tstart,
                 std::vector<int> *item_begin, std::vector<int> *item_pmax) {
    std::vector<int> &order = *ids;
    const i64 nsys = (i64)order.size();
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) {
        return offsets_host[i + 1] - offsets_host[i] > offsets_host[j + 1] - offsets_host[j];
    });
    tstart->assign(nsys, 0);
    item_begin->assign(1, 0);
    item_pmax->clear();
    int used = 0, pmax = 0;
    for (i64 k = 0; k < nsys; ++k) {
        const i64 len = offsets_host[order[k] + 1] - offsets_host[order[k]];
        const int P = (int)((len + v.M - 1) / v.M);
        if (used + P > v.NT) {  // close the current item (next fit, longest first)
            item_begin->push_back((int)k);
            item_pmax->push_back(pmax);
            used = 0;
            pmax = 0;
        }
        (*tstart)[k] = used;
        used += P;
        pmax = std::max(pmax, P);
    }
    item_begin->push_back((int)nsys);
    item_pmax->push_back(pmax);
}

namespace {

// Schedule of the systems `ids` (packed longest first into work items of at
// most NT tiles) for variant v.
hipError_t build_ids(const int64_t *offsets_host, std::vector<int> ids, int prec, const VarlenVariant &v,
                     VarlenSchedule *sc) {
    const i64 nsys = (i64)ids.size();
    sc->prec = prec;
    sc->M = v.M;
    sc->NT = v.NT;
    sc->nsys = nsys;
    std::vector<int> &order = ids;
    std::vector<int> tstart, item_begin, item_pmax;
    varlen_pack(offsets_host, &order, v, &tstart, &item_begin, &item_pmax);
    sc->nitems = (int)item_pmax.size();
    // one device allocation: off | order | tstart | item_begin | item_pmax | counter
    // (off holds every system's offsets; order names the systems of this schedule)
    const i64 nall = 1 + *std::max_element(order.begin(), order.end());
    const size_t b_off = sizeof(i64) * (nall + 1), b_ord = sizeof(int) * nsys, b_ts = sizeof(int) * nsys;
    const size_t b_ib = sizeof(int) * item_begin.size(), b_ip = sizeof(int) * item_pmax.size();
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t total = up(b_off) + up(b_ord) + up(b_ts) + up(b_ib) + up(b_ip) + 256;
    hipError_t e = hipMalloc(&sc->dev, total);
    if (e != hipSuccess) {
        sc->dev = nullptr;
        return e;
    }
    char *p = static_cast<char *>(sc->dev);
    sc->off = reinterpret_cast<i64 *>(p);
    p += up(b_off);
    sc->order = reinterpret_cast<int *>(p);
    p += up(b_ord);
    sc->tstart = reinterpret_cast<int *>(p);
    p += up(b_ts);
    sc->item_begin = reinterpret_cast<int *>(p);
    p += up(b_ib);
    sc->item_pmax = reinterpret_cast<int *>(p);
    p += up(b_ip);
    sc->counter = reinterpret_cast<int *>(p);
    if ((e = hipMemcpy(sc->off, offsets_host, b_off, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(sc->order, order.data(), b_ord, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(sc->tstart, tstart.data(), b_ts, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(sc->item_begin, item_begin.data(), b_ib, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(sc->item_pmax, item_pmax.data(), b_ip, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemset(sc->counter, 0, 2 * sizeof(int))) != hipSuccess) return e;
    sc->thomas = v.thomas;
    sc->nblocks =
        with_kernel(prec, v.M, v.NT, v.thomas, [&](auto k, int nt, size_t lds) { return occupancy_blocks(k, nt, lds); });
    sc->nblocks = std::max(1, std::min(sc->nblocks, sc->nitems));
    return hipSuccess;
}

}  // namespace

namespace {

// The systems longer than kVarlenMaxTiled: their list and the chunked solve's
// workspace (sized for the longest).
hipError_t build_long(const int64_t *off, const std::vector<int> &ids, int prec, VarlenSchedule *sc) {
    size_t ws = 0;
    for (int k : ids) {
        const i64 n = off[k + 1] - off[k];
        sc->long_off.push_back(off[k]);
        sc->long_len.push_back(n);
        LineReq q;
        q.f64 = prec == 0;
        q.inner = 1;
        q.n = n;
        q.outer = 1;
        ws = std::max(ws, prec == 2 ? long_refine_workspace(n, 1) : long_lines_workspace(q));
    }
    if (!ws) return hipSuccess;
    hipError_t e = hipMalloc(&sc->long_ws, ws);
    if (e != hipSuccess) sc->long_ws = nullptr;
    return e;
}

// The long systems, one chunked solve each (three launches; five passes for
// the refinement).
hipError_t launch_long_systems(const VarlenSchedule &sc, const void *a, const void *b, const void *c, const void *d,
                               void *x, hipStream_t s) {
    std::string err;
    for (size_t i = 0; i < sc.long_off.size(); ++i) {
        const i64 o = sc.long_off[i], n = sc.long_len[i];
        hipError_t e;
        if (sc.prec == 2) {
            LongRefineReq q;
            q.a = static_cast<const float *>(a) + o;
            q.b = static_cast<const float *>(b) + o;
            q.c = static_cast<const float *>(c) + o;
            q.d = static_cast<const double *>(d) + o;
            q.d_f64 = true;
            q.x = static_cast<double *>(x) + o;
            q.n = n;
            q.lines = 1;
            e = launch_long_refine(q, sc.long_ws, s, &err);
        } else {
            const size_t w = sc.prec == 0 ? 8 : 4;
            LineReq q;
            q.f64 = sc.prec == 0;
            q.mode = Mode::Arrays;
            q.out = Out::Store;
            q.a = static_cast<const char *>(a) + o * w;
            q.b = static_cast<const char *>(b) + o * w;
            q.c = static_cast<const char *>(c) + o * w;
            q.d = static_cast<const char *>(d) + o * w;
            q.x = static_cast<char *>(x) + o * w;
            q.inner = 1;
            q.n = n;
            q.outer = 1;
            e = launch_long_lines(q, sc.long_ws, s, &err);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t varlen_build(const int64_t *offsets_host, i64 nsys, int prec, const VarlenVariant &v, VarlenSchedule *sc,
                        const VarlenVariant *small) {
    std::vector<int> all, lng_all;
    for (i64 k = 0; k < nsys; ++k)
        (offsets_host[k + 1] - offsets_host[k] > kVarlenMaxTiled ? lng_all : all).push_back((int)k);
    hipError_t e = build_long(offsets_host, lng_all, prec, sc);
    if (e != hipSuccess) return e;
    if (all.empty()) {  // every system takes the chunked solve
        sc->prec = prec;
        sc->M = v.M;
        sc->NT = v.NT;
        sc->thomas = v.thomas;
        sc->wave = v.wave;
        sc->nsys = nsys;
        sc->nitems = 0;
        sc->nblocks = 0;
        return hipSuccess;
    }
    if (v.wave) return varlen_wave_build(offsets_host, all, prec, v, sc);
    if (!small) return build_ids(offsets_host, all, prec, v, sc);
    const i64 cap = (i64)small->M * small->NT;  // longest system the small-block variant holds
    std::vector<int> lng, shr;
    for (int k : all) (offsets_host[k + 1] - offsets_host[k] > cap ? lng : shr).push_back(k);
    if (lng.empty()) return build_ids(offsets_host, shr, prec, *small, sc);
    if (shr.empty()) return build_ids(offsets_host, lng, prec, v, sc);
    e = build_ids(offsets_host, lng, prec, v, sc);
    if (e != hipSuccess) return e;
    sc->next = new VarlenSchedule();
    return build_ids(offsets_host, shr, prec, *small, sc->next);
}

static hipError_t varlen_launch_tiled(const VarlenSchedule &sc, const void *a, const void *b, const void *c,
                                      const void *d, void *x, hipStream_t s);

hipError_t varlen_launch(const VarlenSchedule &sc, const void *a, const void *b, const void *c, const void *d,
                         void *x, hipStream_t s) {
    if (sc.nitems > 0) {
        hipError_t e = sc.wave ? varlen_wave_launch(sc, a, b, c, d, x, s) : varlen_launch_tiled(sc, a, b, c, d, x, s);
        if (e != hipSuccess) return e;
    }
    return launch_long_systems(sc, a, b, c, d, x, s);
}

static hipError_t varlen_launch_tiled(const VarlenSchedule &sc, const void *a, const void *b, const void *c,
                                      const void *d, void *x, hipStream_t s) {
    VarlenArgs g;
    g.a = a;
    g.b = b;
    g.c = c;
    g.d = d;
    g.x = x;
    g.off = sc.off;
    g.order = sc.order;
    g.tstart = sc.tstart;
    g.item_begin = sc.item_begin;
    g.item_pmax = sc.item_pmax;
    g.counter = sc.counter;
    g.nitems = sc.nitems;
    hipError_t e = with_kernel(sc.prec, sc.M, sc.NT, sc.thomas,
                               [&](auto k, int nt, size_t lds) { return launch_persistent(k, nt, lds, sc, g, s); });
    if (e != hipSuccess || !sc.next) return e;
    return varlen_launch_tiled(*sc.next, a, b, c, d, x, s);
}

void varlen_free(VarlenSchedule *sc) {
    sc->graphs.clear([](const VarlenSchedule::GraphKey &k, hipGraphExec_t g) {
        destroy_graph_exec(g, std::get<5>(k));
    });
    if (sc->dev) (void)hipFree(sc->dev);
    sc->dev = nullptr;
    if (sc->long_ws) (void)hipFree(sc->long_ws);
    sc->long_ws = nullptr;
    if (sc->next) {
        varlen_free(sc->next);
        delete sc->next;
        sc->next = nullptr;
    }
}

}  // namespace trid
