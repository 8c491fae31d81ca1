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

// Block-local assignment of threads to (system, tile) for one work item.
// Returns, per thread: system id (or -1), tile p, tile count P, row count n, row offset.
template <int M, int NT>
__device__ __forceinline__ void varlen_assign(const VarlenArgs &g, int item, short *s_sys, short *s_p, int &sys,
                                              int &p, int &P, int &n, i64 &base) {
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
    if (j >= 0) {
        sys = g.order[ib + j];
        base = g.off[sys];
        n = (int)(g.off[sys + 1] - base);
        P = (n + M - 1) / M;
        p = s_p[t];
    } else {
        sys = -1;
        base = 0;
        n = 0;
        P = 1;
        p = 0;
    }
}

// Last block out resets the work counters (vector atomics and stores only).
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

template <typename T, int M, int NT>
__global__ __launch_bounds__(NT) void k_varlen_plain(VarlenArgs g) {
    __shared__ int s_item;
    __shared__ short s_sys[NT], s_p[NT];
    __shared__ T red[6 * NT];
    const T *a = static_cast<const T *>(g.a), *b = static_cast<const T *>(g.b);
    const T *c = static_cast<const T *>(g.c), *d = static_cast<const T *>(g.d);
    T *x = static_cast<T *>(g.x);
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) s_item = atomicAdd(&g.counter[0], 1);
        __syncthreads();
        const int item = s_item;
        if (item >= g.nitems) break;
        int sys, p, P, n;
        i64 base;
        varlen_assign<M, NT>(g, item, s_sys, s_p, sys, p, P, n, base);
        const bool act = sys >= 0;
        T ra[M], rb[M], rc[M], rd[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int r = p * M + k;
            const bool v = act && r < n;
            const i64 o = base + r;
            ra[k] = (v && r > 0) ? a[o] : T(0);
            rb[k] = v ? b[o] : T(1);
            rc[k] = (v && r < n - 1) ? c[o] : T(0);
            rd[k] = v ? d[o] : T(0);
        }
        TileState<T, M> ts;
        tile_eliminate<T, M>(ra, rb, rc, rd, ts);
        T f, lv;
        reduced_pcr<T, M>(ts, red, NT, P, p, t, 1, f, lv, g.item_pmax[item]);
        T u[M];
        tile_backsub<T, M>(ts, f, lv, u);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int r = p * M + k;
            if (act && r < n) x[base + r] = u[k];
        }
        __syncthreads();  // s_item, s_sys and red are reused by the next item
    }
    varlen_finish(g.counter);
}

template <int M, int NT>
__global__ __launch_bounds__(NT) void k_varlen_refine(VarlenArgs g) {
    __shared__ int s_item;
    __shared__ short s_sys[NT], s_p[NT];
    __shared__ double xb[2 * NT];
    __shared__ float red[6 * NT];
    const float *a = static_cast<const float *>(g.a), *b = static_cast<const float *>(g.b);
    const float *c = static_cast<const float *>(g.c);
    const double *d = static_cast<const double *>(g.d);
    double *x = static_cast<double *>(g.x);
    const int t = threadIdx.x;
    for (;;) {
        if (t == 0) s_item = atomicAdd(&g.counter[0], 1);
        __syncthreads();
        const int item = s_item;
        if (item >= g.nitems) break;
        int sys, p, P, n;
        i64 base;
        varlen_assign<M, NT>(g, item, s_sys, s_p, sys, p, P, n, base);
        const bool act = sys >= 0;
        RefCoef<M, false> cf;
        cf.g0 = p * M;
        cf.n = act ? n : 0;
        double dd[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int r = p * M + k;
            const bool v = act && r < n;
            const i64 o = base + r;
            cf.a[k] = v ? a[o] : 0.f;
            cf.b[k] = v ? b[o] : 1.f;
            cf.c[k] = v ? c[o] : 0.f;
            dd[k] = v ? d[o] : 0.0;
        }
        double out[M];
        refine_tile<M, false>(cf, dd, red, xb, NT, P, p, t, 1, out, g.item_pmax[item]);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int r = p * M + k;
            if (act && r < n) x[base + r] = out[k];
        }
        __syncthreads();
    }
    varlen_finish(g.counter);
}

// ------------------------------------------------------------------- host --

namespace {

template <class K>
int occupancy_blocks(K kernel, int nt) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
    return per_cu * cus;
}

template <typename K>
hipError_t launch_persistent(K kernel, int nt, const VarlenSchedule &sc, const VarlenArgs &g, hipStream_t s) {
    hipLaunchKernelGGL(kernel, dim3((unsigned)sc.nblocks), dim3(nt), 0, s, g);
    return hipGetLastError();
}

}  // namespace

// The (M, NT) variants compiled for each precision.
const std::vector<VarlenVariant> &varlen_variants(int prec) {
    static const std::vector<VarlenVariant> f64 = {{16, 512}, {8, 1024}, {32, 256}};
    static const std::vector<VarlenVariant> f32 = {{16, 512}, {32, 256}, {8, 1024}};
    static const std::vector<VarlenVariant> ref = {{16, 512}, {32, 256}};
    return prec == 0 ? f64 : (prec == 1 ? f32 : ref);
}

namespace {

template <class F>
auto with_kernel(int prec, int M, int NT, F &&f) -> decltype(f(k_varlen_refine<16, 512>, 512)) {
    if (prec == 2) {
        if (M == 16 && NT == 512) return f(k_varlen_refine<16, 512>, 512);
        return f(k_varlen_refine<32, 256>, 256);
    }
    if (prec == 0) {
        if (M == 16 && NT == 512) return f(k_varlen_plain<double, 16, 512>, 512);
        if (M == 8 && NT == 1024) return f(k_varlen_plain<double, 8, 1024>, 1024);
        return f(k_varlen_plain<double, 32, 256>, 256);
    }
    if (M == 16 && NT == 512) return f(k_varlen_plain<float, 16, 512>, 512);
    if (M == 8 && NT == 1024) return f(k_varlen_plain<float, 8, 1024>, 1024);
    return f(k_varlen_plain<float, 32, 256>, 256);
}

}  // namespace

bool varlen_variant_fits(const VarlenVariant &v, i64 maxlen) { return (maxlen + v.M - 1) / v.M <= v.NT; }

hipError_t varlen_build(const int64_t *offsets_host, i64 nsys, int prec, const VarlenVariant &v,
                        VarlenSchedule *sc) {
    sc->prec = prec;
    sc->M = v.M;
    sc->NT = v.NT;
    sc->nsys = nsys;
    std::vector<int> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int i, int j) {
        return offsets_host[i + 1] - offsets_host[i] > offsets_host[j + 1] - offsets_host[j];
    });
    std::vector<int> tstart(nsys), item_begin(1, 0), item_pmax;
    int used = 0, pmax = 0;
    for (i64 k = 0; k < nsys; ++k) {
        const i64 len = offsets_host[order[k] + 1] - offsets_host[order[k]];
        const int P = (int)((len + v.M - 1) / v.M);
        if (used + P > v.NT) {  // close the current item (next fit, longest first)
            item_begin.push_back((int)k);
            item_pmax.push_back(pmax);
            used = 0;
            pmax = 0;
        }
        tstart[k] = used;
        used += P;
        pmax = std::max(pmax, P);
    }
    item_begin.push_back((int)nsys);
    item_pmax.push_back(pmax);
    sc->nitems = (int)item_pmax.size();
    // one device allocation: off | order | tstart | item_begin | item_pmax | counter
    const size_t b_off = sizeof(i64) * (nsys + 1), b_ord = sizeof(int) * nsys, b_ts = sizeof(int) * nsys;
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
    sc->nblocks = with_kernel(prec, v.M, v.NT, [&](auto k, int nt) { return occupancy_blocks(k, nt); });
    sc->nblocks = std::max(1, std::min(sc->nblocks, sc->nitems));
    return hipSuccess;
}

hipError_t varlen_launch(const VarlenSchedule &sc, const void *a, const void *b, const void *c, const void *d,
                         void *x, hipStream_t s) {
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
    return with_kernel(sc.prec, sc.M, sc.NT, [&](auto k, int nt) { return launch_persistent(k, nt, sc, g, s); });
}

void varlen_free(VarlenSchedule *sc) {
    for (auto &kv : sc->graphs) hipGraphExecDestroy(kv.second);
    sc->graphs.clear();
    if (sc->dev) hipFree(sc->dev);
    sc->dev = nullptr;
}

}  // namespace trid
