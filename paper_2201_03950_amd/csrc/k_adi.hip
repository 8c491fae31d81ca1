// k_adi.hip -- the explicit-stencil right-hand side of the ADI step (Alg. 3,
// line 2) fused with the x-line solve (Alg. 3, line 3): u is read once, the RHS
// d = 2 s L u is formed while staging the block's x lines into LDS, the rows
// (-s, 1 + 2 s, -s) are generated in-kernel (Section IV-A: coefficient
// generation fused into the solver), and only d is written.
#include <algorithm>

#include "dispatch.hpp"
#include "lines.hpp"

namespace trid {

// Staged source of the fused RHS (per-point s or constant s0).  Region 0 is
// d = 2 s L u computed while staging (7-point stencil in 3D, 5-point in 2D,
// zero outside the mesh); region 1 (per-point s only) is s itself.
template <typename T, bool PP, int NDIM>
struct StgRhs {
    static constexpr int kRegions = PP ? 2 : 1;
    const T *u;
    const T *s;
    T s0;
    int ny, nz;  // lines of one mesh = ny * nz (nz = 1 in 2D)

    template <int M>
    __device__ __forceinline__ void stage(int r, T *__restrict__ sh, i64 o0, int nl, int n, int ls,
                                          void *scratch) const {
        if (r == 1) {
            stage_in<T, M>(sh, s + o0 * n, nl * n, n, ls);
            return;
        }
        // neighbour-existence flags of the block's lines: bit0 y-1, bit1 y+1, bit2 z-1, bit3 z+1
        int *flags = static_cast<int *>(scratch);
        for (int ll = threadIdx.x; ll < nl; ll += blockDim.x) {
            const i64 o = o0 + ll;
            const int j = (int)(o % ny);
            const int k = (int)((o / ny) % nz);
            flags[ll] = (j > 0 ? 1 : 0) | (j < ny - 1 ? 2 : 0) | (k > 0 ? 4 : 0) | (k < nz - 1 ? 8 : 0);
        }
        __syncthreads();
        const i64 off = o0 * n;
        const i64 sy = n, sz = (i64)ny * n;
        const int cnt = nl * n;
        const int nt = blockDim.x;
        // each thread handles at most M elements (see stage_in): gather all
        // loads first so they are in flight together
        T uc[M], sum[M], sv[M];
        int ll = threadIdx.x / n, i = threadIdx.x % n;
        const int dl = nt / n, di = nt % n;
        int lls[M], is[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            lls[k] = ll;
            is[k] = i;
            const int e = threadIdx.x + k * nt;
            const bool v = e < cnt;
            const i64 q = off + e;
            const int f = v ? flags[ll] : 0;
            uc[k] = v ? u[q] : T(0);
            T acc = (v && i > 0) ? u[q - 1] : T(0);
            acc += (v && i < n - 1) ? u[q + 1] : T(0);
            if (f & 1) acc += u[q - sy];
            if (f & 2) acc += u[q + sy];
            if (NDIM == 3) {
                if (f & 4) acc += u[q - sz];
                if (f & 8) acc += u[q + sz];
            }
            sum[k] = acc;
            sv[k] = PP ? (v ? s[q] : T(0)) : s0;
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
            if (e < cnt) sh[staged_pos<M>(lls[k], is[k], ls)] = T(2) * sv[k] * (sum[k] - T(2 * NDIM) * uc[k]);
        }
    }

    template <int M>
    __device__ __forceinline__ void take(int r, const T *__restrict__ sh, int pos, int g0, int n, bool act,
                                         T (&ra)[M], T (&rb)[M], T (&rc)[M], T (&rd)[M]) const {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const int g = g0 + k;
            const bool v = act && g < n;
            if (r == 0) {
                rd[k] = v ? sh[pos + k] : T(0);
                if (!PP) {
                    const T sv = v ? s0 : T(0);
                    ra[k] = (g > 0) ? -sv : T(0);
                    rb[k] = T(1) + T(2) * sv;
                    rc[k] = (g < n - 1) ? -sv : T(0);
                }
            } else {
                const T sv = v ? sh[pos + k] : T(0);
                ra[k] = (g > 0) ? -sv : T(0);
                rb[k] = T(1) + T(2) * sv;
                rc[k] = (g < n - 1) ? -sv : T(0);
            }
        }
    }
};

namespace {

constexpr int kMaxThreads = 256;
constexpr size_t kMaxShmem = 64 * 1024;

i64 cdiv(i64 a, i64 b) { return (a + b - 1) / b; }

template <typename T, int M, bool PP, int NDIM>
hipError_t go(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    StagedGeom g;
    g.nlines = r.ny * r.nz * r.batch;
    g.n = (int)r.nx;
    g.L = pl.L;
    g.P = pl.P;
    g.ls = pl.ls;
    StgRhs<T, PP, NDIM> src{static_cast<const T *>(r.u), static_cast<const T *>(r.s), (T)r.s0,
                            (int)r.ny, (int)r.nz};
    StgOut<T> out{static_cast<T *>(r.d)};
    hipLaunchKernelGGL((k_staged<T, M, kMaxThreads, StgRhs<T, PP, NDIM>, StgOut<T>>),
                       dim3((unsigned)pl.nblocks), dim3(pl.threads()), pl.shmem, s, g, src, out);
    return hipGetLastError();
}

template <typename T, int M>
hipError_t go_m(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    const bool pp = r.s != nullptr;
    if (r.ndim == 3) return pp ? go<T, M, true, 3>(r, pl, s) : go<T, M, false, 3>(r, pl, s);
    return pp ? go<T, M, true, 2>(r, pl, s) : go<T, M, false, 2>(r, pl, s);
}

template <typename T>
hipError_t go_t(const AdiReq &r, const LinePlan &pl, hipStream_t s) {
    switch (pl.M) {
        case 8: return go_m<T, 8>(r, pl, s);
        case 16: return go_m<T, 16>(r, pl, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool plan_rhs_x(const AdiReq &r, LinePlan *pl, std::string *err) {
    const int w = r.f64 ? 8 : 4;
    LinePlan p;
    int M = r.force_M ? r.force_M : (r.f64 ? 8 : 16);
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
    int L = r.force_L ? r.force_L : std::max(1, kMaxThreads / (int)P);
    auto bytes = [&](int LL) {
        // one staging region + reduced-solve scratch (which also holds L ints of flags)
        return (size_t)LL * ls * w + std::max((size_t)6 * LL * P * w, (size_t)LL * 4);
    };
    while (bytes(L) > kMaxShmem && L > 1) L /= 2;
    if (bytes(L) > kMaxShmem || (i64)L * P > kMaxThreads) {
        *err = "fused stencil + x solve does not fit in LDS";
        return false;
    }
    p.M = M;
    p.P = (int)P;
    p.L = L;
    p.staged = true;
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
    return r.f64 ? go_t<double>(r, pl, s) : go_t<float>(r, pl, s);
}

}  // namespace trid
