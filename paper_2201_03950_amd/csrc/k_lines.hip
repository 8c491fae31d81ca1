// k_lines.cpp -- tile plans and launches of the batched line solves (gtsv along any
// axis, coefficient arrays / constants / per-point s, plain, update and adjoint
// epilogues).  Compiled as HIP for gfx950.
#include <algorithm>

#include "dispatch.hpp"
#include "adj_staged.hpp"
#include "lines.hpp"

namespace trid {

namespace {

constexpr int kStridedMaxThreads = 1024;
constexpr int kStagedMaxThreads = 256;

// Largest strided block for a tile of M rows of w-byte words: a thread keeps
// about 3M words of tile state plus its raw rows in VGPRs, so bigger tiles get
// fewer threads per block (and more VGPRs per thread) to avoid spills.  Wide
// epilogues (the update and the adjoints) keep more words per row in flight,
// so they drop one step earlier.
constexpr int strided_max_threads(int M, int w, bool wide = false) {
    const int b = wide ? 2 * M * w : M * w;
    return b <= 64 ? 1024 : (b <= 128 ? 512 : 256);
}
constexpr size_t kMaxShmem = 64 * 1024;

// Register-lean strided s-form solves (k_strided_lean): a thread keeps its
// tile's s and d (and a wide epilogue's M prefetched words), so up to 1024
// threads per block.  Used for lines of at least kLeanMinRows rows, where the
// general kernel's tile state limits a block to few adjacent lines.
constexpr int kLeanMinRows = 512;
constexpr int lean_max_threads(int M, int w, bool wide) {
    // 1024 threads (128 VGPRs) hold tiles of up to 64 bytes of s, and 16 FP64
    // rows without a wide epilogue; larger tiles take 512
    return (M * w <= 64 || (w == 8 && M == 16 && !wide)) ? 1024 : 512;
}

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

int staged_regions(Mode m) {
    switch (m) {
        case Mode::Arrays: return 4;
        case Mode::Const: return 1;
        case Mode::S: return 2;
        default: return 0;
    }
}

}  // namespace

bool plan_lines(const LineReq &r, LinePlan *pl, std::string *err) {
    const int w = r.f64 ? 8 : 4;
    LinePlan p;
    const bool adj_s = r.mode == Mode::ST && r.out == Out::AdjS;  // transposed s solve
    // the staged transposed solve keeps more arrays in flight: 8-row tiles
    // whenever a block can hold the line that way
    const bool adj_x = adj_s && r.inner == 1 && !r.force_strided && cdiv(r.n, 8) <= kStagedMaxThreads;
    int M = r.force_M ? r.force_M : ((r.f64 || adj_x) ? 8 : 16);
    // FP64 coefficient arrays on strided lines: 16-row tiles (fewer reduced-solve
    // levels for the four input streams; measured 8-12% faster than 8 rows)
    if (!r.force_M && r.f64 && r.mode == Mode::Arrays && r.inner > 1) M = 16;
    // FP64 generated rows on long strided lines (>= 128 tiles of 8): 16-row
    // tiles in 512-thread blocks (measured 7% faster on 1024-row y lines)
    if (!r.force_M && r.f64 && r.mode != Mode::Arrays && r.inner > 1 && cdiv(r.n, 8) >= 128) M = 16;
    // FP64 generated rows on x lines of about 1000 rows or more: 16-row staged
    // tiles when they fill their wavefronts as well as 8-row tiles do (measured
    // 3-12% faster on 1000-, 1024- and 2048-row lines; on 1536-row lines, whose
    // 96 tiles leave half a wavefront idle, 7% slower)
    if (!r.force_M && r.f64 && (r.mode == Mode::S || r.mode == Mode::Const) && r.inner == 1 &&
        r.out == Out::Store && r.n >= 1000) {
        auto fill = [](i64 tiles) { return (double)tiles / (64.0 * (double)cdiv(tiles, 64)); };
        if (fill(cdiv(r.n, 16)) >= fill(cdiv(r.n, 8))) M = 16;
    }
    if (M != 8 && M != 16 && M != 32) {
        *err = "tile size must be 8, 16 or 32";
        return false;
    }
    const bool wide = r.out != Out::Store;
    i64 P = cdiv(r.n, M);
    while (!r.force_M && P > strided_max_threads(M, w, wide) / 2 && M < 32) {
        M *= 2;
        P = cdiv(r.n, M);
    }
    int maxt = strided_max_threads(M, w, wide);
    if (P > maxt) {
        *err = "line too long for one workgroup";
        return false;
    }
    p.M = M;
    p.P = (int)P;
    // strided lines of per-point s, long enough that the general kernel's
    // block would hold few lines: the register-lean kernel, as many adjacent
    // lines per block as its 1024 threads allow (longer row segments); FP64
    // blocks stop at 512 threads, so two share a CU (measured 4% faster on
    // 1024-row lines in the grouped block order; FP32 was 8% slower so)
    if (r.mode == Mode::S && r.inner > 1 && r.n >= kLeanMinRows && r.n * r.inner < ((i64)1 << 31) &&
        (r.out == Out::Store || r.out == Out::Add || r.out == Out::AddKeep)) {
        const int Ml = r.force_M ? r.force_M : 16;
        const i64 Pl = cdiv(r.n, Ml);
        const int lmaxt = lean_max_threads(Ml, w, wide);
        if (Pl <= lmaxt) {
            const int tgt = r.f64 ? std::min(lmaxt, 512) : lmaxt;
            int L = r.force_L ? r.force_L : pow2_floor(std::max<i64>(1, tgt / Pl));
            if (!r.force_L) {
                if (r.inner < L) L = std::max(1, pow2_ceil(r.inner));
                while (L > 4 && cdiv(r.inner, L) * r.outer < 512) L /= 2;
            }
            if ((i64)L * Pl <= lmaxt) {
                p.M = Ml;
                p.P = (int)Pl;
                p.L = L;
                p.lean = true;
                p.shmem = (size_t)6 * L * Pl * w;
                p.nblocks = cdiv(r.inner, L) * r.outer;
                if (p.nblocks < (i64)1 << 31) {
                    *pl = p;
                    return true;
                }
            }
        }
    }
    const int regions = staged_regions(r.mode);
    // The staged kernel holds a line of up to kStagedMaxThreads tiles: longer
    // x lines take bigger tiles there when the LDS holds the line (measured
    // 1.6-2.0x faster than the strided kernel on 4096-row FP64 lines with
    // 16-row tiles, 2.0-2.7x on 8192-row FP32 lines with 32-row tiles)
    int Ms = M;
    i64 Ps = P;
    if (r.inner == 1 && !r.force_M && regions > 0 && r.out == Out::Store)
        while (Ps > kStagedMaxThreads && Ms < 32) {
            Ms *= 2;
            Ps = cdiv(r.n, Ms);
        }
    const bool want_staged = r.inner == 1 && !r.force_strided &&
                             ((regions > 0 && r.out == Out::Store) || (adj_s && M <= 16)) &&
                             Ps <= kStagedMaxThreads;
    if (want_staged) {
        // about one wavefront per block: the block's barriers then cost little
        // and many blocks per CU overlap their load, solve and store phases
        // (measured faster than 256-thread blocks for line lengths 128..256)
        int L = r.force_L ? r.force_L : std::max(1, 64 / (int)Ps);
        L = std::max(1, std::min(L, pow2_ceil(r.outer)));
        const int ls = (int)Ps * (Ms + 1);
        auto bytes = [&](int LL) {  // one staging region + reduced-solve scratch
            return (size_t)LL * ls * w + (size_t)6 * LL * Ps * w;
        };
        while (bytes(L) > kMaxShmem && L > 1) L /= 2;
        if (bytes(L) <= kMaxShmem && L * Ps <= kStagedMaxThreads) {
            p.M = Ms;
            p.P = (int)Ps;
            p.staged = true;
            p.L = L;
            p.ls = ls;
            p.shmem = bytes(L);
            p.nblocks = cdiv(r.outer, L);
            *pl = p;
            return true;
        }
    }
    // x lines of over 4096 rows that do not stage (FP64 lines whose 32-row
    // tiles exceed the LDS): each lane reads its own tile's rows, and 8-row
    // tiles (the most lanes per line, the shortest per-lane segments) stream
    // best: measured 1.3-1.5x faster than 16 or 32 rows on 8192-row FP64 lines
    if (r.inner == 1 && !r.force_M && M != 8 && r.n > 4096 && r.out == Out::Store &&
        (r.mode == Mode::S || r.mode == Mode::Arrays) && cdiv(r.n, 8) <= strided_max_threads(8, w, wide)) {
        M = 8;
        P = cdiv(r.n, 8);
        maxt = strided_max_threads(8, w, wide);
        p.M = M;
        p.P = (int)P;
    }
    int L = r.force_L;
    if (!L) {
        if (r.mode == Mode::Arrays || r.mode == Mode::ArraysT) {
            L = std::min(64, pow2_floor(maxt / P));  // four input streams: long row segments
        } else {
            // 64-byte row segments per tile; twice that when the grid would
            // otherwise be small (fewer than 4096 blocks)
            L = 64 / w;
            if (cdiv(r.inner, L) * r.outer < 4096) L *= 2;
            L = std::min(L, pow2_floor(maxt / P));
        }
        if (r.inner < L) L = std::max(1, pow2_ceil(r.inner));
        // small batches are latency-bound: keep at least two blocks per CU
        while (L > 4 && cdiv(r.inner, L) * r.outer < 512) L /= 2;
    }
    if ((i64)L * P > maxt) {
        *err = "plan exceeds 1024 threads per block";
        return false;
    }
    p.staged = false;
    p.L = L;
    p.shmem = (size_t)6 * L * P * w;
    p.nblocks = cdiv(r.inner, L) * r.outer;
    if (p.nblocks >= (i64)1 << 31) {
        *err = "too many blocks";
        return false;
    }
    *pl = p;
    return true;
}

namespace {

template <typename T, int M, class Src, class Epi>
hipError_t go_strided(const LineReq &r, const LinePlan &pl, Src src, Epi epi, hipStream_t s) {
    StridedGeom g;
    g.inner = r.inner;
    g.nib = cdiv(r.inner, pl.L);
    g.n = (int)r.n;
    g.L = pl.L;
    g.P = pl.P;
    constexpr int MAXT = strided_max_threads(M, (int)sizeof(T), Epi::kWide);
    launch((k_strided<T, M, MAXT, Src, Epi>), dim3((unsigned)pl.nblocks),
                       dim3(pl.threads()), pl.shmem, s, g, src, epi);
    return hipGetLastError();
}

template <typename T, class Src, class Epi>
hipError_t strided_M(const LineReq &r, const LinePlan &pl, Src src, Epi epi, hipStream_t s) {
    switch (pl.M) {
        case 8: return go_strided<T, 8>(r, pl, src, epi, s);
        case 16: return go_strided<T, 16>(r, pl, src, epi, s);
        case 32: return go_strided<T, 32>(r, pl, src, epi, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int M, int OUT>
hipError_t go_lean(const LineReq &r, const LinePlan &pl, hipStream_t s) {
    StridedGeom g;
    g.inner = r.inner;
    g.nib = cdiv(r.inner, pl.L);
    g.n = (int)r.n;
    g.L = pl.L;
    g.P = pl.P;
    constexpr int MAXT = lean_max_threads(M, (int)sizeof(T), OUT != 0);
    launch((k_strided_lean<T, M, MAXT, OUT>), dim3((unsigned)pl.nblocks), dim3(pl.threads()), pl.shmem, s, g,
           static_cast<const T *>(r.s), static_cast<const T *>(r.d), static_cast<T *>(r.x), static_cast<T *>(r.x2));
    return hipGetLastError();
}

template <typename T, int OUT>
hipError_t lean_M(const LineReq &r, const LinePlan &pl, hipStream_t s) {
    switch (pl.M) {
        case 8: return go_lean<T, 8, OUT>(r, pl, s);
        case 16: return go_lean<T, 16, OUT>(r, pl, s);
        case 32: return go_lean<T, 32, OUT>(r, pl, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int M, class Src>
hipError_t go_staged(const LineReq &r, const LinePlan &pl, Src src, hipStream_t s) {
    StagedGeom g;
    g.nlines = r.outer;
    g.n = (int)r.n;
    g.L = pl.L;
    g.P = pl.P;
    g.ls = pl.ls;
    StgOut<T> out{static_cast<T *>(r.x)};
    launch((k_staged<T, M, kStagedMaxThreads, Src, StgOut<T>>),
                       dim3((unsigned)pl.nblocks), dim3(pl.threads()), pl.shmem, s, g, src, out);
    return hipGetLastError();
}

template <typename T, class Src>
hipError_t staged_M(const LineReq &r, const LinePlan &pl, Src src, hipStream_t s) {
    switch (pl.M) {
        case 8: return go_staged<T, 8>(r, pl, src, s);
        case 16: return go_staged<T, 16>(r, pl, src, s);
        case 32: return go_staged<T, 32>(r, pl, src, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int M>
hipError_t go_staged_adj_s(const LineReq &r, const LinePlan &pl, hipStream_t s) {
    StagedGeom g;
    g.nlines = r.outer;
    g.n = (int)r.n;
    g.L = pl.L;
    g.P = pl.P;
    g.ls = pl.ls;
    const T *grhs = static_cast<const T *>(r.d ? r.d : r.g);
    launch((k_staged_adj_s<T, M>), dim3((unsigned)pl.nblocks), dim3(pl.threads()), pl.shmem, s, g,
                       static_cast<const T *>(r.s), grhs, static_cast<const T *>(r.xf), static_cast<T *>(r.g),
                       static_cast<T *>(r.gs));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_typed(const LineReq &r, const LinePlan &pl, hipStream_t s) {
    const T *a = static_cast<const T *>(r.a), *b = static_cast<const T *>(r.b);
    const T *c = static_cast<const T *>(r.c), *sp = static_cast<const T *>(r.s);
    const T *d = static_cast<const T *>(r.d);
    T *x = static_cast<T *>(r.x);
    if (pl.lean) {
        switch (r.out) {
            case Out::Store: return lean_M<T, 0>(r, pl, s);
            case Out::Add: return lean_M<T, 1>(r, pl, s);
            case Out::AddKeep: return lean_M<T, 2>(r, pl, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (pl.staged && r.out == Out::AdjS) {
        switch (pl.M) {
            case 8: return go_staged_adj_s<T, 8>(r, pl, s);
            case 16: return go_staged_adj_s<T, 16>(r, pl, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (pl.staged) {
        switch (r.mode) {
            case Mode::Arrays: return staged_M<T>(r, pl, StgArrays<T>{a, b, c, d}, s);
            case Mode::Const:
                return staged_M<T>(r, pl, StgConst<T>{(T)r.ca, (T)r.cb, (T)r.cc, d}, s);
            case Mode::S: return staged_M<T>(r, pl, StgS<T>{sp, d}, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (r.out == Out::Store) {
        switch (r.mode) {
            case Mode::Arrays: return strided_M<T>(r, pl, SrcArrays<T>{a, b, c, d}, EpiStore<T>{x}, s);
            case Mode::Const:
                return strided_M<T>(r, pl, SrcConst<T>{(T)r.ca, (T)r.cb, (T)r.cc, d}, EpiStore<T>{x}, s);
            case Mode::S: return strided_M<T>(r, pl, SrcS<T>{sp, d}, EpiStore<T>{x}, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (r.out == Out::Add) {
        switch (r.mode) {
            case Mode::Const:
                return strided_M<T>(r, pl, SrcConst<T>{(T)r.ca, (T)r.cb, (T)r.cc, d}, EpiAdd<T>{x}, s);
            case Mode::S: return strided_M<T>(r, pl, SrcS<T>{sp, d}, EpiAdd<T>{x}, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (r.out == Out::AddKeep && r.mode == Mode::S)
        return strided_M<T>(r, pl, SrcS<T>{sp, d}, EpiAddKeep<T>{x, static_cast<T *>(r.x2)}, s);
    const T *xf = static_cast<const T *>(r.xf);
    // adjoint right-hand side: r.d if given (out of place), else g itself
    const T *grhs = r.d ? d : static_cast<const T *>(r.g);
    if (r.out == Out::AdjArrays && r.mode == Mode::ArraysT) {
        EpiAdjArrays<T> e{xf, static_cast<T *>(r.g), static_cast<T *>(r.ga), static_cast<T *>(r.gb),
                          static_cast<T *>(r.gc)};
        return strided_M<T>(r, pl, SrcArraysT<T>{a, b, c, grhs}, e, s);
    }
    if (r.out == Out::AdjS && r.mode == Mode::ST) {
        EpiAdjS<T> e{xf, static_cast<T *>(r.g), static_cast<T *>(r.gs)};
        return strided_M<T>(r, pl, SrcST<T>{sp, grhs}, e, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_lines(const LineReq &r, const LinePlan &pl, hipStream_t s) {
    return r.f64 ? launch_typed<double>(r, pl, s) : launch_typed<float>(r, pl, s);
}

}  // namespace trid
