// dispatch.hpp -- host-side description of one batched line-solve launch and the
// launch entry points implemented by the kernel translation units.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace trid {

using i64 = int64_t;

enum class Mode {
    Arrays,   // per-point a, b, c
    Const,    // scalar a, b, c
    S,        // a = c = -s, b = 1 + 2 s
    ArraysT,  // transposed per-point rows (adjoint)
    ST        // transposed s rows (adjoint)
};

enum class Out {
    Store,      // x = solution
    Add,        // x += solution
    AddKeep,    // x += solution and x2 = solution (a step that keeps its intermediates)
    AdjArrays,  // g = lambda; ga, gb, gc = coefficient gradients
    AdjS        // g = lambda; gs += lambda * second difference of xf
};

// Kernel launch used by every entry point.  When a per-kernel timer has armed
// a pair of events for this thread (and the stream is not being captured),
// the dispatch itself stamps the kernel's start and end into them
// (hipExtLaunchKernel), so a timed kernel's duration excludes the queue gaps
// that separately recorded events would include.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
LaunchEvents &launch_events();  // this thread's armed pair (defined with the timer)

template <typename... Args, typename F = void (*)(Args...)>
inline void launch(F kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t s, Args... args) {
    LaunchEvents &ev = launch_events();
    if (ev.start) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone) {
            hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)shmem, s, ev.start, ev.stop, 0u, args...);
            ev.used = true;
            return;
        }
    }
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

// Tile plan of a launch: M rows per tile, P tiles per line, L lines per block.
struct LinePlan {
    int M = 0;
    int L = 0;
    int P = 0;
    bool staged = false;  // contiguous lines through LDS (axis 0)
    bool lean = false;    // strided s-form lines, register-lean tiles (k_strided_lean)
    bool lanes = false;   // 64 / P whole lines per wavefront, 256 threads (fused stencil + x)
    bool vec = false;     // fused stencil + x, n = P M: 16-byte register-window staging (k_rhs_pp)
    int ls = 0;           // staged: LDS elements per line
    size_t shmem = 0;     // dynamic LDS bytes
    i64 nblocks = 0;
    int threads() const { return (lanes || vec) ? 256 : L * P; }
};

struct LineReq {
    bool f64 = true;
    Mode mode = Mode::Arrays;
    Out out = Out::Store;
    // d: right-hand side (adjoint epilogues: optional out-of-place rhs; NULL = g)
    const void *a = nullptr, *b = nullptr, *c = nullptr, *s = nullptr, *d = nullptr;
    double ca = 0, cb = 0, cc = 0;
    void *x = nullptr;         // Store / Add target
    void *x2 = nullptr;        // AddKeep: copy of the solution
    const void *xf = nullptr;  // forward solution (adjoints)
    void *g = nullptr, *ga = nullptr, *gb = nullptr, *gc = nullptr, *gs = nullptr;
    i64 inner = 1, n = 1, outer = 1;  // line stride, length, number of outer indices
    int force_M = 0, force_L = 0;     // plan overrides (0 = automatic)
    int force_strided = 0;            // 1: never use the staged kernel
};

// Choose the tile plan of a request (no HIP calls).  Returns false (with a
// message) when the line length is beyond what one workgroup can hold.
bool plan_lines(const LineReq &r, LinePlan *pl, std::string *err);

// Enqueue the solve described by r on stream s.
hipError_t launch_lines(const LineReq &r, const LinePlan &pl, hipStream_t s);

// ADI: RHS stencil fused with the x-line solve.  d = X^{-1} (2 s L u) for
// `batch` meshes of nx*ny*nz points (nz = 1 in 2D), s per point (s != NULL)
// or the constant s0.
struct AdiReq {
    bool f64 = true;
    int ndim = 3;
    const void *u = nullptr;
    const void *s = nullptr;
    double s0 = 0;
    void *d = nullptr;
    i64 nx = 1, ny = 1, nz = 1, batch = 1;
    int force_M = 0, force_L = 0;
};
bool plan_rhs_x(const AdiReq &r, LinePlan *pl, std::string *err);
hipError_t launch_rhs_x(const AdiReq &r, const LinePlan &pl, hipStream_t s);

// Constant-row fast path (host-tabulated elimination).  *_M return the tile
// size to use, or 0 when the request does not qualify (then the general
// kernels run).
int const_lines_M(const LineReq &r);
hipError_t launch_const_lines(const LineReq &r, int M, hipStream_t s);
int const_rhs_M(const AdiReq &r);
hipError_t launch_const_rhs_x(const AdiReq &r, int M, hipStream_t s);
// Launch geometry of launch_const_rhs_x (host only).
void const_rhs_geometry(const AdiReq &r, int M, int *threads, int *L, size_t *shmem, i64 *nblocks);

// Adjoint of the ADI right-hand side d = 2 s L u (per-point s), pointwise:
//   sbar += 2 rbar (L u);   ubar += 2 L (s rbar)   (L symmetric, zero ghosts).
struct StencilAdjReq {
    bool f64 = true;
    int ndim = 3;
    const void *u = nullptr, *s = nullptr, *rbar = nullptr;
    void *ubar = nullptr, *sbar = nullptr;
    i64 nx = 1, ny = 1, nz = 1, batch = 1;
};
hipError_t launch_stencil_adjoint(const StencilAdjReq &r, hipStream_t s);

// p[0..n) = v in dtype FP64 (f64) or FP32.
hipError_t launch_fill(void *p, bool f64, double v, i64 n, hipStream_t s);

}  // namespace trid
