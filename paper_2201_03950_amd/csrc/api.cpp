// api.cpp -- the extern "C" boundary declared in include/trid.h: handles,
// argument validation (always before any HIP call), tile planning, workspace,
// hipGraph capture of ADI steps, and dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/trid.h"
#include "dispatch.hpp"
#include "ext.hpp"
#include "graph_cache.hpp"
#include "long_lines.hpp"
#include "resident.hpp"

using trid::i64;

namespace {

std::string g_create_error;

// Identity of a captured ADI run: everything the captured launches depend on,
// including the forced tile plan (trid_set_tile).
struct GraphKey {
    const void *u, *s;
    double s0;
    int dt, ndim;
    i64 nx, ny, nz, batch;
    int nsteps;
    int force_M, force_L;
    hipStream_t stream;
    bool operator<(const GraphKey &o) const {
        return std::tie(u, s, s0, dt, ndim, nx, ny, nz, batch, nsteps, force_M, force_L, stream) <
               std::tie(o.u, o.s, o.s0, o.dt, o.ndim, o.nx, o.ny, o.nz, o.batch, o.nsteps, o.force_M, o.force_L,
                        o.stream);
    }
};

// Captured ADI runs kept per handle (least recently used evicted beyond this).
constexpr size_t kAdiGraphCap = 16;

}  // namespace

struct trid_handle_s {
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    bool used = false;                // work has been enqueued on `stream`
    hipEvent_t order_ev = nullptr;    // orders work across a stream switch
    std::string err;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    trid::LruMap<GraphKey, hipGraphExec_t> graphs{kAdiGraphCap};
    trid::ExtState ext;  // state of the extension entry points (refine, varlen, adjoint, plans)
};

namespace {

int fail(trid_handle_t h, int code, const std::string &msg) {
    if (h) h->err = msg;
    return code;
}

int hip_fail(trid_handle_t h, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(h, TRID_ERR_HIP, m);
}

bool dtype_ok(int dt) { return dt == TRID_F32 || dt == TRID_F64; }

// Validate mesh arguments; on success fill the line geometry of `axis`.
// long_ok: contiguous lines up to TRID_MAX_LONG_LINE are accepted (the
// chunked solve of run_lines).
int check_mesh(trid_handle_t h, int ndim, const int64_t *dims, int axis, int64_t batch, i64 *inner,
               i64 *n, i64 *outer, bool long_ok = false) {
    if (ndim < 1 || ndim > 3) return fail(h, TRID_ERR_ARG, "ndim must be 1, 2 or 3");
    if (!dims) return fail(h, TRID_ERR_ARG, "dims is NULL");
    if (axis < 0 || axis >= ndim) return fail(h, TRID_ERR_ARG, "axis out of range");
    if (batch < 1) return fail(h, TRID_ERR_ARG, "batch must be >= 1");
    i64 total = batch;
    for (int k = 0; k < ndim; ++k) {
        if (dims[k] < 1) return fail(h, TRID_ERR_ARG, "every dim must be >= 1");
        if (total > ((i64)1 << 50) / dims[k]) return fail(h, TRID_ERR_ARG, "mesh too large");
        total *= dims[k];
    }
    i64 in = 1, out = batch;
    for (int k = 0; k < axis; ++k) in *= dims[k];
    for (int k = axis + 1; k < ndim; ++k) out *= dims[k];
    if (dims[axis] > TRID_MAX_LINE) {
        if (!long_ok || in != 1)
            return fail(h, TRID_ERR_UNSUPPORTED, "line length exceeds TRID_MAX_LINE");
        if (dims[axis] > TRID_MAX_LONG_LINE)
            return fail(h, TRID_ERR_UNSUPPORTED, "line length exceeds TRID_MAX_LONG_LINE");
        if (out * 2 * ((dims[axis] + 2047) / 2048) >= ((i64)1 << 31))
            return fail(h, TRID_ERR_UNSUPPORTED, "too many long lines in one call");
    }
    *inner = in;
    *n = dims[axis];
    *outer = out;
    return TRID_OK;
}

int run_long_lines(trid_handle_t h, const trid::LineReq &r);

void drop_adi_graph(const GraphKey &k, hipGraphExec_t g) { trid::destroy_graph_exec(g, k.stream); }

int run_lines(trid_handle_t h, const trid::LineReq &r) {
    h->used = true;
    if (r.n > TRID_MAX_LINE) return run_long_lines(h, r);
    trid::LinePlan pl;
    std::string msg;
    trid::LineReq rr = r;
    h->ext.apply_overrides(&rr);
    hipError_t e;
    const int cm = trid::const_lines_M(rr);
    if (cm) {
        e = h->ext.timer.time(rr.inner == 1 ? "gtsv_const_staged" : "gtsv_const_strided", h->stream,
                              [&] { return trid::launch_const_lines(rr, cm, h->stream); });
        if (e != hipSuccess) return hip_fail(h, e, "line-solve launch");
        h->err.clear();
        return TRID_OK;
    }
    if (!trid::plan_lines(rr, &pl, &msg)) return fail(h, TRID_ERR_UNSUPPORTED, msg);
    e = h->ext.timer.time(pl.staged ? "gtsv_staged" : "gtsv_strided", h->stream,
                          [&] { return trid::launch_lines(rr, pl, h->stream); });
    if (e != hipSuccess) return hip_fail(h, e, "line-solve launch");
    h->err.clear();
    return TRID_OK;
}

}  // namespace

// ------------------------------------------------------------------ handle --

namespace trid {

hipStream_t handle_stream(trid_handle_t h) {
    h->used = true;  // every caller of this enqueues work on the stream
    return h->stream;
}
size_t handle_adi_graphs(trid_handle_t h) { return h->graphs.size(); }
size_t handle_adi_graph_cap() { return kAdiGraphCap; }
ExtState &handle_ext(trid_handle_t h) { return h->ext; }
int handle_fail(trid_handle_t h, int code, const std::string &msg) { return fail(h, code, msg); }
int handle_hip_fail(trid_handle_t h, hipError_t e, const char *what) { return hip_fail(h, e, what); }
int handle_check_mesh(trid_handle_t h, int ndim, const int64_t *dims, int axis, int64_t batch,
                      i64 *inner, i64 *n, i64 *outer, bool long_ok) {
    return check_mesh(h, ndim, dims, axis, batch, inner, n, outer, long_ok);
}
int handle_run_lines(trid_handle_t h, const LineReq &r) { return run_lines(h, r); }

// With TRID_FAIL_ALLOC set (to anything), every workspace allocation fails
// with TRID_ERR_ALLOC before any HIP call: a host-forced failure for testing
// the error path.
bool alloc_failure_forced() { return getenv("TRID_FAIL_ALLOC") != nullptr; }

// Grow the handle's workspace to at least `bytes` (invalidates captured graphs).
int handle_workspace(trid_handle_t h, size_t bytes, void **ptr) {
    if (alloc_failure_forced()) return fail(h, TRID_ERR_ALLOC, "workspace allocation failed (TRID_FAIL_ALLOC)");
    if (h->ws_bytes < bytes) {
        if (h->ws) {
            hipError_t e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "hipStreamSynchronize");
            h->graphs.clear(drop_adi_graph);
            hipFree(h->ws);
            h->ws = nullptr;
            h->ws_bytes = 0;
        }
        hipError_t e = hipMalloc(&h->ws, bytes);
        if (e != hipSuccess) {
            h->ws = nullptr;
            return fail(h, TRID_ERR_ALLOC, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
        }
        h->ws_bytes = bytes;
    }
    *ptr = h->ws;
    return TRID_OK;
}

}  // namespace trid

namespace {

// Contiguous lines longer than TRID_MAX_LINE: chunk pass, reduced lines, solve
// pass, with the reduced rows in the handle's workspace.
int run_long_lines(trid_handle_t h, const trid::LineReq &r) {
    h->used = true;
    void *ws = nullptr;
    int rc = trid::handle_workspace(h, trid::long_lines_workspace(r), &ws);
    if (rc) return rc;
    std::string msg;
    hipError_t e = h->ext.timer.time_recorded("gtsv_long", h->stream,
                                              [&] { return trid::launch_long_lines(r, ws, h->stream, &msg); });
    if (e != hipSuccess) {
        if (!msg.empty()) return fail(h, TRID_ERR_UNSUPPORTED, msg);
        return hip_fail(h, e, "long line-solve launch");
    }
    h->err.clear();
    return TRID_OK;
}

}  // namespace

extern "C" {

int trid_version(void) { return 10100; }

int trid_create(trid_handle_t *h) {
    if (!h) {
        g_create_error = "h is NULL";
        return TRID_ERR_ARG;
    }
    *h = nullptr;
    trid_handle_t p = new (std::nothrow) trid_handle_s();
    if (!p) {
        g_create_error = "out of host memory";
        return TRID_ERR_ALLOC;
    }
    *h = p;
    // TRID_PLAN_CACHE names a plan file: loaded here when it exists, written
    // back when the handle is destroyed
    if (const char *path = getenv("TRID_PLAN_CACHE")) {
        if (FILE *f = fopen(path, "r")) {
            fclose(f);
            trid_plan_load(p, path);
        }
    }
    return TRID_OK;
}

int trid_destroy(trid_handle_t h) {
    if (!h) return TRID_OK;
    if (const char *path = getenv("TRID_PLAN_CACHE"))
        if (!h->ext.tuned.empty()) trid_plan_save(h, path);
    if (h->ws || h->graphs.size() || h->capture_stream || h->ext.has_device_state()) {
        hipStreamSynchronize(h->stream);
        h->graphs.clear(drop_adi_graph);
        h->ext.release();
        if (h->ws) hipFree(h->ws);
        if (h->capture_stream) hipStreamDestroy(h->capture_stream);
    }
    if (h->order_ev) hipEventDestroy(h->order_ev);
    delete h;
    return TRID_OK;
}

int trid_set_stream(trid_handle_t h, trid_stream_t stream) {
    if (!h) return TRID_ERR_ARG;
    hipStream_t ns = static_cast<hipStream_t>(stream);
    if (ns == h->stream) return TRID_OK;
    if (h->used) {
        // The handle's workspace, work counters and schedules are shared by its
        // calls: work enqueued on the new stream waits for the work already
        // enqueued on the old one, so calls of one handle never overlap.  (Not
        // possible across a graph capture; a capturing caller keeps one stream.)
        hipStreamCaptureStatus c0 = hipStreamCaptureStatusNone, c1 = hipStreamCaptureStatusNone;
        hipError_t e = hipStreamIsCapturing(h->stream, &c0);
        if (e == hipSuccess) e = hipStreamIsCapturing(ns, &c1);
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamIsCapturing");
        if (c0 == hipStreamCaptureStatusNone && c1 == hipStreamCaptureStatusNone) {
            if (!h->order_ev) {
                e = hipEventCreateWithFlags(&h->order_ev, hipEventDisableTiming);
                if (e != hipSuccess) {
                    h->order_ev = nullptr;
                    return hip_fail(h, e, "hipEventCreate");
                }
            }
            e = hipEventRecord(h->order_ev, h->stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(ns, h->order_ev, 0);
            if (e != hipSuccess) return hip_fail(h, e, "stream switch ordering");
        }
    }
    h->stream = ns;
    return TRID_OK;
}

const char *trid_last_error(trid_handle_t h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int trid_gtsv_batched(trid_handle_t h, trid_dtype_t dt, const void *a, const void *b, const void *c,
                      void *d, int ndim, const int64_t *dims, int axis, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (!dtype_ok(dt)) return fail(h, TRID_ERR_ARG, "bad dtype");
    if (!a || !b || !c || !d) return fail(h, TRID_ERR_ARG, "NULL data pointer");
    trid::LineReq r;
    int rc = check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer, true);
    if (rc) return rc;
    r.f64 = dt == TRID_F64;
    r.mode = trid::Mode::Arrays;
    r.out = trid::Out::Store;
    r.a = a;
    r.b = b;
    r.c = c;
    r.d = d;
    r.x = d;
    return run_lines(h, r);
}

int trid_gtsv_batched_const(trid_handle_t h, trid_dtype_t dt, double a, double b, double c, void *d,
                            int ndim, const int64_t *dims, int axis, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (!dtype_ok(dt)) return fail(h, TRID_ERR_ARG, "bad dtype");
    if (!d) return fail(h, TRID_ERR_ARG, "NULL data pointer");
    trid::LineReq r;
    int rc = check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer, true);
    if (rc) return rc;
    r.f64 = dt == TRID_F64;
    r.mode = trid::Mode::Const;
    r.out = trid::Out::Store;
    r.ca = a;
    r.cb = b;
    r.cc = c;
    r.d = d;
    r.x = d;
    return run_lines(h, r);
}

int trid_gtsv_batched_s(trid_handle_t h, trid_dtype_t dt, const void *s, void *d, int ndim,
                        const int64_t *dims, int axis, int64_t batch) {
    if (!h) return TRID_ERR_ARG;
    if (!dtype_ok(dt)) return fail(h, TRID_ERR_ARG, "bad dtype");
    if (!s || !d) return fail(h, TRID_ERR_ARG, "NULL data pointer");
    trid::LineReq r;
    int rc = check_mesh(h, ndim, dims, axis, batch, &r.inner, &r.n, &r.outer, true);
    if (rc) return rc;
    r.f64 = dt == TRID_F64;
    r.mode = trid::Mode::S;
    r.out = trid::Out::Store;
    r.s = s;
    r.d = d;
    r.x = d;
    return run_lines(h, r);
}

// Enqueue the launches of `nsteps` ADI steps on stream `st`.
static int adi_enqueue(trid_handle_t h, bool f64, void *u, const void *s, double s0, int ndim,
                       i64 nx, i64 ny, i64 nz, i64 batch, int nsteps, void *dws, hipStream_t st,
                       bool timed = true) {
    trid::AdiReq ar;
    ar.f64 = f64;
    ar.ndim = ndim;
    ar.u = u;
    ar.s = s;
    ar.s0 = s0;
    ar.d = dws;
    ar.nx = nx;
    ar.ny = ny;
    ar.nz = nz;
    ar.batch = batch;
    h->ext.apply_adi_overrides(&ar);
    trid::LinePlan px, py, pz;
    std::string msg;
    const int cmx = trid::const_rhs_M(ar);
    if (!cmx && !trid::plan_rhs_x(ar, &px, &msg)) return fail(h, TRID_ERR_UNSUPPORTED, msg);
    trid::LineReq ry;
    ry.f64 = f64;
    ry.mode = s ? trid::Mode::S : trid::Mode::Const;
    ry.ca = -s0;
    ry.cb = 1.0 + 2.0 * s0;
    ry.cc = -s0;
    ry.s = s;
    ry.d = dws;
    ry.inner = nx;
    ry.n = ny;
    ry.outer = nz * batch;
    ry.out = (ndim == 2) ? trid::Out::Add : trid::Out::Store;
    ry.x = (ndim == 2) ? u : dws;
    h->ext.apply_overrides(&ry);
    const int cmy = trid::const_lines_M(ry);
    if (!cmy && !trid::plan_lines(ry, &py, &msg)) return fail(h, TRID_ERR_UNSUPPORTED, msg);
    trid::LineReq rz = ry;
    int cmz = 0;
    if (ndim == 3) {
        rz.inner = nx * ny;
        rz.n = nz;
        rz.outer = batch;
        rz.out = trid::Out::Add;
        rz.x = u;
        h->ext.apply_overrides(&rz);
        cmz = trid::const_lines_M(rz);
        if (!cmz && !trid::plan_lines(rz, &pz, &msg)) return fail(h, TRID_ERR_UNSUPPORTED, msg);
    }
    auto run_x = [&]() {
        return cmx ? trid::launch_const_rhs_x(ar, cmx, st) : trid::launch_rhs_x(ar, px, st);
    };
    auto run_y = [&]() {
        return cmy ? trid::launch_const_lines(ry, cmy, st) : trid::launch_lines(ry, py, st);
    };
    auto run_z = [&]() {
        return cmz ? trid::launch_const_lines(rz, cmz, st) : trid::launch_lines(rz, pz, st);
    };
    trid::KernelTimer notimer;  // graph capture records no events
    trid::KernelTimer &tm = (timed && st == h->stream) ? h->ext.timer : notimer;
    for (int it = 0; it < nsteps; ++it) {
        hipError_t e = tm.time("adi_stencil_x", st, run_x);
        if (e != hipSuccess) return hip_fail(h, e, "stencil + x-solve launch");
        e = tm.time(ndim == 3 ? "adi_y" : "adi_y_update", st, run_y);
        if (e != hipSuccess) return hip_fail(h, e, "y-solve launch");
        if (ndim == 3) {
            e = tm.time("adi_z_update", st, run_z);
            if (e != hipSuccess) return hip_fail(h, e, "z-solve launch");
        }
    }
    return TRID_OK;
}

int trid_adi_step(trid_handle_t h, trid_dtype_t dt, void *u, const void *s, double s0, int ndim,
                  const int64_t *dims, int64_t batch, int nsteps, unsigned flags) {
    if (!h) return TRID_ERR_ARG;
    if (!dtype_ok(dt)) return fail(h, TRID_ERR_ARG, "bad dtype");
    if (!u) return fail(h, TRID_ERR_ARG, "u is NULL");
    if (ndim != 2 && ndim != 3) return fail(h, TRID_ERR_ARG, "ADI needs ndim 2 or 3");
    if (nsteps < 0) return fail(h, TRID_ERR_ARG, "nsteps must be >= 0");
    if (flags & ~(TRID_ADI_GRAPH | TRID_ADI_STREAM)) return fail(h, TRID_ERR_ARG, "unknown flags");
    i64 inner, n, outer;
    for (int ax = 0; ax < ndim; ++ax) {
        int rc = check_mesh(h, ndim, dims, ax, batch, &inner, &n, &outer);
        if (rc) return rc;
    }
    if (nsteps == 0) return TRID_OK;
    h->used = true;
    const bool f64 = dt == TRID_F64;
    const i64 nx = dims[0], ny = dims[1], nz = ndim == 3 ? dims[2] : 1;
    if (ndim == 2 && !(flags & TRID_ADI_STREAM)) {
        trid::ResidentReq rr;
        rr.f64 = f64;
        rr.u = u;
        rr.s = s;
        rr.s0 = s0;
        rr.nx = nx;
        rr.ny = ny;
        rr.batch = batch;
        rr.nsteps = nsteps;
        if (trid::resident_fits(rr)) {
            hipError_t e = h->ext.timer.time("adi2d_resident", h->stream,
                                             [&] { return trid::launch_resident(rr, h->stream); });
            if (e != hipSuccess) return hip_fail(h, e, "resident ADI launch");
            h->err.clear();
            return TRID_OK;
        }
    }
    const size_t bytes = (size_t)(nx * ny * nz * batch) * (f64 ? 8 : 4);
    void *dws = nullptr;
    int rc = trid::handle_workspace(h, bytes, &dws);
    if (rc) return rc;
    if (!(flags & TRID_ADI_GRAPH)) {
        rc = adi_enqueue(h, f64, u, s, s0, ndim, nx, ny, nz, batch, nsteps, dws, h->stream);
        if (rc == TRID_OK) h->err.clear();
        return rc;
    }
    GraphKey key{u, s, s ? 0.0 : s0, (int)dt, ndim, nx, ny, nz, batch, nsteps, h->ext.force_M, h->ext.force_L,
                 h->stream};
    hipGraphExec_t *it = h->graphs.find(key);
    if (!it) {
        hipError_t e;
        if (!h->capture_stream) {
            e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                h->capture_stream = nullptr;
                return hip_fail(h, e, "hipStreamCreate");
            }
        }
        e = hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamBeginCapture");
        rc = adi_enqueue(h, f64, u, s, s0, ndim, nx, ny, nz, batch, nsteps, dws, h->capture_stream);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(h->capture_stream, &graph);
        if (rc) {
            if (graph) hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
        it = h->graphs.insert(key, exec, drop_adi_graph);
    }
    hipError_t e = hipGraphLaunch(*it, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
    h->err.clear();
    return TRID_OK;
}

}  // extern "C"

// ------------------------------------------------------ no-allocation step --
//
// The mesh-sized d workspace of the per-step ADI kernels lives, for
// trid_adi_step_noalloc, in this statically sized device array: each GPU the
// library runs on holds its own copy from module load until the process ends.
// In host code `scratch` names a host-side stand-in, not a device address, so
// the address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that looked-up address is ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[TRID_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the first
// call on that device).
int noalloc_scratch(trid_handle_t h, void **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(h, e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(h, TRID_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(h, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return TRID_OK;
}

}  // namespace

extern "C" int trid_adi_step_noalloc(trid_handle_t h, trid_dtype_t dt, void *u, const void *s, double s0, int ndim,
                                     const int64_t *dims, int64_t batch, int nsteps, unsigned flags) {
    if (!h) return TRID_ERR_ARG;
    if (!dtype_ok(dt)) return fail(h, TRID_ERR_ARG, "bad dtype");
    if (!u) return fail(h, TRID_ERR_ARG, "u is NULL");
    if (ndim != 2 && ndim != 3) return fail(h, TRID_ERR_ARG, "ADI needs ndim 2 or 3");
    if (nsteps < 0) return fail(h, TRID_ERR_ARG, "nsteps must be >= 0");
    if (flags & ~(unsigned)TRID_ADI_STREAM)
        return fail(h, TRID_ERR_ARG, "flags: only TRID_ADI_STREAM (a captured graph would allocate)");
    i64 inner, n, outer;
    for (int ax = 0; ax < ndim; ++ax) {
        int rc = check_mesh(h, ndim, dims, ax, batch, &inner, &n, &outer);
        if (rc) return rc;
    }
    if (nsteps == 0) return TRID_OK;
    const bool f64 = dt == TRID_F64;
    const i64 nx = dims[0], ny = dims[1], nz = ndim == 3 ? dims[2] : 1;
    if (ndim == 2 && !(flags & TRID_ADI_STREAM)) {  // the LDS-resident loop uses no scratch
        trid::ResidentReq rr;
        rr.f64 = f64;
        rr.u = u;
        rr.s = s;
        rr.s0 = s0;
        rr.nx = nx;
        rr.ny = ny;
        rr.batch = batch;
        rr.nsteps = nsteps;
        if (trid::resident_fits(rr)) {
            h->used = true;
            hipError_t e = trid::launch_resident(rr, h->stream);
            if (e != hipSuccess) return hip_fail(h, e, "resident ADI launch");
            h->err.clear();
            return TRID_OK;
        }
    }
    const size_t bytes = (size_t)(nx * ny * nz * batch) * (f64 ? 8 : 4);
    if (bytes > (size_t)TRID_NOALLOC_SCRATCH_BYTES)
        return fail(h, TRID_ERR_UNSUPPORTED, "mesh larger than the no-allocation scratch (TRID_NOALLOC_SCRATCH_BYTES)");
    void *dws = nullptr;
    int rc = noalloc_scratch(h, &dws);
    if (rc) return rc;
    h->used = true;
    rc = adi_enqueue(h, f64, u, s, s0, ndim, nx, ny, nz, batch, nsteps, dws, h->stream, /*timed=*/false);
    if (rc == TRID_OK) h->err.clear();
    return rc;
}

