// ext.hpp -- per-handle state shared by the entry points beyond the plain solves
// (tile-plan overrides and the tuned-plan cache), and the accessors that let
// those entry points live in their own translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "dispatch.hpp"
#include "graph_cache.hpp"

typedef struct trid_handle_s *trid_handle_t;

namespace trid {

struct VarlenSchedule;  // defined with the uneven-batch solver

// Optional per-kernel timing.  When on, time() arms a pair of events that the
// next kernel launch on this thread stamps from its own dispatch (start and
// end of the kernel, see launch()); time_recorded() brackets work that is not
// a direct kernel launch (a graph launch) with two events recorded on the
// stream.  flush() waits for them and accumulates (count, milliseconds) per
// name.  Launches under graph capture are not timed.  A non-empty `only`
// restricts timing to launches of that name (the others run without events);
// `every` > 1 times only every `every`-th launch of each timed name, counting
// from the first after the selection.
struct KernelTimer {
    bool on = false;
    std::string only;
    long every = 1;
    std::map<std::string, long> seen;
    bool wants(const char *name) {
        if (!on) return false;
        if (!only.empty() && only != name) return false;
        return every <= 1 || seen[name]++ % every == 0;
    }
    struct Pending {
        std::string name;
        hipEvent_t e0, e1;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<long, double>> acc;

    hipEvent_t take() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // f() enqueues one kernel through launch() on st.
    template <class F>
    hipError_t time(const char *name, hipStream_t st, F &&f) {
        (void)st;
        if (!wants(name)) return f();
        hipEvent_t e0 = take(), e1 = take();
        if (!e0 || !e1) return f();
        LaunchEvents &ev = launch_events();
        ev.start = e0;
        ev.stop = e1;
        ev.used = false;
        hipError_t e = f();
        const bool used = ev.used;
        ev = LaunchEvents{};
        if (used) {
            pending.push_back({name, e0, e1});
        } else {
            pool.push_back(e0);
            pool.push_back(e1);
        }
        return e;
    }
    // f() enqueues work on st that is not a direct kernel launch.
    template <class F>
    hipError_t time_recorded(const char *name, hipStream_t st, F &&f) {
        if (!wants(name)) return f();
        hipEvent_t e0 = take(), e1 = take();
        if (!e0 || !e1) return f();
        hipEventRecord(e0, st);
        hipError_t e = f();
        hipEventRecord(e1, st);
        pending.push_back({name, e0, e1});
        return e;
    }
    hipError_t flush() {
        for (auto &p : pending) {
            hipError_t e = hipEventSynchronize(p.e1);
            if (e != hipSuccess) return e;
            float ms = 0.f;
            hipEventElapsedTime(&ms, p.e0, p.e1);
            auto &a = acc[p.name];
            a.first += 1;
            a.second += ms;
            pool.push_back(p.e0);
            pool.push_back(p.e1);
        }
        pending.clear();
        return hipSuccess;
    }
    void release() {
        flush();
        for (auto e : pool) hipEventDestroy(e);
        pool.clear();
        acc.clear();
    }
};

// A tuned uneven-batch plan: tile rows, threads per work item, reduced solve
// (thomas), wavefront-level kernel (wave).
struct TunedPlan {
    int M = 0, NT = 0, thomas = 0, wave = 0;
};

// One plan the uneven-batch autotuner considered: the model's prediction and,
// when it was among those timed, the measured time (else < 0).
struct TuneRecord {
    int M = 0, NT = 0, thomas = 0, split = 0, wave = 0;
    int nlong = 0;  // systems longer than one workgroup holds (chunked solve, every plan)
    int blocks = 0, blocks_small = 0;  // persistent workgroups of the launch(es)
    double pred_us = 0, meas_us = -1;
};

struct ExtState {
    int force_M = 0;  // forced tile rows (0: automatic)
    int force_L = 0;  // forced lines per block (0: automatic)
    // tuned plans: key -> plan
    std::map<std::string, TunedPlan> tuned;
    // uneven-batch schedules keyed by a hash of the offsets (least recently
    // used evicted beyond the capacity)
    LruMap<std::string, VarlenSchedule *> varlen{32};
    std::vector<TuneRecord> last_tune;  // the most recent autotuning run
    // scratch for adjoint / refinement entry points
    void *ws2 = nullptr;
    size_t ws2_bytes = 0;
    KernelTimer timer;
    hipStream_t capture_stream = nullptr;  // graph capture of the uneven-batch launch

    void apply_overrides(LineReq *r) const {
        if (force_M) r->force_M = force_M;
        if (force_L) r->force_L = force_L;
    }
    void apply_adi_overrides(AdiReq *r) const {
        if (force_M == 8 || force_M == 16) r->force_M = force_M;
        if (force_L) r->force_L = force_L;
    }
    bool has_device_state() const {
        return ws2 != nullptr || varlen.size() || !timer.pool.empty() || !timer.pending.empty() ||
               capture_stream != nullptr;
    }
    void release();
};

hipStream_t handle_stream(trid_handle_t h);
ExtState &handle_ext(trid_handle_t h);
int handle_fail(trid_handle_t h, int code, const std::string &msg);
int handle_hip_fail(trid_handle_t h, hipError_t e, const char *what);
// long_ok: contiguous lines up to TRID_MAX_LONG_LINE are accepted
int handle_check_mesh(trid_handle_t h, int ndim, const int64_t *dims, int axis, int64_t batch,
                      i64 *inner, i64 *n, i64 *outer, bool long_ok = false);
int handle_run_lines(trid_handle_t h, const LineReq &r);
int handle_workspace(trid_handle_t h, size_t bytes, void **ptr);
bool alloc_failure_forced();  // TRID_FAIL_ALLOC is set: workspace allocations fail
int handle_workspace2(trid_handle_t h, size_t bytes, void **ptr);
size_t handle_adi_graphs(trid_handle_t h);  // captured ADI runs held by the handle
size_t handle_adi_graph_cap();              // and their maximum number

}  // namespace trid
