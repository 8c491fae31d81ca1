// varlen.hpp -- host-side schedule of the uneven-batch persistent solver.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <tuple>
#include <vector>

#include "graph_cache.hpp"

namespace trid {

using i64 = int64_t;

// A compiled tile plan: M rows per tile, NT threads (tiles) per work item;
// thomas = 1: reduced systems solved by Thomas on one thread per system
// (the Thomas-Thomas hybrid), else by PCR across the system's tiles;
// wave = 1: the wavefront-level kernels (each wavefront stages and solves its
// 64 tiles on its own; NT = 64 x wavefronts per workgroup).
struct VarlenVariant {
    int M, NT;
    int thomas = 0;
    int wave = 0;
};

struct VarlenSchedule {
    int prec = 0;  // 0: FP64, 1: FP32, 2: FP32 + FP64 refinement
    int M = 16, NT = 512, thomas = 0, wave = 0;
    i64 nsys = 0;
    int nitems = 0, nblocks = 0;
    void *dev = nullptr;  // single device allocation holding the arrays below
    i64 *off = nullptr;
    int *order = nullptr, *tstart = nullptr, *item_begin = nullptr, *item_pmax = nullptr;
    int *counter = nullptr;
    int *wdesc = nullptr;  // wavefront variants: {first, count, w0 | flag << 8, k} per wavefront slot
    int *rec = nullptr;    // wavefront variants: {first row lo, hi, rows, first lane} per system
    float tuned_us = 0.f;  // measured time when chosen by the autotuner
    // split schedule: the systems too long for a small-block variant run in
    // this launch, the rest in `next` (launched right after, same arrays)
    VarlenSchedule *next = nullptr;
    // systems longer than kVarlenMaxTiled rows: solved one after another by the
    // chunked solve (k_long.hip) after the persistent launch, with a workspace
    // owned by the schedule (stable for captured graphs)
    std::vector<i64> long_off, long_len;
    void *long_ws = nullptr;
    // captured launches keyed by (a, b, c, d, x, stream), least recently used
    // evicted beyond the capacity
    using GraphKey = std::tuple<const void *, const void *, const void *, const void *, void *, hipStream_t>;
    LruMap<GraphKey, hipGraphExec_t> graphs{8};
};

// Longest system the persistent launch takes (one workgroup's tiles); longer
// ones go to the chunked solve.
constexpr i64 kVarlenMaxTiled = 8192;

const std::vector<VarlenVariant> &varlen_variants(int prec);
bool varlen_variant_fits(const VarlenVariant &v, i64 maxlen);
// Work items of a schedule: sorts *ids longest first and packs the systems (next
// fit) into items of at most v.NT tiles; tstart[k] is the first tile of the
// k-th system in its item, item_begin the first system of each item (plus the
// end), item_pmax each item's most tiles of one system.  Host only.
void varlen_pack(const int64_t *offsets_host, std::vector<int> *ids, const VarlenVariant &v, std::vector<int> *tstart,
                 std::vector<int> *item_begin, std::vector<int> *item_pmax);
// Persistent blocks a launch of variant v runs with (occupancy x CUs; HIP query).
int varlen_blocks(int prec, const VarlenVariant &v);
// Schedule for all systems with variant v; with `small` given, the systems of at
// most small.M * small.NT rows go to a second launch with that variant.
hipError_t varlen_build(const int64_t *offsets_host, i64 nsys, int prec, const VarlenVariant &v, VarlenSchedule *sc,
                        const VarlenVariant *small = nullptr);
hipError_t varlen_launch(const VarlenSchedule &sc, const void *a, const void *b, const void *c, const void *d,
                         void *x, hipStream_t s);
void varlen_free(VarlenSchedule *sc);

// Wavefront variants (k_varlen_wave.hip): wavefronts per workgroup of tile
// size M, the packing into wavefront slots (long systems on consecutive
// wavefronts of one item, short systems several per wavefront; per slot
// {first, count, w0, k}, flattened), persistent workgroups, build, launch.
int varlen_wave_NW(int prec, int M);
void varlen_wave_pack(const int64_t *offsets_host, std::vector<int> ids, int M, int NW, std::vector<int> *order,
                      std::vector<int> *tstart, std::vector<int> *wdesc);
int varlen_wave_blocks(int prec, int M);
hipError_t varlen_wave_build(const int64_t *offsets_host, std::vector<int> ids, int prec, const VarlenVariant &v,
                             VarlenSchedule *sc);
hipError_t varlen_wave_launch(const VarlenSchedule &sc, const void *a, const void *b, const void *c, const void *d,
                              void *x, hipStream_t s);

}  // namespace trid
