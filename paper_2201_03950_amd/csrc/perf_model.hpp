// perf_model.hpp -- predictive performance model of the line-solve launches
// and of the uneven-batch schedules: bytes over bandwidth, launch cost, and the
// latency share of the per-tile sweeps (the GPU counterpart of the paper's
// analytic FPGA latency model of Sections III and IV: data movement +
// pipeline latency per call).
#pragma once

#include <string>
#include <vector>

#include "dispatch.hpp"
#include "varlen.hpp"

namespace trid {

// Model constants of the line-solve launches.  t0: fixed cost of a launch;
// bw: streaming bandwidth; a strided kernel whose lanes read row segments of
// `seg` contiguous bytes streams at bw * seg / (seg + seg_half), a staged
// (contiguous-line) kernel at bw * staged_eff, a strided kernel on contiguous
// lines (one line per tile column) at bw * xs_eff; the coefficient-array form
// (five streams) at arr_eff of that.  One workgroup's critical path is lat +
// M rows at row_ns (FP64: times f64_factor) + the reduced-solve levels at
// lvl_ns each, plus lvl_wave_ns per level for each 256 threads of the
// workgroup when the levels go through LDS; the issue bound is the
// grid's wavefronts over the 1024 SIMD slots of the chip times M rows at
// issue_row_ns plus the levels at issue_lvl_ns.
struct LinesParams {
    double t0_us, bw_gbs, seg_half, staged_eff, xs_eff, arr_eff;
    double lat_us, row_ns, f64_factor, lvl_ns, lvl_wave_ns, issue_row_ns, issue_lvl_ns;
};
// Model constants of the uneven-batch persistent launch: a work item costs lat
// + its bytes at cu_gbs (one workgroup's stream) + M rows at row_ns (FP64 and
// the refinement: times f64_factor) + its reduced solve (PCR: lvl_ns per level
// of its longest system; Thomas: thomas_ns per reduced row); the launch takes
// t0 + the larger of (all bytes at bw) and (the items' costs over the
// workgroups, at least the longest item).
struct VarlenParams {
    double t0_us, bw_gbs, lat_us, cu_gbs, row_ns, f64_factor, lvl_ns, thomas_ns;
};
// The same cost form for the wavefront-level plans (a work item is a
// workgroup's wavefront slots, solved without block barriers), with its own
// constants: the tile sweep's M rows cost row_ns each (times f64_factor for
// FP64, ref_factor for the refinement), the in-wavefront reduced solve six
// lane-move levels of lvl_ns / 4 and a long system's exchange one lvl_ns (both
// twice for the refinement).
struct VarlenWaveParams {
    double t0_us, bw_gbs, lat_us, cu_gbs, row_ns, f64_factor, lvl_ns, ref_factor;
};
// Model constants of the ADI-step kernels and of the resident time loops, on top
// of LinesParams (t0, bw): the stencil + x kernels and the constant-row y/z
// kernels each stream at bw * eff with a per-round latency blk_us (rounds =
// the grid's workgroups over what the CUs hold at once); a resident loop costs,
// per round of meshes, one mesh's points per thread (units) times io_ns for
// its load and store plus, per step, res_ns (FP64: times res_f64; the
// Hundsdorfer-Verwer step: hv_ns); the HV predictor stencils stream at
// bw * pred_eff.
struct AdiParams {
    double sx_eff, sx_blk_us, cs_eff, cs_blk_us, res_io_ns, res_ns, res_f64, hv_ns, pred_eff;
};
const LinesParams &lines_params();
const VarlenParams &varlen_params();
const VarlenWaveParams &varlen_wave_params();
const AdiParams &adi_params();

struct ModelTerms {
    double us = 0;       // predicted kernel duration
    double t_bytes = 0;  // bandwidth term (us)
    double t_lat = 0;    // latency term (us)
    double bytes = 0;    // bytes the launch must move
    double rounds = 0;   // workgroup rounds (lines) or items per block (uneven batch)
    int per_cu = 0;      // workgroups resident per CU (estimate)
};

// One launch of the general line-solve kernels (k_staged / k_strided) for
// request r with plan pl.  Host only.
ModelTerms model_lines(const LineReq &r, const LinePlan &pl);

// One uneven-batch schedule: the systems `ids` of the batch with variant v,
// `blocks` persistent workgroups (varlen_blocks).  prec as VarlenSchedule.
ModelTerms model_varlen(const int64_t *offsets_host, std::vector<int> ids, int prec, const VarlenVariant &v,
                        int blocks);

// One kernel of a modelled call: its name (as the library's kernel timer names
// it), the call's predicted time in it (all launches), launches, bytes and
// workgroup rounds per launch, and the class whose constants it uses.
struct KernelPred {
    std::string name, cls;
    double us = 0;
    int launches = 0;
    double bytes = 0, rounds = 0;
    double units = 0;  // resident loops: one mesh's points per thread and step
};

// `nsteps` ADI steps of request r (Alg. 3; the per-step kernels, or the
// resident 2D loop where it applies and stream is false).  Host only; r's
// pointers only decide alignment-dependent plans.
bool model_adi(const AdiReq &r, int nsteps, bool stream, std::vector<KernelPred> *ks, std::string *err);
// `nsteps` Hundsdorfer-Verwer steps of batch meshes of nx * ny points (the
// SLV stand-in): resident loop, or fill + four predictors + four s-form solves
// per step.
bool model_hv(bool f64, i64 nx, i64 ny, i64 batch, int nsteps, bool stream, std::vector<KernelPred> *ks,
              std::string *err);

}  // namespace trid
