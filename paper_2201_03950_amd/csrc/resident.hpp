// resident.hpp -- host entry of the LDS-resident 2D ADI time loop (k_resident.hip).
#pragma once

#include "dispatch.hpp"

namespace trid {

// `nsteps` 2D ADI steps of `batch` meshes of nx * ny points, each mesh held in
// one workgroup's LDS for the whole time loop (u read from HBM once, written
// once).  s per point (s != NULL) or the constant s0.  With hv set, the steps
// are instead Hundsdorfer-Verwer steps of u_t = a u_xx + b u_yy + c u_xy
// (per-point a, b, c, step dt, parameter theta); s and s0 are then unused.
struct ResidentReq {
    bool f64 = true;
    void *u = nullptr;
    const void *s = nullptr;
    double s0 = 0;
    i64 nx = 1, ny = 1, batch = 1;
    int nsteps = 1;
    bool hv = false;
    const void *a = nullptr, *b = nullptr, *c = nullptr;
    double dt = 0, theta = 0;
};

// Whether the request fits the resident kernel (lines of at most 128 points,
// the mesh's arrays within one workgroup's LDS); no HIP calls.
bool resident_fits(const ResidentReq &r);
// The LDS layout the resident kernels use for r (tile size forced unless 0):
// {tile rows, tiles per x line, tiles per y line, row pitch, skew per block of
// tile rows, pad per tile, elements per array, coefficient arrays staged (HV),
// threads per workgroup, LDS bytes}.  Host only.
bool resident_layout(const ResidentReq &r, int force_M, int64_t out[10]);
hipError_t launch_resident(const ResidentReq &r, hipStream_t s);

}  // namespace trid
