// hv.hpp -- host entry of the predictor stencils of the Hundsdorfer-Verwer
// step (k_hv.hip), the synthetic stand-in for Alg. 4's call structure.
#pragma once

#include "dispatch.hpp"

namespace trid {

struct HvReq {
    bool f64 = true;
    void *u = nullptr;                                // mesh field, in place
    void *r = nullptr, *z = nullptr;                  // two mesh-sized work arrays
    const void *a = nullptr, *b = nullptr, *c = nullptr;
    void *sa = nullptr, *sb = nullptr;                // solve coefficients theta dt a, theta dt b
    i64 nx = 1, ny = 1, batch = 1;
    double dt = 0, theta = 0;
};

// which: 0..3 run predictor 0..3 of a step; 4 fills sa and sb.
hipError_t launch_hv_pred(const HvReq &q, int which, hipStream_t s);

}  // namespace trid
