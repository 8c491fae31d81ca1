// refine.hpp -- host-side description of the FP32 + FP64-refinement solves.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace trid {

using i64 = int64_t;

struct RefPtrs {
    const float *a, *b, *c;  // coefficient arrays (arrays form)
    const float *s;          // diffusion numbers (s form)
};

struct RefineReq {
    bool smode = false;  // rows from s instead of a, b, c
    bool d_f64 = true;   // dtype of d
    RefPtrs src{};
    const void *d = nullptr;
    double *x = nullptr;
    i64 inner = 1, n = 1, outer = 1;
    int force_M = 0, force_L = 0;
};

struct RefPlan {
    int M = 16, L = 1, P = 1, ls = 0;
    bool staged = false;
    bool lean = false;  // s-form lines, register-lean tiles (k_refine_lean; staged: k_refine_staged_lean)
    size_t shmem = 0;
    i64 nblocks = 0;
};

bool plan_refine(const RefineReq &r, RefPlan *pl, std::string *err);
hipError_t launch_refine(const RefineReq &r, const RefPlan &pl, hipStream_t s);

}  // namespace trid
