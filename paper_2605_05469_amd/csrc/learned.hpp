// learned.hpp -- flexible PCG with the U-Net warm start / preconditioner (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/pic.h"
#include "solver_state.hpp"

namespace pic {

struct Learned;

// What the flexible solver borrows from the context.
struct LearnedEnv {
    SweepGeo geo;
    int64_t n3;
    double inv_h2, minv, h, rtol;
    int64_t max_iter;
    int check_every, window;
    DevState* st;
    DevState* st_host;
    double* partials;
    double* r;
    double* p0;
    double* p1;
};

int learned_create(Learned** out, int n, int64_t n3);
void learned_destroy(Learned* l);
size_t learned_bytes(int n);
const char* learned_last_error();
int learned_solve(Learned* l, const LearnedEnv* env, const double* b, double* x,
                  pic_solve_info* info, hipStream_t s);

}  // namespace pic
