// Internal declarations of the trajectory optimisation through the tomogram
// (Sec. III-E): the launcher behind pct_traj_eval and pct_traj_optimize.
#pragma once

#include "pct_internal.h"

namespace pct {

// Weights, limits and the maps of one robot, widened to FP64 on the host.
struct TrajArgs {
    const float* cost;    // c^T [N][ny][nx]
    const float* ground;  // e^G
    const float* ceil;    // e^C
    int nx, ny, N;
    double x0, y0, res;
    double w_z, w_c, w_v, w_a, w_h, w_T;
    double c_safe, v_max2, a_max2, d_ref, d_min;
    int K;   // samples per piece (K + 1 times, ends included)
    int M;   // pieces per trajectory
};

// iters < 0: evaluate the objective, its gradient and (optionally) the
// coefficients once; iters >= 0: run that many optimiser iterations in place.
pct_status launch_traj(const TrajArgs& a, int n_traj, const double* bound, const int* slice, double* knots,
                       double* tau, double* phi, double* gknots, double* gtau, double* coef, int iters, double step,
                       int* iters_done, hipStream_t s);

}  // namespace pct
