// Internal declarations of the path search through the slices (Sec. III-D):
// workspace size and the launchers behind pct_plan_distance / pct_plan_path.
#pragma once

#include "pct_internal.h"

namespace pct {

constexpr double kPlanDefaultBand = 16384.0;   // distance band per round of the path search

size_t plan_ws_bytes(int nx, int ny, int L);
pct_status launch_plan(const float* cost, const float* ground, int nx, int ny, const int* h_layers, int L, float cB,
                       int sx, int sy, int sl, double* dist, void* ws_base, int* h_rounds, long long* h_tiles,
                       hipStream_t s, double delta, long long goal = -1, double* h_settled = nullptr);
pct_status launch_plan_path(const double* dist, int nx, int ny, int L, int sx, int sy, int sl, int gx, int gy, int gl,
                            int* path, int max_len, void* ws_base, int* h_len, hipStream_t s);

}  // namespace pct
