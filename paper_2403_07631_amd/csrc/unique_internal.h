// Internal declarations of the sparse unique-cell storage (Sec. III-C).
#pragma once

#include "pct_internal.h"

namespace pct {

size_t unique_ws_bytes(int nx, int ny, int N);
pct_status launch_unique(const float* ground, const float* ceil, const float* cost, int nx, int ny, int N, float cB,
                         const uint8_t* h_keep, long long capacity, int* cell, float* g_out, float* c_out,
                         float* t_out, long long* h_slice_off, long long* h_count, void* ws, hipStream_t s);

}  // namespace pct
