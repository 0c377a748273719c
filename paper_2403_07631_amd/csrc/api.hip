// Host side of libpct: argument validation, parameter tables, workspace
// sizing and launch orchestration.  Nothing here allocates device memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "pct_internal.h"
#include "plan_internal.h"
#include "traj_internal.h"
#include "unique_internal.h"

namespace pct {

namespace {
thread_local char g_err[512] = "";
}

pct_status fail(pct_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = 0; }

namespace {

bool finite_f(float v) { return isfinite(v) != 0; }

pct_status check_grid(const pct_grid* g) {
    if (!g) return fail(PCT_ERR_ARG, "grid is null");
    if (!finite_f(g->x0) || !finite_f(g->y0)) return fail(PCT_ERR_ARG, "grid origin must be finite");
    if (!(g->res > 0.0f) || !finite_f(g->res)) return fail(PCT_ERR_ARG, "grid res must be > 0");
    if (!(g->slice_dz > 0.0f) || !finite_f(g->slice_dz)) return fail(PCT_ERR_ARG, "slice_dz must be > 0");
    if (g->nx < 1 || g->ny < 1 || g->nx > PCT_MAX_GRID_SIDE || g->ny > PCT_MAX_GRID_SIDE)
        return fail(PCT_ERR_ARG, "grid size %d x %d outside [1, %d]", g->nx, g->ny, PCT_MAX_GRID_SIDE);
    return PCT_OK;
}

// Eq. (6) weight in FP64 from the float parameters; weights within 1e-6
// of 1 or 0 are taken as exactly 1 or 0 (lattice distances that equal d_inf
// or the outer edge in decimal land a few 1e-8 off after the parameters
// are stored as floats).
double kernel_weight(const pct_robot& r, float res, int a, int j) {
    const double rr = (double)res;
    const double dist = rr * sqrt((double)(a * a + j * j));
    double k = 1.0 - (dist - (double)r.d_inf) / ((double)r.d_sm - rr);
    k = std::max(0.0, std::min(k, 1.0));
    if (k >= 1.0 - 1e-6) k = 1.0;
    if (k <= 1e-6) k = 0.0;
    return k;
}

int kernel_radius(const pct_robot& r, float res) {
    int R = 0;
    for (int a = 0; a <= PCT_MAX_KERNEL_RADIUS + 1; ++a)
        for (int j = 0; j <= a; ++j)
            if (kernel_weight(r, res, a, j) > 0.0) R = a;
    return R;
}

pct_status check_robot(const pct_robot* r, float res) {
    if (!r) return fail(PCT_ERR_ARG, "robot is null");
    const float v[] = {r->d_min, r->d_ref, r->theta_b, r->theta_s, r->theta_p, r->c_barrier,
                       r->alpha_d, r->alpha_b, r->alpha_s, r->d_inf, r->d_sm};
    for (float x : v)
        if (!finite_f(x)) return fail(PCT_ERR_ARG, "robot parameters must be finite");
    if (!(r->c_barrier > 0.0f)) return fail(PCT_ERR_ARG, "c_barrier must be > 0");
    if (!(r->theta_b > 0.0f) || !(r->theta_s > 0.0f)) return fail(PCT_ERR_ARG, "theta_b and theta_s must be > 0");
    // the step threshold theta_b * 2r is compared in single precision
    if (!finite_f((float)((double)r->theta_b * 2.0 * (double)res)))
        return fail(PCT_ERR_ARG, "theta_b * 2 res overflows single precision");
    if (r->theta_p < 0.0f) return fail(PCT_ERR_ARG, "theta_p must be >= 0");
    if (r->alpha_d < 0.0f || r->alpha_b < 0.0f || r->alpha_s < 0.0f) return fail(PCT_ERR_ARG, "scaling factors must be >= 0");
    if (r->d_inf < 0.0f) return fail(PCT_ERR_ARG, "d_inf must be >= 0");
    if (!(r->d_sm > res)) return fail(PCT_ERR_ARG, "d_sm (%g) must exceed the grid resolution (%g)", r->d_sm, res);
    if (r->patch_radius < 1 || r->patch_radius > PCT_MAX_PATCH_RADIUS)
        return fail(PCT_ERR_ARG, "patch_radius must be in [1, %d]", PCT_MAX_PATCH_RADIUS);
    if (kernel_radius(*r, res) > PCT_MAX_KERNEL_RADIUS)
        return fail(PCT_ERR_CAPACITY, "inflation kernel radius exceeds %d cells", PCT_MAX_KERNEL_RADIUS);
    return PCT_OK;
}

pct_status check_extent(const pct_extent* e) {
    if (!e) return fail(PCT_ERR_ARG, "extent is null");
    if (e->n_slices < 0 || e->n_slices > PCT_MAX_SLICES)
        return fail(PCT_ERR_CAPACITY, "n_slices %d outside [0, %d]", e->n_slices, PCT_MAX_SLICES);
    if (e->n_slices > 0 && (!finite_f(e->z_min) || !finite_f(e->z_max)))
        return fail(PCT_ERR_ARG, "extent heights must be finite");
    return PCT_OK;
}

// Number of planes for an extent (Sec. III-A): the least N with
// h_{N-1} > z_max; -1 if consecutive planes coincide, -2 if N > cap.
int plane_count(float zmin, float zmax, float ds, int cap) {
    float prev = -INFINITY;
    for (int k = 0; k < cap; ++k) {
        const float h = plane_height(zmin, ds, k);
        if (!(h > prev)) return -1;
        if (h > zmax) return k + 1;
        prev = h;
    }
    return -2;
}

}  // namespace

pct_status make_eval_params(const pct_robot& r, const pct_grid& g, int N, EvalParams* out) {
    EvalParams p{};
    p.nx = g.nx;
    p.ny = g.ny;
    p.N = N;
    p.plane = (long long)g.nx * g.ny;
    p.wx0 = 0;
    p.wy0 = 0;
    p.wx1 = g.nx;
    p.wy1 = g.ny;
    p.R = kernel_radius(r, g.res);
    if (p.R > PCT_MAX_KERNEL_RADIUS) return fail(PCT_ERR_CAPACITY, "inflation kernel radius exceeds %d", PCT_MAX_KERNEL_RADIUS);
    p.d_min = r.d_min;
    p.d_ref = r.d_ref;
    p.cB = r.c_barrier;
    p.alpha_d = r.alpha_d;
    const double two_r = 2.0 * (double)g.res;
    const double tb = (double)r.theta_b * two_r, ts = (double)r.theta_s * two_r;
    p.Tb = (float)tb;
    p.Ts2 = (float)(ts * ts);
    p.As = (float)((double)r.alpha_s / (ts * ts));
    p.Ab = (float)((double)r.alpha_b / (tb * tb));
    p.rp = r.patch_radius;
    const int np = (2 * r.patch_radius + 1) * (2 * r.patch_radius + 1) - 1;
    p.kp = (int)floor((double)r.theta_p * (double)np);
    for (int a = 0; a < kKmax; ++a)
        for (int j = 0; j < kKmax; ++j) p.K[a][j] = (float)kernel_weight(r, g.res, a, j);
    *out = p;
    return PCT_OK;
}

}  // namespace pct

namespace pct {

void digest_params(Digest& d, const EvalParams& p) {
    d.add(p.nx), d.add(p.ny), d.add(p.N), d.add(p.R), d.add(p.plane);
    d.add(p.d_min), d.add(p.d_ref), d.add(p.cB), d.add(p.alpha_d), d.add(p.Tb), d.add(p.Ts2), d.add(p.As), d.add(p.Ab);
    d.add(p.rp), d.add(p.kp), d.add(p.wx0), d.add(p.wy0), d.add(p.wx1), d.add(p.wy1);
    for (int a = 0; a < kKmax; ++a)
        for (int j = 0; j < kKmax; ++j) d.add(p.K[a][j]);
}

namespace {
std::mutex g_res_mu;
std::map<std::pair<const void*, int>, uint64_t> g_resident;
}  // namespace

pct_status resident_tables(const void* region, int kind, uint64_t digest, bool upload) {
    std::lock_guard<std::mutex> lk(g_res_mu);
    const auto key = std::make_pair(region, kind);
    if (upload) {
        g_resident[key] = digest;
        return PCT_OK;
    }
    auto it = g_resident.find(key);
    if (it == g_resident.end())
        return fail(PCT_ERR_ARG, "PCT_DESCRIPTORS_RESIDENT: no descriptor tables were uploaded to this workspace");
    if (it->second != digest)
        return fail(PCT_ERR_ARG, "PCT_DESCRIPTORS_RESIDENT: the workspace holds the tables of other items, robots or "
                                 "tile shapes (tuning changed them?): call once without the flag to upload them");
    return PCT_OK;
}

namespace {

pct_status eval_traversability(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                               const pct_extent* extent, const pct_robot* h_robots, int32_t n_robots, float* d_cost,
                               uint8_t* d_keep, void* d_ws, size_t ws_bytes, hipStream_t s) {
    const int N = extent->n_slices;
    const long long per_robot = (long long)N * grid->nx * grid->ny;
    for (int i = 0; i < n_robots; ++i) {
        EvalParams p;
        pct_status st = make_eval_params(h_robots[i], *grid, N, &p);
        if (st != PCT_OK) return st;
        float* cost = d_cost + per_robot * i;
        st = launch_eval_simplify(d_ground, d_ceil, p, cost, d_keep ? d_keep + (size_t)N * i : nullptr, d_ws, ws_bytes, s);
        if (st != PCT_OK) return st;
    }
    return PCT_OK;
}

pct_status check_eval_args(const float* d_ground, const float* d_ceil, const pct_grid* grid, const pct_extent* extent,
                           const pct_robot* h_robots, int32_t n_robots, const float* d_cost) {
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    if (n_robots < 1 || !h_robots) return fail(PCT_ERR_ARG, "at least one robot is required");
    for (int i = 0; i < n_robots; ++i) {
        st = check_robot(&h_robots[i], grid->res);
        if (st != PCT_OK) return st;
    }
    if (extent->n_slices > 0 && (!d_ground || !d_ceil || !d_cost)) return fail(PCT_ERR_ARG, "device pointers are null");
    return PCT_OK;
}

// The static scratch of pct_eval_traversability_static.  In host code
// `scratch` names a host-side stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device, kept per device.
static __device__ __align__(256) unsigned char scratch[PCT_STATIC_WORKSPACE_BYTES];
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;   // indexed by device ordinal

pct_status static_scratch(hipStream_t s, void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(PCT_ERR_DEVICE, "hipGetDevice failed");
    hipDevice_t sdev = -1;
    hipError_t e = hipStreamGetDevice(s, &sdev);
    if (e != hipSuccess) return fail(PCT_ERR_DEVICE, "hipStreamGetDevice failed: %s", hipGetErrorString(e));
    if ((int)sdev != dev)
        return fail(PCT_ERR_ARG, "the stream belongs to device %d but device %d is current", (int)sdev, dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
    if (!g_scratch_addr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PCT_ERR_DEVICE, "hipGetSymbolAddress of the static scratch failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_addr[dev] = ptr;
    }
    *out = g_scratch_addr[dev];
    return PCT_OK;
}

}  // namespace
}  // namespace pct

namespace pct {
namespace {

// Mean time of `reps` calls of fn (after one untimed call) on stream s.
template <class F>
pct_status time_calls(F fn, hipStream_t s, int reps, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(PCT_ERR_DEVICE, "hipEventCreate failed");
    }
    pct_status st = fn(0);
    if (st == PCT_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(PCT_ERR_DEVICE, "hipEventRecord failed");
    for (int r = 0; r < reps && st == PCT_OK; ++r) st = fn(PCT_DESCRIPTORS_RESIDENT);
    if (st == PCT_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(ms, e0, e1) != hipSuccess))
        st = fail(PCT_ERR_DEVICE, "timing the candidates failed");
    if (st == PCT_OK) *ms /= (float)reps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

// Device buffers of one size class's trial runs, released on scope exit.
struct TrialBuffers {
    void* p[4] = {nullptr, nullptr, nullptr, nullptr};
    ~TrialBuffers() {
        for (void* q : p)
            if (q) (void)hipFree(q);
    }
};

pct_status current_arch(char* out, size_t n) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(PCT_ERR_DEVICE, "hipGetDeviceProperties failed");
    snprintf(out, n, "%s", prop.gcnArchName);
    for (char* c = out; *c; ++c)
        if (*c == ' ') *c = '_';
    return PCT_OK;
}

}  // namespace
}  // namespace pct

using namespace pct;

extern "C" {

int32_t pct_abi_version(void) { return PCT_ABI_VERSION; }

const char* pct_last_error(void) { return g_err; }

pct_status pct_validate_grid(const pct_grid* grid) {
    clear_error();
    return check_grid(grid);
}

pct_status pct_validate_robot(const pct_robot* robot, float res) {
    clear_error();
    if (!(res > 0.0f)) return fail(PCT_ERR_ARG, "res must be > 0");
    return check_robot(robot, res);
}

pct_status pct_kernel_radius(const pct_robot* robot, float res, int32_t* radius_out) {
    clear_error();
    if (!radius_out) return fail(PCT_ERR_ARG, "radius_out is null");
    pct_status st = pct_validate_robot(robot, res);
    if (st != PCT_OK) return st;
    *radius_out = kernel_radius(*robot, res);
    return PCT_OK;
}

pct_status pct_robot_from_physical(float min_interval, float nominal_height, float max_slope_deg, float max_step,
                                   float inflation_radius, float safe_margin, float res, pct_robot* out) {
    clear_error();
    if (!out) return fail(PCT_ERR_ARG, "out is null");
    if (!(res > 0.0f) || !(min_interval > 0.0f) || !(nominal_height > 0.0f) || !(max_step > 0.0f) ||
        !(inflation_radius >= 0.0f) || !(safe_margin > 0.0f))
        return fail(PCT_ERR_ARG, "sizes must be positive");
    if (!(max_slope_deg > 0.0f && max_slope_deg < 90.0f)) return fail(PCT_ERR_ARG, "max slope must be in (0, 90) degrees");
    pct_robot r{};
    r.d_min = min_interval;
    r.d_ref = nominal_height;
    r.theta_s = (float)tan((double)max_slope_deg * M_PI / 180.0);
    r.theta_b = (float)((double)max_step / (2.0 * (double)res));
    r.theta_p = 0.20f;
    r.c_barrier = 50.0f;
    r.alpha_d = 20.0f;
    r.alpha_b = 20.0f;
    r.alpha_s = 15.0f;
    r.d_inf = inflation_radius;
    r.d_sm = safe_margin;
    r.patch_radius = 1;
    *out = r;
    return PCT_OK;
}

pct_status pct_plane_heights(const pct_extent* extent, float slice_dz, float* h_out, int32_t cap) {
    clear_error();
    pct_status st = check_extent(extent);
    if (st != PCT_OK) return st;
    if (!(slice_dz > 0.0f)) return fail(PCT_ERR_ARG, "slice_dz must be > 0");
    if (extent->n_slices > cap) return fail(PCT_ERR_CAPACITY, "h_out holds %d planes, %d needed", cap, extent->n_slices);
    if (extent->n_slices > 0 && !h_out) return fail(PCT_ERR_ARG, "h_out is null");
    for (int k = 0; k < extent->n_slices; ++k) h_out[k] = plane_height(extent->z_min, slice_dz, k);
    return PCT_OK;
}

size_t pct_extent_workspace_bytes(int64_t n) { return extent_ws_bytes(n); }

pct_status pct_tomogram_extent(const float* d_xyz, int64_t n, const pct_grid* grid, pct_extent* h_out, void* d_ws,
                               size_t ws_bytes, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    if (!h_out) return fail(PCT_ERR_ARG, "h_out is null");
    if (n < 0 || n > (int64_t)INT32_MAX) return fail(PCT_ERR_ARG, "point count %lld outside [0, 2^31)", (long long)n);
    pct_extent e{};
    e.z_min = INFINITY;
    e.z_max = -INFINITY;
    if (n == 0) {
        *h_out = e;
        return PCT_OK;
    }
    if (!d_xyz) return fail(PCT_ERR_ARG, "d_xyz is null");
    if (!d_ws || ws_bytes < extent_ws_bytes(n))
        return fail(PCT_ERR_WORKSPACE, "extent workspace too small: %zu < %zu", ws_bytes, extent_ws_bytes(n));
    hipStream_t s = (hipStream_t)stream;
    GridDev g = make_grid_dev(*grid);
    ExtentDev* d_out = (ExtentDev*)((char*)d_ws + extent_ws_bytes(n) - align_up(sizeof(ExtentDev)));
    st = launch_extent(d_xyz, n, g, d_ws, d_out, s);
    if (st != PCT_OK) return st;
    ExtentDev hx{};
    PCT_HIP(hipMemcpyAsync(&hx, d_out, sizeof hx, hipMemcpyDeviceToHost, s));
    PCT_HIP(hipStreamSynchronize(s));
    e.n_used = (int64_t)hx.used;
    e.n_dropped = n - e.n_used;
    if (e.n_used > 0) {
        e.z_min = hx.zmin;
        e.z_max = hx.zmax;
        int N = plane_count(hx.zmin, hx.zmax, grid->slice_dz, PCT_MAX_SLICES);
        if (N == -1) return fail(PCT_ERR_ARG, "slice planes coincide in FP32 (slice_dz too small for z range)");
        if (N == -2) return fail(PCT_ERR_CAPACITY, "more than %d slices needed", PCT_MAX_SLICES);
        e.n_slices = N;
    }
    *h_out = e;
    return PCT_OK;
}

pct_status pct_tomogram_extent_device(const float* d_xyz, int64_t n, const pct_grid* grid, pct_extent* d_out,
                                      void* d_ws, size_t ws_bytes, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    if (!d_out) return fail(PCT_ERR_ARG, "d_out is null");
    if (n < 0 || n > (int64_t)INT32_MAX) return fail(PCT_ERR_ARG, "point count %lld outside [0, 2^31)", (long long)n);
    if (n > 0 && !d_xyz) return fail(PCT_ERR_ARG, "d_xyz is null");
    if (!d_ws || ws_bytes < extent_ws_bytes(n))
        return fail(PCT_ERR_WORKSPACE, "extent workspace too small: %zu < %zu", ws_bytes, extent_ws_bytes(n));
    return launch_extent_record(d_xyz, n, make_grid_dev(*grid), grid->slice_dz, d_ws, d_out, (hipStream_t)stream);
}

size_t pct_build_workspace_bytes(int64_t n, const pct_grid* grid, const pct_extent* extent) {
    (void)extent;
    if (!grid || check_grid(grid) != PCT_OK || n < 0) return 0;
    return build_ws_bytes(n, make_grid_dev(*grid), true);
}

pct_status pct_build_tomogram(const float* d_xyz, int64_t n, const pct_grid* grid, const pct_extent* extent,
                              float* d_ground, float* d_ceil, int32_t* d_arg_ground, int32_t* d_arg_ceil, void* d_ws,
                              size_t ws_bytes, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    if (n < 0 || n > (int64_t)INT32_MAX) return fail(PCT_ERR_ARG, "point count %lld outside [0, 2^31)", (long long)n);
    if ((d_arg_ground == nullptr) != (d_arg_ceil == nullptr))
        return fail(PCT_ERR_ARG, "d_arg_ground and d_arg_ceil must both be given or both be null");
    if (extent->n_slices == 0) return PCT_OK;
    if (!d_ground || !d_ceil) return fail(PCT_ERR_ARG, "output pointers are null");
    if (n > 0 && !d_xyz) return fail(PCT_ERR_ARG, "d_xyz is null");
    if (plane_count(extent->z_min, extent->z_max, grid->slice_dz, PCT_MAX_SLICES) != extent->n_slices)
        return fail(PCT_ERR_ARG, "extent does not match the plane rule for this slice_dz");
    GridDev g = make_grid_dev(*grid);
    const bool ids = d_arg_ground != nullptr;
    if (!d_ws || ws_bytes < build_ws_bytes(n, g, ids))
        return fail(PCT_ERR_WORKSPACE, "build workspace too small: %zu < %zu", ws_bytes, build_ws_bytes(n, g, ids));
    return launch_build(d_xyz, n, g, extent->z_min, grid->slice_dz, extent->n_slices, d_ground, d_ceil, d_arg_ground,
                        d_arg_ceil, d_ws, ws_bytes, (hipStream_t)stream);
}

size_t pct_eval_workspace_bytes(const pct_grid* grid, const pct_extent* extent, int32_t n_robots) {
    if (!grid || !extent || extent->n_slices < 0) return 0;
    return eval_ws_bytes(std::max(1, (int)extent->n_slices), n_robots);
}


pct_status pct_eval_traversability(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                   const pct_extent* extent, const pct_robot* h_robots, int32_t n_robots,
                                   float* d_cost, uint8_t* d_keep, void* d_ws, size_t ws_bytes, void* stream) {
    clear_error();
    pct_status st = check_eval_args(d_ground, d_ceil, grid, extent, h_robots, n_robots, d_cost);
    if (st != PCT_OK) return st;
    const int N = extent->n_slices;
    if (N == 0) return PCT_OK;
    if (d_keep && (!d_ws || ws_bytes < eval_ws_bytes(N, n_robots)))
        return fail(PCT_ERR_WORKSPACE, "eval workspace too small: %zu < %zu", ws_bytes, eval_ws_bytes(N, n_robots));
    return eval_traversability(d_ground, d_ceil, grid, extent, h_robots, n_robots, d_cost, d_keep, d_ws, ws_bytes,
                               (hipStream_t)stream);
}

pct_status pct_eval_traversability_static(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                          const pct_extent* extent, const pct_robot* h_robots, int32_t n_robots,
                                          float* d_cost, uint8_t* d_keep, void* stream) {
    clear_error();
    pct_status st = check_eval_args(d_ground, d_ceil, grid, extent, h_robots, n_robots, d_cost);
    if (st != PCT_OK) return st;
    const int N = extent->n_slices;
    if (N == 0) return PCT_OK;
    const size_t need = eval_ws_min_bytes(N);
    if (d_keep && need > PCT_STATIC_WORKSPACE_BYTES)
        return fail(PCT_ERR_CAPACITY, "the slice test needs %zu bytes of scratch, the static array holds %u", need,
                    (unsigned)PCT_STATIC_WORKSPACE_BYTES);
    hipStream_t s = (hipStream_t)stream;
    void* ws = nullptr;
    if (d_keep) {
        st = static_scratch(s, &ws);
        if (st != PCT_OK) return st;
    }
    return eval_traversability(d_ground, d_ceil, grid, extent, h_robots, n_robots, d_cost, d_keep, ws,
                               PCT_STATIC_WORKSPACE_BYTES, s);
}

pct_status pct_autotune_traversability(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                       const pct_extent* extent, const pct_robot* h_robot, float* d_cost,
                                       int32_t* h_best_rows, int32_t* h_best_waves, int32_t* h_rows,
                                       int32_t* h_waves, float* h_ms, int32_t n_max, int32_t* h_count, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    if (!h_robot) return fail(PCT_ERR_ARG, "h_robot is null");
    st = check_robot(h_robot, grid->res);
    if (st != PCT_OK) return st;
    if (!h_best_rows || !h_count) return fail(PCT_ERR_ARG, "h_best_rows and h_count are required");
    if (n_max < 0) return fail(PCT_ERR_ARG, "n_max must be >= 0");
    *h_best_rows = 0;
    if (h_best_waves) *h_best_waves = 0;
    *h_count = 0;
    const int N = extent->n_slices;
    if (N == 0) return PCT_OK;
    if (!d_ground || !d_ceil || !d_cost) return fail(PCT_ERR_ARG, "device pointers are null");
    EvalParams p;
    st = make_eval_params(*h_robot, *grid, N, &p);
    if (st != PCT_OK) return st;
    EvalShape best{0, 0}, cand[24];
    float ms[24];
    int count = 0;
    st = autotune_eval(d_ground, d_ceil, p, d_cost, (hipStream_t)stream, &best, cand, ms, 24, &count);
    if (st != PCT_OK) return st;
    for (int i = 0; i < count && i < n_max; ++i) {
        if (h_rows) h_rows[i] = cand[i].rows;
        if (h_waves) h_waves[i] = cand[i].nw;
        if (h_ms) h_ms[i] = ms[i];
    }
    *h_best_rows = best.rows;
    if (h_best_waves) *h_best_waves = best.nw;
    *h_count = count;
    return PCT_OK;
}

pct_status pct_autotune_reset(void) {
    clear_error();
    autotune_reset();
    return PCT_OK;
}

pct_status pct_autotune_set_traversability(const pct_grid* grid, const pct_extent* extent, const pct_robot* h_robot,
                                           int32_t rows, int32_t waves) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    if (!h_robot) return fail(PCT_ERR_ARG, "h_robot is null");
    st = check_robot(h_robot, grid->res);
    if (st != PCT_OK) return st;
    if (rows != 0 && (rows < 16 || rows > PCT_MAX_STRIP_ROWS))
        return fail(PCT_ERR_ARG, "rows %d is neither 0 nor in [16, %d]", rows, PCT_MAX_STRIP_ROWS);
    if (rows != 0 && waves != 1 && waves != 2 && waves != PCT_STRIP_WAVES)
        return fail(PCT_ERR_ARG, "waves %d is not 1, 2 or %d", waves, PCT_STRIP_WAVES);
    EvalParams p;
    st = make_eval_params(*h_robot, *grid, std::max(1, (int)extent->n_slices), &p);
    if (st != PCT_OK) return st;
    if (rows > 0 && p.rp == 1 && p.R <= 8 && !strip_shape_fits(p, EvalShape{rows, waves}))
        return fail(PCT_ERR_CAPACITY, "strips of %d rows give too many wavefronts for this map", rows);
    autotune_set(p, EvalShape{rows, waves});
    return PCT_OK;
}


namespace {

pct_status check_sampling(const pct_grid* grid, const pct_extent* extent, const pct_robot* robot, int32_t T, int32_t W,
                          const void* wp, const void* slice) {
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    st = check_robot(robot, grid->res);
    if (st != PCT_OK) return st;
    if (T < 0 || W < 0) return fail(PCT_ERR_ARG, "trajectory counts must be >= 0");
    if ((long long)T * W > (long long)INT32_MAX) return fail(PCT_ERR_CAPACITY, "too many waypoints");
    if ((long long)T * W > 0 && (!wp || !slice)) return fail(PCT_ERR_ARG, "waypoint pointers are null");
    return PCT_OK;
}

}  // namespace

pct_status pct_sample_cost_fwd(const float* d_cost, const float* d_ground, const pct_grid* grid,
                               const pct_extent* extent, const pct_robot* h_robot, float w_z, const float* d_wp,
                               const int32_t* d_wp_slice, int32_t n_traj, int32_t n_wp, float* d_f, void* stream) {
    clear_error();
    pct_status st = check_sampling(grid, extent, h_robot, n_traj, n_wp, d_wp, d_wp_slice);
    if (st != PCT_OK) return st;
    if (!isfinite(w_z)) return fail(PCT_ERR_ARG, "w_z must be finite");
    if (n_traj == 0) return PCT_OK;
    if (!d_f) return fail(PCT_ERR_ARG, "d_f is null");
    if (extent->n_slices > 0 && (!d_cost || !d_ground)) return fail(PCT_ERR_ARG, "grid pointers are null");
    return launch_sample_fwd(d_cost, d_ground, *grid, extent->n_slices, h_robot->d_ref, w_z, d_wp, d_wp_slice, n_traj,
                             n_wp, d_f, (hipStream_t)stream);
}

pct_status pct_sample_cost_bwd(const float* d_cost, const float* d_ground, const pct_grid* grid,
                               const pct_extent* extent, const pct_robot* h_robot, float w_z, const float* d_wp,
                               const int32_t* d_wp_slice, int32_t n_traj, int32_t n_wp, const float* d_gf,
                               float* d_gwp, float* d_gcost, float* d_gground, int32_t flags, void* stream) {
    clear_error();
    pct_status st = check_sampling(grid, extent, h_robot, n_traj, n_wp, d_wp, d_wp_slice);
    if (st != PCT_OK) return st;
    if (!isfinite(w_z)) return fail(PCT_ERR_ARG, "w_z must be finite");
    hipStream_t s = (hipStream_t)stream;
    const bool fixed = flags & PCT_FIXED_POINT;
    const long long cells = (long long)extent->n_slices * grid->nx * grid->ny * (fixed ? 2 : 1);
    if (!(flags & PCT_ACCUMULATE)) {
        st = launch_zero(d_gcost, cells, s);
        if (st != PCT_OK) return st;
        st = launch_zero(d_gground, cells, s);
        if (st != PCT_OK) return st;
    }
    if ((long long)n_traj * n_wp == 0) return PCT_OK;
    if (!d_gf || !d_gwp) return fail(PCT_ERR_ARG, "d_gf and d_gwp are required");
    if (extent->n_slices > 0 && (!d_cost || !d_ground)) return fail(PCT_ERR_ARG, "grid pointers are null");
    return launch_sample_bwd(d_cost, d_ground, nullptr, *grid, extent->n_slices, h_robot->d_ref, w_z, d_wp, d_wp_slice,
                             n_traj, n_wp, d_gf, d_gwp, d_gcost, d_gground, nullptr, nullptr, nullptr, nullptr, 0, fixed,
                             s);
}

pct_status pct_eval_traversability_bwd(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                       const pct_extent* extent, const pct_robot* h_robot, const float* d_gcost,
                                       float* d_gground, float* d_gceil, int32_t flags, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    st = check_robot(h_robot, grid->res);
    if (st != PCT_OK) return st;
    const int N = extent->n_slices;
    if (N == 0) return PCT_OK;
    if (!d_ground || !d_ceil || !d_gcost || !d_gground || !d_gceil) return fail(PCT_ERR_ARG, "device pointers are null");
    EvalParams p;
    st = make_eval_params(*h_robot, *grid, N, &p);
    if (st != PCT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const bool fixed = flags & PCT_FIXED_POINT;
    if (!(flags & PCT_ACCUMULATE)) {
        st = launch_zero(d_gground, p.plane * N * (fixed ? 2 : 1), s);
        if (st != PCT_OK) return st;
        st = launch_zero(d_gceil, p.plane * N * (fixed ? 2 : 1), s);
        if (st != PCT_OK) return st;
    }
    return launch_eval_bwd(d_ground, d_ceil, d_gcost, p, d_gground, d_gceil, fixed, s);
}

pct_status pct_route_grad_to_points(const float* d_gground, const float* d_gceil, const int32_t* d_arg_ground,
                                    const int32_t* d_arg_ceil, const pct_grid* grid, const pct_extent* extent,
                                    int64_t n_points, float* d_gz, int32_t flags, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    if (n_points < 0) return fail(PCT_ERR_ARG, "n_points must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const bool fixed = flags & PCT_FIXED_POINT;
    if (!(flags & PCT_ACCUMULATE)) {
        st = launch_zero(d_gz, n_points * (fixed ? 2 : 1), s);
        if (st != PCT_OK) return st;
    }
    if (extent->n_slices == 0 || n_points == 0) return PCT_OK;
    if (!d_gz || !d_gground || !d_arg_ground) return fail(PCT_ERR_ARG, "device pointers are null");
    if (d_gceil && !d_arg_ceil) return fail(PCT_ERR_ARG, "d_arg_ceil is required with d_gceil");
    return launch_route(d_gground, d_gceil, d_arg_ground, d_arg_ceil, (long long)grid->nx * grid->ny,
                        extent->n_slices, n_points, d_gz, fixed, s);
}

pct_status pct_trajectory_cost_bwd(const float* d_ground, const float* d_ceil, const float* d_cost,
                                   const int32_t* d_arg_ground, const int32_t* d_arg_ceil, const pct_grid* grid,
                                   const pct_extent* extent, const pct_robot* h_robot, float w_z, const float* d_wp,
                                   const int32_t* d_wp_slice, int32_t n_traj, int32_t n_wp, const float* d_gf,
                                   int64_t n_points, float* d_gwp, float* d_gz, int32_t flags, void* stream) {
    clear_error();
    pct_status st = check_sampling(grid, extent, h_robot, n_traj, n_wp, d_wp, d_wp_slice);
    if (st != PCT_OK) return st;
    if (!isfinite(w_z)) return fail(PCT_ERR_ARG, "w_z must be finite");
    if (n_points < 0) return fail(PCT_ERR_ARG, "n_points must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    const bool fixed = flags & PCT_FIXED_POINT;
    if (!(flags & PCT_ACCUMULATE)) {
        st = launch_zero(d_gz, n_points * (fixed ? 2 : 1), s);
        if (st != PCT_OK) return st;
    }
    const int N = extent->n_slices;
    if ((long long)n_traj * n_wp == 0) return PCT_OK;
    if (!d_gf || !d_gwp || !d_gz) return fail(PCT_ERR_ARG, "d_gf, d_gwp and d_gz are required");
    if (N > 0 && (!d_ground || !d_ceil || !d_cost || !d_arg_ground || !d_arg_ceil))
        return fail(PCT_ERR_ARG, "grid pointers are null");
    EvalParams p;
    st = make_eval_params(*h_robot, *grid, std::max(N, 1), &p);
    if (st != PCT_OK) return st;
    p.N = N;
    return launch_sample_bwd(d_cost, d_ground, d_ceil, *grid, N, h_robot->d_ref, w_z, d_wp, d_wp_slice, n_traj, n_wp,
                             d_gf, d_gwp, nullptr, nullptr, &p, d_arg_ground, d_arg_ceil, d_gz, n_points, fixed, s);
}

namespace {

// Host table of device item descriptors (grids tiled, bases assigned).
// `tuned`: construction tiles as tall as the size class's tuned height when
// that is taller than the default (so never more tiles than the default,
// which sizes the workspace).
pct_status make_items(const pct_item* h, int n_items, int64_t n_total, bool need_extent, std::vector<BuildItemDev>* out,
                      bool tuned = false) {
    if (n_items < 1 || !h) return fail(PCT_ERR_ARG, "a batch needs at least one item");
    out->resize(n_items);
    int tile_base = 0, chunk_base = 0, echunk_base = 0;
    for (int i = 0; i < n_items; ++i) {
        pct_status st = check_grid(&h[i].grid);
        char msg[512];
        if (st != PCT_OK) {
            snprintf(msg, sizeof msg, "%s", g_err);
            return fail(st, "item %d: %s", i, msg);
        }
        if (h[i].xyz_offset < 0 || h[i].n_points < 0 || h[i].xyz_offset + h[i].n_points > n_total)
            return fail(PCT_ERR_ARG, "item %d: points [%lld, +%lld) outside the %lld given", i,
                        (long long)h[i].xyz_offset, (long long)h[i].n_points, (long long)n_total);
        if (n_total > (int64_t)INT32_MAX) return fail(PCT_ERR_ARG, "point count outside [0, 2^31)");
        BuildItemDev& d = (*out)[i];
        d.g = make_grid_dev(h[i].grid);
        if (h[i].grid.nx <= 128) {
            // narrow submap: 512-cell tiles as wide as the map
            const int tw = h[i].grid.nx <= 64 ? 64 : 128;
            d.g = tile_shape(d.g, tw, 512 / tw);
        } else if (tuned) {
            const int th = batch_build_th(size_class(h[i].grid.nx), size_class(h[i].grid.ny));
            if (th > d.g.th) d.g = tile_shape(d.g, d.g.tw, th);
        }
        d.xyz_off = h[i].xyz_offset;
        d.n = h[i].n_points;
        if (need_extent) {
            st = check_extent(&h[i].extent);
            if (st != PCT_OK) {
                snprintf(msg, sizeof msg, "%s", g_err);
                return fail(st, "item %d: %s", i, msg);
            }
            if (h[i].extent.n_slices > 0 &&
                plane_count(h[i].extent.z_min, h[i].extent.z_max, h[i].grid.slice_dz, PCT_MAX_SLICES) != h[i].extent.n_slices)
                return fail(PCT_ERR_ARG, "item %d: extent does not match the plane rule", i);
            if (h[i].out_offset < 0) return fail(PCT_ERR_ARG, "item %d: negative out_offset", i);
        }
        d.zmin = h[i].extent.z_min;
        d.ds = h[i].grid.slice_dz;
        d.N = h[i].extent.n_slices;
        d.out_off = h[i].out_offset;
        d.tile_base = tile_base;
        d.chunk_base = chunk_base;
        d.echunk_base = echunk_base;
        tile_base += d.g.ntiles;
        chunk_base += (int)((d.n + kBatchChunk - 1) / kBatchChunk);
        echunk_base += (int)std::max<int64_t>(1, (d.n + kBatchEChunk - 1) / kBatchEChunk);
    }
    return PCT_OK;
}

}  // namespace

// Batch workspace layout (one size query serves all three batched calls):
//   [0, A)            the construction's item table (kept for PCT_DESCRIPTORS_RESIDENT)
//   [A, F)            transient: the extent's table and partials, or the
//                     construction's records and counters
//   [end - E, end)    the evaluation's job table and slice-test scratch
// A = item table bytes, F = max(A + extent bytes, construction bytes with
// ids), E = evaluation bytes for the call's robots.  The three regions never
// overlap, so resident tables survive the other calls.
struct BatchLayout {
    size_t A, F, E;
};

static BatchLayout batch_layout(const pct_item* h_items, const std::vector<BuildItemDev>& it, int n_items, int n_robots) {
    BatchLayout L{};
    L.A = align_up(sizeof(BuildItemDev) * (size_t)n_items);
    L.F = align_up(std::max(L.A + batch_extent_ws_bytes(it.data(), n_items), batch_build_ws_bytes(it.data(), n_items, true)));
    L.E = align_up(batch_eval_ws_bytes(h_items, n_items, std::max(1, n_robots)));
    return L;
}

size_t pct_batch_workspace_bytes(const pct_item* h_items, int32_t n_items, int32_t n_robots, int32_t with_ids) {
    (void)with_ids;   // sized for point ids either way, so one workspace serves both
    std::vector<BuildItemDev> it;
    int64_t tot = 0;
    for (int i = 0; h_items && i < n_items; ++i)
        tot = std::max<int64_t>(tot, h_items[i].xyz_offset + h_items[i].n_points);
    if (make_items(h_items, n_items, tot, false, &it) != PCT_OK) return 0;
    const BatchLayout L = batch_layout(h_items, it, n_items, n_robots);
    return L.F + L.E;
}

pct_status pct_tomogram_extent_batched(const float* d_xyz, int64_t n_total, pct_item* h_items, int32_t n_items,
                                       int64_t* total_cells, int64_t* total_slices, void* d_ws, size_t ws_bytes,
                                       void* stream) {
    clear_error();
    std::vector<BuildItemDev> it;
    pct_status st = make_items(h_items, n_items, n_total, false, &it);
    if (st != PCT_OK) return st;
    if (n_total > 0 && !d_xyz) return fail(PCT_ERR_ARG, "d_xyz is null");
    const size_t A = align_up(sizeof(BuildItemDev) * (size_t)n_items);
    const size_t need = A + batch_extent_ws_bytes(it.data(), n_items);
    if (!d_ws || ws_bytes < need) return fail(PCT_ERR_WORKSPACE, "batch extent workspace too small: %zu < %zu", ws_bytes, need);
    std::vector<ExtentDev> ex(n_items);
    st = launch_extent_batched(d_xyz, it.data(), n_items, (char*)d_ws + A, ex.data(), 1, (hipStream_t)stream);
    if (st != PCT_OK) return st;
    int64_t cells = 0, slices = 0;
    for (int i = 0; i < n_items; ++i) {
        pct_extent e{};
        e.z_min = INFINITY;
        e.z_max = -INFINITY;
        e.n_used = (int64_t)ex[i].used;
        e.n_dropped = h_items[i].n_points - e.n_used;
        if (e.n_used > 0) {
            e.z_min = ex[i].zmin;
            e.z_max = ex[i].zmax;
            const int N = plane_count(e.z_min, e.z_max, h_items[i].grid.slice_dz, PCT_MAX_SLICES);
            if (N == -1) return fail(PCT_ERR_ARG, "item %d: slice planes coincide in FP32", i);
            if (N == -2) return fail(PCT_ERR_CAPACITY, "item %d: more than %d slices needed", i, PCT_MAX_SLICES);
            e.n_slices = N;
        }
        h_items[i].extent = e;
        h_items[i].out_offset = cells;
        h_items[i].keep_offset = slices;
        cells += (int64_t)e.n_slices * h_items[i].grid.nx * h_items[i].grid.ny;
        slices += e.n_slices;
    }
    if (total_cells) *total_cells = cells;
    if (total_slices) *total_slices = slices;
    return PCT_OK;
}

pct_status pct_build_tomogram_batched(const float* d_xyz, int64_t n_total, const pct_item* h_items, int32_t n_items,
                                      float* d_ground, float* d_ceil, int32_t* d_arg_ground, int32_t* d_arg_ceil,
                                      int32_t flags, void* d_ws, size_t ws_bytes, void* stream) {
    clear_error();
    std::vector<BuildItemDev> it;
    pct_status st = make_items(h_items, n_items, n_total, true, &it, true);
    if (st != PCT_OK) return st;
    if ((d_arg_ground == nullptr) != (d_arg_ceil == nullptr))
        return fail(PCT_ERR_ARG, "d_arg_ground and d_arg_ceil must both be given or both be null");
    if (n_total > 0 && !d_xyz) return fail(PCT_ERR_ARG, "d_xyz is null");
    if (!d_ground || !d_ceil) return fail(PCT_ERR_ARG, "output pointers are null");
    return launch_build_batched(d_xyz, it.data(), n_items, d_ground, d_ceil, d_arg_ground, d_arg_ceil, d_ws, ws_bytes,
                                !(flags & PCT_DESCRIPTORS_RESIDENT), (hipStream_t)stream);
}

pct_status pct_eval_traversability_batched(const float* d_ground, const float* d_ceil, const pct_item* h_items,
                                           int32_t n_items, const pct_robot* h_robots, int32_t n_robots,
                                           float* d_cost, uint8_t* d_keep, int32_t flags, void* d_ws,
                                           size_t ws_bytes, void* stream) {
    clear_error();
    std::vector<BuildItemDev> it;
    int64_t tot = 0;
    for (int i = 0; h_items && i < n_items; ++i) tot = std::max<int64_t>(tot, h_items[i].xyz_offset + h_items[i].n_points);
    pct_status st = make_items(h_items, n_items, tot, true, &it);
    if (st != PCT_OK) return st;
    if (n_robots < 1 || !h_robots) return fail(PCT_ERR_ARG, "at least one robot is required");
    for (int r = 0; r < n_robots; ++r) {
        for (int i = 0; i < n_items; ++i) {
            st = check_robot(&h_robots[r], h_items[i].grid.res);
            if (st != PCT_OK) return st;
        }
    }
    if (!d_ground || !d_ceil || !d_cost) return fail(PCT_ERR_ARG, "device pointers are null");
    const BatchLayout L = batch_layout(h_items, it, n_items, n_robots);
    if (!d_ws || ws_bytes < L.F + L.E)
        return fail(PCT_ERR_WORKSPACE, "batch workspace too small: %zu < %zu", ws_bytes, L.F + L.E);
    const size_t eval_off = (ws_bytes - L.E) / 256 * 256;   // the last E bytes, 256-aligned
    return launch_eval_batched(d_ground, d_ceil, h_items, n_items, h_robots, n_robots, d_cost, d_keep,
                               (char*)d_ws + eval_off, ws_bytes - eval_off, !(flags & PCT_DESCRIPTORS_RESIDENT),
                               (hipStream_t)stream);
}

pct_status pct_autotune_batched(const float* d_xyz, int64_t n_total, const pct_item* h_items, int32_t n_items,
                                const pct_robot* h_robot, pct_tune_entry* h_out, int32_t n_max, int32_t* h_count,
                                void* stream) {
    clear_error();
    std::vector<BuildItemDev> it;
    pct_status st = make_items(h_items, n_items, n_total, true, &it);
    if (st != PCT_OK) return st;
    if (!h_robot) return fail(PCT_ERR_ARG, "h_robot is null");
    for (int i = 0; i < n_items; ++i) {
        st = check_robot(h_robot, h_items[i].grid.res);
        if (st != PCT_OK) return st;
    }
    if (n_total > 0 && !d_xyz) return fail(PCT_ERR_ARG, "d_xyz is null");
    if (n_max < 0 || (n_max > 0 && !h_out) || !h_count) return fail(PCT_ERR_ARG, "bad report arguments");
    *h_count = 0;
    hipStream_t s = (hipStream_t)stream;
    // the items with slices, by (class x, class y, R)
    std::map<std::vector<int>, std::vector<int>> groups;
    for (int i = 0; i < n_items; ++i) {
        if (h_items[i].extent.n_slices <= 0) continue;
        EvalParams p;
        st = make_eval_params(*h_robot, h_items[i].grid, h_items[i].extent.n_slices, &p);
        if (st != PCT_OK) return st;
        groups[{size_class(h_items[i].grid.nx), size_class(h_items[i].grid.ny), p.R}].push_back(i);
    }
    std::vector<pct_tune_entry> rep;
    std::map<std::pair<int, int>, bool> built;
    for (const auto& gkv : groups) {
        const int cx = gkv.first[0], cy = gkv.first[1], R = gkv.first[2];
        std::vector<pct_item> sub;
        long long cells = 0, slices = 0;
        for (int i : gkv.second) {
            pct_item t = h_items[i];
            t.out_offset = cells;
            t.keep_offset = slices;
            cells += (long long)t.extent.n_slices * t.grid.nx * t.grid.ny;
            slices += t.extent.n_slices;
            sub.push_back(t);
        }
        const int ns = (int)sub.size();
        const size_t ws_bytes = pct_batch_workspace_bytes(sub.data(), ns, 1, 0);
        if (ws_bytes == 0) return fail(PCT_ERR_ARG, "sizing the trial workspace failed");
        TrialBuffers tb;
        if (hipMalloc(&tb.p[0], sizeof(float) * cells) != hipSuccess ||
            hipMalloc(&tb.p[1], sizeof(float) * cells) != hipSuccess ||
            hipMalloc(&tb.p[2], sizeof(float) * cells) != hipSuccess || hipMalloc(&tb.p[3], ws_bytes) != hipSuccess)
            return fail(PCT_ERR_DEVICE, "allocating the trial buffers failed");
        float* G = (float*)tb.p[0];
        float* Cc = (float*)tb.p[1];
        float* cost = (float*)tb.p[2];
        void* ws = tb.p[3];
        auto build = [&](int flags) {
            return pct_build_tomogram_batched(d_xyz, n_total, sub.data(), ns, G, Cc, nullptr, nullptr, flags, ws,
                                              ws_bytes, s);
        };
        const int n_before = (int)rep.size();
        // construction tile height, once per (class x, class y), for maps
        // wider than 128 cells (narrower ones take tiles as wide as the map)
        if (!built[{cx, cy}] && cx >= 8) {
            built[{cx, cy}] = true;
            int th_min = 2;
            for (const pct_item& t : sub) th_min = std::max(th_min, make_grid_dev(t.grid).th);
            const int old = batch_build_th(cx, cy);
            float best = INFINITY;
            int best_th = 0;
            for (int th = th_min; th <= 8; th *= 2) {
                set_batch_build_th(cx, cy, th);
                float ms = 0.0f;
                st = time_calls(build, s, 3, &ms);
                if (st != PCT_OK) {
                    set_batch_build_th(cx, cy, old);
                    return st;
                }
                rep.push_back(pct_tune_entry{0, cx, cy, -1, th, 0, ns, 0, ms});
                if (ms < best) best = ms, best_th = th;
            }
            set_batch_build_th(cx, cy, best_th == th_min ? 0 : best_th);
            for (size_t k = n_before; k < rep.size(); ++k) rep[k].chosen = rep[k].rows == best_th;
        }
        st = build(0);
        if (st != PCT_OK) return st;
        // evaluation strip shape
        auto eval = [&](int flags) {
            return pct_eval_traversability_batched(G, Cc, sub.data(), ns, h_robot, 1, cost, nullptr, flags, ws,
                                                   ws_bytes, s);
        };
        EvalParams p0;
        const EvalShape old = batch_eval_shape(cx, cy, R);
        set_batch_eval_shape(cx, cy, R, EvalShape{0, 0});   // {0, 0} below: the default shape
        const EvalShape shapes[] = {{0, 0},  {32, 1},  {64, 1},  {128, 1}, {256, 1},
                                    {32, 4}, {64, 4},  {128, 4}, {256, 4}};
        const size_t e_before = rep.size();
        float best = INFINITY;
        EvalShape best_sh{0, 0};
        std::vector<std::vector<int>> tried;   // launches already timed (a shape that changes nothing is skipped)
        for (const EvalShape& sh : shapes) {
            bool fits = true;
            std::vector<int> sig;
            for (const pct_item& t : sub) {
                st = make_eval_params(*h_robot, t.grid, t.extent.n_slices, &p0);
                if (st != PCT_OK) {
                    set_batch_eval_shape(cx, cy, R, old);
                    return st;
                }
                if (sh.rows > 0 && !strip_shape_fits(p0, sh)) fits = false;
                int g4[4];
                batch_strip_signature(p0, sh, g4);
                sig.insert(sig.end(), g4, g4 + 4);
            }
            if (!fits || std::find(tried.begin(), tried.end(), sig) != tried.end()) continue;
            tried.push_back(sig);
            set_batch_eval_shape(cx, cy, R, sh);
            float ms = 0.0f;
            st = time_calls(eval, s, 3, &ms);
            if (st != PCT_OK) {
                set_batch_eval_shape(cx, cy, R, old);
                return st;
            }
            rep.push_back(pct_tune_entry{1, cx, cy, R, sh.rows, sh.nw, ns, 0, ms});
            if (ms < best) best = ms, best_sh = sh;
        }
        set_batch_eval_shape(cx, cy, R, best_sh);
        for (size_t k = e_before; k < rep.size(); ++k)
            rep[k].chosen = rep[k].rows == best_sh.rows && rep[k].waves == best_sh.nw;
    }
    for (int k = 0; k < (int)rep.size() && k < n_max; ++k) h_out[k] = rep[k];
    *h_count = (int32_t)rep.size();
    return PCT_OK;
}

pct_status pct_autotune_save(const char* path) {
    clear_error();
    if (!path) return fail(PCT_ERR_ARG, "path is null");
    char arch[256];
    pct_status st = current_arch(arch, sizeof arch);
    if (st != PCT_OK) return st;
    return tune_save(path, arch);
}

pct_status pct_autotune_load(const char* path, int32_t* n_applied) {
    clear_error();
    if (!path) return fail(PCT_ERR_ARG, "path is null");
    char arch[256];
    pct_status st = current_arch(arch, sizeof arch);
    if (st != PCT_OK) return st;
    int n = 0;
    st = tune_load(path, arch, &n);
    if (st == PCT_OK && n_applied) *n_applied = n;
    return st;
}

size_t pct_trajectory_multi_workspace_bytes(int32_t n_profiles) {
    if (n_profiles < 1) return 0;
    return align_up(sizeof(EvalParams) * (size_t)n_profiles);
}

pct_status pct_trajectory_cost_multi(const float* d_ground, const float* d_ceil, const int32_t* d_arg_ground,
                                     const int32_t* d_arg_ceil, const pct_grid* grid, const pct_extent* extent,
                                     const pct_robot* h_robots, int32_t n_profiles, float w_z, const float* d_wp,
                                     const int32_t* d_wp_slice, int32_t n_traj, int32_t n_wp, const float* d_gf,
                                     float* d_f, float* d_gwp, float* d_gground, float* d_gceil, int64_t n_points,
                                     float* d_gz, int32_t flags, void* d_ws, size_t ws_bytes, void* stream) {
    clear_error();
    if (n_profiles < 1 || !h_robots) return fail(PCT_ERR_ARG, "at least one profile is required");
    for (int i = 0; i < n_profiles; ++i) {
        pct_status st = check_sampling(grid, extent, &h_robots[i], n_traj, n_wp, d_wp, d_wp_slice);
        if (st != PCT_OK) return st;
    }
    if ((long long)n_profiles * n_traj * n_wp > (long long)INT32_MAX) return fail(PCT_ERR_CAPACITY, "too many waypoints");
    if (!isfinite(w_z)) return fail(PCT_ERR_ARG, "w_z must be finite");
    if (n_points < 0) return fail(PCT_ERR_ARG, "n_points must be >= 0");
    if ((long long)n_traj > 0 && !d_f) return fail(PCT_ERR_ARG, "d_f is null");
    if (d_gf && (long long)n_traj * n_wp > 0 && !d_gwp) return fail(PCT_ERR_ARG, "d_gwp is required with d_gf");
    if (d_gf && d_gz && n_points > 0 && (!d_arg_ground || !d_arg_ceil))
        return fail(PCT_ERR_ARG, "d_gz needs d_arg_ground and d_arg_ceil");
    const int N = extent->n_slices;
    if (N > 0 && (!d_ground || !d_ceil)) return fail(PCT_ERR_ARG, "grid pointers are null");
    const size_t need = pct_trajectory_multi_workspace_bytes(n_profiles);
    if (!d_ws || ws_bytes < need) return fail(PCT_ERR_WORKSPACE, "workspace too small: %zu < %zu", ws_bytes, need);
    std::vector<EvalParams> ps(n_profiles);
    for (int i = 0; i < n_profiles; ++i) {
        pct_status st = make_eval_params(h_robots[i], *grid, std::max(N, 1), &ps[i]);
        if (st != PCT_OK) return st;
        ps[i].N = N;
    }
    hipStream_t s = (hipStream_t)stream;
    const bool fixed = flags & PCT_FIXED_POINT;
    const int words = fixed ? 2 : 1;
    if (d_gf && !(flags & PCT_ACCUMULATE)) {
        const long long cells = (long long)N * grid->nx * grid->ny;
        pct_status st = launch_zero(d_gground, cells * words, s);
        if (st == PCT_OK) st = launch_zero(d_gceil, cells * words, s);
        if (st == PCT_OK) st = launch_zero(d_gz, d_gz ? n_points * words : 0, s);
        if (st != PCT_OK) return st;
    }
    EvalParams* d_ps = (EvalParams*)d_ws;
    Digest dg;
    for (const EvalParams& p : ps) digest_params(dg, p);
    if (pct_status st = resident_tables(d_ps, 2, dg.h, !(flags & PCT_DESCRIPTORS_RESIDENT))) return st;
    if (!(flags & PCT_DESCRIPTORS_RESIDENT)) {
        // ps is released on return: wait until the copy has read it
        PCT_HIP(hipMemcpyAsync(d_ps, ps.data(), sizeof(EvalParams) * n_profiles, hipMemcpyHostToDevice, s));
        PCT_HIP(hipStreamSynchronize(s));
    }
    if ((long long)n_traj * n_wp == 0) {
        if (n_traj > 0) return launch_zero(d_f, (long long)n_profiles * n_traj, s);
        return PCT_OK;
    }
    return launch_traj_value_grad(d_ground, d_ceil, d_arg_ground, d_arg_ceil, *grid, N, d_ps, n_profiles, w_z, d_wp,
                                  d_wp_slice, n_traj, n_wp, d_gf, d_f, d_gwp, d_gground, d_gceil, d_gz, n_points,
                                  fixed, s);
}

pct_status pct_fixed_to_float(const int64_t* d_acc, int64_t n, float* d_out, void* stream) {
    clear_error();
    if (n < 0) return fail(PCT_ERR_ARG, "n must be >= 0");
    if (n == 0) return PCT_OK;
    if (!d_acc || !d_out) return fail(PCT_ERR_ARG, "device pointers are null");
    const char* a = (const char*)d_acc;
    const char* o = (const char*)d_out;
    if (o < a + 8 * n && a < o + 4 * n) return fail(PCT_ERR_ARG, "d_out overlaps d_acc");
    return launch_fixed_to_float(d_acc, n, d_out, (hipStream_t)stream);
}

size_t pct_plan_workspace_bytes(int32_t nx, int32_t ny, int32_t n_layers) {
    if (nx < 1 || ny < 1 || n_layers < 1) return 0;
    return plan_ws_bytes(nx, ny, n_layers);
}

static pct_status check_node(const pct_grid* g, int32_t n_layers, int32_t x, int32_t y, int32_t l, const char* what) {
    if (x < 0 || y < 0 || x >= g->nx || y >= g->ny || l < 0 || l >= n_layers)
        return fail(PCT_ERR_ARG, "%s node (%d, %d, layer %d) outside the %d x %d x %d map", what, x, y, l, g->nx,
                    g->ny, n_layers);
    return PCT_OK;
}

pct_status pct_plan_distance(const float* d_cost, const float* d_ground, const pct_grid* grid,
                             const pct_extent* extent, const pct_robot* h_robot, const int32_t* h_layers,
                             int32_t n_layers, int32_t sx, int32_t sy, int32_t s_layer, double band, double* d_dist,
                             void* d_ws, size_t ws_bytes, int32_t* h_rounds, int64_t* h_tiles, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    st = check_robot(h_robot, grid->res);
    if (st != PCT_OK) return st;
    const int N = extent->n_slices;
    if (n_layers < 1 || n_layers > N) return fail(PCT_ERR_ARG, "n_layers %d outside [1, %d]", n_layers, N);
    if (!h_layers) return fail(PCT_ERR_ARG, "h_layers is null");
    for (int l = 0; l < n_layers; ++l) {
        if (h_layers[l] < 0 || h_layers[l] >= N || (l > 0 && h_layers[l] <= h_layers[l - 1]))
            return fail(PCT_ERR_ARG, "layers must be strictly increasing slice indices in [0, %d)", N);
    }
    st = check_node(grid, n_layers, sx, sy, s_layer, "start");
    if (st != PCT_OK) return st;
    if (!d_cost || !d_ground || !d_dist) return fail(PCT_ERR_ARG, "device pointers are null");
    if (!(band >= 0.0)) return fail(PCT_ERR_ARG, "band must be >= 0");
    const size_t need = plan_ws_bytes(grid->nx, grid->ny, n_layers);
    if (!d_ws || ws_bytes < need) return fail(PCT_ERR_WORKSPACE, "plan workspace too small: %zu < %zu", ws_bytes, need);
    int rounds = 0;
    long long tiles = 0;
    st = launch_plan(d_cost, d_ground, grid->nx, grid->ny, h_layers, n_layers, h_robot->c_barrier, sx, sy, s_layer,
                     d_dist, d_ws, &rounds, &tiles, (hipStream_t)stream, band > 0.0 ? band : kPlanDefaultBand);
    if (h_rounds) *h_rounds = rounds;
    if (h_tiles) *h_tiles = tiles;
    return st;
}

pct_status pct_plan_query(const float* d_cost, const float* d_ground, const pct_grid* grid, const pct_extent* extent,
                          const pct_robot* h_robot, const int32_t* h_layers, int32_t n_layers, int32_t sx, int32_t sy,
                          int32_t s_layer, int32_t gx, int32_t gy, int32_t g_layer, double band, double* d_dist,
                          void* d_ws, size_t ws_bytes, double* h_goal_dist, double* h_settled, int32_t* h_rounds,
                          int64_t* h_tiles, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    st = check_robot(h_robot, grid->res);
    if (st != PCT_OK) return st;
    const int N = extent->n_slices;
    if (n_layers < 1 || n_layers > N) return fail(PCT_ERR_ARG, "n_layers %d outside [1, %d]", n_layers, N);
    if (!h_layers) return fail(PCT_ERR_ARG, "h_layers is null");
    for (int l = 0; l < n_layers; ++l) {
        if (h_layers[l] < 0 || h_layers[l] >= N || (l > 0 && h_layers[l] <= h_layers[l - 1]))
            return fail(PCT_ERR_ARG, "layers must be strictly increasing slice indices in [0, %d)", N);
    }
    st = check_node(grid, n_layers, sx, sy, s_layer, "start");
    if (st != PCT_OK) return st;
    st = check_node(grid, n_layers, gx, gy, g_layer, "goal");
    if (st != PCT_OK) return st;
    if (!d_cost || !d_ground || !d_dist) return fail(PCT_ERR_ARG, "device pointers are null");
    if (!(band >= 0.0)) return fail(PCT_ERR_ARG, "band must be >= 0");
    const size_t need = plan_ws_bytes(grid->nx, grid->ny, n_layers);
    if (!d_ws || ws_bytes < need) return fail(PCT_ERR_WORKSPACE, "plan workspace too small: %zu < %zu", ws_bytes, need);
    const long long plane = (long long)grid->nx * grid->ny;
    const long long goal = (long long)g_layer * plane + (long long)gy * grid->nx + gx;
    int rounds = 0;
    long long tiles = 0;
    double settled = INFINITY;
    hipStream_t s = (hipStream_t)stream;
    st = launch_plan(d_cost, d_ground, grid->nx, grid->ny, h_layers, n_layers, h_robot->c_barrier, sx, sy, s_layer,
                     d_dist, d_ws, &rounds, &tiles, s, band > 0.0 ? band : kPlanDefaultBand, goal, &settled);
    if (st != PCT_OK) return st;
    double dg = INFINITY;
    PCT_HIP(hipMemcpyAsync(&dg, d_dist + goal, sizeof dg, hipMemcpyDeviceToHost, s));
    PCT_HIP(hipStreamSynchronize(s));
    if (h_goal_dist) *h_goal_dist = dg;
    if (h_settled) *h_settled = settled;
    if (h_rounds) *h_rounds = rounds;
    if (h_tiles) *h_tiles = tiles;
    return PCT_OK;
}

pct_status pct_plan_path(const double* d_dist, const pct_grid* grid, int32_t n_layers, int32_t sx, int32_t sy,
                         int32_t s_layer, int32_t gx, int32_t gy, int32_t g_layer, int32_t* d_path, int32_t max_len,
                         int32_t* h_len, void* d_ws, size_t ws_bytes, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    if (n_layers < 1 || n_layers > PCT_MAX_SLICES) return fail(PCT_ERR_ARG, "n_layers %d outside [1, %d]", n_layers,
                                                               PCT_MAX_SLICES);
    st = check_node(grid, n_layers, sx, sy, s_layer, "start");
    if (st != PCT_OK) return st;
    st = check_node(grid, n_layers, gx, gy, g_layer, "goal");
    if (st != PCT_OK) return st;
    if (max_len < 1) return fail(PCT_ERR_ARG, "max_len must be >= 1");
    if (!d_dist || !d_path || !h_len) return fail(PCT_ERR_ARG, "pointers are null");
    const size_t need = plan_ws_bytes(grid->nx, grid->ny, n_layers);
    if (!d_ws || ws_bytes < need) return fail(PCT_ERR_WORKSPACE, "plan workspace too small: %zu < %zu", ws_bytes, need);
    int len = 0;
    st = launch_plan_path(d_dist, grid->nx, grid->ny, n_layers, sx, sy, s_layer, gx, gy, g_layer, d_path, max_len,
                          d_ws, &len, (hipStream_t)stream);
    if (st != PCT_OK) return st;
    if (len == -2) return fail(PCT_ERR_CAPACITY, "path has more than %d nodes", max_len);
    if (len < 0) return fail(PCT_ERR_ARG, "d_dist is not a distance field of this graph");
    *h_len = len;
    return PCT_OK;
}

size_t pct_unique_workspace_bytes(const pct_grid* grid, const pct_extent* extent) {
    if (!grid || !extent || grid->nx < 1 || grid->ny < 1 || extent->n_slices < 1) return 0;
    return unique_ws_bytes(grid->nx, grid->ny, extent->n_slices);
}

pct_status pct_unique_cells(const float* d_ground, const float* d_ceil, const float* d_cost, const uint8_t* d_keep,
                            const pct_grid* grid, const pct_extent* extent, const pct_robot* h_robot,
                            int64_t capacity, int32_t* d_cell, float* d_ground_out, float* d_ceil_out,
                            float* d_cost_out, int64_t* h_slice_off, int64_t* h_count, void* d_ws, size_t ws_bytes,
                            void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    st = check_robot(h_robot, grid->res);
    if (st != PCT_OK) return st;
    if (!h_count) return fail(PCT_ERR_ARG, "h_count is null");
    if (capacity < 0) return fail(PCT_ERR_ARG, "capacity must be >= 0");
    const int N = extent->n_slices;
    if (N == 0) {
        *h_count = 0;
        if (h_slice_off) h_slice_off[0] = 0;
        return PCT_OK;
    }
    if (!d_ground || !d_ceil || !d_cost || !d_keep) return fail(PCT_ERR_ARG, "device pointers are null");
    if (d_cell && (!d_ground_out || !d_ceil_out || !d_cost_out))
        return fail(PCT_ERR_ARG, "with d_cell, the three value outputs are required");
    const size_t need = unique_ws_bytes(grid->nx, grid->ny, N);
    if (!d_ws || ws_bytes < need) return fail(PCT_ERR_WORKSPACE, "unique-cell workspace too small: %zu < %zu", ws_bytes,
                                              need);
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint8_t> keep((size_t)N);
    PCT_HIP(hipMemcpyAsync(keep.data(), d_keep, (size_t)N, hipMemcpyDeviceToHost, s));
    PCT_HIP(hipStreamSynchronize(s));
    long long count = 0;
    st = launch_unique(d_ground, d_ceil, d_cost, grid->nx, grid->ny, N, h_robot->c_barrier, keep.data(), capacity,
                       d_cell, d_ground_out, d_ceil_out, d_cost_out, (long long*)h_slice_off, &count, d_ws, s);
    *h_count = count;
    return st;
}

size_t pct_insert_workspace_bytes(int64_t n, const pct_grid* grid) {
    if (!grid || check_grid(grid) != PCT_OK || n < 0) return 0;
    const GridDev g = make_grid_dev(*grid);
    return std::max(extent_ws_bytes(std::max<int64_t>(n, 1)) + align_up(4 * sizeof(int)), build_ws_bytes(n, g, true));
}

pct_status pct_tomogram_insert(const float* d_xyz, int64_t n, int32_t id_base, const pct_grid* grid,
                               pct_extent* extent, float* d_ground, float* d_ceil, int32_t* d_arg_ground,
                               int32_t* d_arg_ceil, int32_t* h_bbox, void* d_ws, size_t ws_bytes, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    if (n < 0 || n > (int64_t)INT32_MAX) return fail(PCT_ERR_ARG, "point count %lld outside [0, 2^31)", (long long)n);
    if (id_base < 0 || (int64_t)id_base + n > (int64_t)INT32_MAX) return fail(PCT_ERR_ARG, "point ids exceed int32");
    if ((d_arg_ground == nullptr) != (d_arg_ceil == nullptr))
        return fail(PCT_ERR_ARG, "d_arg_ground and d_arg_ceil must both be given or both be null");
    const int N = extent->n_slices;
    if (N == 0) return fail(PCT_ERR_ARG, "the tomogram has no slices: build it first");
    if (!d_ground || !d_ceil) return fail(PCT_ERR_ARG, "output pointers are null");
    if (n > 0 && !d_xyz) return fail(PCT_ERR_ARG, "d_xyz is null");
    if (plane_count(extent->z_min, extent->z_max, grid->slice_dz, PCT_MAX_SLICES) != N)
        return fail(PCT_ERR_ARG, "extent does not match the plane rule for this slice_dz");
    if (h_bbox) h_bbox[0] = h_bbox[1] = 0, h_bbox[2] = h_bbox[3] = -1;
    if (n == 0) return PCT_OK;
    const size_t need = pct_insert_workspace_bytes(n, grid);
    if (!d_ws || ws_bytes < need) return fail(PCT_ERR_WORKSPACE, "insert workspace too small: %zu < %zu", ws_bytes, need);
    hipStream_t s = (hipStream_t)stream;
    const GridDev g = make_grid_dev(*grid);
    // heights and cells of the new points
    ExtentDev* d_out = (ExtentDev*)((char*)d_ws + extent_ws_bytes(n) - align_up(sizeof(ExtentDev)));
    int* d_bb = (int*)((char*)d_ws + extent_ws_bytes(n));
    st = launch_extent(d_xyz, n, g, d_ws, d_out, s);
    if (st != PCT_OK) return st;
    st = launch_cell_bbox(d_xyz, n, g, d_bb, s);
    if (st != PCT_OK) return st;
    ExtentDev hx{};
    int bb[4];
    PCT_HIP(hipMemcpyAsync(&hx, d_out, sizeof hx, hipMemcpyDeviceToHost, s));
    PCT_HIP(hipMemcpyAsync(bb, d_bb, sizeof bb, hipMemcpyDeviceToHost, s));
    PCT_HIP(hipStreamSynchronize(s));
    if (hx.used > 0) {
        // the union's planes must be the same: no new point below z_min, none
        // at or above the top plane
        const float top = plane_height(extent->z_min, grid->slice_dz, N - 1);
        if (hx.zmin < extent->z_min || !(hx.zmax < top))
            return fail(PCT_ERR_ARG, "new heights [%g, %g] leave [z_min %g, top plane %g): the planes change, rebuild",
                        (double)hx.zmin, (double)hx.zmax, (double)extent->z_min, (double)top);
        st = launch_build(d_xyz, n, g, extent->z_min, grid->slice_dz, N, d_ground, d_ceil, d_arg_ground, d_arg_ceil,
                          d_ws, ws_bytes, s, true, id_base);
        if (st != PCT_OK) return st;
        extent->z_max = std::max(extent->z_max, hx.zmax);
        if (h_bbox) {
            for (int i = 0; i < 4; ++i) h_bbox[i] = bb[i];
        }
    }
    extent->n_used += (int64_t)hx.used;
    extent->n_dropped += n - (int64_t)hx.used;
    return PCT_OK;
}

pct_status pct_eval_traversability_window(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                          const pct_extent* extent, const pct_robot* h_robot, int32_t x0, int32_t y0,
                                          int32_t x1, int32_t y1, float* d_cost, uint8_t* d_keep, void* d_ws,
                                          size_t ws_bytes, void* stream) {
    clear_error();
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    st = check_robot(h_robot, grid->res);
    if (st != PCT_OK) return st;
    const int N = extent->n_slices;
    if (N == 0) return PCT_OK;
    if (!d_ground || !d_ceil || !d_cost) return fail(PCT_ERR_ARG, "device pointers are null");
    x0 = std::max(x0, 0);
    y0 = std::max(y0, 0);
    x1 = std::min(x1, grid->nx);
    y1 = std::min(y1, grid->ny);
    if (d_keep && (!d_ws || ws_bytes < eval_ws_bytes(N, 1)))
        return fail(PCT_ERR_WORKSPACE, "eval workspace too small: %zu < %zu", ws_bytes, eval_ws_bytes(N, 1));
    hipStream_t s = (hipStream_t)stream;
    EvalParams p;
    st = make_eval_params(*h_robot, *grid, N, &p);
    if (st != PCT_OK) return st;
    if (x0 < x1 && y0 < y1) {
        p.wx0 = x0;
        p.wy0 = y0;
        p.wx1 = x1;
        p.wy1 = y1;
        st = launch_eval(d_ground, d_ceil, p, d_cost, s);
        if (st != PCT_OK) return st;
        p.wx0 = 0;
        p.wy0 = 0;
        p.wx1 = grid->nx;
        p.wy1 = grid->ny;
    }
    if (d_keep) return launch_simplify(d_ground, d_cost, p, d_keep, d_ws, ws_bytes, s);
    return PCT_OK;
}

struct pct_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

pct_status pct_graph_begin(void* stream) {
    clear_error();
    if (!stream) return fail(PCT_ERR_ARG, "graph capture needs a stream other than the null stream");
    PCT_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return PCT_OK;
}

pct_status pct_graph_end(void* stream, pct_graph* out) {
    clear_error();
    if (!stream || !out) return fail(PCT_ERR_ARG, "stream and out are required");
    *out = nullptr;
    hipGraph_t g = nullptr;
    PCT_HIP(hipStreamEndCapture((hipStream_t)stream, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(PCT_ERR_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(err));
    }
    pct_graph h = new pct_graph_s{g, e};
    *out = h;
    return PCT_OK;
}

pct_status pct_graph_launch(pct_graph graph, void* stream) {
    clear_error();
    if (!graph) return fail(PCT_ERR_ARG, "graph is null");
    PCT_HIP(hipGraphLaunch(graph->exec, (hipStream_t)stream));
    return PCT_OK;
}

pct_status pct_graph_destroy(pct_graph graph) {
    clear_error();
    if (!graph) return PCT_OK;
    const hipError_t e1 = hipGraphExecDestroy(graph->exec);
    const hipError_t e2 = hipGraphDestroy(graph->graph);
    delete graph;
    if (e1 != hipSuccess || e2 != hipSuccess) return fail(PCT_ERR_DEVICE, "destroying the graph failed");
    return PCT_OK;
}

namespace {

pct_status traj_args(const float* d_cost, const float* d_ground, const float* d_ceil, const pct_grid* grid,
                     const pct_extent* extent, const pct_traj_params* h_prm, int32_t n_traj, int32_t n_pieces,
                     const void* d_bound, const void* d_slice, const void* d_knots, const void* d_tau,
                     const void* d_phi, pct::TrajArgs* out) {
    pct_status st = check_grid(grid);
    if (st != PCT_OK) return st;
    st = check_extent(extent);
    if (st != PCT_OK) return st;
    if (!h_prm) return fail(PCT_ERR_ARG, "h_prm is null");
    const pct_traj_params& p = *h_prm;
    const float w[] = {p.w_z, p.w_c, p.w_v, p.w_a, p.w_h, p.w_T};
    for (float x : w)
        if (!(x >= 0.0f) || !isfinite(x)) return fail(PCT_ERR_ARG, "penalty weights must be finite and >= 0");
    if (!isfinite(p.c_safe) || !isfinite(p.d_ref) || !isfinite(p.d_min))
        return fail(PCT_ERR_ARG, "c_safe, d_ref and d_min must be finite");
    if (!(p.v_max > 0.0f) || !(p.a_max > 0.0f) || !isfinite(p.v_max) || !isfinite(p.a_max))
        return fail(PCT_ERR_ARG, "v_max and a_max must be finite and > 0");
    if (p.samples < 1 || p.samples > PCT_MAX_TRAJ_SAMPLES)
        return fail(PCT_ERR_ARG, "samples must be in [1, %d]", PCT_MAX_TRAJ_SAMPLES);
    if (n_traj < 0) return fail(PCT_ERR_ARG, "n_traj must be >= 0");
    if (n_pieces < 1 || n_pieces > PCT_MAX_PIECES) return fail(PCT_ERR_ARG, "n_pieces must be in [1, %d]", PCT_MAX_PIECES);
    if (n_traj > 0) {
        if (!d_bound || !d_slice || !d_tau || !d_phi) return fail(PCT_ERR_ARG, "trajectory pointers are null");
        if (n_pieces > 1 && !d_knots) return fail(PCT_ERR_ARG, "d_knots is null");
        if (extent->n_slices > 0 && (!d_cost || !d_ground || !d_ceil)) return fail(PCT_ERR_ARG, "map pointers are null");
    }
    pct::TrajArgs a{};
    a.cost = d_cost;
    a.ground = d_ground;
    a.ceil = d_ceil;
    a.nx = grid->nx;
    a.ny = grid->ny;
    a.N = extent->n_slices;
    a.x0 = grid->x0;
    a.y0 = grid->y0;
    a.res = grid->res;
    a.w_z = p.w_z;
    a.w_c = p.w_c;
    a.w_v = p.w_v;
    a.w_a = p.w_a;
    a.w_h = p.w_h;
    a.w_T = p.w_T;
    a.c_safe = p.c_safe;
    a.v_max2 = (double)p.v_max * (double)p.v_max;
    a.a_max2 = (double)p.a_max * (double)p.a_max;
    a.d_ref = p.d_ref;
    a.d_min = p.d_min;
    a.K = p.samples;
    a.M = n_pieces;
    *out = a;
    return PCT_OK;
}

}  // namespace

pct_status pct_traj_eval(const float* d_cost, const float* d_ground, const float* d_ceil, const pct_grid* grid,
                         const pct_extent* extent, const pct_traj_params* h_prm, int32_t n_traj, int32_t n_pieces,
                         const double* d_bound, const int32_t* d_slice, const double* d_knots, const double* d_tau,
                         double* d_phi, double* d_gknots, double* d_gtau, double* d_coef, void* stream) {
    clear_error();
    pct::TrajArgs a;
    pct_status st = traj_args(d_cost, d_ground, d_ceil, grid, extent, h_prm, n_traj, n_pieces, d_bound, d_slice,
                              d_knots, d_tau, d_phi, &a);
    if (st != PCT_OK) return st;
    if (n_traj > 0 && (!d_gtau || (n_pieces > 1 && !d_gknots))) return fail(PCT_ERR_ARG, "gradient pointers are null");
    return pct::launch_traj(a, n_traj, d_bound, d_slice, const_cast<double*>(d_knots), const_cast<double*>(d_tau),
                            d_phi, d_gknots, d_gtau, d_coef, -1, 0.0, nullptr, (hipStream_t)stream);
}

pct_status pct_traj_optimize(const float* d_cost, const float* d_ground, const float* d_ceil, const pct_grid* grid,
                             const pct_extent* extent, const pct_traj_params* h_prm, int32_t n_traj,
                             int32_t n_pieces, const double* d_bound, const int32_t* d_slice, double* d_knots,
                             double* d_tau, int32_t iters, double step, double* d_phi, int32_t* d_iters,
                             void* stream) {
    clear_error();
    pct::TrajArgs a;
    pct_status st = traj_args(d_cost, d_ground, d_ceil, grid, extent, h_prm, n_traj, n_pieces, d_bound, d_slice,
                              d_knots, d_tau, d_phi, &a);
    if (st != PCT_OK) return st;
    if (iters < 0) return fail(PCT_ERR_ARG, "iters must be >= 0");
    if (!(step > 0.0) || !isfinite(step)) return fail(PCT_ERR_ARG, "step must be finite and > 0");
    return pct::launch_traj(a, n_traj, d_bound, d_slice, d_knots, d_tau, d_phi, nullptr, nullptr, nullptr, iters,
                            step, d_iters, (hipStream_t)stream);
}

}  // extern "C"
