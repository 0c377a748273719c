// Internal declarations of libpct: device parameter blocks, launch helpers
// and the kernel launchers shared between the API and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "pct.h"

namespace pct {

// ---------------------------------------------------------------- errors
pct_status fail(pct_status code, const char* fmt, ...);
void clear_error();

#define PCT_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::pct::fail(PCT_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define PCT_LAUNCH_CHECK()                                                                \
    do {                                                                                  \
        hipError_t e_ = hipGetLastError();                                                \
        if (e_ != hipSuccess)                                                             \
            return ::pct::fail(PCT_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

__host__ __device__ inline size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------- grids
// Construction tiles are `tw` cells wide, 256 by default (each output row
// of a tile is one contiguous 1 KB run per slice), and `th` cells tall; th
// grows with the grid so that the tile count fits the LDS-privatised
// counters of the binning kernels.  Batched submaps narrower than 256 cells
// take tiles of 64 or 128 cells by 8 or 4, so that most of a tile's 512
// cells lie inside the map.
constexpr int kBuildTileW = 256;
constexpr int kMaxLdsTiles = 8192;

struct GridDev {
    float x0, y0, res, fnx, fny;
    int nx, ny;
    int th, ntx, nty;   // construction tiling
    int ntiles;
    int tw;
};

GridDev make_grid_dev(const pct_grid& g);
GridDev tile_shape(GridDev g, int tw, int th);

// On-device rasterisation (Sec. III-A): one FP32 subtraction and one
// correctly rounded FP32 division per axis, then the half-open range test.
__device__ __forceinline__ bool rasterize(float x, float y, const GridDev& g, int& ix, int& iy) {
    float qx = (x - g.x0) / g.res;
    float qy = (y - g.y0) / g.res;
    if (!(qx >= 0.0f && qx < g.fnx)) return false;
    if (!(qy >= 0.0f && qy < g.fny)) return false;
    ix = (int)qx;
    iy = (int)qy;
    return true;
}

// Plane k: z_min + (k+1) * d_s as one FP32 multiply and one FP32 add
// (the library is compiled with contraction off, so no FMA forms here).
__host__ __device__ __forceinline__ float plane_height(float zmin, float ds, int k) {
    float step = (float)(k + 1) * ds;
    return zmin + step;
}

// ---------------------------------------------------------------- extent
struct ExtentDev {
    float zmin, zmax;
    unsigned long long used;
};

// ---------------------------------------------------------------- batches
// One item of a batch (a submap): its points, grid, planes and where its
// outputs go.  Uploaded to the workspace as a device table.
struct BuildItemDev {
    GridDev g;
    long long xyz_off, n;
    float zmin, ds;
    int N;
    long long out_off;      // element offset of the item's [N][ny][nx] outputs
    int tile_base;          // first global construction tile
    int chunk_base;         // first global binning chunk
    int echunk_base;        // first global extent chunk
};

constexpr int kBatchChunk = 8192;     // points per workgroup in batched binning
constexpr int kBatchEChunk = 65536;   // points per workgroup in batched extents

// ---------------------------------------------------------------- eval
constexpr int kEvalTileW = 64;
constexpr int kEvalTileH = 16;
constexpr int kKmax = PCT_MAX_KERNEL_RADIUS + 1;

struct EvalParams {
    int nx, ny, N, R;
    long long plane;
    float d_min, d_ref, cB, alpha_d;
    float Tb;    // barrier:  max(|dx|, |dy|) > theta_b * 2r   (dx, dy: raw ground differences)
    float Ts2;   // gentle:   dx^2 + dy^2 < (theta_s * 2r)^2
    float As;    // gentle cost  alpha_s / (theta_s * 2r)^2 * (dx^2 + dy^2)
    float Ab;    // step cost    alpha_b / (theta_b * 2r)^2 * max(dx^2, dy^2)
    int rp, kp;  // patch radius, count threshold floor(theta_p * P)
    int wx0, wy0, wx1, wy1;  // cells evaluated: [wx0, wx1) x [wy0, wy1) (the whole map unless a window is asked)
    float K[kKmax][kKmax];  // K[a][j]: Eq. (6) weight at horizontal offset a, vertical offset j
};

pct_status make_eval_params(const pct_robot& r, const pct_grid& g, int N, EvalParams* out);

// ---------------------------------------------------------------- launchers
pct_status launch_extent(const float* xyz, int64_t n, const GridDev& g, void* ws, ExtentDev* d_out,
                         hipStream_t s);
size_t extent_ws_bytes(int64_t n);
pct_status launch_extent_record(const float* xyz, int64_t n, const GridDev& g, float ds, void* ws, pct_extent* d_out,
                                hipStream_t s);

size_t build_ws_bytes(int64_t n, const GridDev& g, bool ids);
pct_status launch_cell_bbox(const float* xyz, int64_t n, const GridDev& g, int* d_bb, hipStream_t s);
pct_status launch_build(const float* xyz, int64_t n, const GridDev& g, float zmin, float ds, int N,
                        float* ground, float* ceil, int32_t* ag, int32_t* ac, void* ws, size_t ws_bytes,
                        hipStream_t s, bool merge = false, int id_base = 0);

size_t eval_ws_bytes(int N, int n_robots);
size_t eval_ws_min_bytes(int N);   // the least scratch the slice test runs in (one copy of the run starts)
// Strip shape of the evaluation: output rows per strip and wavefronts per
// workgroup sharing one strip (1: each wavefront its own strip);
// rows = 0: the tuned shape for the map if recorded, else the default.
struct EvalShape {
    int rows, nw;
};
pct_status launch_eval(const float* ground, const float* ceil, const EvalParams& p, float* cost, hipStream_t s,
                       EvalShape shape = EvalShape{0, 0});
pct_status autotune_eval(const float* ground, const float* ceil, const EvalParams& p, float* cost, hipStream_t s,
                         EvalShape* best, EvalShape* cand, float* cand_ms, int n_max, int* n_cand);
void autotune_reset();
void autotune_set(const EvalParams& p, EvalShape shape);
bool strip_shape_fits(const EvalParams& p, EvalShape shape);
pct_status launch_eval_simplify(const float* ground, const float* ceil, const EvalParams& p, float* cost, uint8_t* keep,
                                void* ws, size_t ws_bytes, hipStream_t s);

// Batch tuning tables, per size class (ceil(log2 nx), ceil(log2 ny)): the
// evaluation's strip shape for a kernel radius ({0, 0}: default) and the
// construction's tile height (0: default).  Saved and loaded as text with the
// single-map table, for one device architecture.
int size_class(int v);
EvalShape batch_eval_shape(int cx, int cy, int R);
void set_batch_eval_shape(int cx, int cy, int R, EvalShape shape);
int batch_build_th(int cx, int cy);
void set_batch_build_th(int cx, int cy, int th);
// What a batched launch of a job with parameters p does with strip shape
// `shape` ({0, 0}: the shape batched calls use now): wavefronts per
// workgroup, strips across and down, and the strip height when it matters.
void batch_strip_signature(const EvalParams& p, EvalShape shape, int out[4]);
pct_status tune_save(const char* path, const char* arch);
pct_status tune_load(const char* path, const char* arch, int* n_applied);

// Descriptor tables kept in a workspace region for PCT_DESCRIPTORS_RESIDENT
// calls: an upload records a digest of the host plan (kind: which table);
// a resident call fails unless its own plan has the recorded digest.
struct Digest {
    uint64_t h = 1469598103934665603ull;
    template <class T>
    void add(const T& v) {
        const unsigned char* b = (const unsigned char*)&v;
        for (size_t i = 0; i < sizeof(T); ++i) h = (h ^ b[i]) * 1099511628211ull;
    }
};
void digest_params(Digest& d, const EvalParams& p);
pct_status resident_tables(const void* region, int kind, uint64_t digest, bool upload);
pct_status launch_simplify(const float* ground, const float* cost, const EvalParams& p, uint8_t* keep,
                           void* ws, size_t ws_bytes, hipStream_t s);

pct_status launch_zero(float* p, long long n, hipStream_t s);

// batched construction (items: device table; host copy for launch sizes)
size_t batch_extent_ws_bytes(const BuildItemDev* items, int n_items);
pct_status launch_extent_batched(const float* xyz, const BuildItemDev* h_items, int n_items, void* ws,
                                 ExtentDev* h_out, int upload, hipStream_t s);
size_t batch_build_ws_bytes(const BuildItemDev* items, int n_items, bool ids);
size_t batch_eval_ws_bytes(const pct_item* items, int n_items, int n_robots);
pct_status launch_eval_batched(const float* ground, const float* ceil, const pct_item* items, int n_items,
                               const pct_robot* robots, int n_robots, float* cost, uint8_t* keep, void* ws,
                               size_t ws_bytes, int upload, hipStream_t s);
pct_status launch_build_batched(const float* xyz, const BuildItemDev* h_items, int n_items, float* ground,
                                float* ceil, int32_t* ag, int32_t* ac, void* ws, size_t ws_bytes, int upload,
                                hipStream_t s);
pct_status launch_sample_fwd(const float* cost, const float* ground, const pct_grid& g, int N, float d_ref, float w_z,
                             const float* wp, const int* slice, int T, int W, float* f, hipStream_t s);
pct_status launch_sample_bwd(const float* cost, const float* ground, const float* ceil, const pct_grid& g, int N,
                             float d_ref, float w_z, const float* wp, const int* slice, int T, int W, const float* gf,
                             float* gwp, float* gcost, float* gground, const EvalParams* ep, const int* aG,
                             const int* aC, float* gz, long long n_points, bool fixed, hipStream_t s);
pct_status launch_eval_bwd(const float* ground, const float* ceil, const float* gcost, const EvalParams& p,
                           float* gground, float* gceil, bool fixed, hipStream_t s);
pct_status launch_traj_value_grad(const float* ground, const float* ceil, const int* aG, const int* aC,
                                  const pct_grid& g, int N, const EvalParams* d_robots, int n_profiles, float w_z,
                                  const float* wp, const int* slice, int T, int W, const float* gf, float* f,
                                  float* gwp, float* gground, float* gceil, float* gz, long long n_points,
                                  bool fixed, hipStream_t s);
pct_status launch_route(const float* gG, const float* gC, const int* aG, const int* aC, long long plane, int N,
                        long long n_points, float* gz, bool fixed, hipStream_t s);
pct_status launch_fixed_to_float(const int64_t* q, long long n, float* out, hipStream_t s);

}  // namespace pct
