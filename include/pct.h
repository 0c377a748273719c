/*
 * pct.h - C ABI of the MI355X (gfx950) point-cloud-tomography library.
 *
 * Method: Yang et al., "Efficient Global Navigational Planning in 3D
 * Structures based on Point Cloud Tomography" (arXiv 2403.07631).
 *   - tomogram construction: Sec. III-A and Algorithm 1 (construction lines);
 *   - traversability: Sec. III-B, Eqs. (1)-(6);
 *   - simplification: Sec. III-C, Eqs. (7)-(9);
 *   - trajectory cost sampling and adjoints: the cost and height terms of the
 *     trajectory optimisation of Sec. III-E, Eq. (11).
 *
 * Conventions shared by every entry point
 *   - Pointers named d_* are device (HBM) pointers owned by the caller; the
 *     library never allocates or frees device memory.  Pointers named h_* or
 *     passed as structs are host pointers, read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All device work is enqueued on it; only pct_tomogram_extent waits for it.
 *   - Grids are stored [slice][iy][ix], ix fastest (row-major, x = column).
 *   - Every entry point validates its arguments before enqueueing anything
 *     and returns a pct_status.  On error nothing is launched and
 *     pct_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).  A HIP error is reported as PCT_ERR_DEVICE.
 *   - Workspaces are caller-provided device buffers of at least the size the
 *     matching *_workspace_bytes function returns, 256-byte aligned.
 *   - Arithmetic is FP32.  Tomograms are exact: every stored height is the
 *     height of an input point.
 */
#ifndef PCT_H
#define PCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pct_status;
#define PCT_OK 0
#define PCT_ERR_ARG (-1)       /* invalid argument (null pointer, bad size, bad parameter) */
#define PCT_ERR_WORKSPACE (-2) /* workspace smaller than required */
#define PCT_ERR_CAPACITY (-3)  /* a size limit below is exceeded */
#define PCT_ERR_DEVICE (-4)    /* a HIP runtime call failed */

#define PCT_ABI_VERSION 1
#define PCT_MAX_SLICES 1024      /* N, the number of slice planes */
#define PCT_MAX_KERNEL_RADIUS 16 /* support radius of the inflation kernel, in cells */
#define PCT_MAX_PATCH_RADIUS 4   /* r_p of the step test's neighbour patch */
#define PCT_MAX_GRID_SIDE 65535  /* nx, ny */
#define PCT_MAX_PIECES 64        /* M, polynomial pieces of one trajectory */
#define PCT_MAX_TRAJ_SAMPLES 64  /* K, penalty samples per piece (K + 1 times) */

/* Grid of Sec. III-A: resolution r_g = res, slice interval d_s = slice_dz.
 * Cell (ix, iy) holds the points with floor((x - x0) / res) = ix and
 * floor((y - y0) / res) = iy, the subtraction and the division each being one
 * correctly rounded FP32 operation.  Points outside [0,nx) x [0,ny) are not
 * part of the map. */
typedef struct {
    float x0, y0, res;
    int32_t nx, ny;
    float slice_dz;
} pct_grid;

/* Vertical extent of the map (Algorithm 1, first line) and the slice count.
 * Plane k (k = 0 .. n_slices-1) is at h_k = z_min + (k+1) * slice_dz, one
 * FP32 multiply then one FP32 add; n_slices is the least N with
 * h_{N-1} > z_max (Sec. III-A).  n_used counts the points that belong to the
 * map (finite and inside the grid), n_dropped the others.  An empty map has
 * n_slices = 0. */
typedef struct {
    float z_min, z_max;
    int32_t n_slices;
    int32_t reserved;
    int64_t n_used, n_dropped;
} pct_extent;

/* Robot parameters of Eqs. (1)-(6) and Table I.  theta_b, theta_s bound the
 * gradient magnitudes m^xy and m^grad of Eq. (2); theta_p bounds the share
 * p_s of gentle neighbours in the (2 patch_radius + 1)^2 patch of Eq. (4);
 * d_inf and d_sm shape the inflation kernel of Eq. (6). */
typedef struct {
    float d_min, d_ref, theta_b, theta_s, theta_p, c_barrier, alpha_d, alpha_b, alpha_s, d_inf, d_sm;
    int32_t patch_radius;
} pct_robot;

/* ABI version of the loaded library (PCT_ABI_VERSION). */
int32_t pct_abi_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* pct_last_error(void);

/* Host only.  Robot parameters from a physical description at grid
 * resolution res: theta_s = tan(max_slope), theta_b = max_step / (2 res)
 * (a central difference across a step of height s is s / 2r, Eq. (2)),
 * d_min = min_interval, d_ref = nominal_height, d_inf = inflation_radius,
 * d_sm = safe_margin; theta_p = 0.2, c^B = 50, alpha_d = 20, alpha_b = 20,
 * alpha_s = 15 from Table I; patch_radius = 1.  PCT_ERR_ARG on a
 * non-positive size or a slope outside (0, 90) degrees. */
pct_status pct_robot_from_physical(float min_interval, float nominal_height, float max_slope_deg,
                                   float max_step, float inflation_radius, float safe_margin, float res,
                                   pct_robot* out);

/* Host only.  Checks a grid (res > 0, slice_dz > 0, 1 <= nx, ny <= 65535,
 * finite origin). */
pct_status pct_validate_grid(const pct_grid* grid);

/* Host only.  Checks a robot at resolution res: finite parameters,
 * c_barrier > 0, theta_b, theta_s > 0 with theta_b * 2 res finite in
 * single precision, d_sm > res (the margin of Eq. (6) must be wider than a
 * cell), 1 <= patch_radius <= 4, kernel radius <= 16. */
pct_status pct_validate_robot(const pct_robot* robot, float res);

/* Host only.  Support radius R (cells) of the Eq. (6) kernel of a robot at
 * resolution res: the largest max(|m|,|n|) with K(m,n) > 0. */
pct_status pct_kernel_radius(const pct_robot* robot, float res, int32_t* radius_out);

/* Host only.  Plane heights h_0 .. h_{N-1} of an extent (see pct_extent),
 * written to h_out[0 .. cap).  PCT_ERR_CAPACITY if N > cap. */
pct_status pct_plane_heights(const pct_extent* extent, float slice_dz, float* h_out, int32_t cap);

/* ---------------------------------------------------------------------- */
/* Tomogram construction (Sec. III-A, Algorithm 1)                        */

/* Workspace bytes for pct_tomogram_extent over n points. */
size_t pct_extent_workspace_bytes(int64_t n);

/* Algorithm 1, first line, and the plane count of Sec. III-A.
 * d_xyz: n points, float32 [n][3] (x, y, z).  Non-finite points and points
 * outside the grid are dropped; -0 heights count as +0.  Writes *h_out and
 * returns after synchronising `stream` (the slice count sizes the outputs
 * of pct_build_tomogram).  PCT_ERR_CAPACITY if more than PCT_MAX_SLICES
 * planes are needed, PCT_ERR_ARG if two planes coincide in FP32. */
pct_status pct_tomogram_extent(const float* d_xyz, int64_t n, const pct_grid* grid, pct_extent* h_out,
                               void* d_ws, size_t ws_bytes, void* stream);

/* pct_tomogram_extent without the host synchronisation, so that it can be
 * enqueued ahead or captured in a graph: the same record, written to
 * d_out (device memory, one pct_extent) when the stream reaches it.  Where
 * the host version fails on the plane rule, n_slices is -1 (two planes
 * coincide in FP32) or -2 (more than PCT_MAX_SLICES planes).  Workspace as
 * for pct_tomogram_extent (at least 256 bytes when n = 0). */
pct_status pct_tomogram_extent_device(const float* d_xyz, int64_t n, const pct_grid* grid, pct_extent* d_out,
                                      void* d_ws, size_t ws_bytes, void* stream);

/* Workspace bytes for pct_build_tomogram. */
size_t pct_build_workspace_bytes(int64_t n, const pct_grid* grid, const pct_extent* extent);

/* Algorithm 1, construction loop: for every slice k and cell, the ground
 * e^G_k = highest height of the cell's points at or below plane h_k and the
 * ceiling e^C_k = lowest height above it (Sec. III-A: the lower group is
 * projected up to the ground layer, the upper group down to the ceiling).
 * Empty sets give e^G = -inf, e^C = +inf.
 * Outputs d_ground, d_ceil: float32 [N][ny][nx], fully overwritten.
 * d_arg_ground, d_arg_ceil (nullable, both or neither): int32 [N][ny][nx],
 * the index in d_xyz of the point that gives the value (lowest index among
 * equal heights), -1 where invalid.  `extent` must come from
 * pct_tomogram_extent on the same points and grid. */
pct_status pct_build_tomogram(const float* d_xyz, int64_t n, const pct_grid* grid, const pct_extent* extent,
                              float* d_ground, float* d_ceil, int32_t* d_arg_ground, int32_t* d_arg_ceil,
                              void* d_ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Traversability (Sec. III-B) and simplification (Sec. III-C)            */

/* Workspace bytes for pct_eval_traversability (any number of robots: they
 * reuse it in turn): the slice test's scratch, each part 256-byte aligned:
 * an N x N bit matrix of in-run comparisons (4 N ceil(N / 32) bytes), one
 * bit per slice marking the slices with a traversable cell (the slice test
 * reads no other slice), and 16 copies of the per-slice largest run starts,
 * 4 KB apart (the many wavefronts that reach a slice together spread their
 * atomics over the copies).  Only d_keep needs it. */
size_t pct_eval_workspace_bytes(const pct_grid* grid, const pct_extent* extent, int32_t n_robots);

/* Eqs. (1)-(6) for every slice, then the slice test of Eqs. (7)-(9), for
 * each of n_robots robots (h_robots: host array).
 *   c^I:   d^I = e^C - e^G; c^B if d^I < d_min else max(0, alpha_d (d_ref - d^I)).
 *   c^G:   central differences of e^G over 2 res; c^B if m^xy > theta_b;
 *          alpha_s (m^grad / theta_s)^2 if m^grad < theta_s; otherwise
 *          alpha_b (m^xy / theta_b)^2 if more than floor(theta_p * P) of the
 *          P = (2 r_p + 1)^2 - 1 patch neighbours are gentle, else c^B.
 *   c^init = min(c^B, c^I + c^G); c^B where there is no ground.  A stencil
 *          reaching off the grid or into a cell without ground gives an
 *          infinite slope.  No ceiling gives c^I = 0.
 *   c^T:   max over the Eq. (6) window of K(m,n) * c^init (off-grid taps
 *          skipped).
 *   keep:  slice k is kept if some cell with c^T < c^B differs from the last
 *          kept slice (higher ground or lower cost; true when none is kept
 *          yet) and from slice k+1 (higher ground there or lower cost here;
 *          true for the last slice).
 * d_ground, d_ceil: float32 [N][ny][nx] from pct_build_tomogram.
 * d_cost: float32 [n_robots][N][ny][nx], fully overwritten with c^T.
 * d_keep: uint8 [n_robots][N], 1 = kept (nullable: skip the slice test). */
pct_status pct_eval_traversability(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                   const pct_extent* extent, const pct_robot* h_robots, int32_t n_robots,
                                   float* d_cost, uint8_t* d_keep, void* d_ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * evaluation and slice test as pct_eval_traversability, with the slice
 * test's scratch (the N x N bit matrix, the slice marks and as many copies
 * of the run starts as fit, at least one) in a library-owned static device
 * array of PCT_STATIC_WORKSPACE_BYTES instead of a caller workspace.  Each GPU the library runs on holds its own copy
 * of that array until the process ends; the first call on a device finds
 * its address (with that device current).  The call allocates nothing and
 * clears the part of the array it uses before using it.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams or threads without ordering) race and give wrong keep flags.
 * The stream must belong to the current device (PCT_ERR_ARG otherwise).
 * PCT_ERR_CAPACITY when the slice test would need more than the array
 * holds (it cannot for n_slices <= PCT_MAX_SLICES).  Other arguments,
 * outputs and errors as pct_eval_traversability. */
#define PCT_STATIC_WORKSPACE_BYTES (136u * 1024u)
pct_status pct_eval_traversability_static(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                          const pct_extent* extent, const pct_robot* h_robots, int32_t n_robots,
                                          float* d_cost, uint8_t* d_keep, void* stream);

/* Autotuner for pct_eval_traversability.  Times the evaluation of this
 * map shape for each candidate strip shape and records the fastest; later
 * evaluations in this process of a map with the same nx, ny, slice count
 * and kernel radius use it.  A strip is the rows of one slice that one
 * workgroup walks down (32, 64, ... up to the first at or above ny, at most
 * 1024), either one wavefront per 64-column strip (waves = 1) or 2 or
 * PCT_STRIP_WAVES wavefronts side by side sharing the inflation's row pass
 * through LDS (waves = 2, PCT_STRIP_WAVES).  At most 24 candidates.
 * Synchronous.
 * d_cost: float32 [N][ny][nx] scratch, overwritten.
 * h_rows/h_waves/h_ms: host arrays of n_max entries for the candidates'
 * heights, wavefronts and times in ms (each nullable); *h_count = the
 * number of candidates; *h_best_rows, *h_best_waves (nullable) = the
 * chosen shape, rows 0 when this robot's evaluation does not use strips
 * (patch radius above 1 or inflation radius above 8). */
#define PCT_STRIP_WAVES 4
pct_status pct_autotune_traversability(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                       const pct_extent* extent, const pct_robot* h_robot, float* d_cost,
                                       int32_t* h_best_rows, int32_t* h_best_waves, int32_t* h_rows,
                                       int32_t* h_waves, float* h_ms, int32_t n_max, int32_t* h_count, void* stream);

/* Forgets every shape the autotuners recorded, single-map and per size
 * class (defaults apply again). */
pct_status pct_autotune_reset(void);

/* Records a strip shape (rows, waves as in the autotuner) for the
 * evaluation of maps of this shape (nx, ny, slice count) and this robot's
 * inflation radius, as the autotuner does with the fastest candidate: for
 * tuning results kept between processes, or to pin a shape.  rows = 0
 * forgets the entry (the default applies).  PCT_ERR_ARG if rows is not 0
 * and outside [16, PCT_MAX_STRIP_ROWS], or waves is not 1, 2 or
 * PCT_STRIP_WAVES; PCT_ERR_CAPACITY if strips that short would need more
 * than 2^30 wavefronts for this map.  No device work. */
#define PCT_MAX_STRIP_ROWS 4096
pct_status pct_autotune_set_traversability(const pct_grid* grid, const pct_extent* extent, const pct_robot* h_robot,
                                           int32_t rows, int32_t waves);

/* ---------------------------------------------------------------------- */
/* Trajectory cost sampling (Sec. III-E) and adjoints                     */

/* Flag for the gradient entry points: add into the gradient outputs instead
 * of overwriting them (without it the outputs are zero-filled first). */
#define PCT_ACCUMULATE 1

/* Flag for the gradient entry points: the summed gradient outputs (d_gcost,
 * d_gground, d_gceil, d_gz; not d_gwp, which is written once per waypoint)
 * are int64_t arrays in fixed point, value = integer * 2^-PCT_FIXED_FRAC_BITS,
 * passed through the same float* parameters (8 bytes per element).  Each
 * contribution is rounded to the nearest multiple of 2^-32 (ties to even)
 * and added as an integer, so a sum is the same whatever the order in which
 * its terms arrive, and the same when the work is split over several calls
 * with PCT_ACCUMULATE: a per-profile loop and pct_trajectory_cost_multi
 * give identical bits.  Without the flag the sums are float atomics whose
 * last bits depend on that order.  Range: a contribution is clamped to
 * +-2^30, NaN adds nothing, and a sum beyond +-2^31 wraps.  Convert with
 * pct_fixed_to_float. */
#define PCT_FIXED_POINT 4
#define PCT_FIXED_FRAC_BITS 32

/* d_out[i] = d_acc[i] * 2^-32 correctly rounded to float32, for i < n: the
 * fixed-point gradient sums of PCT_FIXED_POINT as floats.  d_acc (int64_t
 * [n]) and d_out (float32 [n]) must not overlap (PCT_ERR_ARG). */
pct_status pct_fixed_to_float(const int64_t* d_acc, int64_t n, float* d_out, void* stream);

/* The cost and height terms of the trajectory optimisation, Eq. (11):
 * travel cost C and preferred height Z_ref = e^G + d_ref along a trajectory.
 * A waypoint (x, y, z) on slice k contributes
 *     f = C_k(x, y) + w_z (z - G_k(x, y) - d_ref)^2,
 * where C_k and G_k interpolate c^T_k and e^G_k bilinearly between cell
 * centres (clamped at the grid edge, zero slope across the clamp); the
 * height term is dropped when one of the four ground corners is missing.
 * A trajectory's cost is the sum over its waypoints; waypoints with a
 * non-finite coordinate or a slice outside [0, N) contribute nothing.
 * d_cost, d_ground: float32 [N][ny][nx] (one robot's c^T and the ground);
 * d_wp: float32 [n_traj][n_wp][3]; d_wp_slice: int32 [n_traj][n_wp];
 * d_f: float32 [n_traj], overwritten.  d_ref is h_robot->d_ref. */
pct_status pct_sample_cost_fwd(const float* d_cost, const float* d_ground, const pct_grid* grid,
                               const pct_extent* extent, const pct_robot* h_robot, float w_z, const float* d_wp,
                               const int32_t* d_wp_slice, int32_t n_traj, int32_t n_wp, float* d_f, void* stream);

/* Adjoint of pct_sample_cost_fwd for upstream gradients d_gf [n_traj]:
 * d_gwp [n_traj][n_wp][3] (overwritten) = dL/d(x, y, z); d_gcost and
 * d_gground [N][ny][nx] (nullable) = dL/dc^T and the height term's dL/de^G
 * (bilinear scatter to the four corners). */
pct_status pct_sample_cost_bwd(const float* d_cost, const float* d_ground, const pct_grid* grid,
                               const pct_extent* extent, const pct_robot* h_robot, float w_z, const float* d_wp,
                               const int32_t* d_wp_slice, int32_t n_traj, int32_t n_wp, const float* d_gf,
                               float* d_gwp, float* d_gcost, float* d_gground, int32_t flags, void* stream);

/* Adjoint of pct_eval_traversability (one robot) for dL/dc^T = d_gcost:
 * dL/de^G and dL/de^C [N][ny][nx].  Each c^T value is K(t) c^init at the
 * maximising tap t of its Eq. (6) window (the first maximum in row-major
 * window order), so its gradient goes to that cell; there Eq. (5) passes it
 * on unless the clip is active, Eq. (1) gives +alpha_d to e^G and -alpha_d
 * to e^C where the interval cost is positive, and the gentle and step costs
 * of Eqs. (3)-(4) differentiate through the central differences (the step
 * cost through its larger axis, x on a tie); barrier branches and the
 * neighbour count give none. */
pct_status pct_eval_traversability_bwd(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                       const pct_extent* extent, const pct_robot* h_robot, const float* d_gcost,
                                       float* d_gground, float* d_gceil, int32_t flags, void* stream);

/* Adjoint of pct_build_tomogram: every ground/ceiling value is the height
 * of the point recorded in d_arg_ground/d_arg_ceil, so d_gz[id] (float32
 * [n_points]) receives the sum of the gradients of the values it holds.
 * d_gceil may be null. */
pct_status pct_route_grad_to_points(const float* d_gground, const float* d_gceil, const int32_t* d_arg_ground,
                                    const int32_t* d_arg_ceil, const pct_grid* grid, const pct_extent* extent,
                                    int64_t n_points, float* d_gz, int32_t flags, void* stream);

/* The three adjoints above in one pass, without dense gradient grids:
 * from d_gf to d_gwp (overwritten) and to d_gz [n_points], the gradient of
 * every point height through the sampled costs, the traversability
 * evaluation and the construction.  d_cost is the robot's c^T. */
pct_status pct_trajectory_cost_bwd(const float* d_ground, const float* d_ceil, const float* d_cost,
                                   const int32_t* d_arg_ground, const int32_t* d_arg_ceil, const pct_grid* grid,
                                   const pct_extent* extent, const pct_robot* h_robot, float w_z, const float* d_wp,
                                   const int32_t* d_wp_slice, int32_t n_traj, int32_t n_wp, const float* d_gf,
                                   int64_t n_points, float* d_gwp, float* d_gz, int32_t flags, void* stream);

/* ---------------------------------------------------------------------- */
/* Batches: many submaps (and robots) per launch                          */

/* Flag: the workspace already holds this batch's descriptor tables from an
 * earlier call with the same items (and robots); nothing is copied from the
 * host, so the call only enqueues kernels and can be captured in a graph.
 * Without the flag the call copies the tables from host memory and waits on
 * the stream until that copy is done (the host tables are temporary). */
#define PCT_DESCRIPTORS_RESIDENT 2

/* One submap of a batch.  The caller sets xyz_offset, n_points and grid;
 * pct_tomogram_extent_batched sets extent and the packing offsets: item i's
 * [N][ny][nx] grids start at element out_offset of the packed grid outputs,
 * its N slice flags at keep_offset of the packed flag outputs. */
typedef struct {
    int64_t xyz_offset;
    int64_t n_points;
    pct_grid grid;
    int32_t reserved;
    pct_extent extent;
    int64_t out_offset;
    int64_t keep_offset;
} pct_item;

/* Workspace bytes for the batched calls (the largest of the three). */
size_t pct_batch_workspace_bytes(const pct_item* h_items, int32_t n_items, int32_t n_robots, int32_t with_ids);

/* Graph capture on a stream, for callers without a framework of their own:
 * pct_graph_begin starts capturing `stream` (thread-local mode); the library
 * calls enqueued on it until pct_graph_end are recorded instead of run, and
 * pct_graph_end returns an instantiated graph that pct_graph_launch replays
 * on any stream.  Only calls that need no host synchronisation can be
 * captured: the batched construction and evaluation with
 * PCT_DESCRIPTORS_RESIDENT, the sampling and gradient calls.  A replay reads
 * and writes the buffers the captured calls named.  pct_graph_end fails
 * (and discards the capture) when a captured call was not capturable.
 * pct_graph_destroy frees the graph. */
typedef struct pct_graph_s* pct_graph;
pct_status pct_graph_begin(void* stream);
pct_status pct_graph_end(void* stream, pct_graph* out);
pct_status pct_graph_launch(pct_graph graph, void* stream);
pct_status pct_graph_destroy(pct_graph graph);

/* pct_tomogram_extent for every item, in one launch and one stream
 * synchronisation.  d_xyz holds n_total points; item i uses points
 * [xyz_offset, xyz_offset + n_points).  Writes h_items[i].extent and the
 * packing offsets; *total_cells (sum of N nx ny) and *total_slices (sum of
 * N) size the packed outputs. */
pct_status pct_tomogram_extent_batched(const float* d_xyz, int64_t n_total, pct_item* h_items, int32_t n_items,
                                       int64_t* total_cells, int64_t* total_slices, void* d_ws, size_t ws_bytes,
                                       void* stream);

/* pct_build_tomogram for every item in one launch per stage (binning, scan,
 * scatter, tile reduce).  Outputs are packed: item i at out_offset.  Point
 * ids index d_xyz.  flags: PCT_DESCRIPTORS_RESIDENT. */
pct_status pct_build_tomogram_batched(const float* d_xyz, int64_t n_total, const pct_item* h_items, int32_t n_items,
                                      float* d_ground, float* d_ceil, int32_t* d_arg_ground, int32_t* d_arg_ceil,
                                      int32_t flags, void* d_ws, size_t ws_bytes, void* stream);

/* pct_eval_traversability for every (item, robot) pair in one launch per
 * stage.  d_cost is [n_robots][total_cells] (robot r, item i at
 * r * total_cells + out_offset), d_keep [n_robots][total_slices] (nullable).
 * flags: PCT_DESCRIPTORS_RESIDENT. */
pct_status pct_eval_traversability_batched(const float* d_ground, const float* d_ceil, const pct_item* h_items,
                                           int32_t n_items, const pct_robot* h_robots, int32_t n_robots,
                                           float* d_cost, uint8_t* d_keep, int32_t flags, void* d_ws,
                                           size_t ws_bytes, void* stream);

/* One timing of pct_autotune_batched: a construction tile height or an
 * evaluation strip shape tried on the items of one size class. */
typedef struct {
    int32_t stage;     /* 0: construction tile height, 1: evaluation strip shape */
    int32_t class_x;   /* ceil(log2 nx) of the class's items */
    int32_t class_y;   /* ceil(log2 ny) */
    int32_t radius;    /* the evaluation's inflation radius R in cells; -1 for the construction */
    int32_t rows;      /* construction: tile height in cells; evaluation: strip rows (0: the default shape) */
    int32_t waves;     /* evaluation: wavefronts per workgroup (1 or PCT_STRIP_WAVES); 0 for the construction */
    int32_t n_items;   /* items in the class */
    int32_t chosen;    /* 1 for the choice recorded for the class */
    float ms;          /* mean time of one batched call over the class's items */
} pct_tune_entry;

/* Tile shapes for batches of submaps (the performance tuning of the batched
 * Sec. III-A construction and Sec. III-B evaluation; results do not depend
 * on them).  Items with slices are grouped into size classes
 * (ceil(log2 nx), ceil(log2 ny), and R for h_robot); for each class the
 * construction is timed at tile heights 2, 4 and 8 (those not below the
 * default) and the evaluation (without slice test) at the default strip
 * shape and at 32, 64, 128 and 256 rows with 1 or PCT_STRIP_WAVES
 * wavefronts, each as a batch of only that class's items, and the fastest
 * is recorded for the class.  Later batched calls use the recorded shapes
 * (the construction never with more tiles than the default, so workspaces
 * sized before tuning still suffice).  h_items must carry extents
 * (pct_tomogram_extent_batched); d_xyz as for pct_build_tomogram_batched.
 * The call allocates and frees its own device buffers and synchronises
 * `stream`; the caller's workspaces are not touched, but their resident
 * descriptor tables no longer match tuned classes: the next batched call on
 * them must upload (no PCT_DESCRIPTORS_RESIDENT), and graphs captured before
 * tuning keep replaying the shapes they captured.  Up to n_max timings go to
 * h_out; *h_count = their number. */
pct_status pct_autotune_batched(const float* d_xyz, int64_t n_total, const pct_item* h_items, int32_t n_items,
                                const pct_robot* h_robot, pct_tune_entry* h_out, int32_t n_max, int32_t* h_count,
                                void* stream);

/* The tuning tables (single-map strip shapes of pct_autotune_traversability
 * and pct_autotune_set_traversability, and the size-class tables of
 * pct_autotune_batched) as a text file, one record a line, each tagged with
 * the current device's architecture name.  pct_autotune_load adds the
 * records of the current architecture to the tables (others are skipped;
 * *n_applied, nullable, counts the added ones) and applies nothing if any
 * line is malformed (PCT_ERR_ARG naming the line). */
pct_status pct_autotune_save(const char* path);
pct_status pct_autotune_load(const char* path, int32_t* n_applied);

/* Workspace bytes for pct_trajectory_cost_multi with n_profiles profiles. */
size_t pct_trajectory_multi_workspace_bytes(int32_t n_profiles);

/* Many robot profiles on one map in one launch (Sec. III-B evaluation with
 * the Sec. III-E / Eq. (11) cost and height terms).  Profile p samples its
 * own trajectories as pct_sample_cost_fwd does with that profile's c^T and,
 * given d_gf, differentiates them as pct_trajectory_cost_bwd does.  No cost
 * map is formed: c^T is evaluated by Eqs. (1)-(6) only at the four bilinear
 * corners of each waypoint, with the same FP32 operations as
 * pct_eval_traversability, so d_f and d_gwp equal the per-profile path's
 * bit for bit.
 * h_robots: host [n_profiles]; d_wp: float32 [n_profiles][n_traj][n_wp][3];
 * d_wp_slice: int32 [n_profiles][n_traj][n_wp]; d_f: float32
 * [n_profiles][n_traj], overwritten.  d_gf: float32 [n_profiles][n_traj] or
 * null (values only).  With d_gf, d_gwp [n_profiles][n_traj][n_wp][3] is
 * required and overwritten, and the nullable d_gground, d_gceil
 * [N][ny][nx] and d_gz [n_points] receive sums over all profiles
 * (zero-filled first unless PCT_ACCUMULATE); d_gz needs d_arg_ground and
 * d_arg_ceil.  flags: PCT_ACCUMULATE, PCT_DESCRIPTORS_RESIDENT (the profile
 * table is already in the workspace from a call with the same profiles). */
pct_status pct_trajectory_cost_multi(const float* d_ground, const float* d_ceil, const int32_t* d_arg_ground,
                                     const int32_t* d_arg_ceil, const pct_grid* grid, const pct_extent* extent,
                                     const pct_robot* h_robots, int32_t n_profiles, float w_z, const float* d_wp,
                                     const int32_t* d_wp_slice, int32_t n_traj, int32_t n_wp, const float* d_gf,
                                     float* d_f, float* d_gwp, float* d_gground, float* d_gceil, int64_t n_points,
                                     float* d_gz, int32_t flags, void* d_ws, size_t ws_bytes, void* stream);

/* ---- path search through the slices (Sec. III-D) ----
 * The graph of the section: nodes are the cells of n_layers chosen slices
 * (normally those the slice test keeps, in increasing order); a node links
 * to its eight planar neighbours on its layer.  Moving onto node v costs
 * c^N(v) + step length (1 or sqrt 2, in cells), where c^N is the least c^T
 * over v and the adjacent layers whose ground elevation at the cell is equal
 * (the same point in space); nodes with c^N >= c^B cannot be entered.  A
 * node whose adjacent layer has the same ground and a strictly lower c^T is
 * a gateway to it (no cost), upwards and downwards.
 * The library computes every node's least path cost from the start (the
 * cost an A* search with the diagonal-distance heuristic ends with) and
 * reads a least-cost path back from it.  Distances are FP64: each edge adds
 * (double)c^N + step in one rounding each, so the result is the least
 * rounded path sum, independent of the order of the parallel work. */

/* Workspace bytes for pct_plan_distance / pct_plan_path on an nx x ny map
 * with n_layers layers. */
size_t pct_plan_workspace_bytes(int32_t nx, int32_t ny, int32_t n_layers);

/* Distances from the start node (sx, sy, layer s_layer) to every node.
 * d_cost, d_ground: float32 [N][ny][nx] (c^T of one robot, e^G); c^B is
 * h_robot->c_barrier.  h_layers: host [n_layers], strictly increasing slice
 * indices in [0, N).  band: width of the distance band whose tiles one
 * round processes (0: the default, 16384); it changes the amount of work,
 * never the result.  d_dist: float64 [n_layers][ny][nx], overwritten
 * (+inf: unreachable).  The workspace keeps the node costs and gateways for
 * pct_plan_path.  Synchronous (one host read-back per round of tiles);
 * *h_rounds (nullable) receives the round count, *h_tiles (nullable) the
 * tiles processed.  The start may itself be a barrier node. */
pct_status pct_plan_distance(const float* d_cost, const float* d_ground, const pct_grid* grid,
                             const pct_extent* extent, const pct_robot* h_robot, const int32_t* h_layers,
                             int32_t n_layers, int32_t sx, int32_t sy, int32_t s_layer, double band, double* d_dist,
                             void* d_ws, size_t ws_bytes, int32_t* h_rounds, int64_t* h_tiles, void* stream);

/* A single query, as the section's A* answers it: pct_plan_distance that
 * stops once the goal's distance is final, i.e. when the least key of the
 * tiles still active (a lower bound on every label they can still lower)
 * exceeds the goal's label.  Then every label below *h_settled is final
 * (equal to pct_plan_distance's), the goal's included; the others are upper
 * bounds.  *h_goal_dist: the goal's least path cost (+inf: unreachable,
 * after a complete search); *h_settled = +inf when the search ran to the
 * end.  pct_plan_path reads the goal's path back from d_dist unchanged.
 * Arguments otherwise as pct_plan_distance; synchronous. */
pct_status pct_plan_query(const float* d_cost, const float* d_ground, const pct_grid* grid, const pct_extent* extent,
                          const pct_robot* h_robot, const int32_t* h_layers, int32_t n_layers, int32_t sx, int32_t sy,
                          int32_t s_layer, int32_t gx, int32_t gy, int32_t g_layer, double band, double* d_dist,
                          void* d_ws, size_t ws_bytes, double* h_goal_dist, double* h_settled, int32_t* h_rounds,
                          int64_t* h_tiles, void* stream);

/* A least-cost path from the start to the goal (gx, gy, layer g_layer),
 * read back from d_dist of the preceding pct_plan_distance call with the
 * same workspace: from the goal, the first predecessor whose distance plus
 * the edge cost equals the node's (gateway from below, gateway from above,
 * then the planar neighbours in row-major order of (dy, dx)), up to the
 * start.  d_path: int32 [max_len][3] (x, y, slice index), start first.
 * *h_len = node count, 0 if the goal is unreachable.  PCT_ERR_CAPACITY if
 * the path has more than max_len nodes, PCT_ERR_ARG if d_dist is not a
 * distance field of this graph.  Synchronous. */
pct_status pct_plan_path(const double* d_dist, const pct_grid* grid, int32_t n_layers, int32_t sx, int32_t sy,
                         int32_t s_layer, int32_t gx, int32_t gy, int32_t g_layer, int32_t* d_path, int32_t max_len,
                         int32_t* h_len, void* d_ws, size_t ws_bytes, void* stream);

/* ---- sparse storage of the simplified tomogram (Sec. III-C) ----
 * Only the unique cells of the kept slices: for kept slice k, with p the
 * last kept slice below it (none for the first), cell c is unique when
 * c^T_k < c^B, and (no p, or e^G_k > e^G_p, or c^T_k < c^T_p), and (k is the
 * last slice, or e^G_{k+1} > e^G_k, or c^T_k < c^T_{k+1}) - Eqs. (8)-(9), the
 * cells that make a slice kept. */

/* Workspace bytes for pct_unique_cells on this grid and extent. */
size_t pct_unique_workspace_bytes(const pct_grid* grid, const pct_extent* extent);

/* The unique cells of the kept slices, slice after slice in increasing
 * order, cells in raster order (index y * nx + x): d_cell int32, and
 * d_ground_out, d_ceil_out, d_cost_out float32 (e^G, e^C, c^T of the cell
 * in its slice), each [capacity].  d_ground, d_ceil, d_cost: float32
 * [N][ny][nx] of one robot; d_keep: uint8 [N] (the slice test's keep flags;
 * copied to the host).  *h_count = the number of unique cells; h_slice_off
 * (host [N+1], nullable): slice k's cells are h_slice_off[k] ..
 * h_slice_off[k+1] (empty for removed slices).  With d_cell null only the
 * count (and offsets) are produced; PCT_ERR_CAPACITY if d_cell is given and
 * the count exceeds capacity (*h_count is still set).  Synchronous. */
pct_status pct_unique_cells(const float* d_ground, const float* d_ceil, const float* d_cost, const uint8_t* d_keep,
                            const pct_grid* grid, const pct_extent* extent, const pct_robot* h_robot,
                            int64_t capacity, int32_t* d_cell, float* d_ground_out, float* d_ceil_out,
                            float* d_cost_out, int64_t* h_slice_off, int64_t* h_count, void* d_ws, size_t ws_bytes,
                            void* stream);

/* ---- incremental updates for streaming scans ---- */

/* Workspace bytes for pct_tomogram_insert of n points. */
size_t pct_insert_workspace_bytes(int64_t n, const pct_grid* grid);

/* Adds n points (ids id_base .. id_base + n - 1) to an existing tomogram in
 * place (Sec. III-A applied to the union): every cell-slice takes the higher
 * ground and the lower ceiling of its stored value and the new points,
 * equal heights keeping the lower point id, so the result equals a build of
 * the union of the old and new points (with the new ids) bit for bit.  The
 * planes must not change: PCT_ERR_ARG if an in-grid new point lies below
 * z_min or at or above the top plane (rebuild instead); nothing is written
 * then.  extent (in/out): n_used, n_dropped and z_max are updated.  d_ground,
 * d_ceil, d_arg_ground, d_arg_ceil: as written by pct_build_tomogram (the
 * ids nullable together).  h_bbox (host [4], nullable): the cells the new
 * points fell in, {x_min, y_min, x_max, y_max} (x_max < x_min when none).
 * Synchronous.  Only tiles that receive points are read and written. */
pct_status pct_tomogram_insert(const float* d_xyz, int64_t n, int32_t id_base, const pct_grid* grid,
                               pct_extent* extent, float* d_ground, float* d_ceil, int32_t* d_arg_ground,
                               int32_t* d_arg_ceil, int32_t* h_bbox, void* d_ws, size_t ws_bytes, void* stream);

/* pct_eval_traversability for one robot on the cells [x0, x1) x [y0, y1)
 * of every slice only (clamped to the grid); the other cells of d_cost are
 * left as they are.  The window's values are those of a whole-map
 * evaluation (the same FP32 operations; neighbours outside the window are
 * read).  After an insertion, the cells whose c^T can change are the new
 * points' cells grown by the inflation radius plus 2 (the stencil and the
 * patch).  With d_keep (uint8 [N]) the slice test then runs on the whole
 * map (workspace as for pct_eval_traversability with one robot). */
pct_status pct_eval_traversability_window(const float* d_ground, const float* d_ceil, const pct_grid* grid,
                                          const pct_extent* extent, const pct_robot* h_robot, int32_t x0, int32_t y0,
                                          int32_t x1, int32_t y1, float* d_cost, uint8_t* d_keep, void* d_ws,
                                          size_t ws_bytes, void* stream);

/* ---- trajectory optimisation (Sec. III-E, Eq. (10)) ---- */

/* Weights and limits of the penalty form of Eq. (10).  Per sample, with G,
 * C, H the bilinear e^G, c^T, e^C of the piece's slice at the sample's (x, y):
 *     w_z (z - G - d_ref)^2 + w_c max(0, C - c_safe)^3
 *   + w_v max(0, |v|^2 - v_max^2)^3 + w_a max(0, |a|^2 - a_max^2)^3
 *   + w_h max(0, G + d_min - z)^3 + w_h max(0, z - H)^3,
 * summed over K + 1 evenly spaced times per piece with trapezoid weights;
 * the objective adds the jerk effort and w_T times the total duration.  All
 * values finite, weights >= 0, v_max and a_max > 0, 1 <= samples <=
 * PCT_MAX_TRAJ_SAMPLES. */
typedef struct {
    float w_z, w_c, w_v, w_a, w_h, w_T;
    float c_safe, v_max, a_max;
    float d_ref, d_min;
    int32_t samples;
} pct_traj_params;

/* Objective, gradient and spline of n_traj trajectories of n_pieces quintic
 * pieces (1 <= n_pieces <= PCT_MAX_PIECES), FP64 (Sec. III-E, Eq. (10)).
 * Each trajectory is the minimum-jerk spline (continuous in derivatives
 * 0..4) through its interior waypoints with durations T_i = exp(tau_i),
 * between fixed start and goal states.
 * d_cost, d_ground, d_ceil: float32 [N][ny][nx], c^T of one robot, e^G, e^C.
 * d_bound: float64 [n][2][3][3], start then goal, rows position, velocity,
 * acceleration.  d_slice: int32 [n][M], the slice each piece is evaluated
 * on (outside [0, N): no map terms).  d_knots: float64 [n][M-1][3] interior
 * waypoints (null when M = 1); d_tau: float64 [n][M].
 * d_phi: float64 [n] objective (+inf where a duration or sample is not
 * finite; the gradients are then NaN).  d_gknots [n][M-1][3], d_gtau [n][M]:
 * its gradient.  d_coef (nullable): float64 [n][M][6][3], the monomial
 * coefficients of each piece in its local time t in [0, T_i].
 * Asynchronous on the stream; no workspace. */
pct_status pct_traj_eval(const float* d_cost, const float* d_ground, const float* d_ceil, const pct_grid* grid,
                         const pct_extent* extent, const pct_traj_params* h_prm, int32_t n_traj, int32_t n_pieces,
                         const double* d_bound, const int32_t* d_slice, const double* d_knots, const double* d_tau,
                         double* d_phi, double* d_gknots, double* d_gtau, double* d_coef, void* stream);

/* iters iterations of gradient descent with Armijo backtracking on the
 * objective of pct_traj_eval, per trajectory, from d_knots / d_tau (updated
 * in place).  The step starts at `step` (> 0, finite), is halved until the
 * objective drops by at least 1e-4 * step * |gradient|^2 (at most 30
 * times; a failed search ends that trajectory's run) and is doubled after
 * each accepted iteration.  d_phi: the final objective; d_iters (nullable):
 * int32 [n], the iterations accepted.  Asynchronous on the stream. */
pct_status pct_traj_optimize(const float* d_cost, const float* d_ground, const float* d_ceil, const pct_grid* grid,
                             const pct_extent* extent, const pct_traj_params* h_prm, int32_t n_traj,
                             int32_t n_pieces, const double* d_bound, const int32_t* d_slice, double* d_knots,
                             double* d_tau, int32_t iters, double step, double* d_phi, int32_t* d_iters,
                             void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PCT_H */
