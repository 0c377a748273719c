// Path search through the tomogram slices (Sec. III-D) on the GPU.
//
// The graph: nodes are the cells of L layers (chosen slices, normally the
// ones the simplification keeps); a node links to its eight planar
// neighbours on its layer; moving onto node v costs c^N(v) + step length
// (1 or sqrt 2 cells), where c^N is the least c^T over the node and the
// adjacent layers with the same ground elevation, and a node with
// c^N >= c^B cannot be entered; a layer whose ground is equal and whose c^T
// is strictly lower is reached at no cost (a gateway, upwards or downwards).
//
// Instead of a sequential A* the library computes every node's
// shortest-path distance from the start with a parallel label-correcting
// method, then reads a least-cost path back from the distances.  A* with its
// admissible, consistent heuristic ends with the same least cost.
//
// Distances are FP64.  Each edge relaxation is one rounding of
// dist(u) + (c^N(v) + step) (the edge cost itself one rounding of the FP32
// node cost plus the step); rounding is monotone and every cycle contains a
// planar step (gateways only lead to strictly cheaper layers), so every
// order of relaxations ends at the same least fixed point - the least
// rounded path sum - which is also what Dijkstra's algorithm computes.
//
// Tiles of 64 x 64 cells of one layer are the unit of work.  A round
// processes every active tile: one wavefront loads the tile's distances and
// a one-cell halo into LDS, takes what gateways offer from the adjacent
// layers, then sweeps the tile left-to-right, right-to-left, top-to-bottom
// and bottom-to-top (a lane per row or column, each step relaxing the edges
// from the previous column or row) until a full set of sweeps changes
// nothing.  Improved cells are written back; a tile whose border cells
// improved activates its planar neighbours, one whose gateway cells improved
// activates the tile of the adjacent layer.  Rounds repeat until no tile is
// active.
#include <math.h>

#include "pct_internal.h"

namespace pct {

namespace {

constexpr int kPT = 64;            // tile side, cells
constexpr int kPS = kPT + 3;       // LDS row stride of the distance tile (doubles; conflict-free columns)
constexpr int kCS = kPT + 1;       // LDS row stride of the node-cost tile (floats)
constexpr double kSqrt2 = 1.4142135623730951;   // sqrt(2) rounded to double

// gateway bits of a node (l, cell)
constexpr unsigned kInFromBelow = 1;   // edge (l-1) -> l
constexpr unsigned kInFromAbove = 2;   // edge (l+1) -> l
constexpr unsigned kOutUp = 4;         // edge l -> (l+1)
constexpr unsigned kOutDown = 8;       // edge l -> (l-1)

struct PlanGeom {
    int nx, ny, L;
    int ntx, nty;
    long long plane;
};

PlanGeom make_plan_geom(int nx, int ny, int L) {
    PlanGeom g;
    g.nx = nx;
    g.ny = ny;
    g.L = L;
    g.ntx = (nx + kPT - 1) / kPT;
    g.nty = (ny + kPT - 1) / kPT;
    g.plane = (long long)nx * ny;
    return g;
}

// Node cost (+inf where the node cannot be entered) and gateway bits.
__global__ __launch_bounds__(256) void k_plan_prep(const float* __restrict__ cost, const float* __restrict__ ground,
                                                   const int* __restrict__ layers, PlanGeom g, float cB,
                                                   float* __restrict__ cn, uint8_t* __restrict__ gw) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.plane * g.L) return;
    const int l = (int)(i / g.plane);
    const long long c = i - (long long)l * g.plane;
    const long long o = (long long)layers[l] * g.plane + c;
    const float e = ground[o], t = cost[o];
    float n = t;
    unsigned bits = 0;
    if (l + 1 < g.L) {
        const long long a = (long long)layers[l + 1] * g.plane + c;
        const float ea = ground[a], ta = cost[a];
        if (ea == e) {
            n = fminf(n, ta);
            if (ta < t) bits |= kOutUp;
            if (t < ta) bits |= kInFromAbove;
        }
    }
    if (l > 0) {
        const long long b = (long long)layers[l - 1] * g.plane + c;
        const float eb = ground[b], tb = cost[b];
        if (eb == e) {
            n = fminf(n, tb);
            if (tb < t) bits |= kOutDown;
            if (t < tb) bits |= kInFromBelow;
        }
    }
    cn[i] = n < cB ? n : INFINITY;
    gw[i] = (uint8_t)bits;
}

__global__ __launch_bounds__(256) void k_plan_init(double* __restrict__ dist, long long n, long long s,
                                                   unsigned* __restrict__ flag, int n_tiles, int t0) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dist[i] = i == s ? 0.0 : INFINITY;
    if (i < n_tiles) flag[i] = i == t0 ? 1u : 0u;
}

// Lane i receives lane i-1's (i+1's) value; the edge lane gets 0.
__device__ __forceinline__ double from_lane_below(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x138, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_lane_above(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Relaxation of one direction over the tile in LDS.  Lane q walks the
// q-th row (horizontal sweeps) or column (vertical sweeps); at each step it
// relaxes the node's three in-edges from the previous step: its own
// previous node and the diagonal ones, which are the neighbour lanes'
// previous nodes (taken from their registers, so the lanes advance in
// lockstep) or, for the edge lanes, halo cells.  A lane touches only its
// own row or column of the tile in LDS during a sweep.
template <bool VERT, bool REV>
__device__ __forceinline__ bool sweep(double* sd, const float* scn, int q) {
    // LDS coordinates: node (r, c) of the tile is sd[(r + 1) * kPS + c + 1]
    bool changed = false;
    const int s0 = REV ? kPT : -1;   // halo position before the first step
    double prev = VERT ? sd[(s0 + 1) * kPS + q + 1] : sd[(q + 1) * kPS + s0 + 1];
#pragma unroll 4
    for (int i = 0; i < kPT; ++i) {
        const int s = REV ? kPT - 1 - i : i;      // step along the sweep
        const int sp = REV ? s + 1 : s - 1;       // previous step
        double* me = VERT ? &sd[(s + 1) * kPS + q + 1] : &sd[(q + 1) * kPS + s + 1];
        const float c = VERT ? scn[s * kCS + q] : scn[q * kCS + s];
        // halo nodes beside lanes 0 and 63 at the previous step
        const double h0 = VERT ? sd[(sp + 1) * kPS] : sd[sp + 1];
        const double h1 = VERT ? sd[(sp + 1) * kPS + kPT + 1] : sd[(kPT + 1) * kPS + sp + 1];
        double a = from_lane_below(prev), b = from_lane_above(prev);
        if (q == 0) a = h0;
        if (q == kPT - 1) b = h1;
        const double ws = (double)c + 1.0, wd = (double)c + kSqrt2;
        const double cand = fmin(prev + ws, fmin(a + wd, b + wd));
        const double old = *me;
        if (cand < old) {
            *me = cand;
            changed = true;
            prev = cand;
        } else {
            prev = old;
        }
    }
    return changed;
}

__global__ __launch_bounds__(64) void k_plan_relax(PlanGeom g, const float* __restrict__ cn,
                                                   const uint8_t* __restrict__ gw, double* __restrict__ dist,
                                                   const unsigned* __restrict__ list, unsigned* __restrict__ flag) {
    __shared__ double sd[(kPT + 2) * kPS];
    __shared__ float scn[kPT * kCS];
    const int q = threadIdx.x;
    const int t = (int)list[blockIdx.x];
    const int tpl = g.ntx * g.nty;
    const int l = t / tpl, tt = t - l * tpl;
    const int ty = tt / g.ntx, tx = tt - ty * g.ntx;
    const int x0 = tx * kPT, y0 = ty * kPT;
    const long long lo = (long long)l * g.plane;

    // distances with a one-cell halo (+inf outside the grid), node costs
    for (int r = 0; r < kPT + 2; ++r) {
        const int y = y0 - 1 + r;
        for (int c = q; c < kPT + 2; c += 64) {
            const int x = x0 - 1 + c;
            const bool in = x >= 0 && y >= 0 && x < g.nx && y < g.ny;
            sd[r * kPS + c] = in ? dist[lo + (long long)y * g.nx + x] : INFINITY;
        }
    }
    __syncthreads();   // lane q now updates column q + 1, written by lane q + 1
    for (int r = 0; r < kPT; ++r) {
        const int y = y0 + r, x = x0 + q;
        const bool in = x < g.nx && y < g.ny;
        float c = INFINITY;
        if (in) {
            const long long i = lo + (long long)y * g.nx + x;
            c = cn[i];
            // gateways into this node: the adjacent layer's distance, at no cost
            const unsigned b = gw[i];
            double d = sd[(r + 1) * kPS + q + 1];
            if (b & kInFromBelow) d = fmin(d, dist[i - g.plane] + 0.0);
            if (b & kInFromAbove) d = fmin(d, dist[i + g.plane] + 0.0);
            sd[(r + 1) * kPS + q + 1] = d;
        }
        scn[r * kCS + q] = c;
    }
    __syncthreads();

    for (;;) {
        bool ch = sweep<false, false>(sd, scn, q);
        __syncthreads();
        ch |= sweep<false, true>(sd, scn, q);
        __syncthreads();
        ch |= sweep<true, false>(sd, scn, q);
        __syncthreads();
        ch |= sweep<true, true>(sd, scn, q);
        __syncthreads();
        if (!__ballot(ch)) break;
    }

    // write back improved nodes; note which neighbours must look again
    bool nb_up = false, nb_dn = false, nb_l = false, nb_r = false;
    bool c_ul = false, c_ur = false, c_dl = false, c_dr = false, g_up = false, g_dn = false;
    const int w = min(kPT, g.nx - x0), h = min(kPT, g.ny - y0);
    if (q < w) {
        for (int r = 0; r < h; ++r) {
            const long long i = lo + (long long)(y0 + r) * g.nx + x0 + q;
            const double nd = sd[(r + 1) * kPS + q + 1];
            if (nd < dist[i]) {
                dist[i] = nd;
                nb_up |= r == 0;
                nb_dn |= r == h - 1;
                nb_l |= q == 0;
                nb_r |= q == w - 1;
                c_ul |= r == 0 && q == 0;
                c_ur |= r == 0 && q == w - 1;
                c_dl |= r == h - 1 && q == 0;
                c_dr |= r == h - 1 && q == w - 1;
                const unsigned b = gw[i];
                g_up |= (b & kOutUp) != 0;
                g_dn |= (b & kOutDown) != 0;
            }
        }
    }
    const unsigned long long m_up = __ballot(nb_up), m_dn = __ballot(nb_dn), m_l = __ballot(nb_l),
                             m_r = __ballot(nb_r), m_ul = __ballot(c_ul), m_ur = __ballot(c_ur),
                             m_dl = __ballot(c_dl), m_dr = __ballot(c_dr), m_gu = __ballot(g_up),
                             m_gd = __ballot(g_dn);
    if (q == 0) {
        auto act = [&](int ll, int yy, int xx) {
            if (ll < 0 || ll >= g.L || yy < 0 || yy >= g.nty || xx < 0 || xx >= g.ntx) return;
            flag[(ll * g.nty + yy) * g.ntx + xx] = 1u;
        };
        if (m_up) act(l, ty - 1, tx);
        if (m_dn) act(l, ty + 1, tx);
        if (m_l) act(l, ty, tx - 1);
        if (m_r) act(l, ty, tx + 1);
        if (m_ul) act(l, ty - 1, tx - 1);
        if (m_ur) act(l, ty - 1, tx + 1);
        if (m_dl) act(l, ty + 1, tx - 1);
        if (m_dr) act(l, ty + 1, tx + 1);
        if (m_gu) act(l + 1, ty, tx);
        if (m_gd) act(l - 1, ty, tx);
    }
}

// Active flags -> next worklist (flags cleared); count[0] must be zero.
__global__ __launch_bounds__(256) void k_plan_compact(unsigned* __restrict__ flag, int n_tiles,
                                                      unsigned* __restrict__ list, unsigned* __restrict__ count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool on = t < n_tiles && flag[t] != 0u;
    const unsigned long long m = __ballot(on);
    const int lane = threadIdx.x & 63;
    unsigned base = 0;
    if (lane == 0 && m) base = atomicAdd(count, (unsigned)__popcll(m));
    base = __shfl(base, 0, 64);
    if (on) {
        flag[t] = 0u;
        list[base + __popcll(m & ((1ull << lane) - 1ull))] = (unsigned)t;
    }
}

__global__ void k_plan_zero1(unsigned* p) { *p = 0u; }

// One wavefront walks back from the goal: lanes 0..9 test the candidate
// predecessors (gateway from below, gateway from above, the eight planar
// neighbours in row-major order of (dy, dx)); the first that matches is
// taken.  out[0] receives the node count (0: goal unreachable, -1: not a
// distance field, -2: more than max_len nodes); path rows are written goal
// first and reversed at the end.
__global__ __launch_bounds__(64) void k_plan_path(PlanGeom g, const float* __restrict__ cn,
                                                  const uint8_t* __restrict__ gw, const double* __restrict__ dist,
                                                  const int* __restrict__ layers, int sx, int sy, int sl, int gx,
                                                  int gy, int gl, int* __restrict__ path, int max_len,
                                                  int* __restrict__ out) {
    const int lane = threadIdx.x;
    long long v = (long long)gl * g.plane + (long long)gy * g.nx + gx;
    const long long s = (long long)sl * g.plane + (long long)sy * g.nx + sx;
    int len = 0, status = 0;
    if (dist[v] < INFINITY) {
        for (;;) {
            if (len >= max_len) {
                status = -2;
                break;
            }
            const int l = (int)(v / g.plane);
            const long long c = v - (long long)l * g.plane;
            const int x = (int)(c % g.nx), y = (int)(c / g.nx);
            if (lane == 0) {
                path[3 * len] = x;
                path[3 * len + 1] = y;
                path[3 * len + 2] = layers[l];
            }
            ++len;
            if (v == s) break;
            const double dv = dist[v];
            long long u = -1;
            bool ok = false;
            if (lane < 2) {
                const int m = lane == 0 ? l - 1 : l + 1;
                if (m >= 0 && m < g.L) {
                    const long long uu = (long long)m * g.plane + c;
                    const unsigned bit = lane == 0 ? kOutUp : kOutDown;
                    if ((gw[uu] & bit) && dist[uu] + 0.0 == dv) {
                        u = uu;
                        ok = true;
                    }
                }
            } else if (lane < 10) {
                const int e = lane - 2;
                const int dy = e < 3 ? -1 : (e < 5 ? 0 : 1);
                const int dx = e < 3 ? e - 1 : (e < 5 ? (e == 3 ? -1 : 1) : e - 6);
                const int x2 = x + dx, y2 = y + dy;
                const float cv = cn[v];
                if (x2 >= 0 && y2 >= 0 && x2 < g.nx && y2 < g.ny && cv < INFINITY) {
                    const long long uu = (long long)l * g.plane + (long long)y2 * g.nx + x2;
                    const double wgt = (double)cv + ((dx != 0 && dy != 0) ? kSqrt2 : 1.0);
                    if (dist[uu] + wgt == dv) {
                        u = uu;
                        ok = true;
                    }
                }
            }
            const unsigned long long m = __ballot(ok);
            if (!m) {
                status = -1;
                break;
            }
            const int first = __ffsll((long long)m) - 1;
            v = __shfl(u, first, 64);
        }
    }
    if (status == 0) {
        // reverse rows: start first
        for (int a = lane; a < len / 2; a += 64) {
            const int b = len - 1 - a;
            for (int k = 0; k < 3; ++k) {
                const int tmp = path[3 * a + k];
                path[3 * a + k] = path[3 * b + k];
                path[3 * b + k] = tmp;
            }
        }
    }
    if (lane == 0) out[0] = status == 0 ? len : status;
}

struct PlanWs {
    float* cn;
    uint8_t* gw;
    unsigned* flag;
    unsigned* list[2];
    unsigned* count;   // [2]
    int* layers;
    int* out;
};

size_t plan_ws_layout(const PlanGeom& g, PlanWs* w, void* base) {
    const long long nn = g.plane * g.L;
    const int nt = g.ntx * g.nty * g.L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return (char*)base + o;
    };
    PlanWs ws;
    ws.cn = (float*)take(sizeof(float) * (size_t)nn);
    ws.gw = (uint8_t*)take((size_t)nn);
    ws.flag = (unsigned*)take(sizeof(unsigned) * (size_t)nt);
    ws.list[0] = (unsigned*)take(sizeof(unsigned) * (size_t)nt);
    ws.list[1] = (unsigned*)take(sizeof(unsigned) * (size_t)nt);
    ws.count = (unsigned*)take(sizeof(unsigned) * 2);
    ws.layers = (int*)take(sizeof(int) * (size_t)g.L);
    ws.out = (int*)take(sizeof(int) * 4);
    if (w) *w = ws;
    return off;
}

}  // namespace

size_t plan_ws_bytes(int nx, int ny, int L) { return plan_ws_layout(make_plan_geom(nx, ny, L), nullptr, nullptr); }

pct_status launch_plan(const float* cost, const float* ground, int nx, int ny, const int* h_layers, int L, float cB,
                       int sx, int sy, int sl, double* dist, void* ws_base, int* h_rounds, long long* h_tiles,
                       hipStream_t s) {
    const PlanGeom g = make_plan_geom(nx, ny, L);
    PlanWs w;
    plan_ws_layout(g, &w, ws_base);
    const long long nn = g.plane * L;
    const int nt = g.ntx * g.nty * L;
    PCT_HIP(hipMemcpyAsync(w.layers, h_layers, sizeof(int) * (size_t)L, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_plan_prep, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, cost, ground, w.layers, g, cB,
                       w.cn, w.gw);
    PCT_LAUNCH_CHECK();
    const long long src = (long long)sl * g.plane + (long long)sy * nx + sx;
    const int t0 = (sl * g.nty + sy / kPT) * g.ntx + sx / kPT;
    const long long ni = std::max<long long>(nn, nt);
    hipLaunchKernelGGL(k_plan_init, dim3((unsigned)((ni + 255) / 256)), dim3(256), 0, s, dist, nn, src, w.flag, nt, t0);
    PCT_LAUNCH_CHECK();
    int rounds = 0;
    long long tiles = 0;
    unsigned n_active = 0;
    for (int cur = 0;; cur ^= 1) {
        // flags -> list[cur]
        hipLaunchKernelGGL(k_plan_zero1, dim3(1), dim3(1), 0, s, w.count + cur);
        hipLaunchKernelGGL(k_plan_compact, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, w.flag, nt,
                           w.list[cur], w.count + cur);
        PCT_LAUNCH_CHECK();
        PCT_HIP(hipMemcpyAsync(&n_active, w.count + cur, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        PCT_HIP(hipStreamSynchronize(s));
        if (n_active == 0) break;
        hipLaunchKernelGGL(k_plan_relax, dim3(n_active), dim3(64), 0, s, g, w.cn, w.gw, dist, w.list[cur], w.flag);
        PCT_LAUNCH_CHECK();
        ++rounds;
        tiles += n_active;
    }
    if (h_rounds) *h_rounds = rounds;
    if (h_tiles) *h_tiles = tiles;
    return PCT_OK;
}

pct_status launch_plan_path(const double* dist, int nx, int ny, int L, int sx, int sy, int sl, int gx, int gy, int gl,
                            int* path, int max_len, void* ws_base, int* h_len, hipStream_t s) {
    const PlanGeom g = make_plan_geom(nx, ny, L);
    PlanWs w;
    plan_ws_layout(g, &w, ws_base);
    hipLaunchKernelGGL(k_plan_path, dim3(1), dim3(64), 0, s, g, w.cn, w.gw, dist, w.layers, sx, sy, sl, gx, gy, gl,
                       path, max_len, w.out);
    PCT_LAUNCH_CHECK();
    int out = 0;
    PCT_HIP(hipMemcpyAsync(&out, w.out, sizeof(int), hipMemcpyDeviceToHost, s));
    PCT_HIP(hipStreamSynchronize(s));
    *h_len = out;
    return PCT_OK;
}

}  // namespace pct
