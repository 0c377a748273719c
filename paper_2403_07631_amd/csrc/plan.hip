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
#include <string.h>

#include "pct_internal.h"
#include "plan_internal.h"

namespace pct {

namespace {

constexpr int kPT = 64;            // tile side, cells
constexpr int kPS = kPT + 1;       // LDS row stride of the distance tile (doubles)
constexpr int kCS = kPT + 1;       // LDS row stride of the node-cost tile (floats)

__device__ __forceinline__ int cidx(int r, int c) { return r * kCS + c; }
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
                                                   unsigned* __restrict__ flag, unsigned long long* __restrict__ key,
                                                   int n_tiles, int t0) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dist[i] = INFINITY;   // the start takes 0 on its tile's first visit
    (void)s;
    if (i < n_tiles) {
        flag[i] = i == t0 ? 1u : 0u;
        key[i] = i == t0 ? 0ull : ~0ull;   // bits of +0.0
    }
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
__device__ __forceinline__ bool sweep(double* sd, const double (*hz)[kPT + 2], const float* scn, int q) {
    // node (r, c) of the tile is sd[r * kPS + c]; the halo lines (row -1,
    // row 64, column -1, column 64, each indexed from -1 to 64) are in hz,
    // a separate array, so that their loads can run ahead of the stores
    bool changed = false;
    double prev = VERT ? hz[REV ? 1 : 0][q + 1] : hz[REV ? 3 : 2][q + 1];   // halo before the first step
#pragma unroll 8
    for (int i = 0; i < kPT; ++i) {
        const int s = REV ? kPT - 1 - i : i;      // step along the sweep
        const int sp = REV ? s + 1 : s - 1;       // previous step
        double* me = VERT ? &sd[s * kPS + q] : &sd[q * kPS + s];
        const float c = VERT ? scn[cidx(s, q)] : scn[cidx(q, s)];
        // halo nodes beside lanes 0 and 63 at the previous step
        const double h0 = VERT ? hz[2][sp + 1] : hz[0][sp + 1];
        const double h1 = VERT ? hz[3][sp + 1] : hz[1][sp + 1];
        const double old = *me;
        double a = from_lane_below(prev), b = from_lane_above(prev);
        a = q == 0 ? h0 : a;
        b = q == kPT - 1 ? h1 : b;
        const double ws = (double)c + 1.0, wd = (double)c + kSqrt2;
        // sums are canonical, so the minima need no NaN quieting
        const double cand = fmin(prev + ws, fmin(a + wd, b + wd));
        const bool lower = cand < old;
        prev = lower ? cand : old;
        *me = prev;
        changed |= lower;
    }
    return changed;
}

// Non-negative doubles order like their bit patterns.
__device__ __forceinline__ unsigned long long dbits(double v) { return __builtin_bit_cast(unsigned long long, v); }

__global__ __launch_bounds__(64) void k_plan_relax(PlanGeom g, const float* __restrict__ cn,
                                                   const uint8_t* __restrict__ gw, double* __restrict__ dist,
                                                   const unsigned* __restrict__ list, unsigned* __restrict__ flag,
                                                   unsigned long long* __restrict__ key, long long src) {
    __shared__ double sd[kPT * kPS];
    __shared__ double hz[4][kPT + 2];
    __shared__ float scn[kPT * kCS];
    const int q = threadIdx.x;
    const int t = (int)list[blockIdx.x];
    const int tpl = g.ntx * g.nty;
    const int l = t / tpl, tt = t - l * tpl;
    const int ty = tt / g.ntx, tx = tt - ty * g.ntx;
    const int x0 = tx * kPT, y0 = ty * kPT;
    const long long lo = (long long)l * g.plane;
    const int x = x0 + q;
    const bool xin = x < g.nx;

    // distances of the tile and its one-cell halo (+inf outside the grid);
    // loads are issued in batches so that many are in flight.  Lane q keeps
    // its column's values (orig) to find the nodes that change.
    double orig[kPT];
    {
        double top, bot;
        constexpr int RB = 22;   // rows -1 .. 64 = 3 batches
#pragma unroll
        for (int r0 = -1; r0 < kPT + 1; r0 += RB) {
            double v[RB];
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                const int y = y0 + r0 + j;
                v[j] = (xin && y >= 0 && y < g.ny) ? dist[lo + (long long)y * g.nx + x] : INFINITY;
            }
#pragma unroll
            for (int j = 0; j < RB; ++j) {
                const int r = r0 + j;
                if (r < 0) top = v[j];
                else if (r >= kPT) bot = v[j];
                else orig[r] = v[j];
            }
        }
        hz[0][q + 1] = top;
        hz[1][q + 1] = bot;
#pragma unroll
        for (int r = 0; r < kPT; ++r) sd[r * kPS + q] = orig[r];
    }
    {
        // halo columns x0 - 1 and x0 + 64 (rows -1 .. 64), and the four
        // corners again in the halo rows: 136 values over the lanes
        double v[3];
        double* dst[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int idx = q + 64 * k;
            int xx, yy;
            dst[k] = nullptr;
            if (idx < 2 * (kPT + 2)) {
                const int side = idx / (kPT + 2), r = idx - side * (kPT + 2);
                xx = side ? x0 + kPT : x0 - 1;
                yy = y0 - 1 + r;
                dst[k] = &hz[2 + side][r];
            } else if (idx < 2 * (kPT + 2) + 4) {
                const int cidx = idx - 2 * (kPT + 2);   // (row -1 | 64) x (column -1 | 64)
                xx = (cidx & 1) ? x0 + kPT : x0 - 1;
                yy = (cidx & 2) ? y0 + kPT : y0 - 1;
                dst[k] = &hz[(cidx & 2) ? 1 : 0][(cidx & 1) ? kPT + 1 : 0];
            } else {
                xx = -1;
                yy = -1;
            }
            const bool in = dst[k] && xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny;
            v[k] = in ? dist[lo + (long long)yy * g.nx + xx] : INFINITY;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (dst[k]) *dst[k] = v[k];
    }
    // node costs; gateways into a node offer the adjacent layer's distance
    // at no cost (lane q updates only its own column here)
    constexpr int CB = 16;
    bool moved = false;                        // some node of the tile can improve
    unsigned long long outup = 0, outdn = 0;   // nodes of column q with a gateway up / down
    for (int r0 = 0; r0 < kPT; r0 += CB) {
        float c[CB];
        unsigned b[CB];
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int y = y0 + r0 + j;
            const bool in = xin && y < g.ny;
            const long long i = lo + (long long)y * g.nx + x;
            c[j] = in ? cn[i] : INFINITY;
            b[j] = in ? (unsigned)gw[i] : 0u;
        }
        double pu[CB];
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const long long i = lo + (long long)(y0 + r0 + j) * g.nx + x;
            double d = INFINITY;
            if (b[j] & kInFromBelow) d = dist[i - g.plane] + 0.0;
            if (b[j] & kInFromAbove) d = fmin(d, dist[i + g.plane] + 0.0);
            pu[j] = d;
        }
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            double* me = &sd[(r0 + j) * kPS + q];
            // the start node enters at distance 0 on the first visit of its tile
            const bool is_src = xin && y0 + r0 + j < g.ny && lo + (long long)(y0 + r0 + j) * g.nx + x == src;
            const double in = is_src ? 0.0 : pu[j];
            if (in < *me) {
                *me = in;
                moved = true;
            }
            scn[cidx(r0 + j, q)] = c[j];
            outup |= (unsigned long long)((b[j] & kOutUp) != 0) << (r0 + j);
            outdn |= (unsigned long long)((b[j] & kOutDown) != 0) << (r0 + j);
        }
    }
    __syncthreads();

    // The tile was at a fixed point of its own edges after its last visit,
    // and only its halo and gateway inputs can have changed since: unless a
    // gateway or the start lowered a node above, or a halo node lowers a
    // border node, nothing in the tile can change.
    {
        auto relax3 = [&](int r, int c, double straight, double d1, double d2) {
            const float cc = scn[cidx(r, c)];
            const double cand = fmin(straight + ((double)cc + 1.0), fmin(d1, d2) + ((double)cc + kSqrt2));
            return cand < sd[r * kPS + c];
        };
        moved |= relax3(0, q, hz[0][q + 1], hz[0][q], hz[0][q + 2]);                    // top
        moved |= relax3(kPT - 1, q, hz[1][q + 1], hz[1][q], hz[1][q + 2]);              // bottom
        moved |= relax3(q, 0, hz[2][q + 1], hz[2][q], hz[2][q + 2]);                    // left
        moved |= relax3(q, kPT - 1, hz[3][q + 1], hz[3][q], hz[3][q + 2]);              // right
    }
    if (!__ballot(moved)) return;

    // Sweep the directions in turn (left-to-right, right-to-left,
    // top-to-bottom, bottom-to-top), skipping a direction when no node has
    // changed since its last sweep: after a sweep, every edge of its
    // direction holds, so the tile is at its fixed point when all four are
    // clean.
    unsigned dirty = 0xFu;
    for (int d = 0; dirty; d = (d + 1) & 3) {
        if (!(dirty & (1u << d))) continue;
        bool ch;
        if (d == 0) ch = sweep<false, false>(sd, hz, scn, q);
        else if (d == 1) ch = sweep<false, true>(sd, hz, scn, q);
        else if (d == 2) ch = sweep<true, false>(sd, hz, scn, q);
        else ch = sweep<true, true>(sd, hz, scn, q);
        dirty &= ~(1u << d);
        if (__ballot(ch)) dirty = 0xFu & ~(1u << d);
        __syncthreads();
    }

    // write back the nodes that changed (values only go down); note which
    // neighbours must look again and the least changed distance (their
    // priority)
    bool nb_up = false, nb_dn = false, nb_l = false, nb_r = false;
    bool c_ul = false, c_ur = false, c_dl = false, c_dr = false, g_up = false, g_dn = false;
    double vmin = INFINITY;
    const int w = min(kPT, g.nx - x0), h = min(kPT, g.ny - y0);
    const bool qin = q < w;
#pragma unroll
    for (int r = 0; r < kPT; ++r) {
        const double nd = sd[r * kPS + q];
        if (qin && r < h && nd < orig[r]) {
            dist[lo + (long long)(y0 + r) * g.nx + x] = nd;
            vmin = fmin(vmin, nd);
            nb_up |= r == 0;
            nb_dn |= r == h - 1;
            nb_l |= q == 0;
            nb_r |= q == w - 1;
            c_ul |= r == 0 && q == 0;
            c_ur |= r == 0 && q == w - 1;
            c_dl |= r == h - 1 && q == 0;
            c_dr |= r == h - 1 && q == w - 1;
            g_up |= ((outup >> r) & 1ull) != 0;
            g_dn |= ((outdn >> r) & 1ull) != 0;
        }
    }
    const unsigned long long m_up = __ballot(nb_up), m_dn = __ballot(nb_dn), m_l = __ballot(nb_l),
                             m_r = __ballot(nb_r), m_ul = __ballot(c_ul), m_ur = __ballot(c_ur),
                             m_dl = __ballot(c_dl), m_dr = __ballot(c_dr), m_gu = __ballot(g_up),
                             m_gd = __ballot(g_dn);
    for (int o = 32; o > 0; o >>= 1) vmin = fmin(vmin, __shfl_xor(vmin, o, 64));
    if (q == 0) {
        const unsigned long long kv = dbits(vmin);
        auto act = [&](int ll, int yy, int xx) {
            if (ll < 0 || ll >= g.L || yy < 0 || yy >= g.nty || xx < 0 || xx >= g.ntx) return;
            const int tn = (ll * g.nty + yy) * g.ntx + xx;
            atomicMin(&key[tn], kv);
            flag[tn] = 1u;
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

// Active tiles whose key (the least distance that activated them) is at
// most the band limit -> worklist (flag and key cleared); the others stay
// active: st[1] counts them and st2 receives their least key.  st[0] (the
// list length), st[1] and st2 must be reset before the launch.
__global__ __launch_bounds__(256) void k_plan_compact(unsigned* __restrict__ flag, unsigned long long* __restrict__ key,
                                                      int n_tiles, unsigned long long band, unsigned* __restrict__ list,
                                                      unsigned* __restrict__ st, unsigned long long* __restrict__ st2,
                                                      unsigned long long* __restrict__ st3) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = t < n_tiles && flag[t] != 0u;
    const unsigned long long kt = act ? key[t] : ~0ull;
    {
        // least key of all active tiles (a lower bound on every label still
        // to be lowered)
        unsigned long long kmin = kt;
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned long long y = __shfl_xor(kmin, o, 64);
            kmin = y < kmin ? y : kmin;
        }
        if ((threadIdx.x & 63) == 0 && kmin != ~0ull) atomicMin(st3, kmin);
    }
    const bool on = act && kt <= band;
    const bool rest = act && !on;
    const unsigned long long m = __ballot(on), mr = __ballot(rest);
    const int lane = threadIdx.x & 63;
    unsigned base = 0;
    if (lane == 0 && m) base = atomicAdd(&st[0], (unsigned)__popcll(m));
    if (lane == 0 && mr) atomicAdd(&st[1], (unsigned)__popcll(mr));
    if (rest) atomicMin(st2, kt);
    base = __shfl(base, 0, 64);
    if (on) {
        flag[t] = 0u;
        key[t] = ~0ull;
        list[base + __popcll(m & ((1ull << lane) - 1ull))] = (unsigned)t;
    }
}

struct PlanStatus {
    unsigned n_list, n_rest;
    unsigned long long rest_key, min_key;
};

__global__ void k_plan_status_reset(PlanStatus* st) {
    st->n_list = 0u;
    st->n_rest = 0u;
    st->rest_key = ~0ull;
    st->min_key = ~0ull;
}



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
    __shared__ int s_layer[PCT_MAX_SLICES];
    __shared__ int s_row[64][3];
    for (int i = lane; i < g.L; i += 64) s_layer[i] = layers[i];
    __syncthreads();
    int len = 0, status = 0;
    // the current node's distance and cost travel with it: each step loads
    // the candidates' distance, cost and gateway bits in one round and takes
    // the chosen one's by a shuffle, so a step waits on one memory round.
    // Path rows collect in LDS and go out 64 at a time (a store in flight
    // would hold up the next step's loads).
    auto flush = [&](int n_rows) {
        __syncthreads();
        if (lane < n_rows) {
            const int r = len - n_rows + lane;
            path[3 * r] = s_row[lane][0];
            path[3 * r + 1] = s_row[lane][1];
            path[3 * r + 2] = s_row[lane][2];
        }
        __syncthreads();
    };
    double dv = dist[v];
    float cv = cn[v];
    int x = gx, y = gy, l = gl;  // v's coordinates travel with it too (no divisions)
    if (dv < INFINITY) {
        for (;;) {
            if (len >= max_len) {
                status = -2;
                break;
            }
            const long long c = (long long)y * g.nx + x;
            if (lane == 0) {
                s_row[len & 63][0] = x;
                s_row[len & 63][1] = y;
                s_row[len & 63][2] = s_layer[l];
            }
            ++len;
            if ((len & 63) == 0) flush(64);
            if (v == s) break;
            long long u = -1;
            double du = 0.0;
            float cu = 0.0f;
            int ux = x, uy = y, ul = l;
            bool ok = false;
            if (lane < 2) {
                const int m = lane == 0 ? l - 1 : l + 1;
                if (m >= 0 && m < g.L) {
                    const long long uu = (long long)m * g.plane + c;
                    const unsigned bit = lane == 0 ? kOutUp : kOutDown;
                    const uint8_t gb = gw[uu];
                    du = dist[uu];
                    cu = cn[uu];
                    ul = m;
                    if ((gb & bit) && du + 0.0 == dv) {
                        u = uu;
                        ok = true;
                    }
                }
            } else if (lane < 10) {
                const int e = lane - 2;
                const int dy = e < 3 ? -1 : (e < 5 ? 0 : 1);
                const int dx = e < 3 ? e - 1 : (e < 5 ? (e == 3 ? -1 : 1) : e - 6);
                const int x2 = x + dx, y2 = y + dy;
                if (x2 >= 0 && y2 >= 0 && x2 < g.nx && y2 < g.ny && cv < INFINITY) {
                    const long long uu = (long long)l * g.plane + (long long)y2 * g.nx + x2;
                    du = dist[uu];
                    cu = cn[uu];
                    ux = x2;
                    uy = y2;
                    const double wgt = (double)cv + ((dx != 0 && dy != 0) ? kSqrt2 : 1.0);
                    if (du + wgt == dv) {
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
            dv = __shfl(du, first, 64);
            cv = __shfl(cu, first, 64);
            x = __shfl(ux, first, 64);
            y = __shfl(uy, first, 64);
            l = __shfl(ul, first, 64);
        }
    }
    if ((len & 63) != 0) flush(len & 63);
    __syncthreads();
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
    unsigned long long* key;
    unsigned* list;
    PlanStatus* st;
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
    ws.key = (unsigned long long*)take(sizeof(unsigned long long) * (size_t)nt);
    ws.list = (unsigned*)take(sizeof(unsigned) * (size_t)nt);
    ws.st = (PlanStatus*)take(sizeof(PlanStatus));
    ws.layers = (int*)take(sizeof(int) * (size_t)g.L);
    ws.out = (int*)take(sizeof(int) * 4);
    if (w) *w = ws;
    return off;
}

}  // namespace

size_t plan_ws_bytes(int nx, int ny, int L) { return plan_ws_layout(make_plan_geom(nx, ny, L), nullptr, nullptr); }

pct_status launch_plan(const float* cost, const float* ground, int nx, int ny, const int* h_layers, int L, float cB,
                       int sx, int sy, int sl, double* dist, void* ws_base, int* h_rounds, long long* h_tiles,
                       hipStream_t s, double delta, long long goal, double* h_settled) {
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
    hipLaunchKernelGGL(k_plan_init, dim3((unsigned)((ni + 255) / 256)), dim3(256), 0, s, dist, nn, src, w.flag, w.key,
                       nt, t0);
    PCT_LAUNCH_CHECK();
    // Rounds take the active tiles whose activating distance lies within
    // a band of width delta above the least one (tiles roughly in order of
    // distance, as Dijkstra's algorithm takes nodes); a band with no tile
    // left moves up to the least remaining key.
    double band = delta;
    int rounds = 0;
    long long tiles = 0;
    PlanStatus hs;
    double settled = INFINITY;
    for (;;) {
        unsigned long long band_bits;
        memcpy(&band_bits, &band, sizeof band_bits);
        hipLaunchKernelGGL(k_plan_status_reset, dim3(1), dim3(1), 0, s, w.st);
        hipLaunchKernelGGL(k_plan_compact, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, w.flag, w.key, nt,
                           band_bits, w.list, &w.st->n_list, &w.st->rest_key, &w.st->min_key);
        PCT_LAUNCH_CHECK();
        PCT_HIP(hipMemcpyAsync(&hs, w.st, sizeof hs, hipMemcpyDeviceToHost, s));
        double dg = INFINITY;
        if (goal >= 0) PCT_HIP(hipMemcpyAsync(&dg, dist + goal, sizeof dg, hipMemcpyDeviceToHost, s));
        PCT_HIP(hipStreamSynchronize(s));
        if (goal >= 0 && (hs.n_list != 0 || hs.n_rest != 0)) {
            // no active tile can lower a label below its key: every label
            // under the least key is final, the goal's among them
            double kmin;
            memcpy(&kmin, &hs.min_key, sizeof kmin);
            if (kmin > dg) {
                settled = kmin;
                break;
            }
        }
        if (hs.n_list == 0) {
            if (hs.n_rest == 0) break;
            double kmin;
            memcpy(&kmin, &hs.rest_key, sizeof kmin);
            band = kmin + delta;
            continue;
        }
        hipLaunchKernelGGL(k_plan_relax, dim3(hs.n_list), dim3(64), 0, s, g, w.cn, w.gw, dist, w.list, w.flag, w.key,
                           src);
        PCT_LAUNCH_CHECK();
        ++rounds;
        tiles += hs.n_list;
    }
    if (h_rounds) *h_rounds = rounds;
    if (h_tiles) *h_tiles = tiles;
    if (h_settled) *h_settled = settled;
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
