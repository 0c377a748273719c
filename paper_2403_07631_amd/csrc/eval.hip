// Traversability (Sec. III-B, Eqs. (1)-(6)) and simplification (Sec. III-C,
// Eqs. (7)-(9)) on gfx950.
//
// One workgroup evaluates a 64 x 16 tile of one slice.  The ground layer is
// staged in LDS with a halo of R + r_p + 1 cells (R: inflation radius, r_p:
// step-patch radius), the gentle flags with a halo of R + r_p, and c^init
// with a halo of R.  Inflation is the weighted max of Eq. (6) split by rows:
//   V_a(x, y) = max_j K(a, j) * max(c(x, y-j), c(x, y+j))       (column pass)
//   c^T(x, y) = max_a max(V_a(x-a, y), V_a(x+a, y))             (row pass)
// Each product K * c is the same FP32 multiply as in the direct 2-D window
// and max is exact, so the result equals the direct FP32 window max.
#include <limits.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "pct_internal.h"

namespace pct {

namespace {

constexpr int kBlock = 256;
constexpr int TW = kEvalTileW, TH = kEvalTileH;

__device__ __forceinline__ float sumsq(float dx, float dy) { return __builtin_fmaf(dx, dx, dy * dy); }

template <int R>
__global__ __launch_bounds__(kBlock) void k_eval(const float* __restrict__ ground, const float* __restrict__ ceil,
                                                 const EvalParams p, float* __restrict__ cost) {
    extern __shared__ float smem[];
    const int k = blockIdx.z;
    const int tx0 = p.wx0 + blockIdx.x * TW, ty0 = p.wy0 + blockIdx.y * TH;
    const int rp = p.rp;
    const int HG = R + rp + 1, HF = R + rp;
    const int WG = TW + 2 * HG, HGt = TH + 2 * HG;
    const int WF = TW + 2 * HF, HFt = TH + 2 * HF;
    constexpr int WC = TW + 2 * R, HC = TH + 2 * R;
    float* sG = smem;
    float* sC = sG + WG * HGt;
    float* sV = sC + WC * HC;
    unsigned char* sF = (unsigned char*)(sV + (R + 1) * TH * WC);
    const float* gk = ground + (long long)k * p.plane;
    const float* ck = ceil + (long long)k * p.plane;
    const int nx = p.nx, ny = p.ny;

    // ground with halo; outside the grid there is no ground
    for (int i = threadIdx.x; i < WG * HGt; i += kBlock) {
        const int u = i % WG, v = i / WG;
        const int gx = tx0 - HG + u, gy = ty0 - HG + v;
        sG[i] = (gx >= 0 && gy >= 0 && gx < nx && gy < ny) ? gk[(long long)gy * nx + gx] : -INFINITY;
    }
    __syncthreads();

    // gentle flags: ground, a full stencil, and m^grad < theta_s
    for (int i = threadIdx.x; i < WF * HFt; i += kBlock) {
        const int u = i % WF, v = i / WF;
        const int su = u + 1, sv = v + 1;
        const float G = sG[sv * WG + su];
        const float l = sG[sv * WG + su - 1], r = sG[sv * WG + su + 1];
        const float d = sG[(sv - 1) * WG + su], up = sG[(sv + 1) * WG + su];
        bool gentle = false;
        if (isfinite(G) && isfinite(l) && isfinite(r) && isfinite(d) && isfinite(up))
            gentle = sumsq(r - l, up - d) < p.Ts2;
        sF[i] = gentle ? 1 : 0;
    }
    __syncthreads();

    // c^init, Eqs. (1)-(5); zero outside the grid (skipped inflation taps)
    for (int i = threadIdx.x; i < WC * HC; i += kBlock) {
        const int u = i % WC, v = i / WC;
        const int gx = tx0 - R + u, gy = ty0 - R + v;
        float ci = 0.0f;
        if (gx >= 0 && gy >= 0 && gx < nx && gy < ny) {
            const int su = u + rp + 1, sv = v + rp + 1;
            const float G = sG[sv * WG + su];
            if (!isfinite(G)) {
                ci = p.cB;
            } else {
                const float C = ck[(long long)gy * nx + gx];
                const float dI = C - G;
                const float cI = dI < p.d_min ? p.cB : fmaxf(0.0f, p.alpha_d * (p.d_ref - dI));
                const float l = sG[sv * WG + su - 1], r = sG[sv * WG + su + 1];
                const float d = sG[(sv - 1) * WG + su], up = sG[(sv + 1) * WG + su];
                float cG = p.cB;
                if (isfinite(l) && isfinite(r) && isfinite(d) && isfinite(up)) {
                    const float dx = r - l, dy = up - d;
                    const float adx = fabsf(dx), ady = fabsf(dy);
                    if (!(fmaxf(adx, ady) > p.Tb)) {
                        const float s2 = sumsq(dx, dy);
                        if (s2 < p.Ts2) {
                            cG = p.As * s2;
                        } else {
                            int cnt = 0;
                            const int fu = u + rp, fv = v + rp;
                            for (int dyp = -rp; dyp <= rp; ++dyp)
                                for (int dxp = -rp; dxp <= rp; ++dxp)
                                    cnt += (dxp | dyp) ? sF[(fv + dyp) * WF + fu + dxp] : 0;
                            if (cnt > p.kp) cG = p.Ab * fmaxf(dx * dx, dy * dy);
                        }
                    }
                }
                ci = fminf(p.cB, cI + cG);
            }
        }
        sC[i] = ci;
    }
    __syncthreads();

    // column pass
    for (int i = threadIdx.x; i < WC * TH; i += kBlock) {
        const int x = i % WC, y = i / WC;
        float P[R + 1];
        P[0] = sC[(y + R) * WC + x];
#pragma unroll
        for (int j = 1; j <= R; ++j) P[j] = fmaxf(sC[(y + R - j) * WC + x], sC[(y + R + j) * WC + x]);
#pragma unroll
        for (int a = 0; a <= R; ++a) {
            float vmax = 0.0f;
#pragma unroll
            for (int j = 0; j <= R; ++j) vmax = fmaxf(vmax, p.K[a][j] * P[j]);
            sV[(a * TH + y) * WC + x] = vmax;
        }
    }
    __syncthreads();

    // row pass and store
    for (int i = threadIdx.x; i < TW * TH; i += kBlock) {
        const int x = i % TW, y = i / TW;
        const int gx = tx0 + x, gy = ty0 + y;
        float v = sV[(0 * TH + y) * WC + x + R];
#pragma unroll
        for (int a = 1; a <= R; ++a)
            v = fmaxf(v, fmaxf(sV[(a * TH + y) * WC + x + R - a], sV[(a * TH + y) * WC + x + R + a]));
        if (gx < p.wx1 && gy < p.wy1) cost[(long long)k * p.plane + (long long)gy * nx + gx] = v;
    }
}

// ------------------------------------------------------------ strip kernels
//
// The common case (patch radius 1, inflation radius <= 8).  A workgroup of
// NW wavefronts (1, 2 or 4) walks down the rows of one slice over a band
// of columns, each wavefront over 64 adjacent columns, keeping the rows it
// still needs in registers:
//   ground rows  y+R .. y+R+2     (the stencil of the newest flag row),
//   gentle flags y+R-1 .. y+R+1   (the 3x3 patch count),
//   c^init rows  y-R   .. y+R     (the column pass of the inflation).
// The central differences of a row are formed once, for its gentle flag,
// and kept for its c^init one step later.  Horizontal neighbours of the
// stencils and the patch count come from adjacent lanes (DPP shifts by one
// lane), so the two lanes at each side of a wavefront only complete the
// stencils of the middle kWgOwn, its own columns.  The row pass of the
// inflation reads the column-pass maxima of the neighbouring columns from
// LDS, where every wavefront leaves those of its own columns; only the
// outer R own columns of the workgroup are halo.  Per element the
// arithmetic is the same sequence of FP32 operations as in the tiled kernel
// above, so both give identical bits.

// bound_ctrl: the edge lane (no source lane) reads 0, so no old value has
// to be copied into the destination first.
__device__ __forceinline__ float from_prev(float v) {   // lane i receives lane i-1
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_next(float v) {   // lane i receives lane i+1
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ int from_prev_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int from_next_i(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }

#ifndef PCT_EVAL_PREFETCH
#define PCT_EVAL_PREFETCH 4
#endif
#ifndef PCT_EVAL_STRIP_ROWS
#define PCT_EVAL_STRIP_ROWS 256
#endif
constexpr int kPrefetch = PCT_EVAL_PREFETCH;   // rows fetched ahead per wavefront
constexpr int kStripRows = PCT_EVAL_STRIP_ROWS; // output rows per strip (upper bound)

struct StripGeom {
    int rows;   // output rows per strip
    int n_sx, n_sy, n_work;
    int nw;     // wavefronts per workgroup (1, 2 or kDefaultWaves)
};

// Max of two non-negative floats (+0 included, no NaN) on their bit patterns:
// for such values the unsigned order of the encodings is the numeric order,
// so this is exact, and it avoids the NaN-quieting moves fmaxf needs.
__device__ __forceinline__ float maxnn(float a, float b) {
    return __builtin_bit_cast(float, max(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b)));
}

// Tap weights known at compile time: weight exactly 1 where a^2 + j^2 <= Q1
// and exactly 0 where a^2 + j^2 >= Q0 (Q1 < 0 and Q0 = kNoZeroTaps: none
// known).  1 * c = c and 0 * c = 0 exactly for the finite c^init >= 0, so
// skipping those multiplies leaves every maximum unchanged.
constexpr int kNoZeroTaps = 1 << 20;

// The largest j <= R with j^2 <= Q1 (0 when Q1 < 1): taps (0, j) up to it have weight 1.
constexpr int weight1_reach(int Q1, int R) {
    int j = 0;
    while (j < R && (j + 1) * (j + 1) <= Q1) ++j;
    return j;
}

constexpr int kWgOwn = 60;                        // own columns of a wavefront
constexpr int kDefaultWaves = PCT_STRIP_WAVES;    // wavefronts of the widest workgroup strip
static_assert(64 * kDefaultWaves == kBlock, "batched jobs run in blocks of kBlock threads");

// V_a of own column i at v[set][row][i * R + a - 1]: the 2R reads of a row
// pass lie within 2R^2 + R words of one address (ds_read2 offsets), and
// lanes R words apart touch distinct banks.  Two rows are exchanged per
// barrier, in two alternating sets.
template <int R, int NW>
struct WgLds {
    float v[2][2][(R > 0 ? R : 1) * kWgOwn * NW];
};

// Raw buffer access to one slice plane (fewer than 2^29 cells): a scalar
// descriptor, the row's byte offset in a scalar register and the lane's
// column offset in a vector register, so that a row step spends no vector
// instruction on addresses.
constexpr int kBufferDword3 = 0x00020000;   // 32-bit elements, gfx9 buffer format
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, long long plane) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(plane * 4), kBufferDword3);
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

// Orders the LDS exchange of one row pass: a workgroup barrier, or for a
// single wavefront (whose LDS operations complete in issue order) only a
// fence that keeps the compiler from moving them.
template <int NW>
__device__ __forceinline__ void row_exchange_sync() {
    if constexpr (NW > 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// One workgroup strip: work item w of a map with parameters p and strip
// geometry sg (ground/ceil/cost already point at the map's first slice).
// The live rows sit in rings of S slots indexed by the step number modulo
// S; the row loop is unrolled S times so that every slot index is a
// compile-time constant and no row is ever moved between registers.  Step t
// handles output row y = Y0 - 2 (R + 2) + t.
// With slice_bits non-null the strip also sets bit k of slice_bits (bit
// k % 32 of word k / 32) when one of its stored costs is traversable
// (c^T < c^B), so that the slice test can pass over slices without any.
template <int R, int Q1, int Q0, int NW>
__device__ __forceinline__ void eval_strip_item(const float* __restrict__ ground, const float* __restrict__ ceil,
                                                const EvalParams& p, float* __restrict__ cost, const StripGeom& sg,
                                                int w, WgLds<R, NW>& lds,
                                                unsigned* __restrict__ slice_bits = nullptr) {
    constexpr int HX = R + 2;
    constexpr int SPAN = kWgOwn * NW;       // own columns of the workgroup
    constexpr int OUTW = SPAN - 2 * R;      // columns it stores
    constexpr int S0 = 2 * R + 1 > 4 ? 2 * R + 1 : 4;
    constexpr int S1 = S0 > kPrefetch ? S0 : kPrefetch;
    constexpr int S = (S1 + 3) / 4 * 4;     // a multiple of 4: the LDS set of step t is (ph >> 1) & 1
    // vertical taps of weight exactly 1: |dy| <= JV (the centre alone when the pattern is not known)
    constexpr int JV = weight1_reach(Q1, R);
    const int gx = w % sg.n_sx;
    const int t0 = w / sg.n_sx;
    const int sy = t0 % sg.n_sy;
    const int k = t0 / sg.n_sy;
    const int wave = NW > 1 ? (int)(threadIdx.x >> 6) : 0;
    const int lane = threadIdx.x & 63;
    const int nx = p.nx, ny = p.ny;
    const int X0 = p.wx0 + gx * OUTW;               // first stored column
    const int i = kWgOwn * wave + lane - 2;         // own-column index (lanes 2 .. 61)
    const int x = X0 - R + i;
    const bool own = lane >= 2 && lane < 2 + kWgOwn;
    const bool xout = own && i >= R && i < SPAN - R && x < p.wx1;
    const int ir = min(max(i, R), SPAN - R - 1);    // row-pass reads stay inside the buffer
    const bool xin = x >= 0 && x < nx;
    const int voff = min(max(x, 0), nx - 1) * 4;    // the lane's column, in bytes
    const int Y0 = p.wy0 + sy * sg.rows, Y1 = min(p.wy1, Y0 + sg.rows);
    const __amdgpu_buffer_rsrc_t rG = plane_rsrc(ground + (long long)k * p.plane, p.plane);
    const __amdgpu_buffer_rsrc_t rC = plane_rsrc(ceil + (long long)k * p.plane, p.plane);
    const __amdgpu_buffer_rsrc_t rO = plane_rsrc(cost + (long long)k * p.plane, p.plane);
    const int row_bytes = nx * 4;
    auto row_off = [&](int row) { return min(max(row, 0), ny - 1) * row_bytes; };

    float gS[S];   // ground, row y+R+2 (newest) at slot ph, row y+R+2-j at slot ph-j
    int fS[S];     // gentle flags, row y+R+1 at slot ph
    float cS[S];   // c^init, row y+R at slot ph
    float gRaw[S], cRaw[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        gS[q] = -INFINITY;
        fS[q] = 0;
        cS[q] = 0.0f;
    }
    // central differences of the row whose c^init is formed next, and
    // whether that row has ground
    float sdx = 0.0f, sdy = 0.0f, ss2 = 0.0f;
    bool sfin = false;
    float h0_even = 0.0f, h0_cur = 0.0f;
    bool skip_even = false;  // the even step's row needs no window maxima (uniform)
    bool any_trav = false;   // a stored cost of this wavefront is below c^B (uniform)
    const int ys = Y0 - 2 * HX;
#pragma unroll
    for (int d = 0; d < kPrefetch; ++d) {
        gRaw[d % S] = buf_load(rG, voff, row_off(ys + HX + d));
        cRaw[d % S] = buf_load(rC, voff, row_off(ys + R + d));
    }
    const int n_steps = Y1 - ys;
    for (int tb = 0; tb < n_steps; tb += S) {
#pragma unroll
        for (int ph = 0; ph < S; ++ph) {
            const int t = tb + ph;
            if (t < n_steps) {   // uniform over the workgroup
                const int y = ys + t;
                const int rg = y + HX, rc = y + R;
                // step t consumes raw slot ph and refills it kPrefetch rows ahead;
                // outside the grid there is no ground
                const float gIn = (xin & (rg >= 0) & (rg < ny)) ? gRaw[ph] : -INFINITY;
                const float cIn = cRaw[ph];
                const bool crow = xin & (rc >= 0) & (rc < ny);
                gRaw[(ph + kPrefetch) % S] = buf_load(rG, voff, row_off(rg + kPrefetch));
                cRaw[(ph + kPrefetch) % S] = buf_load(rC, voff, row_off(rc + kPrefetch));
                gS[ph] = gIn;
                const float g3 = gS[ph], g2 = gS[(ph + S - 1) % S], g1 = gS[(ph + S - 2) % S];   // rows y+R+2, +1, +0

                // Ground values are finite or -inf.  A difference of two
                // such values is finite only when both are finite (else it
                // is +-inf or NaN), so a test that fails on inf and NaN
                // (s2 < Ts2, |d| <= Tb with Tb finite) already carries the
                // finiteness of the stencil neighbours.

                // stencil and gentle flag of row y+R+1
                const float ndx = from_next(g2) - from_prev(g2), ndy = g3 - g1;
                const float ns2 = sumsq(ndx, ndy);
                const bool nfin = isfinite(g2);
                fS[ph] = (nfin & (ns2 < p.Ts2)) ? 1 : 0;
                const int f2 = fS[ph], f1 = fS[(ph + S - 1) % S], f0 = fS[(ph + S - 2) % S];  // rows y+R+1, +0, -1

                // c^init of row y+R, Eqs. (1)-(5), without branches, from the
                // stencil formed one step earlier
                {
                    const float G = g1;
                    const int colsum = f0 + f1 + f2;
                    const int cnt = colsum + from_prev_i(colsum) + from_next_i(colsum) - f1;
                    const float dI = cIn - G;
                    const float cI = dI < p.d_min ? p.cB : fmaxf(0.0f, p.alpha_d * (p.d_ref - dI));
                    const float c_gentle = p.As * ss2;
                    // max(dx^2, dy^2) = max(|dx|, |dy|)^2: squaring is monotone in |d|
                    const float m = fmaxf(fabsf(sdx), fabsf(sdy));
                    const float c_edge = p.Ab * (m * m);
                    const float c_step = cnt > p.kp ? c_edge : p.cB;
                    float cG = ss2 < p.Ts2 ? c_gentle : c_step;
                    // both differences within the step bound (false for inf and NaN)
                    const bool passable = (fabsf(sdx) <= p.Tb) & (fabsf(sdy) <= p.Tb);
                    cG = passable ? cG : p.cB;
                    const float ci = sfin ? fminf(p.cB, cI + cG) : p.cB;
                    cS[ph] = crow ? ci : 0.0f;
                }
                sdx = ndx;
                sdy = ndy;
                ss2 = ns2;
                sfin = nfin;

                // inflation of row y: c^init rows y-R .. y+R are slots ph-2R .. ph
                // (column pass from registers; all operands are >= 0)
                float P[R + 1];
                P[0] = cS[(ph + S - R) % S];
#pragma unroll
                for (int jj = 1; jj <= R; ++jj)
                    P[jj] = maxnn(cS[(ph + S - R - jj) % S], cS[(ph + S - R + jj) % S]);
                // One-wavefront strips skip the window maxima of a row that is
                // not stored (the rows before Y0 only fill the rings), and of a
                // row whose every stored output is already known to be c^B:
                // c^init <= c^B everywhere, so an output whose window holds a
                // cell with c^init = c^B at a tap of weight exactly 1 (the
                // vertical taps |dy| <= JV of its own column) is c^B.  The
                // vote is the wavefront's own; its exchange buffer is read by
                // its own lanes only.
                bool skip = false;
                if constexpr (NW == 1) {
                    float vm = P[0];
#pragma unroll
                    for (int jj = 1; jj <= JV; ++jj) vm = maxnn(vm, P[jj]);
                    skip = y < Y0 || __ballot(xout && vm < p.cB) == 0ull;
                }
                if ((ph & 1) == 0) skip_even = skip;
                if (!skip) {
                float h[R + 1];
#pragma unroll
                for (int a = 0; a <= R; ++a) {
                    float v = 0.0f;
#pragma unroll
                    for (int jj = 0; jj <= R; ++jj) {
                        const int q = a * a + jj * jj;
                        if (q <= Q1) v = maxnn(v, P[jj]);                      // weight 1
                        else if (q < Q0) v = maxnn(v, p.K[a][jj] * P[jj]);     // weight in (0, 1)
                    }
                    h[a] = v;
                }
                // row pass: rows of even and odd steps go to the two rows of a
                // set; the exchange and the row passes follow the odd step (or
                // the last one)
                float* buf = lds.v[(ph >> 1) & 1][ph & 1];
                if (own) {
#pragma unroll
                    for (int a = 1; a <= R; ++a) buf[i * R + a - 1] = h[a];
                }
                if ((ph & 1) == 0) h0_even = h[0];
                else h0_cur = h[0];
                }
                if ((ph & 1) == 1 || t == n_steps - 1) {
                    row_exchange_sync<NW>();
#pragma unroll
                    for (int r2 = 0; r2 < 2; ++r2) {
                        if (r2 == 0 && (ph & 1) == 0) continue;   // a lone even step: its row only
                        const int yy = r2 == 0 ? y - 1 : y;
                        const bool even = r2 == 0 || (ph & 1) == 0;
                        float v = p.cB;
                        if (!(even ? skip_even : skip)) {
                            const float* rb = lds.v[(ph >> 1) & 1][r2 == 0 ? 0 : (ph & 1)] + (ir - R) * R;
                            v = even ? h0_even : h0_cur;
#pragma unroll
                            for (int a = 1; a <= R; ++a)
                                v = maxnn(v, maxnn(rb[(R - a) * R + a - 1], rb[(R + a) * R + a - 1]));
                        }
                        if (yy >= Y0 && xout) buf_store(v, rO, voff, yy * row_bytes);
                        if (slice_bits && yy >= Y0 && !any_trav)   // uniform
                            any_trav = __ballot(xout && v < p.cB) != 0ull;
                    }
                }
            }
        }
    }
    if (any_trav && lane == 0) {
        // the hundreds of strips of a slice with traversable cells end at
        // about the same time, and atomics on one word queue behind each
        // other: strips that find the bit set already leave it (a stale
        // read only costs an atomic)
        unsigned* word = &slice_bits[k >> 5];
        const unsigned bit = 1u << (k & 31);
        if ((*(volatile unsigned*)word & bit) == 0u) atomicOr(word, bit);
    }
}

template <int R, int Q1, int Q0, int NW>
__global__ __launch_bounds__(64 * NW) void k_eval_strip(const float* __restrict__ ground, const float* __restrict__ ceil,
                                                        const EvalParams p, float* __restrict__ cost,
                                                        const StripGeom sg, unsigned* __restrict__ slice_bits) {
    __shared__ WgLds<R, NW> lds;
    // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin; each
    // XCD gets a contiguous range of strips, so neighbours share an L2
    const int per_xcd = gridDim.x / 8;
    const int w = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (w >= sg.n_work) return;   // the whole workgroup
    eval_strip_item<R, Q1, Q0, NW>(ground, ceil, p, cost, sg, w, lds, slice_bits);
}

// A batch: jobs are (map, robot) pairs with their own parameters, strip
// geometry and offsets; one launch covers every job's strips.  A block of
// kBlock threads is one strip of a job whose workgroups have kDefaultWaves
// wavefronts, or kBlock / 64 strips of one wavefront each.
struct EvalJob {
    EvalParams p;
    StripGeom sg;
    long long in_off, out_off, keep_off;   // element offsets of ground/ceil, cost, keep
    long long cell_base;                   // first global cell of the job (slice test)
    long long ws_off;                      // byte offset of the job's slice-test scratch
    int block_base;                        // first global block of the job
    int n_blocks;
};

// A job's slice-test scratch at ws + ws_off: the largest run starts (N
// ints), the N x W bit matrix, then W words of slice marks (bit k: slice
// k has a traversable cell), W = ceil(N / 32).
struct JobScratch {
    int* maxp0;
    unsigned* urun;
    unsigned* marks;
};
__host__ __device__ __forceinline__ size_t job_scratch_bytes(int N) {
    const size_t W = (size_t)(N + 31) / 32;
    return align_up(sizeof(int) * (size_t)N) + align_up(sizeof(unsigned) * (size_t)N * W) +
           align_up(sizeof(unsigned) * W);
}
__device__ __forceinline__ JobScratch job_scratch(char* ws, const EvalJob& jb) {
    const int N = jb.p.N;
    const size_t W = (size_t)(N + 31) / 32;
    char* b = ws + jb.ws_off;
    JobScratch js;
    js.maxp0 = (int*)b;
    js.urun = (unsigned*)(b + align_up(sizeof(int) * (size_t)N));
    js.marks = (unsigned*)(b + align_up(sizeof(int) * (size_t)N) + align_up(sizeof(unsigned) * (size_t)N * W));
    return js;
}

__device__ __forceinline__ int find_job_block(const EvalJob* __restrict__ jobs, int n_jobs, int b) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].block_base <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int R, int Q1, int Q0>
__global__ __launch_bounds__(kBlock) void k_eval_strip_jobs(const float* __restrict__ ground,
                                                            const float* __restrict__ ceil,
                                                            const EvalJob* __restrict__ jobs, int n_jobs, int n_blocks,
                                                            float* __restrict__ cost, char* __restrict__ marks_ws) {
    static_assert(sizeof(WgLds<R, kDefaultWaves>) == (kBlock / 64) * sizeof(WgLds<R, 1>), "LDS of one-wave strips");
    __shared__ WgLds<R, kDefaultWaves> lds;
    const int per_xcd = gridDim.x / 8;
    const int b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= n_blocks) return;   // the whole workgroup
    const int j = __builtin_amdgcn_readfirstlane(find_job_block(jobs, n_jobs, b));
    const EvalJob& jb = jobs[j];
    // slice marks for the slice test (marks_ws: the jobs' scratch, nullable)
    unsigned* marks = marks_ws ? job_scratch(marks_ws, jb).marks : nullptr;
    if (jb.sg.nw > 1) {
        if (b - jb.block_base >= jb.n_blocks) return;
        eval_strip_item<R, Q1, Q0, kDefaultWaves>(ground + jb.in_off, ceil + jb.in_off, jb.p, cost + jb.out_off,
                                                  jb.sg, b - jb.block_base, lds, marks);
    } else {
        const int wave = (int)(threadIdx.x >> 6);
        const int w = (b - jb.block_base) * (kBlock / 64) + wave;
        WgLds<R, 1>& mine = reinterpret_cast<WgLds<R, 1>*>(&lds)[wave];
        if (w < jb.sg.n_work)
            eval_strip_item<R, Q1, Q0, 1>(ground + jb.in_off, ceil + jb.in_off, jb.p, cost + jb.out_off, jb.sg, w,
                                          mine, marks);
    }
}

// Strip shapes chosen by the autotuner, per map shape and kernel radius.
struct TuneKey {
    int nx, ny, N, R;
    bool operator<(const TuneKey& o) const {
        return nx != o.nx ? nx < o.nx : ny != o.ny ? ny < o.ny : N != o.N ? N < o.N : R < o.R;
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, EvalShape> g_tune;

EvalShape tuned_shape(const EvalParams& p) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(TuneKey{p.nx, p.ny, p.N, p.R});
    return it == g_tune.end() ? EvalShape{0, 0} : it->second;
}

int strip_outw(int R, int nw) { return kWgOwn * std::max(1, nw) - 2 * R; }

// shape.rows = 0: the tuned shape if one is recorded, else the default
// (workgroup or wavefront strips as the columns fit best, 256 rows halved
// while there are fewer than 16384 wavefronts, down to 32).
StripGeom strip_geom(const EvalParams& p, EvalShape shape = EvalShape{0, 0}, bool two_wave = true) {
    if (shape.rows <= 0) shape = tuned_shape(p);
    const int wnx = p.wx1 - p.wx0, wny = p.wy1 - p.wy0;
    // default: the kind that spends fewer lanes on the window's columns
    // (workgroup strips on a tie)
    auto lanes = [&](int w) { return (long long)(wnx + strip_outw(p.R, w) - 1) / strip_outw(p.R, w) * 64 * w; };
    int nw = shape.rows > 0 ? std::max(1, shape.nw) : kDefaultWaves;
    if (shape.rows <= 0)
        for (int w : {2, 1})
            if ((w != 2 || two_wave) && lanes(w) < lanes(nw)) nw = w;
    if (nw == 2 && !two_wave) nw = kDefaultWaves;
    const int outw = strip_outw(p.R, nw);
    StripGeom g{};
    g.nw = nw;
    g.n_sx = (wnx + outw - 1) / outw;
    auto work = [&](int r) { return (long long)p.N * g.n_sx * ((wny + r - 1) / r); };
    if (shape.rows > 0) {
        g.rows = shape.rows;
    } else {
        g.rows = kStripRows;
        while (g.rows > 32 && work(g.rows) * nw < 16384) g.rows /= 2;
    }
    g.n_sy = (wny + g.rows - 1) / g.rows;
    g.n_work = (int)work(g.rows);
    return g;
}

template <int R, int Q1 = -1, int Q0 = kNoZeroTaps>
pct_status launch_eval_strip(const float* ground, const float* ceil, const EvalParams& p, float* cost, hipStream_t s,
                             const StripGeom& sg, unsigned* slice_bits) {
    const int blocks = (sg.n_work + 7) / 8 * 8;
    if (sg.nw == kDefaultWaves)
        hipLaunchKernelGGL((k_eval_strip<R, Q1, Q0, kDefaultWaves>), dim3(blocks), dim3(64 * kDefaultWaves), 0, s,
                           ground, ceil, p, cost, sg, slice_bits);
    else if (sg.nw == 2)
        hipLaunchKernelGGL((k_eval_strip<R, Q1, Q0, 2>), dim3(blocks), dim3(128), 0, s, ground, ceil, p, cost, sg,
                           slice_bits);
    else
        hipLaunchKernelGGL((k_eval_strip<R, Q1, Q0, 1>), dim3(blocks), dim3(64), 0, s, ground, ceil, p, cost, sg,
                           slice_bits);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

template <int R>
size_t eval_lds(int rp) {
    const int HG = R + rp + 1, HF = R + rp;
    const int WG = TW + 2 * HG, HGt = TH + 2 * HG;
    const int WF = TW + 2 * HF, HFt = TH + 2 * HF;
    const int WC = TW + 2 * R, HC = TH + 2 * R;
    return sizeof(float) * ((size_t)WG * HGt + (size_t)WC * HC + (size_t)(R + 1) * TH * WC) + (size_t)WF * HFt;
}

template <int R>
pct_status launch_eval_r(const float* ground, const float* ceil, const EvalParams& p, float* cost, hipStream_t s) {
    const size_t lds = eval_lds<R>(p.rp);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_eval<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return fail(PCT_ERR_DEVICE, "eval LDS request of %zu bytes refused: %s", lds, hipGetErrorString(e));
    }
    dim3 grid((p.wx1 - p.wx0 + TW - 1) / TW, (p.wy1 - p.wy0 + TH - 1) / TH, p.N);
    hipLaunchKernelGGL(k_eval<R>, grid, dim3(kBlock), lds, s, ground, ceil, p, cost);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

// ------------------------------------------------------------ simplification
//
// The slice test compares slice k with the last kept slice p, which depends
// on earlier decisions.  Per cell, the "differs from below" condition of
// Eq. (8) holds for every p before the run of slices whose ground equals
// e^G_k (ground is non-decreasing in k), and inside that run only where
// c_k < c_p.  The flags kernel therefore records, for every k, the largest
// run start over the cells that are traversable and satisfy Eq. (9), and a
// bit matrix of the in-run slices p with c_p > c_k.  The sequential chain
// then runs over these N x N bits (one wavefront for a single map, one
// thread per job in a batch).

// Reductions over a whole wavefront (every lane active) by DPP moves:
// row_shr 1, 2, 4, 8 leave each row's result in its lane 15, row_bcast:15
// into rows 1 and 3 and row_bcast:31 into rows 2 and 3 leave the
// wavefront's in lane 63.  Lanes whose source is outside their row, and
// rows outside the row mask, take the identity `id` instead.
template <class Op>
__device__ __forceinline__ int wave_reduce_dpp(int v, int id, Op op) {
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = op(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_max_i(int v) {
    return wave_reduce_dpp(v, INT_MIN, [](int a, int b) { return max(a, b); });
}
__device__ __forceinline__ int wave_min_i(int v) {
    return wave_reduce_dpp(v, INT_MAX, [](int a, int b) { return min(a, b); });
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
    return (unsigned)wave_reduce_dpp((int)v, 0, [](int a, int b) { return a | b; });
}

__global__ __launch_bounds__(kBlock) void k_simp_init(int* __restrict__ maxp0, unsigned* __restrict__ urun,
                                                      unsigned* __restrict__ slice_bits, int N, int W,
                                                      int copies, int cstride) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N * W; i += gridDim.x * kBlock) urun[i] = 0u;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < copies * cstride; i += gridDim.x * kBlock) maxp0[i] = -1;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < W; i += gridDim.x * kBlock) slice_bits[i] = 0u;
}

// Slice-test flags of kSimpCells cells per lane, cells cell0 + c * STRIDE
// for c < nact (nact <= kSimpCells; all lanes of a wavefront must call it
// together, lanes without cells pass nact = 0).  Several cells per lane
// divide the wavefront reductions and atomics per cell; STRIDE = 64
// interleaves the lanes of a wavefront, so that each load instruction reads
// 256 contiguous bytes.
//
// slice_bits (nullable): bit k set when slice k has a traversable cell.  A
// slice without one has no cell that Eqs. (8)-(9) can make unique, so it
// is passed over without reading; the cells' run starts are then followed
// across it lazily: a later slice with the ground of the last slice read
// continues that run (ground is non-decreasing in k), any other starts a
// run whose start is found, if a kept-slice test needs it, by reading the
// ground below.
constexpr int kSimpCells = 2;

template <int STRIDE>
__device__ __forceinline__ void simp_flags_cells(const float* __restrict__ ground, const float* __restrict__ cost,
                                                 long long plane, int N, float cB, int W, int* __restrict__ maxp0,
                                                 unsigned* __restrict__ urun, long long cell0, int nact,
                                                 const unsigned* __restrict__ slice_bits = nullptr,
                                                 int copies = 1, int cstride = 0) {
    constexpr int CPT = kSimpCells;
    const int lane = threadIdx.x & 63;
    // the largest run starts go to one of `copies` copies of maxp0 (cstride
    // ints apart, on separate cache lines), by wavefront: thousands of
    // wavefronts reach each slice together, and atomics on one line queue
    // behind each other
    maxp0 += (int)((((long long)blockIdx.x * kBlock + threadIdx.x) >> 6) % copies) * cstride;
    // bit j of sb0 / sb1: slice 32 * (k / 32) + j / + 32 + j holds a traversable cell
    auto bits_word = [&](int w) -> unsigned {   // uniform
        if (!slice_bits) return ~0u;
        return w < W ? slice_bits[w] : 0u;
    };
    unsigned sb0 = bits_word(0), sb1 = bits_word(1);
    // slice j is read when bit j is set; j < 32 (k / 32) + 64
    auto bit_of = [&](int j, int kw) -> bool {   // uniform; kw = 32 (k / 32)
        if (j >= N) return false;
        const int o = j - kw;
        return ((o < 32 ? sb0 >> o : sb1 >> (o - 32)) & 1u) != 0u;
    };
    // ring of the slices read ahead: slot j % Q holds ground and cost of
    // slice j at the lane's cells, loaded Q - 1 slices before slice j is
    // tested, so that loads of several slices are in flight.  The loads are
    // unconditional (clamped addresses, masks applied where the values are
    // used), so each step issues the same number and a wait for an older
    // slot need not drain the newer ones.
    constexpr int Q = 4;
    float eQ[Q][CPT], cQ[Q][CPT];
    long long cidx[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) cidx[c] = min(cell0 + (long long)c * STRIDE, plane - 1);
    auto load_slot = [&](int slot, int j) {
        const long long base = (long long)min(j, N - 1) * plane;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            eQ[slot][c] = ground[base + cidx[c]];
            cQ[slot][c] = cost[base + cidx[c]];
        }
    };
    if (slice_bits) {   // uniform: no marked slice at all
        unsigned any = 0u;
        for (int w = 0; w < W; ++w) any |= slice_bits[w];
        if (any == 0u) return;
    }
#pragma unroll
    for (int q = 0; q < Q - 1; ++q) load_slot(q, q);
    // per cell: ground of the last slice read, start of its run (-1: below
    // k, not known), and the largest cost of the run's slices below k (an
    // in-run slice can only make k unique where it costs more than c_k)
    float eprev[CPT], rmax[CPT];
    int p0[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        eprev[c] = -INFINITY;
        rmax[c] = -INFINITY;
        p0[c] = 0;
    }
    bool prev_read = false;   // slice k-1 was read (uniform)
    for (int kb = 0; kb < N; kb += Q) {
        if ((kb & 31) == 0 && kb > 0) {   // the next pair of words
            sb0 = sb1;
            sb1 = bits_word((kb >> 5) + 1);
        }
        const int kw = kb & ~31;
        if ((kb & 31) == 0 && sb0 == 0u) {   // uniform: no traversable cell in these 32 slices
            prev_read = false;
            if (sb1 != 0u) {   // the ring for the next word
#pragma unroll
                for (int q = 0; q < Q - 1; ++q) load_slot(q, kb + 32 + q);
            }
            kb += 32 - Q;
            continue;
        }
#pragma unroll
        for (int ph = 0; ph < Q; ++ph) {
            const int k = kb + ph;
            if (k >= N) break;   // uniform
            load_slot((ph + Q - 1) % Q, k + Q - 1);   // slice k + Q - 1 into the slot of slice k - 1
            if (!bit_of(k, kw)) {   // uniform: no traversable cell in slice k
                prev_read = false;
                continue;
            }
            float ek[CPT], ck[CPT], ek1[CPT], ck1[CPT];
            // slice k+1 (Eq. (9)); without a traversable cell its costs are c^B
            const bool rk1 = bit_of(k + 1, kw);
            const int s1 = (ph + 1) % Q;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const bool act = c < nact;
                ek[c] = act ? eQ[ph][c] : -INFINITY;
                ck[c] = act ? cQ[ph][c] : cB;
                ek1[c] = act && rk1 ? eQ[s1][c] : -INFINITY;
                ck1[c] = act && rk1 ? cQ[s1][c] : cB;
            }
            int mloc = -1, pminloc = 0x7fffffff;
            bool runA[CPT];
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                if (k > 0 && ek[c] != eprev[c]) {
                    // a new run: it starts at k when slice k-1 was read, else
                    // below k at a slice not known yet, whose costs are not known
                    p0[c] = prev_read ? k : -1;
                    rmax[c] = prev_read ? -INFINITY : cB;
                } else if (!prev_read && k > 0) {
                    rmax[c] = cB;   // the run continues over slices without a traversable cell (cost c^B)
                }
                const bool trav = c < nact && ck[c] < cB;
                const bool upper = (k == N - 1) || !rk1 || (ek1[c] > ek[c]) || (ck[c] < ck1[c]);
                const bool A = trav && upper;
                if (A && p0[c] < 0) {   // the run start: the lowest slice with this ground
                    int q = k;
                    while (q > 0 && ground[(long long)(q - 1) * plane + cell0 + c * STRIDE] == ek[c]) --q;
                    p0[c] = q;
                }
                if (A) mloc = max(mloc, p0[c]);
                runA[c] = A && p0[c] < k && rmax[c] > ck[c];
                if (runA[c]) pminloc = min(pminloc, p0[c]);
                rmax[c] = fmaxf(rmax[c], ck[c]);
            }
            if (__ballot(mloc >= 0)) {
                const int m = wave_max_i(mloc);
                if (lane == 0) atomicMax(&maxp0[k], m);
            }
            if (__ballot(pminloc != 0x7fffffff)) {
                const int pmin = wave_min_i(pminloc);
                for (int w = pmin / 32; w <= (k - 1) / 32; ++w) {
                    unsigned bits = 0;
                    const int pb = max(pmin, w * 32), pe = min(k, w * 32 + 32);
                    // eight earlier slices at a time, their loads issued together
                    for (int pp0 = pb; pp0 < pe; pp0 += 8) {
                        float cv[8][CPT];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int pp = pp0 + u;
#pragma unroll
                            for (int c = 0; c < CPT; ++c)
                                cv[u][c] = (pp < pe && runA[c] && pp >= p0[c])
                                               ? cost[(long long)pp * plane + cell0 + c * STRIDE]
                                               : -INFINITY;
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
#pragma unroll
                            for (int c = 0; c < CPT; ++c)
                                if (cv[u][c] > ck[c]) bits |= 1u << (pp0 + u - w * 32);
                        }
                    }
                    bits = wave_or(bits);
                    if (lane == 0 && bits) atomicOr(&urun[(long long)k * W + w], bits);
                }
            }
#pragma unroll
            for (int c = 0; c < CPT; ++c) eprev[c] = ek[c];
            prev_read = true;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_simp_flags(const float* __restrict__ ground, const float* __restrict__ cost,
                                                       const int nx, const int ny, const int N, const float cB,
                                                       const int W, int* __restrict__ maxp0, unsigned* __restrict__ urun,
                                                       const unsigned* __restrict__ slice_bits, int copies,
                                                       int cstride) {
    const long long plane = (long long)nx * ny;
    // the wavefront's 64 x kSimpCells cells, lane-interleaved
    const long long wave0 = ((long long)blockIdx.x * kBlock + (threadIdx.x & ~63)) * kSimpCells;
    const long long cell0 = wave0 + (threadIdx.x & 63);
    const long long left = plane - cell0;
    const int nact = left <= 0 ? 0 : (int)std::min<long long>(kSimpCells, (left + 63) / 64);
    simp_flags_cells<64>(ground, cost, plane, N, cB, W, maxp0, urun, nact > 0 ? cell0 : 0, nact, slice_bits, copies,
                         cstride);
}

__device__ void keep_chain(const int* __restrict__ maxp0, const unsigned* __restrict__ urun, int N, int W,
                           uint8_t* __restrict__ keep) {
    int p = -1;
    for (int k = 0; k < N; ++k) {
        const int m = maxp0[k];
        bool u;
        if (p < 0) u = m >= 0;
        else u = p < m || ((urun[(long long)k * W + p / 32] >> (p % 32)) & 1u);
        keep[k] = u ? 1 : 0;
        if (u) p = k;
    }
}

// One wavefront: the copies of the run starts merged per slice, then the
// chain 64 slices at a time.  With p the last kept slice, the lanes test
// the next 64 slices against p together; the first that passes is kept and
// those before it are not (each would have been tested against the same
// p), and the next step starts after it.  Steps: one per kept slice and
// one per 64 slices, instead of one per slice.
__global__ __launch_bounds__(64) void k_keep_chain(const int* __restrict__ maxp0, const unsigned* __restrict__ urun,
                                                   int N, int W, uint8_t* __restrict__ keep, int copies, int cstride) {
    __shared__ int s_m[PCT_MAX_SLICES];
    const int lane = threadIdx.x;
    for (int k = lane; k < N; k += 64) {
        int m = maxp0[k];
        for (int c = 1; c < copies; ++c) m = max(m, maxp0[c * cstride + k]);
        s_m[k] = m;
    }
    __syncthreads();
    int p = -1, k0 = 0;   // uniform
    while (k0 < N) {
        const int k = k0 + lane;
        bool u = false;
        if (k < N) {
            const int m = s_m[k];
            u = p < 0 ? m >= 0 : (p < m || ((urun[(long long)k * W + p / 32] >> (p % 32)) & 1u) != 0u);
        }
        const unsigned long long b = __ballot(u);
        const int f = b ? __ffsll((long long)b) - 1 : 64;   // the first kept lane, 64: none
        if (k < N && lane <= f) keep[k] = lane == f ? 1 : 0;
        if (f < 64) {
            p = k0 + f;
            k0 = p + 1;
        } else {
            k0 += 64;
        }
    }
}

// ---- batched slice test: one workgroup per job for the init and chain,
// job cell ranges padded to whole wavefronts for the flags

__device__ __forceinline__ int find_job_cell(const EvalJob* __restrict__ jobs, int n_jobs, long long c) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].cell_base <= c) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_simp_init_jobs(const EvalJob* __restrict__ jobs, char* __restrict__ ws) {
    const EvalJob& jb = jobs[blockIdx.x];
    const int N = jb.p.N, W = (N + 31) / 32;
    const JobScratch js = job_scratch(ws, jb);
    for (int i = threadIdx.x; i < N * W; i += kBlock) js.urun[i] = 0u;
    for (int i = threadIdx.x; i < N; i += kBlock) js.maxp0[i] = -1;
    for (int i = threadIdx.x; i < W; i += kBlock) js.marks[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void k_simp_flags_jobs(const float* __restrict__ ground,
                                                            const float* __restrict__ cost,
                                                            const EvalJob* __restrict__ jobs, int n_jobs,
                                                            char* __restrict__ ws, int marked) {
    // global padded cell of this lane's first cell; a wavefront's 64 x kSimpCells
    // cells never span two jobs (job ranges are padded to that)
    const long long wave0 = ((long long)blockIdx.x * kBlock + (threadIdx.x & ~63)) * kSimpCells;
    const int j = __builtin_amdgcn_readfirstlane(find_job_cell(jobs, n_jobs, wave0));
    const EvalJob& jb = jobs[j];
    // the wavefront's cells, lane-interleaved as in the single-map kernel
    const long long cell0 = wave0 - jb.cell_base + (threadIdx.x & 63);
    const long long left = jb.p.plane - cell0;
    const int nact = (cell0 < 0 || left <= 0) ? 0 : (int)std::min<long long>(kSimpCells, (left + 63) / 64);
    const int N = jb.p.N, W = (N + 31) / 32;
    const JobScratch js = job_scratch(ws, jb);
    // marked: the evaluation marked the slices with a traversable cell
    simp_flags_cells<64>(ground + jb.in_off, cost + jb.out_off, jb.p.plane, N, jb.p.cB, W, js.maxp0, js.urun,
                         nact > 0 ? cell0 : 0, nact, marked ? js.marks : nullptr);
}

__global__ void k_keep_chain_jobs(const EvalJob* __restrict__ jobs, int n_jobs, const char* __restrict__ ws,
                                  uint8_t* __restrict__ keep) {
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= n_jobs) return;
    const EvalJob& jb = jobs[j];
    const int N = jb.p.N, W = (N + 31) / 32;
    const JobScratch js = job_scratch(const_cast<char*>(ws), jb);
    keep_chain(js.maxp0, js.urun, N, W, keep + jb.keep_off);
}

}  // namespace

// The single-map slice test's scratch: the N x N bit matrix, the slice
// marks, then `copies` copies of the largest run starts, 4 KB apart.
constexpr int kRunStartCopies = 16;
inline size_t run_start_stride(int N) { return align_up(sizeof(int) * (size_t)N, 4096); }
inline size_t simp_base_bytes(int N) {
    const int W = (N + 31) / 32;
    return align_up(sizeof(unsigned) * (size_t)N * W) + align_up(sizeof(unsigned) * (size_t)W);
}

size_t eval_ws_bytes(int N, int) { return simp_base_bytes(N) + kRunStartCopies * run_start_stride(N); }
size_t eval_ws_min_bytes(int N) { return simp_base_bytes(N) + run_start_stride(N); }

// The compiled tap-weight patterns: for radius R >= 2, weight exactly 1 for
// a^2 + j^2 <= (R-2)^2 and exactly 0 for a^2 + j^2 >= (R+1)^2 (an inflation
// radius of R-2 cells with a 3-cell margin, as a 0.1 m grid with a 0.4 m
// smoothing distance gives).  True when p's weights follow it exactly.
static bool weights_follow_pattern(const EvalParams& p) {
    const int R = p.R;
    if (R < 2 || R > 8) return false;
    const int q1 = (R - 2) * (R - 2), q0 = (R + 1) * (R + 1);
    for (int a = 0; a <= R; ++a)
        for (int j = 0; j <= R; ++j) {
            const int q = a * a + j * j;
            if (q <= q1 && p.K[a][j] != 1.0f) return false;
            if (q >= q0 && p.K[a][j] != 0.0f) return false;
        }
    return true;
}

// Strip kernels: patch radius 1, inflation radius <= 8, and slice planes
// small enough for 32-bit buffer offsets.
bool strip_kernel_applies(const EvalParams& p) { return p.rp == 1 && p.R <= 8 && p.plane < (1LL << 29); }

namespace {

// The strip evaluation with geometry sg (slice_bits: nullable, the slices
// with a traversable cell), or the tiled kernel where the strips do not
// apply (which leaves slice_bits alone).
pct_status launch_eval_geom(const float* ground, const float* ceil, const EvalParams& p, float* cost, hipStream_t s,
                            const StripGeom& sg, unsigned* slice_bits) {
    if (strip_kernel_applies(p)) {
        if (weights_follow_pattern(p)) {
            switch (p.R) {
#define PCT_P(r) case r: return launch_eval_strip<r, (r - 2) * (r - 2), (r + 1) * (r + 1)>(ground, ceil, p, cost, s, sg, slice_bits);
                PCT_P(2) PCT_P(3) PCT_P(4) PCT_P(5) PCT_P(6) PCT_P(7) PCT_P(8)
#undef PCT_P
                default: break;
            }
        }
        switch (p.R) {
#define PCT_S(r) case r: return launch_eval_strip<r>(ground, ceil, p, cost, s, sg, slice_bits);
            PCT_S(0) PCT_S(1) PCT_S(2) PCT_S(3) PCT_S(4) PCT_S(5) PCT_S(6) PCT_S(7) PCT_S(8)
#undef PCT_S
            default: break;
        }
    }
    switch (p.R) {
#define PCT_R(r) case r: return launch_eval_r<r>(ground, ceil, p, cost, s);
        PCT_R(0) PCT_R(1) PCT_R(2) PCT_R(3) PCT_R(4) PCT_R(5) PCT_R(6) PCT_R(7) PCT_R(8)
        PCT_R(9) PCT_R(10) PCT_R(11) PCT_R(12) PCT_R(13) PCT_R(14) PCT_R(15) PCT_R(16)
#undef PCT_R
        default: return fail(PCT_ERR_CAPACITY, "inflation radius %d exceeds %d", p.R, PCT_MAX_KERNEL_RADIUS);
    }
}

}  // namespace

pct_status launch_eval(const float* ground, const float* ceil, const EvalParams& p, float* cost, hipStream_t s,
                       EvalShape shape) {
    const StripGeom sg = strip_kernel_applies(p) ? strip_geom(p, shape) : StripGeom{};
    return launch_eval_geom(ground, ceil, p, cost, s, sg, nullptr);
}

// Times the strip evaluation of this map shape for each candidate shape
// (one wavefront per strip, or kDefaultWaves per workgroup, by strip
// height) and records the fastest in the tuning table (synchronous).
pct_status autotune_eval(const float* ground, const float* ceil, const EvalParams& p, float* cost, hipStream_t s,
                         EvalShape* best_shape, EvalShape* cand, float* cand_ms, int n_max, int* n_cand) {
    *best_shape = EvalShape{0, 0};
    *n_cand = 0;
    if (!strip_kernel_applies(p)) return PCT_OK;   // the tiled kernel has no strip shape
    EvalShape shapes[24];
    int nc = 0;
    for (int nw : {kDefaultWaves, 2, 1})
        for (int r = 32; r <= 1024 && nc < 24; r *= 2) {
            if (!strip_shape_fits(p, EvalShape{r, nw})) continue;
            shapes[nc++] = EvalShape{r, nw};
            if (r >= p.ny) break;
        }
    hipEvent_t e0, e1;
    PCT_HIP(hipEventCreate(&e0));
    PCT_HIP(hipEventCreate(&e1));
    float best = INFINITY;
    pct_status st = PCT_OK;
    for (int i = 0; i < nc && st == PCT_OK; ++i) {
        st = launch_eval(ground, ceil, p, cost, s, shapes[i]);   // warm-up
        if (st != PCT_OK) break;
        if (hipEventRecord(e0, s) != hipSuccess) { st = fail(PCT_ERR_DEVICE, "hipEventRecord failed"); break; }
        for (int rep = 0; rep < 3 && st == PCT_OK; ++rep) st = launch_eval(ground, ceil, p, cost, s, shapes[i]);
        if (st != PCT_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = fail(PCT_ERR_DEVICE, "timing the candidates failed");
            break;
        }
        ms /= 3.0f;
        if (i < n_max) {
            if (cand) cand[i] = shapes[i];
            if (cand_ms) cand_ms[i] = ms;
        }
        if (ms < best) {
            best = ms;
            *best_shape = shapes[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PCT_OK) return st;
    *n_cand = nc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[TuneKey{p.nx, p.ny, p.N, p.R}] = *best_shape;
    return PCT_OK;
}

// Batch tables, per size class (ceil(log2 nx), ceil(log2 ny)): the
// evaluation's strip shape (and kernel radius) and the construction's tile
// height.
struct ClassKey {
    int cx, cy, R;
    bool operator<(const ClassKey& o) const {
        return cx != o.cx ? cx < o.cx : cy != o.cy ? cy < o.cy : R < o.R;
    }
};
std::map<ClassKey, EvalShape> g_batch_eval;
std::map<ClassKey, int> g_batch_build;   // R = -1

int size_class(int v) {
    int c = 0;
    while (c < 31 && (1 << c) < v) ++c;
    return c;
}

EvalShape batch_eval_shape(int cx, int cy, int R) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_batch_eval.find(ClassKey{cx, cy, R});
    return it == g_batch_eval.end() ? EvalShape{0, 0} : it->second;
}

void set_batch_eval_shape(int cx, int cy, int R, EvalShape shape) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (shape.rows > 0) g_batch_eval[ClassKey{cx, cy, R}] = shape;
    else g_batch_eval.erase(ClassKey{cx, cy, R});
}

int batch_build_th(int cx, int cy) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_batch_build.find(ClassKey{cx, cy, -1});
    return it == g_batch_build.end() ? 0 : it->second;
}

void set_batch_build_th(int cx, int cy, int th) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (th > 0) g_batch_build[ClassKey{cx, cy, -1}] = th;
    else g_batch_build.erase(ClassKey{cx, cy, -1});
}

void autotune_reset() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    g_batch_eval.clear();
    g_batch_build.clear();
}

void batch_strip_signature(const EvalParams& p, EvalShape shape, int out[4]) {
    const StripGeom g = strip_geom(p, shape.rows > 0 ? shape : batch_eval_shape(size_class(p.nx), size_class(p.ny), p.R),
                                   false);
    out[0] = g.nw;
    out[1] = g.n_sx;
    out[2] = g.n_sy;
    out[3] = g.n_sy > 1 ? g.rows : 0;   // one strip row: the height does not matter
}

// Text form of the tables, one record a line, for the current device's
// architecture `arch`:
//   <arch> map <nx> <ny> <N> <R> <rows> <waves>
//   <arch> batch_eval <cx> <cy> <R> <rows> <waves>
//   <arch> batch_build <cx> <cy> <th>
// Lines starting with '#' are comments.
pct_status tune_save(const char* path, const char* arch) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE* fp = fopen(path, "w");
    if (!fp) return fail(PCT_ERR_ARG, "cannot write %s", path);
    fprintf(fp, "# libpct tuning tables v1\n");
    for (const auto& kv : g_tune)
        fprintf(fp, "%s map %d %d %d %d %d %d\n", arch, kv.first.nx, kv.first.ny, kv.first.N, kv.first.R,
                kv.second.rows, kv.second.nw);
    for (const auto& kv : g_batch_eval)
        fprintf(fp, "%s batch_eval %d %d %d %d %d\n", arch, kv.first.cx, kv.first.cy, kv.first.R, kv.second.rows,
                kv.second.nw);
    for (const auto& kv : g_batch_build)
        fprintf(fp, "%s batch_build %d %d %d\n", arch, kv.first.cx, kv.first.cy, kv.second);
    const bool bad = ferror(fp) != 0;
    if (fclose(fp) != 0 || bad) return fail(PCT_ERR_ARG, "writing %s failed", path);
    return PCT_OK;
}

pct_status tune_load(const char* path, const char* arch, int* n_applied) {
    FILE* fp = fopen(path, "r");
    if (!fp) return fail(PCT_ERR_ARG, "cannot read %s", path);
    std::map<TuneKey, EvalShape> m;
    std::map<ClassKey, EvalShape> be;
    std::map<ClassKey, int> bb;
    char line[512];
    int ln = 0;
    pct_status st = PCT_OK;
    while (fgets(line, sizeof line, fp)) {
        ++ln;
        char a[256], kind[32];
        int v[6], used = 0;
        if (line[0] == '#' || line[0] == '\n') continue;
        if (sscanf(line, "%255s %31s%n", a, kind, &used) != 2) { st = fail(PCT_ERR_ARG, "%s:%d: malformed", path, ln); break; }
        const char* rest = line + used;
        const bool mine = strcmp(a, arch) == 0;
        if (strcmp(kind, "map") == 0) {
            if (sscanf(rest, "%d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) != 6 || v[0] < 1 ||
                v[1] < 1 || v[0] > PCT_MAX_GRID_SIDE || v[1] > PCT_MAX_GRID_SIDE || v[2] < 1 || v[2] > PCT_MAX_SLICES ||
                v[3] < 0 || v[3] > PCT_MAX_KERNEL_RADIUS || v[4] < 16 || v[4] > PCT_MAX_STRIP_ROWS ||
                (v[5] != 1 && v[5] != 2 && v[5] != 4)) {
                st = fail(PCT_ERR_ARG, "%s:%d: bad map record", path, ln);
                break;
            }
            if (mine) m[TuneKey{v[0], v[1], v[2], v[3]}] = EvalShape{v[4], v[5]};
        } else if (strcmp(kind, "batch_eval") == 0) {
            if (sscanf(rest, "%d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4]) != 5 || v[0] < 0 || v[0] > 16 ||
                v[1] < 0 || v[1] > 16 || v[2] < 0 || v[2] > PCT_MAX_KERNEL_RADIUS || v[3] < 16 ||
                v[3] > PCT_MAX_STRIP_ROWS || (v[4] != 1 && v[4] != 4)) {
                st = fail(PCT_ERR_ARG, "%s:%d: bad batch_eval record", path, ln);
                break;
            }
            if (mine) be[ClassKey{v[0], v[1], v[2]}] = EvalShape{v[3], v[4]};
        } else if (strcmp(kind, "batch_build") == 0) {
            if (sscanf(rest, "%d %d %d", &v[0], &v[1], &v[2]) != 3 || v[0] < 0 || v[0] > 16 || v[1] < 0 || v[1] > 16 ||
                (v[2] != 2 && v[2] != 4 && v[2] != 8)) {
                st = fail(PCT_ERR_ARG, "%s:%d: bad batch_build record", path, ln);
                break;
            }
            if (mine) bb[ClassKey{v[0], v[1], -1}] = v[2];
        } else {
            st = fail(PCT_ERR_ARG, "%s:%d: unknown record '%s'", path, ln, kind);
            break;
        }
    }
    fclose(fp);
    if (st != PCT_OK) return st;   // nothing applied
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : m) g_tune[kv.first] = kv.second;
    for (const auto& kv : be) g_batch_eval[kv.first] = kv.second;
    for (const auto& kv : bb) g_batch_build[kv.first] = kv.second;
    if (n_applied) *n_applied = (int)(m.size() + be.size() + bb.size());
    return PCT_OK;
}

bool strip_shape_fits(const EvalParams& p, EvalShape shape) {
    const long long outw = strip_outw(p.R, shape.nw);
    if (outw <= 0 || shape.rows <= 0) return false;
    const long long wnx = p.wx1 - p.wx0, wny = p.wy1 - p.wy0;
    const long long work = (long long)p.N * ((wnx + outw - 1) / outw) * ((wny + shape.rows - 1) / shape.rows);
    return work * std::max(1, shape.nw) <= (1LL << 30);
}

void autotune_set(const EvalParams& p, EvalShape shape) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (shape.rows > 0) g_tune[TuneKey{p.nx, p.ny, p.N, p.R}] = shape;
    else g_tune.erase(TuneKey{p.nx, p.ny, p.N, p.R});
}

namespace {

// The slice test's scratch: per-slice largest run start, the N x N bit
// matrix (W words per slice) and the bits of the slices with a traversable
// cell.
struct SimpScratch {
    int* maxp0;
    unsigned* urun;
    unsigned* slice_bits;
    int W, copies, cstride;
};

// ws_bytes >= eval_ws_min_bytes(N): as many copies of the run starts as fit, up to 16
SimpScratch simp_scratch(void* ws, int N, size_t ws_bytes) {
    SimpScratch sc;
    sc.W = (N + 31) / 32;
    sc.urun = (unsigned*)ws;
    sc.slice_bits = (unsigned*)((char*)ws + align_up(sizeof(unsigned) * (size_t)N * sc.W));
    sc.maxp0 = (int*)((char*)ws + simp_base_bytes(N));
    const size_t stride = run_start_stride(N);
    sc.copies = (int)std::max<size_t>(1, std::min<size_t>(kRunStartCopies, (ws_bytes - simp_base_bytes(N)) / stride));
    sc.cstride = (int)(stride / sizeof(int));
    return sc;
}

// Flags and chain over a cleared scratch (slice_bits: nullable).
pct_status launch_simp_flags(const float* ground, const float* cost, const EvalParams& p, uint8_t* keep,
                             const SimpScratch& sc, const unsigned* slice_bits, hipStream_t s) {
    const long long blocks = (p.plane + (long long)kBlock * kSimpCells - 1) / ((long long)kBlock * kSimpCells);
    hipLaunchKernelGGL(k_simp_flags, dim3((unsigned)blocks), dim3(kBlock), 0, s, ground, cost, p.nx, p.ny, p.N, p.cB,
                       sc.W, sc.maxp0, sc.urun, slice_bits, sc.copies, sc.cstride);
    PCT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_keep_chain, dim3(1), dim3(64), 0, s, sc.maxp0, sc.urun, p.N, sc.W, keep, sc.copies,
                       sc.cstride);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

}  // namespace

pct_status launch_simplify(const float* ground, const float* cost, const EvalParams& p, uint8_t* keep, void* ws,
                           size_t ws_bytes, hipStream_t s) {
    SimpScratch sc = simp_scratch(ws, p.N, ws_bytes);
    hipLaunchKernelGGL(k_simp_init, dim3(std::max(1, std::min(1024, (p.N * sc.W + kBlock - 1) / kBlock))), dim3(kBlock),
                       0, s, sc.maxp0, sc.urun, sc.slice_bits, p.N, sc.W, sc.copies, sc.cstride);
    PCT_LAUNCH_CHECK();
    return launch_simp_flags(ground, cost, p, keep, sc, nullptr, s);
}

// Evaluation of one robot on the whole map or a window, then (keep
// non-null) the slice test.  On a whole map the strip kernels mark the
// slices that hold a traversable cell, and the slice test passes over the
// others without reading them.
pct_status launch_eval_simplify(const float* ground, const float* ceil, const EvalParams& p, float* cost, uint8_t* keep,
                                void* ws, size_t ws_bytes, hipStream_t s) {
    if (!keep) return launch_eval(ground, ceil, p, cost, s);
    const bool whole = p.wx0 == 0 && p.wy0 == 0 && p.wx1 == p.nx && p.wy1 == p.ny;
    if (!(strip_kernel_applies(p) && whole)) {
        pct_status st = launch_eval(ground, ceil, p, cost, s);
        if (st != PCT_OK) return st;
        return launch_simplify(ground, cost, p, keep, ws, ws_bytes, s);
    }
    SimpScratch sc = simp_scratch(ws, p.N, ws_bytes);
    hipLaunchKernelGGL(k_simp_init, dim3(std::max(1, std::min(1024, (p.N * sc.W + kBlock - 1) / kBlock))), dim3(kBlock),
                       0, s, sc.maxp0, sc.urun, sc.slice_bits, p.N, sc.W, sc.copies, sc.cstride);
    PCT_LAUNCH_CHECK();
    pct_status st = launch_eval_geom(ground, ceil, p, cost, s, strip_geom(p), sc.slice_bits);
    if (st != PCT_OK) return st;
    return launch_simp_flags(ground, cost, p, keep, sc, sc.slice_bits, s);
}

// ------------------------------------------------------------ batches (host)

namespace {

struct JobPlan {
    std::vector<EvalJob> jobs;
    int n_blocks = 0;
    long long cells = 0;     // padded cells of all jobs
    size_t scratch = 0;      // bytes of slice-test scratch
    int R = -1;
    bool strip = true;       // every job can use the strip kernel with one R
    bool pattern = true;     // ... and every job's weights follow the compiled pattern
};

pct_status plan_jobs(const pct_item* items, int n_items, const pct_robot* robots, int n_robots, JobPlan* jp) {
    long long total_cells = 0, total_slices = 0;
    for (int i = 0; i < n_items; ++i) {
        total_cells = std::max<long long>(total_cells, items[i].out_offset +
                                                           (long long)items[i].extent.n_slices * items[i].grid.nx * items[i].grid.ny);
        total_slices = std::max<long long>(total_slices, items[i].keep_offset + items[i].extent.n_slices);
    }
    for (int r = 0; r < n_robots; ++r)
        for (int i = 0; i < n_items; ++i) {
            const int N = items[i].extent.n_slices;
            if (N <= 0) continue;
            EvalJob jb{};
            pct_status st = make_eval_params(robots[r], items[i].grid, N, &jb.p);
            if (st != PCT_OK) return st;
            // blocks of kBlock threads: 1 or 4 wavefronts; the size class's
            // tuned shape if one is recorded
            jb.sg = strip_geom(jb.p, batch_eval_shape(size_class(jb.p.nx), size_class(jb.p.ny), jb.p.R), false);
            jb.in_off = items[i].out_offset;
            jb.out_off = (long long)r * total_cells + items[i].out_offset;
            jb.keep_off = (long long)r * total_slices + items[i].keep_offset;
            jb.cell_base = jp->cells;
            jb.ws_off = (long long)jp->scratch;
            jb.block_base = jp->n_blocks;
            jb.n_blocks = jb.sg.nw > 1 ? jb.sg.n_work : (jb.sg.n_work + kBlock / 64 - 1) / (kBlock / 64);
            jp->cells += (jb.p.plane + 64 * kSimpCells - 1) / (64 * kSimpCells) * (64 * kSimpCells);
            jp->scratch += job_scratch_bytes(N);
            jp->n_blocks += jb.n_blocks;
            if (jp->R < 0) jp->R = jb.p.R;
            if (jb.p.R != jp->R || !strip_kernel_applies(jb.p)) jp->strip = false;
            if (!weights_follow_pattern(jb.p)) jp->pattern = false;
            jp->jobs.push_back(jb);
        }
    return PCT_OK;
}

template <int R, int Q1 = -1, int Q0 = kNoZeroTaps>
pct_status launch_jobs_r(const float* ground, const float* ceil, const EvalJob* d_jobs, int n_jobs, int n_blocks,
                         float* cost, char* marks_ws, hipStream_t s) {
    const int blocks = (n_blocks + 7) / 8 * 8;
    hipLaunchKernelGGL((k_eval_strip_jobs<R, Q1, Q0>), dim3(blocks), dim3(kBlock), 0, s, ground, ceil, d_jobs, n_jobs,
                       n_blocks, cost, marks_ws);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

}  // namespace

size_t batch_eval_ws_bytes(const pct_item* items, int n_items, int n_robots) {
    std::vector<pct_robot> rs(n_robots);
    for (auto& r : rs) {
        r = pct_robot{};
        r.d_sm = 1.0f;
        r.patch_radius = 1;
        r.c_barrier = 1.0f;
    }
    JobPlan jp;
    if (plan_jobs(items, n_items, rs.data(), n_robots, &jp) != PCT_OK) return 0;
    return align_up(sizeof(EvalJob) * jp.jobs.size()) + jp.scratch;
}

pct_status launch_eval_batched(const float* ground, const float* ceil, const pct_item* items, int n_items,
                               const pct_robot* robots, int n_robots, float* cost, uint8_t* keep, void* ws,
                               size_t ws_bytes, int upload, hipStream_t s) {
    JobPlan jp;
    pct_status st = plan_jobs(items, n_items, robots, n_robots, &jp);
    if (st != PCT_OK) return st;
    const int n_jobs = (int)jp.jobs.size();
    if (n_jobs == 0) return PCT_OK;
    const size_t need = align_up(sizeof(EvalJob) * n_jobs) + jp.scratch;
    if (!ws || ws_bytes < need) return fail(PCT_ERR_WORKSPACE, "batch eval workspace too small: %zu < %zu", ws_bytes, need);
    EvalJob* d_jobs = (EvalJob*)ws;
    char* scratch = (char*)ws + align_up(sizeof(EvalJob) * n_jobs);
    Digest dg;
    for (const EvalJob& jb : jp.jobs) {
        digest_params(dg, jb.p);
        dg.add(jb.sg.rows), dg.add(jb.sg.n_sx), dg.add(jb.sg.n_sy), dg.add(jb.sg.n_work), dg.add(jb.sg.nw);
        dg.add(jb.in_off), dg.add(jb.out_off), dg.add(jb.keep_off), dg.add(jb.cell_base), dg.add(jb.ws_off);
        dg.add(jb.block_base), dg.add(jb.n_blocks);
    }
    st = resident_tables(ws, 1, dg.h, upload != 0);
    if (st != PCT_OK) return st;
    if (upload) {
        // jp.jobs is released on return: wait until the copy has read it
        PCT_HIP(hipMemcpyAsync(d_jobs, jp.jobs.data(), sizeof(EvalJob) * n_jobs, hipMemcpyHostToDevice, s));
        PCT_HIP(hipStreamSynchronize(s));
    }
    // the slice test's scratch is cleared first: the strip kernels mark the
    // slices with a traversable cell in it
    if (keep) {
        hipLaunchKernelGGL(k_simp_init_jobs, dim3(n_jobs), dim3(kBlock), 0, s, d_jobs, scratch);
        PCT_LAUNCH_CHECK();
    }
    char* marks_ws = keep && jp.strip ? scratch : nullptr;
    if (jp.strip) {
        switch (jp.R) {
#define PCT_J(r)                                                                                       \
    case r:                                                                                            \
        st = (jp.pattern && r >= 2)                                                                    \
                 ? launch_jobs_r<r, (r - 2) * (r - 2), (r + 1) * (r + 1)>(ground, ceil, d_jobs, n_jobs, jp.n_blocks, cost, marks_ws, s) \
                 : launch_jobs_r<r>(ground, ceil, d_jobs, n_jobs, jp.n_blocks, cost, marks_ws, s);                 \
        break;
            PCT_J(0) PCT_J(1) PCT_J(2) PCT_J(3) PCT_J(4) PCT_J(5) PCT_J(6) PCT_J(7) PCT_J(8)
#undef PCT_J
            default: return fail(PCT_ERR_CAPACITY, "inflation radius %d", jp.R);
        }
        if (st != PCT_OK) return st;
    } else {
        // mixed radii or patch sizes: one launch per job
        for (const EvalJob& jb : jp.jobs) {
            st = launch_eval(ground + jb.in_off, ceil + jb.in_off, jb.p, cost + jb.out_off, s);
            if (st != PCT_OK) return st;
        }
    }
    if (keep) {
        hipLaunchKernelGGL(k_simp_flags_jobs, dim3((unsigned)((jp.cells + (long long)kBlock * kSimpCells - 1) /
                                                             ((long long)kBlock * kSimpCells))),
                           dim3(kBlock), 0, s,
                           ground, cost, d_jobs, n_jobs, scratch, marks_ws ? 1 : 0);
        PCT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_keep_chain_jobs, dim3((n_jobs + 63) / 64), dim3(64), 0, s, d_jobs, n_jobs, scratch, keep);
        PCT_LAUNCH_CHECK();
    }
    return PCT_OK;
}

}  // namespace pct
