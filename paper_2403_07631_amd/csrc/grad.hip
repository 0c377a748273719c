// Trajectory cost sampling and adjoints on gfx950.
//
// Sampling (the cost and height terms of the trajectory optimisation of
// Sec. III-E, Eq. (11)): a waypoint (x, y, z) on slice k contributes
//     f = C_k(x, y) + w_z (z - G_k(x, y) - d_ref)^2,
// with C_k, G_k cell-centred bilinear interpolations of c^T_k and e^G_k
// (clamped at the grid edge, zero slope across the clamp); the height term
// is dropped when a ground corner is missing; a trajectory sums its
// waypoints.  Waypoints with a non-finite coordinate or a slice outside
// [0, N) contribute nothing.
//
// Adjoints: bilinear weights scatter dL/dC and dL/dG to the four corners;
// the traversability adjoint routes dL/dc^T through the maximising tap of
// the Eq. (6) window (first maximum in row-major window order) into the
// Eq. (1)-(5) derivatives at that cell; the construction adjoint adds each
// ground/ceiling gradient to the z of the point that holds the value.  The
// maximising tap is found by recomputing c^init with the same FP32
// operation sequence as the forward kernels, so it reproduces the forward
// maximum exactly.
//
// Gradient sums: float atomics by default, whose result depends on the
// order in which the additions land; with PCT_FIXED_POINT, 64-bit integer
// atomics on contributions rounded to multiples of 2^-32, whose sum does
// not depend on that order (nor on how the work is split into launches).
#include <limits.h>

#include "pct_internal.h"

namespace pct {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ float sumsq(float dx, float dy) { return __builtin_fmaf(dx, dx, dy * dy); }

__device__ __forceinline__ float gval(const float* __restrict__ gk, int nx, int ny, int x, int y) {
    return (x >= 0 && y >= 0 && x < nx && y < ny) ? gk[(long long)y * nx + x] : -INFINITY;
}

__device__ bool gentle_at(const float* __restrict__ gk, int nx, int ny, int x, int y, const EvalParams& p) {
    const float G = gval(gk, nx, ny, x, y);
    const float l = gval(gk, nx, ny, x - 1, y), r = gval(gk, nx, ny, x + 1, y);
    const float d = gval(gk, nx, ny, x, y - 1), u = gval(gk, nx, ny, x, y + 1);
    if (!(isfinite(G) && isfinite(l) && isfinite(r) && isfinite(d) && isfinite(u))) return false;
    return sumsq(r - l, u - d) < p.Ts2;
}

struct Cinit {
    float ci, dx, dy, dI;
    int branch;   // 0 no ground, 1 barrier, 2 gentle, 3 step, 4 step without support
    bool ipos;    // interval term active: d^I >= d_min and alpha_d (d_ref - d^I) > 0
    bool pass;    // c^I + c^G < c^B (the clip of Eq. (5) is not active)
};

// c^init of cell (x, y) of one slice, Eqs. (1)-(5), with the values needed
// by its adjoint.  Same FP32 operation sequence as the forward kernels.
__device__ Cinit cinit_at(const float* __restrict__ gk, const float* __restrict__ ck, int x, int y,
                          const EvalParams& p) {
    const int nx = p.nx, ny = p.ny;
    Cinit o{};
    const float G = gk[(long long)y * nx + x];
    if (!isfinite(G)) {
        o.ci = p.cB;
        o.branch = 0;
        return o;
    }
    const float C = ck[(long long)y * nx + x];
    o.dI = C - G;
    const float cI = o.dI < p.d_min ? p.cB : fmaxf(0.0f, p.alpha_d * (p.d_ref - o.dI));
    o.ipos = !(o.dI < p.d_min) && p.alpha_d * (p.d_ref - o.dI) > 0.0f;
    const float l = gval(gk, nx, ny, x - 1, y), r = gval(gk, nx, ny, x + 1, y);
    const float d = gval(gk, nx, ny, x, y - 1), u = gval(gk, nx, ny, x, y + 1);
    float cG = p.cB;
    o.branch = 1;
    if (isfinite(l) && isfinite(r) && isfinite(d) && isfinite(u)) {
        o.dx = r - l;
        o.dy = u - d;
        if (!(fmaxf(fabsf(o.dx), fabsf(o.dy)) > p.Tb)) {
            const float s2 = sumsq(o.dx, o.dy);
            if (s2 < p.Ts2) {
                cG = p.As * s2;
                o.branch = 2;
            } else {
                int cnt = 0;
                for (int dyp = -p.rp; dyp <= p.rp; ++dyp)
                    for (int dxp = -p.rp; dxp <= p.rp; ++dxp)
                        if (dxp | dyp) cnt += gentle_at(gk, nx, ny, x + dxp, y + dyp, p) ? 1 : 0;
                if (cnt > p.kp) {
                    cG = p.Ab * fmaxf(o.dx * o.dx, o.dy * o.dy);
                    o.branch = 3;
                } else {
                    o.branch = 4;
                }
            }
        }
    }
    const float s = cI + cG;
    o.pass = s < p.cB;
    o.ci = fminf(p.cB, s);
    return o;
}

// A contribution in fixed point: v * 2^32 rounded to the nearest integer
// (ties to even), clamped to +-2^62 so that the conversion is defined; NaN
// adds nothing.
__device__ __forceinline__ unsigned long long to_fixed(float v) {
    const float q = rintf(v * 0x1p32f);
    if (!(q == q)) return 0ull;
    return (unsigned long long)(long long)fminf(fmaxf(q, -0x1p62f), 0x1p62f);
}

// Gradient sum: a float array, or with `fixed` an int64 array of 2^-32 units
// (two's complement, so integer addition wraps to the signed sum).
__device__ __forceinline__ void grad_add(float* p, long long i, float v, bool fixed) {
    if (fixed) atomicAdd((unsigned long long*)p + i, to_fixed(v));
    else atomicAdd(p + i, v);
}

// Gradient sink: dense grids (nullable) and/or point heights via the ids.
struct Sink {
    float* gG;          // [N][ny][nx] or null
    float* gC;          // [N][ny][nx] or null
    const int* aG;      // point ids, for routing to gz (null: no routing)
    const int* aC;
    float* gz;
    long long n_points;
    int fixed;          // the sums are int64 fixed point (gG, gC, gz)
};

__device__ __forceinline__ void add_ground(const Sink& s, long long i, float v) {
    if (v == 0.0f) return;
    if (s.gG) grad_add(s.gG, i, v, s.fixed);
    if (s.gz) {
        const int id = s.aG[i];
        if (id >= 0 && id < s.n_points) grad_add(s.gz, id, v, s.fixed);
    }
}
__device__ __forceinline__ void add_ceil(const Sink& s, long long i, float v) {
    if (v == 0.0f) return;
    if (s.gC) grad_add(s.gC, i, v, s.fixed);
    if (s.gz) {
        const int id = s.aC[i];
        if (id >= 0 && id < s.n_points) grad_add(s.gz, id, v, s.fixed);
    }
}

// c^T of cell (x, y) of one slice, evaluated on demand: the maximum over
// the Eq. (6) window of K * c^init (first maximum in row-major window
// order), with the maximising cell and its c^init details.  The same FP32
// products and maxima as the full-map kernels, so the same value.
struct WinMax {
    float v, k;
    int qx, qy;
    Cinit q;
};

// The window maxima of the four bilinear corners of a waypoint at once:
// corners (cx[c], cy[c]) lie in a 2 x 2 block, so their windows share most
// cells.  The union of the windows is walked once in row-major order,
// computing each cell's c^init once; every cell updates the corners whose
// window holds it.  Row-major order over the union is row-major order over
// each corner's window, so each corner gets the same first maximum as a walk
// over its own window.
__device__ void window_max4(const float* __restrict__ gk, const float* __restrict__ ck, const int (&cx)[4],
                            const int (&cy)[4], const EvalParams& p, WinMax (&o)[4]) {
    const int nx = p.nx, ny = p.ny, R = p.R;
    int xlo = cx[0], xhi = cx[0], ylo = cy[0], yhi = cy[0];
#pragma unroll
    for (int c = 1; c < 4; ++c) {
        xlo = min(xlo, cx[c]);
        xhi = max(xhi, cx[c]);
        ylo = min(ylo, cy[c]);
        yhi = max(yhi, cy[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        o[c] = WinMax{};
        o[c].v = -INFINITY;
    }
    for (int qy = max(0, ylo - R); qy <= min(ny - 1, yhi + R); ++qy) {
        for (int qx = max(0, xlo - R); qx <= min(nx - 1, xhi + R); ++qx) {
            bool need = false;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int m = abs(qx - cx[c]), n = abs(qy - cy[c]);
                need |= m <= R && n <= R && p.K[m][n] > 0.0f;
            }
            if (!need) continue;
            const Cinit q = cinit_at(gk, ck, qx, qy, p);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int m = abs(qx - cx[c]), n = abs(qy - cy[c]);
                if (m > R || n > R) continue;
                const float kw = p.K[m][n];
                if (kw <= 0.0f) continue;
                const float v = kw * q.ci;
                if (v > o[c].v) {
                    o[c].v = v;
                    o[c].k = kw;
                    o[c].qx = qx;
                    o[c].qy = qy;
                    o[c].q = q;
                }
            }
        }
    }
}

// window_max4 over c^init values already in `box` (rows of bw cells from
// column bx0, row by0, covering every window): the same row-major walk,
// products and first maxima; the maximising cells' c^init details (o[c].q)
// are recomputed when `details` is set.
__device__ void window_max4_box(const float* __restrict__ box, int bx0, int by0, int bw,
                                const float* __restrict__ gk, const float* __restrict__ ck, const int (&cx)[4],
                                const int (&cy)[4], const EvalParams& p, bool details, WinMax (&o)[4]) {
    const int nx = p.nx, ny = p.ny, R = p.R;
    int xlo = cx[0], xhi = cx[0], ylo = cy[0], yhi = cy[0];
#pragma unroll
    for (int c = 1; c < 4; ++c) {
        xlo = min(xlo, cx[c]);
        xhi = max(xhi, cx[c]);
        ylo = min(ylo, cy[c]);
        yhi = max(yhi, cy[c]);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        o[c] = WinMax{};
        o[c].v = -INFINITY;
    }
    for (int qy = max(0, ylo - R); qy <= min(ny - 1, yhi + R); ++qy) {
        const float* row = box + (qy - by0) * bw - bx0;
        for (int qx = max(0, xlo - R); qx <= min(nx - 1, xhi + R); ++qx) {
            const float ci = row[qx];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int m = abs(qx - cx[c]), n = abs(qy - cy[c]);
                if (m > R || n > R) continue;
                const float kw = p.K[m][n];
                if (kw <= 0.0f) continue;
                const float v = kw * ci;
                if (v > o[c].v) {
                    o[c].v = v;
                    o[c].k = kw;
                    o[c].qx = qx;
                    o[c].qy = qy;
                }
            }
        }
    }
    if (details) {
#pragma unroll
        for (int c = 0; c < 4; ++c) o[c].q = cinit_at(gk, ck, o[c].qx, o[c].qy, p);
    }
}

__device__ __forceinline__ int wave_min_int(int v) {
    for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
    return v;
}
__device__ __forceinline__ int wave_max_int(int v) {
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
    return v;
}

// LDS written by some lanes of a wavefront, then read by others.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// c^init cells a wavefront shares per round of 64 waypoints (8 KB each).
constexpr int kTrajBox = 2048;

// Eq. (1)-(5) adjoint at the maximising cell of a window, for gradient gq
// of its c^init.
__device__ void cinit_adjoint(const Cinit& q, long long iq, int nx, float gq, const EvalParams& p, const Sink& s) {
    if (q.branch == 0 || !q.pass) return;
    if (q.ipos) {
        add_ground(s, iq, p.alpha_d * gq);
        add_ceil(s, iq, -p.alpha_d * gq);
    }
    float ddx = 0.0f, ddy = 0.0f;
    if (q.branch == 2) {
        ddx = 2.0f * p.As * q.dx * gq;
        ddy = 2.0f * p.As * q.dy * gq;
    } else if (q.branch == 3) {
        if (fabsf(q.dx) >= fabsf(q.dy)) ddx = 2.0f * p.Ab * q.dx * gq;
        else ddy = 2.0f * p.Ab * q.dy * gq;
    }
    if (ddx != 0.0f) {
        add_ground(s, iq + 1, ddx);
        add_ground(s, iq - 1, -ddx);
    }
    if (ddy != 0.0f) {
        add_ground(s, iq + nx, ddy);
        add_ground(s, iq - nx, -ddy);
    }
}

// dL/dc^T(k, x, y) = gc: inflation argmax, then the Eq. (1)-(5) adjoint.
__device__ void eval_adjoint_cell(const float* __restrict__ ground, const float* __restrict__ ceil, int k, int x,
                                  int y, float gc, const EvalParams& p, const Sink& s) {
    const long long base = (long long)k * p.plane;
    const float* gk = ground + base;
    const float* ck = ceil + base;
    const int nx = p.nx, ny = p.ny, R = p.R;
    float best = -INFINITY, bk = 0.0f;
    int bx = x, by = y;
    for (int n = -R; n <= R; ++n) {
        const int qy = y + n;
        if (qy < 0 || qy >= ny) continue;
        for (int m = -R; m <= R; ++m) {
            const int qx = x + m;
            const float kw = p.K[abs(m)][abs(n)];
            if (kw <= 0.0f || qx < 0 || qx >= nx) continue;
            const float v = kw * cinit_at(gk, ck, qx, qy, p).ci;
            if (v > best) {
                best = v;
                bk = kw;
                bx = qx;
                by = qy;
            }
        }
    }
    const Cinit q = cinit_at(gk, ck, bx, by, p);
    if (q.branch == 0 || !q.pass) return;
    const float gq = bk * gc;
    const long long iq = base + (long long)by * nx + bx;
    if (q.ipos) {
        add_ground(s, iq, p.alpha_d * gq);
        add_ceil(s, iq, -p.alpha_d * gq);
    }
    float ddx = 0.0f, ddy = 0.0f;   // dL/d(dx), dL/d(dy) for the raw differences
    if (q.branch == 2) {
        ddx = 2.0f * p.As * q.dx * gq;
        ddy = 2.0f * p.As * q.dy * gq;
    } else if (q.branch == 3) {
        if (fabsf(q.dx) >= fabsf(q.dy)) ddx = 2.0f * p.Ab * q.dx * gq;
        else ddy = 2.0f * p.Ab * q.dy * gq;
    }
    if (ddx != 0.0f) {
        add_ground(s, iq + 1, ddx);
        add_ground(s, iq - 1, -ddx);
    }
    if (ddy != 0.0f) {
        add_ground(s, iq + nx, ddy);
        add_ground(s, iq - nx, -ddy);
    }
}

// ----------------------------------------------------------------- sampling
struct SampleArgs {
    float x0, y0, res, inv_res, d_ref, w_z;
    int nx, ny, N;
    long long plane;
    int T, W;
};

struct Bil {
    bool ok, hterm;
    long long c00, c10, c01, c11;
    float fu, fv, du, dv;
};

// Cell-centred coordinate u = (x - x0) / r - 1/2 split into an integer
// part and a fraction.  Far from the origin u is large (2000 cells on a
// 200 m map) and one FP32 rounding of u would cost ~1e-4 of a cell; here
// the subtraction's error (two-sum) and the exact remainder of the
// correctly rounded quotient, fma(-q, r, dx), give the fraction to ~1e-7.
__device__ __forceinline__ void split_coord(float x, float x0, float r, int& i, float& f) {
    // dx + e = x - x0 exactly (two-sum)
    const float dx = x - x0;
    const float bb = dx - x;
    const float e = (x - (dx - bb)) + (-x0 - bb);
    const float q = dx / r;
    const float rem = __builtin_fmaf(-q, r, dx) + e;
    const float qs = q - 0.5f;
    const float fl = floorf(qs);
    f = (qs - fl) + rem / r;
    i = (int)fl;
    if (f < 0.0f) { f += 1.0f; --i; }
    else if (f >= 1.0f) { f -= 1.0f; ++i; }
}

// Clamp to the grid edge (zero slope across the clamp): u = i + f.
__device__ __forceinline__ void axis(int i, float f, int n, int& i0, int& i1, float& fr, float& dq) {
    if (n == 1) {
        i0 = i1 = 0;
        fr = 0.0f;
        dq = 0.0f;
        return;
    }
    dq = 1.0f;
    if (i < 0) {                                   // u < 0
        i = 0;
        f = 0.0f;
        dq = 0.0f;
    } else if (i > n - 1 || (i == n - 1 && f > 0.0f)) {   // u > n - 1
        i = n - 1;
        f = 0.0f;
        dq = 0.0f;
    }
    if (i > n - 2) {                               // u = n - 1 exactly
        i = n - 2;
        f += 1.0f;
    }
    i0 = i;
    i1 = i + 1;
    fr = f;
}

__device__ Bil bilinear(const float* __restrict__ ground, const SampleArgs& a, float x, float y, float z, int k) {
    Bil b{};
    if (k < 0 || k >= a.N || !isfinite(x) || !isfinite(y) || !isfinite(z)) return b;
    b.ok = true;
    int iu, iv, i0, i1, j0, j1;
    float fu, fv;
    split_coord(x, a.x0, a.res, iu, fu);
    split_coord(y, a.y0, a.res, iv, fv);
    axis(iu, fu, a.nx, i0, i1, b.fu, b.du);
    axis(iv, fv, a.ny, j0, j1, b.fv, b.dv);
    b.du *= a.inv_res;
    b.dv *= a.inv_res;
    const long long base = (long long)k * a.plane;
    b.c00 = base + (long long)j0 * a.nx + i0;
    b.c10 = base + (long long)j0 * a.nx + i1;
    b.c01 = base + (long long)j1 * a.nx + i0;
    b.c11 = base + (long long)j1 * a.nx + i1;
    b.hterm = isfinite(ground[b.c00]) && isfinite(ground[b.c10]) && isfinite(ground[b.c01]) && isfinite(ground[b.c11]);
    return b;
}

__global__ __launch_bounds__(kBlock) void k_sample_fwd(const float* __restrict__ cost, const float* __restrict__ ground,
                                                       const float* __restrict__ wp, const int* __restrict__ slice,
                                                       SampleArgs a, float* __restrict__ f) {
    const int t = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x / 64);
    if (t >= a.T) return;
    const int lane = threadIdx.x & 63;
    float acc = 0.0f;
    for (int w = lane; w < a.W; w += 64) {
        const long long i = (long long)t * a.W + w;
        const float x = wp[3 * i], y = wp[3 * i + 1], z = wp[3 * i + 2];
        const Bil b = bilinear(ground, a, x, y, z, slice[i]);
        if (!b.ok) continue;
        const float w00 = (1.0f - b.fu) * (1.0f - b.fv), w10 = b.fu * (1.0f - b.fv);
        const float w01 = (1.0f - b.fu) * b.fv, w11 = b.fu * b.fv;
        acc += w00 * cost[b.c00] + w10 * cost[b.c10] + w01 * cost[b.c01] + w11 * cost[b.c11];
        if (b.hterm) {
            const float G = w00 * ground[b.c00] + w10 * ground[b.c10] + w01 * ground[b.c01] + w11 * ground[b.c11];
            const float e = z - G - a.d_ref;
            acc += a.w_z * e * e;
        }
    }
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane == 0) f[t] = acc;
}

// Per waypoint: dL/dwp (written), the bilinear scatter of dL/dC to c^T
// (dense gcost and/or, with `eval`, straight through the traversability
// adjoint into the sink) and of the height term to e^G.
__global__ __launch_bounds__(kBlock) void k_sample_bwd(const float* __restrict__ cost, const float* __restrict__ ground,
                                                       const float* __restrict__ ceil, const float* __restrict__ wp,
                                                       const int* __restrict__ slice, SampleArgs a,
                                                       const float* __restrict__ gf, float* __restrict__ gwp,
                                                       float* __restrict__ gcost, const EvalParams ep, int eval,
                                                       Sink s) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= (long long)a.T * a.W) return;
    const int t = (int)(i / a.W);
    const float x = wp[3 * i], y = wp[3 * i + 1], z = wp[3 * i + 2];
    const int k = slice[i];
    const Bil b = bilinear(ground, a, x, y, z, k);
    float gx = 0.0f, gy = 0.0f, gzw = 0.0f;
    if (b.ok) {
        const float g = gf[t];
        const float w00 = (1.0f - b.fu) * (1.0f - b.fv), w10 = b.fu * (1.0f - b.fv);
        const float w01 = (1.0f - b.fu) * b.fv, w11 = b.fu * b.fv;
        const float c00 = cost[b.c00], c10 = cost[b.c10], c01 = cost[b.c01], c11 = cost[b.c11];
        const float dCdu = (1.0f - b.fv) * (c10 - c00) + b.fv * (c11 - c01);
        const float dCdv = (1.0f - b.fu) * (c01 - c00) + b.fu * (c11 - c10);
        gx = g * dCdu * b.du;
        gy = g * dCdv * b.dv;
        const long long cs[4] = {b.c00, b.c10, b.c01, b.c11};
        const float ws[4] = {w00, w10, w01, w11};
        if (b.hterm) {
            const float G00 = ground[b.c00], G10 = ground[b.c10], G01 = ground[b.c01], G11 = ground[b.c11];
            const float G = w00 * G00 + w10 * G10 + w01 * G01 + w11 * G11;
            const float de = 2.0f * a.w_z * (z - G - a.d_ref) * g;
            const float dGdu = (1.0f - b.fv) * (G10 - G00) + b.fv * (G11 - G01);
            const float dGdv = (1.0f - b.fu) * (G01 - G00) + b.fu * (G11 - G10);
            gx -= de * dGdu * b.du;
            gy -= de * dGdv * b.dv;
            gzw = de;
            for (int c = 0; c < 4; ++c) add_ground(s, cs[c], -de * ws[c]);
        }
        for (int c = 0; c < 4; ++c) {
            const float gc = g * ws[c];
            if (gcost && gc != 0.0f) grad_add(gcost, cs[c], gc, s.fixed);
            if (eval && gc != 0.0f) {
                const long long local = cs[c] - (long long)k * a.plane;
                eval_adjoint_cell(ground, ceil, k, (int)(local % a.nx), (int)(local / a.nx), gc, ep, s);
            }
        }
    }
    gwp[3 * i] = gx;
    gwp[3 * i + 1] = gy;
    gwp[3 * i + 2] = gzw;
}

// Dense traversability adjoint: one thread per cell-slice with a gradient.
__global__ __launch_bounds__(kBlock) void k_eval_bwd(const float* __restrict__ ground, const float* __restrict__ ceil,
                                                     const float* __restrict__ gcost, const EvalParams p, Sink s) {
    const long long total = p.plane * p.N;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < total;
         i += (long long)gridDim.x * kBlock) {
        const float gc = gcost[i];
        if (gc == 0.0f) continue;
        const int k = (int)(i / p.plane);
        const long long c = i - (long long)k * p.plane;
        eval_adjoint_cell(ground, ceil, k, (int)(c % p.nx), (int)(c / p.nx), gc, p, s);
    }
}

// Construction adjoint: per cell, walk the slices and add each run of
// values held by the same point in one atomic.
__global__ __launch_bounds__(kBlock) void k_route(const float* __restrict__ gG, const float* __restrict__ gC,
                                                  const int* __restrict__ aG, const int* __restrict__ aC,
                                                  long long plane, int N, long long n_points, float* __restrict__ gz,
                                                  int fixed) {
    const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= plane) return;
    for (int which = 0; which < 2; ++which) {
        const float* g = which ? gC : gG;
        const int* a = which ? aC : aG;
        if (!g) continue;
        int cur = -1;
        float acc = 0.0f;
        for (int k = 0; k < N; ++k) {
            const long long i = (long long)k * plane + c;
            const int id = a[i];
            if (id != cur) {
                if (cur >= 0 && cur < n_points && acc != 0.0f) grad_add(gz, cur, acc, fixed);
                cur = id;
                acc = 0.0f;
            }
            acc += g[i];
        }
        if (cur >= 0 && cur < n_points && acc != 0.0f) grad_add(gz, cur, acc, fixed);
    }
}

// Fixed-point sums to float32: the integer correctly rounded, times 2^-32.
__global__ __launch_bounds__(kBlock) void k_fixed_to_float(const long long* __restrict__ q, long long n,
                                                           float* __restrict__ out) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = (float)q[i] * 0x1p-32f;
}

__global__ __launch_bounds__(kBlock) void k_zero(float* __restrict__ p, long long n) {
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = 0.0f;
}

int grid_for(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + kBlock - 1) / kBlock, 1 << 16)); }

// Value and gradient for many robot profiles in one launch, each profile
// with its own trajectories, with c^T evaluated on demand at the bilinear
// corners (no cost maps).  One wavefront per (profile, trajectory), lanes
// over its waypoints; per waypoint the value and the waypoint gradient are
// the same FP32 sequences as k_sample_fwd / k_sample_bwd on a materialised
// map, and the maximising taps found for the value feed the traversability
// adjoint directly.
__global__ __launch_bounds__(kBlock) void k_traj_value_grad(const float* __restrict__ ground,
                                                            const float* __restrict__ ceil,
                                                            const EvalParams* __restrict__ robots, SampleArgs a,
                                                            int n_profiles, const float* __restrict__ wp,
                                                            const int* __restrict__ slice,
                                                            const float* __restrict__ gf, float* __restrict__ f,
                                                            float* __restrict__ gwp, Sink s) {
    const long long wave = (long long)blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
    if (wave >= (long long)n_profiles * a.T) return;
    const int prof = __builtin_amdgcn_readfirstlane((int)(wave / a.T));
    const EvalParams& p = robots[prof];
    const int lane = threadIdx.x & 63;
    const float g = gf ? gf[wave] : 0.0f;
    __shared__ float s_box[kBlock / 64][kTrajBox];
    float* box = s_box[threadIdx.x / 64];
    float acc = 0.0f;
    // rounds of 64 waypoints; a round whose waypoints share a slice and whose
    // windows fit one box has the wavefront compute each c^init of the box
    // once (consecutive waypoints of a trajectory are close, so their
    // windows overlap) and every lane take its window maxima from it
    for (int w0 = 0; w0 < a.W; w0 += 64) {
        const int w = w0 + lane;
        const bool act = w < a.W;
        const long long i = wave * a.W + min(w, a.W - 1);
        const float x = wp[3 * i], y = wp[3 * i + 1], z = wp[3 * i + 2];
        const int k = slice[i];
        Bil b = bilinear(ground, a, x, y, z, k);
        b.ok = b.ok && act;
        int cx[4] = {0, 0, 0, 0}, cy[4] = {0, 0, 0, 0};
        if (b.ok) {
            const long long base = (long long)k * a.plane;
            const long long cs[4] = {b.c00, b.c10, b.c01, b.c11};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const long long local = cs[c] - base;
                cx[c] = (int)(local % a.nx);
                cy[c] = (int)(local / a.nx);
            }
        }
        const unsigned long long okm = __ballot(b.ok);
        bool use_box = false;
        int bx0 = 0, by0 = 0, bw = 0;
        if (okm != 0ull) {   // uniform
            const int kb = __shfl(k, (int)__builtin_ctzll(okm), 64);
            const bool same_k = __ballot(b.ok && k != kb) == 0ull;
            const int xlo = wave_min_int(b.ok ? min(min(cx[0], cx[1]), min(cx[2], cx[3])) : INT_MAX);
            const int xhi = wave_max_int(b.ok ? max(max(cx[0], cx[1]), max(cx[2], cx[3])) : INT_MIN);
            const int ylo = wave_min_int(b.ok ? min(min(cy[0], cy[1]), min(cy[2], cy[3])) : INT_MAX);
            const int yhi = wave_max_int(b.ok ? max(max(cy[0], cy[1]), max(cy[2], cy[3])) : INT_MIN);
            bx0 = max(0, xlo - p.R);
            by0 = max(0, ylo - p.R);
            bw = min(a.nx - 1, xhi + p.R) - bx0 + 1;
            const int bh = min(a.ny - 1, yhi + p.R) - by0 + 1;
            use_box = same_k && (long long)bw * bh <= kTrajBox;
            if (use_box) {
                const long long base = (long long)kb * a.plane;
                for (int idx = lane; idx < bw * bh; idx += 64)
                    box[idx] = cinit_at(ground + base, ceil + base, bx0 + idx % bw, by0 + idx / bw, p).ci;
                wave_lds_sync();
            }
        }
        float gx = 0.0f, gy = 0.0f, gzw = 0.0f;
        if (b.ok) {
            const long long base = (long long)k * a.plane;
            const float* gk = ground + base;
            const float* ck = ceil + base;
            const long long cs[4] = {b.c00, b.c10, b.c01, b.c11};
            WinMax wm[4];
            if (use_box) window_max4_box(box, bx0, by0, bw, gk, ck, cx, cy, p, gf != nullptr, wm);
            else window_max4(gk, ck, cx, cy, p, wm);
            const float w00 = (1.0f - b.fu) * (1.0f - b.fv), w10 = b.fu * (1.0f - b.fv);
            const float w01 = (1.0f - b.fu) * b.fv, w11 = b.fu * b.fv;
            const float ws[4] = {w00, w10, w01, w11};
            acc += w00 * wm[0].v + w10 * wm[1].v + w01 * wm[2].v + w11 * wm[3].v;
            float G00 = 0.0f, G10 = 0.0f, G01 = 0.0f, G11 = 0.0f, G = 0.0f;
            if (b.hterm) {
                G00 = ground[b.c00];
                G10 = ground[b.c10];
                G01 = ground[b.c01];
                G11 = ground[b.c11];
                G = w00 * G00 + w10 * G10 + w01 * G01 + w11 * G11;
                const float e = z - G - p.d_ref;
                acc += a.w_z * e * e;
            }
            if (gf) {
                const float dCdu = (1.0f - b.fv) * (wm[1].v - wm[0].v) + b.fv * (wm[3].v - wm[2].v);
                const float dCdv = (1.0f - b.fu) * (wm[2].v - wm[0].v) + b.fu * (wm[3].v - wm[1].v);
                gx = g * dCdu * b.du;
                gy = g * dCdv * b.dv;
                if (b.hterm) {
                    const float de = 2.0f * a.w_z * (z - G - p.d_ref) * g;
                    const float dGdu = (1.0f - b.fv) * (G10 - G00) + b.fv * (G11 - G01);
                    const float dGdv = (1.0f - b.fu) * (G01 - G00) + b.fu * (G11 - G10);
                    gx -= de * dGdu * b.du;
                    gy -= de * dGdv * b.dv;
                    gzw = de;
                    for (int c = 0; c < 4; ++c) add_ground(s, cs[c], -de * ws[c]);
                }
                for (int c = 0; c < 4; ++c) {
                    const float gc = g * ws[c];
                    if (gc == 0.0f) continue;
                    cinit_adjoint(wm[c].q, base + (long long)wm[c].qy * a.nx + wm[c].qx, a.nx, wm[c].k * gc, p, s);
                }
            }
        }
        if (gwp && act) {
            gwp[3 * i] = gx;
            gwp[3 * i + 1] = gy;
            gwp[3 * i + 2] = gzw;
        }
        if (use_box) wave_lds_sync();   // the next round refills the box
    }
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane == 0) f[wave] = acc;
}

}  // namespace

pct_status launch_zero(float* p, long long n, hipStream_t s) {
    if (!p || n <= 0) return PCT_OK;
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

static SampleArgs make_sample_args(const pct_grid& g, int N, float d_ref, float w_z, int T, int W) {
    SampleArgs a{};
    a.x0 = g.x0;
    a.y0 = g.y0;
    a.res = g.res;
    a.inv_res = (float)(1.0 / (double)g.res);
    a.d_ref = d_ref;
    a.w_z = w_z;
    a.nx = g.nx;
    a.ny = g.ny;
    a.N = N;
    a.plane = (long long)g.nx * g.ny;
    a.T = T;
    a.W = W;
    return a;
}

pct_status launch_sample_fwd(const float* cost, const float* ground, const pct_grid& g, int N, float d_ref, float w_z,
                             const float* wp, const int* slice, int T, int W, float* f, hipStream_t s) {
    const SampleArgs a = make_sample_args(g, N, d_ref, w_z, T, W);
    const int blocks = (T + kBlock / 64 - 1) / (kBlock / 64);
    hipLaunchKernelGGL(k_sample_fwd, dim3(blocks), dim3(kBlock), 0, s, cost, ground, wp, slice, a, f);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

pct_status launch_sample_bwd(const float* cost, const float* ground, const float* ceil, const pct_grid& g, int N,
                             float d_ref, float w_z, const float* wp, const int* slice, int T, int W, const float* gf,
                             float* gwp, float* gcost, float* gground, const EvalParams* ep, const int* aG,
                             const int* aC, float* gz, long long n_points, bool fixed, hipStream_t s) {
    const SampleArgs a = make_sample_args(g, N, d_ref, w_z, T, W);
    Sink sk{};
    sk.fixed = fixed;
    sk.gG = gground;
    sk.gC = nullptr;
    sk.aG = aG;
    sk.aC = aC;
    sk.gz = gz;
    sk.n_points = n_points;
    EvalParams p = ep ? *ep : EvalParams{};
    const long long n = (long long)T * W;
    if (n == 0) return PCT_OK;
    hipLaunchKernelGGL(k_sample_bwd, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, cost, ground, ceil,
                       wp, slice, a, gf, gwp, gcost, p, ep ? 1 : 0, sk);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

pct_status launch_eval_bwd(const float* ground, const float* ceil, const float* gcost, const EvalParams& p,
                           float* gground, float* gceil, bool fixed, hipStream_t s) {
    Sink sk{};
    sk.fixed = fixed;
    sk.gG = gground;
    sk.gC = gceil;
    hipLaunchKernelGGL(k_eval_bwd, dim3(grid_for(p.plane * p.N)), dim3(kBlock), 0, s, ground, ceil, gcost, p, sk);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

pct_status launch_route(const float* gG, const float* gC, const int* aG, const int* aC, long long plane, int N,
                        long long n_points, float* gz, bool fixed, hipStream_t s) {
    hipLaunchKernelGGL(k_route, dim3((unsigned)((plane + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, gG, gC, aG, aC,
                       plane, N, n_points, gz, fixed ? 1 : 0);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

pct_status launch_fixed_to_float(const int64_t* q, long long n, float* out, hipStream_t s) {
    if (n <= 0) return PCT_OK;
    hipLaunchKernelGGL(k_fixed_to_float, dim3(grid_for(n)), dim3(kBlock), 0, s, (const long long*)q, n, out);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

pct_status launch_traj_value_grad(const float* ground, const float* ceil, const int* aG, const int* aC,
                                  const pct_grid& g, int N, const EvalParams* d_robots, int n_profiles, float w_z,
                                  const float* wp, const int* slice, int T, int W, const float* gf, float* f,
                                  float* gwp, float* gground, float* gceil, float* gz, long long n_points,
                                  bool fixed, hipStream_t s) {
    const SampleArgs a = make_sample_args(g, N, 0.0f, w_z, T, W);
    Sink sk{};
    sk.fixed = fixed;
    if (gf) {
        sk.gG = gground;
        sk.gC = gceil;
        sk.aG = aG;
        sk.aC = aC;
        sk.gz = n_points > 0 ? gz : nullptr;
        sk.n_points = n_points;
    }
    const long long waves = (long long)n_profiles * T;
    if (waves == 0) return PCT_OK;
    const unsigned blocks = (unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64));
    hipLaunchKernelGGL(k_traj_value_grad, dim3(blocks), dim3(kBlock), 0, s, ground, ceil, d_robots, a, n_profiles, wp,
                       slice, gf, f, gf ? gwp : nullptr, sk);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

}  // namespace pct
