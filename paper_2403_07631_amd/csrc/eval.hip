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
    const int tx0 = blockIdx.x * TW, ty0 = blockIdx.y * TH;
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
        if (gx < nx && gy < ny) cost[(long long)k * p.plane + (long long)gy * nx + gx] = v;
    }
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
    dim3 grid((p.nx + TW - 1) / TW, (p.ny + TH - 1) / TH, p.N);
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
// bit matrix of the in-run slices p with c_p > c_k.  A single thread then
// runs the sequential chain over these N x N bits.

__device__ __forceinline__ int wave_max_i(int v) {
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
    for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m, 64));
    return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
    for (int m = 32; m >= 1; m >>= 1) v |= __shfl_xor(v, m, 64);
    return v;
}

__global__ __launch_bounds__(kBlock) void k_simp_init(int* __restrict__ maxp0, unsigned* __restrict__ urun, int N, int W) {
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N * W; i += gridDim.x * kBlock) urun[i] = 0u;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) maxp0[i] = -1;
}

__global__ __launch_bounds__(kBlock) void k_simp_flags(const float* __restrict__ ground, const float* __restrict__ cost,
                                                       const int nx, const int ny, const int N, const float cB,
                                                       const int W, int* __restrict__ maxp0, unsigned* __restrict__ urun) {
    const long long plane = (long long)nx * ny;
    const long long cell = (long long)blockIdx.x * kBlock + threadIdx.x;
    const bool active = cell < plane;
    const int lane = threadIdx.x & 63;
    float ek = active ? ground[cell] : -INFINITY;
    float ck = active ? cost[cell] : cB;
    float eprev = -INFINITY;
    int p0 = 0;
    for (int k = 0; k < N; ++k) {
        float ek1 = -INFINITY, ck1 = cB;
        if (k + 1 < N && active) {
            ek1 = ground[(long long)(k + 1) * plane + cell];
            ck1 = cost[(long long)(k + 1) * plane + cell];
        }
        if (k > 0 && ek != eprev) p0 = k;
        const bool trav = active && ck < cB;
        const bool upper = (k == N - 1) || (ek1 > ek) || (ck < ck1);
        const bool A = trav && upper;
        const int m = wave_max_i(A ? p0 : -1);
        if (lane == 0 && m >= 0) atomicMax(&maxp0[k], m);
        const bool runA = A && p0 < k;
        if (__ballot(runA)) {
            const int pmin = wave_min_i(runA ? p0 : 0x7fffffff);
            for (int w = pmin / 32; w <= (k - 1) / 32; ++w) {
                unsigned bits = 0;
                const int pb = max(pmin, w * 32), pe = min(k, w * 32 + 32);
                for (int pp = pb; pp < pe; ++pp) {
                    const float cp = active ? cost[(long long)pp * plane + cell] : 0.0f;
                    if (runA && pp >= p0 && cp > ck) bits |= 1u << (pp - w * 32);
                }
                bits = wave_or(bits);
                if (lane == 0 && bits) atomicOr(&urun[(long long)k * W + w], bits);
            }
        }
        eprev = ek;
        ek = ek1;
        ck = ck1;
    }
}

__global__ void k_keep_chain(const int* __restrict__ maxp0, const unsigned* __restrict__ urun, int N, int W,
                             uint8_t* __restrict__ keep) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
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

}  // namespace

size_t eval_ws_bytes(int N, int) {
    const int W = (N + 31) / 32;
    return align_up(sizeof(int) * (size_t)N) + align_up(sizeof(unsigned) * (size_t)N * W);
}

pct_status launch_eval(const float* ground, const float* ceil, const EvalParams& p, float* cost, hipStream_t s) {
    switch (p.R) {
#define PCT_R(r) case r: return launch_eval_r<r>(ground, ceil, p, cost, s);
        PCT_R(0) PCT_R(1) PCT_R(2) PCT_R(3) PCT_R(4) PCT_R(5) PCT_R(6) PCT_R(7) PCT_R(8)
        PCT_R(9) PCT_R(10) PCT_R(11) PCT_R(12) PCT_R(13) PCT_R(14) PCT_R(15) PCT_R(16)
#undef PCT_R
        default: return fail(PCT_ERR_CAPACITY, "inflation radius %d exceeds %d", p.R, PCT_MAX_KERNEL_RADIUS);
    }
}

pct_status launch_simplify(const float* ground, const float* cost, const EvalParams& p, uint8_t* keep, void* ws,
                           hipStream_t s) {
    const int W = (p.N + 31) / 32;
    int* maxp0 = (int*)ws;
    unsigned* urun = (unsigned*)((char*)ws + align_up(sizeof(int) * (size_t)p.N));
    hipLaunchKernelGGL(k_simp_init, dim3(std::max(1, std::min(1024, (p.N * W + kBlock - 1) / kBlock))), dim3(kBlock), 0, s,
                       maxp0, urun, p.N, W);
    PCT_LAUNCH_CHECK();
    const long long blocks = (p.plane + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_simp_flags, dim3((unsigned)blocks), dim3(kBlock), 0, s, ground, cost, p.nx, p.ny, p.N, p.cB, W,
                       maxp0, urun);
    PCT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_keep_chain, dim3(1), dim3(64), 0, s, maxp0, urun, p.N, W, keep);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

}  // namespace pct
