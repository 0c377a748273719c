// Tomogram construction on gfx950 (Sec. III-A, Algorithm 1).
//
// Algorithm 1 compares every point with every plane.  Here the points are
// first binned by a counting sort into construction tiles (256 x th cells),
// with LDS-privatised integer counters; then one workgroup per tile sorts
// each cell's heights in LDS and sweeps the planes once:
//   ground e^G_k = the largest height <= h_k, ceiling e^C_k = the next one.
// This equals Algorithm 1's per-plane max/min exactly (only comparisons are
// involved) and writes each output element once, coalesced along x.
#include "pct_internal.h"

namespace pct {

namespace {

constexpr int kBlock = 256;
// LDS record capacity of the tile reduce: at least these (with point ids,
// without), raised per launch towards the mean records per tile, up to
// kReduceCapMax, so that a dense map reduces each tile in one pass.
constexpr int kReduceCapIds = 4096;
constexpr int kReduceCap = 6144;
constexpr int kReduceCapMax = 16384;

__device__ __forceinline__ float wave_min(float v) {
    for (int m = 32; m >= 1; m >>= 1) v = fminf(v, __shfl_xor(v, m, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Points 4q .. 4q+3 as three 16-byte loads (xyz 16-byte aligned): each
// lane reads 48 contiguous bytes, a wavefront 3 KB, instead of three
// 4-byte loads per point.
typedef float pts_f4 __attribute__((vector_size(16)));
__device__ __forceinline__ void load_quad(const float* __restrict__ xyz, int64_t q, float (&px)[4], float (&py)[4],
                                          float (&pz)[4]) {
    const pts_f4* p = (const pts_f4*)(xyz + 12 * q);
    const pts_f4 a = p[0], b = p[1], c = p[2];
    px[0] = a[0], py[0] = a[1], pz[0] = a[2];
    px[1] = a[3], py[1] = b[0], pz[1] = b[1];
    px[2] = b[2], py[2] = b[3], pz[2] = c[0];
    px[3] = c[1], py[3] = c[2], pz[3] = c[3];
}

// Points [4q, 4q + 4) clipped to [.., n): x, y, z and whether each exists;
// whole quads of an aligned array by load_quad, others point by point.
__device__ __forceinline__ void load_points4(const float* __restrict__ xyz, int64_t n, int64_t q, bool vec,
                                             float (&px)[4], float (&py)[4], float (&pz)[4], bool (&ok)[4]) {
    if (vec && 4 * q + 3 < n) {
        load_quad(xyz, q, px, py, pz);
#pragma unroll
        for (int e = 0; e < 4; ++e) ok[e] = true;
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int64_t i = 4 * q + e;
        ok[e] = i < n;
        px[e] = ok[e] ? xyz[3 * i] : 0.0f;
        py[e] = ok[e] ? xyz[3 * i + 1] : 0.0f;
        pz[e] = ok[e] ? xyz[3 * i + 2] : 0.0f;
    }
}

__device__ __forceinline__ bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// ------------------------------------------------------------------ extent
__global__ __launch_bounds__(kBlock) void k_extent(const float* __restrict__ xyz, int64_t n, GridDev g,
                                                   float* __restrict__ pmin, float* __restrict__ pmax,
                                                   unsigned long long* __restrict__ pused) {
    float lo = INFINITY, hi = -INFINITY;
    unsigned long long used = 0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const bool vec = aligned16(xyz);
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; 4 * q < n; q += stride) {
        float px[4], py[4], pz[4];
        bool ok[4];
        load_points4(xyz, n, q, vec, px, py, pz, ok);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float z = pz[e];
            int ix, iy;
            if (!ok[e] || !isfinite(z) || !rasterize(px[e], py[e], g, ix, iy)) continue;
            z = z + 0.0f;
            lo = fminf(lo, z);
            hi = fmaxf(hi, z);
            ++used;
        }
    }
    __shared__ float s_lo[kBlock / 64], s_hi[kBlock / 64];
    __shared__ unsigned long long s_u[kBlock / 64];
    lo = wave_min(lo);
    hi = wave_max(hi);
    used = wave_sum(used);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s_lo[w] = lo;
        s_hi[w] = hi;
        s_u[w] = used;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i) {
            lo = fminf(lo, s_lo[i]);
            hi = fmaxf(hi, s_hi[i]);
            used += s_u[i];
        }
        pmin[blockIdx.x] = lo;
        pmax[blockIdx.x] = hi;
        pused[blockIdx.x] = used;
    }
}

__global__ __launch_bounds__(kBlock) void k_extent_final(const float* __restrict__ pmin,
                                                         const float* __restrict__ pmax,
                                                         const unsigned long long* __restrict__ pused,
                                                         int nb, ExtentDev* __restrict__ out) {
    float lo = INFINITY, hi = -INFINITY;
    unsigned long long used = 0;
    for (int i = threadIdx.x; i < nb; i += kBlock) {
        lo = fminf(lo, pmin[i]);
        hi = fmaxf(hi, pmax[i]);
        used += pused[i];
    }
    __shared__ float s_lo[kBlock / 64], s_hi[kBlock / 64];
    __shared__ unsigned long long s_u[kBlock / 64];
    lo = wave_min(lo);
    hi = wave_max(hi);
    used = wave_sum(used);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s_lo[w] = lo;
        s_hi[w] = hi;
        s_u[w] = used;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i) {
            lo = fminf(lo, s_lo[i]);
            hi = fmaxf(hi, s_hi[i]);
            used += s_u[i];
        }
        out->zmin = lo;
        out->zmax = hi;
        out->used = used;
    }
}

constexpr int kExtentBlocks = 2048;

// ------------------------------------------------------------------ binning
__device__ __forceinline__ bool bin_xyz(float x, float y, float zin, const GridDev& g, int& tile, unsigned& cell,
                                        float& z) {
    z = zin;
    int ix, iy;
    if (!isfinite(z) || !rasterize(x, y, g, ix, iy)) return false;
    z = z + 0.0f;
    int tx = ix / g.tw, ty = iy / g.th;
    tile = ty * g.ntx + tx;
    cell = (unsigned)((iy - ty * g.th) * g.tw + (ix - tx * g.tw));
    return true;
}

__device__ __forceinline__ bool bin_point(const float* __restrict__ xyz, int64_t i, const GridDev& g,
                                          int& tile, unsigned& cell, float& z) {
    float x = xyz[3 * i], y = xyz[3 * i + 1];
    z = xyz[3 * i + 2];
    int ix, iy;
    if (!isfinite(z) || !rasterize(x, y, g, ix, iy)) return false;
    z = z + 0.0f;
    int tx = ix / g.tw, ty = iy / g.th;
    tile = ty * g.ntx + tx;
    cell = (unsigned)((iy - ty * g.th) * g.tw + (ix - tx * g.tw));
    return true;
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(unsigned* __restrict__ p, int64_t n, unsigned v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

// Exclusive scan over a workgroup of one value per thread (every thread
// calls it): the thread's prefix, and the workgroup's total in `total`.
// Inclusive scans within each wavefront by shuffles, then the wavefront
// totals through LDS (s_w: one word per wavefront).
__device__ __forceinline__ unsigned block_scan_excl(unsigned v, unsigned* s_w, unsigned& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    unsigned incl = v;
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned u = __shfl(incl, lane - d, 64);
        if (lane >= d) incl += u;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    unsigned before = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        const unsigned t = s_w[i];
        tot += t;
        if (i < w) before += t;
    }
    __syncthreads();   // s_w is free again
    total = tot;
    return before + incl - v;
}

// Exclusive scan of len counts into out (which may be cnt itself) by one
// workgroup of 1024 threads, in rounds of four consecutive counts per
// thread (loaded together); returns the total.  cursor (nullable) receives
// the offsets too.
__device__ unsigned block_scan_counts(const unsigned* cnt, unsigned* out, unsigned* cursor, int len) {
    __shared__ unsigned s_w[16];
    unsigned carry = 0;
    for (int base = 0; base < len; base += 4 * 1024) {
        const int i0 = base + 4 * (int)threadIdx.x;
        unsigned v[4], sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[q] = i0 + q < len ? cnt[i0 + q] : 0u;
            sum += v[q];
        }
        unsigned total;
        unsigned run = carry + block_scan_excl(sum, s_w, total);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (i0 + q < len) {
                out[i0 + q] = run;
                if (cursor) cursor[i0 + q] = run;
            }
            run += v[q];
        }
        carry += total;
    }
    return carry;
}

// Exclusive scan of the tile counts (one workgroup): off[0..ntiles], and
// the scatter cursors start at the offsets.
__global__ __launch_bounds__(1024) void k_scan_tiles(const unsigned* __restrict__ cnt, int ntiles,
                                                     unsigned* __restrict__ off, unsigned* __restrict__ cursor) {
    const unsigned total = block_scan_counts(cnt, off, cursor, ntiles);
    if (threadIdx.x == 0) off[ntiles] = total;
}

// Two-level binning into construction tiles (a stable-free counting sort).
// Level 1 sorts points into super-tiles, runs of G consecutive tile ids;
// level 2 sorts each super-tile's records into its tiles.  With at most
// 128 buckets per level, each workgroup appends on the order of a hundred
// records per bucket, so the scattered writes of a workgroup fill whole
// cache lines instead of touching thousands of lines with a few bytes each.
// Every level: a per-workgroup LDS histogram written as one column of a
// bucket-major count matrix, an exclusive scan along each bucket's row
// (one wavefront per bucket), bucket offsets, then a scatter through LDS
// cursors.  Positions depend only on the counts, not on timing; the order
// of records inside one workgroup's run of a bucket is left to the LDS
// atomics, which the tile reduce does not depend on.
constexpr int kBinBlock = 512;
constexpr int64_t kBinChunk = 4096;     // points (level 1) or records (level 2) per workgroup
constexpr int kBinPPT = (int)kBinChunk / kBinBlock;   // per thread
constexpr int kSuperTarget = 128;       // buckets per level
constexpr int kMaxSuperG = 8192;        // tiles per super-tile (LDS counters of level 2)
constexpr int kMaxStaged = 1024;        // buckets of a scatter that stages its chunk in LDS

struct BinPlan {
    int G, S1, CT;     // tiles per super-tile, super-tiles, cells per tile
    int nb1;           // level-1 workgroups
    int nb2;           // level-2 workgroups (upper bound; surplus ones exit)
    bool two_level;
    bool staged1, staged2;   // scatters staged in LDS (bucket counts within kMaxStaged)
};

BinPlan make_bin_plan(int64_t n, const GridDev& g) {
    BinPlan b{};
    b.CT = g.tw * g.th;
    int64_t G = (g.ntiles + kSuperTarget - 1) / kSuperTarget;
    if (G < 1) G = 1;
    if (G > kMaxSuperG) G = kMaxSuperG;
    b.G = (int)G;
    b.S1 = (int)((g.ntiles + G - 1) / G);
    b.two_level = b.G > 1;
    b.nb1 = (int)std::max<int64_t>(1, (n + kBinChunk - 1) / kBinChunk);
    b.nb2 = b.two_level ? b.nb1 + b.S1 : 0;
    b.staged1 = b.S1 <= kMaxStaged;
    b.staged2 = b.G <= kMaxStaged;
    return b;
}

// Level-1 histogram: column b of cnt1 [S1][nb1].
__global__ __launch_bounds__(kBinBlock) void k_bin1_hist(const float* __restrict__ xyz, int64_t n, GridDev g,
                                                         int G, int S1, int nb1, unsigned* __restrict__ cnt1) {
    extern __shared__ unsigned s_cnt[];
    for (int t = threadIdx.x; t < S1; t += kBinBlock) s_cnt[t] = 0;
    __syncthreads();
    // the chunk's points as quads (kBinChunk is a multiple of 4)
    const int64_t q0 = (int64_t)blockIdx.x * (kBinChunk / 4), q1 = min((n + 3) / 4, q0 + kBinChunk / 4);
    const bool vec = aligned16(xyz);
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kBinBlock) {
        float px[4], py[4], pz[4];
        bool ok[4];
        load_points4(xyz, n, q, vec, px, py, pz, ok);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            int tile;
            unsigned cell;
            float z;
            if (ok[e] && bin_xyz(px[e], py[e], pz[e], g, tile, cell, z)) atomicAdd(&s_cnt[tile / G], 1u);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < S1; t += kBinBlock) cnt1[(int64_t)t * nb1 + blockIdx.x] = s_cnt[t];
}

// Exclusive scan of row[0..len) in place by one wavefront; returns the total
// (in every lane).
__device__ unsigned wave_scan_row(unsigned* __restrict__ row, int len) {
    const int lane = threadIdx.x & 63;
    unsigned carry = 0;
    // four 64-entry pieces per pass, their loads issued together (one
    // wavefront per row leaves the loop bound by load latency otherwise)
    for (int base = 0; base < len; base += 256) {
        unsigned v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = base + 64 * q + lane;
            v[q] = i < len ? row[i] : 0u;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = base + 64 * q + lane;
            unsigned incl = v[q];
            for (int d = 1; d < 64; d <<= 1) {
                const unsigned u = __shfl(incl, lane - d, 64);
                if (lane >= d) incl += u;
            }
            if (i < len) row[i] = carry + incl - v[q];
            carry += __shfl(incl, 63, 64);
        }
    }
    return carry;
}

// Level-1 rows: bucket s (one workgroup of 1024 per bucket) scans its row
// of cnt1 in place; the total goes to tot1[s].
__global__ __launch_bounds__(1024) void k_bin1_rows(unsigned* __restrict__ cnt1, int nb1, unsigned* __restrict__ tot1) {
    unsigned* row = cnt1 + (int64_t)blockIdx.x * nb1;
    const unsigned t = block_scan_counts(row, row, nullptr, nb1);
    if (threadIdx.x == 0) tot1[blockIdx.x] = t;
}

// One workgroup: super-tile offsets off1[0..S1] and the level-2 workgroup
// bases cbase[0..S1] (each super-tile gets ceil(tot1 / kBinChunk) of them).
__global__ __launch_bounds__(1024) void k_bin1_offsets(const unsigned* __restrict__ tot1, int S1,
                                                       unsigned* __restrict__ off1, unsigned* __restrict__ cbase) {
    __shared__ unsigned s_a[1024], s_b[1024];
    const int per = (S1 + 1023) / 1024;
    const int b = threadIdx.x * per, e = min(b + per, S1);
    unsigned sa = 0, sb = 0;
    for (int i = b; i < e; ++i) {
        sa += tot1[i];
        sb += (unsigned)((tot1[i] + kBinChunk - 1) / kBinChunk);
    }
    s_a[threadIdx.x] = sa;
    s_b[threadIdx.x] = sb;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const unsigned va = threadIdx.x >= (unsigned)d ? s_a[threadIdx.x - d] : 0u;
        const unsigned vb = threadIdx.x >= (unsigned)d ? s_b[threadIdx.x - d] : 0u;
        __syncthreads();
        s_a[threadIdx.x] += va;
        s_b[threadIdx.x] += vb;
        __syncthreads();
    }
    unsigned ra = s_a[threadIdx.x] - sa, rb = s_b[threadIdx.x] - sb;
    for (int i = b; i < e; ++i) {
        off1[i] = ra;
        cbase[i] = rb;
        ra += tot1[i];
        rb += (unsigned)((tot1[i] + kBinChunk - 1) / kBinChunk);
    }
    if (threadIdx.x == 1023) {
        off1[S1] = s_a[1023];
        cbase[S1] = s_b[1023];
    }
}

// Level-1 scatter.  FINAL (one tile per super-tile): records go straight to
// the tile arrays as (height, cell-in-tile[, id]); otherwise to the level-1
// arrays with key = tile-in-super-tile * CT + cell.
template <bool IDS, bool FINAL>
__global__ __launch_bounds__(kBinBlock) void k_bin1_scatter(const float* __restrict__ xyz, int64_t n, GridDev g,
                                                            int G, int S1, int CT, int nb1,
                                                            const unsigned* __restrict__ cnt1,
                                                            const unsigned* __restrict__ off1, float* __restrict__ oz,
                                                            unsigned* __restrict__ okey, int* __restrict__ oid) {
    extern __shared__ unsigned s_cur[];
    for (int t = threadIdx.x; t < S1; t += kBinBlock) s_cur[t] = off1[t] + cnt1[(int64_t)t * nb1 + blockIdx.x];
    __syncthreads();
    const int64_t b0 = (int64_t)blockIdx.x * kBinChunk, b1 = min(n, b0 + kBinChunk);
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kBinBlock) {
        int tile;
        unsigned cell;
        float z;
        if (!bin_point(xyz, i, g, tile, cell, z)) continue;
        const int st = tile / G;
        const unsigned pos = atomicAdd(&s_cur[st], 1u);
        oz[pos] = z;
        okey[pos] = FINAL ? cell : (unsigned)(tile - st * G) * (unsigned)CT + cell;
        if (IDS) oid[pos] = (int)i;
    }
}

// Exclusive scan of cnt[0..B) into start[0..B] by the first wavefront.
__device__ __forceinline__ void wave_scan_lds(const unsigned* __restrict__ cnt, unsigned* __restrict__ start, int B) {
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    unsigned carry = 0;
    for (int base = 0; base < B; base += 64) {
        const unsigned v = base + lane < B ? cnt[base + lane] : 0u;
        unsigned incl = v;
        for (int d = 1; d < 64; d <<= 1) {
            const unsigned u = __shfl(incl, lane - d, 64);
            if (lane >= d) incl += u;
        }
        if (base + lane < B) start[base + lane] = carry + incl - v;
        carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) start[B] = carry;
}

// The bucket of sorted position p: the last b with start[b] <= p.
__device__ __forceinline__ int bucket_of(const unsigned* __restrict__ start, int B, unsigned p) {
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (start[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Staged scatter (both levels): the workgroup's records are first sorted by
// bucket in LDS, then written so that consecutive threads write consecutive
// addresses of a bucket's run.  LDS: 3 B + 1 counters, then the chunk's
// heights, keys (and ids).
inline size_t staged_lds_bytes(int B, bool ids) {
    return sizeof(unsigned) * (3 * (size_t)B + 1) + (size_t)kBinChunk * (ids ? 12 : 8);
}

template <bool IDS>
__device__ __forceinline__ void staged_write(unsigned* s_mem, int B, const float (&z)[kBinPPT],
                                             const unsigned (&key)[kBinPPT], const int (&id)[kBinPPT],
                                             const int (&bk)[kBinPPT], const unsigned (&rank)[kBinPPT],
                                             float* __restrict__ oz, unsigned* __restrict__ okey,
                                             int* __restrict__ oid) {
    unsigned* s_cnt = s_mem;
    unsigned* s_start = s_cnt + B;          // B + 1
    unsigned* s_gb = s_start + B + 1;       // global start of this workgroup's run of each bucket
    float* s_z = (float*)(s_gb + B);
    unsigned* s_key = (unsigned*)(s_z + kBinChunk);
    int* s_id = (int*)(s_key + kBinChunk);
    wave_scan_lds(s_cnt, s_start, B);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBinPPT; ++j) {
        if (bk[j] < 0) continue;
        const unsigned p = s_start[bk[j]] + rank[j];
        s_z[p] = z[j];
        s_key[p] = key[j];
        if (IDS) s_id[p] = id[j];
    }
    __syncthreads();
    const unsigned total = s_start[B];
    for (unsigned p = threadIdx.x; p < total; p += kBinBlock) {
        const int b = bucket_of(s_start, B, p);
        const unsigned pos = s_gb[b] + (p - s_start[b]);
        oz[pos] = s_z[p];
        okey[pos] = s_key[p];
        if (IDS) oid[pos] = s_id[p];
    }
}

template <bool IDS, bool FINAL>
__global__ __launch_bounds__(kBinBlock) void k_bin1_scatter_staged(const float* __restrict__ xyz, int64_t n, GridDev g,
                                                                   int G, int S1, int CT, int nb1,
                                                                   const unsigned* __restrict__ cnt1,
                                                                   const unsigned* __restrict__ off1,
                                                                   float* __restrict__ oz, unsigned* __restrict__ okey,
                                                                   int* __restrict__ oid) {
    extern __shared__ unsigned s_mem[];
    unsigned* s_cnt = s_mem;
    unsigned* s_gb = s_cnt + 2 * S1 + 1;
    for (int t = threadIdx.x; t < S1; t += kBinBlock) {
        s_cnt[t] = 0;
        s_gb[t] = off1[t] + cnt1[(int64_t)t * nb1 + blockIdx.x];
    }
    __syncthreads();
    float z[kBinPPT];
    unsigned key[kBinPPT], rank[kBinPPT];
    int id[kBinPPT], bk[kBinPPT];
    // quads m kBinBlock + threadIdx.x of the chunk: points 4 q .. 4 q + 3
    static_assert(kBinPPT % 4 == 0, "whole quads per thread");
    const int64_t q0 = (int64_t)blockIdx.x * (kBinChunk / 4);
    const bool vec = aligned16(xyz);
#pragma unroll
    for (int m = 0; m < kBinPPT / 4; ++m) {
        const int64_t q = q0 + (int64_t)m * kBinBlock + threadIdx.x;
        float px[4], py[4], pz[4];
        bool ok[4];
        load_points4(xyz, n, q, vec, px, py, pz, ok);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int j = 4 * m + e;
            int tile;
            unsigned cell;
            bk[j] = -1;
            id[j] = (int)(4 * q + e);
            if (ok[e] && bin_xyz(px[e], py[e], pz[e], g, tile, cell, z[j])) {
                const int st = tile / G;
                bk[j] = st;
                key[j] = FINAL ? cell : (unsigned)(tile - st * G) * (unsigned)CT + cell;
                rank[j] = atomicAdd(&s_cnt[st], 1u);
            }
        }
    }
    __syncthreads();
    staged_write<IDS>(s_mem, S1, z, key, id, bk, rank, oz, okey, oid);
}

// Level-2 workgroup q covers records [off1[s] + j kBinChunk, ...) of
// super-tile s, with cbase[s] <= q = cbase[s] + j < cbase[s+1].
__device__ __forceinline__ int bin2_super(const unsigned* __restrict__ cbase, int S1, unsigned q) {
    int lo = 0, hi = S1 - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (cbase[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Level-2 histogram: column q of cnt2 [G][nb2].
__global__ __launch_bounds__(kBinBlock) void k_bin2_hist(const unsigned* __restrict__ key1,
                                                         const unsigned* __restrict__ off1,
                                                         const unsigned* __restrict__ cbase, int S1, int G, int CT,
                                                         int nb2, unsigned* __restrict__ cnt2) {
    extern __shared__ unsigned s_cnt[];
    const unsigned q = blockIdx.x;
    if (q >= cbase[S1]) return;   // surplus workgroup (uniform)
    const int st = bin2_super(cbase, S1, q);
    const unsigned r0 = off1[st] + (q - cbase[st]) * (unsigned)kBinChunk;
    const unsigned r1 = min(off1[st + 1], r0 + (unsigned)kBinChunk);
    for (int t = threadIdx.x; t < G; t += kBinBlock) s_cnt[t] = 0;
    __syncthreads();
    for (unsigned r = r0 + threadIdx.x; r < r1; r += kBinBlock) atomicAdd(&s_cnt[key1[r] / (unsigned)CT], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < G; t += kBinBlock) cnt2[(int64_t)t * nb2 + q] = s_cnt[t];
}

// Level-2 rows: tile t = st G + l scans its workgroups' counts (the
// columns cbase[st] .. cbase[st+1] of row l of cnt2); the total goes to
// tot[t].
__global__ __launch_bounds__(kBlock) void k_bin2_rows(unsigned* __restrict__ cnt2, const unsigned* __restrict__ cbase,
                                                      int G, int ntiles, int nb2, unsigned* __restrict__ tot) {
    const int t = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x / 64);
    if (t >= ntiles) return;
    const int st = t / G, l = t - st * G;
    const unsigned c0 = cbase[st], c1 = cbase[st + 1];
    const unsigned total = wave_scan_row(cnt2 + (int64_t)l * nb2 + c0, (int)(c1 - c0));
    if ((threadIdx.x & 63) == 0) tot[t] = total;
}

// Level-2 scatter into the tile arrays: (height, cell-in-tile[, id]).
template <bool IDS>
__global__ __launch_bounds__(kBinBlock) void k_bin2_scatter(const float* __restrict__ z1,
                                                            const unsigned* __restrict__ key1,
                                                            const int* __restrict__ id1,
                                                            const unsigned* __restrict__ off1,
                                                            const unsigned* __restrict__ cbase, int S1, int G, int CT,
                                                            int nb2, const unsigned* __restrict__ cnt2,
                                                            const unsigned* __restrict__ off, float* __restrict__ rz,
                                                            unsigned* __restrict__ rmeta, int* __restrict__ rid) {
    extern __shared__ unsigned s_cur[];
    const unsigned q = blockIdx.x;
    if (q >= cbase[S1]) return;
    const int st = bin2_super(cbase, S1, q);
    const unsigned r0 = off1[st] + (q - cbase[st]) * (unsigned)kBinChunk;
    const unsigned r1 = min(off1[st + 1], r0 + (unsigned)kBinChunk);
    const int tbase = st * G;
    for (int t = threadIdx.x; t < G; t += kBinBlock) s_cur[t] = off[tbase + t] + cnt2[(int64_t)t * nb2 + q];
    __syncthreads();
    for (unsigned r = r0 + threadIdx.x; r < r1; r += kBinBlock) {
        const unsigned key = key1[r];
        const unsigned l = key / (unsigned)CT;
        const unsigned pos = atomicAdd(&s_cur[l], 1u);
        rz[pos] = z1[r];
        rmeta[pos] = key - l * (unsigned)CT;
        if (IDS) rid[pos] = id1[r];
    }
}

template <bool IDS>
__global__ __launch_bounds__(kBinBlock) void k_bin2_scatter_staged(const float* __restrict__ z1,
                                                                   const unsigned* __restrict__ key1,
                                                                   const int* __restrict__ id1,
                                                                   const unsigned* __restrict__ off1,
                                                                   const unsigned* __restrict__ cbase, int S1, int G,
                                                                   int CT, int nb2, const unsigned* __restrict__ cnt2,
                                                                   const unsigned* __restrict__ off,
                                                                   float* __restrict__ rz, unsigned* __restrict__ rmeta,
                                                                   int* __restrict__ rid) {
    extern __shared__ unsigned s_mem[];
    const unsigned q = blockIdx.x;
    if (q >= cbase[S1]) return;   // surplus workgroup (uniform)
    const int st = bin2_super(cbase, S1, q);
    const unsigned r0 = off1[st] + (q - cbase[st]) * (unsigned)kBinChunk;
    const unsigned r1 = min(off1[st + 1], r0 + (unsigned)kBinChunk);
    const int tbase = st * G;
    unsigned* s_cnt = s_mem;
    unsigned* s_gb = s_cnt + 2 * G + 1;
    for (int t = threadIdx.x; t < G; t += kBinBlock) {
        s_cnt[t] = 0;
        s_gb[t] = off[tbase + t] + cnt2[(int64_t)t * nb2 + q];
    }
    __syncthreads();
    float z[kBinPPT];
    unsigned key[kBinPPT], rank[kBinPPT];
    int id[kBinPPT], bk[kBinPPT];
#pragma unroll
    for (int j = 0; j < kBinPPT; ++j) {
        const unsigned r = r0 + (unsigned)(j * kBinBlock) + threadIdx.x;
        bk[j] = -1;
        id[j] = 0;
        if (r < r1) {
            const unsigned k = key1[r];
            const unsigned l = k / (unsigned)CT;
            z[j] = z1[r];
            key[j] = k - l * (unsigned)CT;
            if (IDS) id[j] = id1[r];
            bk[j] = (int)l;
            rank[j] = atomicAdd(&s_cnt[l], 1u);
        }
    }
    __syncthreads();
    staged_write<IDS>(s_mem, G, z, key, id, bk, rank, rz, rmeta, rid);
}

// ------------------------------------------------------------------ reduce
constexpr int kReduceBlock = 512;   // one cell per thread for the 512-cell tiles
__device__ __forceinline__ bool rec_less(float za, int ia, float zb, int ib, bool ids) {
    return za < zb || (ids && za == zb && ia < ib);
}

// Merge of a cell-slice's value with the one already stored (insertion
// into an existing tomogram): the higher ground / lower ceiling wins, equal
// heights keep the lower point id (-1 only goes with the infinities).
__device__ __forceinline__ void merge_vals(float og, float oc, int oi, int oj, float& gz, int& gi, float& cz, int& ci) {
    if (og > gz) {
        gz = og;
        gi = oi;
    } else if (og == gz) {
        gi = min(gi, oi);
    }
    if (oc < cz) {
        cz = oc;
        ci = oj;
    } else if (oc == cz) {
        ci = min(ci, oj);
    }
}

template <bool IDS>
__device__ __forceinline__ void merge_old(int64_t o, const float* __restrict__ ground, const float* __restrict__ ceil,
                                          const int* __restrict__ ag, const int* __restrict__ ac, float& gz, int& gi,
                                          float& cz, int& ci) {
    merge_vals(ground[o], ceil[o], IDS ? ag[o] : 0, IDS ? ac[o] : 0, gz, gi, cz, ci);
}

// One cell: sort its heights (ties by point id) and sweep the planes.
// MERGE: combine with the stored values instead of overwriting them (ids
// are offset by id_base); a cell without records is left as it is.
template <bool IDS, bool MERGE>
__device__ void sweep_cell(float* zs, int* is, int n, int ix, int iy, const GridDev& g, float zmin, float ds,
                           int N, float* __restrict__ ground, float* __restrict__ ceil, int* __restrict__ ag,
                           int* __restrict__ ac, int id_base) {
    if (MERGE && n == 0) return;
    // Shell sort by (height, id) with Ciura's gaps when merging (a scan can
    // pile many new points into few cells); a plain insertion sort (gap 1)
    // otherwise.  The order is total (ids are unique), so the result does
    // not depend on the gaps.
    constexpr int kGaps[] = {701, 301, 132, 57, 23, 10, 4, 1};
    for (int gi = MERGE ? 0 : 7; gi < 8; ++gi) {
        const int gap = kGaps[gi];
        if (gap >= n) continue;
        for (int a = gap; a < n; ++a) {
            float z = zs[a];
            int id = IDS ? is[a] : 0;
            int b = a - gap;
            while (b >= 0 && rec_less(z, id, zs[b], IDS ? is[b] : 0, IDS)) {
                zs[b + gap] = zs[b];
                if (IDS) is[b + gap] = is[b];
                b -= gap;
            }
            zs[b + gap] = z;
            if (IDS) is[b + gap] = id;
        }
    }
    const int64_t plane = (int64_t)g.nx * g.ny;
    int64_t o = (int64_t)iy * g.nx + ix;
    int j = 0, rs = 0;
    float znext = n > 0 ? zs[0] : INFINITY;
    // MERGE reads the stored values of kAhead planes before it writes
    // any of them, so that their loads overlap
    constexpr int kAhead = MERGE ? 8 : 1;
    for (int k0 = 0; k0 < N; k0 += kAhead) {
        float og[kAhead], oc[kAhead];
        int oi[kAhead], oj[kAhead];
        if (MERGE) {
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                if (k0 + u >= N) break;
                const int64_t q = o + u * plane;
                og[u] = ground[q];
                oc[u] = ceil[q];
                oi[u] = IDS ? ag[q] : 0;
                oj[u] = IDS ? ac[q] : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < kAhead; ++u, o += plane) {
            const int k = k0 + u;
            if (k >= N) break;
            const float hk = plane_height(zmin, ds, k);
            while (j < n && znext <= hk) {
                if (j == 0 || znext != zs[j - 1]) rs = j;
                ++j;
                znext = j < n ? zs[j] : INFINITY;
            }
            float gz = j > 0 ? zs[j - 1] : -INFINITY, cz = znext;
            int gi = IDS && j > 0 ? is[rs] + id_base : -1, ci = IDS && j < n ? is[j] + id_base : -1;
            if (MERGE) merge_vals(og[u], oc[u], oi[u], oj[u], gz, gi, cz, ci);
            // streaming stores: the grids are far larger than the caches
            __builtin_nontemporal_store(gz, &ground[o]);
            __builtin_nontemporal_store(cz, &ceil[o]);
            if (IDS) {
                __builtin_nontemporal_store(gi, &ag[o]);
                __builtin_nontemporal_store(ci, &ac[o]);
            }
        }
    }
}

// A cell with more points than the LDS holds: per plane, a block-wide
// max/min reduction over the tile's records (ties to the lowest id).
template <bool IDS, bool MERGE>
__device__ void huge_cell(unsigned c, unsigned r0, unsigned r1, const float* __restrict__ rz,
                          const unsigned* __restrict__ rmeta, const int* __restrict__ rid, int ix, int iy,
                          const GridDev& g, float zmin, float ds, int N, float* __restrict__ ground,
                          float* __restrict__ ceil, int* __restrict__ ag, int* __restrict__ ac, int id_base) {
    __shared__ float s_gz[kReduceBlock], s_cz[kReduceBlock];
    __shared__ int s_gi[kReduceBlock], s_ci[kReduceBlock];
    const int64_t plane = (int64_t)g.nx * g.ny;
    for (int k = 0; k < N; ++k) {
        const float hk = plane_height(zmin, ds, k);
        float gz = -INFINITY, cz = INFINITY;
        int gi = 0x7fffffff, ci = 0x7fffffff;
        for (unsigned r = r0 + threadIdx.x; r < r1; r += kReduceBlock) {
            if (rmeta[r] != c) continue;
            float z = rz[r];
            int id = IDS ? rid[r] : 0;
            if (z <= hk) {
                if (z > gz || (z == gz && id < gi)) { gz = z; gi = id; }
            } else {
                if (z < cz || (z == cz && id < ci)) { cz = z; ci = id; }
            }
        }
        s_gz[threadIdx.x] = gz; s_gi[threadIdx.x] = gi;
        s_cz[threadIdx.x] = cz; s_ci[threadIdx.x] = ci;
        __syncthreads();
        for (int s = kReduceBlock / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                float z2 = s_gz[threadIdx.x + s];
                int i2 = s_gi[threadIdx.x + s];
                if (z2 > s_gz[threadIdx.x] || (z2 == s_gz[threadIdx.x] && i2 < s_gi[threadIdx.x])) {
                    s_gz[threadIdx.x] = z2; s_gi[threadIdx.x] = i2;
                }
                z2 = s_cz[threadIdx.x + s];
                i2 = s_ci[threadIdx.x + s];
                if (z2 < s_cz[threadIdx.x] || (z2 == s_cz[threadIdx.x] && i2 < s_ci[threadIdx.x])) {
                    s_cz[threadIdx.x] = z2; s_ci[threadIdx.x] = i2;
                }
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            int64_t o = (int64_t)k * plane + (int64_t)iy * g.nx + ix;
            float gz = s_gz[0], cz = s_cz[0];
            int gi = IDS && isfinite(gz) ? s_gi[0] + id_base : -1, ci = IDS && isfinite(cz) ? s_ci[0] + id_base : -1;
            if (MERGE) merge_old<IDS>(o, ground, ceil, ag, ac, gz, gi, cz, ci);
            ground[o] = gz;
            ceil[o] = cz;
            if (IDS) {
                ag[o] = gi;
                ac[o] = ci;
            }
        }
        __syncthreads();
    }
}

// One construction tile: records off[tg] .. off[tg+1] of the tile whose
// position in its grid is tl.  Shared by the single-map and batched kernels.
template <bool IDS, bool MERGE = false>
__device__ void reduce_tile(int tg, int tl, const unsigned* __restrict__ off, const float* __restrict__ rz,
                            const unsigned* __restrict__ rmeta, const int* __restrict__ rid, const GridDev& g,
                            float zmin, float ds, int N, float* __restrict__ ground, float* __restrict__ ceil,
                            int* __restrict__ ag, int* __restrict__ ac, int CAP, int id_base = 0) {
    extern __shared__ unsigned s_mem[];
    const int cells = g.tw * g.th;
    unsigned* s_cnt = s_mem;                 // cells
    unsigned* s_start = s_cnt + cells;       // cells + 1
    float* s_z = (float*)(s_start + cells + 1);
    int* s_id = (int*)(s_z + CAP);

    const int tx = tl % g.ntx, ty = tl / g.ntx;
    const unsigned r0 = off[tg], r1 = off[tg + 1];
    if (MERGE && r0 == r1) return;   // an insertion leaves tiles without new points alone

    for (int c = threadIdx.x; c < cells; c += kReduceBlock) s_cnt[c] = 0;
    __syncthreads();
    for (unsigned r = r0 + threadIdx.x; r < r1; r += kReduceBlock) atomicAdd(&s_cnt[rmeta[r]], 1u);
    __syncthreads();
    // exclusive scan of the per-cell counts; thread i owns a contiguous run
    {
        __shared__ unsigned s_part[kReduceBlock];
        const int per = (cells + kReduceBlock - 1) / kReduceBlock;
        const int b = threadIdx.x * per, e = min(b + per, cells);
        unsigned sum = 0;
        for (int i = b; i < e; ++i) sum += s_cnt[i];
        s_part[threadIdx.x] = sum;
        __syncthreads();
        for (int d = 1; d < kReduceBlock; d <<= 1) {
            unsigned v = threadIdx.x >= (unsigned)d ? s_part[threadIdx.x - d] : 0u;
            __syncthreads();
            s_part[threadIdx.x] += v;
            __syncthreads();
        }
        unsigned run = s_part[threadIdx.x] - sum;
        for (int i = b; i < e; ++i) {
            s_start[i] = run;
            run += s_cnt[i];
        }
        if (threadIdx.x == kReduceBlock - 1) s_start[cells] = s_part[kReduceBlock - 1];
    }
    __syncthreads();

    int c_lo = 0;
    while (c_lo < cells) {
        // largest group [c_lo, c_hi) whose records fit in LDS
        int lo = c_lo + 1, hi = cells;
        if (s_start[c_lo + 1] - s_start[c_lo] > (unsigned)CAP) {
            hi = c_lo + 1;
        } else {
            while (lo < hi) {
                int mid = (lo + hi + 1) / 2;
                if (s_start[mid] - s_start[c_lo] <= (unsigned)CAP) lo = mid;
                else hi = mid - 1;
            }
            hi = lo;
        }
        const int c_hi = hi;
        const unsigned g0 = s_start[c_lo];
        if (c_hi == c_lo + 1 && s_start[c_hi] - g0 > (unsigned)CAP) {
            const int ix = tx * g.tw + (c_lo % g.tw);
            const int iy = ty * g.th + c_lo / g.tw;
            huge_cell<IDS, MERGE>((unsigned)c_lo, r0, r1, rz, rmeta, rid, ix, iy, g, zmin, ds, N, ground, ceil, ag, ac,
                                  id_base);
        } else {
            for (int c = c_lo + threadIdx.x; c < c_hi; c += kReduceBlock) s_cnt[c] = 0;
            __syncthreads();
            for (unsigned r = r0 + threadIdx.x; r < r1; r += kReduceBlock) {
                unsigned c = rmeta[r];
                if ((int)c < c_lo || (int)c >= c_hi) continue;
                unsigned pos = s_start[c] - g0 + atomicAdd(&s_cnt[c], 1u);
                s_z[pos] = rz[r];
                if (IDS) s_id[pos] = rid[r];
            }
            __syncthreads();
            for (int c = c_lo + threadIdx.x; c < c_hi; c += kReduceBlock) {
                const int ix = tx * g.tw + (c % g.tw);
                const int iy = ty * g.th + c / g.tw;
                if (ix >= g.nx || iy >= g.ny) continue;
                const unsigned s = s_start[c] - g0;
                sweep_cell<IDS, MERGE>(s_z + s, s_id + s, (int)(s_start[c + 1] - s_start[c]), ix, iy, g, zmin, ds,
                                       N, ground, ceil, ag, ac, id_base);
            }
        }
        __syncthreads();
        c_lo = c_hi;
    }
}

template <bool IDS, bool MERGE>
__global__ __launch_bounds__(kReduceBlock) void k_tile_reduce(const unsigned* __restrict__ off,
                                                        const float* __restrict__ rz,
                                                        const unsigned* __restrict__ rmeta,
                                                        const int* __restrict__ rid, GridDev g, float zmin,
                                                        float ds, int N, float* __restrict__ ground,
                                                        float* __restrict__ ceil, int* __restrict__ ag,
                                                        int* __restrict__ ac, int cap, int id_base) {
    reduce_tile<IDS, MERGE>((int)blockIdx.x, (int)blockIdx.x, off, rz, rmeta, rid, g, zmin, ds, N, ground, ceil, ag,
                            ac, cap, id_base);
}

// Record capacity for n points over the grid's tiles: the floor, or 1.25x
// the mean per tile (rounded up to 1024) when that is larger, up to the cap.
inline int reduce_cap(int64_t n, const GridDev& g, bool ids) {
    const int64_t mean = g.ntiles > 0 ? n / g.ntiles : 0;
    const int64_t want = (mean + mean / 4 + 1023) / 1024 * 1024;
    return (int)std::min<int64_t>(kReduceCapMax, std::max<int64_t>(ids ? kReduceCapIds : kReduceCap, want));
}

inline size_t reduce_lds_bytes(const GridDev& g, bool ids, int cap) {
    const int cells = g.tw * g.th;
    return sizeof(unsigned) * (2 * cells + 1) + (size_t)cap * (ids ? 8 : 4);
}

// Kernels may take more than 64 KB of LDS only once asked for.
pct_status allow_lds(const void* fn, size_t bytes) {
    if (bytes <= 64 * 1024) return PCT_OK;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return fail(PCT_ERR_DEVICE, "tile reduce LDS request of %zu bytes refused: %s", bytes,
                                     hipGetErrorString(e));
    return PCT_OK;
}

struct BuildWs {
    BinPlan bp;
    unsigned *cnt1, *tot1, *off1, *cbase;   // level 1
    unsigned *cnt2;                          // level 2
    unsigned *count, *off, *cursor;          // tiles
    float* z1;                               // level-1 records
    unsigned* key1;
    int* id1;
    float* rz;                               // tile records
    unsigned* rmeta;
    int* rid;
    size_t bytes;
};

BuildWs carve_build_ws(void* base, int64_t n, const GridDev& g, bool ids) {
    BuildWs w{};
    char* p = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* r = p ? p + o : nullptr;
        o += align_up(bytes);
        return r;
    };
    w.bp = make_bin_plan(n, g);
    const BinPlan& b = w.bp;
    w.cnt1 = (unsigned*)take(sizeof(unsigned) * (size_t)b.S1 * b.nb1);
    w.tot1 = (unsigned*)take(sizeof(unsigned) * (size_t)(b.S1 + 1));
    w.off1 = (unsigned*)take(sizeof(unsigned) * (size_t)(b.S1 + 1));
    w.cbase = (unsigned*)take(sizeof(unsigned) * (size_t)(b.S1 + 1));
    if (b.two_level) {
        w.cnt2 = (unsigned*)take(sizeof(unsigned) * (size_t)b.G * b.nb2);
        w.z1 = (float*)take(sizeof(float) * (size_t)n);
        w.key1 = (unsigned*)take(sizeof(unsigned) * (size_t)n);
        w.id1 = ids ? (int*)take(sizeof(int) * (size_t)n) : nullptr;
    }
    w.count = (unsigned*)take(sizeof(unsigned) * (g.ntiles + 1));
    w.off = (unsigned*)take(sizeof(unsigned) * (g.ntiles + 1));
    w.cursor = (unsigned*)take(sizeof(unsigned) * (g.ntiles + 1));
    w.rz = (float*)take(sizeof(float) * (size_t)n);
    w.rmeta = (unsigned*)take(sizeof(unsigned) * (size_t)n);
    w.rid = ids ? (int*)take(sizeof(int) * (size_t)n) : nullptr;
    w.bytes = o;
    return w;
}

}  // namespace

// ------------------------------------------------------------------ batches
//
// Many submaps in one launch per stage.  Workgroups are dealt out over
// global chunks (binning, extents) or global tiles (reduce); each finds its
// item by binary search over the item table's bases.

__device__ __forceinline__ int find_base(const BuildItemDev* __restrict__ items, int n_items, int v, int which) {
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        const int b = which == 0 ? items[mid].chunk_base : (which == 1 ? items[mid].tile_base : items[mid].echunk_base);
        if (b <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_bextent(const float* __restrict__ xyz, const BuildItemDev* __restrict__ items,
                                                    int n_items, float* __restrict__ pmin, float* __restrict__ pmax,
                                                    unsigned long long* __restrict__ pused) {
    const int c = blockIdx.x;
    const int it = find_base(items, n_items, c, 2);
    const BuildItemDev& d = items[it];
    const long long b0 = (long long)(c - d.echunk_base) * kBatchEChunk, b1 = min(d.n, b0 + kBatchEChunk);
    float lo = INFINITY, hi = -INFINITY;
    unsigned long long used = 0;
    for (long long i = b0 + threadIdx.x; i < b1; i += kBlock) {
        const long long j = d.xyz_off + i;
        float x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
        int ix, iy;
        if (!isfinite(z) || !rasterize(x, y, d.g, ix, iy)) continue;
        z = z + 0.0f;
        lo = fminf(lo, z);
        hi = fmaxf(hi, z);
        ++used;
    }
    __shared__ float s_lo[kBlock / 64], s_hi[kBlock / 64];
    __shared__ unsigned long long s_u[kBlock / 64];
    lo = wave_min(lo);
    hi = wave_max(hi);
    used = wave_sum(used);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s_lo[w] = lo;
        s_hi[w] = hi;
        s_u[w] = used;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i) {
            lo = fminf(lo, s_lo[i]);
            hi = fmaxf(hi, s_hi[i]);
            used += s_u[i];
        }
        pmin[c] = lo;
        pmax[c] = hi;
        pused[c] = used;
    }
}

// one workgroup per item: reduce its chunks' partials
__global__ __launch_bounds__(kBlock) void k_bextent_final(const BuildItemDev* __restrict__ items, int n_items,
                                                          int n_echunks, const float* __restrict__ pmin,
                                                          const float* __restrict__ pmax,
                                                          const unsigned long long* __restrict__ pused,
                                                          ExtentDev* __restrict__ out) {
    const int it = blockIdx.x;
    const int c0 = items[it].echunk_base, c1 = it + 1 < n_items ? items[it + 1].echunk_base : n_echunks;
    float lo = INFINITY, hi = -INFINITY;
    unsigned long long used = 0;
    for (int c = c0 + threadIdx.x; c < c1; c += kBlock) {
        lo = fminf(lo, pmin[c]);
        hi = fmaxf(hi, pmax[c]);
        used += pused[c];
    }
    __shared__ float s_lo[kBlock / 64], s_hi[kBlock / 64];
    __shared__ unsigned long long s_u[kBlock / 64];
    lo = wave_min(lo);
    hi = wave_max(hi);
    used = wave_sum(used);
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        s_lo[w] = lo;
        s_hi[w] = hi;
        s_u[w] = used;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i) {
            lo = fminf(lo, s_lo[i]);
            hi = fmaxf(hi, s_hi[i]);
            used += s_u[i];
        }
        out[it].zmin = lo;
        out[it].zmax = hi;
        out[it].used = used;
    }
}

// Per-chunk tile counts of the chunk's item: LDS histogram, one global
// atomic per touched tile.
__global__ __launch_bounds__(kBlock) void k_bcount(const float* __restrict__ xyz, const BuildItemDev* __restrict__ items,
                                                   int n_items, unsigned* __restrict__ gcount) {
    extern __shared__ unsigned s_cnt[];
    const int c = blockIdx.x;
    const int it = find_base(items, n_items, c, 0);
    const BuildItemDev& d = items[it];
    const bool lds = d.g.ntiles <= kMaxLdsTiles;
    if (lds)
        for (int t = threadIdx.x; t < d.g.ntiles; t += kBlock) s_cnt[t] = 0;
    __syncthreads();
    const long long b0 = (long long)(c - d.chunk_base) * kBatchChunk, b1 = min(d.n, b0 + kBatchChunk);
    for (long long i = b0 + threadIdx.x; i < b1; i += kBlock) {
        int tile;
        unsigned cell;
        float z;
        if (!bin_point(xyz, d.xyz_off + i, d.g, tile, cell, z)) continue;
        if (lds) atomicAdd(&s_cnt[tile], 1u);
        else atomicAdd(&gcount[d.tile_base + tile], 1u);
    }
    __syncthreads();
    if (lds)
        for (int t = threadIdx.x; t < d.g.ntiles; t += kBlock)
            if (s_cnt[t]) atomicAdd(&gcount[d.tile_base + t], s_cnt[t]);
}

template <bool IDS>
__global__ __launch_bounds__(kBlock) void k_bscatter(const float* __restrict__ xyz, const BuildItemDev* __restrict__ items,
                                                     int n_items, unsigned* __restrict__ cursor, float* __restrict__ rz,
                                                     unsigned* __restrict__ rmeta, int* __restrict__ rid) {
    extern __shared__ unsigned s_mem[];
    const int c = blockIdx.x;
    const int it = find_base(items, n_items, c, 0);
    const BuildItemDev& d = items[it];
    const bool lds = d.g.ntiles <= kMaxLdsTiles;
    unsigned* s_cnt = s_mem;
    unsigned* s_base = s_mem + (lds ? d.g.ntiles : 0);
    if (lds)
        for (int t = threadIdx.x; t < d.g.ntiles; t += kBlock) s_cnt[t] = 0;
    __syncthreads();
    const long long b0 = (long long)(c - d.chunk_base) * kBatchChunk, b1 = min(d.n, b0 + kBatchChunk);
    if (lds) {
        for (long long i = b0 + threadIdx.x; i < b1; i += kBlock) {
            int tile;
            unsigned cell;
            float z;
            if (bin_point(xyz, d.xyz_off + i, d.g, tile, cell, z)) atomicAdd(&s_cnt[tile], 1u);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < d.g.ntiles; t += kBlock) {
            const unsigned k = s_cnt[t];
            if (k) s_base[t] = atomicAdd(&cursor[d.tile_base + t], k);
            s_cnt[t] = 0;
        }
        __syncthreads();
    }
    for (long long i = b0 + threadIdx.x; i < b1; i += kBlock) {
        int tile;
        unsigned cell;
        float z;
        if (!bin_point(xyz, d.xyz_off + i, d.g, tile, cell, z)) continue;
        const unsigned pos = lds ? s_base[tile] + atomicAdd(&s_cnt[tile], 1u) : atomicAdd(&cursor[d.tile_base + tile], 1u);
        rz[pos] = z;
        rmeta[pos] = cell;
        if (IDS) rid[pos] = (int)(d.xyz_off + i);
    }
}

template <bool IDS>
__global__ __launch_bounds__(kReduceBlock) void k_breduce(const unsigned* __restrict__ off, const float* __restrict__ rz,
                                                    const unsigned* __restrict__ rmeta, const int* __restrict__ rid,
                                                    const BuildItemDev* __restrict__ items, int n_items,
                                                    float* __restrict__ ground, float* __restrict__ ceil,
                                                    int* __restrict__ ag, int* __restrict__ ac, int cap) {
    const int tg = blockIdx.x;
    const int it = find_base(items, n_items, tg, 1);
    const BuildItemDev& d = items[it];
    if (d.N <= 0) return;
    const long long o = d.out_off;
    reduce_tile<IDS>(tg, tg - d.tile_base, off, rz, rmeta, rid, d.g, d.zmin, d.ds, d.N, ground + o, ceil + o,
                     IDS ? ag + o : nullptr, IDS ? ac + o : nullptr, cap);
}

struct BatchWs {
    BuildItemDev* items;
    unsigned *count, *off, *cursor;
    float* rz;
    unsigned* rmeta;
    int* rid;
    size_t bytes;
    int total_tiles, total_chunks;
    long long total_points;
};

BatchWs carve_batch_ws(void* base, const BuildItemDev* h, int n_items, bool ids) {
    BatchWs w{};
    char* p = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char* r = p ? p + o : nullptr;
        o += align_up(bytes);
        return r;
    };
    for (int i = 0; i < n_items; ++i) {
        w.total_tiles += h[i].g.ntiles;
        w.total_chunks += (int)((h[i].n + kBatchChunk - 1) / kBatchChunk);
        w.total_points += h[i].n;
    }
    w.items = (BuildItemDev*)take(sizeof(BuildItemDev) * (size_t)n_items);
    w.count = (unsigned*)take(sizeof(unsigned) * (size_t)(w.total_tiles + 1));
    w.off = (unsigned*)take(sizeof(unsigned) * (size_t)(w.total_tiles + 1));
    w.cursor = (unsigned*)take(sizeof(unsigned) * (size_t)(w.total_tiles + 1));
    w.rz = (float*)take(sizeof(float) * (size_t)w.total_points);
    w.rmeta = (unsigned*)take(sizeof(unsigned) * (size_t)w.total_points);
    w.rid = ids ? (int*)take(sizeof(int) * (size_t)w.total_points) : nullptr;
    w.bytes = o;
    return w;
}

size_t extent_ws_bytes(int64_t) {
    return align_up(sizeof(float) * kExtentBlocks) * 2 + align_up(sizeof(unsigned long long) * kExtentBlocks) +
           align_up(sizeof(ExtentDev));
}

pct_status launch_extent(const float* xyz, int64_t n, const GridDev& g, void* ws, ExtentDev* d_out,
                         hipStream_t s) {
    char* p = (char*)ws;
    float* pmin = (float*)p;
    float* pmax = (float*)(p + align_up(sizeof(float) * kExtentBlocks));
    unsigned long long* pused = (unsigned long long*)(p + 2 * align_up(sizeof(float) * kExtentBlocks));
    int nb = (int)std::min<int64_t>(kExtentBlocks, std::max<int64_t>(1, (n + kBlock * 8 - 1) / (kBlock * 8)));
    hipLaunchKernelGGL(k_extent, dim3(nb), dim3(kBlock), 0, s, xyz, n, g, pmin, pmax, pused);
    PCT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_extent_final, dim3(1), dim3(kBlock), 0, s, pmin, pmax, pused, nb, d_out);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

// The extent record on the device, with the plane count of the plane rule
// (-1: two planes coincide in FP32; -2: more than PCT_MAX_SLICES planes).
__global__ void k_extent_record(const ExtentDev* __restrict__ x, int64_t n, float ds, pct_extent* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    pct_extent e{};
    e.z_min = INFINITY;
    e.z_max = -INFINITY;
    const unsigned long long used = n > 0 ? x->used : 0ull;
    e.n_used = (int64_t)used;
    e.n_dropped = n - (int64_t)used;
    if (used > 0) {
        e.z_min = x->zmin;
        e.z_max = x->zmax;
        int N = -2;
        float prev = -INFINITY;
        for (int k = 0; k < PCT_MAX_SLICES; ++k) {
            const float h = plane_height(e.z_min, ds, k);
            if (!(h > prev)) {
                N = -1;
                break;
            }
            if (h > e.z_max) {
                N = k + 1;
                break;
            }
            prev = h;
        }
        e.n_slices = N;
    }
    *out = e;
}

pct_status launch_extent_record(const float* xyz, int64_t n, const GridDev& g, float ds, void* ws, pct_extent* d_out,
                                hipStream_t s) {
    ExtentDev* d_x = (ExtentDev*)((char*)ws + extent_ws_bytes(n) - align_up(sizeof(ExtentDev)));
    if (n > 0) {
        pct_status st = launch_extent(xyz, n, g, ws, d_x, s);
        if (st != PCT_OK) return st;
    }
    hipLaunchKernelGGL(k_extent_record, dim3(1), dim3(64), 0, s, d_x, n, ds, d_out);
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

size_t build_ws_bytes(int64_t n, const GridDev& g, bool ids) { return carve_build_ws(nullptr, n, g, ids).bytes; }

pct_status launch_build(const float* xyz, int64_t n, const GridDev& g, float zmin, float ds, int N, float* ground,
                        float* ceil, int32_t* ag, int32_t* ac, void* ws, size_t ws_bytes, hipStream_t s, bool merge,
                        int id_base) {
    const bool ids = ag != nullptr;
    BuildWs w = carve_build_ws(ws, n, g, ids);
    if (w.bytes > ws_bytes) return fail(PCT_ERR_WORKSPACE, "build workspace too small: %zu < %zu", ws_bytes, w.bytes);
    const BinPlan& b = w.bp;
    if (n == 0) {
        hipLaunchKernelGGL(k_fill_u32, dim3(std::min(1024, g.ntiles / kBlock + 1)), dim3(kBlock), 0, s, w.count,
                           (int64_t)g.ntiles + 1, 0u);
        PCT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, w.count, g.ntiles, w.off, w.cursor);
        PCT_LAUNCH_CHECK();
    } else {
        // level 1: points -> super-tiles (the tiles themselves when G = 1)
        const size_t l1 = sizeof(unsigned) * (size_t)b.S1;
        hipLaunchKernelGGL(k_bin1_hist, dim3(b.nb1), dim3(kBinBlock), l1, s, xyz, n, g, b.G, b.S1, b.nb1, w.cnt1);
        PCT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_bin1_rows, dim3(b.S1), dim3(1024), 0, s, w.cnt1, b.nb1, w.tot1);
        PCT_LAUNCH_CHECK();
        if (!b.two_level) {
            hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, w.tot1, g.ntiles, w.off, w.cursor);
            PCT_LAUNCH_CHECK();
            const size_t ls = staged_lds_bytes(b.S1, ids);
            if (b.staged1 && ids)
                hipLaunchKernelGGL((k_bin1_scatter_staged<true, true>), dim3(b.nb1), dim3(kBinBlock), ls, s, xyz, n, g,
                                   b.G, b.S1, b.CT, b.nb1, w.cnt1, w.off, w.rz, w.rmeta, w.rid);
            else if (b.staged1)
                hipLaunchKernelGGL((k_bin1_scatter_staged<false, true>), dim3(b.nb1), dim3(kBinBlock), ls, s, xyz, n, g,
                                   b.G, b.S1, b.CT, b.nb1, w.cnt1, w.off, w.rz, w.rmeta, w.rid);
            else if (ids)
                hipLaunchKernelGGL((k_bin1_scatter<true, true>), dim3(b.nb1), dim3(kBinBlock), l1, s, xyz, n, g, b.G,
                                   b.S1, b.CT, b.nb1, w.cnt1, w.off, w.rz, w.rmeta, w.rid);
            else
                hipLaunchKernelGGL((k_bin1_scatter<false, true>), dim3(b.nb1), dim3(kBinBlock), l1, s, xyz, n, g, b.G,
                                   b.S1, b.CT, b.nb1, w.cnt1, w.off, w.rz, w.rmeta, w.rid);
            PCT_LAUNCH_CHECK();
        } else {
            hipLaunchKernelGGL(k_bin1_offsets, dim3(1), dim3(1024), 0, s, w.tot1, b.S1, w.off1, w.cbase);
            PCT_LAUNCH_CHECK();
            const size_t ls = staged_lds_bytes(b.S1, ids);
            if (b.staged1 && ids)
                hipLaunchKernelGGL((k_bin1_scatter_staged<true, false>), dim3(b.nb1), dim3(kBinBlock), ls, s, xyz, n,
                                   g, b.G, b.S1, b.CT, b.nb1, w.cnt1, w.off1, w.z1, w.key1, w.id1);
            else if (b.staged1)
                hipLaunchKernelGGL((k_bin1_scatter_staged<false, false>), dim3(b.nb1), dim3(kBinBlock), ls, s, xyz, n,
                                   g, b.G, b.S1, b.CT, b.nb1, w.cnt1, w.off1, w.z1, w.key1, w.id1);
            else if (ids)
                hipLaunchKernelGGL((k_bin1_scatter<true, false>), dim3(b.nb1), dim3(kBinBlock), l1, s, xyz, n, g, b.G,
                                   b.S1, b.CT, b.nb1, w.cnt1, w.off1, w.z1, w.key1, w.id1);
            else
                hipLaunchKernelGGL((k_bin1_scatter<false, false>), dim3(b.nb1), dim3(kBinBlock), l1, s, xyz, n, g, b.G,
                                   b.S1, b.CT, b.nb1, w.cnt1, w.off1, w.z1, w.key1, w.id1);
            PCT_LAUNCH_CHECK();
            // level 2: each super-tile's records -> its tiles
            const size_t l2 = sizeof(unsigned) * (size_t)b.G;
            hipLaunchKernelGGL(k_bin2_hist, dim3(b.nb2), dim3(kBinBlock), l2, s, w.key1, w.off1, w.cbase, b.S1, b.G,
                               b.CT, b.nb2, w.cnt2);
            PCT_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_bin2_rows, dim3((g.ntiles + 3) / 4), dim3(kBlock), 0, s, w.cnt2, w.cbase, b.G,
                               g.ntiles, b.nb2, w.count);
            PCT_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, w.count, g.ntiles, w.off, w.cursor);
            PCT_LAUNCH_CHECK();
            const size_t ls2 = staged_lds_bytes(b.G, ids);
            if (b.staged2 && ids)
                hipLaunchKernelGGL(k_bin2_scatter_staged<true>, dim3(b.nb2), dim3(kBinBlock), ls2, s, w.z1, w.key1,
                                   w.id1, w.off1, w.cbase, b.S1, b.G, b.CT, b.nb2, w.cnt2, w.off, w.rz, w.rmeta, w.rid);
            else if (b.staged2)
                hipLaunchKernelGGL(k_bin2_scatter_staged<false>, dim3(b.nb2), dim3(kBinBlock), ls2, s, w.z1, w.key1,
                                   w.id1, w.off1, w.cbase, b.S1, b.G, b.CT, b.nb2, w.cnt2, w.off, w.rz, w.rmeta, w.rid);
            else if (ids)
                hipLaunchKernelGGL(k_bin2_scatter<true>, dim3(b.nb2), dim3(kBinBlock), l2, s, w.z1, w.key1, w.id1,
                                   w.off1, w.cbase, b.S1, b.G, b.CT, b.nb2, w.cnt2, w.off, w.rz, w.rmeta, w.rid);
            else
                hipLaunchKernelGGL(k_bin2_scatter<false>, dim3(b.nb2), dim3(kBinBlock), l2, s, w.z1, w.key1, w.id1,
                                   w.off1, w.cbase, b.S1, b.G, b.CT, b.nb2, w.cnt2, w.off, w.rz, w.rmeta, w.rid);
            PCT_LAUNCH_CHECK();
        }
    }
    const int cap = reduce_cap(n, g, ids);
    const size_t rl = reduce_lds_bytes(g, ids, cap);
    if (ids && merge) {
        if (pct_status st = allow_lds((const void*)k_tile_reduce<true, true>, rl)) return st;
        hipLaunchKernelGGL((k_tile_reduce<true, true>), dim3(g.ntiles), dim3(kReduceBlock), rl, s, w.off, w.rz, w.rmeta,
                           w.rid, g, zmin, ds, N, ground, ceil, ag, ac, cap, id_base);
    } else if (merge) {
        if (pct_status st = allow_lds((const void*)k_tile_reduce<false, true>, rl)) return st;
        hipLaunchKernelGGL((k_tile_reduce<false, true>), dim3(g.ntiles), dim3(kReduceBlock), rl, s, w.off, w.rz, w.rmeta,
                           w.rid, g, zmin, ds, N, ground, ceil, ag, ac, cap, id_base);
    } else if (ids) {
        if (pct_status st = allow_lds((const void*)k_tile_reduce<true, false>, rl)) return st;
        hipLaunchKernelGGL((k_tile_reduce<true, false>), dim3(g.ntiles), dim3(kReduceBlock), rl, s, w.off, w.rz, w.rmeta,
                           w.rid, g, zmin, ds, N, ground, ceil, ag, ac, cap, 0);
    } else {
        if (pct_status st = allow_lds((const void*)k_tile_reduce<false, false>, rl)) return st;
        hipLaunchKernelGGL((k_tile_reduce<false, false>), dim3(g.ntiles), dim3(kReduceBlock), rl, s, w.off, w.rz,
                           w.rmeta, w.rid, g, zmin, ds, N, ground, ceil, ag, ac, cap, 0);
    }
    PCT_LAUNCH_CHECK();
    return PCT_OK;
}

// Bounding box of the cells that the in-grid points of a batch fall in:
// bb = {x_min, y_min, x_max, y_max}, to be initialised to {INT_MAX, INT_MAX,
// -1, -1}.
__global__ __launch_bounds__(256) void k_cell_bbox(const float* __restrict__ xyz, int64_t n, GridDev g,
                                                   int* __restrict__ bb) {
    int x0 = 0x7fffffff, y0 = 0x7fffffff, x1 = -1, y1 = -1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
        int ix, iy;
        if (!isfinite(x) || !isfinite(y) || !isfinite(z) || !rasterize(x, y, g, ix, iy)) continue;
        x0 = min(x0, ix);
        y0 = min(y0, iy);
        x1 = max(x1, ix);
        y1 = max(y1, iy);
    }
    for (int o = 32; o > 0; o >>= 1) {
        x0 = min(x0, __shfl_xor(x0, o, 64));
        y0 = min(y0, __shfl_xor(y0, o, 64));
        x1 = max(x1, __shfl_xor(x1, o, 64));
        y1 = max(y1, __shfl_xor(y1, o, 64));
    }
    // one set of atomics per workgroup: they all go to the same four words
    __shared__ int s_bb[4][4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_bb[w][0] = x0;
        s_bb[w][1] = y0;
        s_bb[w][2] = x1;
        s_bb[w][3] = y1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < 4; ++v) {
            x0 = min(x0, s_bb[v][0]);
            y0 = min(y0, s_bb[v][1]);
            x1 = max(x1, s_bb[v][2]);
            y1 = max(y1, s_bb[v][3]);
        }
    }
    if (threadIdx.x == 0 && x1 >= 0) {
        atomicMin(&bb[0], x0);
        atomicMin(&bb[1], y0);
        atomicMax(&bb[2], x1);
        atomicMax(&bb[3], y1);
    }
}

__global__ void k_bbox_init(int* bb) {
    bb[0] = 0x7fffffff;
    bb[1] = 0x7fffffff;
    bb[2] = -1;
    bb[3] = -1;
}

pct_status launch_cell_bbox(const float* xyz, int64_t n, const GridDev& g, int* d_bb, hipStream_t s) {
    hipLaunchKernelGGL(k_bbox_init, dim3(1), dim3(1), 0, s, d_bb);
    PCT_LAUNCH_CHECK();
    if (n > 0) {
        const int64_t blocks = std::min<int64_t>(512, (n + 255) / 256);
        hipLaunchKernelGGL(k_cell_bbox, dim3((unsigned)blocks), dim3(256), 0, s, xyz, n, g, d_bb);
        PCT_LAUNCH_CHECK();
    }
    return PCT_OK;
}

GridDev make_grid_dev(const pct_grid& gr) {
    GridDev g{};
    g.x0 = gr.x0;
    g.y0 = gr.y0;
    g.res = gr.res;
    g.nx = gr.nx;
    g.ny = gr.ny;
    g.fnx = (float)gr.nx;
    g.fny = (float)gr.ny;
    g.tw = kBuildTileW;
    g.ntx = (gr.nx + kBuildTileW - 1) / kBuildTileW;
    g.th = 2;
    while (g.th < 8 && (int64_t)g.ntx * ((gr.ny + g.th - 1) / g.th) > kMaxLdsTiles) g.th *= 2;
    g.nty = (gr.ny + g.th - 1) / g.th;
    g.ntiles = g.ntx * g.nty;
    return g;
}

GridDev tile_shape(GridDev g, int tw, int th) {
    g.tw = tw;
    g.th = th;
    g.ntx = (g.nx + tw - 1) / tw;
    g.nty = (g.ny + th - 1) / th;
    g.ntiles = g.ntx * g.nty;
    return g;
}

size_t batch_extent_ws_bytes(const BuildItemDev* items, int n_items) {
    long long nch = 0;
    for (int i = 0; i < n_items; ++i) nch += std::max<long long>(1, (items[i].n + kBatchEChunk - 1) / kBatchEChunk);
    return align_up(sizeof(BuildItemDev) * (size_t)n_items) + 2 * align_up(sizeof(float) * (size_t)nch) +
           align_up(sizeof(unsigned long long) * (size_t)nch) + align_up(sizeof(ExtentDev) * (size_t)n_items);
}

pct_status launch_extent_batched(const float* xyz, const BuildItemDev* h_items, int n_items, void* ws,
                                 ExtentDev* h_out, int upload, hipStream_t s) {
    long long nch = 0;
    for (int i = 0; i < n_items; ++i) nch += std::max<long long>(1, (h_items[i].n + kBatchEChunk - 1) / kBatchEChunk);
    char* p = (char*)ws;
    BuildItemDev* d_items = (BuildItemDev*)p;
    p += align_up(sizeof(BuildItemDev) * (size_t)n_items);
    float* pmin = (float*)p;
    p += align_up(sizeof(float) * (size_t)nch);
    float* pmax = (float*)p;
    p += align_up(sizeof(float) * (size_t)nch);
    unsigned long long* pused = (unsigned long long*)p;
    p += align_up(sizeof(unsigned long long) * (size_t)nch);
    ExtentDev* d_out = (ExtentDev*)p;
    if (upload) {
        PCT_HIP(hipMemcpyAsync(d_items, h_items, sizeof(BuildItemDev) * n_items, hipMemcpyHostToDevice, s));
        PCT_HIP(hipStreamSynchronize(s));   // the host table is temporary
    }
    hipLaunchKernelGGL(k_bextent, dim3((unsigned)nch), dim3(kBlock), 0, s, xyz, d_items, n_items, pmin, pmax, pused);
    PCT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_bextent_final, dim3(n_items), dim3(kBlock), 0, s, d_items, n_items, (int)nch, pmin, pmax, pused,
                       d_out);
    PCT_LAUNCH_CHECK();
    if (h_out) {
        PCT_HIP(hipMemcpyAsync(h_out, d_out, sizeof(ExtentDev) * n_items, hipMemcpyDeviceToHost, s));
        PCT_HIP(hipStreamSynchronize(s));
    }
    return PCT_OK;
}

size_t batch_build_ws_bytes(const BuildItemDev* items, int n_items, bool ids) {
    return carve_batch_ws(nullptr, items, n_items, ids).bytes;
}

pct_status launch_build_batched(const float* xyz, const BuildItemDev* h_items, int n_items, float* ground, float* ceil,
                                int32_t* ag, int32_t* ac, void* ws, size_t ws_bytes, int upload, hipStream_t s) {
    const bool ids = ag != nullptr;
    BatchWs w = carve_batch_ws(ws, h_items, n_items, ids);
    if (w.bytes > ws_bytes) return fail(PCT_ERR_WORKSPACE, "batch workspace too small: %zu < %zu", ws_bytes, w.bytes);
    Digest dg;
    for (int i = 0; i < n_items; ++i) {
        const BuildItemDev& d = h_items[i];
        dg.add(d.g.x0), dg.add(d.g.y0), dg.add(d.g.res), dg.add(d.g.nx), dg.add(d.g.ny), dg.add(d.g.th), dg.add(d.g.tw);
        dg.add(d.g.ntiles), dg.add(d.xyz_off), dg.add(d.n), dg.add(d.zmin), dg.add(d.ds), dg.add(d.N);
        dg.add(d.out_off), dg.add(d.tile_base), dg.add(d.chunk_base), dg.add(d.echunk_base);
    }
    if (pct_status st = resident_tables(w.items, 0, dg.h, upload != 0)) return st;
    if (upload) {
        // the table lives in pageable host memory that the caller releases
        // on return: wait until the copy has read it
        PCT_HIP(hipMemcpyAsync(w.items, h_items, sizeof(BuildItemDev) * n_items, hipMemcpyHostToDevice, s));
        PCT_HIP(hipStreamSynchronize(s));
    }
    int max_tiles_lds = 0, cap = 0;
    for (int i = 0; i < n_items; ++i) {
        if (h_items[i].g.ntiles <= kMaxLdsTiles) max_tiles_lds = std::max(max_tiles_lds, h_items[i].g.ntiles);
        cap = std::max(cap, reduce_cap(h_items[i].n, h_items[i].g, ids));
    }
    cap = std::max(cap, ids ? kReduceCapIds : kReduceCap);
    // the largest tile (tw x th cells) of any item sizes the counters
    size_t max_reduce_lds = 0;
    for (int i = 0; i < n_items; ++i) max_reduce_lds = std::max(max_reduce_lds, reduce_lds_bytes(h_items[i].g, ids, cap));
    if (pct_status st = allow_lds(ids ? (const void*)k_breduce<true> : (const void*)k_breduce<false>, max_reduce_lds))
        return st;
    hipLaunchKernelGGL(k_fill_u32, dim3(std::min(1024, w.total_tiles / kBlock + 1)), dim3(kBlock), 0, s, w.count,
                       (int64_t)w.total_tiles + 1, 0u);
    PCT_LAUNCH_CHECK();
    if (w.total_chunks > 0) {
        hipLaunchKernelGGL(k_bcount, dim3(w.total_chunks), dim3(kBlock), sizeof(unsigned) * max_tiles_lds, s, xyz, w.items,
                           n_items, w.count);
        PCT_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, w.count, w.total_tiles, w.off, w.cursor);
    PCT_LAUNCH_CHECK();
    if (w.total_chunks > 0) {
        const size_t lb = 2 * sizeof(unsigned) * max_tiles_lds;
        if (ids)
            hipLaunchKernelGGL(k_bscatter<true>, dim3(w.total_chunks), dim3(kBlock), lb, s, xyz, w.items, n_items,
                               w.cursor, w.rz, w.rmeta, w.rid);
        else
            hipLaunchKernelGGL(k_bscatter<false>, dim3(w.total_chunks), dim3(kBlock), lb, s, xyz, w.items, n_items,
                               w.cursor, w.rz, w.rmeta, w.rid);
        PCT_LAUNCH_CHECK();
    }
    if (w.total_tiles > 0) {
        if (ids)
            hipLaunchKernelGGL(k_breduce<true>, dim3(w.total_tiles), dim3(kReduceBlock), max_reduce_lds, s, w.off, w.rz, w.rmeta,
                               w.rid, w.items, n_items, ground, ceil, ag, ac, cap);
        else
            hipLaunchKernelGGL(k_breduce<false>, dim3(w.total_tiles), dim3(kReduceBlock), max_reduce_lds, s, w.off, w.rz,
                               w.rmeta, w.rid, w.items, n_items, ground, ceil, ag, ac, cap);
        PCT_LAUNCH_CHECK();
    }
    return PCT_OK;
}

}  // namespace pct
