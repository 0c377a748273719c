// Sparse storage of the simplified tomogram (the closing remark of
// Sec. III-C): only the unique cells of the kept slices, Eqs. (8)-(9), each
// as its cell index and its e^G, e^C, c^T, slice after slice in raster
// order.
//
// Two passes over the kept slices: the first counts the unique cells of
// every 1024-cell block, an exclusive scan turns the counts into output
// offsets, the second recomputes the flags and writes each block's unique
// cells at its offset in raster order (ranks from wavefront ballots).
#include <vector>

#include "pct_internal.h"
#include "unique_internal.h"

namespace pct {

namespace {

constexpr int kUBlock = 256;
constexpr int kUCells = 4;                      // cells per lane
constexpr int kUSpan = kUBlock * kUCells;      // cells per workgroup

// Kept slice j: its slice k, the last kept slice p below it (-1: none) and
// whether k is the last slice of the tomogram.
struct UniqSlice {
    int k, p, last;
};

// Unique flags of a lane's four cells c0 .. c0+3 of kept slice sl.
template <bool VEC>
__device__ __forceinline__ unsigned uniq_flags(const float* __restrict__ ground, const float* __restrict__ cost,
                                               long long plane, float cB, UniqSlice sl, long long c0, int nact) {
    float ek[kUCells], ck[kUCells], ep[kUCells], cp[kUCells], eu[kUCells], cu[kUCells];
    const long long ok = (long long)sl.k * plane + c0;
    auto load = [&](const float* a, long long off, float fill, float* v) {
        if (VEC && nact == kUCells) {
            const float4 x = *(const float4*)(a + off);
            v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        } else {
#pragma unroll
            for (int i = 0; i < kUCells; ++i) v[i] = i < nact ? a[off + i] : fill;
        }
    };
    load(ground, ok, -INFINITY, ek);
    load(cost, ok, cB, ck);
    if (sl.p >= 0) {
        const long long op = (long long)sl.p * plane + c0;
        load(ground, op, -INFINITY, ep);
        load(cost, op, cB, cp);
    }
    if (!sl.last) {
        load(ground, ok + plane, -INFINITY, eu);
        load(cost, ok + plane, cB, cu);
    }
    unsigned f = 0;
#pragma unroll
    for (int i = 0; i < kUCells; ++i) {
        const bool trav = i < nact && ck[i] < cB;
        const bool lower = sl.p < 0 || ek[i] > ep[i] || ck[i] < cp[i];
        const bool upper = sl.last || eu[i] > ek[i] || ck[i] < cu[i];
        f |= (trav && lower && upper) ? 1u << i : 0u;
    }
    return f;
}

template <bool VEC>
__global__ __launch_bounds__(kUBlock) void k_uniq_count(const float* __restrict__ ground,
                                                        const float* __restrict__ cost, long long plane, float cB,
                                                        const UniqSlice* __restrict__ slices, int nb,
                                                        unsigned long long* __restrict__ counts) {
    __shared__ unsigned s_wave[kUBlock / 64];
    const int j = blockIdx.y, b = blockIdx.x;
    const long long c0 = (long long)b * kUSpan + (long long)threadIdx.x * kUCells;
    const long long left = plane - c0;
    const int nact = left <= 0 ? 0 : (left < kUCells ? (int)left : kUCells);
    const unsigned f = nact > 0 ? uniq_flags<VEC>(ground, cost, plane, cB, slices[j], c0, nact) : 0u;
    int n = __popc(f);
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x / 64] = (unsigned)n;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = 0;
        for (int w = 0; w < kUBlock / 64; ++w) t += s_wave[w];
        counts[(long long)j * nb + b] = t;
    }
}

// Exclusive scan of n counts in place (one workgroup of 16 wavefronts),
// 4096 counts at a time: four consecutive counts per thread, an inclusive
// scan of the thread sums within each wavefront by shuffles, then the
// wavefront totals across the workgroup.  total[0] receives the sum.
__global__ __launch_bounds__(1024) void k_uniq_scan(unsigned long long* __restrict__ v, long long n,
                                                    unsigned long long* __restrict__ total) {
    __shared__ unsigned long long s_wave[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long carry = 0;
    for (long long base = 0; base < n; base += 4096) {
        const long long i0 = base + 4 * (long long)threadIdx.x;
        unsigned long long x[4], sum = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            x[c] = i0 + c < n ? v[i0 + c] : 0ull;
            sum += x[c];
        }
        unsigned long long incl = sum;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long y = __shfl(incl, lane - o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        unsigned long long before = carry, chunk = 0;
        for (int w = 0; w < 16; ++w) {
            const unsigned long long t = s_wave[w];
            if (w < wave) before += t;
            chunk += t;
        }
        unsigned long long run = before + incl - sum;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (i0 + c < n) v[i0 + c] = run;
            run += x[c];
        }
        carry += chunk;
        __syncthreads();
    }
    if (threadIdx.x == 0) total[0] = carry;
}

template <bool VEC>
__global__ __launch_bounds__(kUBlock) void k_uniq_write(const float* __restrict__ ground,
                                                        const float* __restrict__ ceil,
                                                        const float* __restrict__ cost, long long plane, float cB,
                                                        const UniqSlice* __restrict__ slices, int nb,
                                                        const unsigned long long* __restrict__ offs,
                                                        int* __restrict__ cell, float* __restrict__ g_out,
                                                        float* __restrict__ c_out, float* __restrict__ t_out) {
    __shared__ unsigned s_wave[kUBlock / 64];
    const int j = blockIdx.y, b = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x / 64;
    const long long c0 = (long long)b * kUSpan + (long long)threadIdx.x * kUCells;
    const long long left = plane - c0;
    const int nact = left <= 0 ? 0 : (left < kUCells ? (int)left : kUCells);
    const UniqSlice sl = slices[j];
    const unsigned f = nact > 0 ? uniq_flags<VEC>(ground, cost, plane, cB, sl, c0, nact) : 0u;
    // rank of this lane's first unique cell within the workgroup (raster order)
    const int n = __popc(f);
    int incl = n;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl(incl, lane - o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) s_wave[wave] = (unsigned)incl;
    __syncthreads();
    unsigned before = 0;
    for (int w = 0; w < wave; ++w) before += s_wave[w];
    unsigned long long o = offs[(long long)j * nb + b] + before + (unsigned)(incl - n);
    const long long ks = (long long)sl.k * plane;
    for (int i = 0; i < kUCells; ++i) {
        if (!(f & (1u << i))) continue;
        const long long c = c0 + i;
        cell[o] = (int)c;
        g_out[o] = ground[ks + c];
        c_out[o] = ceil[ks + c];
        t_out[o] = cost[ks + c];
        ++o;
    }
}

__global__ void k_uniq_firsts(const unsigned long long* __restrict__ offs, int nb, int L,
                              unsigned long long* __restrict__ first) {
    for (int j = threadIdx.x; j < L; j += blockDim.x) first[j] = offs[(long long)j * nb];
}

}  // namespace

size_t unique_ws_bytes(int nx, int ny, int N) {
    const long long plane = (long long)nx * ny;
    const long long nb = (plane + kUSpan - 1) / kUSpan;
    return align_up(sizeof(UniqSlice) * (size_t)N) + align_up(sizeof(unsigned long long) * (size_t)(nb * N)) +
           align_up(sizeof(unsigned long long) * (size_t)(N + 1));
}

pct_status launch_unique(const float* ground, const float* ceil, const float* cost, int nx, int ny, int N, float cB,
                         const uint8_t* h_keep, long long capacity, int* cell, float* g_out, float* c_out,
                         float* t_out, long long* h_slice_off, long long* h_count, void* ws, hipStream_t s) {
    const long long plane = (long long)nx * ny;
    const int nb = (int)((plane + kUSpan - 1) / kUSpan);
    UniqSlice h_sl[PCT_MAX_SLICES];
    int L = 0, p = -1;
    for (int k = 0; k < N; ++k) {
        if (!h_keep[k]) continue;
        h_sl[L++] = UniqSlice{k, p, k == N - 1 ? 1 : 0};
        p = k;
    }
    long long total = 0;
    std::vector<unsigned long long> first((size_t)L + 1, 0ull);
    const bool vec = plane % 4 == 0 && ((uintptr_t)ground & 15) == 0 && ((uintptr_t)cost & 15) == 0;
    UniqSlice* d_sl = (UniqSlice*)ws;
    unsigned long long* offs = (unsigned long long*)((char*)ws + align_up(sizeof(UniqSlice) * (size_t)N));
    unsigned long long* d_first =
        (unsigned long long*)((char*)offs + align_up(sizeof(unsigned long long) * (size_t)((long long)nb * N)));
    const dim3 grid((unsigned)nb, (unsigned)L);
    if (L > 0) {
        PCT_HIP(hipMemcpyAsync(d_sl, h_sl, sizeof(UniqSlice) * L, hipMemcpyHostToDevice, s));
        if (vec)
            hipLaunchKernelGGL(k_uniq_count<true>, grid, dim3(kUBlock), 0, s, ground, cost, plane, cB, d_sl, nb, offs);
        else
            hipLaunchKernelGGL(k_uniq_count<false>, grid, dim3(kUBlock), 0, s, ground, cost, plane, cB, d_sl, nb, offs);
        PCT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_uniq_scan, dim3(1), dim3(1024), 0, s, offs, (long long)nb * L, d_first + L);
        PCT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_uniq_firsts, dim3(1), dim3(256), 0, s, offs, nb, L, d_first);
        PCT_LAUNCH_CHECK();
        // the host copy of h_sl must outlive the upload: wait here
        PCT_HIP(hipMemcpyAsync(first.data(), d_first, sizeof(unsigned long long) * (size_t)(L + 1),
                               hipMemcpyDeviceToHost, s));
        PCT_HIP(hipStreamSynchronize(s));
        total = (long long)first[(size_t)L];
    }
    if (h_slice_off) {
        // slice k starts after the unique cells of the kept slices below it
        int j = 0;
        for (int k = 0; k < N; ++k) {
            while (j < L && h_sl[j].k < k) ++j;
            h_slice_off[k] = (long long)first[(size_t)j];
        }
        h_slice_off[N] = total;
    }
    if (cell && total > capacity) {
        *h_count = total;
        return fail(PCT_ERR_CAPACITY, "%lld unique cells exceed the capacity %lld", total, capacity);
    }
    if (cell && total > 0) {
        if (vec)
            hipLaunchKernelGGL(k_uniq_write<true>, grid, dim3(kUBlock), 0, s, ground, ceil, cost, plane, cB, d_sl, nb,
                               offs, cell, g_out, c_out, t_out);
        else
            hipLaunchKernelGGL(k_uniq_write<false>, grid, dim3(kUBlock), 0, s, ground, ceil, cost, plane, cB, d_sl, nb,
                               offs, cell, g_out, c_out, t_out);
        PCT_LAUNCH_CHECK();
    }
    *h_count = total;
    return PCT_OK;
}

}  // namespace pct
