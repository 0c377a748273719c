// CPU stand-in for the parts of the HIP runtime and device intrinsics that
// libpct's kernel sources use, so that the same sources can be compiled by
// the host compiler (with AddressSanitizer) and executed on the CPU.
//
// Execution model: the blocks of a launch run one after another on one OS
// thread; the threads of a block run as cooperative fibers that switch only
// at __syncthreads() and at cross-lane operations (__shfl, __shfl_xor,
// __ballot, DPP moves, readfirstlane).  A cross-lane operation completes
// when every live lane of the 64-lane wavefront has reached it; a barrier
// completes when every live thread of the block has reached it.  A block
// whose live threads are all waiting without either condition holding is
// reported as a divergent synchronisation and the process aborts.
//
// Memory: device pointers are host pointers.  Dynamic LDS is a fresh heap
// allocation of exactly the launch's byte count, static LDS arrays are
// function-local statics (one block runs at a time), so AddressSanitizer
// reports out-of-bounds accesses to either, and to global buffers.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <tuple>
#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __constant__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)

struct alignas(16) float4 {
    float x, y, z, w;
};

struct dim3 {
    unsigned x, y, z;
    constexpr dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct emu_uint3 {
    unsigned x, y, z;
};
extern emu_uint3 threadIdx, blockIdx, blockDim, gridDim;

typedef enum hipError_t {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorInvalidConfiguration = 9,
    hipErrorLaunchFailure = 719,
} hipError_t;
typedef struct emu_stream* hipStream_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipGetLastError();
const char* hipGetErrorString(hipError_t e);
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute attr, int value);
// One device (ordinal 0); a __device__ variable's address is its host address.
typedef int hipDevice_t;
hipError_t hipGetDevice(int* device);
hipError_t hipStreamGetDevice(hipStream_t s, hipDevice_t* device);
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol);
#define HIP_SYMBOL(x) ((const void*)&(x))
// Device memory is host memory (calloc'd, so the sanitizer sees its bounds).
hipError_t hipMalloc(void** ptr, size_t n);
hipError_t hipFree(void* ptr);
struct hipDeviceProp_t {
    char gcnArchName[256];
};
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int device);
typedef struct emu_event* hipEvent_t;
hipError_t hipEventCreate(hipEvent_t* e);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b);
// Graph capture is not emulated: the calls fail with "invalid argument".
typedef struct emu_graph* hipGraph_t;
typedef struct emu_graph_exec* hipGraphExec_t;
typedef struct emu_graph_node* hipGraphNode_t;
enum hipStreamCaptureMode { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal, hipStreamCaptureModeRelaxed };
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode mode);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g);
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t* err_node, char* log, size_t log_size);
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s);
hipError_t hipGraphExecDestroy(hipGraphExec_t e);
hipError_t hipGraphDestroy(hipGraph_t g);

namespace emu {

enum WaveOp { OP_SHFL = 1, OP_SHFL_XOR, OP_BALLOT, OP_DPP, OP_READFIRSTLANE };

// Suspends the calling lane until every live lane of its wavefront has
// reached a cross-lane operation of the same kind, then returns this lane's
// result.  `arg` is the source lane / xor mask / DPP control, `old` the DPP
// fallback value.
uint64_t wave_op(int op, uint64_t value, int arg, uint64_t old);
void syncthreads();
void* dyn_smem();
unsigned lane_id();

bool begin_launch(const char* name, const void* fn, dim3 grid, dim3 block, size_t smem);
// Aborts when the running launch has more threads per workgroup than the
// kernel's __launch_bounds__ (the hardware would not run such a launch).
void check_launch_bound(int bound, const char* fn);
void run_blocks(void (*thunk)(void*), void* ctx);

template <class T>
uint64_t to_bits(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lane values only");
    uint64_t b = 0;
    memcpy(&b, &v, sizeof(T));
    return b;
}
template <class T>
T from_bits(uint64_t b) {
    T v;
    memcpy(&v, &b, sizeof(T));
    return v;
}

template <class F>
void thunk(void* p) {
    (*static_cast<F*>(p))();
}

template <class... P, class... A>
void launch(const char* name, void (*k)(P...), dim3 grid, dim3 block, size_t smem, hipStream_t, A&&... a) {
    static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
    if (!begin_launch(name, (const void*)k, grid, block, smem)) return;
    std::tuple<std::decay_t<P>...> args(static_cast<std::decay_t<P>>(a)...);
    auto body = [&]() { std::apply(k, args); };
    run_blocks(&thunk<decltype(body)>, &body);
}

}  // namespace emu

#define hipLaunchKernelGGL(k, grid, block, smem, stream, ...) \
    ::emu::launch(#k, k, dim3(grid), dim3(block), (size_t)(smem), stream, ##__VA_ARGS__)

#define __syncthreads() ::emu::syncthreads()

template <class T>
inline T __shfl(T v, int src, int width = 64) {
    (void)width;
    return emu::from_bits<T>(emu::wave_op(emu::OP_SHFL, emu::to_bits(v), src, 0));
}
template <class T>
inline T __shfl_xor(T v, int mask, int width = 64) {
    (void)width;
    return emu::from_bits<T>(emu::wave_op(emu::OP_SHFL_XOR, emu::to_bits(v), mask, 0));
}
inline unsigned long long __ballot(int pred) { return emu::wave_op(emu::OP_BALLOT, pred ? 1u : 0u, 0, 0); }
// Lanes whose source lane is outside the wavefront or inactive get `old`,
// or 0 with bound_ctrl.
// DPP moves: wave_shr:1, wave_shl:1, row_shr:1..15, row_bcast:15 and
// row_bcast:31; lanes of rows outside row_mask keep `old` (so a row mask
// needs bound_ctrl off, where invalid sources give `old` too).
inline int emu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    if (bank_mask != 0xf || (row_mask != 0xf && bound_ctrl)) __builtin_trap();
    return emu::from_bits<int>(emu::wave_op(emu::OP_DPP, emu::to_bits(src), ctrl | (row_mask << 12),
                                            emu::to_bits(bound_ctrl ? 0 : old)));
}
template <class T>
inline T emu_readlane(T v, int lane) {
    return emu::from_bits<T>(emu::wave_op(emu::OP_SHFL, emu::to_bits(v), lane, 0));
}
inline int emu_readfirstlane(int v) { return emu::from_bits<int>(emu::wave_op(emu::OP_READFIRSTLANE, emu::to_bits(v), 0, 0)); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
inline int __popc(unsigned v) { return __builtin_popcount(v); }
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
#define __builtin_amdgcn_update_dpp emu_update_dpp
#define __builtin_nontemporal_store(v, p) (void)(*(p) = (v))
#define __builtin_amdgcn_readfirstlane emu_readfirstlane
#define __builtin_amdgcn_readlane emu_readlane

// Raw buffer access (stride 0): offset = voffset + soffset bytes from the
// descriptor's base.  The hardware returns 0 for reads and drops writes
// beyond num_records; the library never relies on that, so here such an
// access aborts.
struct emu_buffer_rsrc {
    char* base;
    unsigned num;
};
typedef emu_buffer_rsrc __amdgpu_buffer_rsrc_t;
inline emu_buffer_rsrc emu_make_buffer_rsrc(void* p, short stride, int num, int flags) {
    (void)flags;
    if (stride != 0) __builtin_trap();
    return emu_buffer_rsrc{(char*)p, (unsigned)num};
}
inline char* emu_buffer_addr(emu_buffer_rsrc r, int voff, int soff) {
    const unsigned long long off = (unsigned long long)(unsigned)voff + (unsigned)soff;
    if (off + 4 > r.num) __builtin_trap();
    return r.base + off;
}
inline unsigned emu_raw_buffer_load_b32(emu_buffer_rsrc r, int voff, int soff, int aux) {
    (void)aux;
    unsigned v;
    memcpy(&v, emu_buffer_addr(r, voff, soff), 4);
    return v;
}
inline unsigned long long emu_raw_buffer_load_b64(emu_buffer_rsrc r, int voff, int soff, int aux) {
    (void)aux;
    const unsigned long long off = (unsigned long long)(unsigned)voff + (unsigned)soff;
    if (off + 8 > r.num) __builtin_trap();
    unsigned long long v;
    memcpy(&v, r.base + off, 8);
    return v;
}
inline void emu_raw_buffer_store_b32(unsigned v, emu_buffer_rsrc r, int voff, int soff, int aux) {
    (void)aux;
    memcpy(emu_buffer_addr(r, voff, soff), &v, 4);
}
#define __builtin_amdgcn_make_buffer_rsrc emu_make_buffer_rsrc
#define __builtin_amdgcn_raw_buffer_load_b32 emu_raw_buffer_load_b32
#define __builtin_amdgcn_raw_buffer_load_b64 emu_raw_buffer_load_b64
#define __builtin_amdgcn_raw_buffer_store_b32 emu_raw_buffer_store_b32
// A wavefront barrier: every live lane of the wavefront arrives before any
// continues (the fences around it need nothing more here).
inline void emu_wave_barrier() { (void)emu::wave_op(emu::OP_BALLOT, 1u, 0, 0); }
#define __builtin_amdgcn_wave_barrier emu_wave_barrier
#define __builtin_amdgcn_fence(order, scope) ((void)0)

// Fibers switch only at the operations above, so read-modify-write needs no
// further protection.
template <class T>
inline T atomicAdd(T* p, T v) {
    T o = *p;
    *p = o + v;
    return o;
}
template <class T>
inline T atomicMax(T* p, T v) {
    T o = *p;
    *p = o > v ? o : v;
    return o;
}
template <class T>
inline T atomicMin(T* p, T v) {
    T o = *p;
    *p = o < v ? o : v;
    return o;
}
template <class T>
inline T atomicOr(T* p, T v) {
    T o = *p;
    *p = o | v;
    return o;
}

template <class T, class U>
inline typename std::common_type<T, U>::type min(T a, U b) {
    typedef typename std::common_type<T, U>::type C;
    return (C)a < (C)b ? (C)a : (C)b;
}
template <class T, class U>
inline typename std::common_type<T, U>::type max(T a, U b) {
    typedef typename std::common_type<T, U>::type C;
    return (C)a > (C)b ? (C)a : (C)b;
}
