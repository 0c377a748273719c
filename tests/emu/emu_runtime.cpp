// Fiber scheduler and runtime entry points of the CPU stand-in declared in
// hip/hip_runtime.h.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <setjmp.h>
#include <sys/mman.h>
#include <ucontext.h>

#include <chrono>
#include <map>
#include <vector>

#include "hip/hip_runtime.h"

#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#else
#define EMU_ASAN 0
#endif

emu_uint3 threadIdx, blockIdx, blockDim, gridDim;

namespace emu {
namespace {

constexpr size_t kStack = 512 * 1024;
constexpr size_t kDefaultLds = 64 * 1024;
constexpr size_t kMaxLds = 160 * 1024;

enum State { RUN, AT_SYNC, AT_WAVE, DONE };

// A fiber is entered the first time with swapcontext (which also switches
// stacks); every later switch is a _setjmp/_longjmp pair, which saves no
// signal mask and so makes no system call.
struct Fiber {
    ucontext_t ctx;
    jmp_buf jb;
    bool started = false;
    char* stack = nullptr;
    State state = RUN;
    int op = 0, arg = 0;
    uint64_t val = 0, old = 0, res = 0;
    void* fake = nullptr;
};

struct Sched {
    ucontext_t main;
    jmp_buf main_jb;
    std::vector<Fiber> f;
    int n = 0, cur = -1;
    void (*thunk)(void*) = nullptr;
    void* ctx = nullptr;
    void* smem = nullptr;
    const char* name = "";
    const void* main_bottom = nullptr;
    size_t main_size = 0;
    void* main_fake = nullptr;
} S;

hipError_t g_last = hipSuccess;
std::map<const void*, size_t> g_lds_limit;
long long g_launches = 0;

void set_tid(int t) {
    threadIdx.x = t % blockDim.x;
    threadIdx.y = (t / blockDim.x) % blockDim.y;
    threadIdx.z = t / (blockDim.x * blockDim.y);
}

void to_main() {
    Fiber& me = S.f[S.cur];
#if EMU_ASAN
    __sanitizer_start_switch_fiber(me.state == DONE ? nullptr : &me.fake, S.main_bottom, S.main_size);
#endif
    if (!_setjmp(me.jb)) _longjmp(S.main_jb, 1);
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(me.fake, &S.main_bottom, &S.main_size);
#endif
}

void fiber_entry() {
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &S.main_bottom, &S.main_size);
#endif
    S.thunk(S.ctx);
    S.f[S.cur].state = DONE;
    to_main();
    __builtin_trap();   // a finished fiber is never resumed
}

void resume(int i) {
    S.cur = i;
    set_tid(i);
    Fiber& f = S.f[i];
#if EMU_ASAN
    __sanitizer_start_switch_fiber(&S.main_fake, f.stack, kStack);
#endif
    if (!_setjmp(S.main_jb)) {
        if (!f.started) {
            f.started = true;
            swapcontext(&S.main, &f.ctx);
        } else {
            _longjmp(f.jb, 1);
        }
    }
#if EMU_ASAN
    __sanitizer_finish_switch_fiber(S.main_fake, nullptr, nullptr);
#endif
    S.cur = -1;
}

[[noreturn]] void die(const char* what) {
    fprintf(stderr, "[emu] %s in kernel %s, block (%u,%u,%u)\n", what, S.name, blockIdx.x, blockIdx.y, blockIdx.z);
    for (int i = 0; i < S.n; ++i)
        if (S.f[i].state != DONE)
            fprintf(stderr, "[emu]   thread %d state %d op %d\n", i, (int)S.f[i].state, S.f[i].op);
    fflush(stderr);
    abort();
}

// Completes the cross-lane operation of wavefront w if all its live lanes
// wait at one.  Returns whether lanes were released.
bool try_wave(int w) {
    const int l0 = w * 64, l1 = std::min(S.n, l0 + 64);
    int op = 0, dpp_ctrl = 0;
    bool any = false;
    for (int i = l0; i < l1; ++i) {
        const Fiber& f = S.f[i];
        if (f.state == DONE) continue;
        if (f.state != AT_WAVE) return false;
        if (any && f.op != op) die("lanes of one wavefront at different cross-lane operations");
        if (any && f.op == OP_DPP && f.arg != dpp_ctrl) die("lanes of one wavefront at different DPP moves");
        op = f.op;
        dpp_ctrl = f.arg;
        any = true;
    }
    if (!any) return false;
    auto live = [&](int lane) { return l0 + lane < l1 && S.f[l0 + lane].state == AT_WAVE; };
    uint64_t ballot = 0;
    int first = -1;
    for (int l = 0; l < l1 - l0; ++l)
        if (live(l)) {
            if (first < 0) first = l;
            if (op == OP_BALLOT && S.f[l0 + l].val) ballot |= 1ull << l;
        }
    const uint64_t poison = 0x7fc00bad7fc00badull;   // value of a lane that has exited
    for (int l = 0; l < l1 - l0; ++l) {
        Fiber& f = S.f[l0 + l];
        if (f.state != AT_WAVE) continue;
        switch (op) {
            case OP_SHFL: {
                const int src = f.arg & 63;
                f.res = live(src) ? S.f[l0 + src].val : poison;
                break;
            }
            case OP_SHFL_XOR: {
                const int src = (l ^ f.arg) & 63;
                f.res = live(src) ? S.f[l0 + src].val : poison;
                break;
            }
            case OP_BALLOT: f.res = ballot; break;
            case OP_READFIRSTLANE: f.res = S.f[l0 + first].val; break;
            case OP_DPP: {
                const int ctrl = f.arg & 0xfff, rmask = (f.arg >> 12) & 0xf, row = l / 16;
                if (!((rmask >> row) & 1)) {   // row not written
                    f.res = f.old;
                    break;
                }
                int src;
                if (ctrl == 0x138) src = l - 1;                                   // wave_shr:1
                else if (ctrl == 0x130) src = l + 1;                              // wave_shl:1
                else if (ctrl > 0x110 && ctrl <= 0x11f) src = (l % 16 >= (ctrl & 0xf)) ? l - (ctrl & 0xf) : -1;  // row_shr
                else if (ctrl == 0x142) src = row >= 1 ? 16 * row - 1 : -1;       // row_bcast:15
                else if (ctrl == 0x143) src = row >= 2 ? 31 : -1;                 // row_bcast:31
                else die("unsupported DPP control");
                f.res = (src >= 0 && src < 64 && live(src)) ? S.f[l0 + src].val : f.old;
                break;
            }
            default: die("unknown cross-lane operation");
        }
    }
    for (int i = l0; i < l1; ++i)
        if (S.f[i].state == AT_WAVE) S.f[i].state = RUN;
    return true;
}

// Order in which runnable wavefronts are resumed within a phase: 0 in
// order, 1 reversed, 2 pseudo-random (EMU_ORDER=fwd|rev|rand).  Lanes of a
// wavefront always run in order.  A missing barrier between wavefronts shows
// up as a result that depends on this order.
int wave_order() {
    static int o = -1;
    if (o < 0) {
        const char* e = getenv("EMU_ORDER");
        o = !e ? 0 : !strcmp(e, "rev") ? 1 : !strcmp(e, "rand") ? 2 : 0;
    }
    return o;
}
uint64_t g_rng = 0x9E3779B97F4A7C15ull;

void run_block() {
    const int n = S.n;
    const int nw = (n + 63) / 64;
    std::vector<int> order(nw);
    for (int w = 0; w < nw; ++w) order[w] = w;
    for (int i = 0; i < n; ++i) {
        Fiber& f = S.f[i];
        f.state = RUN;
        f.fake = nullptr;
        f.started = false;
        getcontext(&f.ctx);
        f.ctx.uc_stack.ss_sp = f.stack;
        f.ctx.uc_stack.ss_size = kStack;
        f.ctx.uc_link = nullptr;
        makecontext(&f.ctx, (void (*)())fiber_entry, 0);
    }
    int live = n;
    while (live > 0) {
        if (wave_order() == 1) {
            for (int w = 0; w < nw; ++w) order[w] = nw - 1 - w;
        } else if (wave_order() == 2) {
            for (int w = nw - 1; w > 0; --w) {
                g_rng ^= g_rng << 13;
                g_rng ^= g_rng >> 7;
                g_rng ^= g_rng << 17;
                std::swap(order[w], order[g_rng % (uint64_t)(w + 1)]);
            }
        }
        for (int oi = 0; oi < nw; ++oi) {
            const int w = order[oi];
            for (int i = w * 64; i < std::min(n, w * 64 + 64); ++i)
                if (S.f[i].state == RUN) resume(i);
        }
        live = 0;
        bool all_sync = true;
        for (int i = 0; i < n; ++i) {
            if (S.f[i].state == DONE) continue;
            ++live;
            if (S.f[i].state != AT_SYNC) all_sync = false;
        }
        if (live == 0) break;
        bool released = false;
        for (int w = 0; w * 64 < n; ++w) released |= try_wave(w);
        if (released) continue;
        if (all_sync) {
            for (int i = 0; i < n; ++i)
                if (S.f[i].state == AT_SYNC) S.f[i].state = RUN;
            continue;
        }
        die("divergent synchronisation (threads wait at different barriers)");
    }
}

}  // namespace

uint64_t wave_op(int op, uint64_t value, int arg, uint64_t old) {
    if (S.cur < 0) {
        fprintf(stderr, "[emu] cross-lane operation outside a kernel\n");
        abort();
    }
    Fiber& me = S.f[S.cur];
    me.op = op;
    me.val = value;
    me.arg = arg;
    me.old = old;
    me.state = AT_WAVE;
    to_main();
    return S.f[S.cur].res;
}

void syncthreads() {
    Fiber& me = S.f[S.cur];
    me.op = 0;
    me.state = AT_SYNC;
    to_main();
}

void* dyn_smem() { return S.smem; }

void check_launch_bound(int bound, const char* fn) {
    const unsigned nt = blockDim.x * blockDim.y * blockDim.z;
    if ((long long)nt > bound) {
        fprintf(stderr, "[emu] %s launched with %u threads per workgroup, above its launch bound %d\n", fn, nt, bound);
        fflush(stderr);
        abort();
    }
}

unsigned lane_id() { return (unsigned)S.cur & 63u; }

bool begin_launch(const char* name, const void* fn, dim3 grid, dim3 block, size_t smem) {
    ++g_launches;
    const unsigned long long nt = (unsigned long long)block.x * block.y * block.z;
    if (grid.x == 0 || grid.y == 0 || grid.z == 0 || nt == 0 || nt > 1024 || grid.y > 65535 || grid.z > 65535) {
        fprintf(stderr, "[emu] invalid launch configuration of %s: grid (%u,%u,%u) block (%u,%u,%u)\n", name, grid.x,
                grid.y, grid.z, block.x, block.y, block.z);
        g_last = hipErrorInvalidConfiguration;
        return false;
    }
    auto it = g_lds_limit.find(fn);
    const size_t lim = it == g_lds_limit.end() ? kDefaultLds : it->second;
    if (smem > lim) {
        fprintf(stderr, "[emu] %s requests %zu bytes of dynamic LDS (limit %zu)\n", name, smem, lim);
        g_last = hipErrorInvalidValue;
        return false;
    }
    S.name = name;
    gridDim = {grid.x, grid.y, grid.z};
    blockDim = {block.x, block.y, block.z};
    S.n = (int)nt;
    free(S.smem);
    S.smem = malloc(smem ? smem : 1);   // exact size, so out-of-range LDS accesses are reported
    memset(S.smem, 0xA5, smem);         // LDS starts with unspecified contents
    if ((int)S.f.size() < S.n) {
        const size_t old = S.f.size();
        S.f.resize(S.n);
        for (size_t i = old; i < S.f.size(); ++i) {
            void* p = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
            if (p == MAP_FAILED) abort();
            S.f[i].stack = (char*)p;
        }
    }
    return true;
}

void run_blocks(void (*thunk)(void*), void* ctx) {
    S.thunk = thunk;
    S.ctx = ctx;
    for (unsigned z = 0; z < gridDim.z; ++z)
        for (unsigned y = 0; y < gridDim.y; ++y)
            for (unsigned x = 0; x < gridDim.x; ++x) {
                blockIdx = {x, y, z};
                run_block();
            }
    free(S.smem);
    S.smem = nullptr;
}

}  // namespace emu

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
    memcpy(dst, src, n);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipGetLastError() {
    hipError_t e = emu::g_last;
    emu::g_last = hipSuccess;
    return e;
}
const char* hipGetErrorString(hipError_t e) {
    switch (e) {
        case hipSuccess: return "no error";
        case hipErrorInvalidValue: return "invalid argument";
        case hipErrorInvalidConfiguration: return "invalid configuration argument";
        default: return "launch failure";
    }
}
hipError_t hipFuncSetAttribute(const void* f, hipFuncAttribute attr, int value) {
    if (attr != hipFuncAttributeMaxDynamicSharedMemorySize || value < 0 || (size_t)value > emu::kMaxLds)
        return hipErrorInvalidValue;
    emu::g_lds_limit[f] = (size_t)value;
    return hipSuccess;
}

hipError_t hipGetDevice(int* device) {
    *device = 0;
    return hipSuccess;
}
hipError_t hipMalloc(void** ptr, size_t n) {
    *ptr = calloc(n ? n : 1, 1);
    return *ptr ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipFree(void* ptr) {
    free(ptr);
    return hipSuccess;
}
hipError_t hipGetDeviceProperties(hipDeviceProp_t* prop, int device) {
    if (device != 0) return hipErrorInvalidValue;
    snprintf(prop->gcnArchName, sizeof prop->gcnArchName, "cpu-emulator");
    return hipSuccess;
}
hipError_t hipStreamGetDevice(hipStream_t, hipDevice_t* device) {
    *device = 0;
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol) {
    *ptr = const_cast<void*>(symbol);
    return symbol ? hipSuccess : hipErrorInvalidValue;
}

// Events: launches run to completion when issued, so an event records the
// host clock at the time it is recorded.
struct emu_event {
    std::chrono::steady_clock::time_point t;
};
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = new emu_event{std::chrono::steady_clock::now()};
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    e->t = std::chrono::steady_clock::now();
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorInvalidValue; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
    *g = nullptr;
    return hipErrorInvalidValue;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, hipGraphNode_t*, char*, size_t) {
    *e = nullptr;
    return hipErrorInvalidValue;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}

extern "C" {
void* emu_alloc(size_t bytes) { return malloc(bytes ? bytes : 1); }
void emu_free(void* p) { free(p); }
long long emu_launch_count() { return emu::g_launches; }
}
