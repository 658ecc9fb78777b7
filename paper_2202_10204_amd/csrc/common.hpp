// Shared definitions of libspai: handle, preconditioner object, error reporting,
// device arithmetic in the precision model of the build, wavefront helpers.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/spai.h"

namespace spai {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

void set_error(const std::string& msg);

struct Status {
    int code = SPAI_OK;
};

#define SPAI_HIP(call)                                                                     \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::spai::set_error(std::string("HIP error in ") + #call + ": " +               \
                              hipGetErrorString(e_));                                      \
            return SPAI_E_HIP;                                                             \
        }                                                                                  \
    } while (0)

#define SPAI_ARG(cond, msg)                                                                \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            ::spai::set_error(std::string("invalid argument: ") + (msg));                 \
            return SPAI_E_ARG;                                                             \
        }                                                                                  \
    } while (0)

// ---------------------------------------------------------------------------
// device memory: grow-only buffers owned by the handle
// ---------------------------------------------------------------------------

// A region of device memory lent to a handle: allocations are taken from it
// front to back and never returned one by one; the lender reclaims the whole
// region once the handle's work in it has completed.
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    size_t used = 0;
    bool owns(const void* p) const { return base && (const char*)p >= base && (const char*)p < base + size; }
};

struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
    Arena from;        // the region it came from (empty: hipMalloc)
};

// Device memory of a handle: from the handle's arena when it has one (a free
// is then a no-op and never waits, where hipFree waits for the whole device;
// an allocation beyond the arena fails with SPAI_E_OOM), else from the
// allocator in force (spai_set_allocator, default hipMalloc / hipFree).
int dev_malloc(spai_handle* h, void** p, size_t bytes);
// the allocator in force, for memory no handle owns (a request server's arena)
int raw_malloc(void** p, size_t bytes, int device, hipStream_t stream);
void raw_free(void* p);
// device address of the workspace array of spai_gmres_ir_noalloc on `device`
// (looked up once per device, with that device current; spai_create does it)
int noalloc_scratch_init(int device);
// whether a solve of n unknowns fits the fused Arnoldi launch on h->num_cu CUs
bool arnoldi_fused_fits(spai_handle* h, int n, int maxit, int ortho);
void dev_free(void* p, const Arena& from);
int buffer_reserve(spai_handle* h, Buffer& b, size_t bytes);
void buffer_free(Buffer& b);

// fixed small device area for counters and reduction results
struct Scalars {
    double h;          // last reduction result
    double norm;       // norm results
    double maxabs[2];  // ||d||_inf, ||x||_inf
    int flag;          // device-side flags
    int count;         // list counters
    int err;           // device-side validation failures
    int pad;
};

struct KernelTimer {
    int every = 0;               // 0: off
    long long seen = 0;          // launches of the class since enabling
    std::vector<hipEvent_t> ev;  // pool of event pairs
    size_t used = 0;             // pairs recorded since the last read
};

}  // namespace spai

struct spai_handle {
    spai::KernelTimer timers[SPAI_KT_COUNT];
    int device = 0;
    hipStream_t stream = nullptr;
    spai::Buffer ws[8];            // scratch buffers, indexed by purpose
    spai::Buffer red;              // reduction partials + ticket counters
    spai::Buffer host_pinned;      // pinned host staging
    int num_cu = 256;
    spai::Arena arena;             // device memory lent by a request server (empty: the allocator in force)
    size_t ws_cap = 0;             // cap on the batched solver's workspace in bytes (0: a quarter of free memory)
    hipEvent_t chunk_ev[2] = {nullptr, nullptr};   // completion of the stop-flag copies of two Arnoldi chunks
    bool no_alloc = false;         // inside spai_gmres_ir_noalloc: no timing events are created
};

struct spai_precond {
    int32_t n = 0;
    int64_t nnz = 0;
    spai_prec val_prec = SPAI_FP32;  // storage format of the values
    spai_prec u_f = SPAI_FP32;       // precision of the build (x0 = P b rounds its input to it)
    int32_t stride = 0;
    int32_t* rowptr = nullptr;  // n+1
    int32_t* col = nullptr;     // nnz
    void* val = nullptr;        // nnz values in val_prec
    double* d = nullptr;        // n
    int32_t* j_ins = nullptr;   // n * stride (build only)
    double* m_ins = nullptr;    // n * stride (build only)
    int32_t* len = nullptr;     // n (build only)
    int32_t* steps = nullptr;   // n (build only)
    double* res = nullptr;      // n (build only)
    int32_t* flags = nullptr;   // n (build only)
    spai::Arena from;             // arena of the building handle (arrays inside it are not freed one by one)
    int32_t side = SPAI_LEFT;     // SPAI_RIGHT: rows hold m_k[i], applied as D (M w)
};

namespace spai {

// workspace slots
enum WsSlot { WS_BUILD0 = 0, WS_BUILD1 = 1, WS_BUILD2 = 2, WS_SOLVE_V = 3, WS_SOLVE_VEC = 4,
              WS_SOLVE_H = 5, WS_MISC = 6, WS_SPARE = 7 };

// per-column flags (device) — the same bits as the public warnings where they overlap
constexpr int CF_EPS = 1 << 0;
constexpr int CF_RANKDEF = 1 << 1;
constexpr int CF_NONFINITE = 1 << 2;
constexpr int CF_DEFERRED = 1 << 3;  // problem exceeded the kernel's capacity: redo in the large kernel
constexpr int CF_FALLBACK = 1 << 4;  // a 16-bit column recomputed in FP32 after a non-finite value

// ---------------------------------------------------------------------------
// device arithmetic.  The build computes in F = float (u_f = FP32/FP16/BF16)
// or F = double (u_f = FP64): every sum is sequential in a stated index order
// and products are accumulated with fused multiply-adds; store<UF>() rounds a
// value at a storage point to u_f (round to nearest even).
// ---------------------------------------------------------------------------

template <int UF> struct UfTraits;
template <> struct UfTraits<SPAI_FP64> { using F = double; };
template <> struct UfTraits<SPAI_FP32> { using F = float; };
template <> struct UfTraits<SPAI_FP16> { using F = float; };
template <> struct UfTraits<SPAI_BF16> { using F = float; };

__device__ __forceinline__ float round_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
    uint32_t bias = 0x7fffu + ((u >> 16) & 1u);
    u = (u + bias) & 0xffff0000u;
    return __uint_as_float(u);
}

// Keeps the compiler from merging the preceding FP32 operation into the
// conversion (v_fma_mixlo_f16 would round a*b+c once, straight to FP16, while
// the model rounds to FP32 first and then to the storage format).
__device__ __forceinline__ float opaque(float x) {
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ float round_fp16(float x) { return __half2float(__float2half_rn(opaque(x))); }

template <int UF, typename F>
__device__ __forceinline__ F store(F x) {
    if constexpr (UF == SPAI_FP16) return round_fp16(x);
    else if constexpr (UF == SPAI_BF16) return round_bf16(x);
    else return x;
}

// FP64 product d * a rounded to u_f (the gathered entries of B = A^T D)
template <int UF>
__device__ __forceinline__ typename UfTraits<UF>::F scaled_entry(double d, double a) {
    using F = typename UfTraits<UF>::F;
    double p = d * a;
    return store<UF, F>(static_cast<F>(p));
}

__device__ __forceinline__ float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fsqrt(float a) { return __builtin_sqrtf(a); }
__device__ __forceinline__ double fsqrt(double a) { return __builtin_sqrt(a); }

// P value formats
template <int VP> struct ValType;
template <> struct ValType<SPAI_FP64> { using T = double; };
template <> struct ValType<SPAI_FP32> { using T = float; };
template <> struct ValType<SPAI_FP16> { using T = __half; };
template <> struct ValType<SPAI_BF16> { using T = __hip_bfloat16; };

__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(__half v) { return (double)__half2float(v); }
__device__ __forceinline__ double to_f64(__hip_bfloat16 v) { return (double)__bfloat162float(v); }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(__half v) { return __half2float(v); }
__device__ __forceinline__ float to_f32(__hip_bfloat16 v) { return __bfloat162float(v); }

// ---------------------------------------------------------------------------
// wavefront helpers
// ---------------------------------------------------------------------------

// Orders LDS accesses of the lanes of one wavefront: the LDS executes a wave's
// instructions in issue order, so only the compiler must be kept from moving
// accesses across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// ---------------------------------------------------------------------------
// sampled launch timing (host)
// ---------------------------------------------------------------------------

// Returns the index of the event pair to close after the launch, or -1.
inline long timer_begin(spai_handle* h, int kc) {
    KernelTimer& t = h->timers[kc];
    if (t.every <= 0 || h->no_alloc) return -1;
    if ((t.seen++ % t.every) != 0) return -1;
    if (2 * t.used + 2 > t.ev.size()) {
        for (int q = 0; q < 2; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return -1;
            t.ev.push_back(e);
        }
    }
    long idx = (long)t.used++;
    (void)hipEventRecord(t.ev[2 * idx], h->stream);
    return idx;
}

inline void timer_end(spai_handle* h, int kc, long idx) {
    if (idx < 0) return;
    (void)hipEventRecord(h->timers[kc].ev[2 * idx + 1], h->stream);
}

}  // namespace spai
