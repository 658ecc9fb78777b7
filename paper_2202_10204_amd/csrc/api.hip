// Handle, error reporting and workspace management of libspai.
#include <cstdlib>
#include <mutex>
#include <string>
#include <unordered_map>

#include "common.hpp"

namespace spai {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string& msg) { g_last_error = msg; }

// The allocator in force (spai_set_allocator; empty: hipMalloc / hipFree) and,
// for every block a caller's allocator returned, the pair that frees it with
// the device and stream it was allocated for.
struct HookAlloc {
    spai_alloc_fn alloc = nullptr;
    spai_free_fn free_ = nullptr;
    void* ctx = nullptr;
};
struct HookBlock {
    HookAlloc by;
    int device;
    hipStream_t stream;
};
static std::mutex g_alloc_mu;
static HookAlloc g_alloc;
static std::unordered_map<void*, HookBlock> g_blocks;

int raw_malloc(void** p, size_t bytes, int device, hipStream_t stream) {
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    HookAlloc by;
    {
        std::lock_guard<std::mutex> l(g_alloc_mu);
        by = g_alloc;
    }
    if (by.alloc) {
        void* q = by.alloc(bytes, device, stream, by.ctx);
        if (!q) {
            set_error("device allocation of " + std::to_string(bytes) + " bytes failed (caller's allocator)");
            return SPAI_E_OOM;
        }
        std::lock_guard<std::mutex> l(g_alloc_mu);
        g_blocks[q] = HookBlock{by, device, stream};
        *p = q;
        return SPAI_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_error(std::string("device allocation of ") + std::to_string(bytes) + " bytes failed: " +
                  hipGetErrorString(e));
        return SPAI_E_OOM;
    }
    return SPAI_OK;
}

void raw_free(void* p) {
    if (!p) return;
    HookBlock b{};
    bool hooked = false;
    {
        std::lock_guard<std::mutex> l(g_alloc_mu);
        auto it = g_blocks.find(p);
        if (it != g_blocks.end()) {
            b = it->second;
            hooked = true;
            g_blocks.erase(it);
        }
    }
    if (hooked) b.by.free_(p, b.device, b.stream, b.by.ctx);
    else (void)hipFree(p);
}

int dev_malloc(spai_handle* h, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    Arena& a = h->arena;
    if (a.base) {
        // a unit of a request server: its memory is the region it was admitted
        // with, never more (admission by footprint is a hard bound)
        const size_t off = (a.used + 255) & ~(size_t)255;
        if (off <= a.size && bytes <= a.size - off) {
            *p = a.base + off;
            a.used = off + bytes;
            return SPAI_OK;
        }
        set_error("device allocation of " + std::to_string(bytes) + " bytes exceeds the " +
                  std::to_string(a.size) + "-byte region the request was admitted with (" +
                  std::to_string(a.used) + " bytes in use)");
        return SPAI_E_OOM;
    }
    return raw_malloc(p, bytes, h->device, h->stream);
}

void dev_free(void* p, const Arena& from) {
    if (!p || from.owns(p)) return;
    raw_free(p);
}

int buffer_reserve(spai_handle* h, Buffer& b, size_t bytes) {
    if (bytes <= b.bytes && b.ptr) return SPAI_OK;
    buffer_free(b);
    size_t want = bytes + bytes / 8 + 256;
    void* p = nullptr;
    int rc = dev_malloc(h, &p, want);
    if (rc) return rc;
    b.ptr = p;
    b.bytes = want;
    b.from = h->arena;
    return SPAI_OK;
}

void buffer_free(Buffer& b) {
    dev_free(b.ptr, b.from);
    b.ptr = nullptr;
    b.bytes = 0;
    b.from = Arena{};
}

}  // namespace spai

static int pinned_reserve(spai::Buffer& b, size_t bytes) {
    if (bytes <= b.bytes && b.ptr) return SPAI_OK;
    if (b.ptr) (void)hipHostFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
    void* p = nullptr;
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        spai::set_error(std::string("pinned host allocation failed: ") + hipGetErrorString(e));
        return SPAI_E_OOM;
    }
    b.ptr = p;
    b.bytes = bytes;
    return SPAI_OK;
}

extern "C" const char* spai_last_error(void) { return spai::g_last_error.c_str(); }

extern "C" int spai_set_allocator(spai_alloc_fn alloc, spai_free_fn free_, void* ctx) {
    if ((alloc == nullptr) != (free_ == nullptr)) {
        spai::set_error("invalid argument: give both allocator functions or neither");
        return SPAI_E_ARG;
    }
    std::lock_guard<std::mutex> l(spai::g_alloc_mu);
    spai::g_alloc = spai::HookAlloc{alloc, free_, alloc ? ctx : nullptr};
    return SPAI_OK;
}

extern "C" int spai_create(spai_handle** h) {
    if (!h) {
        spai::set_error("invalid argument: NULL handle pointer");
        return SPAI_E_ARG;
    }
    *h = nullptr;
    int dev = 0;
    SPAI_HIP(hipGetDevice(&dev));
    spai_handle* H = new spai_handle();
    H->device = dev;
    H->stream = nullptr;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) H->num_cu = prop.multiProcessorCount;
    int rc = pinned_reserve(H->host_pinned, 4096);
    if (rc == SPAI_OK) rc = spai::noalloc_scratch_init(dev);
    for (int q = 0; q < 2 && rc == SPAI_OK; ++q)
        if (hipEventCreateWithFlags(&H->chunk_ev[q], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            spai::set_error("hipEventCreateWithFlags failed");
            rc = SPAI_E_HIP;
        }
    if (rc) {
        for (hipEvent_t e : H->chunk_ev)
            if (e) (void)hipEventDestroy(e);
        if (H->host_pinned.ptr) (void)hipHostFree(H->host_pinned.ptr);
        delete H;
        return rc;
    }
    *h = H;
    return SPAI_OK;
}

extern "C" int spai_destroy(spai_handle* h) {
    if (!h) return SPAI_OK;
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    for (auto& t : h->timers)
        for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->chunk_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& b : h->ws) spai::buffer_free(b);
    spai::buffer_free(h->red);
    if (h->host_pinned.ptr) (void)hipHostFree(h->host_pinned.ptr);
    delete h;
    return SPAI_OK;
}

extern "C" int spai_set_stream(spai_handle* h, hipStream_t stream) {
    if (!h) {
        spai::set_error("invalid argument: NULL handle");
        return SPAI_E_ARG;
    }
    h->stream = stream;
    return SPAI_OK;
}

extern "C" int spai_timing_enable(spai_handle* h, int kc, int every) {
    if (!h || kc < 0 || kc >= SPAI_KT_COUNT) {
        spai::set_error("invalid argument: handle or kernel class");
        return SPAI_E_ARG;
    }
    auto& t = h->timers[kc];
    t.every = every > 0 ? every : 0;
    t.seen = 0;
    t.used = 0;
    return SPAI_OK;
}

extern "C" int spai_timing_read(spai_handle* h, int kc, int64_t* launches, double* total_ms) {
    if (!h || kc < 0 || kc >= SPAI_KT_COUNT || !launches || !total_ms) {
        spai::set_error("invalid argument: handle, kernel class or outputs");
        return SPAI_E_ARG;
    }
    auto& t = h->timers[kc];
    SPAI_HIP(hipStreamSynchronize(h->stream));
    double tot = 0.0;
    for (size_t q = 0; q < t.used; ++q) {
        float ms = 0.0f;
        SPAI_HIP(hipEventElapsedTime(&ms, t.ev[2 * q], t.ev[2 * q + 1]));
        tot += ms;
    }
    *launches = (int64_t)t.used;
    *total_ms = tot;
    t.used = 0;
    t.seen = 0;
    return SPAI_OK;
}
