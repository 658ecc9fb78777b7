// Request server of libspai: independent SPAI-GMRES-IR solves admitted as they
// arrive, by device footprint, and run concurrently on batch lanes (many small
// systems per launch) and one device lane (one large system on the whole chip).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace spai {
namespace {

using Clock = std::chrono::steady_clock;

constexpr int MAX_LANES = 16;
constexpr int64_t MIB = 1 << 20;

struct Request {
    int64_t id = 0;
    int32_t n = 0, nnz = 0, jnnz = 0;
    std::vector<int32_t> rowptr, col, jptr, jidx;
    std::vector<double> val, b;
    spai_build_params bp{};
    spai_ir_params ip{};
    bool small = false;
    std::vector<double> x;
    spai_serve_result res{};
    std::string err;
    bool done = false;
    bool claimed = false;   // a caller is waiting for it
};

// Requests that can share one batch: the same build and solve parameters and
// the same kind of initial pattern.
bool same_key(const Request& a, const Request& b) {
    return a.bp.eps == b.bp.eps && a.bp.alpha == b.bp.alpha && a.bp.beta == b.bp.beta && a.bp.side == b.bp.side &&
           a.bp.qr_update == b.bp.qr_update && a.bp.kernel_cfg == b.bp.kernel_cfg &&
           a.bp.maxfill == b.bp.maxfill && a.bp.u_f == b.bp.u_f && a.ip.u_r == b.ip.u_r && a.ip.tau == b.ip.tau &&
           a.ip.imax == b.ip.imax && a.ip.maxit == b.ip.maxit && a.ip.tol_ir == b.ip.tol_ir && a.ip.u == b.ip.u &&
           a.jptr.empty() == b.jptr.empty();
}

// Shared / exclusive use of the device: batches and builds hold it shared, the
// device lane's solve (whose launches need every workgroup resident) holds it
// exclusively.  A waiting exclusive user blocks new shared users.
struct Gate {
    std::mutex m;
    std::condition_variable cv;
    int readers = 0, writers_waiting = 0;
    bool writer = false;
    void lock_shared() {
        std::unique_lock<std::mutex> l(m);
        cv.wait(l, [&] { return !writer && writers_waiting == 0; });
        ++readers;
    }
    void unlock_shared() {
        std::lock_guard<std::mutex> l(m);
        if (--readers == 0) cv.notify_all();
    }
    void lock() {
        std::unique_lock<std::mutex> l(m);
        ++writers_waiting;
        cv.wait(l, [&] { return !writer && readers == 0; });
        --writers_waiting;
        writer = true;
    }
    void unlock() {
        std::lock_guard<std::mutex> l(m);
        writer = false;
        cv.notify_all();
    }
};

size_t val_bytes(spai_prec p) { return p == SPAI_FP64 ? 8 : p == SPAI_FP32 ? 4 : 2; }

// Structure of a host CSR-like array pair: ptr runs from 0 to nnz without
// decreasing and every index lies in [0, n).  Checked on the host before
// anything is copied, so a malformed request never reaches a kernel that other
// requests share.
int check_structure(int32_t n, int32_t nnz, const int32_t* ptr, const int32_t* idx, const char* what) {
    if (ptr[0] != 0 || ptr[n] != nnz) {
        set_error(std::string("invalid argument: ") + what + " pointers must run from 0 to the entry count");
        return SPAI_E_ARG;
    }
    for (int32_t i = 0; i < n; ++i) {
        if (ptr[i + 1] < ptr[i]) {
            set_error(std::string("invalid argument: ") + what + " pointers decrease at row " + std::to_string(i));
            return SPAI_E_ARG;
        }
    }
    for (int32_t q = 0; q < nnz; ++q) {
        if (idx[q] < 0 || idx[q] >= n) {
            set_error(std::string("invalid argument: ") + what + " index " + std::to_string(idx[q]) +
                      " at entry " + std::to_string(q) + " outside [0, n)");
            return SPAI_E_ARG;
        }
    }
    return SPAI_OK;
}

int check_request(const spai_serve_request* r) {
    SPAI_ARG(r, "NULL request");
    SPAI_ARG(r->n > 0 && r->nnz >= 0, "n <= 0 or nnz < 0");
    SPAI_ARG(r->rowptr && r->b && (r->nnz == 0 || (r->col && r->val)), "NULL array in the request");
    int rc = check_structure(r->n, r->nnz, r->rowptr, r->col, "matrix row");
    if (rc) return rc;
    if (r->jptr) {
        SPAI_ARG(r->jnnz >= 0 && (r->jnnz == 0 || r->jidx), "pattern without indices");
        if ((rc = check_structure(r->n, r->jnnz, r->jptr, r->jidx, "pattern column"))) return rc;
    }
    const spai_build_params& p = r->build;
    SPAI_ARG(p.eps > 0 && p.alpha >= 0 && p.beta >= 0 && p.maxfill >= 1 && p.maxfill <= 63,
             "bad build parameters");
    SPAI_ARG(p.u_f == SPAI_FP64 || p.u_f == SPAI_FP32 || p.u_f == SPAI_FP16 || p.u_f == SPAI_BF16, "bad u_f");
    SPAI_ARG(p.side == SPAI_LEFT || p.side == SPAI_RIGHT, "bad side");
    SPAI_ARG(p.qr_update == 0 || p.qr_update == 1, "bad qr_update");
    SPAI_ARG(p.kernel_cfg >= 0 && p.kernel_cfg <= SPAI_KCFG_COUNT, "bad kernel_cfg");
    const spai_ir_params& q = r->ir;
    SPAI_ARG(q.imax >= 1 && q.imax <= 32 && q.maxit >= 1 && q.tau >= 0, "bad solve parameters");
    SPAI_ARG(q.u_r == SPAI_DD || q.u_r == SPAI_FP64, "bad u_r");
    SPAI_ARG(q.u == SPAI_FP64 || (q.u == SPAI_FP32 && q.u_r == SPAI_FP64 && p.u_f != SPAI_FP64),
             "bad working precision");
    return SPAI_OK;
}

// Upper estimate of everything the request holds on the device: A, b, x and the
// pattern; P with the build's per-column arrays (stride = the longest column
// J_k can reach); the build's workspace; the single-system solve's basis and
// vectors (a batched system uses its lane's workspace instead, but the
// estimate does not depend on where it runs).
int64_t footprint_of(const spai_serve_request* r) {
    const int64_t n = r->n, nnz = r->nnz;
    int64_t stride = r->build.maxfill;
    if (r->jptr)
        for (int32_t k = 0; k < r->n; ++k) stride = std::max<int64_t>(stride, r->jptr[k + 1] - r->jptr[k]);
    const int64_t maxit = std::min<int64_t>(r->ir.maxit, n);
    int64_t b = 12 * nnz + 4 * (n + 1) + 16 * n;                              // A, b, x
    if (r->jptr) b += 4 * (n + 1) + 4 * (int64_t)r->jnnz;                    // pattern
    b += 4 * (n + 1) + 8 * n + (int64_t)(4 + val_bytes(r->build.u_f)) * n * stride;  // P
    b += 12 * n * stride + 28 * n;                                           // insertion order, stats
    b += 48 * n + 4 * nnz;                                                   // build workspace
    b += 8 * n * (maxit + 4) + 8 * (maxit + 2) * (maxit + 2) * 4;            // basis, vectors, H
    return b + b / 8 + 4 * MIB;
}

double seconds_since(Clock::time_point t0) {
    return std::chrono::duration<double>(Clock::now() - t0).count();
}

// First-fit allocator of contiguous regions of the server's device arena
// (offsets and sizes in bytes, 256-byte granules); freed regions merge with
// their free neighbours.
struct Regions {
    std::map<int64_t, int64_t> free_;   // offset -> size
    void init(int64_t size) { free_ = {{0, size}}; }
    static int64_t granule(int64_t b) { return (b + 255) & ~(int64_t)255; }
    int64_t largest() const {
        int64_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
    int64_t take(int64_t size) {   // -1 when no free region is large enough
        size = granule(size);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < size) continue;
            const int64_t off = it->first, rest = it->second - size;
            free_.erase(it);
            if (rest > 0) free_.emplace(off + size, rest);
            return off;
        }
        return -1;
    }
    void give(int64_t off, int64_t size) {
        size = granule(size);
        auto it = free_.emplace(off, size).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

// Admitted work for one lane: its requests and the arena region they hold.
struct Unit {
    std::vector<Request*> rs;
    int64_t off = -1, size = 0;
};

}  // namespace
}  // namespace spai

using spai::Request;

struct spai_server {
    spai_serve_params prm{};
    int device = 0;
    char* arena = nullptr;       // hbm_budget bytes of device memory, lent to lanes region by region
    spai::Regions regions;       // free parts of the arena
    spai::Clock::time_point t0;
    std::mutex m;
    std::condition_variable cv;  // new work, freed regions, finished requests
    std::deque<Request*> small, large;   // waiting, in arrival order
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs;
    int64_t next_id = 1;
    bool stop = false;
    spai::Gate gate;
    std::vector<std::thread> threads;
};

namespace spai {
namespace {

// Per-lane device state: a non-blocking stream, a handle that allocates from
// the arena region of its current unit of work, and grow-only pinned host
// staging.
struct LaneCtx {
    spai_server* S = nullptr;
    int lane = -1;
    hipStream_t stream = nullptr;
    hipStream_t solve_stream = nullptr;   // device lane with reserved CUs: the solve's stream
    int all_cus = 0, solve_cus = 0;
    spai_handle* h = nullptr;
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
};

// CU masks on gfx950: bit i of a stream's mask enables a CU of XCD i mod 8 (the
// driver deals consecutive bits to the XCDs in turn, and within an XCD to its
// shader engines in turn), so bits [0, 8K) enable K CUs in every XCD and a grid
// dealt round-robin to the XCDs finds K CUs in each.
constexpr int XCDS = 8;

int masked_stream(hipStream_t* s, int num_cu, int lo, int hi) {
    std::vector<uint32_t> mask((num_cu + 31) / 32, 0u);
    for (int b = lo; b < hi; ++b) mask[b / 32] |= 1u << (b % 32);
    SPAI_HIP(hipExtStreamCreateWithCUMask(s, (uint32_t)mask.size(), mask.data()));
    return SPAI_OK;
}

int lane_init(LaneCtx& L, size_t ws_cap) {
    SPAI_HIP(hipSetDevice(L.S->device));
    int rc = spai_create(&L.h);
    if (rc) return rc;
    const int num_cu = L.h->num_cu, rsv = XCDS * L.S->prm.device_lane_cus;
    L.all_cus = num_cu;
    if (rsv > 0 && L.lane >= 0) {
        // batch lane: the CUs outside the device lane's reservation
        if ((rc = masked_stream(&L.stream, num_cu, rsv, num_cu))) return rc;
        L.h->num_cu = num_cu - rsv;
    } else {
        SPAI_HIP(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
    }
    if (rsv > 0 && L.lane < 0) {
        if ((rc = masked_stream(&L.solve_stream, num_cu, 0, rsv))) return rc;
        L.solve_cus = rsv;
    }
    L.h->stream = L.stream;
    L.h->ws_cap = ws_cap;
    return SPAI_OK;
}

void lane_fini(LaneCtx& L) {
    if (L.h) (void)spai_destroy(L.h);
    if (L.pinned) (void)hipHostFree(L.pinned);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    if (L.solve_stream) (void)hipStreamDestroy(L.solve_stream);
}

int pinned(LaneCtx& L, size_t bytes, char** out) {
    if (bytes > L.pinned_bytes) {
        if (L.pinned) (void)hipHostFree(L.pinned);
        L.pinned = nullptr;
        L.pinned_bytes = 0;
        const size_t want = bytes + bytes / 4 + 4096;
        SPAI_HIP(hipHostMalloc(&L.pinned, want, hipHostMallocDefault));
        L.pinned_bytes = want;
    }
    *out = (char*)L.pinned;
    return SPAI_OK;
}

// Forget the handle's workspaces (they live in the unit's region) so that the
// next unit allocates in its own region.
void lane_trim(LaneCtx& L) {
    for (auto& b : L.h->ws) buffer_free(b);
}

// Device arrays of one unit of work, taken from the unit's region.
struct DevArrays {
    LaneCtx* L;
    std::vector<void*> ptrs;
    explicit DevArrays(LaneCtx* l) : L(l) {}
    template <typename T>
    int alloc(T** p, size_t count) {
        int rc = dev_malloc(L->h, (void**)p, sizeof(T) * (count ? count : 1));
        if (rc) return rc;
        ptrs.push_back(*p);
        return SPAI_OK;
    }
    ~DevArrays() {
        for (void* q : ptrs) dev_free(q, L->h->arena);
    }
};

// Concatenation of the requests of one unit of work (one request on the device
// lane) as a block-diagonal system, staged through pinned memory.
struct Staged {
    int32_t n = 0, nnz = 0, jnnz = 0;
    std::vector<int32_t> sys_ptr;
    int32_t *rowptr = nullptr, *col = nullptr, *jptr = nullptr, *jidx = nullptr;
    double *val = nullptr, *b = nullptr, *x = nullptr;
};

int stage(LaneCtx& L, const std::vector<Request*>& rs, DevArrays& D, Staged& g) {
    int64_t n = 0, nnz = 0, jnnz = 0;
    for (Request* r : rs) {
        n += r->n;
        nnz += r->nnz;
        jnnz += r->jnnz;
    }
    SPAI_ARG(n < (1ll << 31) && nnz < (1ll << 31) && jnnz < (1ll << 31), "batch exceeds int32 indices");
    const bool pat = !rs[0]->jptr.empty();
    g.n = (int32_t)n;
    g.nnz = (int32_t)nnz;
    g.jnnz = (int32_t)jnnz;
    const size_t bytes = 4 * (size_t)(n + 1) * (pat ? 2 : 1) + 4 * (size_t)nnz + 8 * (size_t)nnz + 8 * (size_t)n +
                         4 * (size_t)jnnz + 64;
    char* hp = nullptr;
    int rc = pinned(L, bytes, &hp);
    if (rc) return rc;
    int32_t* h_rp = (int32_t*)hp;
    int32_t* h_jp = h_rp + (n + 1);
    int32_t* h_ci = pat ? h_jp + (n + 1) : h_jp;
    int32_t* h_ji = h_ci + nnz;
    double* h_v = (double*)(((uintptr_t)(h_ji + jnnz) + 7) & ~(uintptr_t)7);
    double* h_b = h_v + nnz;
    g.sys_ptr.assign(1, 0);
    int64_t r0 = 0, q0 = 0, p0 = 0;
    for (Request* r : rs) {
        for (int32_t i = 0; i < r->n; ++i) h_rp[r0 + i] = (int32_t)(q0 + r->rowptr[i]);
        for (int32_t q = 0; q < r->nnz; ++q) h_ci[q0 + q] = (int32_t)(r0 + r->col[q]);
        std::memcpy(h_v + q0, r->val.data(), 8 * (size_t)r->nnz);
        std::memcpy(h_b + r0, r->b.data(), 8 * (size_t)r->n);
        if (pat) {
            for (int32_t i = 0; i < r->n; ++i) h_jp[r0 + i] = (int32_t)(p0 + r->jptr[i]);
            for (int32_t q = 0; q < r->jnnz; ++q) h_ji[p0 + q] = (int32_t)(r0 + r->jidx[q]);
        }
        r0 += r->n;
        q0 += r->nnz;
        p0 += r->jnnz;
        g.sys_ptr.push_back((int32_t)r0);
    }
    h_rp[n] = (int32_t)nnz;
    if (pat) h_jp[n] = (int32_t)jnnz;
    if ((rc = D.alloc(&g.rowptr, n + 1)) || (rc = D.alloc(&g.col, nnz)) || (rc = D.alloc(&g.val, nnz)) ||
        (rc = D.alloc(&g.b, n)) || (rc = D.alloc(&g.x, n)))
        return rc;
    const hipStream_t s = L.stream;
    SPAI_HIP(hipMemcpyAsync(g.rowptr, h_rp, 4 * (size_t)(n + 1), hipMemcpyHostToDevice, s));
    SPAI_HIP(hipMemcpyAsync(g.col, h_ci, 4 * (size_t)nnz, hipMemcpyHostToDevice, s));
    SPAI_HIP(hipMemcpyAsync(g.val, h_v, 8 * (size_t)nnz, hipMemcpyHostToDevice, s));
    SPAI_HIP(hipMemcpyAsync(g.b, h_b, 8 * (size_t)n, hipMemcpyHostToDevice, s));
    if (pat) {
        if ((rc = D.alloc(&g.jptr, n + 1)) || (rc = D.alloc(&g.jidx, jnnz))) return rc;
        SPAI_HIP(hipMemcpyAsync(g.jptr, h_jp, 4 * (size_t)(n + 1), hipMemcpyHostToDevice, s));
        SPAI_HIP(hipMemcpyAsync(g.jidx, h_ji, 4 * (size_t)jnnz, hipMemcpyHostToDevice, s));
    }
    // the staging buffer is reused by the next unit: wait for the copies
    SPAI_HIP(hipStreamSynchronize(s));
    return SPAI_OK;
}

// Copy x and the row pointer of P back and split them per request.
int unstage(LaneCtx& L, const std::vector<Request*>& rs, const Staged& g, const spai_precond* P) {
    char* hp = nullptr;
    int rc = pinned(L, 8 * (size_t)g.n + 4 * ((size_t)g.n + 1) + 64, &hp);
    if (rc) return rc;
    double* h_x = (double*)hp;
    int32_t* h_pp = (int32_t*)(h_x + g.n);
    SPAI_HIP(hipMemcpyAsync(h_x, g.x, 8 * (size_t)g.n, hipMemcpyDeviceToHost, L.stream));
    SPAI_HIP(hipMemcpyAsync(h_pp, P->rowptr, 4 * ((size_t)g.n + 1), hipMemcpyDeviceToHost, L.stream));
    SPAI_HIP(hipStreamSynchronize(L.stream));
    for (size_t q = 0; q < rs.size(); ++q) {
        const int32_t a = g.sys_ptr[q], e = g.sys_ptr[q + 1];
        rs[q]->x.assign(h_x + a, h_x + e);
        rs[q]->res.nnz_p = (int64_t)h_pp[e] - h_pp[a];
    }
    return SPAI_OK;
}

void finish(spai_server* S, const Unit& u, int rc_fail, const std::string& msg) {
    const double t = seconds_since(S->t0);
    {
        std::lock_guard<std::mutex> l(S->m);
        S->regions.give(u.off, u.size);
        for (Request* r : u.rs) {
            if (rc_fail < 0) {
                r->res.rc = rc_fail;
                r->err = msg;
                r->x.clear();
            }
            r->res.t_done = t;
            r->done = true;
            r->rowptr = {};   // inputs are not needed any more
            r->col = {};
            r->val = {};
            r->b = {};
            r->jptr = {};
            r->jidx = {};
        }
    }
    S->cv.notify_all();
}

// One batch on a batch lane.
int run_batch(LaneCtx& L, const std::vector<Request*>& rs) {
    spai_server* S = L.S;
    DevArrays D(&L);
    Staged g;
    int rc = stage(L, rs, D, g);
    if (rc < 0) return rc;
    spai_csr A{g.n, g.nnz, g.rowptr, g.col, g.val};
    spai_pattern J{g.n, g.jnnz, g.jptr, g.jidx};
    const int nsys = (int)rs.size();
    spai_precond* P = nullptr;
    std::vector<spai_ir_stats> st(nsys);
    spai_ir_params ip = rs[0]->ip;
    ip.ortho = SPAI_ORTHO_MGS;
    S->gate.lock_shared();
    int rb = spai_build_batched(L.h, &A, nsys, g.sys_ptr.data(), g.jptr ? &J : nullptr, &rs[0]->bp, &P, nullptr);
    const double ts = seconds_since(S->t0);
    int rs_ = rb < 0 ? rb : spai_gmres_ir_batched(L.h, &A, P, nsys, g.sys_ptr.data(), g.b, g.x, &ip, st.data());
    S->gate.unlock_shared();
    if (rb < 0 || rs_ < 0) {
        if (P) spai_precond_destroy(P);
        return rb < 0 ? rb : rs_;
    }
    // per-system build warnings from the per-column flags
    std::vector<int32_t> flags(g.n);
    rc = SPAI_OK;
    if (hipMemcpyAsync(flags.data(), P->flags, 4 * (size_t)g.n, hipMemcpyDeviceToHost, L.stream) != hipSuccess)
        rc = SPAI_E_HIP;
    if (!rc) rc = unstage(L, rs, g, P);
    spai_precond_destroy(P);
    if (rc) return rc;
    for (int q = 0; q < nsys; ++q) {
        int w = 0;
        for (int32_t k = g.sys_ptr[q]; k < g.sys_ptr[q + 1]; ++k) w |= flags[k];
        int warn = ((w & CF_EPS) ? SPAI_W_EPS : 0) | ((w & CF_RANKDEF) ? SPAI_W_RANKDEF : 0) |
                   ((w & CF_NONFINITE) ? SPAI_W_NONFINITE : 0);
        rs[q]->res.ir = st[q];
        rs[q]->res.rc = warn | st[q].status;
        rs[q]->res.batch_size = nsys;
        rs[q]->res.t_solve = ts;
        rs[q]->res.cus = L.h->num_cu;
    }
    return SPAI_OK;
}

// One large system on the device lane.
int run_single(LaneCtx& L, Request* r) {
    spai_server* S = L.S;
    DevArrays D(&L);
    Staged g;
    std::vector<Request*> rs{r};
    int rc = stage(L, rs, D, g);
    if (rc < 0) return rc;
    spai_csr A{g.n, g.nnz, g.rowptr, g.col, g.val};
    spai_pattern J{g.n, g.jnnz, g.jptr, g.jidx};
    spai_precond* P = nullptr;
    spai_build_stats bst{};
    S->gate.lock_shared();
    int rb = spai_build(L.h, &A, g.jptr ? &J : nullptr, &r->bp, &P, &bst);
    S->gate.unlock_shared();
    if (rb < 0) return rb;
    lane_trim(L);   // the build's workspace is not needed by the solve
    spai_ir_stats st{};
    int rs_;
    // on the reserved CUs when the fused Arnoldi launch fits them (batches go on
    // beside it), else on the whole device with no batch running
    L.h->num_cu = L.solve_cus;
    const bool masked = L.solve_cus > 0 && arnoldi_fused_fits(L.h, g.n, r->ip.maxit, r->ip.ortho);
    L.h->num_cu = L.all_cus;
    if (masked) {
        L.h->num_cu = L.solve_cus;
        L.h->stream = L.solve_stream;
        r->res.t_solve = seconds_since(S->t0);
        rs_ = spai_gmres_ir(L.h, &A, P, g.b, g.x, &r->ip, &st);
        L.h->stream = L.stream;
        L.h->num_cu = L.all_cus;
    } else {
        S->gate.lock();
        r->res.t_solve = seconds_since(S->t0);
        rs_ = spai_gmres_ir(L.h, &A, P, g.b, g.x, &r->ip, &st);
        S->gate.unlock();
    }
    r->res.cus = masked ? L.solve_cus : L.all_cus;
    if (rs_ < 0) {
        spai_precond_destroy(P);
        return rs_;
    }
    rc = unstage(L, rs, g, P);
    spai_precond_destroy(P);
    if (rc) return rc;
    r->res.ir = st;
    r->res.rc = rb | rs_;
    r->res.batch_size = 1;
    return SPAI_OK;
}

// Admission (under the server lock).  A batch starts with the oldest waiting
// small request and takes every later one with the same parameters, in arrival
// order, while the batch caps allow and the batch (its requests' footprints
// plus one lane workspace) fits the largest free region of the arena; the
// device lane takes the oldest large request when its footprint fits.  A
// request that does not fit waits: later ones of its kind are not admitted
// ahead of it.  The unit's region is taken at admission and returned when the
// unit has finished.
constexpr int64_t UNIT_SLACK = 16 * MIB;   // small buffers and alignment of one unit

bool take_batch(spai_server* S, int lane, Unit& u) {
    if (S->small.empty()) return false;
    Request* head = S->small.front();
    const int64_t room = S->regions.largest();
    int64_t need = S->prm.lane_workspace + UNIT_SLACK;
    if (need + head->res.footprint > room) return false;
    const double t = seconds_since(S->t0);
    int64_t rows = 0;
    for (auto it = S->small.begin(); it != S->small.end();) {
        Request* r = *it;
        if (!same_key(*head, *r)) {
            ++it;
            continue;
        }
        if ((int)u.rs.size() >= S->prm.batch_max_systems || rows + r->n >= (1ll << 31) - 1 ||
            need + r->res.footprint > room)
            break;
        need += r->res.footprint;
        rows += r->n;
        r->res.t_admit = t;
        r->res.lane = lane;
        u.rs.push_back(r);
        it = S->small.erase(it);
    }
    u.size = need;
    u.off = S->regions.take(need);
    return true;
}

// The device lane serves the oldest large request, or, with a positive
// age limit, the smallest waiting one (shortest job first: one large system
// holds the whole device for its solve) unless the oldest has waited longer
// than the limit.
bool take_large(spai_server* S, Unit& u) {
    if (S->large.empty()) return false;
    const double now = seconds_since(S->t0);
    auto pick = S->large.begin();
    if (S->prm.sjf_age_ms > 0 && now - (*pick)->res.t_submit <= 1e-3 * S->prm.sjf_age_ms)
        for (auto it = S->large.begin(); it != S->large.end(); ++it)
            if ((*it)->n < (*pick)->n) pick = it;
    Request* r = *pick;
    const int64_t need = r->res.footprint + UNIT_SLACK;
    if (need > S->regions.largest()) return false;
    r->res.t_admit = now;
    r->res.lane = -1;
    u.rs.push_back(r);
    u.size = need;
    u.off = S->regions.take(need);
    S->large.erase(pick);
    return true;
}

void lane_main(spai_server* S, int lane) {
    LaneCtx L;
    L.S = S;
    L.lane = lane;
    const bool batch = lane >= 0;
    int rc0 = lane_init(L, batch ? (size_t)S->prm.lane_workspace : 0);
    for (;;) {
        Unit u;
        {
            std::unique_lock<std::mutex> l(S->m);
            S->cv.wait(l, [&] {
                if (batch ? take_batch(S, lane, u) : take_large(S, u)) return true;
                return S->stop && (batch ? S->small.empty() : S->large.empty());
            });
        }
        if (u.rs.empty()) break;
        int rc = rc0;
        if (!rc) {
            L.h->arena = Arena{S->arena + u.off, (size_t)u.size, 0};
            rc = batch ? run_batch(L, u.rs) : run_single(L, u.rs[0]);
            lane_trim(L);
            L.h->arena = Arena{};
        }
        finish(S, u, rc < 0 ? rc : 0, rc < 0 ? std::string(spai_last_error()) : std::string());
    }
    lane_fini(L);
}

}  // namespace
}  // namespace spai

extern "C" int spai_serve_footprint(const spai_serve_request* r, int64_t* bytes) {
    if (!bytes) {
        spai::set_error("invalid argument: NULL output");
        return SPAI_E_ARG;
    }
    int rc = spai::check_request(r);
    if (rc) return rc;
    *bytes = spai::footprint_of(r);
    return SPAI_OK;
}

extern "C" int spai_serve_create(const spai_serve_params* p, spai_server** out) {
    if (!p || !out) {
        spai::set_error("invalid argument: NULL parameters or output");
        return SPAI_E_ARG;
    }
    *out = nullptr;
    SPAI_ARG(p->batch_lanes >= 1 && p->batch_lanes <= spai::MAX_LANES, "batch_lanes outside 1..16");
    SPAI_ARG(p->batch_max_n >= 1 && p->batch_max_systems >= 1, "batch_max_n and batch_max_systems must be >= 1");
    SPAI_ARG(p->hbm_budget > 0 && p->lane_workspace >= 0, "bad budget");
    SPAI_ARG(p->sjf_age_ms >= 0, "sjf_age_ms must be non-negative");
    SPAI_ARG(p->device_lane_cus >= 0, "device_lane_cus must be non-negative");
    if (p->device_lane_cus > 0) {
        int dev0 = 0;
        hipDeviceProp_t prop;
        SPAI_HIP(hipGetDevice(&dev0));
        SPAI_HIP(hipGetDeviceProperties(&prop, dev0));
        SPAI_ARG(prop.multiProcessorCount % spai::XCDS == 0 &&
                     p->device_lane_cus < prop.multiProcessorCount / spai::XCDS,
                 "device_lane_cus must leave every XCD a CU for the batch lanes");
    }
    spai_serve_params prm = *p;
    if (prm.lane_workspace == 0)
        prm.lane_workspace = std::min<int64_t>(8ll << 30, prm.hbm_budget / 4 / prm.batch_lanes);
    SPAI_ARG(prm.lane_workspace + spai::UNIT_SLACK + 64 * spai::MIB <= prm.hbm_budget,
             "hbm_budget does not hold a lane workspace");
    int dev = 0;
    SPAI_HIP(hipGetDevice(&dev));
    void* arena = nullptr;
    if (spai::raw_malloc(&arena, (size_t)prm.hbm_budget, dev, nullptr) != SPAI_OK) {
        spai::set_error(std::string("device allocation of the server's ") + std::to_string(prm.hbm_budget) +
                        " bytes failed");
        return SPAI_E_OOM;
    }
    spai_server* S = new spai_server();
    S->prm = prm;
    S->device = dev;
    S->arena = (char*)arena;
    S->regions.init(prm.hbm_budget);
    S->t0 = spai::Clock::now();
    for (int l = 0; l < prm.batch_lanes; ++l) S->threads.emplace_back(spai::lane_main, S, l);
    S->threads.emplace_back(spai::lane_main, S, -1);
    *out = S;
    return SPAI_OK;
}

extern "C" int spai_serve_submit(spai_server* S, const spai_serve_request* r, int64_t* id) {
    SPAI_ARG(S && id, "NULL server or id");
    int rc = spai::check_request(r);
    if (rc) return rc;
    const int64_t fp = spai::footprint_of(r);
    // right preconditioners run on the device lane (the batched solver applies left ones)
    const bool small = r->n <= S->prm.batch_max_n && r->build.side == SPAI_LEFT;
    const int64_t need = fp + spai::UNIT_SLACK + (small ? S->prm.lane_workspace : 0);
    if (need > S->prm.hbm_budget) {
        spai::set_error("request needs " + std::to_string(need) + " bytes of device memory (footprint " +
                        std::to_string(fp) + (small ? " plus a lane workspace" : "") + "), more than the budget of " +
                        std::to_string(S->prm.hbm_budget) + " bytes");
        return SPAI_E_OOM;
    }
    auto q = std::make_unique<Request>();
    q->n = r->n;
    q->nnz = r->nnz;
    q->rowptr.assign(r->rowptr, r->rowptr + r->n + 1);
    q->col.assign(r->col, r->col + r->nnz);
    q->val.assign(r->val, r->val + r->nnz);
    q->b.assign(r->b, r->b + r->n);
    if (r->jptr) {
        q->jnnz = r->jnnz;
        q->jptr.assign(r->jptr, r->jptr + r->n + 1);
        q->jidx.assign(r->jidx, r->jidx + r->jnnz);
    }
    q->bp = r->build;
    q->ip = r->ir;
    q->ip.x_given = 0;        // a request starts from x0 = P b
    q->ip.x_true = nullptr;   // requests are host data; no device pointer is kept
    q->small = small;
    q->res.footprint = fp;
    {
        std::lock_guard<std::mutex> l(S->m);
        SPAI_ARG(!S->stop, "server is shutting down");
        q->id = S->next_id++;
        q->res.t_submit = spai::seconds_since(S->t0);
        Request* raw = q.get();
        *id = q->id;
        S->reqs.emplace(q->id, std::move(q));
        (raw->small ? S->small : S->large).push_back(raw);
    }
    S->cv.notify_all();
    return SPAI_OK;
}

extern "C" int spai_serve_wait(spai_server* S, int64_t id, double* x, spai_serve_result* res) {
    SPAI_ARG(S, "NULL server");
    std::unique_ptr<Request> q;
    {
        std::unique_lock<std::mutex> l(S->m);
        auto it = S->reqs.find(id);
        SPAI_ARG(it != S->reqs.end(), "unknown request id");
        Request* r = it->second.get();
        SPAI_ARG(!r->claimed, "another caller is already waiting for this request");
        r->claimed = true;
        S->cv.wait(l, [&] { return r->done; });
        // the wait dropped the lock: submissions may have rehashed the map, so
        // the entry is looked up again (the request object itself has not moved)
        auto again = S->reqs.find(id);
        q = std::move(again->second);
        S->reqs.erase(again);
    }
    if (x && !q->x.empty()) std::memcpy(x, q->x.data(), 8 * q->x.size());
    if (res) *res = q->res;
    if (q->res.rc < 0) spai::set_error(q->err);
    return q->res.rc;
}

extern "C" int spai_serve_destroy(spai_server* S) {
    if (!S) return SPAI_OK;
    {
        std::lock_guard<std::mutex> l(S->m);
        S->stop = true;
    }
    S->cv.notify_all();
    for (auto& t : S->threads) t.join();
    (void)hipDeviceSynchronize();
    spai::raw_free(S->arena);
    delete S;
    return SPAI_OK;
}
