// SPAI construction on gfx950: Algorithm 1 (Section 2.2) on B = A^T D with the
// one-sided column scaling of Section 4, producing the left preconditioner
// P = M^T D of Algorithm 3.
//
// Work decomposition.  The Frobenius norm decouples into n independent column
// problems (eq. fronormmin).  A group of G lanes of one wavefront owns one
// column k; a 64-wide wavefront holds floor(64/G) groups and a workgroup is one
// wavefront, so groups never need a workgroup barrier.  The reduced matrix
// A-bar = B(I_k, J_k) and e-bar live in LDS (column-major, odd leading
// dimension): lane c of the group owns column c of A-bar and lane p owns e-bar,
// so the Householder updates of the trailing columns run in parallel while
// every inner sum runs sequentially over the rows in ascending order.  That is
// the rounding model of the build, stated with the arithmetic helpers in
// common.hpp: one precision F, sequential sums in a fixed index order, fused
// multiply-adds for sums of products, and rounding to u_f at the storage points.
// Index work (shadows, candidate sets) uses per-group bitonic sorts in LDS.
//
// Problems that exceed a kernel's LDS capacity (rows of the shadow, gathered
// entries, raw candidates) are deferred to a launch of a larger configuration
// over the deferred list (and what that one defers to the largest).
#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "common.hpp"

namespace spai {

// ---------------------------------------------------------------------------
// preprocessing kernels
// ---------------------------------------------------------------------------

struct PrepOut {
    int err;        // bit 0: bad rowptr, 1: column out of range / unsorted, 2: non-finite value,
                    // 3: all-zero row, 4: bad pattern
    int max_row;    // max nnz per row of A
    int max_col;    // max nnz per column of A
    int max_pat;    // longest initial pattern column
};

// Reductions of one value per lane over the 64 lanes of a wave (every lane takes
// part).  Atomics on one address serialise at the memory side (one per wave
// already, the compiler combining a wave's lanes), so the counters and maxima of
// the build are reduced over a whole block of a grid-stride launch first.
constexpr int RED_BLOCK = 256;   // threads of the grid-stride reduction kernels

__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

__global__ __launch_bounds__(RED_BLOCK) void k_validate_scale(int n, int nnz, const int* __restrict__ rp,
                                                               const int* __restrict__ ci,
                                 const double* __restrict__ av, double* __restrict__ d,
                                 int* __restrict__ colcount, PrepOut* out) {
    __shared__ int sh[RED_BLOCK / 64];
    int len = 0;
    for (int j = blockIdx.x * RED_BLOCK + threadIdx.x; j < n; j += gridDim.x * RED_BLOCK) {
        int s = rp[j], e = rp[j + 1];
        int err = 0;
        if (j == 0 && s != 0) err |= 1;
        if (j == n - 1 && e != nnz) err |= 1;
        if (e < s || s < 0 || e > nnz) {
            atomicOr(&out->err, err | 1);
            d[j] = 1.0;
        } else {
            double mx = 0.0;
            int prev = -1;
            for (int q = s; q < e; ++q) {
                int c = ci[q];
                double v = av[q];
                if (c < 0 || c >= n || c <= prev) err |= 2;
                prev = c;
                if (!isfinite(v)) err |= 4;
                double a = fabs(v);
                if (a > mx) mx = a;
                if (c >= 0 && c < n) atomicAdd(&colcount[c], 1);
            }
            if (!(mx > 0.0)) err |= 8;
            // Section 4: scale so that the largest entry of every column of A^T D is 1
            d[j] = mx > 0.0 ? 1.0 / mx : 1.0;
            if (err) atomicOr(&out->err, err);
            len = max(len, e - s);
        }
    }
    len = wave_max_i(len);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = len;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < RED_BLOCK / 64; ++w) len = max(len, sh[w]);
        atomicMax(&out->max_row, len);
    }
}

// ||B(:,j)||^2 = sum over row j of A (CSR order) of (u_f(d_j a_jl))^2, in F
template <int UF>
__global__ void k_colnorm(int n, const int* __restrict__ rp, const double* __restrict__ av,
                          const double* __restrict__ d, typename UfTraits<UF>::F* __restrict__ bn) {
    using F = typename UfTraits<UF>::F;
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double dj = d[j];
    F s = F(0);
    for (int q = rp[j]; q < rp[j + 1]; ++q) {
        F b = scaled_entry<UF>(dj, av[q]);
        s = ffma(b, b, s);
    }
    bn[j] = s;
}

__global__ __launch_bounds__(RED_BLOCK) void k_max_count(int n, const int* __restrict__ cnt, PrepOut* out) {
    __shared__ int sh[RED_BLOCK / 64];
    int v = 0;
    for (int j = blockIdx.x * RED_BLOCK + threadIdx.x; j < n; j += gridDim.x * RED_BLOCK) v = max(v, cnt[j]);
    v = wave_max_i(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < RED_BLOCK / 64; ++w) v = max(v, sh[w]);
        atomicMax(&out->max_col, v);
    }
}

// CSC(A): rows j of every column l, and b_lj = u_f(d_j a_jl) (the entries of B by
// row); the order inside a column is irrelevant (the column kernel sorts them)
template <int UF>
__global__ void k_fill_csc(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ av, const double* __restrict__ d, int* __restrict__ cursor,
                           int* __restrict__ ri, typename UfTraits<UF>::F* __restrict__ bcv) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double dj = d[j];
    for (int q = rp[j]; q < rp[j + 1]; ++q) {
        int pos = atomicAdd(&cursor[ci[q]], 1);
        ri[pos] = j;
        bcv[pos] = scaled_entry<UF>(dj, av[q]);
    }
}

__global__ void k_validate_pattern(int n, int pnnz, const int* __restrict__ pp, const int* __restrict__ pi,
                                   PrepOut* out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    int err = 0, len = 0;
    if (k < n) {
        const int s = pp[k], e = pp[k + 1];
        if (s < 0 || e < s || e > pnnz || (k == 0 && s != 0) || (k == n - 1 && e != pnnz)) {
            err = 16;
        } else {
            if (e == s) err = 16;      // every column needs at least one index
            len = e - s;
            if (len <= 32) {
                // the column in registers, compared pairwise (distinct fillers past its end)
                int v[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) v[u] = u < len ? pi[s + u] : -1 - u;
                bool bad = false;
#pragma unroll
                for (int u = 0; u < 32; ++u) {
                    bad |= u < len && (v[u] < 0 || v[u] >= n);
#pragma unroll
                    for (int u2 = 0; u2 < u; ++u2) bad |= v[u] == v[u2];
                }
                if (bad) err = 16;
            } else {
                for (int q = s; q < e; ++q) {
                    int j = pi[q];
                    if (j < 0 || j >= n) err = 16;
                    for (int q2 = s; q2 < q; ++q2)
                        if (pi[q2] == j) err = 16;
                }
            }
        }
    }
    // one atomic per wave (a word updated by every thread serialises the launch)
    len = wave_max_i(len);
    err = wave_max_i(err);
    if ((threadIdx.x & 63) == 0) {
        if (err) atomicOr(&out->err, err);
        if (len) atomicMax(&out->max_pat, len);
    }
}

// exclusive scan of n ints into out[0..n], out[n] = total (three passes)
constexpr int SCAN_BLOCK = 1024;

__global__ void k_scan_block(int n, const int* __restrict__ in, int* __restrict__ out,
                             int* __restrict__ block_sums) {
    __shared__ int sh[SCAN_BLOCK];
    int i = blockIdx.x * SCAN_BLOCK + threadIdx.x;
    int v = i < n ? in[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        int t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = sh[threadIdx.x] - v;
    if (threadIdx.x == SCAN_BLOCK - 1) block_sums[blockIdx.x] = sh[threadIdx.x];
}

// exclusive scan of the block sums by one block of SCAN_BLOCK threads: each
// thread scans a contiguous run of them, the runs' totals are scanned in LDS
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_sums(int nb, int* __restrict__ block_sums,
                                                          int* __restrict__ total) {
    __shared__ int sh[SCAN_BLOCK];
    const int t = threadIdx.x;
    const int per = (nb + SCAN_BLOCK - 1) / SCAN_BLOCK;
    const int lo = min(nb, t * per), hi = min(nb, lo + per);
    int run = 0;
    for (int b = lo; b < hi; ++b) run += block_sums[b];
    sh[t] = run;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        const int v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int base = sh[t] - run;
    for (int b = lo; b < hi; ++b) {
        const int v = block_sums[b];
        block_sums[b] = base;
        base += v;
    }
    if (t == SCAN_BLOCK - 1) *total = sh[t];
}

__global__ void k_scan_add(int n, int* __restrict__ out, const int* __restrict__ block_sums,
                           const int* __restrict__ total) {
    int i = blockIdx.x * SCAN_BLOCK + threadIdx.x;
    if (i < n) out[i] += block_sums[blockIdx.x];
    if (i == 0) out[n] = *total;
}

// ---------------------------------------------------------------------------
// the column kernel
// ---------------------------------------------------------------------------

struct ColArgs {
    int n;
    const int* rp;
    const int* ci;
    const double* av;
    const int* cp;      // CSC(A) structure: column l -> rows j with a_jl != 0
    const int* ri;
    const double* d;
    const void* bnrm2;  // F per column of B
    const void* bcv;    // F per CSC(A) entry (column l, row j): b_lj = u_f(d_j a_jl)
    const int* pat_ptr;  // initial pattern (NULL: identity)
    const int* pat_idx;
    double eps;
    int alpha, beta, maxfill;
    const int* cols;    // problems to solve (NULL: 0..ncols-1)
    int ncols;
    int stride;
    int* len;
    int* jout;
    double* mout;
    int* steps;
    double* res;
    int* flags;
    int* nI;
    int* defer_list;
    int* defer_count;
    int qr_update;      // keep each column's QR across augmentation steps (same results)
};

// AMAX_: capacity of A-bar in elements when the QR is recomputed per solve: A-bar
// is stored with the odd leading dimension m | 1 of the solve at hand, and a
// column whose (|J| + 1) (m | 1) exceeds it is deferred (the default holds the
// largest problem of the shape)
// AREG_: A-bar lives in registers (lane c holds column c, e-bar in lane p) for the
// QR; only the Householder vector being applied, R and Q^T e-bar pass through LDS.
// FP32 arithmetic only (u_f = FP32, FP16, BF16).
constexpr int clog2(int x) {
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
}

template <int UF_, int G_, int MAXM_, int EMAX_, int CMAX_, int AMAX_ = G_ * (MAXM_ + 1), bool AREG_ = false>
struct Cfg {
    static constexpr int UF = UF_;
    static constexpr bool AREG = AREG_ && UF_ != SPAI_FP64;
    using F = typename UfTraits<UF_>::F;
    static constexpr int G = G_;           // lanes per problem
    static constexpr int MAXP = G_ - 1;    // columns of A-bar; lane MAXP can hold e-bar
    static constexpr int MAXM = MAXM_;     // rows of A-bar
    static constexpr int LD = MAXM_ + 1;   // odd leading dimension
    static constexpr int EMAX = EMAX_;     // gathered entries of B(:, J) (power of two)
    // Sort keys of the gathered entries, (row, slot): 32 bits (row relative to the
    // smallest gathered row, then log2(EMAX) slot bits) when EMAX <= 256, so a
    // column whose rows span 2^(32 - log2 EMAX) or more is deferred; the largest
    // configuration keeps (row << 32 | slot).
    static constexpr bool KEY32 = EMAX_ <= 256;
    using Key = std::conditional_t<KEY32, uint32_t, uint64_t>;
    static constexpr int SB = EMAX_ <= 64 ? 6 : EMAX_ <= 128 ? 7 : EMAX_ <= 256 ? 8 : 32;
    using Seg = std::conditional_t<(EMAX_ <= 255), uint8_t, uint16_t>;   // holds 0 .. EMAX
    static constexpr int CMAX = CMAX_;     // raw candidate entries (power of two)
    // Candidate keys (j, rank of the row l, slot): 32 bits when j relative to the
    // smallest candidate fits in the bits left (CJB >= 15; a column whose
    // candidates span more is deferred), else (j << 32 | rank << 16 | slot).
    // Ranks run to 2 MAXM; CMARK, above them all, marks the indices of J.
    static constexpr int CSB = clog2(CMAX_);
    static constexpr int CRB = clog2(2 * MAXM_ + 2);
    static constexpr int CJB = 32 - CSB - CRB;
    static constexpr bool CKEY32 = CJB >= 15;
    using CKey = std::conditional_t<CKEY32, uint32_t, uint64_t>;
    static constexpr int CMARK = CKEY32 ? (1 << CRB) - 1 : 0xFFFF;
    // scores of the unique candidates, in the space of the gathered values
    static constexpr int RHOCAP = EMAX_ + EMAX_ / (int)sizeof(F);
    static constexpr int AMAX = AMAX_;     // A-bar elements (recomputed QR)
    static constexpr int PPW = 64 / G_;    // problems per wavefront
};

// A-bar (columns in J order, Householder vectors below the diagonal, R above)
// and e-bar in column p, and the candidate arrays.  When the QR is updated across
// augmentation steps (INC) the factorisation must survive the candidate phase, so
// the two get their own space; otherwise they share it.
template <class C, bool INC> struct QrCand;
// The raw candidate keys are sorted in key[] and the unique candidates are
// compacted into its front in place (each is written at or before the position
// it is read from).
template <class C> struct QrCand<C, false> {
    using F = typename C::F;
    union {
        F A[C::AMAX];                 // leading dimension m | 1
        struct {
            typename C::CKey key[C::CMAX];   // candidate keys, sorted; then the unique j (ascending)
            F val[C::CMAX];                  // b_lj by slot
        } c;
    };
};
template <class C> struct QrCand<C, true> {
    using F = typename C::F;
    F A[(C::MAXP + 1) * C::LD];       // leading dimension LD (kept across solves)
    struct {
        typename C::CKey key[C::CMAX];
        F val[C::CMAX];
    } c;
    F tau[C::MAXP + 1];      // tau_t of each reflector
    uint8_t rz[C::MAXP + 1]; // reflector t skipped (zero column norm)
};

// A-bar in registers: the row position of every gathered slot (read while the
// columns are loaded into registers), the Householder vector being applied
// (rows t .. m-1, zero elsewhere), then R (column c: rows 0 .. c, packed) and
// Q^T e-bar for the back substitution; the candidate arrays share the space.
template <class C> struct QrCandReg {
    using F = typename C::F;
    union {
        uint8_t spos[C::EMAX];
        struct {
            F vb[C::MAXM];
            F R[C::MAXP * (C::MAXP + 1) / 2];
            F qe[C::MAXP + 1];
        } r;
        struct {
            typename C::CKey key[C::CMAX];
            F val[C::CMAX];
        } c;
    };
};

template <class C, bool INC>
struct alignas(16) Smem {
    using F = typename C::F;
    typename C::Key gkey[C::EMAX];  // (row, slot), sorted by row then slot
    std::conditional_t<C::AREG && !INC, QrCandReg<C>, QrCand<C, INC>> u;

    union {
        struct {
            F gval[C::EMAX];         // u_f(d_j a_ji) by slot
            uint8_t gcol[C::EMAX];   // position of j in J by slot
        };
        F rho[C::RHOCAP];            // candidate scores (the gathered values are dead by then)
    };
    uint8_t gpos[C::EMAX];   // row position in I of sorted entry e
    int I[C::MAXM];          // shadow in insertion order: earlier solves' rows, then new rows ascending
    uint8_t dpos[C::MAXM];   // position in I of the d-th row in ascending order
    typename C::Seg seg[C::MAXM + 1];   // first sorted entry of the d-th row in ascending order
    F s[C::MAXM];            // residual s-bar (rows in insertion order)
    int J[C::MAXP + 1];
    F mb[C::MAXP + 1];
    F Rd[C::MAXP + 1];
    F fs[4];
    int is[8];
};

__device__ __forceinline__ int next_pow2(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

template <int G, typename K>
__device__ void group_sort(K* keys, int N, int lane) {
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < (N >> 1); t += G) {
                int i = 2 * t - (t & (stride - 1));
                int l = i + stride;
                bool asc = (i & size) == 0;
                K a = keys[i], b = keys[l];
                if ((a > b) == asc) {
                    keys[i] = b;
                    keys[l] = a;
                }
            }
            wave_sync();
        }
    }
}

// rows and slots of the sort keys (rbase: the smallest gathered row of the
// column, for the 32-bit keys); key_rel orders keys by row alone
template <class C>
__device__ __forceinline__ uint32_t key_rel(typename C::Key k) {
    if constexpr (C::KEY32) return k >> C::SB;
    else return (uint32_t)(k >> 32);
}
template <class C>
__device__ __forceinline__ int key_row(typename C::Key k, int rbase) {
    if constexpr (C::KEY32) return (int)(k >> C::SB) + rbase;
    else return (int)(uint32_t)(k >> 32);
}
template <class C>
__device__ __forceinline__ int key_slot(typename C::Key k) {
    if constexpr (C::KEY32) return (int)(k & ((1u << C::SB) - 1u));
    else return (int)(uint32_t)(k & 0xffffffffu);
}

template <class C>
__device__ __forceinline__ typename C::CKey ckey_j(typename C::CKey k) {
    if constexpr (C::CKEY32) return k >> (C::CSB + C::CRB);
    else return k >> 32;
}
template <class C>
__device__ __forceinline__ int ckey_rank(typename C::CKey k) {
    if constexpr (C::CKEY32) return (int)((k >> C::CSB) & ((1u << C::CRB) - 1u));
    else return (int)((k >> 16) & 0xffffu);
}
template <class C>
__device__ __forceinline__ int ckey_slot(typename C::CKey k) {
    if constexpr (C::CKEY32) return (int)(k & ((1u << C::CSB) - 1u));
    else return (int)(k & 0xffffu);
}

template <class C, bool INC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(C::AREG && !INC ? 3 : 1))) void k_spai_columns(ColArgs a) {
    using F = typename C::F;
    constexpr int G = C::G;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int wl = threadIdx.x;
    const int g = wl / G;
    const int lane = wl - g * G;
    const int gl0 = wl - lane;                // first lane of the group (lane permutes stay inside it)
    if (g >= C::PPW) return;
    const int prob = blockIdx.x * C::PPW + g;
    if (prob >= a.ncols) return;
    Smem<C, INC>& S = reinterpret_cast<Smem<C, INC>*>(smem_raw)[g];
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (g * G));
    const uint64_t below = (wl == 0) ? 0ull : ((~0ull) >> (64 - wl));
    const F* bnrm2 = reinterpret_cast<const F*>(a.bnrm2);
    const F* bcv = reinterpret_cast<const F*>(a.bcv);
    using CKey = typename C::CKey;

    const int k = a.cols ? a.cols[prob] : prob;
    int p;
    bool defer = false;
    // initial pattern, ascending (Algorithm 1 input J; identity when absent)
    if (a.pat_ptr) {
        int s0 = a.pat_ptr[k];
        p = a.pat_ptr[k + 1] - s0;
        if (p > C::MAXP || p < 1) {
            defer = (p > C::MAXP);
            p = 0;
        } else {
            int my = lane < p ? a.pat_idx[s0 + lane] : INT_MAX;
            int rank = 0;
            for (int t = 0; t < p; ++t) {
                int o = a.pat_idx[s0 + t];
                rank += (o < my);
            }
            if (lane < p) S.J[rank] = my;
        }
    } else {
        p = 1;
        if (lane == 0) S.J[0] = k;
    }
    wave_sync();
    const int cap = a.maxfill > p ? a.maxfill : p;
    int flags = 0, step = 0, m = 0, kpos = -1, p_prev = 0;
    int rbase = 0;                            // smallest gathered row (32-bit keys)
    F res = F(0);
    if (p == 0 && !defer) flags |= CF_EPS;

    for (step = 0; p > 0 && !defer; ++step) {
        // ---- shadow I_k and A-bar = B(I_k, J_k), e-bar = e_k(I_k) ----
        // The rows of the previous solve keep their positions and the rows the new
        // columns bring in follow in ascending order.  The columns factored before
        // are zero in the new rows, so their Householder reflectors do not change:
        // the QR below equals an incremental update of the previous one.
        const int m_prev = m;
        int myj = 0, mys = 0, myn = 0;
        if (lane < p) {
            myj = S.J[lane];
            mys = a.rp[myj];
            myn = a.rp[myj + 1] - mys;
        }
        int off = 0, E = 0;
        for (int t = 0; t < G; ++t) {
            const int v = __shfl(myn, gl0 + t, 64);
            off += (t < lane) ? v : 0;
            E += v;
        }
        if (E > C::EMAX) { defer = true; break; }
        int rlo = INT_MAX, rhi = -1;
        if (lane < p) {
            double dj = a.d[myj];
            // unrolled by 4: four entries' index and value loads in flight (each
            // entry has its own slot, so the order does not matter)
#pragma unroll 4
            for (int q = 0; q < myn; ++q) {
                int slot = off + q;
                int i = a.ci[mys + q];
                if constexpr (C::KEY32) {
                    S.gkey[slot] = (uint32_t)i;        // the row; made a key below
                    rlo = min(rlo, i);
                    rhi = max(rhi, i);
                } else {
                    S.gkey[slot] = ((uint64_t)(uint32_t)i << 32) | (uint32_t)slot;
                }
                S.gval[slot] = scaled_entry<C::UF>(dj, a.av[mys + q]);
                S.gcol[slot] = (uint8_t)lane;
            }
        }
        if constexpr (C::KEY32) {
            // rows relative to the smallest one, with the slot in the low bits
            const int mylo = rlo, myhi = rhi;
            for (int t = 0; t < G; ++t) {
                rlo = min(rlo, __shfl(mylo, gl0 + t, 64));
                rhi = max(rhi, __shfl(myhi, gl0 + t, 64));
            }
            wave_sync();                          // the raw rows are in gkey
            rbase = rlo;
            if (E > 0 && (unsigned)(rhi - rlo) >= (1u << (32 - C::SB)) - 1u) { defer = true; break; }
            for (int e = lane; e < E; e += G) S.gkey[e] = ((S.gkey[e] - (uint32_t)rlo) << C::SB) | (uint32_t)e;
        }
        const int E2 = next_pow2(E > 0 ? E : 1);
        for (int e = E + lane; e < E2; e += G) S.gkey[e] = ~typename C::Key(0);
        wave_sync();
        group_sort<G>(S.gkey, E2, lane);
        // count distinct rows
        m = 0;
        for (int base = 0; base < E; base += G) {
            int e = base + lane;
            bool head = false;
            if (e < E) {
                const uint32_t i = key_rel<C>(S.gkey[e]);
                head = (e == 0) || (key_rel<C>(S.gkey[e - 1]) != i);
            }
            m += __popcll(ballot(head) & gmask);
        }
        if (m > C::MAXM) { defer = true; break; }
        const int ld = INC ? C::LD : (m | 1);   // leading dimension of A-bar
        if (!INC && !C::AREG && (p + 1) * ld > C::AMAX) { defer = true; break; }
        // sorted rows, their segments, and their positions in I.  A row is old
        // (in the previous shadow) iff the first entry of its segment comes from a
        // column of the previous solve (slots follow the column order); old rows
        // appear in the same relative order as in the previous sorted list, so the
        // previous dpos gives their positions.  Pass 1 reads the previous lists and
        // leaves each head's position (other entries: their sorted row index) in
        // gpos; pass 2 writes the new lists; pass 3 maps every entry to its position.
        {
            int run = 0, nnew = 0, nold = 0;
            for (int base = 0; base < E; base += G) {
                int e = base + lane;
                bool head = false, old = false;
                if (e < E) {
                    const uint32_t i = key_rel<C>(S.gkey[e]);
                    head = (e == 0) || (key_rel<C>(S.gkey[e - 1]) != i);
                    old = head && S.gcol[key_slot<C>(S.gkey[e])] < p_prev;
                }
                const bool fresh = head && !old;
                uint64_t bal = ballot(head) & gmask, obal = ballot(old) & gmask, nbal = ballot(fresh) & gmask;
                if (e < E) {
                    if (head)
                        S.gpos[e] = old ? S.dpos[nold + __popcll(obal & below)]
                                        : (uint8_t)(m_prev + nnew + __popcll(nbal & below));
                    else
                        S.gpos[e] = (uint8_t)(run + __popcll(bal & below) - 1);
                }
                run += __popcll(bal);
                nold += __popcll(obal);
                nnew += __popcll(nbal);
            }
            wave_sync();
            run = 0;
            for (int base = 0; base < E; base += G) {
                int e = base + lane;
                bool head = false;
                uint32_t i = 0;
                if (e < E) {
                    i = key_rel<C>(S.gkey[e]);
                    head = (e == 0) || (key_rel<C>(S.gkey[e - 1]) != i);
                }
                uint64_t bal = ballot(head) & gmask;
                if (head) {
                    const int d = run + __popcll(bal & below);
                    const int pos = S.gpos[e];
                    S.seg[d] = (typename C::Seg)e;
                    S.dpos[d] = (uint8_t)pos;
                    if (pos >= m_prev) S.I[pos] = key_row<C>(S.gkey[e], rbase);
                }
                run += __popcll(bal);
            }
            if (lane == 0) {
                S.seg[m] = (typename C::Seg)E;
                S.is[0] = -1;
            }
        }
        wave_sync();
        for (int e = lane; e < E; e += G) {
            const bool head = (e == 0) || (key_rel<C>(S.gkey[e - 1]) != key_rel<C>(S.gkey[e]));
            if (!head) S.gpos[e] = S.dpos[S.gpos[e]];
        }
        // With the update (INC), columns 0 .. p_old-1 and e-bar (in column p_old)
        // still hold the factorisation of the previous solve over its m_prev rows:
        // the new rows are zero in those columns, so only the new columns are
        // gathered, the old reflectors are applied to them, and the QR continues at
        // column p_old.  Without it (p_old = 0) everything is rebuilt: the same
        // operations on the same values, so the same bits.
        const int p_old = (INC && step > 0) ? p_prev : 0;
        constexpr bool AR = C::AREG && !INC;
        F colr[AR ? C::MAXM : 1];
        if constexpr (AR) {
            // every slot's row position, then each lane takes its column's entries
            // (lane c: column c of J; lane p: e-bar)
            for (int e = lane; e < E; e += G) S.u.spos[key_slot<C>(S.gkey[e])] = S.gpos[e];
            wave_sync();
#pragma unroll
            for (int i = 0; i < C::MAXM; ++i) colr[i] = F(0);
            if (lane < p) {
                for (int q = 0; q < myn; ++q) {
                    const int pos = S.u.spos[off + q];
                    const F v = S.gval[off + q];
#pragma unroll
                    for (int i = 0; i < C::MAXM; ++i) colr[i] = (i == pos) ? v : colr[i];
                }
            }
            for (int e = lane; e < E; e += G)
                if (S.I[S.gpos[e]] == k) S.is[0] = S.gpos[e];
            wave_sync();
            kpos = S.is[0];
            if (lane == p && kpos >= 0) {
#pragma unroll
                for (int i = 0; i < C::MAXM; ++i) colr[i] = (i == kpos) ? F(1) : colr[i];
            }
        }
        if constexpr (!AR) {
            if (p_old > 0 && lane == p) {
                // e-bar after the previous reflectors moves from column p_old to column p
                const F* src = &S.u.A[p_old * ld];
                F* dst = &S.u.A[p * ld];
                for (int i = 0; i < m_prev; ++i) dst[i] = src[i];
                for (int i = m_prev; i < m; ++i) dst[i] = F(0);
            }
        }
        wave_sync();
        if constexpr (!AR) {
            if (lane < p_old) {
                F* col = &S.u.A[lane * ld];
                for (int i = m_prev; i < m; ++i) col[i] = F(0);
            } else if (lane < p || (p_old == 0 && lane == p)) {
                F* col = &S.u.A[lane * ld];
                for (int i = 0; i < m; ++i) col[i] = F(0);
            }
            wave_sync();
            for (int e = lane; e < E; e += G) {
                int slot = key_slot<C>(S.gkey[e]);
                int pos = S.gpos[e];
                if (S.gcol[slot] >= p_old) S.u.A[S.gcol[slot] * ld + pos] = S.gval[slot];
                if (S.I[pos] == k) S.is[0] = pos;
            }
            wave_sync();
            kpos = S.is[0];
            // e-bar = e_k(I): the 1 is placed by a full build, or by the update when k is a new row
            if (lane == 0 && kpos >= 0 && (p_old == 0 || kpos >= m_prev)) S.u.A[p * ld + kpos] = F(1);
        }
        wave_sync();

        // ---- Householder QR of A-bar, applied to e-bar as well ----
        // For x = A(t:m, t): sigma = ||x||, alpha = -sgn(x_t) sigma (sgn(0) = +1),
        // v = x - alpha e_1 with v^T v = 2 sigma (sigma + |x_t|), so the reflector
        // maps a column a to a - (v^T a / tau) v with tau = sigma (sigma + |x_t|).
        // Sums run over the rows t .. m-1 (the stored zeros of the new rows add
        // nothing), so the update equals the factorisation from scratch.
        bool rankdef = false;
        const int qsteps = p < m ? p : m;
        // reflectors of the previous solve: t < min(p_old, m_prev) (later ones met only
        // zeros then and meet only zeros now: the loop below finds them rank deficient)
        const int qold = min(min(p_old, m_prev), qsteps);
        if constexpr (INC)
            for (int t = 0; t < qold; ++t) rankdef |= S.u.rz[t] != 0;
        if constexpr (INC) if (lane >= p_old && lane < p) {
            // the previous reflectors on a new column, one after the other
            F* col = &S.u.A[lane * ld];
            for (int t = 0; t < qold; ++t) {
                if (S.u.rz[t]) continue;
                const F* v = &S.u.A[t * ld];
                F dot = F(0);
                for (int i = t; i < m; ++i) dot = ffma(v[i], col[i], dot);
                F f = dot / S.u.tau[t];
                for (int i = t; i < m; ++i) col[i] = store<C::UF>(ffma(-f, v[i], col[i]));
            }
        }
        wave_sync();
        if constexpr (AR) {
            // The same operations as below on the register columns, rows in chunks
            // of 8.  The sums run over whole chunks: the rows outside t .. m-1
            // contribute exact zeros (the Householder vector is zero there, the
            // rows past m are zero padding), and an ascending sum that starts at
            // +0 and adds +-0 terms keeps its value, so the bits equal the sums
            // over t .. m-1; chunks wholly above row t are skipped (t is uniform).
            // The squared norm of the next pivot column (rows t+1 .. m-1, in
            // ascending order, of the values just stored) is summed during the
            // update of reflector t, the same sum the pivot lane would form next.
            static_assert(C::MAXM % 8 == 0, "chunks of 8 rows");
            constexpr int NCH = C::MAXM / 8;
            F sig2n = F(0);
            bool sig_ok = false;                // sig2n holds rows t .. m-1 of this column
            for (int t = 0; t < qsteps; ++t) {
                const int c0 = t >> 3;          // first chunk with rows >= t
                if (lane == t) {
                    F sig2 = sig2n;
                    if (!sig_ok) {
                        sig2 = F(0);
#pragma unroll
                        for (int i = 0; i < C::MAXM; ++i) {
                            const F xi = i >= t ? colr[i] : F(0);
                            sig2 = ffma(xi, xi, sig2);
                        }
                    }
                    const F sigma = fsqrt(sig2);
                    if (sigma == F(0)) {
                        S.Rd[t] = F(0);
                        S.is[1] = 1;
                    } else {
                        F xt = F(0);
#pragma unroll
                        for (int i = 0; i < C::MAXM; ++i) xt = i == t ? colr[i] : xt;
                        const F alpha = (xt >= F(0)) ? -sigma : sigma;
                        const F vt = store<C::UF>(xt - alpha);
                        // R(0 .. t-1, t) is final: staged for the back substitution
                        F* rc = &S.u.r.R[t * (t + 1) / 2];
#pragma unroll
                        for (int i = 0; i < C::MAXP; ++i)
                            if (i < t) rc[i] = colr[i];
                        // the Householder vector: rows t .. m-1 (zero above t and past m)
                        float4* vb4 = reinterpret_cast<float4*>(S.u.r.vb);
#pragma unroll
                        for (int q = 0; q < C::MAXM / 4; ++q) {
                            float4 o;
                            const int i = 4 * q;
                            o.x = i + 0 < t ? F(0) : (i + 0 == t ? vt : colr[i + 0]);
                            o.y = i + 1 < t ? F(0) : (i + 1 == t ? vt : colr[i + 1]);
                            o.z = i + 2 < t ? F(0) : (i + 2 == t ? vt : colr[i + 2]);
                            o.w = i + 3 < t ? F(0) : (i + 3 == t ? vt : colr[i + 3]);
                            vb4[q] = o;
                        }
                        S.fs[0] = sigma * (sigma + fabs(xt));
                        S.Rd[t] = store<C::UF>(alpha);
                        S.is[1] = 0;
                    }
                }
                wave_sync();
                if (S.is[1]) {
                    rankdef = true;
                    sig_ok = false;             // the columns did not change: norms from scratch
                    continue;
                }
                const F tau = S.fs[0];
                if (lane > t && lane <= p) {
                    const float4* vb4 = reinterpret_cast<const float4*>(S.u.r.vb);
                    F dot = F(0);
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        if (ch < c0) continue;  // rows above t: zero terms
                        const float4 a0 = vb4[2 * ch], a1 = vb4[2 * ch + 1];
                        const int i = 8 * ch;
                        dot = ffma(a0.x, colr[i + 0], dot);
                        dot = ffma(a0.y, colr[i + 1], dot);
                        dot = ffma(a0.z, colr[i + 2], dot);
                        dot = ffma(a0.w, colr[i + 3], dot);
                        dot = ffma(a1.x, colr[i + 4], dot);
                        dot = ffma(a1.y, colr[i + 5], dot);
                        dot = ffma(a1.z, colr[i + 6], dot);
                        dot = ffma(a1.w, colr[i + 7], dot);
                    }
                    const F f = dot / tau;
                    F sn = F(0);
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        if (ch < c0) continue;
                        const float4 a0 = vb4[2 * ch], a1 = vb4[2 * ch + 1];
                        const F vv[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int i = 8 * ch + q;
                            const F y = store<C::UF>(ffma(-f, vv[q], colr[i]));
                            colr[i] = i >= t ? y : colr[i];
                            const F z = i > t ? y : F(0);
                            sn = ffma(z, z, sn);
                        }
                    }
                    sig2n = sn;
                    sig_ok = true;
                }
                wave_sync();
            }
            // columns that never became pivots (p > m) stage R now; Q^T e-bar (rows 0 .. p-1)
            if (lane >= qsteps && lane < p) {
                F* rc = &S.u.r.R[lane * (lane + 1) / 2];
#pragma unroll
                for (int i = 0; i < C::MAXP; ++i)
                    if (i <= lane) rc[i] = colr[i];
            } else if (lane == p) {
#pragma unroll
                for (int i = 0; i < C::MAXP; ++i)
                    if (i < p) S.u.r.qe[i] = colr[i];
            }
            wave_sync();
        }
        if constexpr (!AR) for (int t = qold; t < qsteps; ++t) {
            if (lane == t) {
                F* x = &S.u.A[t * ld];
                F sig2 = F(0);
                for (int i = t; i < m; ++i) sig2 = ffma(x[i], x[i], sig2);
                F sigma = fsqrt(sig2);
                if (sigma == F(0)) {
                    S.Rd[t] = F(0);
                    if constexpr (INC) S.u.rz[t] = 1;
                    S.is[1] = 1;
                } else {
                    F xt = x[t];
                    F alpha = (xt >= F(0)) ? -sigma : sigma;
                    x[t] = store<C::UF>(xt - alpha);
                    S.fs[0] = sigma * (sigma + fabs(xt));
                    if constexpr (INC) {
                        S.u.tau[t] = S.fs[0];
                        S.u.rz[t] = 0;
                    }
                    S.Rd[t] = store<C::UF>(alpha);
                    S.is[1] = 0;
                }
            }
            wave_sync();
            if (S.is[1]) {
                rankdef = true;
                continue;
            }
            const F tau = S.fs[0];
            if (lane > t && lane <= p) {
                const F* v = &S.u.A[t * ld];
                F* col = &S.u.A[lane * ld];
                F dot = F(0);
                for (int i = t; i < m; ++i) dot = ffma(v[i], col[i], dot);
                F f = dot / tau;
                for (int i = t; i < m; ++i) col[i] = store<C::UF>(ffma(-f, v[i], col[i]));
            }
            wave_sync();
        }
        if (p > m) rankdef = true;
        // back substitution, c = p-1 down to 0, inner sum over c' ascending
        if constexpr (AR) {
            // m-bar in registers, R read at fixed offsets of its packed columns
            if (lane == 0) {
                F mbr[C::MAXP];
                int rd = 0;
#pragma unroll
                for (int c = C::MAXP - 1; c >= 0; --c) {
                    mbr[c] = F(0);
                    if (c < p) {
                        if (c >= m || S.Rd[c] == F(0)) {
                            rd = 1;
                        } else {
                            F s = S.u.r.qe[c];
#pragma unroll
                            for (int c2 = c + 1; c2 < C::MAXP; ++c2)
                                s = c2 < p ? ffma(-S.u.r.R[c2 * (c2 + 1) / 2 + c], mbr[c2], s) : s;
                            mbr[c] = store<C::UF>(s / S.Rd[c]);
                        }
                    }
                }
#pragma unroll
                for (int c = 0; c < C::MAXP; ++c)
                    if (c < p) S.mb[c] = mbr[c];
                S.is[2] = rd;
            }
        } else if (lane == 0) {
            int rd = 0;
            for (int c = p - 1; c >= 0; --c) {
                if (c >= m || S.Rd[c] == F(0)) {
                    S.mb[c] = F(0);
                    rd = 1;
                    continue;
                }
                if constexpr (!AR) {
                    F s = S.u.A[p * ld + c];
                    for (int c2 = c + 1; c2 < p; ++c2) s = ffma(-S.u.A[c2 * ld + c], S.mb[c2], s);
                    S.mb[c] = store<C::UF>(s / S.Rd[c]);
                }
            }
            S.is[2] = rd;
        }
        wave_sync();
        if (S.is[2]) rankdef = true;
        if (rankdef) flags |= CF_RANKDEF;

        // ---- residual s-bar = A-bar m-bar - e-bar over the stored entries ----
        for (int d = lane; d < m; d += G) {
            F acc = F(0);
            for (int e = S.seg[d]; e < S.seg[d + 1]; ++e) {
                int slot = key_slot<C>(S.gkey[e]);
                acc = ffma(S.gval[slot], S.mb[S.gcol[slot]], acc);
            }
            const int pos = S.dpos[d];
            S.s[pos] = acc - ((pos == kpos) ? F(1) : F(0));
        }
        wave_sync();
        if (lane == 0) {
            F r2 = F(0);
            for (int pos = 0; pos < m; ++pos) r2 = ffma(S.s[pos], S.s[pos], r2);
            // row k of the full residual is -1 when k lies outside the shadow
            if (kpos < 0) r2 = r2 + F(1);
            S.fs[1] = r2;
            S.is[3] = 0;                      // candidate phase: entries, smallest and largest j
            S.is[4] = INT_MAX;
            S.is[5] = -1;
        }
        wave_sync();
        const F res2 = S.fs[1];
        res = fsqrt(res2);
        if (!isfinite(res)) { flags |= CF_NONFINITE; break; }
        if ((double)res <= a.eps) break;                        // stopping test
        if (step >= a.alpha || p >= cap) { flags |= CF_EPS; break; }

        // ---- candidates: L = I u {k}, J~ = (union of N_l) \ J ----
        // One entry per pair (l, j) with l in L and b_lj != 0, read from CSC(B):
        // its key orders by j, then by the row l (the rank of l among L in
        // ascending order: 2d + 1 for the d-th row of I, 2 #{rows of I < k} for k
        // outside I), then the slot holding b_lj; every j of J adds a marker that
        // sorts after its entries.  After the sort, the entries of candidate j are
        // contiguous and in ascending row order, which is the order of the sum
        // r^T B e_j over the rows of B(:, j) that lie in L.
        constexpr int RPL = (C::MAXM + G - 1) / G;   // shadow rows per lane
        int rq0[RPL], rcnt[RPL], roff[RPL];
        int cnt = 0, rk = 0;
#pragma unroll
        for (int it = 0; it < RPL; ++it) {
            const int d = lane + it * G;
            int l = 0;
            if (d < m) l = key_row<C>(S.gkey[S.seg[d]], rbase);
            rq0[it] = d < m ? a.cp[l] : 0;
            rcnt[it] = d < m ? a.cp[l + 1] - rq0[it] : 0;
            cnt += rcnt[it];
            rk += __popcll(ballot(d < m && l < k) & gmask);
        }
        const int kq0 = a.cp[k], kcnt = kpos < 0 ? a.cp[k + 1] - kq0 : 0;
        const int mine = cnt + (lane == 0 ? kcnt : 0) + (lane < p ? 1 : 0);
        // slots in any order: the keys are distinct without them, so the sorted
        // order and every sum below do not depend on it
        int coff = atomicAdd(&S.is[3], mine);
        wave_sync();
        const int Ec = S.is[3];
        if (Ec > C::CMAX) { defer = true; break; }
        int jlo = INT_MAX, jhi = -1;
        auto fill = [&](int q0, int qn) {
            for (int qb = 0; qb < qn; qb += 8) {
                int jj[8];
                F bb[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int q = q0 + min(qb + u, qn - 1);
                    jj[u] = a.ri[q];
                    bb[u] = bcv[q];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (qb + u < qn) {
                        S.u.c.key[coff] = (CKey)jj[u];
                        S.u.c.val[coff] = bb[u];
                        ++coff;
                        jlo = min(jlo, jj[u]);
                        jhi = max(jhi, jj[u]);
                    }
            }
        };
#pragma unroll
        for (int it = 0; it < RPL; ++it) {
            roff[it] = coff;
            fill(rq0[it], rcnt[it]);
        }
        const int koff = coff;
        if (lane == 0) fill(kq0, kcnt);
        const int moff = coff;
        if (lane < p) {
            const int jm = S.J[lane];
            S.u.c.key[moff] = (CKey)jm;
            jlo = min(jlo, jm);
            jhi = max(jhi, jm);
        }
        if (jhi >= 0) {
            atomicMin(&S.is[4], jlo);
            atomicMax(&S.is[5], jhi);
        }
        wave_sync();
        const int jbase = S.is[4];
        if constexpr (C::CKEY32) {
            if ((unsigned)(S.is[5] - jbase) >= (1u << C::CJB) - 1u) { defer = true; break; }
        }
        auto mk = [&](int slot, int rank) {
            const CKey j = S.u.c.key[slot];
            if constexpr (C::CKEY32)
                S.u.c.key[slot] = ((j - (CKey)jbase) << (C::CSB + C::CRB)) | ((CKey)rank << C::CSB) | (CKey)slot;
            else
                S.u.c.key[slot] = (j << 32) | ((CKey)rank << 16) | (CKey)slot;
        };
#pragma unroll
        for (int it = 0; it < RPL; ++it)
            for (int e = 0; e < rcnt[it]; ++e) mk(roff[it] + e, 2 * (lane + it * G) + 1);
        if (lane == 0)
            for (int e = 0; e < kcnt; ++e) mk(koff + e, 2 * rk);
        if (lane < p) mk(moff, C::CMARK);
        const int Ec2 = next_pow2(Ec > 0 ? Ec : 1);
        for (int e = Ec + lane; e < Ec2; e += G) S.u.c.key[e] = ~CKey(0);
        wave_sync();
        group_sort<G>(S.u.c.key, Ec2, lane);
        // unique candidates outside J, in ascending j: the first entry of each run
        // of equal j sums its run (a marker at the end of the run: j is in J) and
        // scores rho_j = sqrt(max(res^2 - (r^T B e_j)^2 / ||B e_j||^2, 0)), r being
        // the residual on L (s-bar on I, -1 at k when k is outside I).  Candidate c
        // goes to key[c] (c is at most the position of its first entry, read
        // before) and rho[c] (the space of the gathered values, unused from here).
        int nc = 0;
        bool over = false;
        CKey jprev = 0;                      // j of the last entry of the previous stride
        for (int base = 0; base < Ec; base += G) {
            const int e = base + lane;
            bool head = false;
            CKey jk = 0;
            if (e < Ec) {
                jk = ckey_j<C>(S.u.c.key[e]);
                // entry e - 1 of the first lane may already hold a compacted candidate
                const CKey jp = lane == 0 ? jprev : ckey_j<C>(S.u.c.key[e - 1]);
                head = (e == 0) || (jp != jk);
            }
            const int last = min(base + G, Ec) - 1;
            jprev = ckey_j<C>(S.u.c.key[last]);
            const int j = (int)jk + (C::CKEY32 ? jbase : 0);
            F bn = F(1), tj = F(0);
            bool inJ = false;
            if (head) {
                bn = bnrm2[j];
                for (int e2 = e; e2 < Ec; ++e2) {
                    const CKey kk = S.u.c.key[e2];
                    if (ckey_j<C>(kk) != jk) break;
                    const int rank = ckey_rank<C>(kk);
                    if (rank == C::CMARK) {
                        inJ = true;
                        break;
                    }
                    const F r = (rank & 1) ? S.s[S.dpos[rank >> 1]] : F(-1);
                    tj = ffma(r, S.u.c.val[ckey_slot<C>(kk)], tj);
                }
            }
            const bool valid = head && !inJ;
            const uint64_t bal = ballot(valid) & gmask;
            if (nc + __popcll(bal) > C::RHOCAP) {
                over = true;
                break;
            }
            if (valid) {
                F r2 = res2 - (tj * tj) / bn;
                if (r2 <= F(0)) r2 = F(0);
                const int c = nc + __popcll(bal & below);
                S.u.c.key[c] = (CKey)j;
                S.rho[c] = fsqrt(r2);
            }
            nc += __popcll(bal);
        }
        if (over) { defer = true; break; }
        wave_sync();
        if (nc == 0) { flags |= CF_EPS; break; }
        if (lane == 0) {
            F rs = F(0);
            for (int c = 0; c < nc; ++c) rs = rs + S.rho[c];   // ascending j
            S.fs[2] = rs / (F)nc;
        }
        wave_sync();
        const F rbar = S.fs[2];
        // acceptable: rho_j <= rho-bar; add the min(beta, #acceptable, cap - |J|)
        // best, ordered by (rho, j): candidate c goes to position p + (its rank in
        // that order) when the rank is below the number taken (every candidate
        // ordered before an acceptable one is acceptable)
        int na = 0;
        for (int base = 0; base < nc; base += G) {
            int c = base + lane;
            bool ok = (c < nc) && (S.rho[c] <= rbar);
            na += __popcll(ballot(ok) & gmask);
        }
        int nsel = a.beta;
        if (na < nsel) nsel = na;
        if (cap - p < nsel) nsel = cap - p;
        if (nsel <= 0) { flags |= CF_EPS; break; }
        for (int c = lane; c < nc; c += G) {
            const F rc = S.rho[c];
            const int jc = (int)S.u.c.key[c];
            if (!(rc <= rbar)) continue;
            int rank = 0;
            for (int c2 = 0; c2 < nc; ++c2) {
                const F r2 = S.rho[c2];
                rank += (r2 < rc || (r2 == rc && (int)S.u.c.key[c2] < jc)) ? 1 : 0;
            }
            if (rank < nsel) S.J[p + rank] = jc;
        }
        wave_sync();
        p_prev = p;
        p += nsel;
    }

    if (defer) {
        if (lane == 0) {
            a.flags[k] = CF_DEFERRED;
            int slot = atomicAdd(a.defer_count, 1);
            a.defer_list[slot] = k;
        }
        return;
    }
    // outputs: J_k in insertion order with m-bar of the last solve
    const size_t o = (size_t)k * (size_t)a.stride;
    for (int c = lane; c < a.stride; c += G) {
        a.jout[o + c] = c < p ? S.J[c] : -1;
        a.mout[o + c] = c < p ? (double)S.mb[c] : 0.0;
    }
    if (lane == 0) {
        a.len[k] = p;
        a.steps[k] = step;
        a.res[k] = (double)res;
        a.flags[k] = flags;
        a.nI[k] = m;
    }
}

// ---------------------------------------------------------------------------
// compaction: row k of P = m_k^T with columns ascending
// ---------------------------------------------------------------------------

template <int VP>
__global__ void k_compact(int n, int stride, const int* __restrict__ len, const int* __restrict__ jin,
                          const double* __restrict__ min_, const int* __restrict__ rowptr,
                          int* __restrict__ col, typename ValType<VP>::T* __restrict__ val) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)n * stride) return;
    int k = (int)(t / stride);
    int c = (int)(t - (long long)k * stride);
    int L = len[k];
    if (c >= L) return;
    const int* J = jin + (size_t)k * stride;
    int j = J[c];
    int rank = 0;
    for (int c2 = 0; c2 < L; ++c2) rank += (J[c2] < j);
    int pos = rowptr[k] + rank;
    col[pos] = j;
    double v = min_[(size_t)k * stride + c];
    using T = typename ValType<VP>::T;
    if constexpr (VP == SPAI_FP64) val[pos] = v;
    else if constexpr (VP == SPAI_FP32) val[pos] = (float)v;
    else if constexpr (VP == SPAI_FP16) val[pos] = __float2half_rn((float)v);
    else val[pos] = T((float)v);
}

struct BuildStatsDev {
    int over_eps, rankdef, nonfinite, max_len, max_steps, max_shadow;
    unsigned long long max_res_bits;
    unsigned long long nnz_numeric;   // entries of P whose value is not zero
    int fallback, pad;
};

__global__ __launch_bounds__(RED_BLOCK) void k_build_stats(int n, int stride, const int* __restrict__ len,
                              const int* __restrict__ steps, const double* __restrict__ res,
                              const int* __restrict__ flags, const int* __restrict__ nI,
                              const double* __restrict__ mval, BuildStatsDev* st) {
    __shared__ int shi[7][RED_BLOCK / 64];
    __shared__ unsigned long long shr[2][RED_BLOCK / 64];
    int c_eps = 0, c_rd = 0, c_nf = 0, c_fb = 0, l = 0, sp = 0, sh = 0;
    unsigned long long rb = 0ull;   // non-negative doubles order as their bit patterns
    unsigned long long nz = 0ull;
    for (int k = blockIdx.x * RED_BLOCK + threadIdx.x; k < n; k += gridDim.x * RED_BLOCK) {
        const int f = flags[k];
        c_eps += (f & CF_EPS) ? 1 : 0;
        c_rd += (f & CF_RANKDEF) ? 1 : 0;
        c_nf += (f & CF_NONFINITE) ? 1 : 0;
        c_fb += (f & CF_FALLBACK) ? 1 : 0;
        const int L = len[k];
        for (int c = 0; c < L; ++c) nz += mval[(size_t)k * stride + c] != 0.0 ? 1ull : 0ull;
        l = max(l, len[k]);
        sp = max(sp, steps[k]);
        sh = max(sh, nI[k]);
        const double r = res[k];
        if (r >= 0.0) {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(r);
            rb = bits > rb ? bits : rb;
        }
    }
    c_eps = wave_sum_i(c_eps);
    c_rd = wave_sum_i(c_rd);
    c_nf = wave_sum_i(c_nf);
    c_fb = wave_sum_i(c_fb);
    l = wave_max_i(l);
    sp = wave_max_i(sp);
    sh = wave_max_i(sh);
    rb = wave_max_u64(rb);
    for (int o = 32; o > 0; o >>= 1) nz += __shfl_xor(nz, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        shi[0][w] = c_eps;
        shi[1][w] = c_rd;
        shi[2][w] = c_nf;
        shi[3][w] = l;
        shi[4][w] = sp;
        shi[5][w] = sh;
        shi[6][w] = c_fb;
        shr[0][w] = rb;
        shr[1][w] = nz;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < RED_BLOCK / 64; ++v) {
            c_eps += shi[0][v];
            c_rd += shi[1][v];
            c_nf += shi[2][v];
            l = max(l, shi[3][v]);
            sp = max(sp, shi[4][v]);
            sh = max(sh, shi[5][v]);
            c_fb += shi[6][v];
            rb = shr[0][v] > rb ? shr[0][v] : rb;
            nz += shr[1][v];
        }
        if (c_eps) atomicAdd(&st->over_eps, c_eps);
        if (c_rd) atomicAdd(&st->rankdef, c_rd);
        if (c_nf) atomicAdd(&st->nonfinite, c_nf);
        if (c_fb) atomicAdd(&st->fallback, c_fb);
        if (nz) atomicAdd(&st->nnz_numeric, nz);
        atomicMax(&st->max_len, l);
        atomicMax(&st->max_steps, sp);
        atomicMax(&st->max_shadow, sh);
        if (rb) atomicMax(&st->max_res_bits, rb);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <class C, bool INC>
static int launch_columns_v(spai_handle* h, const ColArgs& a, hipStream_t s) {
    size_t sh = sizeof(Smem<C, INC>) * C::PPW;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [&] {
        attr_err = hipFuncSetAttribute((const void*)k_spai_columns<C, INC>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
    });
    SPAI_HIP(attr_err);
    int grid = (a.ncols + C::PPW - 1) / C::PPW;
    long tk = timer_begin(h, SPAI_KT_COLUMNS);
    hipLaunchKernelGGL((k_spai_columns<C, INC>), dim3(grid), dim3(64), sh, s, a);
    timer_end(h, SPAI_KT_COLUMNS, tk);
    SPAI_HIP(hipGetLastError());
    return SPAI_OK;
}

template <class C>
static int launch_columns(spai_handle* h, const ColArgs& a, hipStream_t s) {
    if (a.ncols <= 0) return SPAI_OK;
    return a.qr_update ? launch_columns_v<C, true>(h, a, s) : launch_columns_v<C, false>(h, a, s);
}

// configurations: lanes per problem G (|J| <= G-1), shadow rows, gathered entries,
// raw candidates; the last one is the large-problem kernel for deferred columns
template <int UF> using CfgS = Cfg<UF, 8, 32, 64, 256>;
template <int UF> using CfgM = Cfg<UF, 16, 64, 128, 256>;
// (the two 21-lane ones store A-bar packed: 640 and 896 elements hold all but a
// fraction of a percent of the columns of their workloads, and bring the
// workgroups per CU from 10 to 12 and from 7 to 9)
template <int UF> using CfgM21s = Cfg<UF, 21, 40, 128, 256, 640>;   // small shadows: more problems per CU
template <int UF> using CfgM21 = Cfg<UF, 21, 64, 128, 256, 896>;
template <int UF> using CfgL = Cfg<UF, 32, 64, 256, 512>;
template <int UF> using CfgX = Cfg<UF, 64, (UF == SPAI_FP64 ? 128 : 256), 1024, 2048>;
// intermediate stage for the columns a configuration of at most 21 lanes defers
// (shadows of up to 96 rows, twice the gathered entries and candidates): they
// run 12 to a CU instead of the large-problem kernel's one
template <int UF> using CfgW = Cfg<UF, 21, 96, 256, 512>;
// A-bar in registers (FP32 arithmetic; with u_f = FP64 these are the LDS shapes):
// the 21-lane shapes, and a 32-lane one with half the candidate space of CfgL
// (a fixed pattern needs none; more candidates are deferred)
template <int UF> using CfgM21sR = Cfg<UF, 21, 40, 128, 256, 21 * 41, true>;
template <int UF> using CfgM21R = Cfg<UF, 21, 64, 128, 256, 21 * 65, true>;
template <int UF> using CfgLR = Cfg<UF, 32, 64, 256, 256, 32 * 65, true>;

// configuration ids of the C ABI (spai_column_config_get, spai_build_params.kernel_cfg)
enum { KC_S = 1, KC_M = 2, KC_M21S = 3, KC_M21 = 4, KC_L = 5, KC_X = 6, KC_M21SR = 7, KC_M21R = 8, KC_LR = 9 };
static_assert(KC_LR == SPAI_KCFG_COUNT, "configuration table and the C ABI disagree");

static int cfg_maxp(int id) {
    switch (id) {
    case KC_S: return CfgS<SPAI_FP32>::MAXP;
    case KC_M: return CfgM<SPAI_FP32>::MAXP;
    case KC_M21S: return CfgM21s<SPAI_FP32>::MAXP;
    case KC_M21: return CfgM21<SPAI_FP32>::MAXP;
    case KC_L: return CfgL<SPAI_FP32>::MAXP;
    case KC_M21SR: return CfgM21sR<SPAI_FP32>::MAXP;
    case KC_M21R: return CfgM21R<SPAI_FP32>::MAXP;
    case KC_LR: return CfgLR<SPAI_FP32>::MAXP;
    default: return CfgX<SPAI_FP32>::MAXP;
    }
}

template <class C>
static void cfg_describe(spai_column_config* o) {
    o->lanes = C::G;
    o->maxp = C::MAXP;
    o->maxm = C::MAXM;
    o->emax = C::EMAX;
    o->cmax = C::CMAX;
    o->problems_per_wave = C::PPW;
    o->lds_bytes_per_problem = (int32_t)sizeof(Smem<C, false>);
}

template <int UF>
static int launch_cfg(spai_handle* h, int id, const ColArgs& a, hipStream_t s) {
    switch (id) {
    case KC_S: return launch_columns<CfgS<UF>>(h, a, s);
    case KC_M: return launch_columns<CfgM<UF>>(h, a, s);
    case KC_M21S: return launch_columns<CfgM21s<UF>>(h, a, s);
    case KC_M21: return launch_columns<CfgM21<UF>>(h, a, s);
    case KC_L: return launch_columns<CfgL<UF>>(h, a, s);
    case KC_M21SR: return launch_columns<CfgM21sR<UF>>(h, a, s);
    case KC_M21R: return launch_columns<CfgM21R<UF>>(h, a, s);
    case KC_LR: return launch_columns<CfgLR<UF>>(h, a, s);
    default: return launch_columns<CfgX<UF>>(h, a, s);
    }
}

// columns whose flags hold `mask`, in any order (list may be NULL: count only)
__global__ void k_flag_list(int n, const int* __restrict__ flags, int mask, int* __restrict__ list,
                            int* __restrict__ count) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !(flags[k] & mask)) return;
    const int at = atomicAdd(count, 1);
    if (list) list[at] = k;
}

__global__ void k_mark_list(int count, const int* __restrict__ list, int bit, int* __restrict__ flags) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) flags[list[t]] |= bit;
}

__global__ void k_strided_list(int count, int stride, int* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = i * stride;
}

// For |J| <= 20: the small-shadow configuration when a strided sample of at
// most 2048 columns defers no more than 2% of its columns to the large-problem
// kernel, else the standard one.  A deferred column is recomputed from scratch
// by the next configuration with the same arithmetic, so the choice changes
// the time, not the result.
template <int UF>
static int launch_columns_m21(spai_handle* h, const ColArgs& a, hipStream_t s, int* sample_list,
                              int* count_host) {
    // the small-shadow shape with A-bar in registers when the arithmetic is FP32
    using Small = std::conditional_t<UF == SPAI_FP64, CfgM21s<UF>, CfgM21sR<UF>>;
    if (a.cols != nullptr || a.ncols < 4096) return launch_columns<CfgM21<UF>>(h, a, s);
    const int ns = 2048, stride = a.ncols / ns;
    hipLaunchKernelGGL(k_strided_list, dim3((ns + 255) / 256), dim3(256), 0, s, ns, stride, sample_list);
    SPAI_HIP(hipGetLastError());
    ColArgs smp = a;
    smp.cols = sample_list;
    smp.ncols = ns;
    SPAI_HIP(hipMemsetAsync(a.defer_count, 0, sizeof(int), s));
    int rc = launch_columns<Small>(h, smp, s);
    if (rc) return rc;
    SPAI_HIP(hipMemcpyAsync(count_host, a.defer_count, sizeof(int), hipMemcpyDeviceToHost, s));
    SPAI_HIP(hipStreamSynchronize(s));
    const bool small = *count_host * 50 <= ns;
    SPAI_HIP(hipMemsetAsync(a.defer_count, 0, sizeof(int), s));
    return small ? launch_columns<Small>(h, a, s) : launch_columns<CfgM21<UF>>(h, a, s);
}

// The column phase: the configuration kcfg (0 = the rule below), then the
// columns it deferred: through the intermediate 21-lane stage when the
// configuration has at most 21 lanes, and what is left on the largest one.
template <int UF>
static int run_columns(spai_handle* h, int pmax, int kcfg, ColArgs a, hipStream_t s, int* defer_list2,
                       int* defer_count_dev, int* defer_count_host, int* cols_deferred) {
    int rc;
    int* dc = a.defer_count;
    int id = kcfg;
    if (id == 0) {
        // the smallest configuration holding pmax indices
        id = pmax <= cfg_maxp(KC_S) ? KC_S : pmax <= cfg_maxp(KC_M) ? KC_M : pmax <= cfg_maxp(KC_M21) ? KC_M21
           : pmax <= cfg_maxp(KC_L) ? KC_L : KC_X;
        // with FP32 arithmetic the 32-lane shape keeps A-bar in registers: three
        // times faster on a fixed 27-point pattern (its smaller candidate space
        // defers more adaptive columns, which the large-problem kernel takes)
        if (UF != SPAI_FP64 && id == KC_L) id = KC_LR;
    }
    if (kcfg == 0 && id == KC_M21) rc = launch_columns_m21<UF>(h, a, s, defer_list2, defer_count_host);
    else rc = launch_cfg<UF>(h, id, a, s);
    if (rc) return rc;
    SPAI_HIP(hipMemcpyAsync(defer_count_host, dc, sizeof(int), hipMemcpyDeviceToHost, s));
    SPAI_HIP(hipStreamSynchronize(s));
    int nd = *defer_count_host;
    *cols_deferred = id == KC_X ? 0 : nd;
    if (nd > 0 && id == KC_X) {
        set_error("a column problem exceeds the largest kernel configuration");
        return SPAI_E_ARG;
    }
    if (nd > 0 && cfg_maxp(id) <= CfgW<UF>::MAXP) {
        // the intermediate stage: reads the first list, defers into the second
        ColArgs b = a;
        b.cols = a.defer_list;
        b.ncols = nd;
        b.defer_list = defer_list2;
        b.defer_count = defer_count_dev;
        SPAI_HIP(hipMemsetAsync(defer_count_dev, 0, sizeof(int), s));
        rc = launch_columns<CfgW<UF>>(h, b, s);
        if (rc) return rc;
        SPAI_HIP(hipMemcpyAsync(defer_count_host, defer_count_dev, sizeof(int), hipMemcpyDeviceToHost, s));
        SPAI_HIP(hipStreamSynchronize(s));
        nd = *defer_count_host;
        if (nd > 0) {
            // the large-problem kernel on the second list (the first one is read by now)
            b.cols = defer_list2;
            b.ncols = nd;
            b.defer_list = a.defer_list;
            b.defer_count = dc;
            SPAI_HIP(hipMemsetAsync(dc, 0, sizeof(int), s));
            rc = launch_columns<CfgX<UF>>(h, b, s);
            if (rc) return rc;
            SPAI_HIP(hipMemcpyAsync(defer_count_host, dc, sizeof(int), hipMemcpyDeviceToHost, s));
            SPAI_HIP(hipStreamSynchronize(s));
            if (*defer_count_host > 0) {
                set_error("a column problem exceeds the largest kernel configuration");
                return SPAI_E_ARG;
            }
        }
    } else if (nd > 0) {
        ColArgs b = a;
        b.cols = a.defer_list;
        b.ncols = nd;
        b.defer_list = defer_list2;
        b.defer_count = defer_count_dev;
        SPAI_HIP(hipMemsetAsync(defer_count_dev, 0, sizeof(int), s));
        rc = launch_columns<CfgX<UF>>(h, b, s);
        if (rc) return rc;
        SPAI_HIP(hipMemcpyAsync(defer_count_host, defer_count_dev, sizeof(int), hipMemcpyDeviceToHost, s));
        SPAI_HIP(hipStreamSynchronize(s));
        if (*defer_count_host > 0) {
            set_error("a column problem exceeds the largest kernel configuration");
            return SPAI_E_ARG;
        }
    }
    return SPAI_OK;
}

// Autotuning measurement: every configuration that holds pmax, with and
// without the QR update, over the columns in `sample` (ns of them), deferred
// columns included; the fastest of `reps` timed runs after an untimed one.
template <int UF>
static int tune_columns(spai_handle* h, int pmax, const ColArgs& a, hipStream_t s, int* sample, int ns,
                        int* defer_list2, int* defer_count_dev, int* defer_count_host, int reps, double* out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SPAI_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error("hipEventCreate failed");
        return SPAI_E_HIP;
    }
    int rc = SPAI_OK;
    for (int id = 1; id <= SPAI_KCFG_COUNT && rc == SPAI_OK; ++id) {
        for (int inc = 0; inc < 2 && rc == SPAI_OK; ++inc) {
            out[2 * (id - 1) + inc] = -1.0;
            if (cfg_maxp(id) < pmax) continue;
            ColArgs b = a;
            b.cols = sample;
            b.ncols = ns;
            b.qr_update = inc;
            float best = -1.0f;
            for (int r = 0; r <= reps && rc == SPAI_OK; ++r) {
                int nd = 0;
                if (hipMemsetAsync(a.defer_count, 0, sizeof(int), s) != hipSuccess ||
                    hipEventRecord(e0, s) != hipSuccess) {
                    rc = SPAI_E_HIP;
                    break;
                }
                if ((rc = run_columns<UF>(h, pmax, id, b, s, defer_list2, defer_count_dev, defer_count_host,
                                          &nd)))
                    break;
                float ms = 0.0f;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = SPAI_E_HIP;
                    break;
                }
                if (r > 0 && (best < 0.0f || ms < best)) best = ms;
            }
            if (rc == SPAI_OK) out[2 * (id - 1) + inc] = (double)best * 1e6 / ns;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SPAI_E_HIP) set_error("a HIP call failed while timing the column configurations");
    return rc;
}

static int blocks_red(int n) { return std::max(1, (n + RED_BLOCK - 1) / RED_BLOCK); }

static int scan_ints(int n, const int* in, int* out, int* tmp_blocks, int* total, hipStream_t s) {
    int nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(SCAN_BLOCK), 0, s, n, in, out, tmp_blocks);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(SCAN_BLOCK), 0, s, nb, tmp_blocks, total);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(SCAN_BLOCK), 0, s, n, out, tmp_blocks, total);
    SPAI_HIP(hipGetLastError());
    return SPAI_OK;
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

static void precond_free(spai_precond* P) {
    if (!P) return;
    void* ptrs[] = {P->rowptr, P->col, P->val, P->d, P->j_ins, P->m_ins, P->len, P->steps, P->res, P->flags};
    for (void* q : ptrs) dev_free(q, P->from);
    delete P;
}

template <typename T>
static int dev_alloc(spai_handle* h, T** p, size_t count) {
    return dev_malloc(h, (void**)p, sizeof(T) * (count ? count : 1));
}

// a new preconditioner whose arrays come from the handle's allocator
static spai_precond* precond_new(spai_handle* h) {
    spai_precond* P = new spai_precond();
    P->from = h->arena;
    return P;
}

static size_t val_size(spai_prec v) {
    switch (v) {
    case SPAI_FP64: return 8;
    case SPAI_FP32: return 4;
    default: return 2;
    }
}

// ---------------------------------------------------------------------------
// CSR transpose (for the right preconditioner): entries are counted per column,
// placed by per-column cursors and each output row is then sorted by column,
// so the result is the unique sorted CSR of the transpose.
// ---------------------------------------------------------------------------

__global__ void k_check_rows(int n, int nnz, const int* __restrict__ rp, const int* __restrict__ ci,
                             int* __restrict__ cnt, int* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = rp[i], e = rp[i + 1];
    if (a < 0 || e < a || e > nnz || (i == 0 && a != 0) || (i == n - 1 && e != nnz)) {
        atomicOr(bad, 1);
        return;
    }
    for (int q = a; q < e; ++q) {
        const int c = ci[q];
        if (c < 0 || c >= n) atomicOr(bad, 1);
        else atomicAdd(&cnt[c], 1);
    }
}

template <typename T>
__global__ void k_scatter_t(int n, const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ v,
                            int* __restrict__ cursor, int* __restrict__ oc, T* __restrict__ ov) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int q = rp[i]; q < rp[i + 1]; ++q) {
        const int pos = atomicAdd(&cursor[ci[q]], 1);
        oc[pos] = i;
        ov[pos] = v[q];
    }
}

template <typename T>
__global__ void k_sort_rows(int n, const int* __restrict__ ptr, int* __restrict__ c, T* __restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a0 = ptr[i], e = ptr[i + 1];
    for (int a = a0 + 1; a < e; ++a) {
        const int key = c[a];
        const T val = v[a];
        int b = a - 1;
        while (b >= a0 && c[b] > key) {
            c[b + 1] = c[b];
            v[b + 1] = v[b];
            --b;
        }
        c[b + 1] = key;
        v[b + 1] = val;
    }
}

// (orp, oci, ov) = transpose of the n x n CSR (rp, ci, v); SPAI_E_ARG for a
// malformed input (checked on the device before anything is placed).
template <typename T>
static int csr_transpose(spai_handle* h, int n, int nnz, const int* rp, const int* ci, const T* v, int* orp,
                         int* oci, T* ov) {
    hipStream_t s = h->stream;
    const int nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK + 1;
    int* tmp = nullptr;
    int rc = dev_alloc(h, &tmp, 2 * (size_t)n + nb + 64);
    if (rc) return rc;
    int* cnt = tmp;
    int* cur = cnt + n + 1;
    int* blk = cur + n;
    int* tot = blk + nb;
    int* bad = tot + 8;
    const int g = (n + 255) / 256;
    auto done = [&](int code) {
        (void)hipStreamSynchronize(s);
        dev_free(tmp, h->arena);
        return code;
    };
    if (hipMemsetAsync(cnt, 0, 4 * ((size_t)n + 1), s) != hipSuccess || hipMemsetAsync(bad, 0, 4, s) != hipSuccess)
        return done(SPAI_E_HIP);
    hipLaunchKernelGGL(k_check_rows, dim3(g), dim3(256), 0, s, n, nnz, rp, ci, cnt, bad);
    int hbad = 0;
    if (hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return done(SPAI_E_HIP);
    if (hbad) {
        set_error("invalid argument: malformed CSR (row pointers or column indices out of range)");
        return done(SPAI_E_ARG);
    }
    if ((rc = scan_ints(n, cnt, orp, blk, tot, s))) return done(rc);
    if (hipMemcpyAsync(cur, orp, 4 * (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess) return done(SPAI_E_HIP);
    hipLaunchKernelGGL((k_scatter_t<T>), dim3(g), dim3(256), 0, s, n, rp, ci, v, cur, oci, ov);
    hipLaunchKernelGGL((k_sort_rows<T>), dim3(g), dim3(256), 0, s, n, (const int*)orp, oci, ov);
    if (hipGetLastError() != hipSuccess) return done(SPAI_E_HIP);
    return done(SPAI_OK);
}

// a tuning run of the build (spai_tune_build): measure, produce no preconditioner
struct TuneReq {
    int sample, reps;
    double* ns_per_col;
};

static int build_right(spai_handle* h, const spai_csr* A, const spai_pattern* J, const spai_build_params* p,
                       spai_precond** P_out, spai_build_stats* st, const TuneReq* tq);

static int build_core(spai_handle* h, const spai_csr* A, const spai_pattern* J, const spai_build_params* p,
                      spai_precond** P_out, spai_build_stats* st, const TuneReq* tq) {
    SPAI_ARG(h && A && p && P_out, "NULL handle, matrix, parameters or output");
    *P_out = nullptr;
    SPAI_ARG(p->side == SPAI_LEFT || p->side == SPAI_RIGHT, "side must be SPAI_LEFT or SPAI_RIGHT");
    SPAI_ARG(tq || p->qr_update == 0 || p->qr_update == 1, "qr_update must be 0 or 1");
    SPAI_ARG(tq || (p->kernel_cfg >= 0 && p->kernel_cfg <= SPAI_KCFG_COUNT),
             "kernel_cfg must lie in 0..SPAI_KCFG_COUNT");
    const int n = A->n;
    SPAI_ARG(n > 0, "n must be positive");
    SPAI_ARG(A->nnz >= n && A->rowptr && A->col && A->val, "matrix arrays missing or nnz < n");
    SPAI_ARG(p->eps > 0.0, "eps must be positive");
    SPAI_ARG(p->alpha >= 0 && p->beta >= 0, "alpha and beta must be non-negative");
    SPAI_ARG(p->maxfill >= 1 && p->maxfill <= 63, "maxfill must lie in 1..63");
    SPAI_ARG(p->u_f == SPAI_FP64 || p->u_f == SPAI_FP32 || p->u_f == SPAI_FP16 || p->u_f == SPAI_BF16,
             "u_f must be FP64, FP32, FP16 or BF16");
    if (J) {
        SPAI_ARG(J->n == n && J->ptr && J->idx && J->nnz >= n, "pattern does not match the matrix");
    }
    if (p->side == SPAI_RIGHT) return build_right(h, A, J, p, P_out, st, tq);
    hipStream_t s = h->stream;
    SPAI_HIP(hipSetDevice(h->device));
    const int nnz = A->nnz;
    const size_t fsz = (p->u_f == SPAI_FP64) ? 8 : 4;

    // workspace: d, bnrm2, col counts, cursor, CSC rows and values, scan blocks, defer lists, stats
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
    const int nb = (n + SCAN_BLOCK - 1) / SCAN_BLOCK + 1;
    size_t o_bn = take(fsz * n), o_cnt = take(4 * (size_t)n + 4), o_cp = take(4 * ((size_t)n + 1)),
           o_cur = take(4 * (size_t)n), o_ri = take(4 * (size_t)nnz), o_bcv = take(fsz * (size_t)nnz),
           o_blk = take(4 * (size_t)nb),
           o_tot = take(16), o_dl = take(4 * (size_t)n), o_dl2 = take(4 * (size_t)n),
           o_dc = take(16), o_prep = take(sizeof(PrepOut)), o_bst = take(sizeof(BuildStatsDev)),
           o_nI = take(4 * (size_t)n), o_sl = take(tq ? 4 * (size_t)n : 0);
    int rc = buffer_reserve(h, h->ws[WS_BUILD0], off);
    if (rc) return rc;
    char* base = (char*)h->ws[WS_BUILD0].ptr;
    void* bn = base + o_bn;
    int* cnt = (int*)(base + o_cnt);
    int* cp = (int*)(base + o_cp);
    int* cur = (int*)(base + o_cur);
    int* ri = (int*)(base + o_ri);
    void* bcv = base + o_bcv;
    int* blk = (int*)(base + o_blk);
    int* tot = (int*)(base + o_tot);
    int* dl = (int*)(base + o_dl);
    int* dl2 = (int*)(base + o_dl2);
    int* dc = (int*)(base + o_dc);
    PrepOut* prep = (PrepOut*)(base + o_prep);
    BuildStatsDev* bst = (BuildStatsDev*)(base + o_bst);
    int* nI = (int*)(base + o_nI);
    int* sl = (int*)(base + o_sl);
    char* hp = (char*)h->host_pinned.ptr;

    spai_precond* P = precond_new(h);
    P->n = n;
    P->val_prec = p->u_f;
    P->u_f = p->u_f;
    auto fail = [&](int code) { precond_free(P); return code; };

    SPAI_HIP(hipMemsetAsync(cnt, 0, 4 * (size_t)n + 4, s));
    SPAI_HIP(hipMemsetAsync(prep, 0, sizeof(PrepOut), s));
    SPAI_HIP(hipMemsetAsync(dc, 0, 16, s));
    SPAI_HIP(hipMemsetAsync(bst, 0, sizeof(BuildStatsDev), s));
    if ((rc = dev_alloc(h, &P->d, n))) return fail(rc);
    const int tb = 256, gb = (n + tb - 1) / tb;
    const int rgb = std::min(blocks_red(n), 4 * std::max(h->num_cu, 1));
    hipLaunchKernelGGL(k_validate_scale, dim3(rgb), dim3(RED_BLOCK), 0, s, n, nnz, A->rowptr, A->col, A->val,
                       P->d, cnt, prep);
    hipLaunchKernelGGL(k_max_count, dim3(rgb), dim3(RED_BLOCK), 0, s, n, cnt, prep);
    if (J)
        hipLaunchKernelGGL(k_validate_pattern, dim3(gb), dim3(tb), 0, s, n, J->nnz, J->ptr, J->idx, prep);
    SPAI_HIP(hipGetLastError());
    SPAI_HIP(hipMemcpyAsync(hp, prep, sizeof(PrepOut), hipMemcpyDeviceToHost, s));
    SPAI_HIP(hipStreamSynchronize(s));
    PrepOut ph;
    std::memcpy(&ph, hp, sizeof(PrepOut));
    if (ph.err) {
        std::string why;
        if (ph.err & 1) why += " rowptr not monotone/consistent with nnz;";
        if (ph.err & 2) why += " column index out of range or columns not strictly ascending;";
        if (ph.err & 4) why += " non-finite value;";
        if (ph.err & 8) why += " a row holds no nonzero value;";
        if (ph.err & 16) why += " pattern malformed (range, duplicates or pointers);";
        set_error("invalid argument:" + why);
        return fail(SPAI_E_ARG);
    }
    const int pinit = J ? ph.max_pat : 1;
    if (pinit > 63) {
        set_error("invalid argument: an initial pattern column holds more than 63 indices");
        return fail(SPAI_E_ARG);
    }
    const int pmax = std::max(p->maxfill, pinit);
    if (!tq && p->kernel_cfg > 0 && cfg_maxp(p->kernel_cfg) < pmax) {
        set_error("invalid argument: kernel_cfg " + std::to_string(p->kernel_cfg) + " holds at most " +
                  std::to_string(cfg_maxp(p->kernel_cfg)) + " indices per column, the build needs " +
                  std::to_string(pmax));
        return fail(SPAI_E_ARG);
    }
    const int stride = pmax;
    P->stride = stride;

    // CSC structure of A (rows of B) and ||B(:, j)||^2
    if ((rc = scan_ints(n, cnt, cp, blk, tot, s))) return fail(rc);
    SPAI_HIP(hipMemcpyAsync(cur, cp, 4 * (size_t)n, hipMemcpyDeviceToDevice, s));
#define SPAI_PREP(UF, T)                                                                                         \
    hipLaunchKernelGGL(k_fill_csc<UF>, dim3(gb), dim3(tb), 0, s, n, A->rowptr, A->col, A->val, P->d, cur, ri,     \
                       (T*)bcv);                                                                                 \
    hipLaunchKernelGGL(k_colnorm<UF>, dim3(gb), dim3(tb), 0, s, n, A->rowptr, A->val, P->d, (T*)bn)
    switch (p->u_f) {
    case SPAI_FP64: SPAI_PREP(SPAI_FP64, double); break;
    case SPAI_FP32: SPAI_PREP(SPAI_FP32, float); break;
    case SPAI_FP16: SPAI_PREP(SPAI_FP16, float); break;
    default: SPAI_PREP(SPAI_BF16, float); break;
    }
#undef SPAI_PREP
    SPAI_HIP(hipGetLastError());

    // per-column outputs
    if ((rc = dev_alloc(h, &P->j_ins, (size_t)n * stride))) return fail(rc);
    if ((rc = dev_alloc(h, &P->m_ins, (size_t)n * stride))) return fail(rc);
    if ((rc = dev_alloc(h, &P->len, n))) return fail(rc);
    if ((rc = dev_alloc(h, &P->steps, n))) return fail(rc);
    if ((rc = dev_alloc(h, &P->res, n))) return fail(rc);
    if ((rc = dev_alloc(h, &P->flags, n))) return fail(rc);

    ColArgs a{};
    a.n = n; a.rp = A->rowptr; a.ci = A->col; a.av = A->val; a.cp = cp; a.ri = ri; a.d = P->d;
    a.bnrm2 = bn;
    a.bcv = bcv;
    a.pat_ptr = J ? J->ptr : nullptr;
    a.pat_idx = J ? J->idx : nullptr;
    a.eps = p->eps; a.alpha = p->alpha; a.beta = p->beta; a.maxfill = p->maxfill;
    a.qr_update = p->qr_update;
    a.cols = nullptr; a.ncols = n; a.stride = stride;
    a.len = P->len; a.jout = P->j_ins; a.mout = P->m_ins; a.steps = P->steps; a.res = P->res;
    a.flags = P->flags; a.nI = nI; a.defer_list = dl; a.defer_count = dc;
    int cols_deferred = 0;
    int* hcount = (int*)(hp + 256);
    if (tq) {
        // strided sample k * floor(n / ns), k < ns
        const int ns = std::min(tq->sample, n);
        hipLaunchKernelGGL(k_strided_list, dim3((ns + 255) / 256), dim3(256), 0, s, ns, n / ns, sl);
        SPAI_HIP(hipGetLastError());
#define SPAI_TUNE(UF) tune_columns<UF>(h, pmax, a, s, sl, ns, dl2, dc + 1, hcount, tq->reps, tq->ns_per_col)
        switch (p->u_f) {
        case SPAI_FP64: rc = SPAI_TUNE(SPAI_FP64); break;
        case SPAI_FP32: rc = SPAI_TUNE(SPAI_FP32); break;
        case SPAI_FP16: rc = SPAI_TUNE(SPAI_FP16); break;
        default: rc = SPAI_TUNE(SPAI_BF16); break;
        }
#undef SPAI_TUNE
        SPAI_HIP(hipStreamSynchronize(s));
        return fail(rc);
    }
    const int kc = p->kernel_cfg;
    switch (p->u_f) {
    case SPAI_FP64: rc = run_columns<SPAI_FP64>(h, pmax, kc, a, s, dl2, dc + 1, hcount, &cols_deferred); break;
    case SPAI_FP32: rc = run_columns<SPAI_FP32>(h, pmax, kc, a, s, dl2, dc + 1, hcount, &cols_deferred); break;
    case SPAI_FP16: rc = run_columns<SPAI_FP16>(h, pmax, kc, a, s, dl2, dc + 1, hcount, &cols_deferred); break;
    default: rc = run_columns<SPAI_BF16>(h, pmax, kc, a, s, dl2, dc + 1, hcount, &cols_deferred); break;
    }
    if (rc) return fail(rc);

    // Overflow of the 16-bit formats: a column with a non-finite value is
    // recomputed from its initial pattern in FP32 (norms of B from the FP32
    // rounding of its entries), marked, and P's values are then stored in FP32.
    bool promoted = false;
    if (p->u_f == SPAI_FP16 || p->u_f == SPAI_BF16) {
        int* fcount = dc + 2;
        SPAI_HIP(hipMemsetAsync(fcount, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_flag_list, dim3(gb), dim3(tb), 0, s, n, (const int*)P->flags, CF_NONFINITE,
                           (int*)nullptr, fcount);
        SPAI_HIP(hipGetLastError());
        SPAI_HIP(hipMemcpyAsync(hcount, fcount, sizeof(int), hipMemcpyDeviceToHost, s));
        SPAI_HIP(hipStreamSynchronize(s));
        const int nf = *hcount;
        if (nf > 0) {
            int* flist = nullptr;
            float* bn32 = nullptr;
            float* bcv32 = nullptr;
            int *ri32 = nullptr, *cur32 = nullptr;
            auto drop = [&]() {
                (void)hipStreamSynchronize(s);
                dev_free(flist, h->arena);
                dev_free(bn32, h->arena);
                dev_free(bcv32, h->arena);
                dev_free(ri32, h->arena);
                dev_free(cur32, h->arena);
            };
            if ((rc = dev_alloc(h, &flist, nf)) || (rc = dev_alloc(h, &bn32, n)) ||
                (rc = dev_alloc(h, &bcv32, (size_t)nnz)) || (rc = dev_alloc(h, &ri32, (size_t)nnz)) ||
                (rc = dev_alloc(h, &cur32, (size_t)n))) {
                drop();
                return fail(rc);
            }
            SPAI_HIP(hipMemsetAsync(fcount, 0, sizeof(int), s));
            hipLaunchKernelGGL(k_flag_list, dim3(gb), dim3(tb), 0, s, n, (const int*)P->flags, CF_NONFINITE, flist,
                               fcount);
            hipLaunchKernelGGL(k_colnorm<SPAI_FP32>, dim3(gb), dim3(tb), 0, s, n, A->rowptr, A->val, P->d, bn32);
            SPAI_HIP(hipMemcpyAsync(cur32, cp, 4 * (size_t)n, hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_fill_csc<SPAI_FP32>, dim3(gb), dim3(tb), 0, s, n, A->rowptr, A->col, A->val, P->d,
                               cur32, ri32, bcv32);
            SPAI_HIP(hipGetLastError());
            ColArgs f = a;
            f.bnrm2 = bn32;
            f.ri = ri32;
            f.bcv = bcv32;
            f.cols = flist;
            f.ncols = nf;
            SPAI_HIP(hipMemsetAsync(dc, 0, 2 * sizeof(int), s));
            int nd_fb = 0;
            rc = run_columns<SPAI_FP32>(h, pmax, 0, f, s, dl2, dc + 1, hcount, &nd_fb);
            if (rc == SPAI_OK) {
                hipLaunchKernelGGL(k_mark_list, dim3((nf + 255) / 256), dim3(256), 0, s, nf, (const int*)flist,
                                   CF_FALLBACK, P->flags);
                if (hipGetLastError() != hipSuccess) rc = SPAI_E_HIP;
            }
            drop();
            if (rc) return fail(rc);
            promoted = true;
        }
    }
    const spai_prec vstore = promoted ? SPAI_FP32 : p->u_f;
    P->val_prec = vstore;

    // compaction into CSR(P)
    if ((rc = dev_alloc(h, &P->rowptr, (size_t)n + 1))) return fail(rc);
    if ((rc = scan_ints(n, P->len, P->rowptr, blk, tot, s))) return fail(rc);
    hipLaunchKernelGGL(k_build_stats, dim3(rgb), dim3(RED_BLOCK), 0, s, n, stride, P->len, P->steps, P->res,
                       P->flags, nI, (const double*)P->m_ins, bst);
    SPAI_HIP(hipMemcpyAsync(hp, tot, sizeof(int), hipMemcpyDeviceToHost, s));
    SPAI_HIP(hipMemcpyAsync(hp + 64, bst, sizeof(BuildStatsDev), hipMemcpyDeviceToHost, s));
    SPAI_HIP(hipStreamSynchronize(s));
    int total = *(int*)hp;
    BuildStatsDev bs;
    std::memcpy(&bs, hp + 64, sizeof(bs));
    P->nnz = total;
    if ((rc = dev_alloc(h, &P->col, (size_t)total))) return fail(rc);
    {
        void* v = nullptr;
        if ((rc = dev_malloc(h, &v, val_size(vstore) * (size_t)std::max(total, 1)))) return fail(rc);
        P->val = v;
    }
    long long work = (long long)n * stride;
    int cg = (int)((work + 255) / 256);
    switch (vstore) {
    case SPAI_FP64: hipLaunchKernelGGL(k_compact<SPAI_FP64>, dim3(cg), dim3(256), 0, s, n, stride, P->len, P->j_ins, P->m_ins, P->rowptr, P->col, (double*)P->val); break;
    case SPAI_FP32: hipLaunchKernelGGL(k_compact<SPAI_FP32>, dim3(cg), dim3(256), 0, s, n, stride, P->len, P->j_ins, P->m_ins, P->rowptr, P->col, (float*)P->val); break;
    case SPAI_FP16: hipLaunchKernelGGL(k_compact<SPAI_FP16>, dim3(cg), dim3(256), 0, s, n, stride, P->len, P->j_ins, P->m_ins, P->rowptr, P->col, (__half*)P->val); break;
    default: hipLaunchKernelGGL(k_compact<SPAI_BF16>, dim3(cg), dim3(256), 0, s, n, stride, P->len, P->j_ins, P->m_ins, P->rowptr, P->col, (__hip_bfloat16*)P->val); break;
    }
    SPAI_HIP(hipGetLastError());
    SPAI_HIP(hipStreamSynchronize(s));

    int warn = 0;
    if (bs.over_eps) warn |= SPAI_W_EPS;
    if (bs.rankdef) warn |= SPAI_W_RANKDEF;
    if (bs.nonfinite) warn |= SPAI_W_NONFINITE;
    if (st) {
        st->nnz = total;
        st->max_len = bs.max_len;
        st->max_steps = bs.max_steps;
        st->max_shadow = bs.max_shadow;
        st->cols_over_eps = bs.over_eps;
        st->cols_rankdef = bs.rankdef;
        st->cols_nonfinite = bs.nonfinite;
        st->cols_deferred = cols_deferred;
        double mr;
        std::memcpy(&mr, &bs.max_res_bits, sizeof(double));
        st->max_res = mr;
        st->nnz_numeric = (int64_t)bs.nnz_numeric;
        st->cols_fallback = bs.fallback;
        st->pad = 0;
    }
    *P_out = P;
    return warn;
}

int build_impl(spai_handle* h, const spai_csr* A, const spai_pattern* J, const spai_build_params* p,
               spai_precond** P_out, spai_build_stats* st) {
    return build_core(h, A, J, p, P_out, st, nullptr);
}

// The right preconditioner: the left build of A^T gives rows m_k with
// A D m_k ~ e_k (D from the rows of A^T, i.e. the columns of A); P = D M is the
// transpose of that CSR with D applied to the output.
static int build_right(spai_handle* h, const spai_csr* A, const spai_pattern* J, const spai_build_params* p,
                       spai_precond** P_out, spai_build_stats* st, const TuneReq* tq) {
    const int n = A->n, nnz = A->nnz;
    SPAI_ARG(n > 0 && nnz >= n && A->rowptr && A->col && A->val, "matrix arrays missing or nnz < n");
    SPAI_HIP(hipSetDevice(h->device));
    int *trp = nullptr, *tci = nullptr;
    double* tv = nullptr;
    int rc;
    auto free_t = [&]() {
        (void)hipStreamSynchronize(h->stream);
        dev_free(trp, h->arena);
        dev_free(tci, h->arena);
        dev_free(tv, h->arena);
    };
    if ((rc = dev_alloc(h, &trp, (size_t)n + 1)) || (rc = dev_alloc(h, &tci, (size_t)nnz)) ||
        (rc = dev_alloc(h, &tv, (size_t)nnz))) {
        free_t();
        return rc;
    }
    if ((rc = csr_transpose<double>(h, n, nnz, A->rowptr, A->col, A->val, trp, tci, tv))) {
        free_t();
        return rc;
    }
    spai_csr At{n, nnz, trp, tci, tv};
    spai_build_params pl = *p;
    pl.side = SPAI_LEFT;
    spai_precond* P = nullptr;
    const int warn = build_core(h, &At, J, &pl, &P, st, tq);
    free_t();
    if (warn < 0 || tq) return warn;
    // transpose the rows m_k into rows i of P = D M
    int *prp = nullptr, *pci = nullptr;
    void* pv = nullptr;
    const int pnz = (int)P->nnz;
    auto fail = [&](int code) {
        (void)hipStreamSynchronize(h->stream);
        dev_free(prp, h->arena);
        dev_free(pci, h->arena);
        dev_free(pv, h->arena);
        precond_free(P);
        return code;
    };
    if ((rc = dev_alloc(h, &prp, (size_t)n + 1)) || (rc = dev_alloc(h, &pci, (size_t)pnz)) ||
        (rc = dev_malloc(h, &pv, val_size(P->val_prec) * (size_t)std::max(pnz, 1))))
        return fail(rc);
    switch (P->val_prec) {
    case SPAI_FP64: rc = csr_transpose<double>(h, n, pnz, P->rowptr, P->col, (const double*)P->val, prp, pci, (double*)pv); break;
    case SPAI_FP32: rc = csr_transpose<float>(h, n, pnz, P->rowptr, P->col, (const float*)P->val, prp, pci, (float*)pv); break;
    default: rc = csr_transpose<uint16_t>(h, n, pnz, P->rowptr, P->col, (const uint16_t*)P->val, prp, pci, (uint16_t*)pv); break;
    }
    if (rc) return fail(rc);
    SPAI_HIP(hipStreamSynchronize(h->stream));
    dev_free(P->rowptr, P->from);
    dev_free(P->col, P->from);
    dev_free(P->val, P->from);
    P->rowptr = prp;
    P->col = pci;
    P->val = pv;
    P->side = SPAI_RIGHT;
    *P_out = P;
    return warn;
}

int precond_import_impl(spai_handle* h, int32_t n, int64_t nnz, const int32_t* rowptr,
                        const int32_t* col, const double* val, spai_prec vp, const double* d,
                        spai_precond** P_out);

}  // namespace spai

// ---------------------------------------------------------------------------
// C ABI: build and preconditioner objects
// ---------------------------------------------------------------------------

template <int VP>
__global__ void k_convert_vals(long long nnz, const double* __restrict__ in, typename spai::ValType<VP>::T* out) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnz) return;
    double v = in[t];
    if constexpr (VP == SPAI_FP64) out[t] = v;
    else if constexpr (VP == SPAI_FP32) out[t] = (float)v;
    else if constexpr (VP == SPAI_FP16) out[t] = __float2half_rn((float)v);
    else out[t] = typename spai::ValType<VP>::T((float)v);
}

int spai::precond_import_impl(spai_handle* h, int32_t n, int64_t nnz, const int32_t* rowptr,
                              const int32_t* col, const double* val, spai_prec vp, const double* d,
                              spai_precond** P_out) {
    SPAI_ARG(h && P_out && rowptr && col && val && d, "NULL argument");
    SPAI_ARG(n > 0 && nnz >= 0 && nnz < (1ll << 31), "bad sizes");
    SPAI_ARG(vp == SPAI_FP64 || vp == SPAI_FP32 || vp == SPAI_FP16 || vp == SPAI_BF16, "bad value format");
    *P_out = nullptr;
    SPAI_HIP(hipSetDevice(h->device));
    hipStream_t s = h->stream;
    spai_precond* P = precond_new(h);
    P->n = n;
    P->nnz = nnz;
    P->val_prec = vp;
    P->u_f = vp;
    auto fail = [&](int code) { precond_free(P); return code; };
    int rc;
    if ((rc = dev_alloc(h, &P->rowptr, (size_t)n + 1))) return fail(rc);
    if ((rc = dev_alloc(h, &P->col, (size_t)nnz))) return fail(rc);
    if ((rc = dev_alloc(h, &P->d, (size_t)n))) return fail(rc);
    {
        void* v = nullptr;
        if ((rc = dev_malloc(h, &v, val_size(vp) * (size_t)std::max<int64_t>(nnz, 1)))) return fail(rc);
        P->val = v;
    }
    SPAI_HIP(hipMemcpyAsync(P->rowptr, rowptr, 4 * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
    SPAI_HIP(hipMemcpyAsync(P->col, col, 4 * (size_t)nnz, hipMemcpyDeviceToDevice, s));
    SPAI_HIP(hipMemcpyAsync(P->d, d, 8 * (size_t)n, hipMemcpyDeviceToDevice, s));
    int g = (int)((nnz + 255) / 256);
    if (g < 1) g = 1;
    switch (vp) {
    case SPAI_FP64: hipLaunchKernelGGL(k_convert_vals<SPAI_FP64>, dim3(g), dim3(256), 0, s, (long long)nnz, val, (double*)P->val); break;
    case SPAI_FP32: hipLaunchKernelGGL(k_convert_vals<SPAI_FP32>, dim3(g), dim3(256), 0, s, (long long)nnz, val, (float*)P->val); break;
    case SPAI_FP16: hipLaunchKernelGGL(k_convert_vals<SPAI_FP16>, dim3(g), dim3(256), 0, s, (long long)nnz, val, (__half*)P->val); break;
    default: hipLaunchKernelGGL(k_convert_vals<SPAI_BF16>, dim3(g), dim3(256), 0, s, (long long)nnz, val, (__hip_bfloat16*)P->val); break;
    }
    SPAI_HIP(hipGetLastError());
    SPAI_HIP(hipStreamSynchronize(s));
    *P_out = P;
    return SPAI_OK;
}

extern "C" int spai_build(spai_handle* h, const spai_csr* A, const spai_pattern* J,
                          const spai_build_params* p, spai_precond** P, spai_build_stats* st) {
    return spai::build_impl(h, A, J, p, P, st);
}

extern "C" int spai_tune_build(spai_handle* h, const spai_csr* A, const spai_pattern* J, const spai_build_params* p,
                               int32_t sample, int32_t reps, double* ns_per_col) {
    if (sample < 1 || reps < 1 || !ns_per_col) {
        spai::set_error("invalid argument: sample and reps must be positive and ns_per_col non-NULL");
        return SPAI_E_ARG;
    }
    spai::TuneReq tq{sample, reps, ns_per_col};
    spai_precond* P = nullptr;
    return spai::build_core(h, A, J, p, &P, nullptr, &tq);
}

extern "C" int spai_column_config_get(int32_t id, spai_column_config* out) {
    if (!out || id < 1 || id > SPAI_KCFG_COUNT) {
        spai::set_error("invalid argument: configuration id outside 1..SPAI_KCFG_COUNT or NULL output");
        return SPAI_E_ARG;
    }
    switch (id) {
    case spai::KC_S: spai::cfg_describe<spai::CfgS<SPAI_FP32>>(out); break;
    case spai::KC_M: spai::cfg_describe<spai::CfgM<SPAI_FP32>>(out); break;
    case spai::KC_M21S: spai::cfg_describe<spai::CfgM21s<SPAI_FP32>>(out); break;
    case spai::KC_M21: spai::cfg_describe<spai::CfgM21<SPAI_FP32>>(out); break;
    case spai::KC_L: spai::cfg_describe<spai::CfgL<SPAI_FP32>>(out); break;
    case spai::KC_M21SR: spai::cfg_describe<spai::CfgM21sR<SPAI_FP32>>(out); break;
    case spai::KC_M21R: spai::cfg_describe<spai::CfgM21R<SPAI_FP32>>(out); break;
    case spai::KC_LR: spai::cfg_describe<spai::CfgLR<SPAI_FP32>>(out); break;
    default: spai::cfg_describe<spai::CfgX<SPAI_FP32>>(out); break;
    }
    return SPAI_OK;
}

extern "C" int spai_precond_import(spai_handle* h, int32_t n, int64_t nnz, const int32_t* rowptr,
                                   const int32_t* col, const double* val, spai_prec val_prec,
                                   const double* d, spai_precond** P) {
    return spai::precond_import_impl(h, n, nnz, rowptr, col, val, val_prec, d, P);
}

extern "C" int spai_precond_view_get(const spai_precond* P, spai_precond_view* v) {
    if (!P || !v) {
        spai::set_error("invalid argument: NULL preconditioner or view");
        return SPAI_E_ARG;
    }
    v->n = P->n;
    v->nnz = P->nnz;
    v->rowptr = P->rowptr;
    v->col = P->col;
    v->val = P->val;
    v->val_prec = P->val_prec;
    v->d = P->d;
    v->stride = P->stride;
    v->j_ins = P->j_ins;
    v->m_ins = P->m_ins;
    v->len = P->len;
    v->steps = P->steps;
    v->res = P->res;
    v->flags = P->flags;
    v->side = P->side;
    v->u_f = P->u_f;
    return SPAI_OK;
}

extern "C" int spai_precond_destroy(spai_precond* P) {
    spai::precond_free(P);
    return SPAI_OK;
}
