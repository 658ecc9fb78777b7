// SPAI-GMRES-IR on gfx950 (Algorithm 3, Section 3.2): x0 = P b in u_f, then per
// refinement step the residual in double-double (u_r), left-preconditioned
// MGS-GMRES in FP64 (u_g = u_p = u, Section 4) and the FP64 update.
//
// Kernels are HBM-bound streaming passes over CSR(A), CSR(P) and the Krylov
// basis V (column-major, n x (maxit+1) FP64).  Every reduction is deterministic:
// each thread sums a fixed set of elements, blocks reduce in a fixed tree, and
// the last block to finish (ticket counter) reduces the per-block partials in
// block order, so repeated runs give bit-identical results.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include <type_traits>

#include "common.hpp"
#include "device_math.hpp"

namespace spai {

constexpr int RB = 256;        // threads per reduction block
constexpr int RBLOCKS = 1024;  // upper bound on reduction blocks

// ---------------------------------------------------------------------------
// solver state shared by the kernels of one refinement step
// ---------------------------------------------------------------------------

struct SolveState {
    double beta0;   // ||P r_i||_2
    double gabs;    // |g_{j+1}| after the last Givens update
    int done;       // 0 running, 1 converged, 2 maxit reached, 3 device error
    int its;        // GMRES iterations of the step once done
    int err;        // 1: a grid-wide sum timed out
    int jcur;       // graph replay: index of the next Arnoldi step (advanced by its launch)
};

// ---------------------------------------------------------------------------
// sparse products (a set `done` flag turns them into no-ops so that steps
// enqueued past convergence cost only their launch; launched from the stream,
// they read the flag once their first loads are out, so that its latency
// overlaps theirs, and then write nothing)
// ---------------------------------------------------------------------------

// w = A v and y = M^T (D w) (row k of P holds m_k, values in VP, FP64
// arithmetic; for a right preconditioner row i holds the m_k[i] and y = D (M w))
// with G lanes per row (G a power of two <= 16).  The product may scale its
// output, w_i = d_i (A v)_i, so that the left application that follows gathers
// only w (the product d_k w_k is the one it would form itself: the same bits,
// one gather per entry instead of two).  The lanes load the
// row's entries with unit stride, keep lane-strided partial sums and add them
// by a fixed xor tree, so every call gives the same bits.  Many more waves than
// one thread per row, and coalesced loads.

// IT: entries per lane of a row whose loads are issued together (1 or 2: the
// lanes per row are chosen so that an average row takes at most 1.5 rounds;
// for a large matrix with short rows, one lane per row and IT = 4..8, a whole
// average row in flight: spmv_shape)
template <int G, int R, int IT>
__global__ __launch_bounds__(256) void k_spmv_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                const double* __restrict__ av, const double* __restrict__ x,
                                                double* __restrict__ y, const double* __restrict__ dout,
                                                const SolveState* __restrict__ st, int by_step) {
    if (by_step) {                           // graph replay: x is column jcur of the basis
        if (st->done) return;
        x += (size_t)st->jcur * n;
    }
    // a block covers R slabs of 256 / G consecutive rows: each slab is read by the whole block at once
    constexpr int GPB = 256 / G;
    const int sub = threadIdx.x & (G - 1);
    const int row0 = (int)blockIdx.x * GPB * R + (int)threadIdx.x / G;
    if (row0 >= n) return;                   // the whole group of G lanes
    // R rows per group: their row pointers, entries and gathers are all in flight together
    int q0[R], q1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = min(row0 + r * GPB, n - 1);
        q0[r] = rp[row] + sub;
        q1[r] = row0 + r * GPB < n ? rp[row + 1] : 0;
    }
    // the first IT entries of every row's lane are loaded before any is used
    // (the index loads, then the value loads and gathers; a position past the
    // row's end loads entry 0, which exists since nnz >= 1, and is not added),
    // the rest of a longer row follows in a loop; each lane sums its entries in
    // ascending order
    double acc[R];
    {
        int qx[R][IT], jx[R][IT];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int q = q0[r] + it * G;
                qx[r][it] = q < q1[r] ? q : 0;
                jx[r][it] = ci[qx[r][it]];
            }
        double va[R][IT], vx[R][IT];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                va[r][it] = av[qx[r][it]];
                vx[r][it] = x[jx[r][it]];
            }
        __asm__ volatile("" ::: "memory");   // the loads above stay ahead of the flag's test
        if (!by_step && st && st->done) return;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const double f = __builtin_fma(va[r][it], vx[r][it], s);
                s = q0[r] + it * G < q1[r] ? f : s;
            }
            acc[r] = s;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double s = acc[r];
        for (int q = q0[r] + IT * G; q < q1[r]; q += G) s = __builtin_fma(av[q], x[ci[q]], s);
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
        if (sub == 0 && row0 + r * GPB < n) y[row0 + r * GPB] = dout ? dout[row0 + r * GPB] * s : s;
    }
}

// SCALED (left only): w already holds D w, the gather of d is skipped
template <int VP, int G, int R, bool RIGHT, bool SCALED, int IT>
__global__ __launch_bounds__(256) void k_apply_P_g(int n, const int* __restrict__ pp, const int* __restrict__ pc,
                                                   const typename ValType<VP>::T* __restrict__ pv,
                                                   const double* __restrict__ d, const double* __restrict__ w,
                                                   double* __restrict__ y, const SolveState* __restrict__ st,
                                                   int by_step) {
    if (by_step) {                           // graph replay: w is column jcur of the basis
        if (st->done) return;
        w += (size_t)st->jcur * n;
    }
    // a block covers R slabs of 256 / G consecutive rows: each slab is read by the whole block at once
    constexpr int GPB = 256 / G;
    const int sub = threadIdx.x & (G - 1);
    const int row0 = (int)blockIdx.x * GPB * R + (int)threadIdx.x / G;
    if (row0 >= n) return;
    int q0[R], q1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int row = min(row0 + r * GPB, n - 1);
        q0[r] = pp[row] + sub;
        q1[r] = row0 + r * GPB < n ? pp[row + 1] : 0;
    }
    // as in k_spmv_g: the first IT entries of every row's lane in flight
    // together (entry 0 standing in past the row's end, not added), the rest in
    // a loop, each lane's sum in ascending order
    double acc[R];
    {
        int qx[R][IT], jx[R][IT];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int q = q0[r] + it * G;
                qx[r][it] = q < q1[r] ? q : 0;
                jx[r][it] = pc[qx[r][it]];
            }
        double vp[R][IT], vw[R][IT];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int j = jx[r][it];
                vp[r][it] = to_f64(pv[qx[r][it]]);
                if constexpr (RIGHT || SCALED) vw[r][it] = w[j];
                else vw[r][it] = d[j] * w[j];
            }
        __asm__ volatile("" ::: "memory");   // the loads above stay ahead of the flag's test
        if (!by_step && st && st->done) return;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double s = 0.0;
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const double f = __builtin_fma(vp[r][it], vw[r][it], s);
                s = q0[r] + it * G < q1[r] ? f : s;
            }
            acc[r] = s;
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        double s = acc[r];
        for (int q = q0[r] + IT * G; q < q1[r]; q += G) {
            const int j = pc[q];
            if constexpr (RIGHT || SCALED) s = __builtin_fma(to_f64(pv[q]), w[j], s);
            else s = __builtin_fma(to_f64(pv[q]), d[j] * w[j], s);
        }
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
        if (sub == 0 && row0 + r * GPB < n) {
            if constexpr (RIGHT) s = d[row0 + r * GPB] * s;   // P = D M: the scaling acts on the output
            y[row0 + r * GPB] = s;
        }
    }
}

// lanes per row for an average of nnz / n entries per row: up to 4 lanes, the
// fewest for which 1.5 entries per lane cover an average row; from 4 on, two
// entries per lane (more loads in flight per lane, fewer idle lanes: the 7-point
// product at 128^3 took 53 us with 4 lanes of two entries against 65 us with 8
// lanes of one)
static inline int lanes_per_row(long long nnz, int n) {
    const double avg = n > 0 ? (double)nnz / n : 0.0;
    int g = 1;
    while (g < 16 && g * (g >= 4 ? 2.0 : 1.5) < avg) g <<= 1;
    return g;
}

// x0 = P b in u_f: z_j = u_f(d_j b_j), products and sums in F, ascending column.
// VP is the storage format of P's values, UF the precision of the build (the
// two differ for a 16-bit build whose overflowing columns were recomputed in
// FP32: the values are then FP32, the rounding of the input stays 16-bit).
template <int VP, int UF, bool RIGHT>
__global__ void k_x0(int n, const int* __restrict__ pp, const int* __restrict__ pc,
                     const typename ValType<VP>::T* __restrict__ pv, const double* __restrict__ d,
                     const double* __restrict__ b, double* __restrict__ x0) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    // entry loops unrolled by 4 (loads in flight together, the same order)
    if constexpr (RIGHT) {
        // P = D M: b rounded to u_f, the row's sum in the arithmetic of u_f, times d_k rounded to u_f
        if constexpr (VP == SPAI_FP64) {
            double s = 0.0;
#pragma unroll 4
            for (int q = pp[k]; q < pp[k + 1]; ++q) s = __builtin_fma(pv[q], b[pc[q]], s);
            x0[k] = d[k] * s;
        } else {
            float s = 0.0f;
#pragma unroll 4
            for (int q = pp[k]; q < pp[k + 1]; ++q)
                s = __builtin_fmaf(to_f32(pv[q]), store<UF, float>((float)b[pc[q]]), s);
            x0[k] = (double)(store<UF, float>((float)d[k]) * s);
        }
    } else if constexpr (VP == SPAI_FP64) {
        double s = 0.0;
#pragma unroll 4
        for (int q = pp[k]; q < pp[k + 1]; ++q) {
            int j = pc[q];
            s = __builtin_fma(pv[q], d[j] * b[j], s);
        }
        x0[k] = s;
    } else {
        float s = 0.0f;
#pragma unroll 4
        for (int q = pp[k]; q < pp[k + 1]; ++q) {
            int j = pc[q];
            float z = store<UF, float>((float)(d[j] * b[j]));
            s = __builtin_fmaf(to_f32(pv[q]), z, s);
        }
        x0[k] = (double)s;
    }
}

// Maxima behind the error measures of Theorems 1 and 2 for the returned x:
// out[0..5] = max |r_i|, max_i sum_j |a_ij|, max |x_i|, max |b_i|,
// max |x_i - xt_i|, max |xt_i| (xt may be NULL).  Non-negative doubles order
// as their bit patterns, so the maxima are taken on the bits (any order, same
// result); out must be zero on entry.
__global__ void k_err_norms(int n, const int* __restrict__ rp, const double* __restrict__ av,
                            const double* __restrict__ r, const double* __restrict__ x,
                            const double* __restrict__ b, const double* __restrict__ xt,
                            unsigned long long* __restrict__ out) {
    double m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        m[0] = fmax(m[0], fabs(r[i]));
        double rs = 0.0;
        for (int q = rp[i]; q < rp[i + 1]; ++q) rs += fabs(av[q]);
        m[1] = fmax(m[1], rs);
        m[2] = fmax(m[2], fabs(x[i]));
        m[3] = fmax(m[3], fabs(b[i]));
        if (xt) {
            m[4] = fmax(m[4], fabs(x[i] - xt[i]));
            m[5] = fmax(m[5], fabs(xt[i]));
        }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        double v = m[q];
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
        if ((threadIdx.x & 63) == 0 && v > 0.0) atomicMax(out + q, (unsigned long long)__double_as_longlong(v));
    }
}

// r = b - A x: products split exactly with an FMA and accumulated in
// double-double, rounded once to FP64 at the end (u_r = DD); or plain FP64
template <bool DD>
__global__ void k_residual(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ av, const double* __restrict__ b,
                           const double* __restrict__ x, double* __restrict__ r) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // entry loops unrolled by 4: four entries' loads in flight, the same order
    if constexpr (DD) {
        double sh = b[i], sl = 0.0;
#pragma unroll 4
        for (int q = rp[i]; q < rp[i + 1]; ++q) {
            double a = av[q], xv = x[ci[q]];
            double ph = a * xv;
            double pl = __builtin_fma(a, xv, -ph);
            dd_add(sh, sl, -ph, -pl, sh, sl);
        }
        r[i] = sh + sl;
    } else {
        double s = b[i];
#pragma unroll 4
        for (int q = rp[i]; q < rp[i + 1]; ++q) s = __builtin_fma(-av[q], x[ci[q]], s);
        r[i] = s;
    }
}

// ---------------------------------------------------------------------------
// the Arnoldi step: one cooperative launch per step
//
// Modified Gram-Schmidt is a chain of j+2 dependent global sums per Arnoldi
// step (h_lj = <y, v_l> with y already reduced by v_0 .. v_{l-1}, then ||y||),
// so its cost is the latency of a grid-wide sum.  The launch keeps y in
// registers (EPT elements per thread), streams each basis vector once and
// prefetches the next one while the sum is in flight.  A grid-wide sum: every
// block publishes its partial into its own write-once slot of the link (an
// agent-scope atomic store of the 64-bit value; slots start as a signalling-NaN
// sentinel no arithmetic produces), wave 0 of every block polls all slots with
// agent-scope atomic loads and adds them in slot order, so every block obtains
// the bit-identical sum.  Slots alternate between two buffers from one launch
// to the next; each launch re-arms the other buffer.  Polls are bounded: a
// timeout aborts every block and is reported through SolveState::err.
// Block 0 then applies the Givens rotations to column j of H (in LDS), updates
// g and sets `done` when |g_{j+1}| <= tau beta0, on an exact breakdown or at
// maxit.
// ---------------------------------------------------------------------------

// Load p[i] where ok, else 0, with an unconditional load of a valid address
// (p[0] is always valid): the loads of a group then stay in one basic block.
__device__ __forceinline__ double ld0(const double* __restrict__ p, size_t i, bool ok) {
    const double v = p[ok ? i : 0];
    return ok ? v : 0.0;
}

// Index for a prefetch: i where ok, else 0 (a valid address).  The raw value is
// kept and masked only where it is used, so that no wait is placed between the
// prefetch and the work it overlaps.
__device__ __forceinline__ size_t pf_index(size_t i, bool ok) { return ok ? i : 0; }

constexpr int AT_DATA = 512;          // threads that hold y and stream the basis (8 waves)
constexpr int AT = AT_DATA + 64;      // plus one wave that only publishes and polls
constexpr int MAX_NB = 256;           // blocks of the Arnoldi kernel (4 slots per poll lane)
constexpr unsigned long long SENTINEL = 0x7ff4dead5eed0001ull;
constexpr long long SPIN_LIMIT = 1ll << 20;   // about a second of polling

struct ArnoldiArgs {
    int n, j, ld, maxit, maxlinks, nb, parity;
    const double* y;     // P A v_j
    double* V;           // basis, column-major n x (maxit + 1)
    double* H;           // ld x maxit
    double* cs;
    double* sn;
    double* g;
    double tau;
    unsigned long long* slots;   // grid-sum slots and mailboxes of both parities
    SolveState* st;
    double* HRp;         // DCGS2: first projections, column-major ld x maxit
    double* HRf;         // DCGS2: completed Hessenberg columns before rotation, row-major (maxit+1) x maxit
    int by_step;         // DCGS2 graph replay: j = st->jcur (parity j & 1), advanced by block 0
    // pipelined DCGS2 with the step's second operator product fused in: y = M mx
    // at the launch's rows, M in CSR (mrp, mcol, and mval of the value type the
    // launch is built for); y above is then neither read nor written
    const int* mrp;
    const int* mcol;
    const void* mval;
    const double* mx;
};

// Grid-wide sum of one double per block, in two hops that keep every polled
// word lightly shared: the poll wave of each block (the last wave, which has no
// other memory traffic, so its loads never queue behind the basis prefetch)
// publishes the block's partial into its write-once slot of the link; the
// reducer block (the last block) loads all nb slots (four independent loads per
// lane, repeated until none is the sentinel), adds them in a fixed order and
// writes the total into one mailbox per block (each on its own 64-byte line);
// every block then polls only its own mailbox.  All blocks obtain the
// bit-identical total.  Returns the total to every thread of the block.
constexpr int MBOX_STRIDE = 8;   // 64-bit words between mailboxes (one cache line)

__device__ __forceinline__ bool poll_word(unsigned long long* p, unsigned long long& v) {
    long long spins = 0;
    while ((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == SENTINEL) {
        if (++spins > SPIN_LIMIT) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

__device__ __forceinline__ double grid_sum(double part, unsigned long long* slot_row, unsigned long long* mbox,
                                           size_t mbox_stride, int nb, double* wsum, double* total, int* abort_flag) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int DW = AT_DATA / 64;
    if (wave < DW) {
        part = wave_sum(part);
        if (lane == 0) wsum[wave] = part;
    }
    __syncthreads();
    if (wave == DW) {
        if (lane == 0) {
            double s = 0.0;
            for (int w = 0; w < DW; ++w) s += wsum[w];
            __hip_atomic_store(&slot_row[blockIdx.x], (unsigned long long)__double_as_longlong(s),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        bool timeout = false;
        if ((int)blockIdx.x == nb - 1) {        // the reducer
            unsigned long long v[MAX_NB / 64];
            bool ready[MAX_NB / 64];
#pragma unroll
            for (int k = 0; k < MAX_NB / 64; ++k) {
                ready[k] = (lane + 64 * k) >= nb;
                v[k] = 0ull;
            }
            long long spins = 0;
            while (true) {
#pragma unroll
                for (int k = 0; k < MAX_NB / 64; ++k)
                    if (!ready[k])
                        v[k] = __hip_atomic_load(&slot_row[lane + 64 * k], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
                bool all = true;
#pragma unroll
                for (int k = 0; k < MAX_NB / 64; ++k) {
                    if (!ready[k]) ready[k] = (v[k] != SENTINEL);
                    all = all && ready[k];
                }
                if (all) break;
                if (++spins > SPIN_LIMIT) {
                    timeout = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            double val = 0.0;
#pragma unroll
            for (int k = 0; k < MAX_NB / 64; ++k)
                if (lane + 64 * k < nb) val += __longlong_as_double((long long)v[k]);
            val = wave_sum(val);
            const unsigned long long bits = timeout ? 0x7ff8000000000000ull : (unsigned long long)__double_as_longlong(val);
#pragma unroll
            for (int k = 0; k < MAX_NB / 64; ++k) {
                int q = lane + 64 * k;
                if (q < nb) __hip_atomic_store(&mbox[(size_t)q * mbox_stride], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (lane == 0) *total = val;
        } else if (lane == 0) {
            unsigned long long v = 0ull;
            if (poll_word(&mbox[(size_t)blockIdx.x * mbox_stride], v)) *total = __longlong_as_double((long long)v);
            else timeout = true;
        }
        uint64_t bad = ballot(timeout);
        if (lane == 0 && bad) *abort_flag = 1;
    }
    __syncthreads();
    return *total;
}

// Apply the Givens rotations 0..m-1 in order to the column hh[0..m]; the
// running entry is carried in a register (same operations as rotating hh in
// place, without a round trip through memory per rotation).
// The operands of 8 rotations are loaded together, so that one LDS latency is
// paid per 8 rotations instead of one per rotation.
__device__ __forceinline__ void apply_rotations(double* hh, int m, const double* csL, const double* snL) {
    if (m <= 0) return;
    double x0 = hh[0];
    for (int l0 = 0; l0 < m; l0 += 8) {
        double x1[8], c[8], s[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int l = min(l0 + k, m - 1);
            x1[k] = hh[l + 1];
            c[k] = csL[l];
            s[k] = snL[l];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (l0 + k < m) {
                hh[l0 + k] = c[k] * x0 + s[k] * x1[k];
                x0 = -s[k] * x0 + c[k] * x1[k];
            }
        }
    }
    hh[m] = x0;
}

// The same rotations applied by the 64 lanes of one wave: lane L owns a
// segment of at most ROT_SEG consecutive rotations; the carried entry obeys the
// affine recurrence x_{l+1} = -s_l x_l + c_l h_{l+1}, whose maps are composed
// over the lanes by an inclusive scan (Kogge-Stone, fixed order), so every lane
// obtains its incoming carry in 6 steps instead of waiting for the whole chain.
// The rounding differs from the sequential order only in how the carry is
// associated.  hh must be visible to the whole wave; on return the rotated
// entries are.
constexpr int ROT_SEG = 8;

__device__ __forceinline__ void wave_rotate(double* hh, int m, const double* csL, const double* snL) {
    const int lane = threadIdx.x & 63;
    if (m <= 0) return;
    if (m > 64 * ROT_SEG) {
        if (lane == 0) apply_rotations(hh, m, csL, snL);
        wave_sync();
        return;
    }
    const int seg = (m + 63) / 64;
    const int lo = min(lane * seg, m), hi = min(lo + seg, m);
    double cv[ROT_SEG], sv[ROT_SEG], xv[ROT_SEG];
    double A = 1.0, B = 0.0;
#pragma unroll
    for (int k = 0; k < ROT_SEG; ++k) {
        cv[k] = 1.0;
        sv[k] = 0.0;
        xv[k] = 0.0;
        if (lo + k < hi) {
            cv[k] = csL[lo + k];
            sv[k] = snL[lo + k];
            xv[k] = hh[lo + k + 1];
            A = -sv[k] * A;
            B = -sv[k] * B + cv[k] * xv[k];
        }
    }
    for (int d = 1; d < 64; d <<= 1) {       // maps of the lanes before come first
        const double Ap = __shfl_up(A, d, 64), Bp = __shfl_up(B, d, 64);
        if (lane >= d) {
            B = A * Bp + B;
            A = A * Ap;
        }
    }
    const double x00 = hh[0];
    const double Ae = __shfl_up(A, 1, 64), Be = __shfl_up(B, 1, 64);
    double x0 = lane == 0 ? x00 : Ae * x00 + Be;
    wave_sync();                              // every read of hh before any write
#pragma unroll
    for (int k = 0; k < ROT_SEG; ++k) {
        if (lo + k < hi) {
            hh[lo + k] = cv[k] * x0 + sv[k] * xv[k];
            x0 = -sv[k] * x0 + cv[k] * xv[k];
        }
    }
    if (lo < hi && hi == m) hh[m] = x0;
    wave_sync();
}

// One wave completes column c of the Hessenberg matrix: hh[0..c+1] holds it
// before rotation (visible to the wave).  Applies rotations 0..c-1, builds
// rotation c, updates g, writes the rotated column into H and takes the
// stopping decision (|g_{c+1}| <= tau beta0 or a zero subdiagonal: converged;
// c + 1 = maxit: iteration cap).
__device__ __forceinline__ void wave_givens_column(const ArnoldiArgs& a, double* hh, int c, const double* csL,
                                                   const double* snL) {
    const int lane = threadIdx.x & 63;
    wave_rotate(hh, c, csL, snL);
    if (lane == 0) {
        const double hs = hh[c + 1];
        const double delta = hypot(hh[c], hs);
        const double cc = hh[c] / delta, sv = hs / delta;
        hh[c] = delta;
        hh[c + 1] = 0.0;
        const double gc = a.g[c];
        a.g[c + 1] = -sv * gc;
        a.g[c] = cc * gc;
        a.cs[c] = cc;
        a.sn[c] = sv;
        const double ga = fabs(-sv * gc);
        a.st->gabs = ga;
        if (ga <= a.tau * a.st->beta0 || hs == 0.0) {
            a.st->its = c + 1;
            a.st->done = 1;
        } else if (c + 1 == a.maxit) {
            a.st->its = c + 1;
            a.st->done = 2;
        }
    }
    wave_sync();
    double* Hc = a.H + (size_t)c * a.ld;
    for (int l = lane; l <= c + 1; l += 64) Hc[l] = hh[l];
}

template <int EPT>
__global__ __launch_bounds__(AT) void k_arnoldi(ArnoldiArgs a) {
    extern __shared__ double dyn[];          // block 0: hcol (maxit+2), cs, sn (maxit each)
    __shared__ double wsum[AT_DATA / 64];
    __shared__ double total;
    __shared__ int abort_flag;
    if (a.st->done) return;                  // uniform: written by an earlier launch
    const int b = blockIdx.x, t = threadIdx.x;
    const bool data = t < AT_DATA;
    const int gstride = a.nb * AT_DATA;
    const int base = b * AT_DATA + t;
    const int n = a.n, j = a.j;
    // slot buffer of one parity: [maxlinks][nb] partials, then [nb][maxlinks] mailboxes (one line each)
    const size_t per_parity = (size_t)a.maxlinks * a.nb * (1 + MBOX_STRIDE);
    unsigned long long* cur = a.slots + (size_t)a.parity * per_parity;
    unsigned long long* nxt = a.slots + (size_t)(1 - a.parity) * per_parity;
    unsigned long long* cur_mbox = cur + (size_t)a.maxlinks * a.nb;
    const size_t mstride = (size_t)a.maxlinks * MBOX_STRIDE;   // between the mailboxes of two blocks
    unsigned long long* nxt_mbox = nxt + (size_t)a.maxlinks * a.nb;
    // re-arm the other buffer for the next launch (links 0 .. j+3)
    const int lim = min(j + 4, a.maxlinks);
    for (int l = t; l < lim; l += AT) {
        nxt[(size_t)l * a.nb + b] = SENTINEL;
        nxt_mbox[((size_t)b * a.maxlinks + l) * MBOX_STRIDE] = SENTINEL;
    }
    double* hcol = dyn;
    double* csL = dyn + (a.maxit + 2);
    double* snL = csL + a.maxit;
    if (t == 0) abort_flag = 0;
    if (b == 0)
        for (int l = t; l < j; l += AT) {
            csL[l] = a.cs[l];
            snL[l] = a.sn[l];
        }
    double y[EPT], v[EPT], vn[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        int i = base + e * gstride;
        bool ok = data && i < n;
        y[e] = ld0(a.y, i, ok);
        v[e] = ld0(a.V, i, ok);
        vn[e] = 0.0;
    }
    __syncthreads();
    // h_lj = <y, v_l>; y -= h_lj v_l  (l = 0 .. j)
    for (int l = 0; l <= j; ++l) {
        if (l < j) {
            const double* vnext = a.V + (size_t)(l + 1) * n;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                int i = base + e * gstride;
                vn[e] = vnext[pf_index(i, data && i < n)];   // masked where used
            }
        }
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) part = __builtin_fma(y[e], v[e], part);
        double h = grid_sum(part, cur + (size_t)l * a.nb, cur_mbox + (size_t)l * MBOX_STRIDE, mstride, a.nb, wsum,
                            &total, &abort_flag);
        if (abort_flag) break;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            y[e] = __builtin_fma(-h, v[e], y[e]);
            v[e] = (data && base + e * gstride < n) ? vn[e] : 0.0;
        }
        if (b == 0 && t == 0) hcol[l] = h;
    }
    // h_{j+1,j} = ||y||; v_{j+1} = y / h_{j+1,j}
    double hn = 0.0;
    if (!abort_flag) {
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) part = __builtin_fma(y[e], y[e], part);
        hn = __builtin_sqrt(grid_sum(part, cur + (size_t)(j + 1) * a.nb, cur_mbox + (size_t)(j + 1) * MBOX_STRIDE,
                                    mstride, a.nb, wsum, &total, &abort_flag));
    }
    if (abort_flag) {
        if (t == 0) {
            a.st->err = 1;
            a.st->done = 3;
        }
        return;
    }
    double* vout = a.V + (size_t)(j + 1) * n;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        int i = base + e * gstride;
        if (data && i < n) vout[i] = y[e] / hn;
    }
    if (b == 0 && t < 64) {
        if (t == 0) hcol[j + 1] = hn;
        wave_sync();
        wave_givens_column(a, hcol, j, csL, snL);
    }
}

// ---------------------------------------------------------------------------
// CGS2 Arnoldi step: classical Gram-Schmidt applied twice
//   h1 = V^T y; y -= V h1; h2 = V^T y; y -= V h2; H(:, j) = h1 + h2; ||y||
// Three grid-wide reductions per step instead of j+2: bandwidth-bound (four
// streaming passes over the basis).  A vector reduction: every block publishes
// its partial vector into write-once slots [l][b]; the owner of column l (block
// l mod nb) adds the nb partials in a fixed order and writes the total into the
// private mailbox row of every block ([b][l], write-once); each block polls its
// own row.  All blocks obtain bit-identical totals.
// ---------------------------------------------------------------------------

// basis vectors in flight per thread: about 16 doubles of loads per thread, so
// that large EPT does not spill (the grouping does not change the arithmetic)
template <int EPT>
constexpr int cg_u() { return EPT >= 16 ? 1 : EPT >= 8 ? 2 : EPT >= 4 ? 4 : 8; }

// per-block partials pvec[l] = sum over the block's rows of V(i, l) y_i, l < L
template <int EPT>
__device__ __forceinline__ void block_vty(const double* __restrict__ V, int n, int L, const double (&y)[EPT],
                                          int base, int gstride, double* wpart, int ldw, double* pvec) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int DW = AT_DATA / 64;
    constexpr int CG_U = cg_u<EPT>();
    if (wave < DW) {
        for (int l0 = 0; l0 < L; l0 += CG_U) {
            double vv[CG_U][EPT];
#pragma unroll
            for (int u = 0; u < CG_U; ++u)
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    int i = base + e * gstride;
                    vv[u][e] = ld0(V + (size_t)min(l0 + u, L - 1) * n, i, l0 + u < L && i < n);
                }
#pragma unroll
            for (int u = 0; u < CG_U; ++u) {
                double p = 0.0;
#pragma unroll
                for (int e = 0; e < EPT; ++e) p = __builtin_fma(vv[u][e], y[e], p);
                p = wave_sum(p);
                if (lane == 0 && l0 + u < L) wpart[wave * ldw + l0 + u] = p;
            }
        }
    }
    __syncthreads();
    for (int l = t; l < L; l += AT) {
        double sacc = 0.0;
        for (int w = 0; w < DW; ++w) sacc += wpart[w * ldw + l];
        pvec[l] = sacc;
    }
    __syncthreads();
}

// y -= V h for the thread's rows, l ascending
template <int EPT>
__device__ __forceinline__ void y_minus_Vh(const double* __restrict__ V, int n, int L, double (&y)[EPT],
                                           const double* h, int base, int gstride) {
    if (threadIdx.x >= AT_DATA) return;
    constexpr int CG_U = cg_u<EPT>();
    for (int l0 = 0; l0 < L; l0 += CG_U) {
        double vv[CG_U][EPT];
#pragma unroll
        for (int u = 0; u < CG_U; ++u)
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                int i = base + e * gstride;
                vv[u][e] = ld0(V + (size_t)min(l0 + u, L - 1) * n, i, l0 + u < L && i < n);
            }
#pragma unroll
        for (int u = 0; u < CG_U; ++u) {
            if (l0 + u < L) {
                const double hl = h[l0 + u];
#pragma unroll
                for (int e = 0; e < EPT; ++e) y[e] = __builtin_fma(-hl, vv[u][e], y[e]);
            }
        }
    }
}

// all-reduce of the per-block vectors pvec (length L) into hout (every block)
__device__ __forceinline__ void grid_vsum(const double* pvec, int L, int nb, unsigned long long* slots,
                                          unsigned long long* mbox, int lmax, double* red, double* hout,
                                          int* abort_flag) {
    const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int l = t; l < L; l += AT)
        __hip_atomic_store(&slots[(size_t)l * nb + b], (unsigned long long)__double_as_longlong(pvec[l]),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();                          // pvec may share its storage with red
    const int owned = L > b ? (L - 1 - b) / nb + 1 : 0;
    bool to = false;
    for (int q = t; q < owned * nb; q += AT) {
        int k = q / nb, src = q - k * nb;
        unsigned long long v = 0ull;
        if (!poll_word(&slots[(size_t)(b + k * nb) * nb + src], v)) to = true;
        red[q] = __longlong_as_double((long long)v);
    }
    __syncthreads();
    for (int k = wave; k < owned; k += AT / 64) {
        double acc = 0.0;
        for (int src = lane; src < nb; src += 64) acc += red[k * nb + src];
        acc = wave_sum(acc);
        const int l = b + k * nb;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(acc);
        for (int q = lane; q < nb; q += 64)
            __hip_atomic_store(&mbox[(size_t)q * lmax + l], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    for (int l = t; l < L; l += AT) {
        unsigned long long v = 0ull;
        if (!poll_word(&mbox[(size_t)b * lmax + l], v)) to = true;
        hout[l] = __longlong_as_double((long long)v);
    }
    if (to) *abort_flag = 1;
    __syncthreads();
}

// slot words of one parity for the CGS2 kernel
__host__ __device__ inline size_t cgs2_parity_words(int maxlinks, int nb) {
    return (size_t)4 * maxlinks * nb + (size_t)nb * (1 + MBOX_STRIDE);
}

template <int EPT>
__global__ __launch_bounds__(AT) void k_arnoldi_cgs2(ArnoldiArgs a) {
    extern __shared__ double dyn[];
    __shared__ double wsum[AT_DATA / 64];
    __shared__ double total;
    __shared__ int abort_flag;
    if (a.st->done) return;                  // uniform: written by an earlier launch
    const int b = blockIdx.x, t = threadIdx.x, nb = a.nb;
    const bool data = t < AT_DATA;
    const int gstride = nb * AT_DATA;
    const int base = b * AT_DATA + t;
    const int n = a.n, j = a.j, L = j + 1, lmax = a.maxlinks;
    constexpr int DW = AT_DATA / 64;
    // LDS: wpart [DW][lmax], pvec, h1, h2 [lmax], red [lmax + nb], cs, sn [maxit]
    double* wpart = dyn;
    double* pvec = wpart + (size_t)DW * lmax;
    double* h1 = pvec + lmax;
    double* h2 = h1 + lmax;
    double* red = h2 + lmax;
    double* csL = red + lmax + nb;
    double* snL = csL + a.maxit;
    const size_t pw = cgs2_parity_words(lmax, nb);
    unsigned long long* cur = a.slots + (size_t)a.parity * pw;
    unsigned long long* nxt = a.slots + (size_t)(1 - a.parity) * pw;
    const size_t blk = (size_t)lmax * nb;    // one slot array or one mailbox array
    // re-arm this block's words of the other buffer for the next launch (L + 1 columns)
    for (int l = t; l < min(L + 1, lmax); l += AT) {
        nxt[0 * blk + (size_t)l * nb + b] = SENTINEL;
        nxt[1 * blk + (size_t)b * lmax + l] = SENTINEL;
        nxt[2 * blk + (size_t)l * nb + b] = SENTINEL;
        nxt[3 * blk + (size_t)b * lmax + l] = SENTINEL;
    }
    if (t == 0) {
        nxt[4 * blk + b] = SENTINEL;
        nxt[4 * blk + nb + (size_t)b * MBOX_STRIDE] = SENTINEL;
        abort_flag = 0;
    }
    if (b == 0)
        for (int l = t; l < j; l += AT) {
            csL[l] = a.cs[l];
            snL[l] = a.sn[l];
        }
    double y[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        int i = base + e * gstride;
        y[e] = ld0(a.y, i, data && i < n);
    }
    __syncthreads();
    block_vty<EPT>(a.V, n, L, y, base, gstride, wpart, lmax, pvec);
    grid_vsum(pvec, L, nb, cur, cur + blk, lmax, red, h1, &abort_flag);
    double hn = 0.0;
    if (!abort_flag) {
        y_minus_Vh<EPT>(a.V, n, L, y, h1, base, gstride);
        block_vty<EPT>(a.V, n, L, y, base, gstride, wpart, lmax, pvec);
        grid_vsum(pvec, L, nb, cur + 2 * blk, cur + 3 * blk, lmax, red, h2, &abort_flag);
    }
    if (!abort_flag) {
        y_minus_Vh<EPT>(a.V, n, L, y, h2, base, gstride);
        double part = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) part = __builtin_fma(y[e], y[e], part);
        hn = __builtin_sqrt(grid_sum(part, cur + 4 * blk, cur + 4 * blk + nb, MBOX_STRIDE, nb, wsum, &total,
                                     &abort_flag));
    }
    if (abort_flag) {
        if (t == 0) {
            a.st->err = 1;
            a.st->done = 3;
        }
        return;
    }
    double* vout = a.V + (size_t)(j + 1) * n;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        int i = base + e * gstride;
        if (data && i < n) vout[i] = y[e] / hn;
    }
    if (b == 0 && t < 64) {
        double* hh = pvec;                      // free now: column j of H
        for (int l = t; l < L; l += 64) hh[l] = h1[l] + h2[l];
        if (t == 0) hh[j + 1] = hn;
        wave_sync();
        wave_givens_column(a, hh, j, csL, snL);
    }
}

// ---------------------------------------------------------------------------
// DCGS2 Arnoldi step: CGS2 with the second projection and the normalisation of
// each new vector delayed by one step, so that a step needs one grid-wide
// reduction and two streaming passes over the basis.  Column j of V holds the
// lagged vector u_j (u_0 = v_0) and y = P A u_j.  Launch j
//   pass 1: block partials of [V_{j-1}^T u_j, u_j^T u_j, V_{j-1}^T y, u_j^T y]
//           (2j + 2 values: a, omega, b, c), all-reduced over the grid;
//   every block: nu = sqrt(omega - a^T a) (nu = 1 for j = 0) and
//           gj = (c - a^T b) / nu, in the same order, so identical everywhere;
//   pass 2: v_j = (u_j - V_{j-1} a) / nu into column j and
//           u_{j+1} = (y - V_{j-1} b - gj v_j) / nu into column j + 1 (skipped
//           by the launch j = maxit, which only completes column maxit - 1);
// while the poll wave of every block, idle during pass 2, completes its rows of
// the Hessenberg matrix: the column j - 1 entries f_r = HRp(r, j-1) + a_r
// (r < j), f_j = nu, and the first projection of M v_j,
//   HRp(r, j) = (gv_r - sum_{m <= j-2} HRf(r, m) a_m - f_r a_{j-1}) / nu,
// with gv = [b; gj] (rows r = b, b + nb, ...); the poll wave of block 0 applies
// the Givens rotations to column j - 1 and takes the stopping decision.
// ---------------------------------------------------------------------------

// LDS of the DCGS2 kernel, in doubles: the (u, y) staging [AT_DATA min(EPT, 8)] double2,
// the block partials / poll buffer [rmax + nb] (one after the other in time),
// the totals [rmax], the Hessenberg column [maxlinks], cs and sn [maxit]
__host__ __device__ constexpr size_t dcgs2_lds_words(int ept, int rmax, int nb, int maxlinks, int maxit) {
    return (size_t)2 * AT_DATA * (ept < 8 ? ept : 8) + (size_t)(rmax + nb) + rmax + maxlinks + 2 * (size_t)maxit;
}

// slot words of one parity for the DCGS2 kernel: [rmax][nb] slots + [nb][rmax] mailboxes
__host__ __device__ inline size_t dcgs2_parity_words(int maxlinks, int nb) {
    return (size_t)2 * (2 * (size_t)maxlinks) * nb;
}

// basis vectors per group in the double-buffered passes: 16 doubles per buffer
// and thread (32 loads in flight per thread with two buffers)
template <int EPT>
constexpr int cg_u2() { return EPT >= 16 ? 1 : 16 / EPT; }

// raw loads of basis vectors l0 .. l0+U-1 (< lim) at the thread's rows; entries
// outside (columns >= lim, rows >= n) are loaded from a valid address and must
// not be used
template <int EPT, int U>
__device__ __forceinline__ void load_cols(const double* __restrict__ V, int n, int l0, int lim, int base, int gstride,
                                          double (&vv)[U][EPT]) {
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            int i = base + e * gstride;
            vv[q][e] = V[(size_t)min(l0 + q, lim - 1) * n + pf_index(i, i < n)];
        }
}

// pass 1 with one wave per basis vector: wave w takes the vectors l = w,
// w + 8, ... over all rows of the block (8 rows per lane and 512-row chunk;
// (u_i, y_i) staged in LDS in the row order of the data threads), so that each
// block partial is reduced once per staged part, by one wave; three buffers of
// loads are in flight while one is used.  At most DCGS2_SE chunks are staged at
// a time (64 KB): with more (EPT = 16) the rows are covered in EPT / DCGS2_SE
// parts and the parts' totals are added.
constexpr int DCGS2_SE = 8;

template <int EPT>
__device__ __forceinline__ void block_dots_cols(const double* __restrict__ V, int n, int j, const double (&u)[EPT],
                                                const double (&yv)[EPT], int gstride, double2* uy, double* wsum2,
                                                double* pvec) {
    const int t = threadIdx.x, lane = t & 63, b = blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // uniform: scalar column bases
    constexpr int DW = AT_DATA / 64;
    constexpr int SE = EPT < DCGS2_SE ? EPT : DCGS2_SE;       // chunks staged per part
    constexpr int NPART = EPT / SE;
    // a load chunk = CE row blocks of 512 (8 CE rows per lane); NCH chunks per vector and part
    constexpr int CE = (EPT <= 2 || NPART > 1) ? 1 : 2;
    constexpr int NCH = SE / CE;
    // EPT <= 2: the lane's 8 EPT pairs (u_i, y_i) are held in registers for the
    // whole pass (LDS reads would cost a fifth of the pass)
    constexpr bool REG = EPT <= 2;
    if (wave < DW) {
        double om = 0.0, c = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            om = __builtin_fma(u[e], u[e], om);
            c = __builtin_fma(u[e], yv[e], c);
        }
        om = wave_sum(om);
        c = wave_sum(c);
        if (lane == 0) {
            wsum2[2 * wave] = om;
            wsum2[2 * wave + 1] = c;
        }
    }
    const int ncol = j > wave ? (j - 1 - wave) / DW + 1 : 0;
    const int total = ncol * NCH;
    // FULL: every 512-row chunk of the thread block lies inside 0 .. n-1 (the
    // loads take a scalar column base plus the lane's offset, no masks)
    const bool all_full = b * AT_DATA + (EPT - 1) * gstride + AT_DATA <= n;
#pragma unroll
    for (int part = 0; part < NPART; ++part) {
        if (wave < DW) {
#pragma unroll
            for (int e = 0; e < SE; ++e) uy[e * AT_DATA + t] = make_double2(u[part * SE + e], yv[part * SE + e]);
        }
        __syncthreads();
        if (wave < DW) {
            double ur[REG ? 8 * EPT : 1], yr[REG ? 8 * EPT : 1];
            if constexpr (REG) {
#pragma unroll
                for (int e = 0; e < EPT; ++e)
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const double2 q = uy[e * AT_DATA + lane + 64 * k];
                        ur[e * 8 + k] = q.x;
                        yr[e * 8 + k] = q.y;
                    }
            }
            auto run = [&](auto fullc) {
                constexpr bool FULL = decltype(fullc)::value;
                double p1 = 0.0, p2 = 0.0;
                auto load = [&](int it, double (&buf)[8 * CE]) {
                    const int l = wave + DW * (it / NCH), c = it % NCH;
                    const double* col = V + (size_t)l * n;
#pragma unroll
                    for (int ee = 0; ee < CE; ++ee) {
                        const int rb = b * AT_DATA + (part * SE + c * CE + ee) * gstride;   // uniform
                        if constexpr (FULL) {
                            const double* cb = col + rb;
#pragma unroll
                            for (int k = 0; k < 8; ++k) buf[ee * 8 + k] = cb[lane + 64 * k];
                        } else {
#pragma unroll
                            for (int k = 0; k < 8; ++k) {
                                const int r = rb + lane + 64 * k;
                                buf[ee * 8 + k] = col[pf_index((size_t)r, r < n)];
                            }
                        }
                    }
                };
                auto consume = [&](int it, const double (&buf)[8 * CE]) {
                    const int c = it % NCH;
#pragma unroll
                    for (int ee = 0; ee < CE; ++ee) {
                        const int e = c * CE + ee;                         // staged chunk
                        const int r0 = b * AT_DATA + (part * SE + e) * gstride + lane;
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            double qx, qy;
                            if constexpr (REG) {
                                qx = ur[e * 8 + k];
                                qy = yr[e * 8 + k];
                            } else {
                                const double2 q = uy[e * AT_DATA + lane + 64 * k];
                                qx = q.x;
                                qy = q.y;
                            }
                            const double vk = (FULL || r0 + 64 * k < n) ? buf[ee * 8 + k] : 0.0;
                            p1 = __builtin_fma(vk, qx, p1);
                            p2 = __builtin_fma(vk, qy, p2);
                        }
                    }
                    if (c == NCH - 1) {
                        const double t1 = wave_sum(p1), t2 = wave_sum(p2);
                        const int l = wave + DW * (it / NCH);
                        if (lane == 0) {
                            pvec[l] = part == 0 ? t1 : pvec[l] + t1;
                            pvec[j + 1 + l] = part == 0 ? t2 : pvec[j + 1 + l] + t2;
                        }
                        p1 = 0.0;
                        p2 = 0.0;
                    }
                };
                // three buffers in turn: the loads of chunks it + 1 and it + 2 are in
                // flight while chunk it is used (a chunk index past the end reloads
                // the last chunk, unused)
                double ba[8 * CE], bb[8 * CE], bc[8 * CE];
                if (total > 0) {
                    load(0, ba);
                    load(min(1, total - 1), bb);
                }
                for (int it = 0; it < total; it += 3) {
                    load(min(it + 2, total - 1), bc);
                    consume(it, ba);
                    if (it + 1 < total) {
                        load(min(it + 3, total - 1), ba);
                        consume(it + 1, bb);
                    }
                    if (it + 2 < total) {
                        load(min(it + 4, total - 1), bb);
                        consume(it + 2, bc);
                    }
                }
            };
            if (all_full)
                run(std::true_type{});
            else
                run(std::false_type{});
        }
        if (NPART > 1) __syncthreads();       // the next part overwrites the staging
    }
    __syncthreads();
    if (t == 0) {
        double om = 0.0, c = 0.0;
        for (int w = 0; w < DW; ++w) {
            om += wsum2[2 * w];
            c += wsum2[2 * w + 1];
        }
        pvec[j] = om;
        pvec[2 * j + 1] = c;
    }
    __syncthreads();
}

// pass 2 (data waves): u and yv are consumed in place; the basis vectors are
// taken in descending order
template <int EPT>
__device__ __forceinline__ void dcgs2_update(const double* __restrict__ V, int n, int j, double (&u)[EPT],
                                             double (&yv)[EPT], const double* acoef, const double* bcoef, double nu,
                                             double gj, int base, int gstride, double* vout, double* uout) {
    if (threadIdx.x >= AT_DATA) return;
    constexpr int CG_U = cg_u2<EPT>();
    // basis vectors in descending order: the most recently read ones (the end of
    // pass 1) come first, while they may still sit in the memory-side cache
    auto use = [&](int l0, const double (&vv)[CG_U][EPT]) {
#pragma unroll
        for (int q = CG_U - 1; q >= 0; --q) {
            if (l0 + q < j) {
                const double al = acoef[l0 + q], bl = bcoef[l0 + q];
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    u[e] = __builtin_fma(-al, vv[q][e], u[e]);
                    yv[e] = __builtin_fma(-bl, vv[q][e], yv[e]);
                }
            }
        }
    };
    // groups of CG_U vectors from the top down, two buffers in turn (a group
    // index below 0 reloads group 0, unused)
    double va[CG_U][EPT], vb[CG_U][EPT];
    const int top = j > 0 ? ((j - 1) / CG_U) * CG_U : 0;
    if (j > 0) load_cols<EPT, CG_U>(V, n, top, j, base, gstride, va);
    for (int l0 = top; l0 >= 0 && j > 0; l0 -= 2 * CG_U) {
        load_cols<EPT, CG_U>(V, n, max(l0 - CG_U, 0), j, base, gstride, vb);
        use(l0, va);
        if (l0 - CG_U >= 0) {
            load_cols<EPT, CG_U>(V, n, max(l0 - 2 * CG_U, 0), j, base, gstride, va);
            use(l0 - CG_U, vb);
        }
    }
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        int i = base + e * gstride;
        if (i < n) {
            double v = j > 0 ? u[e] / nu : u[e];
            if (j > 0) vout[i] = v;
            uout[i] = __builtin_fma(-gj, v, yv[e]) / nu;
        }
    }
}

// poll wave of every block: its rows of the Hessenberg matrix
__device__ __forceinline__ void dcgs2_rows(const ArnoldiArgs& a, const double* hv, double nu, double gj) {
    const int lane = threadIdx.x & 63, j = a.j, nb = a.nb, ld = a.ld, mx = a.maxit;
    for (int r = blockIdx.x; r <= j; r += nb) {
        double f = 0.0;                       // completed entry (r, j-1)
        if (j >= 1) {
            f = r < j ? a.HRp[(size_t)(j - 1) * ld + r] + hv[r] : nu;
            if (lane == 0) a.HRf[(size_t)r * mx + (j - 1)] = f;
        }
        if (j >= mx) continue;
        // sum_{m = max(0, r-1)}^{j-2} HRf(r, m) a_m, lanes over m, then a fixed tree
        double part = 0.0;
        for (int m = max(0, r - 1) + lane; m <= j - 2; m += 64)
            part = __builtin_fma(a.HRf[(size_t)r * mx + m], hv[m], part);
        part = wave_sum(part);
        if (lane == 0) {
            double s = (r < j ? hv[j + 1 + r] : gj) - part;
            if (j >= 1) s = __builtin_fma(-f, hv[j - 1], s);
            a.HRp[(size_t)j * ld + r] = s / nu;
        }
    }
}

// poll wave of block 0: Givens step on the completed column j - 1; hh holds
// HRp(0:j-1, j-1), loaded at the start of the launch
__device__ __forceinline__ void dcgs2_givens(const ArnoldiArgs& a, const double* hv, double nu, double* hh,
                                             const double* csL, const double* snL) {
    const int j = a.j, lane = threadIdx.x & 63;
    for (int l = lane; l < j; l += 64) hh[l] += hv[l];
    if (lane == 0) hh[j] = nu;
    wave_sync();
    wave_givens_column(a, hh, j - 1, csL, snL);
}

template <int EPT>
__global__ __launch_bounds__(AT) void k_arnoldi_dcgs2(ArnoldiArgs a) {
    extern __shared__ __align__(16) double dyn[];
    __shared__ double nu_s, gj_s;
    __shared__ double wsum2[2 * (AT_DATA / 64)];
    __shared__ int abort_flag;
    if (a.st->done) return;                  // uniform: written by an earlier launch
    if (a.by_step) {                         // graph replay: the step comes from the solver state
        a.j = a.st->jcur;
        a.parity = a.j & 1;
    }
    const int b = blockIdx.x, t = threadIdx.x, nb = a.nb, lane = t & 63, wave = t >> 6;
    const bool data = t < AT_DATA;
    const int gstride = nb * AT_DATA;
    const int base = b * AT_DATA + t;
    const int n = a.n, j = a.j, rmax = 2 * a.maxlinks, R = 2 * j + 2;
    constexpr int DW = AT_DATA / 64;
    // LDS (dcgs2_lds_words): (u, y) staging, block partials = poll buffer, totals,
    // Hessenberg column, cs, sn
    double* pvec = dyn + (size_t)2 * AT_DATA * (EPT < DCGS2_SE ? EPT : DCGS2_SE);
    double* red = pvec;                      // free once the partials are published
    double* hv = pvec + rmax + nb;
    double* hh = hv + rmax;
    double* csL = hh + a.maxlinks;
    double* snL = csL + a.maxit;
    const size_t pw = dcgs2_parity_words(a.maxlinks, nb);
    unsigned long long* cur = a.slots + (size_t)a.parity * pw;
    unsigned long long* nxt = a.slots + (size_t)(1 - a.parity) * pw;
    const size_t blk = (size_t)rmax * nb;
    // re-arm this block's words of the other buffer for the next launch (2j + 4 values)
    for (int r = t; r < min(R + 2, rmax); r += AT) {
        nxt[(size_t)r * nb + b] = SENTINEL;
        nxt[blk + (size_t)b * rmax + r] = SENTINEL;
    }
    if (t == 0) abort_flag = 0;
    if (b == 0) {
        for (int l = t; l + 1 < j; l += AT) {
            csL[l] = a.cs[l];
            snL[l] = a.sn[l];
        }
        if (wave == DW)                       // first projections of column j - 1
            for (int l = lane; l < j; l += 64) hh[l] = a.HRp[(size_t)(j - 1) * a.ld + l];
    }
    double u[EPT], yv[EPT];
    const double* uj = a.V + (size_t)j * n;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        int i = base + e * gstride;
        bool ok = data && i < n;
        u[e] = ld0(uj, i, ok);
        yv[e] = ld0(a.y, i, ok);
    }
    __syncthreads();
    block_dots_cols<EPT>(a.V, n, j, u, yv, gstride, (double2*)dyn, wsum2, pvec);
    grid_vsum(pvec, R, nb, cur, cur + blk, rmax, red, hv, &abort_flag);
    if (abort_flag) {
        if (t == 0) {
            a.st->err = 1;
            a.st->done = 3;
        }
        return;
    }
    if (wave == DW) {
        double q = 0.0, ab = 0.0;
        for (int l = lane; l < j; l += 64) {
            q = __builtin_fma(hv[l], hv[l], q);
            ab = __builtin_fma(hv[l], hv[j + 1 + l], ab);
        }
        q = wave_sum(q);
        ab = wave_sum(ab);
        if (lane == 0) {
            double nu = 1.0;
            if (j > 0) {
                double qq = hv[j] - q;
                nu = qq > 0.0 ? __builtin_sqrt(qq) : 0.0;
            }
            nu_s = nu;
            gj_s = (hv[2 * j + 1] - ab) / nu;
        }
    }
    __syncthreads();
    const double nu = nu_s, gj = gj_s;
    if (wave < DW) {
        if constexpr (EPT <= DCGS2_SE) {     // reload from the staging instead of holding them through pass 1
            const double2* uy = (const double2*)dyn;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                u[e] = uy[e * AT_DATA + t].x;
                yv[e] = uy[e * AT_DATA + t].y;
            }
        }
        if (j < a.maxit)
            dcgs2_update<EPT>(a.V, n, j, u, yv, hv, hv + j + 1, nu, gj, base, gstride, a.V + (size_t)j * n,
                              a.V + (size_t)(j + 1) * n);
    } else {
        // the poll wave's bookkeeping is a short dependent chain next to the
        // streaming data waves: raise its issue priority while it runs
        __builtin_amdgcn_s_setprio(3);
        dcgs2_rows(a, hv, nu, gj);
        if (b == 0 && j >= 1) dcgs2_givens(a, hv, nu, hh, csL, snL);
        // every block read the step index before publishing its partial sums,
        // which this block has received: the next launch's index can be set
        if (a.by_step && b == 0 && lane == 0) a.st->jcur = j + 1;
        __builtin_amdgcn_s_setprio(0);
    }
}

// ---------------------------------------------------------------------------
// Pipelined DCGS2 step: the step of k_arnoldi_dcgs2 with its grid-wide sum
// split by groups of DCGS2P_GS basis vectors, so that pass 2 trails pass 1 by
// LAG groups instead of waiting for the whole of pass 1.  A thread keeps the
// basis entries it loaded for a group's pass 1 (in registers for LR groups,
// then, where the LDS holds them, in its own LDS words for NL more)
// and runs that group's pass 2 on them, so the basis is read from memory once
// per step; the latency of the sums is hidden behind the streaming of the
// next LAG groups.  Every data thread owns EPT consecutive rows; group g =
// vectors GS g .. GS g + GS - 1:
//   pass 1: per vector l, the thread's products with (u_j, y) summed over its
//           rows (FMA chain), a fixed tree over the wave, then the 8 waves in
//           order by the last wave to arrive, which publishes the block's
//           partials of a_l and b_l into the write-once slots;
//   sums:   the poll wave of block l mod nb owns vector l: it adds the nb
//           partials (lane-strided in block order, then a fixed tree) and
//           writes a_l and b_l into every block's mailbox; every poll wave
//           moves its mailbox into LDS in vector order and raises `ready`;
//   pass 2: u_j -= a_l v_l and y -= b_l v_l for the vectors of group
//           g - LAG, ascending l, once `ready` covers them.
// omega and c (block partials formed first) are owned by block j mod nb.  The
// poll wave then forms nu and gj, releases the data waves for the final
// scaling (v_j, u_{j+1}) and completes its Hessenberg rows and the Givens step
// as in the two-pass launch.  All sums have a fixed order, so the results do
// not depend on timing.  Deadlock-free by induction over the groups given
// co-residency (a thread waits only for sums of groups every block has
// already published or will publish without waiting); every wait is bounded.
// ---------------------------------------------------------------------------
constexpr int DCGS2P_GS = 4;                   // basis vectors per group
static_assert(64 % (2 * DCGS2P_GS) == 0, "a lane set of the poll wave holds one group's values");
// Register ring of a thread (7 buffers of a group at 163 VGPRs): LR groups kept
// after their pass 1 and the loads of PF groups ahead.  With the LDS extension
// LR = 4, PF = 2 (a fixed 400-step solve at 512^2: 45.7 ms against 46.7 for
// LR = 5, PF = 1, 46.2 for 3 and 3, 47.1 for 2 and 4); without it the lag has
// no slack to give up: LR = 5, PF = 1.
__host__ __device__ constexpr int dcgs2p_lr(int nl) { return nl > 0 ? 4 : 5; }
__host__ __device__ constexpr int dcgs2p_pf(int nl) { return nl > 0 ? 2 : 1; }
// LDS slots that extend the lag: a thread moves the oldest group of its register
// ring into LDS instead of running its pass 2 at once, and pass 2 reads it back
// NL groups later (128 KB of LDS per block at either EPT); NL = 0: no extension
template <int EPT>
constexpr int dcgs2p_nl_ext() { return 8 / EPT; }
__host__ __device__ constexpr int dcgs2p_ring(int nl) { return dcgs2p_lr(nl) + nl + 2; }   // wave partials in flight

__host__ __device__ constexpr size_t dcgs2p_lds_words(int rmax, int maxlinks, int maxit, int nl, int ept) {
    return (size_t)rmax + (size_t)maxlinks + 2 * (size_t)maxit +
           (size_t)dcgs2p_ring(nl) * (AT_DATA / 64) * 2 * DCGS2P_GS + (size_t)nl * DCGS2P_GS * ept * AT_DATA;
}

// Ordering of LDS traffic between the waves of a block.  A wave's LDS
// operations are performed in order, so a flag stored (or an atomic performed)
// after data stores is seen after them; what must not happen is that the
// compiler moves the accesses across each other, and a workgroup fence would
// also wait for the wave's outstanding global loads (the prefetch of the next
// group).  So: wait for the wave's LDS operations only (s_waitcnt lgkmcnt(0),
// the other counters at their maximum) and a compiler barrier.
__device__ __forceinline__ void lds_order() {
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __asm__ volatile("" ::: "memory");
}

// A data wave's wait for the poll wave: until *flag >= need, or the poll wave
// gave up (its own waits are bounded); bounded too, with a bound beyond the poll
// wave's, so that it only trips if the poll wave stopped without a word.
__device__ __forceinline__ bool wait_lds_at_least(int* flag, int need, const int* abort_flag) {
    long long spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < need) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) return false;
        if (++spins > 16 * SPIN_LIMIT) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    lds_order();
    return true;
}

// Wave totals of eight values per lane at once: three halving exchanges (lanes
// 32, 16, 8 apart: each lane keeps half of its values and adds its partner's
// half, so that after them lane L holds value L / 8 summed over 8 lanes), then
// the sum over the 8 lanes of each group (xor 1 and xor 2 by DPP moves, xor 4
// by a lane permute).  Lane 8v returns the total of value v; a fixed tree.
__device__ __forceinline__ double wave_sum8(const double (&x)[8], int lane) {
    double c4[4], c2[2];
    const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const double send = h32 ? x[m] : x[m + 4];
        c4[m] = (h32 ? x[m + 4] : x[m]) + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const double send = h16 ? c4[m] : c4[m + 2];
        c2[m] = (h16 ? c4[m + 2] : c4[m]) + __shfl_xor(send, 16, 64);
    }
    const double send = h8 ? c2[0] : c2[1];
    double w = (h8 ? c2[1] : c2[0]) + dpp_mov<0x128>(send);   // row_ror:8 = lane xor 8 in a row of 16
    w += dpp_mov<0xB1>(w);                                      // quad_perm xor 1
    w += dpp_mov<0x4E>(w);                                      // quad_perm xor 2
    w += __shfl_xor(w, 4, 64);
    return w;
}

// The poll wave of a pipelined DCGS2 launch (groups of GS basis vectors): the
// block partials of omega and c, the event loop of the grid-wide sums (mailbox
// words of the lane sets' groups, the partials of the owned columns), then nu
// and gj for the data waves, the block's Hessenberg rows and (block 0) the
// Givens step.  ready, fin, abort_flag, nu_s and gj_s are the block's LDS words.
template <int GS>
__device__ __forceinline__ void dcgs2p_poll(ArnoldiArgs& a, int b, int nb, int lane, int j, int G, int rmax,
                                            unsigned long long* slots, unsigned long long* mbox, double* hv,
                                            double* hh, const double* csL, const double* snL, const double* wsum2,
                                            int& ready, int& fin, int& abort_flag, double& nu_s, double& gj_s) {
    constexpr int DW = AT_DATA / 64, GV = 2 * GS;
    // ---- poll wave: block partials of omega and c, the sums, then the bookkeeping ----
    __builtin_amdgcn_s_setprio(3);
    if (lane == 0) {
        double om = 0.0, c = 0.0;
        for (int w = 0; w < DW; ++w) {
            om += wsum2[2 * w];
            c += wsum2[2 * w + 1];
        }
        __hip_atomic_store(&slots[(size_t)j * nb + b], (unsigned long long)__double_as_longlong(om),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&slots[(size_t)(2 * j + 1) * nb + b], (unsigned long long)__double_as_longlong(c),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // An event loop, so that no single wait holds up the others: each pass
    // polls (once, without waiting) the mailbox words of eight groups at a time
    // (lanes 8q .. 8q + 7 take the groups q, q + 8, ... in order, lane 8q + k
    // the value k of its group: a_l for even k, b_l for odd k) and the slots of
    // the next column this block owns (columns b, b + nb, ..., then omega and c
    // as column j); `ready` is raised to the groups complete in every lane set.
    constexpr int SETS = 64 / GV;
    const int q4 = lane / GV, k16 = lane % GV;
    int gq = q4;                          // this lane set's group
    bool have = false;                    // this lane's value of group gq is in hv
    int own = b < j ? b : (j % nb == b ? j : -1);   // next owned column (j: omega and c)
    unsigned long long ov[8];             // owned column: partials of sources lane, lane + 64, ... (a, b)
    unsigned omask = 0u;
    bool ready_c = false;                 // omega and c are in hv
    long long idle = 0;
    bool to = false;
    const unsigned omask_all = [&] {
        unsigned m = 0u;
        for (int s4 = 0; s4 < 4; ++s4)
            if (lane + 64 * s4 < nb) m |= 3u << (2 * s4);
        return m;
    }();
    for (;;) {
        bool progress = false;
        // every load of the pass is issued before any of them is used, so that
        // one memory round trip serves the mailbox words of the lane sets'
        // groups, omega and c, and the partials of the owned column
        const int l = GS * gq + (k16 >> 1);
        const bool want_m = gq < G && l < j && !have;
        const int rm = (k16 & 1) ? j + 1 + l : l;
        const bool want_c = !ready_c && lane < 2;
        const int rc = lane ? 2 * j + 1 : j;
        const int r1 = own < j ? own : j, r2 = own < j ? j + 1 + own : 2 * j + 1;
        unsigned long long mv = SENTINEL, cv = SENTINEL, nv[8];
        if (want_m) mv = __hip_atomic_load(&mbox[(size_t)b * rmax + rm], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (want_c) cv = __hip_atomic_load(&mbox[(size_t)b * rmax + rc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int src = lane + 64 * s4;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                nv[2 * s4 + h] = SENTINEL;
                if (own >= 0 && src < nb && !(omask & (1u << (2 * s4 + h))))
                    nv[2 * s4 + h] = __hip_atomic_load(&slots[(size_t)(h ? r2 : r1) * nb + src], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (want_m && mv != SENTINEL) {
            hv[rm] = __longlong_as_double((long long)mv);
            have = true;
        }
        if (gq < G && l >= j) have = true;
        if (want_c) {
            if (cv != SENTINEL) hv[rc] = __longlong_as_double((long long)cv);
            ready_c = cv != SENTINEL;
        }
        ready_c = (__builtin_amdgcn_ballot_w64(ready_c) & 3ull) == 3ull;
        // a lane set whose group is complete moves to its next group
        const unsigned long long hb = __builtin_amdgcn_ballot_w64(have || gq >= G);
        constexpr unsigned long long SETMASK = GV == 64 ? ~0ull : ((1ull << GV) - 1ull);
        const bool set_done = ((hb >> (GV * q4)) & SETMASK) == SETMASK;
        if (set_done && gq < G) {
            gq += SETS;
            have = false;
            progress = true;
        }
        // groups complete in every set: the smallest group a set still waits for
        int gmin = gq;
#pragma unroll
        for (int off = GV; off < 64; off <<= 1) gmin = min(gmin, __shfl_xor(gmin, off, 64));
        const int rdy = min(GS * min(gmin, G), j);
        lds_order();
        if (lane == 0 && rdy > __hip_atomic_load(&ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
            __hip_atomic_store(&ready, rdy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        // the owned column: its partials, then the totals into every mailbox
        if (own >= 0) {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (nv[k] != SENTINEL) {
                    ov[k] = nv[k];
                    omask |= 1u << k;
                }
            if (__builtin_amdgcn_ballot_w64(omask != omask_all) == 0ull) {
                double s1 = 0.0, s2 = 0.0;
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
                    if (lane + 64 * s4 < nb) {
                        s1 += __longlong_as_double((long long)ov[2 * s4]);
                        s2 += __longlong_as_double((long long)ov[2 * s4 + 1]);
                    }
                s1 = wave_sum(s1);
                s2 = wave_sum(s2);
                const unsigned long long w1 = (unsigned long long)__double_as_longlong(s1);
                const unsigned long long w2 = (unsigned long long)__double_as_longlong(s2);
                for (int q = lane; q < nb; q += 64) {
                    __hip_atomic_store(&mbox[(size_t)q * rmax + r1], w1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&mbox[(size_t)q * rmax + r2], w2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                omask = 0u;
                own = own == j ? -1 : (own + nb < j ? own + nb : (j % nb == b ? j : -1));
                progress = true;
            }
        }
        if (gmin >= G && ready_c && own < 0) break;
        if (progress) {
            idle = 0;
        } else {
            if (++idle > SPIN_LIMIT) {
                to = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    if (to) {
        if (lane == 0) {
            __hip_atomic_store(&abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            a.st->err = 1;
            a.st->done = 3;
        }
        return;
    }
    lds_order();
    double q = 0.0, ab = 0.0;
    for (int l = lane; l < j; l += 64) {
        q = __builtin_fma(hv[l], hv[l], q);
        ab = __builtin_fma(hv[l], hv[j + 1 + l], ab);
    }
    q = wave_sum(q);
    ab = wave_sum(ab);
    double nu = 1.0;
    if (j > 0) {
        double qq = hv[j] - q;
        nu = qq > 0.0 ? __builtin_sqrt(qq) : 0.0;
    }
    const double gj = (hv[2 * j + 1] - ab) / nu;
    if (lane == 0) {
        nu_s = nu;
        gj_s = gj;
    }
    lds_order();
    if (lane == 0) __hip_atomic_store(&fin, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    dcgs2_rows(a, hv, nu, gj);
    if (b == 0 && j >= 1) dcgs2_givens(a, hv, nu, hh, csL, snL);
    // every block read the step index before publishing its partial sums,
    // which this block has received: the next launch's index can be set
    if (a.by_step && b == 0 && lane == 0) a.st->jcur = j + 1;
    __builtin_amdgcn_s_setprio(0);
}

// The step's second operator product inside the pipelined launch: y = M x at a
// data thread's EPT consecutive rows.  The 64 EPT rows of a wave own one
// contiguous run of CSR entries, which the wave reads coalesced in chunks of
// 64 K entries (entry c0 + 64 k + lane on lane `lane`); each lane multiplies its
// entries by the gathered x and stages the products in the wave's own columns
// of the lag extension (word k AT_DATA + lane of `stage`, free until the lag
// first moves a group there), and each thread then adds its rows' products in
// ascending entry order.  The sums and their order do not depend on the launch
// shape beyond EPT.  pr: the row pointers of the thread's rows and the one after
// (clamped to n, so rows past n - 1 are empty).
template <int EPT, int K, typename T>
__device__ __forceinline__ void fused_rows(const int (&pr)[EPT + 1], const int* __restrict__ mcol,
                                           const T* __restrict__ mval, const double* __restrict__ x,
                                           double* stage, int lane, double (&y)[EPT]) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) y[e] = 0.0;
    const int lo = __builtin_amdgcn_readlane(pr[0], 0), hi = __builtin_amdgcn_readlane(pr[EPT], 63);
    for (int c0 = lo; c0 < hi; c0 += 64 * K) {
        int cj[K];
        T cv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int q = c0 + 64 * k + lane;
            const int qq = q < hi ? q : c0;  // past the run: entry c0 again, not staged
            cj[k] = mcol[qq];
            cv[k] = mval[qq];
        }
        double xv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) xv[k] = x[cj[k]];
#pragma unroll
        for (int k = 0; k < K; ++k) stage[(size_t)k * AT_DATA + lane] = to_f64(cv[k]) * xv[k];
        lds_order();                         // a wave's LDS operations complete in order
        const int c1 = min(hi, c0 + 64 * K);
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            double s = y[e];
            for (int q = max(pr[e], c0); q < min(pr[e + 1], c1); ++q) {
                const int o = q - c0;
                s += stage[(size_t)(o >> 6) * AT_DATA + (o & 63)];
            }
            y[e] = s;
        }
        lds_order();                         // read before the next chunk overwrites
    }
}
// entries per lane and chunk of the fused product (the stage holds 32 words per lane)
constexpr int DCGS2P_FK = 24;

// MV < 0: y is read from a.y; MV = a value precision (SPAI_FP64 ..): y = M mx
// computed in the launch (fused_rows), M's values of that precision
template <int EPT, int NL, int MV>
__global__ __launch_bounds__(AT) void k_arnoldi_dcgs2p(ArnoldiArgs a) {
    static_assert(MV < 0 || DCGS2P_FK <= NL * DCGS2P_GS * EPT, "the fused product stages in the lag extension");
    constexpr int RING = dcgs2p_ring(NL);
    constexpr int LR = dcgs2p_lr(NL), PF = dcgs2p_pf(NL);
    constexpr int LAG = LR + NL;             // groups between pass 1 and pass 2
    extern __shared__ __align__(16) double dyn[];
    __shared__ double nu_s, gj_s;
    __shared__ double wsum2[2 * (AT_DATA / 64)];
    __shared__ int abort_flag, ready, fin;
    __shared__ int arrived[RING];
    const bool by_step = a.by_step;
    if (by_step) {                           // graph replay: the step comes from the solver state
        if (a.st->done) return;              // uniform: written by an earlier launch
        a.j = a.st->jcur;
        a.parity = a.j & 1;
    }
    const int b = blockIdx.x, t = threadIdx.x, nb = a.nb, lane = t & 63, wave = t >> 6;
    // a data thread's rows: EPT consecutive ones from row0 (at EPT = 2 one 16-byte
    // load per vector)
    const int row0 = EPT * (b * AT_DATA + t);
    const int n = a.n, j = a.j, rmax = 2 * a.maxlinks, R = 2 * j + 2;
    constexpr int DW = AT_DATA / 64;
    // LDS (dcgs2p_lds_words): totals hv (a_l = hv[l], omega = hv[j], b_l = hv[j+1+l],
    // c = hv[2j+1]), the Hessenberg column, cs, sn, the wave partials [RING][DW][2 GS],
    // the lag extension [NL][GS * EPT][AT_DATA] (a thread's own words)
    double* hv = dyn;
    double* hh = hv + rmax;
    double* csL = hh + a.maxlinks;
    double* snL = csL + a.maxit;
    double* wpart = snL + a.maxit;
    double* ext = wpart + (size_t)RING * (AT_DATA / 64) * 2 * DCGS2P_GS;
    const size_t pw = dcgs2_parity_words(a.maxlinks, nb);
    unsigned long long* cur = a.slots + (size_t)a.parity * pw;
    unsigned long long* nxt = a.slots + (size_t)(1 - a.parity) * pw;
    const size_t blk = (size_t)rmax * nb;
    unsigned long long* slots = cur;         // [rmax][nb]
    unsigned long long* mbox = cur + blk;    // [nb][rmax]
    constexpr int GS = DCGS2P_GS, GV = 2 * GS;   // vectors and values per group
    const int G = (j + GS - 1) / GS;
    // loads of group gl's vectors at the thread's rows (a vector past j - 1 reads vector 0, unused)
    auto load_group = [&](int gl, double (&v)[GS][EPT]) {
#pragma unroll
        for (int c = 0; c < GS; ++c) {
            const int l = GS * gl + c;
            const double* col = a.V + (size_t)(l < j ? l : 0) * n;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int i = row0 + e;
                // at EPT = 2 a row past n - 1 is not clamped: the rows end below 2n
                // (one row per thread did not cover n), so it reads vector l + 1,
                // which the basis holds (l + 1 <= j <= maxit); its product is not added
                if constexpr (EPT >= 2) v[c][e] = col[i];
                else v[c][e] = col[pf_index(i, i < n)];
            }
        }
    };
    constexpr int NBUF = LR + 1 + PF;        // register buffers: groups g - LR .. g + PF
    double B[NBUF][GS][EPT];
    double u[EPT], yv[EPT];
    int pr[EPT + 1];
    if (wave < DW) {
        // u_j, y (or the row pointers of the fused product) and the first group
        // go out before the launch looks at the stop flag, so that its latency
        // overlaps theirs (all in bounds: j <= maxit)
        const double* uj = a.V + (size_t)j * n;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = row0 + e;
            const bool ok = i < n;
            u[e] = ld0(uj, i, ok);
            if constexpr (MV < 0) yv[e] = ld0(a.y, i, ok);
        }
        if constexpr (MV >= 0)
#pragma unroll
            for (int e = 0; e <= EPT; ++e) pr[e] = a.mrp[min(row0 + e, n)];
#pragma unroll
        for (int q = 0; q < PF; ++q) load_group(q, B[q]);   // in flight through the block's first barrier
    }
    if (!by_step && a.st->done) return;      // uniform: written by an earlier launch
    // re-arm this block's words of the other buffer for the next launch (2j + 4 values)
    for (int r = t; r < min(R + 2, rmax); r += AT) {
        nxt[(size_t)r * nb + b] = SENTINEL;
        nxt[blk + (size_t)b * rmax + r] = SENTINEL;
    }
    if (t == 0) {
        abort_flag = 0;
        ready = 0;
        fin = 0;
    }
    if (t < RING) arrived[t] = 0;
    if (b == 0) {
        for (int l = t; l + 1 < j; l += AT) {
            csL[l] = a.cs[l];
            snL[l] = a.sn[l];
        }
        if (wave == DW)                       // first projections of column j - 1
            for (int l = lane; l < j; l += 64) hh[l] = a.HRp[(size_t)(j - 1) * a.ld + l];
    }
    if (wave < DW) {
        if constexpr (MV >= 0)
            fused_rows<EPT, DCGS2P_FK>(pr, a.mcol, (const typename ValType<MV < 0 ? 0 : MV>::T*)a.mval, a.mx,
                                       ext + 64 * wave, lane, yv);
        double om = 0.0, c = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            om = __builtin_fma(u[e], u[e], om);
            c = __builtin_fma(u[e], yv[e], c);
        }
        om = wave_sum(om);
        c = wave_sum(c);
        if (lane == 0) {
            wsum2[2 * wave] = om;
            wsum2[2 * wave + 1] = c;
        }
    }
    __syncthreads();
    if (wave == DW) {
        dcgs2p_poll<GS>(a, b, nb, lane, j, G, rmax, slots, mbox, hv, hh, csL, snL, wsum2, ready, fin, abort_flag,
                        nu_s, gj_s);
        return;
    }
    // ---- data waves: pass 1 of group g and pass 2 of group g - LAG ----
    const bool update = j < a.maxit;         // launch maxit only completes column maxit - 1
    double au[EPT], ay[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        au[e] = u[e];
        ay[e] = yv[e];
    }
    // one step g: the loads of group g + PF into vn, pass 1 of group g from vc
    // (loaded PF steps before), pass 2 of group g - LAG from the values this
    // thread loaded for that group's pass 1 (so the basis is read once from
    // memory): from vp, the register buffer of group g - LR, or with the LDS
    // extension from its LDS slot, into which vp then moves; NBUF register
    // buffers in turn, one loop trip per NBUF steps
    bool ok = true;
    double* mine = ext + t;                  // this thread's LDS words: [slot][GS * EPT] stride AT_DATA
    auto step = [&](int g, double (&vc)[GS][EPT], double (&vn)[GS][EPT], double (&vp)[GS][EPT]) {
        const int g2 = g - LAG;
        // unconditional (past the last group the loads fall on vector 0): a load
        // under a branch makes the compiler's wait counts assume the loads of the
        // step before are the most recent, so pass 1 would wait for every load
        load_group(g + PF, vn);
        if (g < G) {
            const int ring = g % RING;
            double* wp = wpart + ((size_t)ring * DW + wave) * GV;
            static_assert(GV == 8, "wave_sum8 reduces the 8 values of a group of 4 vectors");
            double pv[GV];
#pragma unroll
            for (int c = 0; c < GS; ++c) {
                double p1 = 0.0, p2 = 0.0;
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    const int i = row0 + e;
                    const double vv = i < n ? vc[c][e] : 0.0;
                    p1 = __builtin_fma(vv, u[e], p1);
                    p2 = __builtin_fma(vv, yv[e], p2);
                }
                pv[2 * c] = p1;
                pv[2 * c + 1] = p2;
            }
            const double tot = wave_sum8(pv, lane);
            if ((lane & 7) == 0) wp[lane >> 3] = tot;
            lds_order();
            int old = 0;
            if (lane == 0) old = __hip_atomic_fetch_add(&arrived[ring], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            old = __builtin_amdgcn_readfirstlane(old);
            if (old == DW - 1) {
                // the last wave of the block to finish the group: the block's partials, waves in order
                lds_order();
                if (lane < GV) {
                    const int c = lane >> 1, l = GS * g + c;
                    double sum = 0.0;
                    for (int w = 0; w < DW; ++w) sum += wpart[((size_t)ring * DW + w) * GV + lane];
                    if (l < j) {
                        const int r = (lane & 1) ? j + 1 + l : l;
                        __hip_atomic_store(&slots[(size_t)r * nb + b], (unsigned long long)__double_as_longlong(sum),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                lds_order();
                if (lane == 0) __hip_atomic_store(&arrived[ring], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        if (g2 >= 0) {
            // the wait also paces the waves of the block when pass 2 is skipped: no
            // wave runs more than LAG + 1 groups ahead of the block's last
            // published group, so a ring entry is free again before its next use
            const int l0 = GS * g2;
            if (ok && !wait_lds_at_least(&ready, min(l0 + GS, j), &abort_flag)) ok = false;
            if (update && ok) {
                double w[GS][EPT];
#pragma unroll
                for (int c = 0; c < GS; ++c)
#pragma unroll
                    for (int e = 0; e < EPT; ++e)
                        w[c][e] = NL > 0 ? mine[((size_t)(g2 % (NL > 0 ? NL : 1)) * GS * EPT + c * EPT + e) * AT_DATA]
                                         : vp[c][e];
#pragma unroll
                for (int c = 0; c < GS; ++c) {
                    const int l = l0 + c;
                    if (l < j) {
                        const double al = hv[l], bl = hv[j + 1 + l];
#pragma unroll
                        for (int e = 0; e < EPT; ++e) {
                            au[e] = __builtin_fma(-al, w[c][e], au[e]);
                            ay[e] = __builtin_fma(-bl, w[c][e], ay[e]);
                        }
                    }
                }
            }
        }
        if constexpr (NL > 0) {
            // the oldest register group moves into the slot just read (g2 = gr - NL)
            const int gr = g - LR;
            if (update && ok && gr >= 0 && gr < G)
#pragma unroll
                for (int c = 0; c < GS; ++c)
#pragma unroll
                    for (int e = 0; e < EPT; ++e)
                        mine[((size_t)(gr % NL) * GS * EPT + c * EPT + e) * AT_DATA] = vp[c][e];
        }
    };
    for (int g = 0; g < G + LAG && ok; g += NBUF) {
        // whole trips, no step under a branch (see load_group above): a step past
        // G + LAG - 1 has no pass 1, no pass 2 and nothing to move, and its wait
        // is for all j sums, which every block receives
#pragma unroll
        for (int k = 0; k < NBUF; ++k) step(g + k, B[k], B[(k + PF) % NBUF], B[(k + NBUF - LR) % NBUF]);
    }
    if (!ok) {
        if (lane == 0) {
            a.st->err = 1;
            a.st->done = 3;
        }
        return;
    }
    if (!update) return;
    if (!wait_lds_at_least(&fin, 1, &abort_flag)) {
        if (lane == 0) {
            a.st->err = 1;
            a.st->done = 3;
        }
        return;
    }
    const double nu = nu_s, gj = gj_s;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = row0 + e;
        if (i < n) {
            const double v = j > 0 ? au[e] / nu : au[e];
            if (j > 0) a.V[(size_t)j * n + i] = v;
            a.V[(size_t)(j + 1) * n + i] = __builtin_fma(-gj, v, ay[e]) / nu;
        }
    }
}

// ---------------------------------------------------------------------------
// Pipelined DCGS2 step for more than 2 rows per thread (the registers cannot
// keep a lag of groups there): groups of one basis vector; u_j and y wait in
// LDS (the thread's own words), and pass 2 of vector g - LAG reads that vector
// again, LAG vectors after its pass 1 read it, into the buffer
// pass 1 of vector g has just released.  That second read misses the L2 (the
// lag spans more than an XCD's L2 holds), and the memory-side cache (256 MB)
// serves what it still holds, so HBM sees between one and two reads of the
// basis per step; the launch gains over the two-pass one mostly by its
// pipelining.  Sums, poll wave and final steps as in k_arnoldi_dcgs2p.
// ---------------------------------------------------------------------------
constexpr int DCGS2M_LAG16 = 3, DCGS2M_LAG8 = 6, DCGS2M_LAG4 = 10;
// vectors between pass 1 and pass 2 by rows per thread: enough to cover the
// grid-wide sum at the time a vector takes to stream, few enough that the
// second read still finds much of its vector in the memory-side cache (swept
// on fixed-step solves: at 16 rows per thread lags 3, 4, 6, 9 gave 283, 284,
// 290, 315 ms; at 8 rows lags 3, 6, 10 gave 65.0, 61.3, 61.8 ms; at 4 rows
// lags 4, 10, 16 gave 38.3, 35.5, 36.2 ms)
__host__ __device__ constexpr int dcgs2m_lag(int ept) { return ept >= 16 ? DCGS2M_LAG16 : ept >= 8 ? DCGS2M_LAG8 : DCGS2M_LAG4; }
__host__ __device__ constexpr int dcgs2m_ring(int ept) { return dcgs2m_lag(ept) + 2; }

__host__ __device__ constexpr size_t dcgs2m_lds_words(int rmax, int maxlinks, int maxit, int ept) {
    return (size_t)rmax + (size_t)maxlinks + 2 * (size_t)maxit + (size_t)dcgs2m_ring(ept) * (AT_DATA / 64) * 2 +
           2 * (size_t)ept * AT_DATA;
}

template <int EPT>
__global__ __launch_bounds__(AT) void k_arnoldi_dcgs2m(ArnoldiArgs a) {
    constexpr int LAG = dcgs2m_lag(EPT), RING = dcgs2m_ring(EPT), DW = AT_DATA / 64;
    extern __shared__ __align__(16) double dyn[];
    __shared__ double nu_s, gj_s;
    __shared__ double wsum2[2 * DW];
    __shared__ int abort_flag, ready, fin;
    __shared__ int arrived[RING];
    const bool by_step = a.by_step;
    if (by_step) {                           // graph replay: the step comes from the solver state
        if (a.st->done) return;              // uniform: written by an earlier launch
        a.j = a.st->jcur;
        a.parity = a.j & 1;
    }
    const int b = blockIdx.x, t = threadIdx.x, nb = a.nb, lane = t & 63, wave = t >> 6;
    const int gstride = nb * AT_DATA;
    const int base = b * AT_DATA + t;
    const int n = a.n, j = a.j, rmax = 2 * a.maxlinks, R = 2 * j + 2;
    // LDS (dcgs2m_lds_words): totals hv, the Hessenberg column, cs, sn, the wave
    // partials [RING][DW][2], then u_j and y at the thread's rows [2][EPT][AT_DATA]
    double* hv = dyn;
    double* hh = hv + rmax;
    double* csL = hh + a.maxlinks;
    double* snL = csL + a.maxit;
    double* wpart = snL + a.maxit;
    double* uy = wpart + (size_t)RING * DW * 2;
    const size_t pw = dcgs2_parity_words(a.maxlinks, nb);
    unsigned long long* cur = a.slots + (size_t)a.parity * pw;
    unsigned long long* nxt = a.slots + (size_t)(1 - a.parity) * pw;
    const size_t blk = (size_t)rmax * nb;
    unsigned long long* slots = cur;         // [rmax][nb]
    unsigned long long* mbox = cur + blk;    // [nb][rmax]
    const int G = j;                         // one vector per group
    // loads of vector l at the thread's rows (l past j - 1 reads vector 0, unused).
    // A row past n - 1 is not clamped: with EPT >= 2 the rows end below 2n
    // (EPT is the smallest power of two that covers n), so it reads vector l + 1,
    // which the basis holds (l + 1 <= j <= maxit); its product is not added.  One
    // row offset then serves every load of the thread.
    auto load_vec = [&](int l, double (&v)[EPT]) {
        const double* col = a.V + (size_t)(l < j ? l : 0) * n + base;
#pragma unroll
        for (int e = 0; e < EPT; ++e) v[e] = col[(size_t)e * gstride];
    };
    double B[2][EPT];
    double au[EPT], ay[EPT];                 // u_j and y, then their updates by pass 2
    if (wave < DW) {
        const double* uj = a.V + (size_t)j * n;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            const int i = base + e * gstride;
            const bool ok = i < n;
            au[e] = ld0(uj, i, ok);
            ay[e] = ld0(a.y, i, ok);
        }
        load_vec(0, B[0]);
    }
    if (!by_step && a.st->done) return;      // uniform: written by an earlier launch
    // re-arm this block's words of the other buffer for the next launch (2j + 4 values)
    for (int r = t; r < min(R + 2, rmax); r += AT) {
        nxt[(size_t)r * nb + b] = SENTINEL;
        nxt[blk + (size_t)b * rmax + r] = SENTINEL;
    }
    if (t == 0) {
        abort_flag = 0;
        ready = 0;
        fin = 0;
    }
    if (t < RING) arrived[t] = 0;
    if (b == 0) {
        for (int l = t; l + 1 < j; l += AT) {
            csL[l] = a.cs[l];
            snL[l] = a.sn[l];
        }
        if (wave == DW)                       // first projections of column j - 1
            for (int l = lane; l < j; l += 64) hh[l] = a.HRp[(size_t)(j - 1) * a.ld + l];
    }
    if (wave < DW) {
        double om = 0.0, c = 0.0;
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            om = __builtin_fma(au[e], au[e], om);
            c = __builtin_fma(au[e], ay[e], c);
            uy[(size_t)e * AT_DATA + t] = au[e];
            uy[(size_t)(EPT + e) * AT_DATA + t] = ay[e];
        }
        om = wave_sum(om);
        c = wave_sum(c);
        if (lane == 0) {
            wsum2[2 * wave] = om;
            wsum2[2 * wave + 1] = c;
        }
    }
    __syncthreads();
    if (wave == DW) {
        dcgs2p_poll<1>(a, b, nb, lane, j, G, rmax, slots, mbox, hv, hh, csL, snL, wsum2, ready, fin, abort_flag,
                       nu_s, gj_s);
        return;
    }
    // ---- data waves: pass 1 of vector g and pass 2 of vector g - LAG ----
    const bool update = j < a.maxit;         // launch maxit only completes column maxit - 1
    const double* us = uy + t;
    const double* ys = uy + (size_t)EPT * AT_DATA + t;
    bool ok = true;
    // one step g: the loads of vector g + 1 into vn, pass 1 of vector g from vc
    // (loaded the step before), then vector g - LAG again into vc for its pass 2;
    // two buffers in turn, whole trips of two steps (a step past G + LAG - 1 only
    // waits for all sums; the loads are unconditional, past the end vector 0)
    auto step = [&](int g, double (&vc)[EPT], double (&vn)[EPT]) {
        const int g2 = g - LAG;
        load_vec(g + 1, vn);
        if (g < G) {
            const int ring = g % RING;
            double p1 = 0.0, p2 = 0.0;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int i = base + e * gstride;
                const double vv = i < n ? vc[e] : 0.0;
                p1 = __builtin_fma(vv, us[(size_t)e * AT_DATA], p1);
                p2 = __builtin_fma(vv, ys[(size_t)e * AT_DATA], p2);
            }
            p1 = wave_sum(p1);
            p2 = wave_sum(p2);
            if (lane == 0) {
                wpart[((size_t)ring * DW + wave) * 2] = p1;
                wpart[((size_t)ring * DW + wave) * 2 + 1] = p2;
            }
            lds_order();
            int old = 0;
            if (lane == 0) old = __hip_atomic_fetch_add(&arrived[ring], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            old = __builtin_amdgcn_readfirstlane(old);
            if (old == DW - 1) {
                // the last wave of the block to finish the vector: the block's partials, waves in order
                lds_order();
                if (lane < 2) {
                    double sum = 0.0;
                    for (int w = 0; w < DW; ++w) sum += wpart[((size_t)ring * DW + w) * 2 + lane];
                    const int r = lane ? j + 1 + g : g;
                    __hip_atomic_store(&slots[(size_t)r * nb + b], (unsigned long long)__double_as_longlong(sum),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                lds_order();
                if (lane == 0) __hip_atomic_store(&arrived[ring], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        if (g2 >= 0) {
            // the wait also paces the waves of the block when pass 2 is skipped (a
            // ring entry is free again before its next use)
            if (ok && !wait_lds_at_least(&ready, min(g2 + 1, j), &abort_flag)) ok = false;
            if (update && ok && g2 < G) {
                load_vec(g2, vc);
                const double al = hv[g2], bl = hv[j + 1 + g2];
#pragma unroll
                for (int e = 0; e < EPT; ++e) {
                    au[e] = __builtin_fma(-al, vc[e], au[e]);
                    ay[e] = __builtin_fma(-bl, vc[e], ay[e]);
                }
            }
        }
    };
    for (int g = 0; g < G + LAG && ok; g += 2) {
        step(g, B[0], B[1]);
        step(g + 1, B[1], B[0]);
    }
    if (!ok) {
        if (lane == 0) {
            a.st->err = 1;
            a.st->done = 3;
        }
        return;
    }
    if (!update) return;
    if (!wait_lds_at_least(&fin, 1, &abort_flag)) {
        if (lane == 0) {
            a.st->err = 1;
            a.st->done = 3;
        }
        return;
    }
    const double nu = nu_s, gj = gj_s;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int i = base + e * gstride;
        if (i < n) {
            const double v = j > 0 ? au[e] / nu : au[e];
            if (j > 0) a.V[(size_t)j * n + i] = v;
            a.V[(size_t)(j + 1) * n + i] = __builtin_fma(-gj, v, ay[e]) / nu;
        }
    }
}

__global__ void k_fill_u64(unsigned long long* p, size_t len, unsigned long long v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) p[i] = v;
}

// ---------------------------------------------------------------------------
// reductions (standalone norms and the per-projection fallback path)
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[RB / 64];
    v = wave_sum(v);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < RB / 64; ++q) t += sh[q];
    __syncthreads();
    return t;   // valid in thread 0
}

// Last-block finalisation: every block writes its partial; the block that takes
// the last ticket sums the partials in block order and writes the result.
__device__ __forceinline__ bool last_block(unsigned* ticket) {
    __shared__ bool is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = atomicAdd(ticket, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    return is_last;
}

__device__ __forceinline__ double sum_partials(const double* partials, int nb) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += RB) acc += partials[q];
    return block_sum(acc);
}

enum { MGS_DOT = 0, MGS_NORM = 1 };

// One projection of the fallback path: if vprev is given, y -= (*hprev) vprev;
// then out = <y, vcur> (MGS_DOT) or ||y||_2 (MGS_NORM).
__global__ __launch_bounds__(RB) void k_mgs(int n, double* __restrict__ y, const double* __restrict__ vprev,
                                            const double* __restrict__ hprev, const double* __restrict__ vcur,
                                            double* __restrict__ out, double* __restrict__ partials,
                                            unsigned* __restrict__ ticket, int mode, const SolveState* st) {
    if (st && st->done) return;
    const double coef = vprev ? *hprev : 0.0;
    double acc = 0.0;
    const int stride = gridDim.x * RB;
    for (int i = blockIdx.x * RB + threadIdx.x; i < n; i += stride) {
        double yi = y[i];
        if (vprev) {
            yi = __builtin_fma(-coef, vprev[i], yi);
            y[i] = yi;
        }
        double vi = (mode == MGS_NORM) ? yi : vcur[i];
        acc = __builtin_fma(yi, vi, acc);
    }
    double bs = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = bs;
    if (last_block(ticket)) {
        double tot = sum_partials(partials, gridDim.x);
        if (threadIdx.x == 0) {
            *out = (mode == MGS_NORM) ? __builtin_sqrt(tot) : tot;
            *ticket = 0u;
        }
    }
}

// v = y / (*h)
__global__ void k_scale(int n, const double* __restrict__ y, const double* __restrict__ h, double* __restrict__ v,
                        const SolveState* st) {
    if (st && st->done) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = y[i] / *h;
}

// Fallback Givens update (one thread): rotations, new rotation, g, stop test.
__global__ void k_givens(int j, int maxit, double* __restrict__ H, int ld, double* __restrict__ cs,
                         double* __restrict__ sn, double* __restrict__ g, double tau, SolveState* st) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || st->done) return;
    double* h = H + (size_t)j * ld;
    double hn = h[j + 1];
    for (int l = 0; l < j; ++l) {
        double a = h[l], c = h[l + 1];
        h[l] = cs[l] * a + sn[l] * c;
        h[l + 1] = -sn[l] * a + cs[l] * c;
    }
    double delta = hypot(h[j], h[j + 1]);
    cs[j] = h[j] / delta;
    sn[j] = h[j + 1] / delta;
    h[j] = delta;
    h[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    st->gabs = fabs(g[j + 1]);
    if (fabs(g[j + 1]) <= tau * st->beta0 || hn == 0.0) {
        st->its = j + 1;
        st->done = 1;
    } else if (j + 1 == maxit) {
        st->its = j + 1;
        st->done = 2;
    }
}

// y = H(0:k, 0:k)^{-1} g(0:k) by column-oriented back substitution (one block)
__global__ __launch_bounds__(RB) void k_backsolve(int k, const double* __restrict__ H, int ld,
                                                  const double* __restrict__ g, double* __restrict__ work,
                                                  double* __restrict__ yk) {
    for (int i = threadIdx.x; i < k; i += RB) work[i] = g[i];
    __syncthreads();
    for (int c = k - 1; c >= 0; --c) {
        double yc = work[c] / H[(size_t)c * ld + c];
        __syncthreads();
        if (threadIdx.x == 0) yk[c] = yc;
        for (int i = threadIdx.x; i < c; i += RB) work[i] = __builtin_fma(-H[(size_t)c * ld + i], yc, work[i]);
        __syncthreads();
    }
}

// The same back substitution for k <= BS_MAXK with the latency of H off the
// critical path: the whole workgroup stages BS_COLS columns of H (rows 0 .. top
// of the block) in LDS with all loads in flight, then wave 0 runs those columns
// with the right-hand side in registers (lane l holds rows l, l + 64, ...) and
// the pivot value broadcast by readlane, no barrier per column.  Same
// operations in the same order as k_backsolve.
constexpr int BS_MAXK = 512;
constexpr int BS_COLS = 32;

__global__ __launch_bounds__(RB) void k_backsolve_lds(int k, const double* __restrict__ H, int ld,
                                                      const double* __restrict__ g, double* __restrict__ yk) {
    constexpr int M = BS_MAXK / 64;
    __shared__ double hb[BS_COLS * BS_MAXK];   // column q of the block at hb[q * BS_MAXK]
    const int t = threadIdx.x, lane = t & 63;
    double wv[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int i = lane + 64 * m;
        wv[m] = i < k ? g[i] : 0.0;
    }
    for (int top = k - 1; top >= 0; top -= BS_COLS) {
        const int c0 = max(top - BS_COLS + 1, 0), nc = top - c0 + 1, rows = top + 1;
        __syncthreads();
        // 16 loads in flight per thread, then their LDS stores
        const int tot = nc * rows;
        for (int e0 = 0; e0 < tot; e0 += 16 * RB) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = min(e0 + u * RB + t, tot - 1);
                const int q = e / rows, i = e - q * rows;
                v[u] = H[(size_t)(c0 + q) * ld + i];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int e = e0 + u * RB + t;
                if (e < tot) {
                    const int q = e / rows, i = e - q * rows;
                    hb[q * BS_MAXK + i] = v[u];
                }
            }
        }
        __syncthreads();
        if (t < 64) {
            for (int c = top; c >= c0; --c) {
                const double* hc = hb + (c - c0) * BS_MAXK;
                const int mc = c >> 6;
                double wc = 0.0;
#pragma unroll
                for (int m = 0; m < M; ++m)
                    if (m == mc) wc = wv[m];
                wc = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(wc), c & 63),
                                      __builtin_amdgcn_readlane(__double2loint(wc), c & 63));
                const double yc = wc / hc[c];
                if (lane == 0) yk[c] = yc;
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int i = lane + 64 * m;
                    if (i < c) wv[m] = __builtin_fma(-hc[i], yc, wv[m]);
                }
            }
        }
    }
}

// x += V_k y; records ||d||_inf and ||x||_inf (non-negative doubles compare as integers).
// The loop over the basis is unrolled by 8 so that eight loads are in flight per
// thread; the sum keeps its order (the same bits).
__global__ void k_update(int n, int k, const double* __restrict__ V, const double* __restrict__ yk,
                         double* __restrict__ x, unsigned long long* __restrict__ maxbits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double dm = 0.0, xm = 0.0;
    if (i < n) {
        double di = 0.0;
#pragma unroll 8
        for (int c = 0; c < k; ++c) di = di + V[(size_t)c * n + i] * yk[c];
        double xi = x[i] + di;
        x[i] = xi;
        dm = fabs(di);
        xm = fabs(xi);
    }
    for (int o = 32; o > 0; o >>= 1) {
        dm = fmax(dm, __shfl_xor(dm, o, 64));
        xm = fmax(xm, __shfl_xor(xm, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&maxbits[0], (unsigned long long)__double_as_longlong(dm));
        atomicMax(&maxbits[1], (unsigned long long)__double_as_longlong(xm));
    }
}

// t = V_k y (the correction before the right preconditioner is applied)
__global__ void k_vy(int n, int k, const double* __restrict__ V, const double* __restrict__ yk,
                     double* __restrict__ t) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double di = 0.0;
#pragma unroll 8
    for (int c = 0; c < k; ++c) di = di + V[(size_t)c * n + i] * yk[c];
    t[i] = di;
}

// x += d; records ||d||_inf and ||x||_inf like k_update
__global__ void k_add_norms(int n, const double* __restrict__ dv, double* __restrict__ x,
                            unsigned long long* __restrict__ maxbits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    double dm = 0.0, xm = 0.0;
    if (i < n) {
        const double di = dv[i];
        const double xi = x[i] + di;
        x[i] = xi;
        dm = fabs(di);
        xm = fabs(xi);
    }
    for (int o = 32; o > 0; o >>= 1) {
        dm = fmax(dm, __shfl_xor(dm, o, 64));
        xm = fmax(xm, __shfl_xor(xm, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&maxbits[0], (unsigned long long)__double_as_longlong(dm));
        atomicMax(&maxbits[1], (unsigned long long)__double_as_longlong(xm));
    }
}

// g = beta0 e_1; fresh solver state
__global__ void k_init_state(double* g, int len, const double* beta0, SolveState* st) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) g[i] = (i == 0) ? *beta0 : 0.0;
    if (i == 0) {
        st->beta0 = *beta0;
        st->done = 0;
        st->its = 0;
        st->err = 0;
        st->jcur = 0;
        st->gabs = *beta0;
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

static inline int blocks_for(int n, int t) { return (n + t - 1) / t; }

static int reduce_blocks(int n) {
    int b = (n + RB * 4 - 1) / (RB * 4);
    return std::max(1, std::min(b, RBLOCKS));
}

// rows per lane group in the sparse products (measured on the 512 x 512
// workload: 2 for A with 5 entries per row, 4 for P with up to 20)
constexpr int SPMV_R = 2;
constexpr int APPLY_R = 4;

// entries per lane whose loads go out together: 2 when an average row is
// longer than the lanes per row, else 1
static inline int row_it(long long nnz, int n, int g) { return (double)nnz > (double)g * n ? 2 : 1; }

// Lanes per row and entries per lane in flight of an application of P.  A
// large preconditioner with 17 to 32 entries per row on average takes 4 lanes
// per row with ceil(average / 4) entries each in flight: measured at 128^3
// (25 per row; a fixed 300-step solve 268 ms against 276 with 16 lanes of two,
// 271 with 8 of four, 270 with 4 of eight, 280 with 2 of fourteen).  Otherwise
// lanes_per_row and row_it.
static inline int apply_it(long long nnz, int n, int g) {
    const double avg = n > 0 ? (double)nnz / n : 0.0;
    if (g == 4 && n >= (1 << 16) && avg > 16.0 && avg <= 32.0) return (int)std::ceil(avg / 4.0);
    return row_it(nnz, n, g);
}
static inline int apply_lanes(long long nnz, int n) {
    const double avg = n > 0 ? (double)nnz / n : 0.0;
    if (n >= (1 << 16) && avg > 16.0 && avg <= 32.0) return 4;
    return lanes_per_row(nnz, n);
}

template <int VP, bool RIGHT, bool SCALED = false>
static void apply_P_g(int g, int n, const spai_precond* P, const double* w, double* y, hipStream_t s,
                      const SolveState* st, int by_step) {
    using T = typename ValType<VP>::T;
    const T* pv = (const T*)P->val;
    const long long groups = ((long long)n + APPLY_R - 1) / APPLY_R;
    const unsigned grid = (unsigned)((groups * g + 255) / 256);
    const int it = apply_it(P->nnz, n, g);
#define SPAI_AP(G, IT)                                                                                       \
    hipLaunchKernelGGL((k_apply_P_g<VP, G, APPLY_R, RIGHT, SCALED, IT>), dim3(grid), dim3(256), 0, s, n, P->rowptr, \
                       P->col, pv, P->d, w, y, st, by_step)
#define SPAI_AP2(G) if (it == 2) SPAI_AP(G, 2); else SPAI_AP(G, 1)
    if (g == 4 && it >= 5) {
        switch (it) {
        case 5: SPAI_AP(4, 5); break;
        case 6: SPAI_AP(4, 6); break;
        case 7: SPAI_AP(4, 7); break;
        default: SPAI_AP(4, 8); break;
        }
    } else switch (g) {
    case 1: SPAI_AP2(1); break;
    case 2: SPAI_AP2(2); break;
    case 4: SPAI_AP2(4); break;
    case 8: SPAI_AP2(8); break;
    default: SPAI_AP2(16); break;
    }
#undef SPAI_AP2
#undef SPAI_AP
}

// scaled: (left preconditioner) w already holds D w, as written by a product
// with output scaling d
// by_step (graph replay, st set): the input is column st->jcur of the basis starting at w
static int launch_apply_P(spai_handle* h, const spai_precond* P, const double* w, double* y, hipStream_t s,
                          const SolveState* st = nullptr, bool scaled = false, int by_step = 0) {
    const int n = P->n, g = apply_lanes(P->nnz, n);
    SPAI_ARG(P->nnz >= 1, "the preconditioner has no entries");   // the kernel reads entry 0 past row ends
    long tk = timer_begin(h, SPAI_KT_APPLY_P);
    const int mode = P->side == SPAI_RIGHT ? 2 : scaled ? 1 : 0;
#define SPAI_AP_MODE(VP)                                     \
    if (mode == 2) apply_P_g<VP, true>(g, n, P, w, y, s, st, by_step);          \
    else if (mode == 1) apply_P_g<VP, false, true>(g, n, P, w, y, s, st, by_step); \
    else apply_P_g<VP, false>(g, n, P, w, y, s, st, by_step);
    switch (P->val_prec) {
    case SPAI_FP64: SPAI_AP_MODE(SPAI_FP64); break;
    case SPAI_FP32: SPAI_AP_MODE(SPAI_FP32); break;
    case SPAI_FP16: SPAI_AP_MODE(SPAI_FP16); break;
    default: SPAI_AP_MODE(SPAI_BF16); break;
    }
#undef SPAI_AP_MODE
    timer_end(h, SPAI_KT_APPLY_P, tk);
    SPAI_HIP(hipGetLastError());
    return SPAI_OK;
}

// Lanes per row and entries per lane in flight of the operator's product.  A
// large matrix with short rows (at least 65,536 rows of at most 8 entries on
// average) takes one lane per row with ceil(average) entries in flight, 4 to 8:
// measured for 5 entries per row at 512^2 (an Arnoldi solve of 400 fixed steps
// 43.5 ms against 44.0 with 4 lanes of two entries) and for 7 at 128^3 (a
// product 46.0 us against 53.5; 46.8 with 8 in flight, 51.8 with 2 lanes of 3).
// Otherwise lanes_per_row and row_it, as for P (small systems keep that shape).
struct SpmvShape {
    int g, it;
};
static SpmvShape spmv_shape(long long nnz, int n) {
    const double avg = n > 0 ? (double)nnz / n : 0.0;
    if (n >= (1 << 16) && avg <= 8.0) return {1, std::max(4, (int)std::ceil(avg))};
    const int g = lanes_per_row(nnz, n);
    return {g, row_it(nnz, n, g)};
}

// dout (may be NULL): output scaling, y_i = dout_i (A x)_i; by_step as launch_apply_P
static int launch_spmv(spai_handle* h, const spai_csr* A, const double* x, double* y, hipStream_t s,
                       const SolveState* st = nullptr, const double* dout = nullptr, int by_step = 0) {
    const int n = A->n;
    const SpmvShape sh = spmv_shape(A->nnz, n);
    const int g = sh.g, it = sh.it;
    SPAI_ARG(A->nnz >= 1, "the matrix has no entries");   // the kernel reads entry 0 past row ends
    // one row per lane in the one-lane shape (twice the waves: 43.0 against 43.2 ms
    // for the 400-step solve at 512^2, 45.2 against 46.9 us for the product at
    // 128^3); SPMV_R rows per lane group otherwise
    const bool one = g == 1 && it >= 4;
    const int rows = one ? 1 : SPMV_R;
    const long long groups = ((long long)n + rows - 1) / rows;
    const unsigned grid = (unsigned)((groups * g + 255) / 256);
    long tk = timer_begin(h, SPAI_KT_SPMV_A);
#define SPAI_SP(G, IT)                                                                                              \
    hipLaunchKernelGGL((k_spmv_g<G, SPMV_R, IT>), dim3(grid), dim3(256), 0, s, n, A->rowptr, A->col, A->val, x, y, \
                       dout, st, by_step)
#define SPAI_SP2(G) if (it == 2) SPAI_SP(G, 2); else SPAI_SP(G, 1)
#define SPAI_SP1(IT)                                                                                           \
    hipLaunchKernelGGL((k_spmv_g<1, 1, IT>), dim3(grid), dim3(256), 0, s, n, A->rowptr, A->col, A->val, x, y, dout, \
                       st, by_step)
    if (one) {
        switch (it) {
        case 4: SPAI_SP1(4); break;
        case 5: SPAI_SP1(5); break;
        case 6: SPAI_SP1(6); break;
        case 7: SPAI_SP1(7); break;
        default: SPAI_SP1(8); break;
        }
    } else switch (g) {
    case 1: SPAI_SP2(1); break;
    case 2: SPAI_SP2(2); break;
    case 4: SPAI_SP2(4); break;
    case 8: SPAI_SP2(8); break;
    default: SPAI_SP2(16); break;
    }
#undef SPAI_SP2
#undef SPAI_SP1
#undef SPAI_SP
    timer_end(h, SPAI_KT_SPMV_A, tk);
    SPAI_HIP(hipGetLastError());
    return SPAI_OK;
}

static int launch_x0(const spai_precond* P, const double* b, double* x0, hipStream_t s) {
    int n = P->n, g = blocks_for(n, 256);
#define SPAI_X0(VP, UF, T, R) hipLaunchKernelGGL((k_x0<VP, UF, R>), dim3(g), dim3(256), 0, s, n, P->rowptr, P->col, (const T*)P->val, P->d, b, x0)
    const bool right = P->side == SPAI_RIGHT;
    switch (P->val_prec) {
    case SPAI_FP64:
        if (right) { SPAI_X0(SPAI_FP64, SPAI_FP64, double, true); } else { SPAI_X0(SPAI_FP64, SPAI_FP64, double, false); }
        break;
    case SPAI_FP32:
        if (P->u_f == SPAI_FP16) {
            if (right) { SPAI_X0(SPAI_FP32, SPAI_FP16, float, true); } else { SPAI_X0(SPAI_FP32, SPAI_FP16, float, false); }
        } else if (P->u_f == SPAI_BF16) {
            if (right) { SPAI_X0(SPAI_FP32, SPAI_BF16, float, true); } else { SPAI_X0(SPAI_FP32, SPAI_BF16, float, false); }
        } else {
            if (right) { SPAI_X0(SPAI_FP32, SPAI_FP32, float, true); } else { SPAI_X0(SPAI_FP32, SPAI_FP32, float, false); }
        }
        break;
    case SPAI_FP16:
        if (right) { SPAI_X0(SPAI_FP16, SPAI_FP16, __half, true); } else { SPAI_X0(SPAI_FP16, SPAI_FP16, __half, false); }
        break;
    default:
        if (right) { SPAI_X0(SPAI_BF16, SPAI_BF16, __hip_bfloat16, true); } else { SPAI_X0(SPAI_BF16, SPAI_BF16, __hip_bfloat16, false); }
        break;
    }
#undef SPAI_X0
    SPAI_HIP(hipGetLastError());
    return SPAI_OK;
}

static int launch_residual(spai_handle* h, const spai_csr* A, const double* b, const double* x, double* r,
                           spai_prec ur, hipStream_t s) {
    int n = A->n, g = blocks_for(n, 256);
    long tk = timer_begin(h, SPAI_KT_RESIDUAL);
    if (ur == SPAI_DD)
        hipLaunchKernelGGL(k_residual<true>, dim3(g), dim3(256), 0, s, n, A->rowptr, A->col, A->val, b, x, r);
    else
        hipLaunchKernelGGL(k_residual<false>, dim3(g), dim3(256), 0, s, n, A->rowptr, A->col, A->val, b, x, r);
    timer_end(h, SPAI_KT_RESIDUAL, tk);
    SPAI_HIP(hipGetLastError());
    return SPAI_OK;
}

static int check_csr(const spai_csr* A) {
    SPAI_ARG(A && A->n > 0 && A->nnz >= 0 && A->rowptr && A->col && A->val, "bad matrix");
    return SPAI_OK;
}

// Launch configuration of the Arnoldi kernel: nb blocks of AT threads, EPT
// elements per thread (a power of two); nb = 0 when the cooperative kernel cannot
// hold the problem (the per-projection MGS path is used instead).
struct ArnoldiCfg {
    int nb = 0;
    int ept = 0;
    int ortho = SPAI_ORTHO_MGS;
    bool ext = false;        // pipelined DCGS2: the lag extended through LDS
    bool reread = false;     // pipelined DCGS2 with more than 2 rows per thread (pass 2 reads its vector again)
    int mv = -1;             // pipelined DCGS2 with the LDS extension: value precision of the fused second product, or -1
    size_t shmem = 0;
    size_t slot_words = 0;   // both parities
};

// DCGS2 with at most 2 rows per thread runs the pipelined launch unless
// SPAI_DCGS2=twopass selects the two-pass one (both give the same iterates up to
// the order of their sums)
static bool dcgs2_pipelined() {
    static const bool p = [] {
        const char* e = getenv("SPAI_DCGS2");
        return !(e && std::string(e) == "twopass");
    }();
    return p;
}

// SPAI_DCGS2_REREAD=0 keeps the two-pass launch for more than 2 rows per thread
static bool dcgs2_reread() {
    static const bool x = [] {
        const char* e = getenv("SPAI_DCGS2_REREAD");
        return !(e && std::string(e) == "0");
    }();
    return x;
}

// SPAI_DCGS2_LDS=0 keeps the pipelined launch's lag to its register ring
static bool dcgs2_lds_ext() {
    static const bool x = [] {
        const char* e = getenv("SPAI_DCGS2_LDS");
        return !(e && std::string(e) == "0");
    }();
    return x;
}

// SPAI_DCGS2_FUSE=0 keeps the step's second operator product a launch of its
// own (read at every solve, so that one process can compare both)
static bool dcgs2_fuse() {
    const char* e = getenv("SPAI_DCGS2_FUSE");
    return !(e && std::string(e) == "0");
}

template <int EPT>
static const void* arnoldi_fn(int ortho, bool ext, bool reread, int mv) {
    switch (ortho) {
    case SPAI_ORTHO_CGS2: return (const void*)k_arnoldi_cgs2<EPT>;
    case SPAI_ORTHO_DCGS2:
        if constexpr (EPT <= 2) {
            constexpr int NE = dcgs2p_nl_ext<EPT>();
            if (dcgs2_pipelined()) {
                if (!ext) return (const void*)k_arnoldi_dcgs2p<EPT, 0, -1>;
                switch (mv) {
                case SPAI_FP64: return (const void*)k_arnoldi_dcgs2p<EPT, NE, SPAI_FP64>;
                case SPAI_FP32: return (const void*)k_arnoldi_dcgs2p<EPT, NE, SPAI_FP32>;
                case SPAI_FP16: return (const void*)k_arnoldi_dcgs2p<EPT, NE, SPAI_FP16>;
                case SPAI_BF16: return (const void*)k_arnoldi_dcgs2p<EPT, NE, SPAI_BF16>;
                default: return (const void*)k_arnoldi_dcgs2p<EPT, NE, -1>;
                }
            }
        } else {
            if (reread) return (const void*)k_arnoldi_dcgs2m<EPT>;
        }
        return (const void*)k_arnoldi_dcgs2<EPT>;
    default: return (const void*)k_arnoldi<EPT>;
    }
}

static const void* arnoldi_fn(int ortho, int ept, bool ext, bool reread, int mv) {
    switch (ept) {
    case 1: return arnoldi_fn<1>(ortho, ext, reread, mv);
    case 2: return arnoldi_fn<2>(ortho, ext, reread, mv);
    case 4: return arnoldi_fn<4>(ortho, ext, reread, mv);
    case 8: return arnoldi_fn<8>(ortho, ext, reread, mv);
    default: return arnoldi_fn<16>(ortho, ext, reread, mv);
    }
}

// mv: value precision of the step's second operator product (fused into the
// pipelined DCGS2 launch where that launch has its LDS extension), or -1
static ArnoldiCfg arnoldi_config(spai_handle* h, int n, int maxit, int ortho, int mv = -1) {
    ArnoldiCfg c;
    c.ortho = ortho;
    if (ortho == SPAI_ORTHO_MGS)
        if (const char* e = getenv("SPAI_ARNOLDI_PATH"))
            if (std::string(e) == "projection") return ArnoldiCfg{};
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, h->device) != hipSuccess || !coop) {
        (void)hipGetLastError();
        return ArnoldiCfg{};
    }
    const int maxlinks = maxit + 2;
    const int rows_nb = std::max(1, blocks_for(n, AT_DATA));
    // MGS: half the CUs (the grid-wide sums get cheaper with fewer blocks while half
    // the chip still streams the basis fast enough); CGS2 streams the basis four
    // times per step and uses every CU
    int nb = ortho != SPAI_ORTHO_MGS ? std::min(std::min(h->num_cu, MAX_NB), rows_nb)
                                     : std::min(std::min(std::max(1, h->num_cu / 2), MAX_NB), rows_nb);
    if ((long long)nb * AT_DATA * 16 < n)    // more blocks rather than more than 16 elements per thread
        nb = std::min(std::min(h->num_cu, MAX_NB), rows_nb);
    if (const char* e = getenv("SPAI_ARNOLDI_BLOCKS")) {
        int want = atoi(e);
        if (want >= 1 && want <= MAX_NB) nb = std::min(want, rows_nb);
    }
    int ept = 1;
    while ((long long)nb * AT_DATA * ept < n) ept <<= 1;
    if (ept > 16) return ArnoldiCfg{};
    if (ortho == SPAI_ORTHO_CGS2) {
        c.shmem = sizeof(double) * ((size_t)(AT_DATA / 64 + 4) * maxlinks + nb + 2 * (size_t)maxit);
        c.slot_words = 2 * cgs2_parity_words(maxlinks, nb);
    } else if (ortho == SPAI_ORTHO_DCGS2) {
        if (ept <= 2 && dcgs2_pipelined()) {
            // the LDS extension of the lag where it fits beside the per-step arrays
            const int nl = ept == 1 ? dcgs2p_nl_ext<1>() : dcgs2p_nl_ext<2>();
            c.shmem = sizeof(double) * dcgs2p_lds_words(2 * maxlinks, maxlinks, maxit, nl, ept);
            c.ext = dcgs2_lds_ext() && c.shmem <= 159 * 1024;
            if (!c.ext) c.shmem = sizeof(double) * dcgs2p_lds_words(2 * maxlinks, maxlinks, maxit, 0, ept);
        } else {
            // more rows per thread: the pipelined launch that reads each vector again
            // for pass 2, where u_j and y fit in LDS beside the per-step arrays
            c.shmem = sizeof(double) * dcgs2m_lds_words(2 * maxlinks, maxlinks, maxit, ept);
            c.reread = dcgs2_pipelined() && dcgs2_reread() && c.shmem <= 159 * 1024;
            if (!c.reread) c.shmem = sizeof(double) * dcgs2_lds_words(ept, 2 * maxlinks, nb, maxlinks, maxit);
        }
        c.slot_words = 2 * dcgs2_parity_words(maxlinks, nb);
    } else {
        c.shmem = sizeof(double) * (size_t)(3 * maxit + 2);
        c.slot_words = (size_t)2 * maxlinks * nb * (1 + MBOX_STRIDE);
    }
    if (c.shmem > 159 * 1024) return ArnoldiCfg{};   // 160 KB of LDS per CU, 1 KB for static arrays
    // whether every block of a launch of fn can be resident at once
    auto admits = [&](const void* fn) {
        if (c.shmem > 48 * 1024 &&
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c.shmem) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, AT, c.shmem) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return per_cu * h->num_cu >= nb;
    };
    if (c.ext && mv >= 0 && dcgs2_fuse() && admits(arnoldi_fn(ortho, ept, true, false, mv))) c.mv = mv;
    if (c.mv < 0 && !admits(arnoldi_fn(ortho, ept, c.ext, c.reread, -1))) return ArnoldiCfg{};
    c.nb = nb;
    c.ept = ept;
    return c;
}

// Whether a solve of n unknowns runs the fused Arnoldi launch on the CUs the
// handle counts (h->num_cu) rather than the separate-kernel path.
bool arnoldi_fused_fits(spai_handle* h, int n, int maxit, int ortho) {
    return arnoldi_config(h, n, std::min(maxit, n), ortho).nb > 0;
}

// The blocks of an Arnoldi launch must be resident together (they wait on each
// other's partial sums).  arnoldi_config admits a configuration only when the
// occupancy query shows that all nb blocks fit on the device at once, so an
// ordinary launch on an otherwise idle device places them all; every wait is
// bounded, so a launch whose blocks were not all placed ends with an error
// instead of hanging.  The cooperative launch API gives the same placement
// with a formal guarantee, but costs about 11 us of queue synchronisation on
// each side of every launch; SPAI_COOPERATIVE=1 selects it.
static bool use_cooperative_launch() {
    static const bool coop = [] {
        const char* e = getenv("SPAI_COOPERATIVE");
        return e && std::string(e) == "1";
    }();
    return coop;
}

static int launch_arnoldi(spai_handle* h, const ArnoldiCfg& c, ArnoldiArgs& a, hipStream_t s) {
    void* args[] = {&a};
    const void* fn = arnoldi_fn(c.ortho, c.ept, c.ext, c.reread, c.mv);
    long tk = timer_begin(h, SPAI_KT_MGS);
    hipError_t e = use_cooperative_launch() ? hipLaunchCooperativeKernel(fn, dim3(c.nb), dim3(AT), args, c.shmem, s)
                                            : hipLaunchKernel(fn, dim3(c.nb), dim3(AT), args, c.shmem, s);
    timer_end(h, SPAI_KT_MGS, tk);
    SPAI_HIP(e);
    return SPAI_OK;
}

int gmres_ir_batched_impl(spai_handle* h, const spai_csr* A, const spai_precond* P, int32_t nsys,
                          const int32_t* sys_ptr, const double* b, double* x, const spai_ir_params* prm,
                          spai_ir_stats* st);

// two events without timing, destroyed with the scope
// ---------------------------------------------------------------------------
// Workspace of spai_gmres_ir_noalloc: one array in every device's memory, for
// callers that cannot allocate.  Host code never passes the array's name to a
// kernel (in host code it is a host-side stand-in); it uses the device address
// hipGetSymbolAddress gives for the device at hand, looked up once per device.
// ---------------------------------------------------------------------------

constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES];

int noalloc_scratch_init(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) {
        set_error("device index " + std::to_string(device) + " beyond the library's table");
        return SPAI_E_ARG;
    }
    std::lock_guard<std::mutex> l(g_scratch_mu);
    if (g_scratch_ptr[device]) return SPAI_OK;
    int cur = -1;
    SPAI_HIP(hipGetDevice(&cur));
    if (cur != device) SPAI_HIP(hipSetDevice(device));
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        set_error(std::string("hipGetSymbolAddress of the no-allocation workspace failed: ") + hipGetErrorString(e));
        return SPAI_E_HIP;
    }
    g_scratch_ptr[device] = ptr;
    return SPAI_OK;
}

static void* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> l(g_scratch_mu);
    return device >= 0 && device < NOALLOC_MAX_DEVICES ? g_scratch_ptr[device] : nullptr;
}

// A chunk of DCGS2 Arnoldi steps as one HIP graph (graph and executable,
// destroyed with the scope).
struct ChunkGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ~ChunkGraph() {
        if (x) (void)hipGraphExecDestroy(x);
        if (g) (void)hipGraphDestroy(g);
    }
};

// The operands of the second operator product when it runs inside the pipelined
// DCGS2 launch: y = A w (right preconditioning) or y = P w with w = D A v_j (left)
static void fused_operands(const ArnoldiCfg& cfg, const spai_csr* A, const spai_precond* P, const double* w,
                           ArnoldiArgs& aa) {
    if (cfg.mv < 0) return;
    if (P->side == SPAI_RIGHT) {
        aa.mrp = A->rowptr;
        aa.mcol = A->col;
        aa.mval = A->val;
    } else {
        aa.mrp = P->rowptr;
        aa.mcol = P->col;
        aa.mval = P->val;
    }
    aa.mx = w;
}

// Captures `steps` Arnoldi steps (operator products, then the DCGS2 launch) on a
// private stream into cg: every kernel takes the step index from st->jcur and
// the DCGS2 launch advances it, so one executable serves every chunk of every
// refinement step of this call.  No timing events are recorded inside.
static int capture_chunk(spai_handle* h, const spai_csr* A, const spai_precond* P, const ArnoldiCfg& cfg,
                         ArnoldiArgs aa, double* V, double* w, double* y, SolveState* sst, int steps,
                         ChunkGraph& cg) {
    hipStream_t cs = nullptr;
    SPAI_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    int saved[SPAI_KT_COUNT];
    for (int k = 0; k < SPAI_KT_COUNT; ++k) {
        saved[k] = h->timers[k].every;
        h->timers[k].every = 0;
    }
    const bool right = P->side == SPAI_RIGHT;
    aa.by_step = 1;
    aa.j = 0;
    aa.parity = 0;
    int rc = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess ? SPAI_OK : SPAI_E_HIP;
    const bool capturing = rc == SPAI_OK;
    const bool fused = cfg.mv >= 0;   // the second product runs inside the Arnoldi launch
    for (int q = 0; q < steps && rc == SPAI_OK; ++q) {
        if (right) {                                               // y = A P v_j
            rc = launch_apply_P(h, P, V, w, cs, sst, false, 1);
            if (!rc && !fused) rc = launch_spmv(h, A, w, y, cs, sst);
        } else {                                                   // y = M^T (D (A v_j))
            rc = launch_spmv(h, A, V, w, cs, sst, P->d, 1);
            if (!rc && !fused) rc = launch_apply_P(h, P, w, y, cs, sst, true);
        }
        if (!rc) rc = launch_arnoldi(h, cfg, aa, cs);
    }
    hipGraph_t g = nullptr;
    if (capturing && hipStreamEndCapture(cs, &g) != hipSuccess && rc == SPAI_OK) rc = SPAI_E_HIP;
    for (int k = 0; k < SPAI_KT_COUNT; ++k) h->timers[k].every = saved[k];
    if (rc == SPAI_OK && g) {
        cg.g = g;
        if (hipGraphInstantiate(&cg.x, g, nullptr, nullptr, 0) != hipSuccess) rc = SPAI_E_HIP;
    } else if (g) {
        (void)hipGraphDestroy(g);
    }
    (void)hipStreamDestroy(cs);
    if (rc == SPAI_E_HIP) set_error("capturing the Arnoldi chunk into a HIP graph failed");
    return rc;
}

// scratch != NULL: the workspace is carved from that device memory of
// scratch_bytes bytes (spai_gmres_ir_noalloc), no device memory is allocated and
// no event, stream or graph is created; working precision FP64 only.
int gmres_ir_impl(spai_handle* h, const spai_csr* A, const spai_precond* P, const double* b, double* x,
                  const spai_ir_params* prm, spai_ir_stats* st, void* scratch = nullptr,
                  size_t scratch_bytes = 0) {
    SPAI_ARG(h && prm, "NULL handle or parameters");
    SPAI_ARG(P, "NULL preconditioner");
    SPAI_ARG(b && x, "NULL right-hand side or solution");
    int rc = check_csr(A);
    if (rc) return rc;
    const int n = A->n;
    SPAI_ARG(P->n == n, "preconditioner size differs from the matrix");
    SPAI_ARG(prm->imax >= 1 && prm->imax <= 32, "imax must lie in 1..32");
    SPAI_ARG(prm->maxit >= 1, "maxit must be positive");
    SPAI_ARG(prm->tau >= 0.0, "tau must be non-negative");
    SPAI_ARG(prm->u_r == SPAI_DD || prm->u_r == SPAI_FP64, "u_r must be DD or FP64");
    SPAI_ARG(prm->ortho == SPAI_ORTHO_MGS || prm->ortho == SPAI_ORTHO_CGS2 || prm->ortho == SPAI_ORTHO_DCGS2,
             "ortho must be MGS, CGS2 or DCGS2");
    SPAI_ARG(prm->u == SPAI_FP64 || prm->u == SPAI_FP32, "the working precision u must be FP64 or FP32");
    const bool right = P->side == SPAI_RIGHT;
    SPAI_ARG(!right || prm->u == SPAI_FP64, "right preconditioning runs in working precision FP64");
    SPAI_ARG(!scratch || prm->u == SPAI_FP64, "the allocation-free solve runs in working precision FP64");
    if (prm->u == SPAI_FP32) {
        // working precision single: the system runs in the batched solver as a batch of one
        SPAI_ARG(prm->ortho == SPAI_ORTHO_MGS, "working precision FP32 orthogonalises with MGS");
        const int32_t one[2] = {0, n};
        spai_ir_stats tmp{};
        rc = gmres_ir_batched_impl(h, A, P, 1, one, b, x, prm, &tmp);
        if (rc >= 0 && st) *st = tmp;
        return rc;
    }
    SPAI_HIP(hipSetDevice(h->device));
    hipStream_t s = h->stream;
    const int maxit = std::min(prm->maxit, n);
    const int ld = maxit + 1;
    // the step's second operator product (A for right, P for left preconditioning)
    // can run inside the pipelined DCGS2 launch
    const ArnoldiCfg cfg = arnoldi_config(h, n, maxit, prm->ortho, P->side == SPAI_RIGHT ? SPAI_FP64 : P->val_prec);
    SPAI_ARG(cfg.nb > 0 || prm->ortho == SPAI_ORTHO_MGS,
             "CGS2 and DCGS2 need the cooperative Arnoldi kernel, which cannot hold this problem");
    const int maxlinks = maxit + 2;

    // workspace: the basis, three vectors, and H with the rotations, reduction
    // partials, solver state and grid-sum slots
    size_t slot_count = cfg.slot_words;
    const bool dcgs2 = prm->ortho == SPAI_ORTHO_DCGS2;
    const size_t hr_words = dcgs2 ? 2 * (size_t)ld * maxit : 0;   // HRp, HRf
    const size_t vbytes = sizeof(double) * (size_t)n * (size_t)(maxit + 1), wbytes = sizeof(double) * (size_t)n * 3;
    size_t hbytes = sizeof(double) * ((size_t)ld * maxit + 4 * (size_t)ld + RBLOCKS + 64 + slot_count + hr_words);
    double *V, *r, *H;
    if (scratch) {
        auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
        const size_t need = up(vbytes) + up(wbytes) + up(hbytes);
        if (need > scratch_bytes) {
            set_error("invalid argument: the allocation-free solve needs " + std::to_string(need) +
                      " bytes of workspace for n = " + std::to_string(n) + ", maxit = " + std::to_string(maxit) +
                      ", more than its " + std::to_string(scratch_bytes) + "-byte array");
            return SPAI_E_ARG;
        }
        V = (double*)scratch;
        r = (double*)((char*)scratch + up(vbytes));
        H = (double*)((char*)r + up(wbytes));
    } else {
        rc = buffer_reserve(h, h->ws[WS_SOLVE_V], vbytes);
        if (rc) return rc;
        rc = buffer_reserve(h, h->ws[WS_SOLVE_VEC], wbytes);
        if (rc) return rc;
        rc = buffer_reserve(h, h->ws[WS_SOLVE_H], hbytes);
        if (rc) return rc;
        V = (double*)h->ws[WS_SOLVE_V].ptr;
        r = (double*)h->ws[WS_SOLVE_VEC].ptr;
        H = (double*)h->ws[WS_SOLVE_H].ptr;
    }
    double* w = r + n;
    double* y = w + n;
    double* cs = H + (size_t)ld * maxit;
    double* sn = cs + ld;
    double* g = sn + ld;
    double* yk = g + ld;
    double* partials = yk + ld;
    double* scal = partials + RBLOCKS;          // [0] beta0, [1] h_{j+1,j} (projection path)
    SolveState* sst = (SolveState*)(scal + 8);
    unsigned long long* maxbits = (unsigned long long*)(scal + 16);
    unsigned* ticket = (unsigned*)(scal + 24);
    unsigned long long* slots = (unsigned long long*)(scal + 64);
    double* HRp = (double*)(slots + slot_count);
    double* HRf = HRp + (size_t)ld * maxit;
    char* hp = (char*)h->host_pinned.ptr;

    const int tb = 256, gb = blocks_for(n, tb);
    const int nbr = reduce_blocks(n);
    SPAI_HIP(hipMemsetAsync(ticket, 0, 16, s));
    const int chunk = 8;   // Arnoldi steps enqueued between checks of the stop flag
    hipEvent_t* ev = h->chunk_ev;   // completion of the flag copies of the last two chunks

    // graph replay of the Arnoldi chunks (DCGS2 with ordinary launches only)
    ChunkGraph cgraph;
    const bool use_graph = prm->graph && dcgs2 && cfg.nb && !use_cooperative_launch() && !scratch;
    if (use_graph) {
        ArnoldiArgs aa{};
        aa.n = n; aa.ld = ld; aa.maxit = maxit; aa.maxlinks = maxlinks; aa.nb = cfg.nb;
        aa.y = y; aa.V = V; aa.H = H; aa.cs = cs; aa.sn = sn; aa.g = g; aa.tau = prm->tau;
        aa.slots = slots; aa.st = sst; aa.HRp = HRp; aa.HRf = HRf;
        fused_operands(cfg, A, P, w, aa);
        if ((rc = capture_chunk(h, A, P, cfg, aa, V, w, y, sst, chunk, cgraph))) return rc;
    }

    int status = 0;
    spai_ir_stats loc{};
    if (!prm->x_given && (rc = launch_x0(P, b, x, s))) return rc;   // x0 = P b in u_f
    double dprev = INFINITY;
    for (int step = 0; step < prm->imax; ++step) {
        if ((rc = launch_residual(h, A, b, x, r, prm->u_r, s))) return rc;
        if (right) SPAI_HIP(hipMemcpyAsync(V, r, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
        else if ((rc = launch_apply_P(h, P, r, V, s))) return rc;          // z = P r into V(:,0)
        hipLaunchKernelGGL(k_mgs, dim3(nbr), dim3(RB), 0, s, n, V, (const double*)nullptr,
                           (const double*)nullptr, (const double*)V, scal, partials, ticket, (int)MGS_NORM,
                           (const SolveState*)nullptr);
        SPAI_HIP(hipGetLastError());
        SPAI_HIP(hipMemcpyAsync(hp, scal, sizeof(double), hipMemcpyDeviceToHost, s));
        SPAI_HIP(hipStreamSynchronize(s));
        double beta0;
        std::memcpy(&beta0, hp, sizeof(double));
        if (beta0 == 0.0) break;   // P r_i = 0: x_i solves the system
        loc.steps = step + 1;
        hipLaunchKernelGGL(k_scale, dim3(gb), dim3(tb), 0, s, n, (const double*)V, (const double*)scal, V,
                           (const SolveState*)nullptr);
        hipLaunchKernelGGL(k_init_state, dim3(blocks_for(ld, 256)), dim3(256), 0, s, g, ld, (const double*)scal, sst);
        if (cfg.nb) {
            size_t len = slot_count;
            hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, s, slots, len, SENTINEL);
        }
        SPAI_HIP(hipGetLastError());
        SolveState ss{};
        int sweep = 0;
        // DCGS2 completes column j - 1 in launch j: launches 0 .. maxit
        const int jend = dcgs2 ? maxit + 1 : maxit;
        // The stop flag of chunk c is read while chunk c + 1 is already queued, so
        // the device never drains between chunks; a chunk enqueued after the stop
        // returns at once on the device (every kernel checks the flag).
        int pending = -1;   // chunk whose flag copy has not been read yet
        bool stopped = false;
        auto read_flag = [&](int c) -> int {
            SPAI_HIP(hipEventSynchronize(ev[c & 1]));
            std::memcpy(&ss, hp + 256 * (c & 1), sizeof(ss));
            return SPAI_OK;
        };
        int cidx = 0;
        for (int j0 = 0; j0 < jend; j0 += chunk, ++cidx) {
            int j1 = std::min(j0 + chunk, jend);
            if (use_graph) {
                // steps j0 .. j0 + chunk - 1; those at or past jend return at once
                // (the stop flag is set by launch maxit at the latest)
                SPAI_HIP(hipGraphLaunch(cgraph.x, s));
                j1 = j0;
            }
            for (int j = j0; j < j1; ++j) {
                double* vj = V + (size_t)j * n;
                const bool fused = cfg.nb && cfg.mv >= 0;   // the second product inside the Arnoldi launch
                if (right) {                                               // y = A P v_j
                    if ((rc = launch_apply_P(h, P, vj, w, s, sst))) return rc;
                    if (!fused && (rc = launch_spmv(h, A, w, y, s, sst))) return rc;
                } else {                                                   // y = M^T (D (A v_j))
                    if ((rc = launch_spmv(h, A, vj, w, s, sst, P->d))) return rc;
                    if (!fused && (rc = launch_apply_P(h, P, w, y, s, sst, true))) return rc;
                }
                if (cfg.nb) {
                    ArnoldiArgs aa{};
                    aa.n = n; aa.j = j; aa.ld = ld; aa.maxit = maxit; aa.maxlinks = maxlinks; aa.nb = cfg.nb;
                    aa.parity = sweep & 1;
                    aa.y = y; aa.V = V; aa.H = H; aa.cs = cs; aa.sn = sn; aa.g = g; aa.tau = prm->tau;
                    aa.slots = slots; aa.st = sst; aa.HRp = HRp; aa.HRf = HRf;
                    fused_operands(cfg, A, P, w, aa);
                    if ((rc = launch_arnoldi(h, cfg, aa, s))) return rc;
                    ++sweep;
                } else {
                    // one launch per projection: h_lj = <y, v_l>, y -= h_lj v_l, l = 0..j
                    double* hcol = H + (size_t)j * ld;
                    for (int l = 0; l <= j; ++l) {
                        const double* vprev = l > 0 ? V + (size_t)(l - 1) * n : nullptr;
                        const double* hprev = l > 0 ? hcol + (l - 1) : nullptr;
                        long tm = timer_begin(h, SPAI_KT_MGS);
                        hipLaunchKernelGGL(k_mgs, dim3(nbr), dim3(RB), 0, s, n, y, vprev, hprev,
                                           (const double*)(V + (size_t)l * n), hcol + l, partials, ticket,
                                           (int)MGS_DOT, (const SolveState*)sst);
                        timer_end(h, SPAI_KT_MGS, tm);
                    }
                    hipLaunchKernelGGL(k_mgs, dim3(nbr), dim3(RB), 0, s, n, y, (const double*)vj,
                                       (const double*)(hcol + j), (const double*)y, hcol + j + 1, partials, ticket,
                                       (int)MGS_NORM, (const SolveState*)sst);
                    hipLaunchKernelGGL(k_scale, dim3(gb), dim3(tb), 0, s, n, (const double*)y,
                                       (const double*)(hcol + j + 1), V + (size_t)(j + 1) * n, (const SolveState*)sst);
                    hipLaunchKernelGGL(k_givens, dim3(1), dim3(1), 0, s, j, maxit, H, ld, cs, sn, g, prm->tau, sst);
                    SPAI_HIP(hipGetLastError());
                }
            }
            SPAI_HIP(hipMemcpyAsync(hp + 256 * (cidx & 1), sst, sizeof(SolveState), hipMemcpyDeviceToHost, s));
            SPAI_HIP(hipEventRecord(ev[cidx & 1], s));
            if (pending >= 0) {
                if ((rc = read_flag(pending))) return rc;
                if (ss.done) {
                    stopped = true;
                    pending = -1;
                    break;
                }
            }
            pending = cidx;
        }
        if (!stopped && pending >= 0) {
            if ((rc = read_flag(pending))) return rc;
        }
        if (ss.done == 3 || ss.err) {
            set_error("a grid-wide sum of the Arnoldi kernel timed out");
            return SPAI_E_INTERNAL;
        }
        if (ss.done == 0) {
            set_error("GMRES ended without a stop decision");
            return SPAI_E_INTERNAL;
        }
        const int kk = ss.its;
        if (ss.done == 2) status |= SPAI_W_MAXIT;
        loc.its[step] = kk;
        loc.total_its += kk;
        if (kk <= BS_MAXK)
            hipLaunchKernelGGL(k_backsolve_lds, dim3(1), dim3(RB), 0, s, kk, (const double*)H, ld, (const double*)g, yk);
        else
            hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(RB), 0, s, kk, (const double*)H, ld, (const double*)g, w,
                               yk);
        SPAI_HIP(hipMemsetAsync(maxbits, 0, 16, s));
        long tu = timer_begin(h, SPAI_KT_UPDATE);
        if (right) {                                                       // d = P (V_k y)
            hipLaunchKernelGGL(k_vy, dim3(gb), dim3(tb), 0, s, n, kk, (const double*)V, (const double*)yk, w);
            if ((rc = launch_apply_P(h, P, w, y, s))) return rc;
            hipLaunchKernelGGL(k_add_norms, dim3(gb), dim3(tb), 0, s, n, (const double*)y, x, maxbits);
        } else {
            hipLaunchKernelGGL(k_update, dim3(gb), dim3(tb), 0, s, n, kk, (const double*)V, (const double*)yk, x,
                               maxbits);
        }
        timer_end(h, SPAI_KT_UPDATE, tu);
        SPAI_HIP(hipGetLastError());
        SPAI_HIP(hipMemcpyAsync(hp, maxbits, 16, hipMemcpyDeviceToHost, s));
        SPAI_HIP(hipStreamSynchronize(s));
        double dn, xn;
        std::memcpy(&dn, hp, 8);
        std::memcpy(&xn, hp + 8, 8);
        loc.gest[step] = ss.gabs / beta0;
        loc.dnorm[step] = dn;
        if (dn <= prm->tol_ir * xn) break;
        if (step >= 2 && dn > 0.5 * dprev) {
            status |= SPAI_W_NOCONV;
            break;
        }
        dprev = dn;
        if (step == prm->imax - 1) status |= SPAI_W_NOCONV;
    }
    loc.status = status;
    // backward and forward error of the returned x (residual in u_r)
    if ((rc = launch_residual(h, A, b, x, r, prm->u_r, s))) return rc;
    SPAI_HIP(hipMemsetAsync(maxbits + 2, 0, 6 * sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_err_norms, dim3(std::min(gb, 4 * std::max(h->num_cu, 1))), dim3(tb), 0, s, n, A->rowptr,
                       A->val, (const double*)r, (const double*)x, b, prm->x_true, maxbits + 2);
    SPAI_HIP(hipGetLastError());
    SPAI_HIP(hipMemcpyAsync(hp, maxbits + 2, 6 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    SPAI_HIP(hipStreamSynchronize(s));
    double nm[6];
    std::memcpy(nm, hp, sizeof(nm));
    const double den = nm[1] * nm[2] + nm[3];
    loc.nbe = den > 0.0 ? nm[0] / den : 0.0;
    loc.ferr = prm->x_true ? (nm[5] > 0.0 ? nm[4] / nm[5] : nm[4]) : -1.0;
    if (st) *st = loc;
    return status;
}

}  // namespace spai

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" int spai_gmres_ir(spai_handle* h, const spai_csr* A, const spai_precond* P, const double* b,
                             double* x, const spai_ir_params* p, spai_ir_stats* st) {
    return spai::gmres_ir_impl(h, A, P, b, x, p, st);
}

extern "C" int spai_gmres_ir_noalloc(spai_handle* h, const spai_csr* A, const spai_precond* P, const double* b,
                                     double* x, const spai_ir_params* p, spai_ir_stats* st) {
    if (!h) {
        spai::set_error("invalid argument: NULL handle");
        return SPAI_E_ARG;
    }
    void* ws = spai::noalloc_scratch(h->device);
    if (!ws) {
        spai::set_error("the no-allocation workspace of this device was not set up");
        return SPAI_E_INTERNAL;
    }
    h->no_alloc = true;
    const int rc = spai::gmres_ir_impl(h, A, P, b, x, p, st, ws, spai::NOALLOC_BYTES);
    h->no_alloc = false;
    return rc;
}

extern "C" int spai_residual(spai_handle* h, const spai_csr* A, const double* b, const double* x, double* r,
                             spai_prec u_r) {
    if (!h || !b || !x || !r) {
        spai::set_error("invalid argument: NULL argument");
        return SPAI_E_ARG;
    }
    int rc = spai::check_csr(A);
    if (rc) return rc;
    if (u_r != SPAI_DD && u_r != SPAI_FP64) {
        spai::set_error("invalid argument: u_r must be DD or FP64");
        return SPAI_E_ARG;
    }
    SPAI_HIP(hipSetDevice(h->device));
    rc = spai::launch_residual(h, A, b, x, r, u_r, h->stream);
    if (rc) return rc;
    SPAI_HIP(hipStreamSynchronize(h->stream));
    return SPAI_OK;
}

extern "C" int spai_precond_apply(spai_handle* h, const spai_precond* P, const double* w, double* y) {
    if (!h || !P || !w || !y) {
        spai::set_error("invalid argument: NULL argument");
        return SPAI_E_ARG;
    }
    SPAI_HIP(hipSetDevice(h->device));
    int rc = spai::launch_apply_P(h, P, w, y, h->stream);
    if (rc) return rc;
    SPAI_HIP(hipStreamSynchronize(h->stream));
    return SPAI_OK;
}

extern "C" int spai_precond_apply_uf(spai_handle* h, const spai_precond* P, const double* b, double* x0) {
    if (!h || !P || !b || !x0) {
        spai::set_error("invalid argument: NULL argument");
        return SPAI_E_ARG;
    }
    SPAI_HIP(hipSetDevice(h->device));
    int rc = spai::launch_x0(P, b, x0, h->stream);
    if (rc) return rc;
    SPAI_HIP(hipStreamSynchronize(h->stream));
    return SPAI_OK;
}

extern "C" int spai_spmv(spai_handle* h, const spai_csr* A, const double* x, double* y) {
    if (!h || !x || !y) {
        spai::set_error("invalid argument: NULL argument");
        return SPAI_E_ARG;
    }
    int rc = spai::check_csr(A);
    if (rc) return rc;
    SPAI_HIP(hipSetDevice(h->device));
    rc = spai::launch_spmv(h, A, x, y, h->stream);
    if (rc) return rc;
    SPAI_HIP(hipStreamSynchronize(h->stream));
    return SPAI_OK;
}
