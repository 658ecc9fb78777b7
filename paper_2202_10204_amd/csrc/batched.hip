// Many independent systems in one call (SPAI-GMRES-IR, Algorithms 1 and 3,
// applied to each system on its own).
//
// A batch is one block-diagonal matrix: system s owns rows and columns
// sys_ptr[s] .. sys_ptr[s+1]-1.  The SPAI build of a block-diagonal matrix is
// the build of each block (a column's shadow, candidates and residual never
// leave its block), so the batched build is one build over all columns.  The
// solve is not: every system has its own Krylov space, iteration counts and
// stopping decisions.  One persistent launch does all of them: each workgroup
// takes the next system from a work counter (largest systems first) and runs
// the whole refinement loop of that system -- x0 = P b in u_f, residuals in
// double-double, left-preconditioned MGS-GMRES in FP64 with workgroup-level
// reductions, back substitution and update -- before taking the next one.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "common.hpp"
#include "device_math.hpp"

namespace spai {

int build_impl(spai_handle* h, const spai_csr* A, const spai_pattern* J, const spai_build_params* p,
               spai_precond** P_out, spai_build_stats* st);

namespace {

constexpr int BT = 256;          // threads per workgroup (4 waves)
constexpr int BW = BT / 64;

// row -> system by binary search in sys_ptr; flags an entry outside the block
__global__ void k_check_blocks(int n, int nsys, const int* __restrict__ sys_ptr, const int* __restrict__ rp,
                               const int* __restrict__ ci, int* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int lo = 0, hi = nsys;                // sys_ptr[lo] <= i < sys_ptr[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (sys_ptr[mid] <= i) lo = mid;
        else hi = mid;
    }
    const int r0 = sys_ptr[lo], r1 = sys_ptr[lo + 1];
    for (int q = rp[i]; q < rp[i + 1]; ++q)
        if (ci[q] < r0 || ci[q] >= r1) atomicOr(bad, 1);
}

struct BatchArgs {
    int nsys;
    const int* order;      // systems in processing order
    const int* sys_ptr;    // nsys + 1
    const int* rp;         // A (block diagonal, global indices)
    const int* ci;
    const double* av;
    const int* pp;         // P = M^T D, same blocks
    const int* pc;
    const void* pv;
    const double* d;
    const double* b;
    double* x;
    const double* x_true;  // exact solution for the forward error (NULL: none)
    int x_given;           // x holds the first iterate (no x0 = P b)
    double tau;
    double tol_ir;
    int imax;
    int maxit;
    int dd;                // residual in double-double (1) or FP64 (0)
    int kmax;              // Krylov dimension the workspace holds
    double* ws;            // per-workgroup slots
    size_t slot;           // doubles per slot
    int cap_n;             // largest system
    int* next;             // work counter
    spai_ir_stats* stats;  // per system
};

// sum over the workgroup; every thread gets the same bits.  The wave totals go
// to one of two buffers in turn (par, flipped here), so one barrier suffices:
// the next sum writes the other buffer, and this one is written again only
// after every thread has passed the next sum's barrier, past its reads here.
template <typename TW>
__device__ __forceinline__ TW wg_sum(TW v, TW* sh2, int& par) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    TW* sh = sh2 + par * BW;
    par ^= 1;
    v = wave_sum(v);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    TW t = 0;
#pragma unroll
    for (int w = 0; w < BW; ++w) t += sh[w];
    return t;
}

template <typename TW>
__device__ __forceinline__ TW wg_max(TW v, TW* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    TW t = 0;
#pragma unroll
    for (int w = 0; w < BW; ++w) t = fmax(t, sh[w]);
    __syncthreads();
    return t;
}

__device__ __forceinline__ float tw_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double tw_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float tw_sqrt(float a) { return __builtin_sqrtf(a); }
__device__ __forceinline__ double tw_sqrt(double a) { return __builtin_sqrt(a); }
template <typename TW, typename T> __device__ __forceinline__ TW to_tw(T v) {
    if constexpr (sizeof(TW) == 8) return to_f64(v);
    else return to_f32(v);
}

// The entry loops of a row are unrolled by 4 so that four entries' index,
// value and gather loads are in flight together; the sums keep their order (the
// same bits).  Measured on the 4096-system batch: the solve 133.0 -> 109.8 ms
// (products and residual; 111.1 with the products alone, 118.1 unrolled by 8).

// y_i = sum_q m_q (d_j w_j) over row i of P in the working precision TW (d
// rounded to TW; rows r0 + i, columns global)
template <int VP, typename TW>
__device__ __forceinline__ TW p_row(const BatchArgs& a, int gi, const TW* w) {
    using T = typename ValType<VP>::T;
    const T* pv = (const T*)a.pv;
    TW s = 0;
#pragma unroll 4
    for (int q = a.pp[gi]; q < a.pp[gi + 1]; ++q) {
        const int j = a.pc[q];
        s = tw_fma(to_tw<TW>(pv[q]), (TW)a.d[j] * w[j], s);
    }
    return s;
}

// r_i = b_i - (A x)_i of global row gi in u_r, before its rounding to the
// working precision: double-double rounded to FP64 (dd), else FP64 fused
// multiply-adds in CSR order (with u = FP32: A and b as rounded to binary32).
template <bool U32>
__device__ __forceinline__ double resid_row(const BatchArgs& a, int gi, const double* x) {
    if (a.dd) {
        double shi = a.b[gi], slo = 0.0;
#pragma unroll 4
        for (int q = a.rp[gi]; q < a.rp[gi + 1]; ++q) {
            const double av = a.av[q], xv = x[a.ci[q]];
            const double ph = av * xv;
            const double pl = __builtin_fma(av, xv, -ph);
            dd_add(shi, slo, -ph, -pl, shi, slo);
        }
        return shi + slo;
    }
    double acc = U32 ? (double)(float)a.b[gi] : a.b[gi];
#pragma unroll 4
    for (int q = a.rp[gi]; q < a.rp[gi + 1]; ++q) {
        const double av = U32 ? (double)(float)a.av[q] : a.av[q];
        acc = __builtin_fma(-av, x[a.ci[q]], acc);
    }
    return acc;
}

__device__ __forceinline__ double wg_max_d(double v, double* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < BW; ++w) t = fmax(t, sh[w]);
    __syncthreads();
    return t;
}

// One system's whole refinement loop in working precision TW (double: u = FP64;
// float: u = FP32, where A, b, the scaling, r, the basis, H, the rotations, d
// and x are binary32 values and the residual is evaluated in binary64).  VP is
// the storage format of P's values, UF the precision of its build (x0 rounds
// D b to it).
template <int VP, typename TW, int UF>
__device__ void solve_system(const BatchArgs& a, int s, double* ws_d, TW* sh, TW* sh2, double* shd,
                             spai_ir_stats& st) {
    using T = typename ValType<VP>::T;
    constexpr bool U32 = sizeof(TW) == 4;
    const int t = threadIdx.x;
    const int r0 = a.sys_ptr[s], n = a.sys_ptr[s + 1] - r0;
    const int mx = min(a.maxit, n);
    const int ld = mx + 1;
    // slot layout (in TW): V [n x (mx+1)] (column stride n), H [ld x mx], cs, sn, g, yk [ld], r, w, y [cap_n]
    TW* ws = (TW*)ws_d;
    TW* V = ws;
    TW* H = V + (size_t)a.cap_n * (a.kmax + 1);
    TW* cs = H + (size_t)(a.kmax + 1) * a.kmax;
    TW* sn = cs + (a.kmax + 1);
    TW* g = sn + (a.kmax + 1);
    TW* yk = g + (a.kmax + 1);
    TW* r = yk + (a.kmax + 1) - r0;   // indexed by global row
    TW* w = r + a.cap_n;
    TW* y = w + a.cap_n;
    double* x = a.x;
    if (t == 0) {                             // statistics of this system (LDS, written by thread 0)
        st.steps = 0;
        st.total_its = 0;
        st.status = 0;
        for (int q = 0; q < 32; ++q) {
            st.its[q] = 0;
            st.gest[q] = 0.0;
            st.dnorm[q] = 0.0;
        }
    }
    // x0 = P b in u_f (products and sums in the arithmetic precision of u_f, column order), stored in u;
    // or the given first iterate (as rounded to u)
    for (int i = t; i < n; i += BT) {
        const int gi = r0 + i;
        if (a.x_given) {
            if constexpr (U32) x[gi] = (double)(float)x[gi];
        } else if constexpr (VP == SPAI_FP64) {
            double acc = 0.0;
            for (int q = a.pp[gi]; q < a.pp[gi + 1]; ++q) {
                const int j = a.pc[q];
                acc = __builtin_fma(((const double*)a.pv)[q], a.d[j] * a.b[j], acc);
            }
            x[gi] = acc;
        } else {
            const T* pv = (const T*)a.pv;
            float acc = 0.0f;
            for (int q = a.pp[gi]; q < a.pp[gi + 1]; ++q) {
                const int j = a.pc[q];
                const float z = store<UF, float>((float)(a.d[j] * a.b[j]));
                acc = __builtin_fmaf(to_f32(pv[q]), z, acc);
            }
            x[gi] = (double)acc;
        }
    }
    __syncthreads();
    TW dprev = INFINITY;
    int status = 0;
    int par = 0;                              // buffer of the next workgroup sum
    for (int step = 0; step < a.imax; ++step) {
        // r = b - A x in u_r, stored in u (A and b as stored in u)
        for (int i = t; i < n; i += BT) r[r0 + i] = (TW)resid_row<U32>(a, r0 + i, x);
        __syncthreads();
        // z = P r into V(:, 0); beta0 = ||z||
        TW part = 0;
        for (int i = t; i < n; i += BT) {
            const TW z = p_row<VP, TW>(a, r0 + i, r);
            V[i] = z;
            part = tw_fma(z, z, part);
        }
        const TW beta0 = tw_sqrt(wg_sum(part, sh2, par));
        if (beta0 == (TW)0) break;           // P r_i = 0: x_i solves the system
        if (t == 0) st.steps = step + 1;
        for (int i = t; i < n; i += BT) V[i] = V[i] / beta0;
        for (int l = t; l <= mx; l += BT) g[l] = l == 0 ? beta0 : (TW)0;
        __syncthreads();
        int k = 0, capped = 0;
        TW gk = beta0;
        for (int jj = 0; jj < mx; ++jj) {
            const TW* vj = V + (size_t)jj * n;
            // w = A v_j (global rows, the system's columns), A as stored in u
            for (int i = t; i < n; i += BT) {
                const int gi = r0 + i;
                TW acc = 0;
#pragma unroll 4
                for (int q = a.rp[gi]; q < a.rp[gi + 1]; ++q) acc = tw_fma((TW)a.av[q], vj[a.ci[q] - r0], acc);
                w[gi] = acc;
            }
            __syncthreads();
            for (int i = t; i < n; i += BT) y[r0 + i] = p_row<VP, TW>(a, r0 + i, w);
            // modified Gram-Schmidt: h_lj = <y, v_l>, y -= h_lj v_l, l = 0 .. jj, then
            // ||y||.  The update by v_l and the partial inner product with v_{l+1}
            // (with y itself after the last projection) share one pass over the
            // rows: the same operations in the same order as separate passes.
            TW* Hc = H + (size_t)jj * ld;
            TW p = 0;
            for (int i = t; i < n; i += BT) p = tw_fma(y[r0 + i], V[i], p);
            for (int l = 0; l <= jj; ++l) {
                const TW* vl = V + (size_t)l * n;
                const TW hl = wg_sum(p, sh2, par);
                if (t == 0) Hc[l] = hl;
                p = 0;
                if (l < jj) {
                    const TW* vn = vl + n;
                    for (int i = t; i < n; i += BT) {
                        const TW yi = tw_fma(-hl, vl[i], y[r0 + i]);
                        y[r0 + i] = yi;
                        p = tw_fma(yi, vn[i], p);
                    }
                } else {
                    for (int i = t; i < n; i += BT) {
                        const TW yi = tw_fma(-hl, vl[i], y[r0 + i]);
                        y[r0 + i] = yi;
                        p = tw_fma(yi, yi, p);
                    }
                }
            }
            const TW hn = tw_sqrt(wg_sum(p, sh2, par));
            TW* vn = V + (size_t)(jj + 1) * n;
            for (int i = t; i < n; i += BT) vn[i] = y[r0 + i] / hn;
            if (t == 0) {
                // previous rotations, new rotation, g update
                Hc[jj + 1] = hn;
                for (int l = 0; l < jj; ++l) {
                    const TW x0 = Hc[l], x1 = Hc[l + 1];
                    Hc[l] = cs[l] * x0 + sn[l] * x1;
                    Hc[l + 1] = -sn[l] * x0 + cs[l] * x1;
                }
                const TW delta = hypot(Hc[jj], Hc[jj + 1]);
                const TW c = Hc[jj] / delta, sv = Hc[jj + 1] / delta;
                Hc[jj] = delta;
                Hc[jj + 1] = 0;
                const TW gj = g[jj];
                g[jj + 1] = -sv * gj;
                g[jj] = c * gj;
                cs[jj] = c;
                sn[jj] = sv;
                sh[BW] = fabs(-sv * gj);
            }
            __syncthreads();
            gk = sh[BW];
            k = jj + 1;
            __syncthreads();
            if (gk <= (TW)a.tau * beta0 || hn == (TW)0) break;
            if (jj + 1 == mx) {
                capped = 1;
                break;
            }
        }
        if (capped) status |= SPAI_W_MAXIT;
        // back substitution H(0:k, 0:k) yk = g(0:k)
        if (t == 0) {
            for (int c = k - 1; c >= 0; --c) {
                TW acc = g[c];
                for (int c2 = c + 1; c2 < k; ++c2) {
                    if constexpr (U32) acc = tw_fma(-H[(size_t)c2 * ld + c], yk[c2], acc);
                    else acc -= H[(size_t)c2 * ld + c] * yk[c2];
                }
                yk[c] = acc / H[(size_t)c * ld + c];
            }
        }
        __syncthreads();
        // d = V_k yk, x += d (in u)
        TW dm = 0, xm = 0;
        for (int i = t; i < n; i += BT) {
            TW di = 0;
            for (int c = 0; c < k; ++c) di = tw_fma(V[(size_t)c * n + i], yk[c], di);
            const TW xi = (TW)x[r0 + i] + di;
            x[r0 + i] = (double)xi;
            dm = fmax(dm, fabs(di));
            xm = fmax(xm, fabs(xi));
        }
        const TW dn = wg_max(dm, sh), xn = wg_max(xm, sh);
        if (t == 0) {
            st.its[step] = k;                 // imax <= 32
            st.gest[step] = (double)(gk / beta0);
            st.dnorm[step] = (double)dn;
            st.total_its += k;
        }
        if ((double)dn <= a.tol_ir * (double)xn) break;
        if (step >= 2 && dn > (TW)0.5 * dprev) {
            status |= SPAI_W_NOCONV;
            break;
        }
        dprev = dn;
        if (step == a.imax - 1) status |= SPAI_W_NOCONV;
    }
    // errors of the returned x (Theorems 1 and 2): residual in u_r, norms in FP64
    {
        double rm = 0.0, am = 0.0, xm = 0.0, bm = 0.0, em = 0.0, tm = 0.0;
        for (int i = t; i < n; i += BT) {
            const int gi = r0 + i;
            rm = fmax(rm, fabs(resid_row<U32>(a, gi, x)));
            double rs = 0.0;
            for (int q = a.rp[gi]; q < a.rp[gi + 1]; ++q) rs += fabs(U32 ? (double)(float)a.av[q] : a.av[q]);
            am = fmax(am, rs);
            xm = fmax(xm, fabs(x[gi]));
            bm = fmax(bm, fabs(U32 ? (double)(float)a.b[gi] : a.b[gi]));
            if (a.x_true) {
                em = fmax(em, fabs(x[gi] - a.x_true[gi]));
                tm = fmax(tm, fabs(a.x_true[gi]));
            }
        }
        rm = wg_max_d(rm, shd);
        am = wg_max_d(am, shd);
        xm = wg_max_d(xm, shd);
        bm = wg_max_d(bm, shd);
        em = wg_max_d(em, shd);
        tm = wg_max_d(tm, shd);
        if (t == 0) {
            const double den = am * xm + bm;
            st.nbe = den > 0.0 ? rm / den : 0.0;
            st.ferr = a.x_true ? (tm > 0.0 ? em / tm : em) : -1.0;
        }
    }
    if (t == 0) {
        st.status = status;
        a.stats[s] = st;
    }
    __syncthreads();
}

template <int VP, typename TW, int UF = VP>
__global__ __launch_bounds__(BT) void k_gmres_ir_batched(BatchArgs a) {
    __shared__ TW sh[BW + 2];
    __shared__ TW sh2[2 * BW];               // the workgroup sums' two buffers
    __shared__ double shd[BW];
    __shared__ int sys;
    __shared__ spai_ir_stats st;
    double* ws = a.ws + (size_t)blockIdx.x * a.slot;
    while (true) {
        if (threadIdx.x == 0) sys = atomicAdd(a.next, 1);
        __syncthreads();
        const int q = sys;
        __syncthreads();
        if (q >= a.nsys) break;
        solve_system<VP, TW, UF>(a, a.order[q], ws, sh, sh2, shd, st);
    }
}

}  // namespace

// Validation of a batch description against the matrix (host sys_ptr).
static int check_batch(const spai_csr* A, int32_t nsys, const int32_t* sys_ptr) {
    SPAI_ARG(A && A->n > 0 && A->rowptr && A->col && A->val, "bad matrix");
    SPAI_ARG(nsys >= 1 && sys_ptr, "nsys must be positive and sys_ptr given");
    SPAI_ARG(sys_ptr[0] == 0 && sys_ptr[nsys] == A->n, "sys_ptr must run from 0 to n");
    for (int s = 0; s < nsys; ++s) SPAI_ARG(sys_ptr[s + 1] > sys_ptr[s], "every system needs at least one row");
    return SPAI_OK;
}

// Copies sys_ptr to the device and checks that A has no entry outside the
// diagonal blocks.
static int upload_and_check_blocks(spai_handle* h, const spai_csr* A, int32_t nsys, const int32_t* sys_ptr,
                                   int** d_sys_ptr) {
    int rc = buffer_reserve(h, h->ws[WS_MISC], sizeof(int) * ((size_t)nsys + 1 + 64));
    if (rc) return rc;
    int* dsp = (int*)h->ws[WS_MISC].ptr;
    int* bad = dsp + nsys + 1;
    hipStream_t s = h->stream;
    SPAI_HIP(hipMemcpyAsync(dsp, sys_ptr, sizeof(int) * ((size_t)nsys + 1), hipMemcpyHostToDevice, s));
    SPAI_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_check_blocks, dim3((A->n + 255) / 256), dim3(256), 0, s, A->n, (int)nsys,
                       (const int*)dsp, A->rowptr, A->col, bad);
    SPAI_HIP(hipGetLastError());
    int hbad = 0;
    SPAI_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    SPAI_HIP(hipStreamSynchronize(s));
    SPAI_ARG(hbad == 0, "the matrix has an entry outside the diagonal blocks given by sys_ptr");
    *d_sys_ptr = dsp;
    return SPAI_OK;
}

int build_batched_impl(spai_handle* h, const spai_csr* A, int32_t nsys, const int32_t* sys_ptr,
                       const spai_pattern* J, const spai_build_params* p, spai_precond** P_out,
                       spai_build_stats* st) {
    SPAI_ARG(h && P_out, "NULL handle or output");
    *P_out = nullptr;
    int rc = check_batch(A, nsys, sys_ptr);
    if (rc) return rc;
    SPAI_HIP(hipSetDevice(h->device));
    int* dsp = nullptr;
    rc = upload_and_check_blocks(h, A, nsys, sys_ptr, &dsp);
    if (rc) return rc;
    return build_impl(h, A, J, p, P_out, st);
}

int gmres_ir_batched_impl(spai_handle* h, const spai_csr* A, const spai_precond* P, int32_t nsys,
                          const int32_t* sys_ptr, const double* b, double* x, const spai_ir_params* prm,
                          spai_ir_stats* st) {
    SPAI_ARG(h && prm && st, "NULL handle, parameters or statistics");
    SPAI_ARG(P, "NULL preconditioner");
    SPAI_ARG(b && x, "NULL right-hand side or solution");
    int rc = check_batch(A, nsys, sys_ptr);
    if (rc) return rc;
    SPAI_ARG(P->n == A->n, "preconditioner size differs from the matrix");
    SPAI_ARG(prm->imax >= 1 && prm->imax <= 32, "imax must lie in 1..32");
    SPAI_ARG(prm->maxit >= 1, "maxit must be positive");
    SPAI_ARG(prm->tau >= 0.0, "tau must be non-negative");
    SPAI_ARG(prm->u_r == SPAI_DD || prm->u_r == SPAI_FP64, "u_r must be DD or FP64");
    SPAI_ARG(prm->ortho == SPAI_ORTHO_MGS, "the batched solver orthogonalises with MGS");
    SPAI_ARG(P->side == SPAI_LEFT, "the batched solver applies left preconditioners");
    SPAI_ARG(prm->u == SPAI_FP64 || prm->u == SPAI_FP32, "the working precision u must be FP64 or FP32");
    if (prm->u == SPAI_FP32) {
        SPAI_ARG(prm->u_r == SPAI_FP64, "with working precision FP32 the residual precision must be FP64");
        SPAI_ARG(P->u_f != SPAI_FP64, "u_f must not be finer than the working precision");
    }
    SPAI_HIP(hipSetDevice(h->device));
    hipStream_t s = h->stream;
    int* dsp = nullptr;
    rc = upload_and_check_blocks(h, A, nsys, sys_ptr, &dsp);
    if (rc) return rc;
    {   // P must have the same blocks (its rows gather only inside their system)
        const spai_csr pc{P->n, (int32_t)std::min<int64_t>(P->nnz, INT32_MAX), P->rowptr, P->col, nullptr};
        int* bad = dsp + nsys + 1;
        SPAI_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
        hipLaunchKernelGGL(k_check_blocks, dim3((P->n + 255) / 256), dim3(256), 0, s, P->n, (int)nsys,
                           (const int*)dsp, pc.rowptr, pc.col, bad);
        SPAI_HIP(hipGetLastError());
        int hbad = 0;
        SPAI_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        SPAI_HIP(hipStreamSynchronize(s));
        SPAI_ARG(hbad == 0, "the preconditioner has an entry outside the diagonal blocks given by sys_ptr");
    }

    // largest systems first
    std::vector<int> order(nsys);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int u, int v) {
        return sys_ptr[u + 1] - sys_ptr[u] > sys_ptr[v + 1] - sys_ptr[v];
    });
    const int cap_n = sys_ptr[order[0] + 1] - sys_ptr[order[0]];
    const int kmax = std::min(prm->maxit, cap_n);
    const size_t slot = (size_t)cap_n * (kmax + 1) + (size_t)(kmax + 1) * kmax + 4 * (size_t)(kmax + 1) +
                        3 * (size_t)cap_n + 64;
    // workgroups: four per CU (16 waves hide the gathers' latency better: the
    // 4096-system batch solve 100 ms against 110 with two per CU, 99 with
    // eight), fewer when the slots would take more than a quarter of free
    // memory (or more than the handle's workspace cap)
    size_t free_b = 0, total_b = 0;
    SPAI_HIP(hipMemGetInfo(&free_b, &total_b));
    long long g = std::min<long long>(nsys, 4LL * h->num_cu);
    const size_t room = h->ws_cap ? std::min(free_b / 4, h->ws_cap) : free_b / 4;
    const long long fit = (long long)(room / (slot * sizeof(double)));
    g = std::max(1LL, std::min(g, fit));

    rc = buffer_reserve(h, h->ws[WS_SPARE], sizeof(double) * slot * (size_t)g);
    if (rc) return rc;
    rc = buffer_reserve(h, h->ws[WS_SOLVE_VEC],
                        sizeof(int) * ((size_t)nsys + 64) + sizeof(spai_ir_stats) * (size_t)nsys + 256);
    if (rc) return rc;
    int* dorder = (int*)h->ws[WS_SOLVE_VEC].ptr;
    int* next = dorder + nsys;
    spai_ir_stats* dst = (spai_ir_stats*)(((uintptr_t)(next + 64) + 255) & ~(uintptr_t)255);
    SPAI_HIP(hipMemcpyAsync(dorder, order.data(), sizeof(int) * (size_t)nsys, hipMemcpyHostToDevice, s));
    SPAI_HIP(hipMemsetAsync(next, 0, sizeof(int), s));

    BatchArgs a{};
    a.nsys = nsys;
    a.order = dorder;
    a.sys_ptr = dsp;
    a.rp = A->rowptr;
    a.ci = A->col;
    a.av = A->val;
    a.pp = P->rowptr;
    a.pc = P->col;
    a.pv = P->val;
    a.d = P->d;
    a.b = b;
    a.x = x;
    a.x_true = prm->x_true;
    a.x_given = prm->x_given ? 1 : 0;
    a.tau = prm->tau;
    a.tol_ir = prm->tol_ir;
    a.imax = prm->imax;
    a.maxit = prm->maxit;
    a.dd = prm->u_r == SPAI_DD;
    a.kmax = kmax;
    a.ws = (double*)h->ws[WS_SPARE].ptr;
    a.slot = slot;
    a.cap_n = cap_n;
    a.next = next;
    a.stats = dst;
    long tk = timer_begin(h, SPAI_KT_MGS);
    const dim3 grid((unsigned)g), blk(BT);
    // P's storage format and the precision of its build (FP32 values of a
    // 16-bit build whose overflowing columns were recomputed in FP32)
    const int vf = P->val_prec == SPAI_FP32 && (P->u_f == SPAI_FP16 || P->u_f == SPAI_BF16) ? 10 + P->u_f
                 : P->val_prec;
    if (prm->u == SPAI_FP32) {
        switch (vf) {
        case SPAI_FP32: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP32, float>), grid, blk, 0, s, a); break;
        case SPAI_FP16: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP16, float>), grid, blk, 0, s, a); break;
        case SPAI_BF16: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_BF16, float>), grid, blk, 0, s, a); break;
        case 10 + SPAI_FP16: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP32, float, SPAI_FP16>), grid, blk, 0, s, a); break;
        default: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP32, float, SPAI_BF16>), grid, blk, 0, s, a); break;
        }
    } else {
        switch (vf) {
        case SPAI_FP64: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP64, double>), grid, blk, 0, s, a); break;
        case SPAI_FP32: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP32, double>), grid, blk, 0, s, a); break;
        case SPAI_FP16: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP16, double>), grid, blk, 0, s, a); break;
        case SPAI_BF16: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_BF16, double>), grid, blk, 0, s, a); break;
        case 10 + SPAI_FP16: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP32, double, SPAI_FP16>), grid, blk, 0, s, a); break;
        default: hipLaunchKernelGGL((k_gmres_ir_batched<SPAI_FP32, double, SPAI_BF16>), grid, blk, 0, s, a); break;
        }
    }
    timer_end(h, SPAI_KT_MGS, tk);
    SPAI_HIP(hipGetLastError());
    SPAI_HIP(hipMemcpyAsync(st, dst, sizeof(spai_ir_stats) * (size_t)nsys, hipMemcpyDeviceToHost, s));
    SPAI_HIP(hipStreamSynchronize(s));
    int status = 0;
    for (int q = 0; q < nsys; ++q) status |= st[q].status;
    return status;
}

}  // namespace spai

extern "C" int spai_build_batched(spai_handle* h, const spai_csr* A, int32_t nsys, const int32_t* sys_ptr,
                                  const spai_pattern* J, const spai_build_params* p, spai_precond** P,
                                  spai_build_stats* st) {
    return spai::build_batched_impl(h, A, nsys, sys_ptr, J, p, P, st);
}

extern "C" int spai_gmres_ir_batched(spai_handle* h, const spai_csr* A, const spai_precond* P, int32_t nsys,
                                     const int32_t* sys_ptr, const double* b, double* x,
                                     const spai_ir_params* p, spai_ir_stats* st) {
    return spai::gmres_ir_batched_impl(h, A, P, nsys, sys_ptr, b, x, p, st);
}
