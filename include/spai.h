/*
 * libspai — SPAI-GMRES-IR on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the GPU library.  The method is the one of Carson & Khan, "Mixed
 * precision iterative refinement with sparse approximate inverse
 * preconditioning": a Frobenius-norm sparse approximate inverse built column by
 * column (Algorithm 1, Section 2.2) and used as the left preconditioner of
 * GMRES-based iterative refinement in five precisions (Algorithm 3,
 * Section 3.2).
 *
 * Conventions for every entry point
 *   - Matrices are CSR with int32 indices, columns sorted ascending within a
 *     row, no duplicate entries, FP64 values; every row must hold a nonzero
 *     value (the column scaling of Section 4 divides by the row's largest
 *     magnitude).  A stored zero is allowed and treated as a structural entry.
 *   - Pointers named "device" point to device memory of the handle's device and
 *     stay owned by the caller; they must stay valid and unmodified until the
 *     call returns.  Host structs are read during the call only.
 *   - Every call enqueues its work on the handle's stream and returns after that
 *     work has completed (the calls need small device-to-host copies for sizes,
 *     statistics and stopping decisions).  Calls on one handle must not overlap.
 *   - Return value: 0 on success; a negative SPAI_E_* code on a hard error (no
 *     output is produced, spai_last_error() describes it); a positive bit mask
 *     of SPAI_W_* warnings when the result was produced but is flagged.
 */
#ifndef SPAI_H
#define SPAI_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Floating-point formats (Table 1 of the paper lists half, single, double, quad). */
typedef enum {
    SPAI_FP64 = 0,
    SPAI_FP32 = 1,
    SPAI_FP16 = 2, /* storage format; arithmetic in FP32 */
    SPAI_BF16 = 3, /* storage format; arithmetic in FP32 */
    SPAI_DD = 4    /* double-double (residual precision u_r only) */
} spai_prec;

enum {
    SPAI_OK = 0,
    SPAI_E_ARG = -1,      /* bad shape, pointer, parameter or CSR structure */
    SPAI_E_OOM = -2,      /* device allocation failed */
    SPAI_E_HIP = -3,      /* a HIP runtime call failed (message has the error) */
    SPAI_E_INTERNAL = -4, /* a device-side consistency check failed */
    SPAI_W_EPS = 1,       /* some columns end with ||e_k - B m_k|| > eps (alpha or fill cap hit) */
    SPAI_W_RANKDEF = 2,   /* a reduced problem was rank deficient (zero Householder norm) */
    SPAI_W_NONFINITE = 4, /* a column is non-finite even after its FP32 recomputation (see spai_build) */
    SPAI_W_MAXIT = 8,     /* some GMRES solve hit maxit */
    SPAI_W_NOCONV = 16    /* refinement stopped at imax or on stagnation */
};

typedef struct spai_handle spai_handle;
typedef struct spai_precond spai_precond;

/* Sparse matrix in CSR, device arrays (rowptr: n+1, col and val: nnz). */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t* rowptr;
    const int32_t* col;
    const double* val;
} spai_csr;

/* Prescribed initial sparsity pattern J (Algorithm 1 input): column k of M has
 * row indices idx[ptr[k] .. ptr[k+1]) (device arrays; any order, no duplicates).
 * Since P = M^T D, these are the column indices of row k of P.  Passing NULL
 * instead of a pattern means the identity pattern (Section 4). */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t* ptr;
    const int32_t* idx;
} spai_pattern;

/* Parameters of Algorithm 1 (its Require line: J, alpha, beta, eps) plus the fill
 * cap of Section 2.2 and the precision u_f of Section 3.1. */
enum { SPAI_LEFT = 0, SPAI_RIGHT = 1 };

typedef struct {
    double eps;      /* column residual tolerance: stop once ||e_k - B m_k||_2 <= eps */
    int32_t alpha;   /* maximum augmentation steps per column (0 = fixed pattern) */
    int32_t beta;    /* maximum indices added per augmentation step */
    int32_t maxfill; /* cap on |J_k| (never truncates the initial pattern) */
    spai_prec u_f;   /* FP64, FP32, FP16 or BF16 */
    int32_t side;    /* SPAI_LEFT (0, default): Algorithm 1 on B = A^T D, P = M^T D, the left
                        preconditioner of Algorithm 3.  SPAI_RIGHT: Algorithm 1 on B = A D with
                        D = diag(1 / max_i |a_ij|) (columns of A scaled to unit maximum), so that
                        A P ~ I with P = D M; spai_gmres_ir then preconditions on the right. */
    int32_t qr_update; /* 0 (default): each augmentation step factors the reduced problem from
                          scratch; 1: the QR of the previous step is updated (its reflectors
                          are applied to the new columns only, Section 2.2's remark), which
                          keeps the factorisation in LDS through the candidate phase: fewer
                          operations, less LDS left for other columns.  Both give the same
                          bits (the shadow rows are kept in insertion order, so the columns
                          factored earlier are zero in the rows an augmentation adds). */
    int32_t kernel_cfg; /* column-kernel configuration: 0 (default) = the library's rule
                           (the smallest configuration holding max(maxfill, longest initial
                           column), with a sampled choice between the two 20-index shapes;
                           when u_f is FP32, FP16 or BF16 the small-shadow 20-index shape
                           and the 31-index shape are the register ones, ids 7 and 9);
                           1..SPAI_KCFG_COUNT = that configuration (spai_column_config), which
                           must hold max(maxfill, longest initial column) indices, else
                           SPAI_E_ARG.  Every configuration gives the same bits: a column that
                           outgrows a configuration's shadow, gather or candidate space is
                           recomputed from scratch by a larger one (after a configuration of
                           at most 21 lanes, an internal 21-lane stage with 96 shadow rows,
                           then the largest configuration).  The choice is a
                           performance choice, made by spai_tune_build's measurements. */
} spai_build_params;

/* Column-kernel configurations of Algorithm 1's per-column solver: `lanes` lanes
 * of a wavefront per column problem (64 / lanes problems per wavefront), at most
 * `maxp` = lanes - 1 indices in J_k, `maxm` shadow rows I_k, `emax` gathered
 * entries of B(:, J_k) and `cmax` raw augmentation candidates staged in LDS.
 * Ids 1-6 keep the reduced matrix A-bar in LDS; ids 7-9 keep it in registers
 * (lane c holds column c) when u_f is FP32, FP16 or BF16 (with u_f = FP64 they
 * run as the LDS shapes): 7 and 8 have the shapes of 3 and 4, 9 that of 5 with
 * 256 candidates.  All give the same bits. */
enum { SPAI_KCFG_COUNT = 9 };
typedef struct {
    int32_t lanes, maxp, maxm, emax, cmax, problems_per_wave;
    int32_t lds_bytes_per_problem; /* for u_f = FP32 with qr_update = 0 */
} spai_column_config;
/* Description of configuration id (1..SPAI_KCFG_COUNT); SPAI_E_ARG otherwise. */
int spai_column_config_get(int32_t id, spai_column_config* out);

/*
 * Autotuning measurement for spai_build: runs the build's preprocessing for
 * (A, J, p) and then, for every configuration id able to hold the pattern
 * (maxp >= max(maxfill, longest initial column)) and for qr_update 0 and 1, the
 * column phase over a strided sample of min(sample, n) columns (the columns
 * sample_k = k * floor(n / count)), including the recomputation of the columns
 * it defers, `reps` times after one untimed run; writes the fastest time per
 * sampled column in nanoseconds to ns_per_col[2 * (id - 1) + qr_update] (host
 * array of 2 * SPAI_KCFG_COUNT doubles; -1 for a configuration that cannot
 * hold the pattern).  p->kernel_cfg and p->qr_update are ignored.  No
 * preconditioner is produced.  Errors as spai_build, plus SPAI_E_ARG for
 * sample < 1, reps < 1 or a NULL ns_per_col.
 */
int spai_tune_build(spai_handle* h, const spai_csr* A, const spai_pattern* J, const spai_build_params* p,
                    int32_t sample, int32_t reps, double* ns_per_col);

typedef struct {
    int64_t nnz;            /* stored entries of P (pattern entries, exact zeros included) */
    int32_t max_len;        /* largest |J_k| */
    int32_t max_steps;      /* largest number of augmentation steps of a column */
    int32_t max_shadow;     /* largest |I_k| at a final solve */
    int32_t cols_over_eps;  /* columns ending above eps */
    int32_t cols_rankdef;   /* columns with a rank-deficient reduced problem */
    int32_t cols_nonfinite; /* columns with a non-finite value */
    int32_t cols_deferred;  /* columns the first configuration deferred to a larger one */
    double max_res;         /* largest final column residual */
    int64_t nnz_numeric;    /* stored entries of P whose value is not zero (what the paper's tables
                               count as nnz of the preconditioner, Section 4) */
    int32_t cols_fallback;  /* FP16/BF16 columns recomputed in FP32 after a non-finite value */
    int32_t pad;
} spai_build_stats;

/* Read-only view of a preconditioner P = M^T D (device pointers owned by P).
 * Row k of P holds m_k: columns col[rowptr[k] .. rowptr[k+1]) ascending with
 * values val (format val_prec); P w = M^T (D w) with d the FP64 scaling.
 * j_ins / m_ins expose the build's per-column result before sorting: column k's
 * indices J_k in insertion order (stride entries, -1 padded) with their values
 * as FP64; steps / res / flags are the per-column statistics (NULL for an
 * imported P). */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int32_t* rowptr;
    const int32_t* col;
    const void* val;
    spai_prec val_prec;
    const double* d;
    int32_t stride;
    const int32_t* j_ins;
    const double* m_ins;
    const int32_t* len;
    const int32_t* steps;
    const double* res;
    const int32_t* flags;
    int32_t side;          /* SPAI_LEFT: row k holds m_k, P w = M^T (D w); SPAI_RIGHT: row i holds the
                              entries m_k[i] (columns k ascending), P w = D (M w) */
    spai_prec u_f;         /* the precision the build ran in; x0 = P b rounds D b (left) or b
                              (right) to it.  Equal to val_prec, except for an FP16/BF16 build with
                              recomputed columns, whose values are stored in FP32 */
} spai_precond_view;

/* Orthogonalisation of the Arnoldi vectors.  Algorithm 3 asks for GMRES; the
 * analysis of Section 3.2 uses modified Gram-Schmidt.  CGS2 (classical
 * Gram-Schmidt applied twice) spans the same Krylov space with orthogonality to
 * working precision and needs three global reductions per iteration instead of
 * j+2.  DCGS2 is CGS2 with the second projection and the normalisation of each
 * new vector delayed to the next iteration: one set of inner products per
 * iteration, reduced over the grid group by group of basis vectors while the
 * second pass trails the first, so that the basis streams from memory about
 * once per iteration; the stopping decision for iteration j is taken one
 * iteration later, so one extra product with P A is computed per solve.
 * Where at most 2 rows per thread suffice, the DCGS2 launch also forms the
 * iteration's second sparse product (P for left, A for right preconditioning)
 * at its own rows, so an iteration is two launches; the environment variable
 * SPAI_DCGS2_FUSE=0 (read at every solve) keeps that product a launch of its own
 * (same iterates up to the rounding order of that product's sums).
 * CGS2 and DCGS2 need the cooperative Arnoldi kernel (SPAI_E_ARG otherwise). */
enum { SPAI_ORTHO_MGS = 0, SPAI_ORTHO_CGS2 = 1, SPAI_ORTHO_DCGS2 = 2 };

/* Parameters of Algorithm 3 (its Require line: i_max, tau) plus the GMRES cap and
 * the refinement stopping rule, the residual precision u_r and the working
 * precision u = u_g = u_p (Section 4 uses u_g = u_p = u).
 * u = SPAI_FP64 (0, default): the precision set (u_f, double, u_r) of Table 3.
 * u = SPAI_FP32: the sets (half, single, double) and (single, single, double) of
 * Tables 4 and 5: A and b are used as rounded to binary32, x0, r_i (evaluated in
 * binary64, so u_r must be SPAI_FP64), the Krylov basis, the Hessenberg
 * matrix, d_i and x are binary32 values (x is returned as doubles), u_f must be
 * FP32, FP16 or BF16, and GMRES orthogonalises with MGS in one workgroup per
 * system (the batched solver's kernel; a single system runs as a batch of one). */
typedef struct {
    spai_prec u_r;  /* residual precision: SPAI_DD (double-double) or SPAI_FP64 */
    double tau;     /* GMRES stops when |g_{j+1}| <= tau ||P r_i||_2 */
    int32_t imax;   /* maximum refinement steps (<= 32) */
    int32_t maxit;  /* maximum GMRES iterations per step */
    double tol_ir;  /* refinement stops when ||d_i||_inf <= tol_ir ||x_{i+1}||_inf */
    int32_t ortho;  /* SPAI_ORTHO_MGS (0, default), SPAI_ORTHO_CGS2 or SPAI_ORTHO_DCGS2 */
    spai_prec u;    /* working precision: SPAI_FP64 (0, default) or SPAI_FP32 */
    int32_t graph;  /* DCGS2 only: 1 = each chunk of 8 Arnoldi steps (the operator's
                       sparse products and the orthogonalisation launch, per step) is one
                       HIP graph, built once per call and replayed; the kernels take the
                       step index from the device solver state.  Same results as 0
                       (stream launches, default); other orthogonalisations ignore it. */
    int32_t x_given;        /* 0 (default): start from x0 = P b in u_f (Algorithm 3).  1: x holds
                               the first iterate on entry (a warm start; with working precision
                               FP32 it is used as rounded to binary32) and refinement step 0 starts
                               from it */
    const double* x_true;   /* optional device array of n values: the exact solution, for the
                               forward error in the statistics (NULL: ferr is reported as -1) */
} spai_ir_params;

typedef struct {
    int32_t steps;      /* refinement steps taken */
    int32_t its[32];    /* GMRES iterations of each step */
    int32_t total_its;
    int32_t status;     /* SPAI_W_MAXIT | SPAI_W_NOCONV bits */
    double gest[32];    /* |g_{k+1}| / ||P r_i|| at the end of each step */
    double dnorm[32];   /* ||d_i||_inf of each step */
    double nbe;         /* normwise backward error of the returned x (Theorem 2):
                           ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf), residual in u_r */
    double ferr;        /* forward error ||x - x_true||_inf / ||x_true||_inf (Theorem 1), or -1
                           when x_true is NULL */
} spai_ir_stats;

/* Handle: binds the current HIP device, a stream (default: the null stream) and a
 * grow-only device workspace.  Destroy frees the workspace. */
int spai_create(spai_handle** h);
int spai_destroy(spai_handle* h);
int spai_set_stream(spai_handle* h, hipStream_t stream);

/* Thread-local description of the last error (never NULL). */
const char* spai_last_error(void);

/*
 * Device memory.  By default the library takes device memory with hipMalloc
 * and returns it with hipFree.  spai_set_allocator routes every later device
 * allocation of the library through the caller's functions instead (for
 * example a framework's caching allocator, so that one owner holds all device
 * memory):
 *   alloc(bytes, device, stream, ctx) returns device memory of at least
 *       `bytes` bytes on `device`, usable by work enqueued on `stream` (the
 *       stream the library will use it on), or NULL when none is available
 *       (the library call then fails with SPAI_E_OOM);
 *   free_(ptr, device, stream, ctx) takes back a block alloc returned, with
 *       the device and stream it was allocated for; work the library enqueued
 *       on that stream before the call may still be using it, so the block may
 *       only be reused for work ordered after that stream's pending work.
 * Every block is freed by the pair that allocated it, also after a later call
 * changed the allocator.  alloc = free_ = NULL restores hipMalloc/hipFree.
 * Process-wide; not to be called while another thread is inside a library
 * call.  Request servers take their arena (one block) through the same path.
 * Returns SPAI_E_ARG when exactly one of the two functions is NULL.
 */
typedef void* (*spai_alloc_fn)(size_t bytes, int device, hipStream_t stream, void* ctx);
typedef void (*spai_free_fn)(void* ptr, int device, hipStream_t stream, void* ctx);
int spai_set_allocator(spai_alloc_fn alloc, spai_free_fn free_, void* ctx);

/*
 * Build the left preconditioner P = M^T D (Algorithm 3, first line, with the
 * scaling of Section 4): D = diag(1 / max_j |a_ij|), Algorithm 1 runs on
 * B = A^T D from the initial pattern J (NULL = identity), and every column solves
 * min ||e_k - B(I_k, J_k) m|| by Householder QR in u_f, growing J_k by at most
 * beta candidates with the smallest scores rho_jk <= mean per step until the
 * residual is <= eps, alpha steps were taken or |J_k| reached maxfill.
 * On success *P receives a new preconditioner owned by the caller (free with
 * spai_precond_destroy) and *st (optional) the statistics.
 * Overflow (Section 4 scales A so that the low precision computations do not
 * overflow; it can still happen when a reduced problem is ill conditioned): an
 * FP16 or BF16 column whose computation gives a non-finite value is recomputed
 * from its initial pattern in FP32 (gather, QR, scores and selection, as with
 * u_f = FP32) and counted in cols_fallback; P's values are then all stored in
 * FP32 (the other columns keep their FP16/BF16 values exactly), while x0 = P b
 * still rounds D b to the build's u_f (spai_precond_view.u_f).  A column that
 * is still non-finite in FP32 keeps its values and sets SPAI_W_NONFINITE.
 * Errors: SPAI_E_ARG for n <= 0, NULL arrays, eps <= 0, beta < 0, alpha < 0,
 * maxfill < 1, maxfill > 63, an unknown u_f, a kernel_cfg outside 0..SPAI_KCFG_COUNT
 * or too small for the pattern, a pattern with a column longer than 63 or a
 * malformed A/pattern (checked on the device); SPAI_E_OOM; SPAI_E_HIP.
 */
int spai_build(spai_handle* h, const spai_csr* A, const spai_pattern* J,
               const spai_build_params* p, spai_precond** P, spai_build_stats* st);

/* Wrap an existing preconditioner given as CSR(M^T) (device, columns ascending,
 * FP64 values that must be exactly representable in val_prec) plus the scaling d
 * (device, n): the data are copied, P is owned by the caller. */
int spai_precond_import(spai_handle* h, int32_t n, int64_t nnz, const int32_t* rowptr,
                        const int32_t* col, const double* val, spai_prec val_prec,
                        const double* d, spai_precond** P);
int spai_precond_view_get(const spai_precond* P, spai_precond_view* view);
int spai_precond_destroy(spai_precond* P);

/*
 * SPAI-GMRES-IR (Algorithm 3): x0 = P b in u_f (the format of P's values; FP32
 * arithmetic for FP16/BF16), then per refinement step r_i = b - A x_i in u_r
 * (stored FP64), left-preconditioned MGS-GMRES on P A d = P r_i in FP64 with zero
 * initial guess, stopped when the Givens estimate |g_{j+1}| <= tau ||P r_i||_2,
 * and x_{i+1} = x_i + d_i in FP64.  With a preconditioner built with
 * side = SPAI_RIGHT the solve preconditions on the right instead (the paper's
 * future-work variant): GMRES on A P y = r_i stopped when |g_{j+1}| <=
 * tau ||r_i||_2, d_i = P y (working precision FP64 only).  Refinement stops when ||d_i||_inf <= tol_ir
 * ||x_{i+1}||_inf, after imax steps, from the third step on when ||d_i||_inf >
 * ||d_{i-1}||_inf / 2, or before a step whose P r_i is exactly zero.
 * b and x are device arrays of n FP64 values (x is output only).
 * Errors: SPAI_E_ARG (sizes differ, imax outside 1..32, maxit < 1, tau < 0, an
 * unknown ortho, CGS2 when the cooperative Arnoldi kernel cannot hold the
 * problem, u other than FP64/FP32, u = FP32 with u_r = DD, ortho other than
 * MGS or u_f = FP64); SPAI_E_INTERNAL when a grid-wide sum times out (about a
 * second); warnings SPAI_W_MAXIT, SPAI_W_NOCONV.
 */
int spai_gmres_ir(spai_handle* h, const spai_csr* A, const spai_precond* P, const double* b,
                  double* x, const spai_ir_params* p, spai_ir_stats* st);

/*
 * spai_gmres_ir without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, semantics and results as
 * spai_gmres_ir (bit for bit), with these limits:
 *   - the workspace (the Krylov basis n (min(maxit, n) + 1) doubles, three
 *     vectors, the Hessenberg matrix and the grid-sum slots of the chosen
 *     orthogonalisation) must fit the library's fixed 64 MiB device array
 *     (about n (maxit + 1) <= 7.5 M doubles with DCGS2 at maxit 500); larger
 *     problems are rejected with SPAI_E_ARG and a message giving the size;
 *   - working precision FP64 only (p->u = SPAI_FP32 is rejected); p->graph is
 *     ignored (stream launches); kernel timing (spai_timing_enable) is not
 *     recorded during the call.
 * The array is one per device, set up by spai_create and held until the
 * process ends; every call on a device uses the same array and leaves its
 * contents behind (each call initialises what it reads), so calls that overlap
 * on one device -- from several handles or threads -- race and must not be
 * made.  No hipMalloc, hipFree, event, stream or graph creation happens inside.
 */
int spai_gmres_ir_noalloc(spai_handle* h, const spai_csr* A, const spai_precond* P, const double* b,
                          double* x, const spai_ir_params* p, spai_ir_stats* st);

/*
 * Batches of independent systems (many systems of different sizes in one call).
 * A batch is one block-diagonal matrix A (the caller concatenates the systems):
 * system s owns rows and columns sys_ptr[s] .. sys_ptr[s+1]-1, with sys_ptr a
 * host array of nsys + 1 int32 values from 0 to n, strictly increasing.
 *
 * spai_build_batched: Algorithm 1 on every column of every system in one build
 * (a block-diagonal matrix's SPAI is the SPAI of each block: a column's shadow,
 * candidates and residual stay inside its block), so the result is the
 * block-diagonal P whose block s is system s's preconditioner, bit-identical to
 * building each system alone with the same parameters.  Errors: those of
 * spai_build, and SPAI_E_ARG for a bad sys_ptr or an entry of A outside the
 * diagonal blocks (checked on the device).
 */
int spai_build_batched(spai_handle* h, const spai_csr* A, int32_t nsys, const int32_t* sys_ptr,
                       const spai_pattern* J, const spai_build_params* p, spai_precond** P,
                       spai_build_stats* st);

/*
 * spai_gmres_ir_batched: Algorithm 3 for every system of the batch on its own
 * (its own x0, residuals, Krylov space, stopping decisions and refinement
 * steps, with the semantics of spai_gmres_ir and maxit capped at the system's
 * size), all systems in one persistent launch: each workgroup takes the next
 * system (largest first) and runs its whole refinement loop.  Orthogonalisation
 * is MGS (p->ortho must be SPAI_ORTHO_MGS); P must be a left preconditioner.  b and x are device arrays of n FP64
 * values in the batch's row order; st is a host array of nsys statistics.
 * Device workspace: up to two workgroups per compute unit, each holding
 * n_max (min(maxit, n_max) + 1) + O(maxit^2) doubles for the largest system
 * n_max (fewer workgroups if that would exceed a quarter of free memory).
 * Returns the bitwise OR of the systems' warnings (SPAI_W_MAXIT,
 * SPAI_W_NOCONV), or a negative error: SPAI_E_ARG (as spai_gmres_ir, a bad
 * sys_ptr, an entry outside the blocks, ortho not MGS), SPAI_E_OOM, SPAI_E_HIP.
 */
int spai_gmres_ir_batched(spai_handle* h, const spai_csr* A, const spai_precond* P, int32_t nsys,
                          const int32_t* sys_ptr, const double* b, double* x, const spai_ir_params* p,
                          spai_ir_stats* st);

/* Kernel timing for measurement: when enabled for a kernel class, every
 * `sample_every`-th launch of that class is bracketed by a pair of HIP events
 * recorded on the handle's stream.  spai_timing_read synchronises the stream,
 * returns the number of timed launches and their summed duration in ms, and
 * clears the counters.  sample_every <= 0 disables timing of the class. */
enum {
    SPAI_KT_COLUMNS = 0,  /* column kernel of Algorithm 1 (all configurations) */
    SPAI_KT_SPMV_A = 1,   /* w = A v */
    SPAI_KT_APPLY_P = 2,  /* y = P w */
    SPAI_KT_MGS = 3,      /* one modified Gram-Schmidt pass */
    SPAI_KT_RESIDUAL = 4, /* r = b - A x in u_r */
    SPAI_KT_UPDATE = 5,   /* x += V y */
    SPAI_KT_COUNT = 6
};
int spai_timing_enable(spai_handle* h, int kernel_class, int sample_every);
int spai_timing_read(spai_handle* h, int kernel_class, int64_t* launches_timed, double* total_ms);

/* Building blocks of Algorithm 3, exposed for testing (device arrays, length n). */
/* r = b - A x evaluated in u_r (SPAI_DD or SPAI_FP64), rounded to FP64. */
int spai_residual(spai_handle* h, const spai_csr* A, const double* b, const double* x, double* r,
                  spai_prec u_r);
/* y = P w = M^T (D w) in FP64. */
int spai_precond_apply(spai_handle* h, const spai_precond* P, const double* w, double* y);
/* x0 = P b in u_f (the format of P's values), stored in FP64. */
int spai_precond_apply_uf(spai_handle* h, const spai_precond* P, const double* b, double* x0);
/* y = A x in FP64. */
int spai_spmv(spai_handle* h, const spai_csr* A, const double* x, double* y);

/*
 * Serving: a request loop inside the library that solves independent systems
 * as they arrive (continuous batching).  Requests are host data (copied at
 * submission); each is admitted once its device footprint fits the server's
 * memory budget, and its matrix, preconditioner and Krylov basis stay on the
 * device from admission until its result is copied back.
 *
 * Two kinds of lanes, each a host thread with its own stream and handle, run
 * admitted work concurrently:
 *   - batch lanes take every waiting system with n <= batch_max_n that shares
 *     the oldest one's parameters (up to batch_max_systems, in arrival order)
 *     and run them as one batch: spai_build_batched, then
 *     spai_gmres_ir_batched (MGS; ortho is ignored).  A lane that finishes
 *     takes the next batch at once, so arrivals join the device while other
 *     batches are still running.
 *   - one device lane runs larger systems one at a time with spai_build and
 *     spai_gmres_ir (the request's ortho), in arrival order or smallest first
 *     (sjf_age_ms).  Its Arnoldi launches synchronise across their whole grid
 *     and need every workgroup resident.  With device_lane_cus = K > 0 the
 *     device lane's solve runs on a stream masked to K CUs of every XCD, its
 *     Arnoldi grid sized to them, and the batch lanes' streams are masked to
 *     the other CUs, so batches start and run beside the solve; a system too
 *     large for the fused Arnoldi launch on the K CUs (or K = 0) takes the
 *     whole device for its solve instead, and then no batch starts while it
 *     runs (running batches finish first).  Builds overlap freely.
 * A system's result does not depend on what else is in flight: a batch gives
 * every system the bits it gets in a batch of its own (every system is solved
 * by one workgroup in a fixed order, and the block-diagonal build equals each
 * block's build), and the device lane's kernels are deterministic.
 * Device memory: the server allocates hbm_budget bytes once and lends each
 * admitted unit of work (a batch, or one device-lane request) a contiguous
 * region of it, first fit; the library's allocations for that unit come from
 * the region (so no lane ever waits on another lane's hipFree), and the region
 * returns to the server when the unit's results are on the host.  A batch
 * needs its requests' footprints plus one lane workspace; a request waits
 * until a free region is large enough.
 */
typedef struct spai_server spai_server;

typedef struct {
    int32_t batch_lanes;       /* concurrent batch lanes, 1..16 */
    int32_t batch_max_n;       /* systems up to this size are batched; larger ones use the device lane */
    int32_t batch_max_systems; /* systems per batch, >= 1 */
    int32_t sjf_age_ms;        /* device lane order: 0 = arrival order; > 0 = smallest waiting system
                                  first unless the oldest has waited longer than this many ms */
    int64_t hbm_budget;        /* device bytes of the server's arena (allocated at creation) */
    int64_t lane_workspace;    /* batched-solver workspace of a batch in bytes (0: min(8 GiB,
                                  hbm_budget / 4 / batch_lanes)) */
    int32_t device_lane_cus;   /* CUs per XCD reserved for the device lane's solves, 0..31 (gfx950:
                                  8 XCDs of 32 CUs): batch lanes run on the other CUs, so batches
                                  keep running beside a device-lane solve; 0 = no reservation */
    int32_t pad;
} spai_serve_params;

/* One system: host CSR A (validated on the device like spai_build's input),
 * host right-hand side b, optional host initial pattern (jptr: n+1, jidx: jnnz;
 * NULL jptr = identity), and the parameters of the build and of the solve
 * (ir.x_given and ir.x_true are ignored: a request starts from x0 = P b). */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t* rowptr;
    const int32_t* col;
    const double* val;
    const double* b;
    int32_t jnnz;
    const int32_t* jptr;
    const int32_t* jidx;
    spai_build_params build;
    spai_ir_params ir;
} spai_serve_request;

typedef struct {
    int32_t rc;             /* the request's outcome: 0, a SPAI_W_* mask, or a negative SPAI_E_* */
    int32_t lane;           /* batch lane index, or -1 for the device lane */
    int32_t batch_size;     /* systems solved in the same batch (1 on the device lane) */
    int32_t cus;            /* CUs the solve could use (the reservation, the batch lanes' share,
                               or the whole device) */
    int64_t footprint;      /* device bytes reserved at admission (an upper estimate) */
    int64_t nnz_p;          /* stored entries of the system's preconditioner */
    double t_submit;        /* seconds since the server was created */
    double t_admit;
    double t_solve;         /* the solve (of the batch, or of the system) was started */
    double t_done;          /* result copied back to the host */
    spai_ir_stats ir;
} spai_serve_result;

/* Upper estimate of a request's device footprint in bytes (host only; also
 * what admission reserves).  SPAI_E_ARG for a malformed request. */
int spai_serve_footprint(const spai_serve_request* r, int64_t* bytes);

/* Create a server on the current device, allocate its arena and start its
 * lanes.  Errors: SPAI_E_ARG (batch_lanes outside 1..16, batch_max_n < 1,
 * batch_max_systems < 1, a budget that does not hold a lane workspace),
 * SPAI_E_OOM (the arena could not be allocated), SPAI_E_HIP (no device). */
int spai_serve_create(const spai_serve_params* p, spai_server** S);

/* Queue a request (its arrays are copied before the call returns) and return
 * its id.  Errors: SPAI_E_ARG (NULL pointers, n <= 0, rowptr not running from 0
 * to nnz, bad parameters), SPAI_E_OOM (its footprint, plus a lane workspace for
 * a batched system, exceeds hbm_budget, so it could never be admitted). */
int spai_serve_submit(spai_server* S, const spai_serve_request* r, int64_t* id);

/* Block until request `id` is done, copy its solution into x (host, n values;
 * may be NULL) and its record into *res (may be NULL), and forget it.  Returns
 * the request's outcome (res->rc; spai_last_error() describes a negative one),
 * or SPAI_E_ARG for an unknown id or one another caller is already waiting for.
 * Waits for different ids may run concurrently from several threads. */
int spai_serve_wait(spai_server* S, int64_t id, double* x, spai_serve_result* res);

/* Finish every queued request, stop the lanes and free the server.  Results not
 * yet collected are dropped.  No other thread may be inside a spai_serve_* call on
 * this server meanwhile. */
int spai_serve_destroy(spai_server* S);

#ifdef __cplusplus
}
#endif

#endif /* SPAI_H */
