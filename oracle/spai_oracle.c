/*
 * CPU ORACLE for SPAI-GMRES-IR — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct implementation of
 *   - the Frobenius-norm sparse approximate inverse of Algorithm 1 (Grote-Huckle
 *     variant, Section 2.2), run in the left form of Algorithm 3 on B = A^T D
 *     with the one-sided column scaling of Section 4, and
 *   - SPAI-GMRES-IR (Algorithm 3, Section 3.2) with left-preconditioned MGS-GMRES,
 *     u_g = u_p = u = FP64 (Section 4) and a residual computed exactly and then
 *     rounded to FP64 (the paper's u_r is quad; an exactly rounded residual is
 *     what any u_r <= u^2 reaches up to one rounding).
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load this
 * code.  It shares nothing with the GPU library: no headers, helpers or tables.
 *
 * Precision model (the same model the GPU library documents and follows).  The
 * build works in an arithmetic precision F — binary64 when u_f = FP64, binary32
 * otherwise — with the five IEEE operations written out one by one (FADD, FSUB,
 * FMUL, FDIV, FSQRT) and the fused multiply-add FFMA; a binary64 value rounded
 * to binary32 after an exact binary32 operation needs no double rounding, since
 * every operand here is already a binary32 value.  Every sum is sequential, in
 * the index order stated next to it, accumulated with FFMA where it is a sum of
 * products.  RS() rounds a value at a storage point to u_f: the gathered entries
 * of A-bar, the Householder vectors and updated trailing entries after each
 * reflector, the diagonal of R and m-bar.  For FP16 and BF16 this is the only
 * place the 16-bit format appears; all arithmetic is binary32.
 * Build with -O2 -ffp-contract=off and no fast-math: no implicit contraction.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_FP64 0
#define OR_FP32 1
#define OR_FP16 2
#define OR_BF16 3

/* ------------------------------------------------------------------------- */
/* rounding to the target formats (round to nearest, ties to even)            */
/* ------------------------------------------------------------------------- */

/* Round x to a binary format with `prec` significand bits (incl. hidden bit),
 * minimum normal exponent emin (x = f * 2^e with 1 <= f < 2) and largest finite
 * value maxv; subnormals keep the quantum 2^(emin - prec + 1).  Overflow gives
 * +-inf.  x / quantum is exact (power-of-two scaling), rint rounds to nearest even. */
static double round_binary(double x, int prec, int emin, double maxv) {
    if (x == 0.0 || isnan(x) || isinf(x)) return x;
    int e2;
    frexp(x, &e2);          /* |x| in [2^(e2-1), 2^e2) */
    int e = e2 - 1;
    if (e < emin) e = emin;
    double q = ldexp(1.0, e - prec + 1);
    double r = rint(x / q) * q;
    if (fabs(r) > maxv) return x > 0 ? INFINITY : -INFINITY;
    return r;
}

double oracle_round_fp16(double x) { return round_binary(x, 11, -14, 65504.0); }
double oracle_round_bf16(double x) {
    return round_binary(x, 8, -126, ldexp(255.0, 120)); /* (2 - 2^-7) * 2^127 */
}
double oracle_round_fp32(double x) { return (double)(float)x; }

static inline double f_add(double a, double b, int p) {
    return p == OR_FP64 ? a + b : (double)((float)a + (float)b);
}
static inline double f_sub(double a, double b, int p) {
    return p == OR_FP64 ? a - b : (double)((float)a - (float)b);
}
static inline double f_mul(double a, double b, int p) {
    return p == OR_FP64 ? a * b : (double)((float)a * (float)b);
}
static inline double f_div(double a, double b, int p) {
    return p == OR_FP64 ? a / b : (double)((float)a / (float)b);
}
static inline double f_sqrt(double a, int p) {
    return p == OR_FP64 ? sqrt(a) : (double)sqrtf((float)a);
}
static inline double f_fma(double a, double b, double c, int p) {
    return p == OR_FP64 ? fma(a, b, c) : (double)fmaf((float)a, (float)b, (float)c);
}
static inline double rs_p(double x, int p) {
    switch (p) {
    case OR_FP64: return x;
    case OR_FP32: return (double)(float)x;
    case OR_FP16: return oracle_round_fp16((double)(float)x);
    default: return oracle_round_bf16((double)(float)x);
    }
}
#define FADD(a, b) f_add((a), (b), uf)
#define FSUB(a, b) f_sub((a), (b), uf)
#define FMUL(a, b) f_mul((a), (b), uf)
#define FDIV(a, b) f_div((a), (b), uf)
#define FSQRT(a) f_sqrt((a), uf)
#define FFMA(a, b, c) f_fma((a), (b), (c), uf)
#define RS(x) rs_p((x), uf)

/* ------------------------------------------------------------------------- */
/* preprocessing (Section 4): d_i = 1 / max_j |a_ij| in FP64;                  */
/* B = A^T D so column j of B is d_j times row j of A;                         */
/* row l of B lists {j : a_jl != 0}, i.e. column l of A.                       */
/* ------------------------------------------------------------------------- */

typedef struct {
    int n;
    const int *rp, *ci;
    const double *av;
    double *d;          /* scaling */
    int *cp, *ri;       /* CSC structure of A: column l -> rows j */
    double *bnrm2;      /* ||B(:,j)||^2 in the arithmetic precision (from stored values) */
} prep_t;

static void prep_build(prep_t* P, int n, const int* rp, const int* ci, const double* av, int uf) {
    P->n = n; P->rp = rp; P->ci = ci; P->av = av;
    P->d = (double*)malloc(sizeof(double) * (size_t)n);
    P->bnrm2 = (double*)malloc(sizeof(double) * (size_t)n);
    int nnz = rp[n];
    P->cp = (int*)calloc((size_t)n + 1, sizeof(int));
    P->ri = (int*)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    for (int j = 0; j < n; ++j) {
        double mx = 0.0;
        for (int t = rp[j]; t < rp[j + 1]; ++t)
            if (fabs(av[t]) > mx) mx = fabs(av[t]);
        P->d[j] = mx > 0.0 ? 1.0 / mx : 1.0;
    }
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int t = rp[j]; t < rp[j + 1]; ++t) {
            double b = RS(P->d[j] * av[t]);
            s = FFMA(b, b, s);                     /* CSR order of row j */
        }
        P->bnrm2[j] = s;
    }
    /* counting sort transpose (rows of each column come out ascending) */
    for (int t = 0; t < nnz; ++t) P->cp[ci[t] + 1]++;
    for (int l = 0; l < n; ++l) P->cp[l + 1] += P->cp[l];
    int* fill = (int*)malloc(sizeof(int) * (size_t)n);
    memcpy(fill, P->cp, sizeof(int) * (size_t)n);
    for (int j = 0; j < n; ++j)
        for (int t = rp[j]; t < rp[j + 1]; ++t) P->ri[fill[ci[t]]++] = j;
    free(fill);
}

static void prep_free(prep_t* P) {
    free(P->d); free(P->bnrm2); free(P->cp); free(P->ri);
}

/* ------------------------------------------------------------------------- */
/* small dynamic int set helpers                                               */
/* ------------------------------------------------------------------------- */

static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

/* sort ascending and drop duplicates; returns new length */
static int sort_unique(int* v, int len) {
    if (len == 0) return 0;
    qsort(v, (size_t)len, sizeof(int), cmp_int);
    int w = 1;
    for (int t = 1; t < len; ++t)
        if (v[t] != v[w - 1]) v[w++] = v[t];
    return w;
}


typedef struct { double rho; int j; } cand_t;

static int cmp_cand(const void* a, const void* b) {
    const cand_t* x = (const cand_t*)a;
    const cand_t* y = (const cand_t*)b;
    if (x->rho < y->rho) return -1;
    if (x->rho > y->rho) return 1;
    return (x->j > y->j) - (x->j < y->j);
}

/* ------------------------------------------------------------------------- */
/* one column of Algorithm 1 on B                                              */
/* ------------------------------------------------------------------------- */

typedef struct {
    int cap_e;       /* capacity for index gathers */
    int* Ibuf;       /* shadow I in insertion order (see column_solve) */
    int* Tbuf;       /* scratch for the rows of the new columns */
    int* Cbuf;       /* candidates */
    double* A0;      /* gathered A-bar, column-major m x p (kept for the residual) */
    double* Aw;      /* working copy for QR, m x (p+1): last column e-bar */
    double* Rd;      /* diagonal of R */
    double* mb;      /* m-bar */
    double* s;       /* residual s-bar on I */
    cand_t* cand;
    int cap_m, cap_p;
} work_t;

static void work_reserve(work_t* W, int m, int p, int e) {
    if (e > W->cap_e) {
        W->cap_e = e * 2;
        W->Ibuf = (int*)realloc(W->Ibuf, sizeof(int) * (size_t)W->cap_e);
        W->Tbuf = (int*)realloc(W->Tbuf, sizeof(int) * (size_t)W->cap_e);
        W->Cbuf = (int*)realloc(W->Cbuf, sizeof(int) * (size_t)W->cap_e);
        W->cand = (cand_t*)realloc(W->cand, sizeof(cand_t) * (size_t)W->cap_e);
    }
    if (m > W->cap_m || p > W->cap_p) {
        if (m > W->cap_m) W->cap_m = m * 2;
        if (p > W->cap_p) W->cap_p = p * 2;
        size_t mp = (size_t)W->cap_m * (size_t)W->cap_p;
        W->A0 = (double*)realloc(W->A0, sizeof(double) * mp);
        W->Aw = (double*)realloc(W->Aw, sizeof(double) * mp);
        W->s = (double*)realloc(W->s, sizeof(double) * (size_t)W->cap_m);
        W->Rd = (double*)realloc(W->Rd, sizeof(double) * (size_t)W->cap_p);
        W->mb = (double*)realloc(W->mb, sizeof(double) * (size_t)W->cap_p);
    }
}

static void work_free(work_t* W) {
    free(W->Ibuf); free(W->Tbuf); free(W->Cbuf); free(W->cand); free(W->A0); free(W->Aw);
    free(W->s); free(W->Rd); free(W->mb);
}

typedef struct {
    /* outputs for one column */
    int len;           /* |J_k| */
    int steps;         /* number of augmentation steps taken */
    int nI;            /* |I_k| at the last solve */
    int flags;         /* bit0 rank-deficient, bit1 residual above eps, bit2 non-finite,
                          bit3 recomputed in FP32 after a non-finite 16-bit result */
    double res;        /* ||e_k - B m_k||_2 at the last solve (as tested) */
    double margin;     /* smallest relative decision margin seen */
    double flops;      /* algorithmic flops of the column's solves (see spai_column) */
} colinfo_t;

#define FLAG_RANKDEF 1
#define FLAG_EPS 2
#define FLAG_NONFINITE 4
#define FLAG_FALLBACK 8

static double dmin(double a, double b) { return a < b ? a : b; }

/* position of key in the shadow list I (insertion order), or -1 */
static int find_pos(const int* I, int m, int key) {
    for (int t = 0; t < m; ++t)
        if (I[t] == key) return t;
    return -1;
}

/* Solve the reduced least-squares problem (eq. redprob) for the current J by
 * Householder QR (Algorithm 1, QR and solve lines) and return res^2.
 * I (insertion order, length m) and J (insertion order, length p) are given. */
static double ls_solve(const prep_t* P, int k, const int* I, int m, const int* J, int p,
                       work_t* W, int uf, int* flags, int* kin) {
    double* A0 = W->A0;
    double* A = W->Aw;
    /* gather A-bar = B(I, J) column-major and e-bar = e_k(I) */
    for (int c = 0; c < p; ++c) {
        int j = J[c];
        for (int i = 0; i < m; ++i) A0[(size_t)c * m + i] = 0.0;
        for (int t = P->rp[j]; t < P->rp[j + 1]; ++t) {
            int pos = find_pos(I, m, P->ci[t]);
            A0[(size_t)c * m + pos] = RS(P->d[j] * P->av[t]);
        }
    }
    memcpy(A, A0, sizeof(double) * (size_t)m * (size_t)p);
    int kpos = find_pos(I, m, k);
    *kin = kpos >= 0;
    for (int i = 0; i < m; ++i) A[(size_t)p * m + i] = (i == kpos) ? 1.0 : 0.0;

    /* Householder QR, column by column (the QR line of Algorithm 1).  For
     * x = A(t:m, t), sigma = ||x||, alpha = -sgn(x_t) sigma (sgn(0) = +1) and
     * v = x - alpha e_1 one has v^T v = 2 sigma (sigma + |x_t|), so the reflector
     * H = I - 2 v v^T / (v^T v) maps a column a to a - (v^T a / tau) v with
     * tau = sigma (sigma + |x_t|).  Column p of the work array holds e-bar, which
     * becomes Q^T e-bar.  Sums run over i = t..m-1 ascending. */
    int rank_def = 0;
    int steps = p < m ? p : m;
    for (int t = 0; t < p; ++t) W->Rd[t] = 0.0;
    double* e = A + (size_t)p * m;
    for (int t = 0; t < steps; ++t) {
        double* x = A + (size_t)t * m;
        double sig2 = 0.0;
        for (int i = t; i < m; ++i) sig2 = FFMA(x[i], x[i], sig2);
        double sigma = FSQRT(sig2);
        if (sigma == 0.0) { rank_def = 1; W->Rd[t] = 0.0; continue; }
        double xt = x[t];
        double alpha = (xt >= 0.0) ? -sigma : sigma;
        x[t] = RS(FSUB(xt, alpha));               /* column t now holds v */
        double tau = FMUL(sigma, FADD(sigma, fabs(xt)));
        for (int c = t + 1; c <= p; ++c) {        /* trailing columns and e-bar */
            double* a = A + (size_t)c * m;
            double dot = 0.0;
            for (int i = t; i < m; ++i) dot = FFMA(x[i], a[i], dot);
            double f = FDIV(dot, tau);
            for (int i = t; i < m; ++i) a[i] = RS(FFMA(-f, x[i], a[i]));
        }
        W->Rd[t] = RS(alpha);
    }
    if (p > m) rank_def = 1;  /* more unknowns than rows: cannot happen for nonsingular B */
    /* back substitution m-bar = R^{-1} (Q^T e-bar)(1:p), c = p-1 down to 0, inner sum
     * over c' = c+1..p-1 ascending; R(c, c') = A(c, c') above the diagonal */
    for (int c = p - 1; c >= 0; --c) {
        if (c >= m || W->Rd[c] == 0.0) { W->mb[c] = 0.0; rank_def = 1; continue; }
        double s = e[c];
        for (int c2 = c + 1; c2 < p; ++c2) s = FFMA(-A[(size_t)c2 * m + c], W->mb[c2], s);
        W->mb[c] = RS(FDIV(s, W->Rd[c]));
    }
    if (rank_def) *flags |= FLAG_RANKDEF;
    /* residual s-bar = A-bar m-bar - e-bar (the residual line of Algorithm 1),
     * evaluated explicitly with the gathered A-bar: row sums over c = 0..p-1 over
     * the stored entries of the row, then ||s-bar||^2 over i ascending */
    double res2 = 0.0;
    for (int i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int c = 0; c < p; ++c)
            if (A0[(size_t)c * m + i] != 0.0) acc = FFMA(A0[(size_t)c * m + i], W->mb[c], acc);
        W->s[i] = FSUB(acc, (i == kpos) ? 1.0 : 0.0);
        res2 = FFMA(W->s[i], W->s[i], res2);
    }
    /* true residual ||e_k - B m_k||: row k contributes 1 when k lies outside the shadow */
    if (kpos < 0) res2 = FADD(res2, 1.0);
    return res2;
}

/* Shadow and reduced least-squares solve for the current J (lines computing I_k,
 * A-bar, e-bar, QR, m-bar and s-bar in Algorithm 1).  The shadow is kept in
 * insertion order: the first m_prev entries of W->Ibuf (the shadow of the
 * previous solve of this column, 0 at the first solve) stay where they are and
 * the rows that the new columns bring in follow in ascending order.  With this
 * row order the Householder reflectors of the columns already factored are
 * unchanged by an augmentation (those columns are zero in the new rows), so the
 * full QR below is exactly what an incremental update of the previous QR
 * computes (the remark on updating the QR in Section 2.2).  Leaves I in W->Ibuf
 * (m entries), m-bar in W->mb and s-bar in W->s; returns
 * res^2 = ||e_k - B m_k||^2. */
static double column_solve(const prep_t* P, int k, const int* J, int p, work_t* W, int uf, int m_prev,
                           int* m_out, int* kin, int* flags) {
    /* shadow I_k = rows touched by the columns J_k (structural; no stored zeros) */
    int ecount = 0;
    for (int c = 0; c < p; ++c) ecount += P->rp[J[c] + 1] - P->rp[J[c]];
    work_reserve(W, ecount + 1, p + 1, ecount + 1);
    int nt = 0;
    for (int c = 0; c < p; ++c)
        for (int t = P->rp[J[c]]; t < P->rp[J[c] + 1]; ++t) W->Tbuf[nt++] = P->ci[t];
    nt = sort_unique(W->Tbuf, nt);
    int m = m_prev;
    for (int t = 0; t < nt; ++t)
        if (find_pos(W->Ibuf, m_prev, W->Tbuf[t]) < 0) W->Ibuf[m++] = W->Tbuf[t];
    work_reserve(W, m + 1, p + 1, ecount + 1);
    *m_out = m;
    return ls_solve(P, k, W->Ibuf, m, J, p, W, uf, flags, kin);
}

/* Candidate indices and their scores (lines from L_k to the mean in Algorithm 1):
 * L = I u {k}; N_l = {j : B(l, j) != 0}; J~ = (union N_l) \ J, ascending;
 * rho_j = sqrt(max(res^2 - (r^T B e_j)^2 / ||B e_j||^2, 0)) with r the full residual
 * on L (r_l = s-bar_l on I, r_k = -1 when k is outside I); rho-bar = mean of rho_j.
 * Fills W->cand[0..nc) in ascending j and returns nc. */
static int column_score(const prep_t* P, int k, const int* J, int p, int m, int kin, double res2,
                        work_t* W, int uf, double* rbar_out) {
    int nl = m + (kin ? 0 : 1);
    int ccount = 0;
    for (int t = 0; t < m; ++t) ccount += P->cp[W->Ibuf[t] + 1] - P->cp[W->Ibuf[t]];
    if (!kin) ccount += P->cp[k + 1] - P->cp[k];
    work_reserve(W, m + 1, p + 1, ccount + nl + 1);
    int nc = 0;
    for (int t = 0; t < m; ++t) {
        int l = W->Ibuf[t];
        for (int q = P->cp[l]; q < P->cp[l + 1]; ++q) W->Cbuf[nc++] = P->ri[q];
    }
    if (!kin)
        for (int q = P->cp[k]; q < P->cp[k + 1]; ++q) W->Cbuf[nc++] = P->ri[q];
    nc = sort_unique(W->Cbuf, nc);
    int w = 0;
    for (int t = 0; t < nc; ++t) {
        int j = W->Cbuf[t], inJ = 0;
        for (int c = 0; c < p; ++c) if (J[c] == j) { inJ = 1; break; }
        if (!inJ) W->Cbuf[w++] = j;
    }
    nc = w;
    double rsum = 0.0;
    for (int t = 0; t < nc; ++t) {
        int j = W->Cbuf[t];
        double tj = 0.0;
        /* rows of B(:, j) in ascending order = columns of row j of A */
        for (int q = P->rp[j]; q < P->rp[j + 1]; ++q) {
            int i = P->ci[q];
            double ri;
            int pos = find_pos(W->Ibuf, m, i);
            if (pos >= 0) ri = W->s[pos];
            else if (i == k) ri = -1.0;  /* k outside the shadow */
            else continue;               /* row not in L */
            double bij = RS(P->d[j] * P->av[q]);
            tj = FFMA(ri, bij, tj);
        }
        double r2 = FSUB(res2, FDIV(FMUL(tj, tj), P->bnrm2[j]));
        if (r2 <= 0.0) r2 = 0.0;
        double rho = FSQRT(r2);
        W->cand[t].rho = rho;
        W->cand[t].j = j;
        rsum = FADD(rsum, rho);                /* candidates in ascending j */
    }
    *rbar_out = nc > 0 ? FDIV(rsum, (double)nc) : 0.0;
    return nc;
}

/* Algorithm 1 for column k.  J0/len0: initial pattern column (any order; sorted here).
 * On return Jout[0..len) holds J_k in insertion order and mout the values m-bar;
 * hist (optional, capacity hcap) the residual norm of every solve. */
static void spai_column(const prep_t* P, int k, const int* J0, int len0, double eps, int alpha,
                        int beta, int maxfill, int uf, work_t* W, int* Jout, double* mout,
                        colinfo_t* info, double* hist, int hcap) {
    int p = len0;
    int cap = (maxfill > len0 ? maxfill : len0);
    int* J = Jout;
    for (int t = 0; t < len0; ++t) J[t] = J0[t];
    p = sort_unique(J, len0);
    info->flags = 0;
    info->margin = INFINITY;
    info->steps = 0;
    info->flops = 0.0;
    int m = 0;
    for (int step = 0;; ++step) {
        int kin = 0;
        double res2 = column_solve(P, k, J, p, W, uf, m, &m, &kin, &info->flags);
        /* algorithmic flops of this solve of an m x p problem: Householder QR
         * 2mp^2 - 2p^3/3, applying the reflectors to e-bar and forming the
         * residual 4mp, back substitution p^2 (Section 2.2: cubic in the number
         * of nonzeros per column) */
        info->flops += 2.0 * m * p * p - 2.0 * p * p * p / 3.0 + 4.0 * m * p + (double)p * p;
        double res = FSQRT(res2);
        if (hist && step < hcap) hist[step] = res;
        info->res = res;
        info->nI = m;
        info->steps = step;
        for (int c = 0; c < p; ++c) mout[c] = W->mb[c];
        info->len = p;
        if (!isfinite(res)) { info->flags |= FLAG_NONFINITE; return; }
        info->margin = dmin(info->margin, fabs(res - eps) / eps);
        if (res <= eps) return;                       /* stopping test */
        if (step >= alpha || p >= cap) { info->flags |= FLAG_EPS; return; }

        double rbar = 0.0;
        int nc = column_score(P, k, J, p, m, kin, res2, W, uf, &rbar);
        if (nc == 0) { info->flags |= FLAG_EPS; return; }
        /* acceptable indices rho_j <= rho-bar, best (smallest rho, then smallest j) first;
         * up to beta of them join J, never beyond the fill cap */
        int na = 0;
        for (int t = 0; t < nc; ++t) {
            if (rbar > 0.0) info->margin = dmin(info->margin, fabs(W->cand[t].rho - rbar) / rbar);
            else info->margin = 0.0;
            if (W->cand[t].rho <= rbar) W->cand[na++] = W->cand[t];
        }
        qsort(W->cand, (size_t)na, sizeof(cand_t), cmp_cand);
        int nsel = beta;
        if (na < nsel) nsel = na;
        if (cap - p < nsel) nsel = cap - p;
        if (nsel > 0 && nsel < na && rbar > 0.0)
            info->margin = dmin(info->margin, fabs(W->cand[nsel].rho - W->cand[nsel - 1].rho) / rbar);
        if (nsel <= 0) { info->flags |= FLAG_EPS; return; }
        for (int t = 0; t < nsel; ++t) J[p++] = W->cand[t].j;
    }
}

/*
 * One solve and scoring step of Algorithm 1 for column k with the given J (insertion
 * order) and the shadow of the previous solve Iprev (mprev rows, 0 for a first
 * solve), for tests.  Outputs: res, I (sorted, *m entries, capacity cap), m-bar (p
 * entries), candidates cj/crho (*nc entries, ascending j, capacity cap) and rho-bar.
 * Returns 0, or -1 when a capacity is too small.
 */
int oracle_spai_probe(int n, const int* rp, const int* ci, const double* av, int k, const int* J,
                      int p, const int* Iprev, int mprev, int uf, int cap, double* res, int* I, int* m,
                      double* mbar, int* cj, double* crho, int* nc, double* rbar, int* flags) {
    prep_t P;
    prep_build(&P, n, rp, ci, av, uf);
    work_t W;
    memset(&W, 0, sizeof(W));
    int kin = 0, mm = 0, fl = 0;
    int ecount = mprev;
    for (int c = 0; c < p; ++c) ecount += rp[J[c] + 1] - rp[J[c]];
    work_reserve(&W, ecount + 1, p + 1, ecount + 1);
    for (int t = 0; t < mprev; ++t) W.Ibuf[t] = Iprev[t];   /* shadow of the previous solve, in order */
    double res2 = column_solve(&P, k, J, p, &W, uf, mprev, &mm, &kin, &fl);
    int rc = 0;
    *res = FSQRT(res2);
    *m = mm;
    *flags = fl;
    if (mm > cap) rc = -1;
    else for (int t = 0; t < mm; ++t) I[t] = W.Ibuf[t];
    for (int c = 0; c < p; ++c) mbar[c] = W.mb[c];
    int ncc = column_score(&P, k, J, p, mm, kin, res2, &W, uf, rbar);
    *nc = ncc;
    if (ncc > cap) rc = -1;
    else for (int t = 0; t < ncc; ++t) { cj[t] = W.cand[t].j; crho[t] = W.cand[t].rho; }
    work_free(&W);
    prep_free(&P);
    return rc;
}

/* ------------------------------------------------------------------------- */
/* exported: SPAI build over a list of columns                                 */
/* ------------------------------------------------------------------------- */

typedef struct {
    const prep_t* P;
    const prep_t* P32;    /* FP32 preprocessing for the recomputation of overflowing 16-bit columns */
    const int* pat_ptr;
    const int* pat_idx;
    const int* cols;
    int c0, c1;
    double eps;
    int alpha, beta, maxfill, uf, stride;
    int* out_len;
    int* out_J;
    double* out_m;
    int* out_steps;
    int* out_nI;
    int* out_flags;
    double* out_res;
    double* out_margin;
    double* out_hist;
    double* out_flops;
} job_t;

static void* run_job(void* arg) {
    job_t* jb = (job_t*)arg;
    work_t W;
    memset(&W, 0, sizeof(W));
    int* Jtmp = (int*)malloc(sizeof(int) * (size_t)(jb->stride + 1));
    double* mtmp = (double*)malloc(sizeof(double) * (size_t)(jb->stride + 1));
    for (int t = jb->c0; t < jb->c1; ++t) {
        int k = jb->cols ? jb->cols[t] : t;
        const int* J0;
        int len0;
        int ident = k;
        if (jb->pat_ptr) { J0 = jb->pat_idx + jb->pat_ptr[k]; len0 = jb->pat_ptr[k + 1] - jb->pat_ptr[k]; }
        else { J0 = &ident; len0 = 1; }
        colinfo_t info;
        double* hist = jb->out_hist ? jb->out_hist + (size_t)t * (size_t)(jb->stride + 1) : NULL;
        if (hist) for (int h = 0; h <= jb->stride; ++h) hist[h] = NAN;
        spai_column(jb->P, k, J0, len0, jb->eps, jb->alpha, jb->beta, jb->maxfill, jb->uf, &W,
                    Jtmp, mtmp, &info, hist, jb->stride + 1);
        if ((info.flags & FLAG_NONFINITE) && jb->P32) {
            /* overflow policy of the 16-bit formats: the whole column again, from its
             * initial pattern, with u_f = FP32 (storage points and arithmetic) */
            if (hist) for (int h = 0; h <= jb->stride; ++h) hist[h] = NAN;
            spai_column(jb->P32, k, J0, len0, jb->eps, jb->alpha, jb->beta, jb->maxfill, OR_FP32, &W,
                        Jtmp, mtmp, &info, hist, jb->stride + 1);
            info.flags |= FLAG_FALLBACK;
        }
        size_t o = (size_t)t * (size_t)jb->stride;
        jb->out_len[t] = info.len;
        for (int c = 0; c < info.len; ++c) { jb->out_J[o + c] = Jtmp[c]; jb->out_m[o + c] = mtmp[c]; }
        for (int c = info.len; c < jb->stride; ++c) { jb->out_J[o + c] = -1; jb->out_m[o + c] = 0.0; }
        if (jb->out_steps) jb->out_steps[t] = info.steps;
        if (jb->out_nI) jb->out_nI[t] = info.nI;
        if (jb->out_flags) jb->out_flags[t] = info.flags;
        if (jb->out_res) jb->out_res[t] = info.res;
        if (jb->out_margin) jb->out_margin[t] = info.margin;
        if (jb->out_flops) jb->out_flops[t] = info.flops;
    }
    free(Jtmp);
    free(mtmp);
    work_free(&W);
    return NULL;
}

/*
 * Run Algorithm 1 on B = A^T D for the columns `cols[0..ncols)` (all columns when
 * cols == NULL and ncols == n).  A is CSR (sorted columns, no stored zeros).
 * pat_ptr/pat_idx give the initial pattern J (column k -> indices); NULL means the
 * identity.  alpha = maximum augmentation steps (0 = fixed pattern).  maxfill caps
 * |J_k| (never truncating the initial pattern).  Outputs are padded with stride
 * `stride` (>= max(maxfill, initial column length)); out_hist (optional) receives
 * the residual norm of every solve, stride + 1 per column, NaN padded.  Returns 0,
 * or -1 on a bad argument.
 */
int oracle_spai(int n, const int* rp, const int* ci, const double* av, const int* pat_ptr,
                const int* pat_idx, double eps, int alpha, int beta, int maxfill, int uf,
                const int* cols, int ncols, int stride, int nthreads, int* out_len, int* out_J,
                double* out_m, int* out_steps, int* out_nI, int* out_flags, double* out_res,
                double* out_margin, double* out_d, double* out_hist, double* out_flops) {
    if (n <= 0 || uf < 0 || uf > 3 || ncols < 0 || stride <= 0) return -1;
    if (nthreads < 1) nthreads = 1;
    prep_t P, P32;
    prep_build(&P, n, rp, ci, av, uf);
    const int low = uf == OR_FP16 || uf == OR_BF16;
    if (low) prep_build(&P32, n, rp, ci, av, OR_FP32);
    if (out_d) memcpy(out_d, P.d, sizeof(double) * (size_t)n);
    if (nthreads > ncols) nthreads = ncols > 0 ? ncols : 1;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
    job_t* jobs = (job_t*)malloc(sizeof(job_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; ++t) {
        job_t* jb = &jobs[t];
        jb->P = &P; jb->P32 = low ? &P32 : NULL; jb->pat_ptr = pat_ptr; jb->pat_idx = pat_idx; jb->cols = cols;
        jb->c0 = (int)((long long)ncols * t / nthreads);
        jb->c1 = (int)((long long)ncols * (t + 1) / nthreads);
        jb->eps = eps; jb->alpha = alpha; jb->beta = beta; jb->maxfill = maxfill; jb->uf = uf;
        jb->stride = stride; jb->out_len = out_len; jb->out_J = out_J; jb->out_m = out_m;
        jb->out_steps = out_steps; jb->out_nI = out_nI; jb->out_flags = out_flags;
        jb->out_res = out_res; jb->out_margin = out_margin; jb->out_hist = out_hist; jb->out_flops = out_flops;
    }
    if (nthreads == 1) run_job(&jobs[0]);
    else {
        for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
        for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    free(th);
    free(jobs);
    prep_free(&P);
    if (low) prep_free(&P32);
    return 0;
}

/* scaling vector only (Section 4): d_i = 1 / max_j |a_ij| */
void oracle_scaling(int n, const int* rp, const double* av, double* d) {
    for (int j = 0; j < n; ++j) {
        double mx = 0.0;
        for (int t = rp[j]; t < rp[j + 1]; ++t)
            if (fabs(av[t]) > mx) mx = fabs(av[t]);
        d[j] = mx > 0.0 ? 1.0 / mx : 1.0;
    }
}

/* ------------------------------------------------------------------------- */
/* exact summation, correctly rounded.  Every finite binary64 value is an      */
/* integer multiple of 2^-1074, so a sum of them is too: the values are added  */
/* as integers into a fixed-point accumulator of 32-bit digits (no rounding at */
/* all), and the exact total is rounded once to binary64 at the end (round to  */
/* nearest, ties to even).                                                     */
/* ------------------------------------------------------------------------- */

#define XDIGITS 72 /* 72 x 32 bits: weights 2^-1074 .. 2^1229, room for 2^200 terms */

double oracle_exact_sum(const double* xs, int len, double* scratch) {
    (void)scratch;
    int64_t acc[XDIGITS];
    memset(acc, 0, sizeof acc);
    for (int t = 0; t < len; ++t) {
        double x = xs[t];
        if (x == 0.0) continue;
        int e;
        double f = frexp(fabs(x), &e);              /* |x| = f 2^e, 1/2 <= f < 1 */
        uint64_t m = (uint64_t)ldexp(f, 53);        /* |x| = m 2^(e-53), m < 2^53, exact */
        int sh = e - 53 + 1074;                     /* |x| = m 2^(sh-1074) */
        if (sh < 0) { m >>= -sh; sh = 0; }          /* subnormal: the dropped bits are zero */
        unsigned __int128 v = (unsigned __int128)m << (sh % 32);
        int q = sh / 32;
        int64_t s = x < 0.0 ? -1 : 1;
        acc[q] += s * (int64_t)(uint32_t)v;
        acc[q + 1] += s * (int64_t)(uint32_t)(v >> 32);
        acc[q + 2] += s * (int64_t)(uint32_t)(v >> 64);
    }
    /* carries: every digit into [0, 2^32), the sign ends in the top digit */
    for (int q = 0; q + 1 < XDIGITS; ++q) {
        int64_t c = acc[q] >> 32;                   /* floor division by 2^32 */
        acc[q] -= c * ((int64_t)1 << 32);
        acc[q + 1] += c;
    }
    double sign = 1.0;
    if (acc[XDIGITS - 1] < 0) {                     /* negative: take the two's complement */
        sign = -1.0;
        int64_t borrow = 0;
        for (int q = 0; q < XDIGITS; ++q) {
            int64_t v = -acc[q] - borrow;
            borrow = 0;
            if (v < 0 && q + 1 < XDIGITS) { v += (int64_t)1 << 32; borrow = 1; }
            acc[q] = v;
        }
    }
    int top = -1;                                   /* index of the highest set bit */
    for (int q = XDIGITS - 1; q >= 0 && top < 0; --q)
        if (acc[q]) for (int b = 31; b >= 0; --b) if ((acc[q] >> b) & 1) { top = 32 * q + b; break; }
    if (top < 0) return 0.0;
#define XBIT(i) ((i) >= 0 ? (int)((acc[(i) / 32] >> ((i) % 32)) & 1) : 0)
    if (top < 53) {                                 /* below 2^-1021: exact as it stands */
        uint64_t m = 0;
        for (int i = top; i >= 0; --i) m = 2 * m + (uint64_t)XBIT(i);
        return sign * ldexp((double)m, -1074);
    }
    uint64_t m = 0;                                 /* the 53 leading bits */
    for (int i = top; i > top - 53; --i) m = 2 * m + (uint64_t)XBIT(i);
    int rbit = XBIT(top - 53), sticky = 0;
    for (int i = top - 54; i >= 0 && !sticky; --i) sticky = XBIT(i);
    if (rbit && (sticky || (m & 1))) ++m;           /* nearest, ties to even (m may reach 2^53: exact) */
#undef XBIT
    return sign * ldexp((double)m, top - 52 - 1074);
}

/* r = fl(b - A x), each component computed exactly and rounded once to FP64
 * (Algorithm 3, residual line, with u_r finer than needed to round exactly).
 * Products a_ij x_j are split exactly into hi + lo with an FMA. */
void oracle_residual(int n, const int* rp, const int* ci, const double* av, const double* b,
                     const double* x, double* r) {
    int maxq = 0;
    for (int i = 0; i < n; ++i) if (rp[i + 1] - rp[i] > maxq) maxq = rp[i + 1] - rp[i];
    double* terms = (double*)malloc(sizeof(double) * (size_t)(2 * maxq + 1));
    double* scratch = (double*)malloc(sizeof(double) * (size_t)(2 * maxq + 1));
    for (int i = 0; i < n; ++i) {
        int nt = 0;
        terms[nt++] = b[i];
        for (int t = rp[i]; t < rp[i + 1]; ++t) {
            double hi = av[t] * x[ci[t]];
            double lo = fma(av[t], x[ci[t]], -hi);
            terms[nt++] = -hi;
            terms[nt++] = -lo;
        }
        r[i] = oracle_exact_sum(terms, nt, scratch);
    }
    free(terms);
    free(scratch);
}

/* ------------------------------------------------------------------------- */
/* SPAI-GMRES-IR (Algorithm 3)                                                 */
/* ------------------------------------------------------------------------- */

/* y = P w = M^T (D w) in FP64 (u_p = u).  Row k of P holds m_k: columns pc, values pv. */
static void apply_P(int n, const int* pp, const int* pc, const double* pv, const double* d,
                    const double* w, double* dw, double* y) {
    for (int j = 0; j < n; ++j) dw[j] = d[j] * w[j];
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int t = pp[k]; t < pp[k + 1]; ++t) s += pv[t] * dw[pc[t]];
        y[k] = s;
    }
}

static void spmv(int n, const int* rp, const int* ci, const double* av, const double* x, double* y) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int t = rp[i]; t < rp[i + 1]; ++t) s += av[t] * x[ci[t]];
        y[i] = s;
    }
}

/* Right preconditioner P = D M (Algorithm 1 run on A with the columns of A scaled
 * to unit maximum, so that A D M ~ I): row i of its CSR holds the entries m_k[i]
 * of the columns k with i in J_k (columns pc, values pv), and y = P w = D (M w):
 * y_i = d_i * sum_k m_k[i] w_k in FP64. */
static void apply_P_right(int n, const int* pp, const int* pc, const double* pv, const double* d,
                          const double* w, double* y) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int t = pp[i]; t < pp[i + 1]; ++t) s += pv[t] * w[pc[t]];
        y[i] = d[i] * s;
    }
}

/* y = P A v (left preconditioning, the paper's Algorithm 3) or y = A P v (right
 * preconditioning); w and dw are scratch vectors. */
static void apply_op(int right, int n, const int* rp, const int* ci, const double* av, const int* pp,
                     const int* pc, const double* pv, const double* d, const double* v, double* w, double* dw,
                     double* y) {
    if (right) {
        apply_P_right(n, pp, pc, pv, d, v, w);
        spmv(n, rp, ci, av, w, y);
    } else {
        spmv(n, rp, ci, av, v, w);
        apply_P(n, pp, pc, pv, d, w, dw, y);
    }
}

static double dot(int n, const double* a, const double* b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static double norm_inf(int n, const double* a) {
    double m = 0.0;
    for (int i = 0; i < n; ++i) if (fabs(a[i]) > m) m = fabs(a[i]);
    return m;
}

/* x0 = P b in u_f (Algorithm 3, initial solve): D b in FP64, rounded to u_f; products
 * and sums in the arithmetic precision of u_f; result stored in FP64. */
void oracle_x0(int n, const int* pp, const int* pc, const double* pv, const double* d,
               const double* b, int uf, double* x0) {
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    for (int j = 0; j < n; ++j) z[j] = RS(d[j] * b[j]);
    for (int k = 0; k < n; ++k) {
        double s = 0.0;
        for (int t = pp[k]; t < pp[k + 1]; ++t) s = FFMA(pv[t], z[pc[t]], s);  /* ascending column */
        x0[k] = s;
    }
    free(z);
}

/* x0 = P b in u_f for a right preconditioner P = D M: b rounded to u_f, each row's
 * sum of m_k[i] b_k in the arithmetic precision of u_f (ascending k, fused
 * multiply-adds), then multiplied by d_i rounded to u_f, in that precision. */
void oracle_x0_right(int n, const int* pp, const int* pc, const double* pv, const double* d,
                     const double* b, int uf, double* x0) {
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    for (int j = 0; j < n; ++j) z[j] = RS(b[j]);
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int t = pp[i]; t < pp[i + 1]; ++t) s = FFMA(pv[t], z[pc[t]], s);
        x0[i] = FMUL(RS(d[i]), s);
    }
    free(z);
}

#define IR_OK 0
#define IR_MAXIT 1       /* some GMRES solve hit maxit */
#define IR_NOCONV 2      /* refinement hit imax without meeting tol_ir */
#define IR_STAGNATED 4   /* correction stopped decreasing */

/* Givens step on column j of the Hessenberg matrix (column-major, leading
 * dimension ld): apply the rotations 0..j-1, build rotation j, update g. */
static void givens_column(double* H, int ld, int j, double* cs, double* sn, double* g) {
    double* h = H + (size_t)j * (size_t)ld;
    for (int l = 0; l < j; ++l) {
        double a = h[l], c2 = h[l + 1];
        h[l] = cs[l] * a + sn[l] * c2;
        h[l + 1] = -sn[l] * a + cs[l] * c2;
    }
    double delta = hypot(h[j], h[j + 1]);
    cs[j] = h[j] / delta;
    sn[j] = h[j + 1] / delta;
    h[j] = delta;
    h[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
}

/*
 * Arnoldi with CGS2 whose second projection (and the normalisation) of each new
 * vector is delayed to the next step, so that one step needs one set of inner
 * products (the delayed-reorthogonalisation CGS2 of the low-synchronisation
 * Gram-Schmidt literature; the steps below are derived from the Arnoldi relation
 * M V_j = V_{j+1} H_j, M = P A, in exact arithmetic).
 *
 * On entry column 0 of V holds v_0 = z / beta0.  Column j of V holds the lagged
 * vector u_j (u_0 = v_0), the once-projected successor of v_{j-1}.  Step j:
 *   a = V_{j-1}^T u_j, omega = u_j^T u_j, nu = sqrt(omega - a^T a)  (j >= 1)
 *   column j-1 of the Hessenberg matrix is complete: HR(0:j-1, j-1) += a,
 *   HR(j, j-1) = nu; Givens step on it and the stopping test (|g_j| <= tau beta0,
 *   nu = 0, or j = maxit), which ends the Arnoldi process with k = j;
 *   y = P A u_j; b = V_{j-1}^T y, c = u_j^T y;
 *   v_j = (u_j - V_{j-1} a) / nu;
 *   gv = [b; (c - a^T b) / nu]  (= V_j^T y);
 *   HR(0:j, j) = (gv - HR(0:j, 0:j-1) a) / nu  (first projection of M v_j);
 *   u_{j+1} = (y - V_j gv) / nu  (= M v_j - V_j HR(0:j, j)).
 * For j = 0 there is no a and nu = 1.  HR keeps the Hessenberg matrix before the
 * rotations, H receives the rotated columns.  Returns k; *maxit_hit is set when
 * k reached maxit without the test being met.
 */
static int arnoldi_dcgs2(int right, int n, const int* rp, const int* ci, const double* av, const int* pp,
                         const int* pc, const double* pv, const double* d, double* V, double* H,
                         double* HR, int ld, double* cs, double* sn, double* g, double beta0, double tau,
                         int maxit, double* w, double* dw, double* y, double* a, double* bb,
                         int* maxit_hit) {
#define HRR(i, j) HR[(size_t)(j) * (size_t)ld + (size_t)(i)]
    int k = 0;
    *maxit_hit = 0;
    for (int j = 0;; ++j) {
        double* uj = V + (size_t)j * n;
        double nu = 1.0;
        if (j > 0) {
            double q = dot(n, uj, uj);
            for (int l = 0; l < j; ++l) {
                a[l] = dot(n, V + (size_t)l * n, uj);
                q -= a[l] * a[l];
            }
            nu = q > 0.0 ? sqrt(q) : 0.0;
            for (int l = 0; l < j; ++l) HRR(l, j - 1) += a[l];
            HRR(j, j - 1) = nu;
            for (int l = 0; l <= j; ++l) H[(size_t)(j - 1) * ld + l] = HRR(l, j - 1);
            givens_column(H, ld, j - 1, cs, sn, g);
            k = j;
            if (fabs(g[j]) <= tau * beta0 || nu == 0.0) break;
            if (j == maxit) {
                *maxit_hit = 1;
                break;
            }
        }
        apply_op(right, n, rp, ci, av, pp, pc, pv, d, uj, w, dw, y);
        for (int l = 0; l < j; ++l) bb[l] = dot(n, V + (size_t)l * n, y);
        double c = dot(n, uj, y);
        if (j > 0) {                     /* per element: l ascending, then the division */
            for (int l = 0; l < j; ++l) {
                const double* vl = V + (size_t)l * n;
                for (int i = 0; i < n; ++i) uj[i] -= a[l] * vl[i];
            }
            for (int i = 0; i < n; ++i) uj[i] /= nu;
        }
        double gj = c;
        for (int l = 0; l < j; ++l) gj -= a[l] * bb[l];
        gj /= nu;
        for (int r = 0; r <= j; ++r) {
            double s = r < j ? bb[r] : gj;
            for (int m = 0; m < j; ++m) s -= HRR(r, m) * a[m];
            HRR(r, j) = s / nu;
        }
        double* un = V + (size_t)(j + 1) * n;
        for (int i = 0; i < n; ++i) un[i] = y[i];
        for (int l = 0; l < j; ++l) {
            const double* vl = V + (size_t)l * n;
            for (int i = 0; i < n; ++i) un[i] -= bb[l] * vl[i];
        }
        for (int i = 0; i < n; ++i) un[i] = (un[i] - gj * uj[i]) / nu;
    }
#undef HRR
    return k;
}

/*
 * SPAI-GMRES-IR.  A: CSR FP64.  right = 0: left preconditioning as in Algorithm 3
 * (GMRES on P A d = P r_i, P = M^T D as for oracle_x0); right = 1: right
 * preconditioning with P = D M given as for apply_P_right (GMRES on A P y = r_i,
 * stopped when |g_{j+1}| <= tau ||r_i||_2, correction d_i = P y; x0 from
 * oracle_x0_right).  ortho selects the orthogonalisation of the Arnoldi
 * vectors: 0 = modified Gram-Schmidt (the variant of the analysis in Section 3.2),
 * 1 = classical Gram-Schmidt applied twice (CGS2), 2 = CGS2 with the second
 * projection delayed by one step (arnoldi_dcgs2).  P = M^T D: CSR rows pp/pc with u_f values pv (held
 * in double) and the FP64 scaling d; uf is the precision of the initial solve.
 * x (out) receives the solution; basis0 (optional, n x maxit) receives the first
 * refinement step's orthonormal Arnoldi vectors v_0 .. v_{k-1}, column by column.  its[0..imax) receives GMRES iterations per
 * refinement step; *nsteps the number of steps.  Left-preconditioned MGS-GMRES
 * with zero initial guess, no restart, stopped when the Givens estimate of the
 * preconditioned residual |g_{j+1}| <= tau * ||P r_i||_2 (or at maxit or on an
 * exact breakdown).  The refinement stops after step i when
 * ||d_i||_inf <= tol_ir ||x_{i+1}||_inf, after imax steps, or (i >= 2) when
 * ||d_i||_inf > ||d_{i-1}||_inf / 2; it ends before step i, which is then not
 * counted, when P r_i = 0 exactly.
 * gest (optional, length imax) receives |g_{k+1}| / beta0 at the end of each step.
 * Returns a bit mask of IR_* flags, or -1 on a bad argument.
 */
int oracle_gmres_ir(int n, const int* rp, const int* ci, const double* av, const int* pp,
                    const int* pc, const double* pv, const double* d, int uf, const double* b,
                    double* x, double tau, int imax, int maxit, double tol_ir, int ortho, int right, int* its,
                    int* nsteps, double* gest, double* dnorm, double* basis0) {
    if (n <= 0 || imax < 1 || maxit < 1 || ortho < 0 || ortho > 2) return -1;
    int status = 0;
    double* r = (double*)malloc(sizeof(double) * (size_t)n);
    double* z = (double*)malloc(sizeof(double) * (size_t)n);
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    double* dw = (double*)malloc(sizeof(double) * (size_t)n);
    double* V = (double*)malloc(sizeof(double) * (size_t)n * (size_t)(maxit + 1));
    double* H = (double*)calloc((size_t)(maxit + 1) * (size_t)maxit, sizeof(double));
    double* cs = (double*)malloc(sizeof(double) * (size_t)maxit);
    double* sn = (double*)malloc(sizeof(double) * (size_t)maxit);
    double* g = (double*)malloc(sizeof(double) * (size_t)(maxit + 1));
    double* yk = (double*)malloc(sizeof(double) * (size_t)maxit);
    double* hp = (double*)malloc(sizeof(double) * (size_t)(maxit + 1));
    double* HR = ortho == 2 ? (double*)calloc((size_t)(maxit + 1) * (size_t)maxit, sizeof(double)) : NULL;
    double* bb = (double*)malloc(sizeof(double) * (size_t)(maxit + 1));
#define HH(i, j) H[(size_t)(j) * (size_t)(maxit + 1) + (size_t)(i)]

    if (right) oracle_x0_right(n, pp, pc, pv, d, b, uf, x);
    else oracle_x0(n, pp, pc, pv, d, b, uf, x);
    double dprev = INFINITY;
    int step;
    *nsteps = 0;
    for (step = 0; step < imax; ++step) {
        oracle_residual(n, rp, ci, av, b, x, r);
        if (right) memcpy(z, r, sizeof(double) * (size_t)n);   /* GMRES on A P y = r_i */
        else apply_P(n, pp, pc, pv, d, r, dw, z);              /* GMRES on P A d = P r_i */
        double beta0 = sqrt(dot(n, z, z));
        if (beta0 == 0.0) break;  /* the (preconditioned) residual is 0: x_i solves the system */
        its[step] = 0;
        if (gest) gest[step] = 0.0;
        if (dnorm) dnorm[step] = 0.0;
        *nsteps = step + 1;
        for (int i = 0; i < n; ++i) V[i] = z[i] / beta0;
        for (int i = 0; i <= maxit; ++i) g[i] = 0.0;
        g[0] = beta0;
        int k = 0;
        if (ortho == 2) {
            for (size_t q = 0; q < (size_t)(maxit + 1) * (size_t)maxit; ++q) HR[q] = 0.0;
            int hit = 0;
            k = arnoldi_dcgs2(right, n, rp, ci, av, pp, pc, pv, d, V, H, HR, maxit + 1, cs, sn, g, beta0, tau,
                              maxit, w, dw, y, hp, bb, &hit);
            if (hit) status |= IR_MAXIT;
        }
        for (int j = 0; j < maxit && ortho != 2; ++j) {
            double* vj = V + (size_t)j * n;
            apply_op(right, n, rp, ci, av, pp, pc, pv, d, vj, w, dw, y);
            if (ortho == 0) {
                for (int l = 0; l <= j; ++l) {        /* modified Gram-Schmidt */
                    double* vl = V + (size_t)l * n;
                    double h = dot(n, y, vl);
                    HH(l, j) = h;
                    for (int i = 0; i < n; ++i) y[i] -= h * vl[i];
                }
            } else {
                /* classical Gram-Schmidt applied twice: h = V^T y, y -= V h,
                 * h2 = V^T y, y -= V h2, H(:, j) = h + h2 */
                for (int l = 0; l <= j; ++l) HH(l, j) = 0.0;
                for (int pass = 0; pass < 2; ++pass) {
                    for (int l = 0; l <= j; ++l) hp[l] = dot(n, y, V + (size_t)l * n);
                    for (int l = 0; l <= j; ++l) {
                        double* vl = V + (size_t)l * n;
                        for (int i = 0; i < n; ++i) y[i] -= hp[l] * vl[i];
                        HH(l, j) += hp[l];
                    }
                }
            }
            double hn = sqrt(dot(n, y, y));
            HH(j + 1, j) = hn;
            for (int l = 0; l < j; ++l) {             /* previous rotations */
                double a = HH(l, j), c2 = HH(l + 1, j);
                HH(l, j) = cs[l] * a + sn[l] * c2;
                HH(l + 1, j) = -sn[l] * a + cs[l] * c2;
            }
            double delta = hypot(HH(j, j), HH(j + 1, j));
            cs[j] = HH(j, j) / delta;
            sn[j] = HH(j + 1, j) / delta;
            HH(j, j) = delta;
            HH(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            if (fabs(g[j + 1]) <= tau * beta0 || hn == 0.0) break;
            if (j + 1 == maxit) { status |= IR_MAXIT; break; }
            double* vn = V + (size_t)(j + 1) * n;
            for (int i = 0; i < n; ++i) vn[i] = y[i] / hn;
        }
        its[step] = k;
        if (gest) gest[step] = fabs(g[k]) / beta0;
        /* inspection: the first step's orthonormal basis v_0 .. v_{k-1} (n x k,
         * column-major; maxit columns reserved by the caller) */
        if (basis0 && step == 0) memcpy(basis0, V, sizeof(double) * (size_t)n * (size_t)k);
        /* back substitution H(1:k,1:k) y = g(1:k) */
        for (int c = k - 1; c >= 0; --c) {
            double s = g[c];
            for (int c2 = c + 1; c2 < k; ++c2) s -= HH(c, c2) * yk[c2];
            yk[c] = s / HH(c, c);
        }
        /* d = V_k y (left) or d = P V_k y (right); x = x + d */
        for (int i = 0; i < n; ++i) {
            double di = 0.0;
            for (int c = 0; c < k; ++c) di += V[(size_t)c * n + i] * yk[c];
            w[i] = di;
        }
        if (right) {
            apply_P_right(n, pp, pc, pv, d, w, y);
            memcpy(w, y, sizeof(double) * (size_t)n);
        }
        double dn = 0.0;
        for (int i = 0; i < n; ++i) {
            const double di = w[i];
            if (fabs(di) > dn) dn = fabs(di);
            x[i] = x[i] + di;
        }
        if (dnorm) dnorm[step] = dn;
        double xn = norm_inf(n, x);
        if (dn <= tol_ir * xn) break;
        if (step >= 2 && dn > 0.5 * dprev) { status |= IR_STAGNATED; break; }
        dprev = dn;
        if (step == imax - 1) status |= IR_NOCONV;
    }
#undef HH
    free(r); free(z); free(w); free(y); free(dw); free(V); free(H); free(cs); free(sn);
    free(g); free(yk); free(hp); free(HR); free(bb);
    return status;
}

/*
 * SPAI-GMRES-IR with working precision u = u_g = u_p = single and residual
 * precision u_r = double (the precision sets (half, single, double) and
 * (single, single, double) of Tables 4 and 5).  Every quantity Algorithm 3
 * stores in u is a binary32 value: A and b (rounded to binary32 on entry; the
 * paper's data are given in u), the scaling d, x0, r_i, the Krylov basis, the
 * Hessenberg matrix, the rotations, d_i and x.  The residual is evaluated in
 * binary64 (products of binary32 values are exact there; the row's terms are
 * subtracted from b_i one by one in CSR order) and then rounded to binary32.
 * P is applied in binary32: D w rounded per element, then each row's sum in
 * ascending column order with fused multiply-adds; A likewise.  Inner products
 * and norms are sequential binary32 sums with fused multiply-adds.  GMRES is
 * MGS with the same stopping rules as oracle_gmres_ir; the refinement stops
 * when ||d_i||_inf <= tol_ir ||x_{i+1}||_inf, after imax steps, on stagnation
 * (from the third step) or before a step whose P r_i is exactly zero.  uf must
 * be a binary32 or 16-bit format (u_f no finer than u).  x (out) receives the
 * binary32 solution as doubles.
 */
static float dot32(int n, const float* a, const float* b) {
    float s = 0.0f;
    for (int i = 0; i < n; ++i) s = fmaf(a[i], b[i], s);
    return s;
}

static void apply_P32(int n, const int* pp, const int* pc, const float* pv, const float* d, const float* w,
                      float* dw, float* y) {
    for (int j = 0; j < n; ++j) dw[j] = d[j] * w[j];
    for (int k = 0; k < n; ++k) {
        float s = 0.0f;
        for (int t = pp[k]; t < pp[k + 1]; ++t) s = fmaf(pv[t], dw[pc[t]], s);
        y[k] = s;
    }
}

static void spmv32(int n, const int* rp, const int* ci, const float* av, const float* x, float* y) {
    for (int i = 0; i < n; ++i) {
        float s = 0.0f;
        for (int t = rp[i]; t < rp[i + 1]; ++t) s = fmaf(av[t], x[ci[t]], s);
        y[i] = s;
    }
}

int oracle_gmres_ir_fp32(int n, const int* rp, const int* ci, const double* av, const int* pp,
                         const int* pc, const double* pv, const double* d, int uf, const double* b,
                         double* x, double tau, int imax, int maxit, double tol_ir, int* its, int* nsteps,
                         double* gest, double* dnorm, const double* x_init, double* xhist, double* gprev) {
    if (n <= 0 || imax < 1 || maxit < 1 || uf == OR_FP64) return -1;
    const int nnz = rp[n], pnz = pp[n];
    float* af = (float*)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    float* pf = (float*)malloc(sizeof(float) * (size_t)(pnz > 0 ? pnz : 1));
    float* df = (float*)malloc(sizeof(float) * (size_t)n);
    float* bf = (float*)malloc(sizeof(float) * (size_t)n);
    float* xf = (float*)malloc(sizeof(float) * (size_t)n);
    float* r = (float*)malloc(sizeof(float) * (size_t)n);
    float* z = (float*)malloc(sizeof(float) * (size_t)n);
    float* w = (float*)malloc(sizeof(float) * (size_t)n);
    float* y = (float*)malloc(sizeof(float) * (size_t)n);
    float* dw = (float*)malloc(sizeof(float) * (size_t)n);
    float* V = (float*)malloc(sizeof(float) * (size_t)n * (size_t)(maxit + 1));
    float* H = (float*)calloc((size_t)(maxit + 1) * (size_t)maxit, sizeof(float));
    float* cs = (float*)malloc(sizeof(float) * (size_t)maxit);
    float* sn = (float*)malloc(sizeof(float) * (size_t)maxit);
    float* g = (float*)malloc(sizeof(float) * (size_t)(maxit + 1));
    float* yk = (float*)malloc(sizeof(float) * (size_t)maxit);
    double* x0 = (double*)malloc(sizeof(double) * (size_t)n);
#define HH(i, j) H[(size_t)(j) * (size_t)(maxit + 1) + (size_t)(i)]
    for (int t = 0; t < nnz; ++t) af[t] = (float)av[t];
    for (int t = 0; t < pnz; ++t) pf[t] = (float)pv[t];
    for (int i = 0; i < n; ++i) {
        df[i] = (float)d[i];
        bf[i] = (float)b[i];
    }
    /* x0 = P b in u_f (as in the double-precision variant), stored in u; or the
     * given first iterate, as rounded to u */
    if (x_init) for (int i = 0; i < n; ++i) xf[i] = (float)x_init[i];
    else {
        oracle_x0(n, pp, pc, pv, d, b, uf, x0);
        for (int i = 0; i < n; ++i) xf[i] = (float)x0[i];
    }
    if (xhist) for (int i = 0; i < n; ++i) xhist[i] = (double)xf[i];
    int status = 0;
    float dprev = INFINITY;
    *nsteps = 0;
    for (int step = 0; step < imax; ++step) {
        for (int i = 0; i < n; ++i) {           /* r = b - A x in double, stored in single */
            double s = (double)bf[i];
            for (int t = rp[i]; t < rp[i + 1]; ++t) s = fma(-(double)af[t], (double)xf[ci[t]], s);
            r[i] = (float)s;
        }
        apply_P32(n, pp, pc, pf, df, r, dw, z);
        const float beta0 = sqrtf(dot32(n, z, z));
        if (beta0 == 0.0f) break;
        its[step] = 0;
        if (gest) gest[step] = 0.0;
        if (dnorm) dnorm[step] = 0.0;
        *nsteps = step + 1;
        for (int i = 0; i < n; ++i) V[i] = z[i] / beta0;
        for (int i = 0; i <= maxit; ++i) g[i] = 0.0f;
        g[0] = beta0;
        int k = 0;
        float glast = beta0, gcur = beta0;   /* |g_{j+1}| of the previous and the current iteration */
        for (int j = 0; j < maxit; ++j) {
            float* vj = V + (size_t)j * n;
            spmv32(n, rp, ci, af, vj, w);
            apply_P32(n, pp, pc, pf, df, w, dw, y);
            for (int l = 0; l <= j; ++l) {             /* modified Gram-Schmidt */
                const float* vl = V + (size_t)l * n;
                const float h = dot32(n, y, vl);
                HH(l, j) = h;
                for (int i = 0; i < n; ++i) y[i] = fmaf(-h, vl[i], y[i]);
            }
            const float hn = sqrtf(dot32(n, y, y));
            HH(j + 1, j) = hn;
            for (int l = 0; l < j; ++l) {
                const float a = HH(l, j), c2 = HH(l + 1, j);
                HH(l, j) = cs[l] * a + sn[l] * c2;
                HH(l + 1, j) = -sn[l] * a + cs[l] * c2;
            }
            const float delta = hypotf(HH(j, j), HH(j + 1, j));
            cs[j] = HH(j, j) / delta;
            sn[j] = HH(j + 1, j) / delta;
            HH(j, j) = delta;
            HH(j + 1, j) = 0.0f;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            glast = gcur;
            gcur = fabsf(g[j + 1]);
            if (fabsf(g[j + 1]) <= (float)tau * beta0 || hn == 0.0f) break;
            if (j + 1 == maxit) { status |= IR_MAXIT; break; }
            float* vn = V + (size_t)(j + 1) * n;
            for (int i = 0; i < n; ++i) vn[i] = y[i] / hn;
        }
        its[step] = k;
        if (gest) gest[step] = (double)(fabsf(g[k]) / beta0);
        /* the estimate one iteration earlier, which did not stop (beta0 for k = 1):
         * with gest it tells how close the stopping test came to another count */
        if (gprev) gprev[step] = (double)(glast / beta0);
        for (int c = k - 1; c >= 0; --c) {
            float s = g[c];
            for (int c2 = c + 1; c2 < k; ++c2) s = fmaf(-HH(c, c2), yk[c2], s);
            yk[c] = s / HH(c, c);
        }
        float dn = 0.0f, xn = 0.0f;
        for (int i = 0; i < n; ++i) {
            float di = 0.0f;
            for (int c = 0; c < k; ++c) di = fmaf(V[(size_t)c * n + i], yk[c], di);
            xf[i] = xf[i] + di;
            if (fabsf(di) > dn) dn = fabsf(di);
            if (fabsf(xf[i]) > xn) xn = fabsf(xf[i]);
        }
        if (dnorm) dnorm[step] = (double)dn;
        if (xhist) for (int i = 0; i < n; ++i) xhist[(size_t)(step + 1) * (size_t)n + i] = (double)xf[i];
        if ((double)dn <= tol_ir * (double)xn) break;
        if (step >= 2 && dn > 0.5f * dprev) { status |= IR_STAGNATED; break; }
        dprev = dn;
        if (step == imax - 1) status |= IR_NOCONV;
    }
#undef HH
    for (int i = 0; i < n; ++i) x[i] = (double)xf[i];
    free(af); free(pf); free(df); free(bf); free(xf); free(r); free(z); free(w); free(y); free(dw);
    free(V); free(H); free(cs); free(sn); free(g); free(yk); free(x0);
    return status;
}

/* y = P w in FP64 (for tests of the application of the preconditioner) */
void oracle_apply_P(int n, const int* pp, const int* pc, const double* pv, const double* d,
                    const double* w, double* y) {
    double* dw = (double*)malloc(sizeof(double) * (size_t)n);
    apply_P(n, pp, pc, pv, d, w, dw, y);
    free(dw);
}
