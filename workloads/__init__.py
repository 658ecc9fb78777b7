"""Seeded synthetic inputs for SPAI-GMRES-IR.

This module is shared by the CPU oracle (``oracle/``) and by the GPU library's
tests and benchmark.  It holds input generators only: sparse matrices, exact
right-hand sides, prescribed sparsity patterns and the parameter sets that go
with each workload.  No step of the sparse approximate inverse construction
(Algorithm 1) or of the refinement loop (Algorithm 3) lives here.

The paper evaluates on SuiteSparse matrices (Section 4, Table ``tab:mats``)
that are not available here, so every workload is a synthetic stand-in with
the structure of the paper's problem class: nonsymmetric sparse matrices with
nonzero diagonals (Section 4 restricts itself to those), solved with an
identity or prescribed initial SPAI pattern.

Exact right-hand sides
----------------------
A forward error of 1e-12 can only be measured against a solution that is
known exactly.  Every value a_ij is a multiple of 2^-p with |a_ij| < 2^m, every
x_true component a multiple of 2^-s with |x| <= 1, and a row holds at most q
entries.  When m + p + s + ceil(log2 q) <= 53 every partial sum of A @ x_true
is an integer multiple of 2^-(p+s) below 2^53 in magnitude, so b = A x_true is
computed exactly (here with int64 arithmetic) and x_true is the exact solution
of A x = b in FP64.  ``exact_rhs`` verifies the budget and fails loudly.

Seeds
-----
Every random draw comes from PCG64 seeded by
``SeedSequence([220210204, config_id, size_tag, purpose])``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

ROOT_SEED = 220210204

# purposes for seed streams
_COEF, _XTRUE, _TRACE, _SIZES = 0, 1, 2, 3


def rng_for(config_id: int, size_tag: int, purpose: int) -> np.random.Generator:
    """PCG64 generator for one (config, size, purpose) stream."""
    ss = np.random.SeedSequence([ROOT_SEED, int(config_id), int(size_tag), int(purpose)])
    return np.random.Generator(np.random.PCG64(ss))


@dataclasses.dataclass
class CSR:
    """Compressed sparse row matrix: int32 indices, sorted columns, FP64 values."""

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def row_nnz(self) -> np.ndarray:
        return np.diff(self.rowptr)


@dataclasses.dataclass
class Pattern:
    """Prescribed SPAI pattern: column k of M has row indices idx[ptr[k]:ptr[k+1]]."""

    n: int
    ptr: np.ndarray
    idx: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.ptr[-1])


def _assemble(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """Sum duplicate (row, col) entries and return sorted CSR without stored zeros."""
    key = rows.astype(np.int64) * n + cols.astype(np.int64)
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    uniq, start = np.unique(key, return_index=True)
    summed = np.add.reduceat(vals, start) if len(vals) else vals
    keep = summed != 0.0
    uniq = uniq[keep]
    summed = summed[keep]
    r = (uniq // n).astype(np.int64)
    c = (uniq % n).astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    if rowptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32")
    return CSR(n, rowptr.astype(np.int32), c, summed.astype(np.float64))


def _quantize(x: np.ndarray, bits: int) -> np.ndarray:
    """Round to the nearest multiple of 2^-bits (ties to even)."""
    return np.ldexp(np.rint(np.ldexp(x, bits)), -bits)


# ---------------------------------------------------------------------------
# 2D convection-diffusion, 5-point stencil, first-order upwind
# ---------------------------------------------------------------------------

def convdiff2d(N: int, peclet: float, kappa_range: Optional[tuple] = None,
               rng: Optional[np.random.Generator] = None, pbits: int = 30) -> CSR:
    """-div(kappa grad u) + w . grad u on (0,1)^2, N x N interior points, h = 1/(N+1).

    Dirichlet boundary values are eliminated and unknowns ordered
    lexicographically (x fastest), the natural ordering the paper uses for
    SPAI-GMRES-IR (Section 4).  w = (Pe/sqrt 2)(1, 1) with Pe = |w| L / nu,
    L = nu = 1.  The equation is scaled by h^2, so a face contributes its
    diffusion coefficient and an upwind (west/south) neighbour additionally
    h*w.  kappa is 1 everywhere when ``kappa_range`` is None, otherwise it is
    drawn per grid point log-uniformly from the range, and a face takes the
    harmonic mean of its two points (the point's own value on the boundary).
    Face coefficients are quantised to multiples of 2^-pbits before assembly
    so the diagonal equals the exact sum of the quantised face terms.
    """
    n = N * N
    h = 1.0 / (N + 1)
    wx = wy = peclet / math.sqrt(2.0)
    if kappa_range is None:
        kap = np.ones((N, N))
    else:
        lo, hi = kappa_range
        kap = np.exp(rng.uniform(math.log(lo), math.log(hi), size=(N, N)))
    idx = np.arange(n).reshape(N, N)  # [iy, ix]

    def hmean(a, b):
        return 2.0 * a * b / (a + b)

    cx = _quantize(h * wx, pbits)
    cy = _quantize(h * wy, pbits)
    rows, cols, vals = [], [], []
    diag = np.zeros((N, N))
    # x-direction faces between (iy, ix) and (iy, ix+1)
    kf = _quantize(hmean(kap[:, :-1], kap[:, 1:]), pbits)
    left, right = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    kfr = kf.ravel()
    rows += [left, right]
    cols += [right, left]
    vals += [-kfr, -kfr - cx]          # right point's west neighbour is upwind
    diag[:, :-1] += kf
    diag[:, 1:] += kf
    # y-direction faces between (iy, ix) and (iy+1, ix)
    kf = _quantize(hmean(kap[:-1, :], kap[1:, :]), pbits)
    low, up = idx[:-1, :].ravel(), idx[1:, :].ravel()
    kfr = kf.ravel()
    rows += [low, up]
    cols += [up, low]
    vals += [-kfr, -kfr - cy]          # upper point's south neighbour is upwind
    diag[:-1, :] += kf
    diag[1:, :] += kf
    # boundary faces
    kb = _quantize(kap, pbits)
    diag[:, 0] += kb[:, 0]
    diag[:, -1] += kb[:, -1]
    diag[0, :] += kb[0, :]
    diag[-1, :] += kb[-1, :]
    diag += cx + cy
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    return _assemble(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


# ---------------------------------------------------------------------------
# 3D anisotropic diffusion, 7-point stencil, coefficient jumps
# ---------------------------------------------------------------------------

def aniso3d(N: int, rng: np.random.Generator, jump: float = 1e4, jump_frac: float = 0.05,
            aniso=(1.0, 1.0, 1e-3), pbits: int = 24) -> CSR:
    """7-point cell-centred diffusion on an N^3 grid (x fastest ordering).

    Cell coefficient c = ``jump`` with probability ``jump_frac``, else 1.  The
    coefficient of the face between two cells is the harmonic mean of theirs
    times the anisotropy factor of the face direction; a boundary face uses
    the cell's own coefficient.  a_ij = -k_face and a_ii = sum of the faces of
    cell i including boundary faces (an M-matrix).  Face values are quantised
    to multiples of 2^-pbits before assembly.
    """
    n = N ** 3
    c = np.where(rng.random((N, N, N)) < jump_frac, jump, 1.0)  # [iz, iy, ix]
    idx = np.arange(n).reshape(N, N, N)
    diag = np.zeros((N, N, N))
    rows, cols, vals = [], [], []
    for axis, fac in zip((2, 1, 0), aniso):  # x, y, z
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[axis] = slice(0, N - 1)
        sl_hi[axis] = slice(1, N)
        a, b = c[tuple(sl_lo)], c[tuple(sl_hi)]
        kf = _quantize(fac * 2.0 * a * b / (a + b), pbits)
        i_lo, i_hi = idx[tuple(sl_lo)].ravel(), idx[tuple(sl_hi)].ravel()
        rows += [i_lo, i_hi]
        cols += [i_hi, i_lo]
        vals += [-kf.ravel(), -kf.ravel()]
        diag[tuple(sl_lo)] += kf
        diag[tuple(sl_hi)] += kf
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = 0
        last[axis] = N - 1
        diag[tuple(first)] += _quantize(fac * c[tuple(first)], pbits)
        diag[tuple(last)] += _quantize(fac * c[tuple(last)], pbits)
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    return _assemble(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


# ---------------------------------------------------------------------------
# random banded nonsymmetric systems
# ---------------------------------------------------------------------------

def random_banded(n: int, rng: np.random.Generator, kmin: int = 4, kmax: int = 12,
                  half_band: int = 32, dominance: float = 1.1, pbits: int = 26) -> CSR:
    """Row i holds k_i ~ U{kmin..kmax} entries including the diagonal.

    Off-diagonal columns are drawn without replacement from
    [i-half_band, i+half_band-1] intersected with [0, n), values N(0,1)
    quantised to 2^-pbits, and a_ii = dominance * sum_{j != i} |a_ij| (then
    quantised), so every row is strictly diagonally dominant.
    """
    rows, cols, vals = [], [], []
    ks = rng.integers(kmin, kmax + 1, size=n)
    for i in range(n):
        lo, hi = max(0, i - half_band), min(n, i + half_band)
        cand = np.array([j for j in range(lo, hi) if j != i])
        k = min(int(ks[i]) - 1, len(cand))
        js = np.sort(rng.choice(cand, size=k, replace=False)) if k > 0 else np.zeros(0, np.int64)
        v = _quantize(rng.standard_normal(k), pbits)
        v[v == 0.0] = 2.0 ** -pbits
        d = _quantize(dominance * np.abs(v).sum(), pbits)
        if d == 0.0:
            d = 1.0
        rows.append(np.full(k + 1, i))
        cols.append(np.concatenate([js, [i]]))
        vals.append(np.concatenate([v, [d]]))
    return _assemble(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


# ---------------------------------------------------------------------------
# exact right-hand side
# ---------------------------------------------------------------------------

def exact_rhs(A: CSR, rng: np.random.Generator, pbits: int, sbits: int):
    """Draw x_true ~ U(-1,1) on the 2^-sbits grid and return (x_true, b = A x_true exactly)."""
    aint = np.ldexp(A.val, pbits)
    if not np.array_equal(aint, np.rint(aint)):
        raise ValueError("matrix values are not multiples of 2^-pbits")
    mbits = int(math.floor(math.log2(np.abs(A.val).max()))) + 1
    q = int(A.row_nnz().max())
    budget = mbits + pbits + sbits + int(math.ceil(math.log2(max(q, 1))))
    if budget > 53:
        raise ValueError(f"exact-RHS bit budget {budget} > 53")
    x = _quantize(rng.uniform(-1.0, 1.0, size=A.n), sbits)
    xint = np.rint(np.ldexp(x, sbits)).astype(np.int64)
    prod = aint.astype(np.int64) * xint[A.col]
    rows = np.repeat(np.arange(A.n), A.row_nnz())
    bint = np.zeros(A.n, dtype=np.int64)
    np.add.at(bint, rows, prod)
    if np.abs(bint).max(initial=0) >= 2**53:
        raise ValueError("exact-RHS sum exceeds 2^53")
    b = np.ldexp(bint.astype(np.float64), -(pbits + sbits))
    return x, b


# ---------------------------------------------------------------------------
# prescribed patterns
# ---------------------------------------------------------------------------

def pattern_of(A: CSR) -> Pattern:
    """pattern(P) = pattern(A): column k of M (row k of P) takes row k of A's columns."""
    return Pattern(A.n, A.rowptr.copy(), A.col.copy())


def pattern_power2_trunc(A: CSR, cap: int) -> Pattern:
    """pattern(P) = pattern(A^2) truncated to ``cap`` entries per row of P.

    Truncation keeps the diagonal, then the largest (|A|^2)_kj, ties to the
    smaller j; rows with at most ``cap`` entries are kept whole.
    """
    S = A.to_scipy()
    S.data = np.abs(S.data)
    S2 = (S @ S).tocsr()
    S2.sort_indices()
    counts = np.diff(S2.indptr)
    if counts.max(initial=0) <= cap:
        return Pattern(A.n, S2.indptr.astype(np.int32), S2.indices.astype(np.int32))
    ptr = [0]
    idx = []
    for k in range(A.n):
        cols = S2.indices[S2.indptr[k]:S2.indptr[k + 1]]
        w = S2.data[S2.indptr[k]:S2.indptr[k + 1]]
        if len(cols) > cap:
            order = sorted(range(len(cols)), key=lambda t: (cols[t] != k, -w[t], cols[t]))
            cols = np.sort(cols[order[:cap]])
        idx.append(cols)
        ptr.append(ptr[-1] + len(cols))
    return Pattern(A.n, np.asarray(ptr, np.int32), np.concatenate(idx).astype(np.int32))


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SpaiParams:
    eps: float
    alpha: int            # maximum augmentation steps (0 = fixed pattern)
    beta: int             # maximum indices added per step
    maxfill: int          # cap on |J_k|
    u_f: str              # "fp64" | "fp32" | "fp16" | "bf16"


@dataclasses.dataclass
class IrParams:
    tau: float            # GMRES relative tolerance
    imax: int             # maximum refinement steps
    maxit: int            # maximum GMRES iterations per refinement step
    tol_ir: float         # refinement stops when ||d||_inf <= tol_ir ||x||_inf
    u: str = "fp64"       # working precision u = u_g = u_p ("fp64" or "fp32")


@dataclasses.dataclass
class Workload:
    name: str
    A: CSR
    x_true: np.ndarray
    b: np.ndarray
    pattern: Optional[Pattern]   # None = identity initial pattern
    spai: SpaiParams
    ir: IrParams
    recipe: str

    @property
    def n(self) -> int:
        return self.A.n


TOL_IR = 2.0 ** -45   # refinement stops once ||d||_inf <= 2^-45 ||x||_inf (about 256 u)
TOL_IR32 = 2.0 ** -16  # the same 256 u for working precision single


def _convdiff_pbits(N: int, peclet: float, sbits: int) -> int:
    """Largest value grid 2^-p that keeps the exact-RHS budget (q = 5 entries per row)."""
    bound = 4.0 + 2.0 * (peclet / math.sqrt(2.0)) / (N + 1)     # max diagonal, kappa <= 1
    mbits = int(math.floor(math.log2(bound))) + 1
    return min(30, 53 - sbits - 3 - mbits)


def convdiff_small(N: int = 32) -> Workload:
    """2D convection-diffusion, Pe 10, fixed SPAI pattern = pattern(A), FP32 SPAI.

    Full size N = 32 (n = 1024, nnz = 4992)."""
    pb = _convdiff_pbits(N, 10.0, 17)
    A = convdiff2d(N, 10.0, None, None, pbits=pb)
    x, b = exact_rhs(A, rng_for(1, N, _XTRUE), pbits=pb, sbits=17)
    return Workload(f"convdiff2d_pe10_{N}x{N}_fixedA", A, x, b, pattern_of(A),
                    SpaiParams(eps=0.5, alpha=0, beta=8, maxfill=max(A.row_nnz().max(), 1), u_f="fp32"),
                    IrParams(tau=1e-10, imax=10, maxit=min(A.n, 500), tol_ir=TOL_IR),
                    f"convdiff2d N={N} Pe=10 kappa=1, values on 2^-{pb} grid, x_true on 2^-17 grid")


def convdiff_adaptive(N: int = 512, u_f: str = "fp32") -> Workload:
    """2D convection-diffusion, Pe 100, kappa log-uniform in [1e-2, 1], adaptive SPAI.

    Identity start, eps = 0.3, beta = 8, alpha = ceil(n/beta), at most 20 entries
    per column, FP32 SPAI, FP64 GMRES with tau = 1e-8.  Full size N = 512
    (n = 262144, nnz = 1,308,672)."""
    pb = _convdiff_pbits(N, 100.0, 17)
    A = convdiff2d(N, 100.0, (1e-2, 1.0), rng_for(2, N, _COEF), pbits=pb)
    x, b = exact_rhs(A, rng_for(2, N, _XTRUE), pbits=pb, sbits=17)
    n = A.n
    return Workload(f"convdiff2d_pe100_logk_{N}x{N}_adaptive", A, x, b, None,
                    SpaiParams(eps=0.3, alpha=-(-n // 8), beta=8, maxfill=20, u_f=u_f),
                    IrParams(tau=1e-8, imax=10, maxit=min(n, 500), tol_ir=TOL_IR),
                    f"convdiff2d N={N} Pe=100 kappa~logU[1e-2,1] harmonic faces, values on 2^-{pb} grid, "
                    f"x_true on 2^-17 grid")


def aniso_fixed(N: int = 128, u_f: str = "fp16") -> Workload:
    """3D anisotropic diffusion with 1e4 jumps in 5% of cells, pattern(A^2) capped at 27."""
    A = aniso3d(N, rng_for(3, N, _COEF), pbits=24)
    x, b = exact_rhs(A, rng_for(3, N, _XTRUE), pbits=24, sbits=10)
    pat = pattern_power2_trunc(A, 27)
    n = A.n
    return Workload(f"aniso3d_{N}^3_fixedA2", A, x, b, pat,
                    SpaiParams(eps=0.5, alpha=0, beta=8, maxfill=27, u_f=u_f),
                    IrParams(tau=1e-8, imax=10, maxit=min(n, 500), tol_ir=TOL_IR),
                    f"aniso3d N={N} jumps 1e4 in 5% cells, anisotropy (1,1,1e-3), values on 2^-24 grid, "
                    f"x_true on 2^-10 grid")


def random_banded_rows(n: int, rng: np.random.Generator, kmin: int = 4, kmax: int = 12,
                       half_band: int = 32, dominance: float = 1.1, pbits: int = 26) -> CSR:
    """The structure of ``random_banded`` drawn row-parallel (its own stream).

    Row i holds k_i ~ U{kmin..kmax} entries including the diagonal; the k_i - 1
    off-diagonal columns are the candidates i + o, o in [-half_band, half_band-1]
    without 0 and inside [0, n), with the smallest of independent U(0,1) keys
    (a uniform draw without replacement); values N(0,1) on the 2^-pbits grid
    (an exact zero becomes 2^-pbits) and a_ii = dominance * sum_j |a_ij| on the
    grid."""
    ks = rng.integers(kmin, kmax + 1, size=n)
    offs = np.concatenate([np.arange(-half_band, 0), np.arange(1, half_band)])
    cand = np.arange(n, dtype=np.int64)[:, None] + offs[None, :]
    valid = (cand >= 0) & (cand < n)
    keys = rng.random(cand.shape)
    keys[~valid] = 2.0
    m = min(kmax - 1, offs.size)               # the m smallest keys of a row, in ascending order
    part = np.argpartition(keys, m - 1, axis=1)[:, :m]
    order = np.take_along_axis(part, np.argsort(np.take_along_axis(keys, part, axis=1), axis=1), axis=1)
    kk = np.minimum(ks - 1, valid.sum(axis=1))
    take = np.arange(m)[None, :] < kk[:, None]
    cols = np.take_along_axis(cand, order, axis=1)[take]
    rows = np.repeat(np.arange(n), kk)
    v = _quantize(rng.standard_normal(cols.size), pbits)
    v[v == 0.0] = 2.0 ** -pbits
    d = _quantize(dominance * np.bincount(rows, weights=np.abs(v), minlength=n), pbits)
    d[d == 0.0] = 1.0
    return _assemble(n, np.concatenate([rows, np.arange(n)]), np.concatenate([cols, np.arange(n)]),
                     np.concatenate([v, d]))


@dataclasses.dataclass
class Batch:
    """Independent systems stored as one block-diagonal matrix: system s owns rows
    and columns sys_ptr[s] .. sys_ptr[s+1]-1."""

    name: str
    sys_ptr: np.ndarray
    A: CSR
    x_true: np.ndarray
    b: np.ndarray
    spai: SpaiParams
    ir: IrParams
    recipe: str

    @property
    def nsys(self) -> int:
        return len(self.sys_ptr) - 1

    @property
    def n(self) -> int:
        return self.A.n

    def system(self, s: int) -> Workload:
        """System s alone (indices rebased), with the batch's parameters."""
        r0, r1 = int(self.sys_ptr[s]), int(self.sys_ptr[s + 1])
        q0, q1 = int(self.A.rowptr[r0]), int(self.A.rowptr[r1])
        A = CSR(r1 - r0, (self.A.rowptr[r0:r1 + 1] - q0).astype(np.int32),
                (self.A.col[q0:q1] - r0).astype(np.int32), self.A.val[q0:q1].copy())
        return Workload(f"{self.name}_sys{s}", A, self.x_true[r0:r1].copy(), self.b[r0:r1].copy(), None,
                        dataclasses.replace(self.spai),
                        dataclasses.replace(self.ir, maxit=min(A.n, self.ir.maxit)), self.recipe)


def random_batch(nsys: int = 4096, nmin: int = 200, nmax: int = 20000) -> Batch:
    """Many independent random banded systems (4-12 entries per row within a band
    of 64, N(0,1), dominance 1.1), sizes log-uniform in [nmin, nmax]; adaptive
    FP32 SPAI (identity start, eps 0.3, beta 8, at most 20 entries per column;
    alpha = ceil(nmin / 8) >= 3 steps, which the fill cap reaches first: at most
    (20 - 1) / 8 + 1 = 3 augmentations), FP64 GMRES-IR with a double-double
    residual, tau 1e-8, maxit min(n_s, 500).  Full size: 4096 systems,
    sum n ~ 1.8e7."""
    sz = rng_for(5, nsys, _SIZES)
    ns = np.rint(np.exp(sz.uniform(math.log(nmin), math.log(nmax), size=nsys))).astype(np.int64)
    ptr = np.zeros(nsys + 1, np.int64)
    ptr[1:] = np.cumsum(ns)
    rps, cols, vals, xs, bs = [], [], [], [], []
    nnz_off = 0
    for s in range(nsys):
        n = int(ns[s])
        A = random_banded_rows(n, rng_for(5, 1_000_000 + s, _COEF))
        x, b = exact_rhs(A, rng_for(5, 1_000_000 + s, _XTRUE), pbits=26, sbits=16)
        rps.append(A.rowptr[:-1].astype(np.int64) + nnz_off)
        cols.append(A.col + ptr[s])
        vals.append(A.val)
        xs.append(x)
        bs.append(b)
        nnz_off += A.nnz
    if nnz_off >= 2**31 or ptr[-1] >= 2**31:
        raise ValueError("batch exceeds int32 indices")
    rowptr = np.concatenate(rps + [np.array([nnz_off])]).astype(np.int32)
    A = CSR(int(ptr[-1]), rowptr, np.concatenate(cols).astype(np.int32), np.concatenate(vals))
    return Batch(f"random_batch_{nsys}_n{nmin}-{nmax}", ptr, A, np.concatenate(xs), np.concatenate(bs),
                 SpaiParams(eps=0.3, alpha=-(-nmin // 8), beta=8, maxfill=20, u_f="fp32"),
                 IrParams(tau=1e-8, imax=10, maxit=500, tol_ir=TOL_IR),
                 f"{nsys} random banded systems, n log-uniform in [{nmin}, {nmax}], 4-12 nnz/row in a band of 64, "
                 f"N(0,1) on 2^-26 grid, diag 1.1 x offdiag abs sum, x_true on 2^-16 grid")


def random_system(n: int, sys_id: int = 0) -> Workload:
    """One random banded nonsymmetric system (4-12 nnz/row, band 64, dominance 1.1), adaptive SPAI."""
    A = random_banded(n, rng_for(4, sys_id * 1000003 + n, _COEF), pbits=26)
    x, b = exact_rhs(A, rng_for(4, sys_id * 1000003 + n, _XTRUE), pbits=26, sbits=16)
    return Workload(f"random_banded_n{n}_s{sys_id}", A, x, b, None,
                    SpaiParams(eps=0.3, alpha=-(-n // 8), beta=8, maxfill=20, u_f="fp32"),
                    IrParams(tau=1e-8, imax=10, maxit=min(n, 500), tol_ir=TOL_IR),
                    f"random banded n={n} 4-12 nnz/row half-band 32, N(0,1) on 2^-26 grid, "
                    f"diag 1.1 x offdiag abs sum, x_true on 2^-16 grid")


# ---------------------------------------------------------------------------
# serving stream: Poisson arrivals of systems of the three families
# ---------------------------------------------------------------------------

SERVE_ALPHA = 125   # augmentation cap of the adaptive families in the stream (see serving_request)


@dataclasses.dataclass
class Arrival:
    t: float      # arrival time in seconds from the start of the stream
    kind: str     # "convdiff" (2D, adaptive), "aniso" (3D, fixed pattern(A^2)), "random" (banded, adaptive)
    size: int     # grid side for convdiff / aniso, n for random
    u_f: str      # "fp16" or "fp32"
    req_id: int


def serving_trace(rate: float = 200.0, duration: float = 60.0, tag: int = 0,
                  max_side_2d: int = 512, max_side_3d: int = 128, max_n_random: int = 20000) -> list:
    """Poisson arrivals at ``rate`` per second for ``duration`` seconds; each request
    is uniform over the three families with sizes log-uniform in: 2D side
    [32, max_side_2d], 3D side [10, max_side_3d], random n [1000, max_n_random]
    (so n spans 1e3 .. 2.1e6 at the defaults), and u_f FP16 or FP32 with equal
    probability."""
    rng = rng_for(6, tag, _TRACE)
    out, t, k = [], 0.0, 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            return out
        kind = ("convdiff", "aniso", "random")[int(rng.integers(0, 3))]
        u = float(rng.random())
        if kind == "convdiff":
            size = int(round(math.exp(math.log(32) + u * (math.log(max_side_2d) - math.log(32)))))
        elif kind == "aniso":
            size = int(round(math.exp(math.log(10) + u * (math.log(max_side_3d) - math.log(10)))))
        else:
            size = int(round(math.exp(math.log(1000) + u * (math.log(max_n_random) - math.log(1000)))))
        u_f = "fp16" if rng.random() < 0.5 else "fp32"
        out.append(Arrival(t, kind, size, u_f, k))
        k += 1


def serving_request(a: Arrival) -> Workload:
    """The system of one arrival, from its own seed streams.  The adaptive
    families use alpha = SERVE_ALPHA for every size (not ceil(n / beta)) so that
    requests of different sizes share parameters and can be batched: from the
    identity start with beta = 8 and at most 20 entries per column a column
    takes at most 3 augmentation steps, so any alpha >= 3 gives the same
    preconditioner."""
    tag = 10_000_000 + a.req_id
    if a.kind == "convdiff":
        N = a.size
        pb = _convdiff_pbits(N, 100.0, 17)
        A = convdiff2d(N, 100.0, (1e-2, 1.0), rng_for(6, tag, _COEF), pbits=pb)
        x, b = exact_rhs(A, rng_for(6, tag, _XTRUE), pbits=pb, sbits=17)
        return Workload(f"serve{a.req_id}_convdiff_{N}x{N}", A, x, b, None,
                        SpaiParams(eps=0.3, alpha=SERVE_ALPHA, beta=8, maxfill=20, u_f=a.u_f),
                        IrParams(tau=1e-8, imax=10, maxit=500, tol_ir=TOL_IR),
                        f"convdiff2d N={N} Pe=100 kappa~logU[1e-2,1], values on 2^-{pb} grid, x_true on 2^-17 grid")
    if a.kind == "aniso":
        N = a.size
        A = aniso3d(N, rng_for(6, tag, _COEF), pbits=24)
        x, b = exact_rhs(A, rng_for(6, tag, _XTRUE), pbits=24, sbits=10)
        return Workload(f"serve{a.req_id}_aniso_{N}^3", A, x, b, pattern_power2_trunc(A, 27),
                        SpaiParams(eps=0.5, alpha=0, beta=8, maxfill=27, u_f=a.u_f),
                        IrParams(tau=1e-8, imax=10, maxit=500, tol_ir=TOL_IR),
                        f"aniso3d N={N} jumps 1e4 in 5% cells, values on 2^-24 grid, x_true on 2^-10 grid")
    n = a.size
    A = random_banded_rows(n, rng_for(6, tag, _COEF))
    x, b = exact_rhs(A, rng_for(6, tag, _XTRUE), pbits=26, sbits=16)
    return Workload(f"serve{a.req_id}_random_n{n}", A, x, b, None,
                    SpaiParams(eps=0.3, alpha=SERVE_ALPHA, beta=8, maxfill=20, u_f=a.u_f),
                    IrParams(tau=1e-8, imax=10, maxit=500, tol_ir=TOL_IR),
                    f"random banded n={n} 4-12 nnz/row half-band 32, N(0,1) on 2^-26 grid, x_true on 2^-16 grid")


# ---------------------------------------------------------------------------
# paper-shaped stand-ins for the matrices of Table tab:mats
# ---------------------------------------------------------------------------

# (shape of the table's row, n, nnz, kappa_inf(A), precision set, epsilons of its tables)
# Set "sdq" = (u_f, u, u_r) = (single, double, quad) of Table 3; "hsd" = (half, single,
# double) of Table 4, also run as (single, single, double) in Table 5.
S0_SHAPES = [
    ("pores_3", 532, 3474, 1.2e6, "sdq", (0.5, 0.4)),
    ("steam1", 240, 2248, 3.1e7, "sdq", (0.2, 0.1)),
    ("steam3", 80, 314, 7.6e10, "sdq", (0.5, 0.1)),
    ("saylr1", 238, 1128, 1.6e9, "sdq", (0.4, 0.3)),
    ("bfwa782", 782, 7514, 6.8e3, "hsd", (0.5, 0.3)),
    ("cage5", 37, 233, 2.9e1, "hsd", (0.5, 0.3)),
    ("gre_115", 115, 421, 1.4e2, "hsd", (0.5, 0.3)),
    ("orsreg_1", 2205, 14133, 7.0e3, "hsd", (0.5, 0.3)),
    ("sherman4", 1104, 3786, 3.1e3, "hsd", (0.5, 0.3)),
]


def kappa_inf(A: CSR) -> float:
    """Dense infinity-norm condition number (small n only)."""
    M = A.to_scipy().toarray()
    return float(np.abs(M).sum(axis=1).max() * np.abs(np.linalg.inv(M)).sum(axis=1).max())


def s0_matrix(k: int) -> Workload:
    """Random nonsymmetric stand-in with the n, nnz and (within 10x) kappa_inf of
    row k of Table tab:mats: off-diagonals N(0,1) at distinct random columns within
    a band of +-min(32, n/4), spread evenly over the rows (nnz - n of them), and a
    positive diagonal s * sum_j |a_ij| whose factor s is found by bisection on
    log kappa_inf (dense).  Parameters follow the paper's protocol (identity
    start, beta = 8, alpha = ceil(n / beta), tau = 1e-8 for u = double and 1e-4
    for u = single); the fill cap is the library's largest, 63 entries per
    column, standing in for the paper's uncapped columns.

    Off-diagonals are clipped to +-7.9.  Values of the "sdq" matrices lie on a
    2^-24 grid with x_true on 2^-16 (exact FP64 right-hand side); those of the
    "hsd" matrices, which Tables 4 and 5 solve with working precision single,
    on a 2^-10 grid with x_true on 2^-5, so that A, x_true and b = A x_true are
    exact in FP32 as well when |a| < 2^5 and a row holds at most 16 entries
    (5 + 10 + 5 + 4 = 24 bits; checked by s0_fp32_exact)."""
    name, n, nnz, kappa, pset, eps = S0_SHAPES[k]
    rng = rng_for(7, k, _COEF)
    pbits, sbits = (24, 16) if pset == "sdq" else (10, 5)
    hb = min(32, n // 4)
    off = nnz - n
    base, extra = divmod(off, n)
    ks = np.full(n, base)
    ks[rng.permutation(n)[:extra]] += 1
    offs = np.concatenate([np.arange(-hb, 0), np.arange(1, hb + 1)])
    rows, cols = [], []
    for i in range(n):
        cand = i + offs
        cand = cand[(cand >= 0) & (cand < n)]
        take = rng.permutation(cand)[:min(int(ks[i]), cand.size)]
        rows.append(np.full(take.size, i))
        cols.append(take)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    v = _quantize(np.clip(rng.standard_normal(cols.size), -7.9, 7.9), pbits)
    v[v == 0.0] = 2.0 ** -pbits
    rs = np.bincount(rows, weights=np.abs(v), minlength=n)

    def assemble(s):
        d = _quantize(s * rs, pbits)
        d[d == 0.0] = 2.0 ** -pbits
        return _assemble(n, np.concatenate([rows, np.arange(n)]), np.concatenate([cols, np.arange(n)]),
                         np.concatenate([v, d]))

    def kap(A):
        try:
            return kappa_inf(A)
        except np.linalg.LinAlgError:
            return np.inf

    # A(s) = offdiag + s diag(rowsum) is singular where -s is a real eigenvalue of
    # diag(rowsum)^-1 offdiag (all inside [-1, 1]); kappa_inf(A(s)) grows without
    # bound as s decreases from 2 to the largest such s*, so bisect on log kappa
    # over (s*, 2]
    off_m = np.zeros((n, n))
    off_m[rows, cols] = v
    lam = np.linalg.eigvals(off_m / rs[:, None])
    real = -lam[np.abs(lam.imag) <= 1e-9 * np.maximum(np.abs(lam), 1.0)].real
    s_star = float(real.max()) if real.size else -1.5
    lo, hi = s_star, 2.0
    A_hi = assemble(hi)
    best = (abs(math.log10(kap(A_hi) / kappa)), hi, A_hi)
    for _ in range(80):
        if best[0] <= 0.3:
            break
        mid = 0.5 * (lo + hi)
        A_mid = assemble(mid)
        km = kap(A_mid)
        if np.isfinite(km) and abs(math.log10(km / kappa)) < best[0]:
            best = (abs(math.log10(km / kappa)), mid, A_mid)
        if km >= kappa:
            lo = mid
        else:
            hi = mid
    A = best[2]
    x, b = exact_rhs(A, rng_for(7, k, _XTRUE), pbits=pbits, sbits=sbits)
    single = pset != "sdq"
    return Workload(f"s0_{name}_shape_n{n}", A, x, b, None,
                    SpaiParams(eps=eps[0], alpha=-(-n // 8), beta=8, maxfill=63, u_f="fp16" if single else "fp32"),
                    IrParams(tau=1e-4 if single else 1e-8, imax=10, maxit=n, tol_ir=TOL_IR32 if single else TOL_IR,
                             u="fp32" if single else "fp64"),
                    f"stand-in for the shape of {name} (n={n}, nnz~{nnz}, kappa_inf~{kappa:.1e}); band "
                    f"+-{hb}, N(0,1) on 2^-{pbits} grid, diagonal factor {best[1]:.4g}, x_true on 2^-{sbits} grid")
