"""CPU oracle for SPAI-GMRES-IR — TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU library
computes, written from the paper (Carson & Khan, "Mixed precision iterative
refinement with sparse approximate inverse preconditioning"):

* ``spai``       — Algorithm 1 (Section 2.2) on B = A^T D with the column
                   scaling of Section 4, step by step in the precision u_f
                   (``spai_oracle.c``, explicit rounding of every operation);
* ``ls_column``  — the plain definition of a fixed-pattern column: the FP64
                   least-squares solution of eq. (redprob) (numpy lstsq);
* ``gmres_ir``   — Algorithm 3 (Section 3.2): x0 = P b in u_f, residuals
                   computed exactly and rounded to FP64, left-preconditioned
                   MGS-GMRES in FP64 (u_g = u_p = u, Section 4); or, for the
                   precision sets of Tables 4-5, everything stored in binary32
                   with residuals in binary64;
* ``residual``   — r = fl(b - A x), each component exactly rounded.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It shares no code with the GPU
library (``paper_2202_10204_amd``), and the library never imports it.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spai_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

UF = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3}

FLAG_RANKDEF, FLAG_EPS, FLAG_NONFINITE, FLAG_FALLBACK = 1, 2, 4, 8
IR_MAXIT, IR_NOCONV, IR_STAGNATED = 1, 2, 4


def build() -> str:
    """Compile the C oracle (plain gcc, no contraction, no fast-math)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", _SO + ".tmp", _SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, f64 = ctypes.c_int, ctypes.c_double
        L.oracle_spai.restype = i32
        L.oracle_spai.argtypes = [i32, P, P, P, P, P, f64, i32, i32, i32, i32, P, i32, i32, i32,
                                  P, P, P, P, P, P, P, P, P, P, P]
        L.oracle_spai_probe.restype = i32
        L.oracle_spai_probe.argtypes = [i32, P, P, P, i32, P, i32, P, i32, i32, i32, P, P, P, P, P, P, P,
                                        P, P]
        L.oracle_gmres_ir.restype = i32
        L.oracle_gmres_ir.argtypes = [i32, P, P, P, P, P, P, P, i32, P, P, f64, i32, i32, f64,
                                      i32, i32, P, P, P, P, P]
        L.oracle_x0_right.restype = None
        L.oracle_x0_right.argtypes = [i32, P, P, P, P, P, i32, P]
        L.oracle_gmres_ir_fp32.restype = i32
        L.oracle_gmres_ir_fp32.argtypes = [i32, P, P, P, P, P, P, P, i32, P, P, f64, i32, i32, f64, P, P, P, P,
                                           P, P, P]
        L.oracle_residual.restype = None
        L.oracle_residual.argtypes = [i32, P, P, P, P, P, P]
        L.oracle_exact_sum.restype = f64
        L.oracle_exact_sum.argtypes = [P, i32, P]
        L.oracle_x0.restype = None
        L.oracle_x0.argtypes = [i32, P, P, P, P, P, i32, P]
        L.oracle_apply_P.restype = None
        L.oracle_apply_P.argtypes = [i32, P, P, P, P, P, P]
        L.oracle_scaling.restype = None
        L.oracle_scaling.argtypes = [i32, P, P, P]
        for name in ("oracle_round_fp16", "oracle_round_bf16", "oracle_round_fp32"):
            fn = getattr(L, name)
            fn.restype = f64
            fn.argtypes = [f64]
        _lib_handle = L
    return _lib_handle


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# precision helpers
# ---------------------------------------------------------------------------

def round_to(x: float, uf: str) -> float:
    """Round a binary64 value to u_f (round to nearest, ties to even)."""
    L = _lib()
    if uf == "fp64":
        return float(x)
    if uf == "fp32":
        return L.oracle_round_fp32(float(x))
    if uf == "fp16":
        return L.oracle_round_fp16(L.oracle_round_fp32(float(x)))
    if uf == "bf16":
        return L.oracle_round_bf16(L.oracle_round_fp32(float(x)))
    raise ValueError(uf)


def scaling(A) -> np.ndarray:
    """d_i = 1 / max_j |a_ij| (Section 4: the largest entry of every column of A^T D is 1)."""
    d = np.empty(A.n)
    _lib().oracle_scaling(A.n, _p(_i32(A.rowptr)), _p(_f64(A.val)), _p(d))
    return d


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SpaiResult:
    cols: np.ndarray      # columns k computed
    length: np.ndarray    # |J_k|
    J: np.ndarray         # [ncols, stride] J_k in insertion order, -1 padded
    m: np.ndarray         # [ncols, stride] m-bar values (u_f values held in FP64)
    steps: np.ndarray     # augmentation steps taken
    nI: np.ndarray        # |I_k| at the final solve
    flags: np.ndarray     # FLAG_* bits
    res: np.ndarray       # ||e_k - B m_k||_2 as tested at the final solve
    margin: np.ndarray    # smallest relative decision margin of the column
    d: np.ndarray         # scaling vector D
    hist: np.ndarray      # [ncols, stride+1] residual norm of every solve (NaN padded)
    flops: np.ndarray     # algorithmic flops of the column's solves, 2mp^2 - 2p^3/3 + 4mp + p^2 per m x p solve

    def P_csr(self, n: int):
        """Row k of P = M^T D holds m_k: CSR (rowptr, col, val) with columns ascending.

        Only valid when ``cols`` is all of 0..n-1.  D is kept separate (``d``)."""
        assert len(self.cols) == n and np.array_equal(self.cols, np.arange(n))
        rowptr = np.zeros(n + 1, np.int32)
        rowptr[1:] = np.cumsum(self.length)
        col = np.empty(rowptr[-1], np.int32)
        val = np.empty(rowptr[-1], np.float64)
        for k in range(n):
            L = self.length[k]
            order = np.argsort(self.J[k, :L], kind="stable")
            col[rowptr[k]:rowptr[k + 1]] = self.J[k, :L][order]
            val[rowptr[k]:rowptr[k + 1]] = self.m[k, :L][order]
        return rowptr, col, val


def spai(A, pattern, eps: float, alpha: int, beta: int, maxfill: int, uf: str,
         cols: Optional[np.ndarray] = None, nthreads: int = 1) -> SpaiResult:
    """Algorithm 1 on B = A^T D for the given columns (all by default).

    ``pattern`` (a ``workloads.Pattern`` or None for the identity) is the
    initial pattern J; ``alpha`` is the maximum number of augmentation steps
    (0 for a fixed pattern), ``beta`` the maximum number of indices added per
    step and ``maxfill`` the cap on |J_k|.  ``spai_oracle.c`` states how it
    reads the points the printed algorithm leaves open (residual on the full
    column, candidates outside J, at most beta best acceptable indices with
    ties to the smaller index, augmentation only while step < alpha).  With
    u_f = FP16/BF16 a column whose computation gives a non-finite value is
    computed again from its initial pattern with u_f = FP32 (FLAG_FALLBACK):
    the overflow policy of the library (Section 4 scales A so that the low
    precision build does not overflow; an ill-conditioned reduced problem can
    still exceed the half range).
    """
    n = A.n
    if cols is None:
        cols = np.arange(n, dtype=np.int32)
    cols = _i32(cols)
    if len(cols) and (cols.min() < 0 or cols.max() >= n):
        raise ValueError("column out of range")
    maxinit = 1 if pattern is None else int(np.diff(pattern.ptr).max(initial=1))
    stride = max(int(maxfill), maxinit, 1)
    nc = len(cols)
    out_len = np.zeros(nc, np.int32)
    out_J = np.full((nc, stride), -1, np.int32)
    out_m = np.zeros((nc, stride), np.float64)
    out_steps = np.zeros(nc, np.int32)
    out_nI = np.zeros(nc, np.int32)
    out_flags = np.zeros(nc, np.int32)
    out_res = np.zeros(nc, np.float64)
    out_margin = np.zeros(nc, np.float64)
    out_d = np.zeros(n, np.float64)
    out_hist = np.zeros((nc, stride + 1), np.float64)
    out_flops = np.zeros(nc, np.float64)
    rp, ci, av = _i32(A.rowptr), _i32(A.col), _f64(A.val)
    pp = None if pattern is None else _i32(pattern.ptr)
    pi = None if pattern is None else _i32(pattern.idx)
    rc = _lib().oracle_spai(n, _p(rp), _p(ci), _p(av), _p(pp), _p(pi), float(eps), int(alpha),
                            int(beta), int(maxfill), UF[uf], _p(cols), nc, stride, int(nthreads),
                            _p(out_len), _p(out_J), _p(out_m), _p(out_steps), _p(out_nI),
                            _p(out_flags), _p(out_res), _p(out_margin), _p(out_d), _p(out_hist),
                            _p(out_flops))
    if rc != 0:
        raise ValueError("oracle_spai: bad argument")
    return SpaiResult(cols, out_len, out_J, out_m, out_steps, out_nI, out_flags, out_res,
                      out_margin, out_d, out_hist, out_flops)


@dataclasses.dataclass
class Probe:
    res: float            # ||e_k - B m_k|| for the given J
    I: np.ndarray         # shadow of J (ascending)
    mbar: np.ndarray      # m-bar on J (insertion order)
    cand: np.ndarray      # candidate indices (ascending)
    rho: np.ndarray       # their scores rho_j
    rbar: float           # mean score
    flags: int


def spai_probe(A, k: int, J, uf: str, cap: int = 4096, Iprev=None) -> Probe:
    """One solve + candidate scoring step of Algorithm 1 for column k and a given J.
    ``Iprev``: the shadow of the previous solve of the column, in its order (its rows
    keep their places, the new rows follow ascending); None for a first solve."""
    J = _i32(J)
    Ip = _i32(Iprev if Iprev is not None else np.zeros(0, np.int32))
    res = np.zeros(1)
    I = np.zeros(cap, np.int32)
    m = np.zeros(1, np.int32)
    mbar = np.zeros(max(len(J), 1))
    cj = np.zeros(cap, np.int32)
    crho = np.zeros(cap)
    nc = np.zeros(1, np.int32)
    rbar = np.zeros(1)
    flags = np.zeros(1, np.int32)
    rp, ci, av = _i32(A.rowptr), _i32(A.col), _f64(A.val)
    rc = _lib().oracle_spai_probe(A.n, _p(rp), _p(ci), _p(av), int(k), _p(J), len(J), _p(Ip), len(Ip), UF[uf], cap,
                                  _p(res), _p(I), _p(m), _p(mbar), _p(cj), _p(crho), _p(nc),
                                  _p(rbar), _p(flags))
    if rc != 0:
        raise ValueError("oracle_spai_probe: capacity too small")
    return Probe(float(res[0]), I[:m[0]].copy(), mbar[:len(J)].copy(), cj[:nc[0]].copy(),
                 crho[:nc[0]].copy(), float(rbar[0]), int(flags[0]))


def ls_column(A, d: np.ndarray, k: int, J) -> tuple:
    """Plain definition of a column for a given J (eq. redprob), in FP64.

    m-bar = argmin || e_k(I) - B(I, J) m ||_2 with B = A^T D and I the shadow
    of J.  Returns (m-bar, residual norm ||e_k - B m_k||_2)."""
    J = [int(j) for j in J]
    I = sorted({int(i) for j in J for i in A.col[A.rowptr[j]:A.rowptr[j + 1]]})
    pos = {i: t for t, i in enumerate(I)}
    Ab = np.zeros((len(I), len(J)))
    for c, j in enumerate(J):
        for t in range(A.rowptr[j], A.rowptr[j + 1]):
            Ab[pos[int(A.col[t])], c] = d[j] * A.val[t]
    e = np.zeros(len(I))
    if k in pos:
        e[pos[k]] = 1.0
    mbar, *_ = np.linalg.lstsq(Ab, e, rcond=None)
    r = Ab @ mbar - e
    res2 = float(r @ r) + (0.0 if k in pos else 1.0)
    return mbar, float(np.sqrt(res2))


# ---------------------------------------------------------------------------
# Algorithm 3
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class IrResult:
    x: np.ndarray
    its: list             # GMRES iterations per refinement step
    status: int           # IR_* bits
    gest: np.ndarray      # |g_{k+1}| / beta0 per step
    dnorm: np.ndarray     # ||d_i||_inf per step
    xhist: Optional[np.ndarray] = None   # u = fp32: x_0 .. x_s (the iterate each step starts from, then the last)
    gprev: Optional[np.ndarray] = None   # u = fp32: |g_k| / beta0, the estimate one iteration before the stop
    basis0: Optional[np.ndarray] = None  # basis=True: the first step's orthonormal Arnoldi vectors (n x its[0])

    @property
    def total(self) -> int:
        return int(sum(self.its))

    def tuple_str(self) -> str:
        return f"{self.total}({', '.join(str(i) for i in self.its)})"


ORTHO = {"mgs": 0, "cgs2": 1, "dcgs2": 2}


def gmres_ir(A, P_rowptr, P_col, P_val, d, uf: str, b, tau: float, imax: int, maxit: int,
             tol_ir: float, ortho: str = "mgs", u: str = "fp64", side: str = "left",
             x_init: Optional[np.ndarray] = None, basis: bool = False) -> IrResult:
    """SPAI-GMRES-IR (Algorithm 3) with P = M^T D given as CSR(M^T) + D.

    ``ortho`` = "mgs" (modified Gram-Schmidt, the variant analysed in Section
    3.2), "cgs2" (classical Gram-Schmidt applied twice) or "dcgs2" (CGS2 with
    the second projection and the normalisation delayed by one step: one set of
    inner products per Arnoldi step).

    ``u`` is the working precision u = u_g = u_p: "fp64" (residual rounded
    exactly to FP64, the precision set of Table 3) or "fp32" (the sets of Tables
    4 and 5: every stored quantity binary32, residual in binary64, MGS only).

    ``side`` = "left" (Algorithm 3: P = M^T D from ``spai``) or "right" (P = D M
    from ``spai_right``, GMRES on A P y = r_i with d_i = P y; working precision
    double only).

    ``x_init`` (u = "fp32" only): start the refinement from this iterate (used
    as rounded to binary32) instead of x0 = P b; the result then also holds the
    iterates each step started from (``xhist``) and the stopping margins.

    ``basis`` (u = "fp64"): also return the first refinement step's Arnoldi
    vectors v_0 .. v_{k-1} (an inspection output: the arithmetic is unchanged)."""
    n = A.n
    x = np.zeros(n)
    its = np.zeros(imax, np.int32)
    nsteps = np.zeros(1, np.int32)
    gest = np.zeros(imax)
    dn = np.zeros(imax)
    rp, ci, av = _i32(A.rowptr), _i32(A.col), _f64(A.val)
    pp, pc, pv = _i32(P_rowptr), _i32(P_col), _f64(P_val)
    dd, bb = _f64(d), _f64(b)
    if side not in ("left", "right") or (side == "right" and u != "fp64"):
        raise ValueError("side must be left or right (right with u = fp64)")
    xhist = gprev = None
    if x_init is not None and u != "fp32":
        raise ValueError("x_init is supported with u = fp32")
    if u == "fp32":
        if ortho != "mgs":
            raise ValueError("the single working precision variant uses MGS")
        xhist = np.zeros((imax + 1, n))
        gprev = np.zeros(imax)
        xi = None if x_init is None else _f64(x_init)
        st = _lib().oracle_gmres_ir_fp32(n, _p(rp), _p(ci), _p(av), _p(pp), _p(pc), _p(pv), _p(dd), UF[uf],
                                         _p(bb), _p(x), float(tau), int(imax), int(maxit), float(tol_ir),
                                         _p(its), _p(nsteps), _p(gest), _p(dn), _p(xi), _p(xhist), _p(gprev))
    elif u == "fp64":
        B0 = np.zeros((maxit, n)) if basis else None
        st = _lib().oracle_gmres_ir(n, _p(rp), _p(ci), _p(av), _p(pp), _p(pc), _p(pv), _p(dd), UF[uf],
                                    _p(bb), _p(x), float(tau), int(imax), int(maxit), float(tol_ir),
                                    ORTHO[ortho], int(side == "right"), _p(its), _p(nsteps), _p(gest), _p(dn),
                                    _p(B0))
    else:
        raise ValueError(f"unknown working precision {u}")
    if st < 0:
        raise ValueError("oracle_gmres_ir: bad argument")
    s = int(nsteps[0])
    return IrResult(x, [int(v) for v in its[:s]], st, gest[:s].copy(), dn[:s].copy(),
                    None if xhist is None else xhist[:s + 1].copy(), None if gprev is None else gprev[:s].copy(),
                    None if u != "fp64" or not basis or s == 0 else B0[:its[0]].T.copy())


def x0(P_rowptr, P_col, P_val, d, b, uf: str) -> np.ndarray:
    """x0 = P b computed in u_f, stored in FP64 (Algorithm 3, initial solve)."""
    n = len(b)
    out = np.zeros(n)
    pp, pc, pv = _i32(P_rowptr), _i32(P_col), _f64(P_val)
    _lib().oracle_x0(n, _p(pp), _p(pc), _p(pv), _p(_f64(d)), _p(_f64(b)), UF[uf], _p(out))
    return out


@dataclasses.dataclass
class _Transposed:
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray


def x0_right(P_rowptr, P_col, P_val, d, b, uf: str) -> np.ndarray:
    """x0 = P b in u_f for a right preconditioner P = D M (rows i hold m_k[i])."""
    n = len(b)
    out = np.zeros(n)
    pp, pc, pv = _i32(P_rowptr), _i32(P_col), _f64(P_val)
    _lib().oracle_x0_right(n, _p(pp), _p(pc), _p(pv), _p(_f64(d)), _p(_f64(b)), UF[uf], _p(out))
    return out


def spai_right(A, pattern, eps: float, alpha: int, beta: int, maxfill: int, uf: str, nthreads: int = 0):
    """Right preconditioner P = D M with A D M ~ I: Algorithm 1 on A itself with its
    columns scaled to unit maximum (D = diag(1 / max_i |a_ij|)), i.e. the left-form
    build of A^T, whose rows m_k become the columns of M.  Returns (R, rowptr, col,
    val, d): R the per-column results of the build on A^T, and the CSR of P by rows
    i (entries m_k[i], columns k ascending) with the scaling d applied to the
    output."""
    import scipy.sparse as _sp
    At = _sp.csr_matrix((np.asarray(A.val), np.asarray(A.col), np.asarray(A.rowptr)), shape=(A.n, A.n)).T.tocsr()
    At.sort_indices()

    T = _Transposed(A.n, At.indptr.astype(np.int32), At.indices.astype(np.int32), At.data.copy())
    R = spai(T, pattern, eps, alpha, beta, maxfill, uf, nthreads=max(1, nthreads))
    pp, pc, pv = R.P_csr(A.n)
    Pt = _sp.csr_matrix((pv, pc, pp), shape=(A.n, A.n)).T.tocsr()
    Pt.sort_indices()
    return R, Pt.indptr.astype(np.int32), Pt.indices.astype(np.int32), Pt.data.copy(), R.d.copy()


def apply_P(P_rowptr, P_col, P_val, d, w) -> np.ndarray:
    """y = M^T (D w) in FP64."""
    n = len(w)
    out = np.zeros(n)
    pp, pc, pv = _i32(P_rowptr), _i32(P_col), _f64(P_val)
    _lib().oracle_apply_P(n, _p(pp), _p(pc), _p(pv), _p(_f64(d)), _p(_f64(w)), _p(out))
    return out


def residual(A, b, x) -> np.ndarray:
    """r = b - A x, every component computed exactly and rounded once to FP64."""
    r = np.zeros(A.n)
    rp, ci, av = _i32(A.rowptr), _i32(A.col), _f64(A.val)
    _lib().oracle_residual(A.n, _p(rp), _p(ci), _p(av), _p(_f64(b)), _p(_f64(x)), _p(r))
    return r


def exact_sum(values) -> float:
    """Correctly rounded sum of a list of binary64 values."""
    v = _f64(values)
    scratch = np.zeros(max(len(v), 1))
    return _lib().oracle_exact_sum(_p(v), len(v), _p(scratch))


# ---------------------------------------------------------------------------
# error measures (Theorems 1 and 2)
# ---------------------------------------------------------------------------

def ferr(x, x_true) -> float:
    """Relative forward error ||x - x_true||_inf / ||x_true||_inf."""
    return float(np.abs(np.asarray(x) - x_true).max() / np.abs(x_true).max())


def nbe(A, b, x) -> float:
    """Normwise backward error ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)."""
    r = residual(A, b, x)
    anorm = np.add.reduceat(np.abs(A.val), A.rowptr[:-1]).max()
    return float(np.abs(r).max() / (anorm * np.abs(x).max() + np.abs(b).max()))
