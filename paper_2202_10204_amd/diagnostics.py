"""Diagnostics of the SPAI build over a range of tolerances (Section 3.1).

For one matrix and a list of epsilons, builds P on the GPU in each requested
u_f and reports what Figures 1 and 2 of the paper plot: the number of stored
entries of P against epsilon (in single and in double precision), and the
infinity-norm condition number of the preconditioned matrix PA beside the
rough estimate (1 + 2 n eps)^2 of eq. `kappaAtest`.  It also reports
||I - PA||_inf, which the column residual test bounds by 2 n eps (eq. `AM1`)
when every column met eps.

The builds run in the library; the dense quantities (PA, its inverse) are
host-side analysis for small n only and are not part of the solver.
"""
from __future__ import annotations

import numpy as np


def dense_p(P) -> np.ndarray:
    """P = M^T D as a dense FP64 host matrix (entry (k, j) = m_k[j] d_j)."""
    rowptr, col, val, d = (t.cpu() for t in P.csr())
    rowptr = rowptr.numpy().astype(np.int64)
    col = col.numpy()
    val = val.double().numpy()
    d = d.numpy()
    n = len(rowptr) - 1
    out = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    out[rows, col] = val * d[col]
    return out


def eps_sweep(h, A_host, eps_values, u_f_values=("fp32", "fp64"), alpha=None, beta=8, maxfill=63,
              pattern=None, dense=True):
    """One build per (u_f, eps): list of dicts with nnz(P), the columns left above
    eps, the largest column residual and, when ``dense``, kappa_inf(PA),
    ||I - PA||_inf, the estimate (1 + 2 n eps)^2 and the bound 2 n eps."""
    import paper_2202_10204_amd as S

    n = int(A_host.n)
    A = S.DeviceCSR.from_host(A_host)
    pat = S.DevicePattern.from_host(pattern) if pattern is not None else None
    a = -(-n // beta) if alpha is None else alpha
    Ad = A_host.to_scipy().toarray() if dense else None
    rows = []
    for u_f in u_f_values:
        for eps in eps_values:
            P, warn, st = h.spai_build(A, pat, float(eps), a, beta, maxfill, u_f)
            r = {"u_f": u_f, "eps": float(eps), "nnz_P": int(st["nnz"]), "cols_over_eps": int(st["cols_over_eps"]),
                 "max_res": float(st["max_res"]), "max_len": int(st["max_len"]), "warnings": int(warn)}
            if dense:
                PA = dense_p(P) @ Ad
                try:
                    inv = np.linalg.inv(PA)
                    kap = float(np.abs(PA).sum(axis=1).max() * np.abs(inv).sum(axis=1).max())
                except np.linalg.LinAlgError:
                    kap = float("inf")
                r.update({"kappa_inf_PA": kap, "estimate_kappa": (1.0 + 2.0 * n * eps) ** 2,
                          "norm_I_minus_PA": float(np.abs(np.eye(n) - PA).sum(axis=1).max()),
                          "bound_I_minus_PA": 2.0 * n * eps})
            rows.append(r)
            del P
    return rows
