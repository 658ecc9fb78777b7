"""Write the oracle's results for the 512x512 convection-diffusion workload.

Calls only oracle/ (and the shared input generators): the full adaptive FP32
SPAI build (digests of every column's insertion-ordered indices and values)
and the SPAI-GMRES-IR solve with each Arnoldi orthogonalisation (MGS, CGS2,
delayed CGS2: iteration tuples, errors).  Output:
convdiff512_oracle.json next to this script.  Takes a few minutes (the oracle's
GMRES is single-threaded).

    python tests/golden/make_convdiff512_golden.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    w = W.convdiff_adaptive(512)
    s, ir = w.spai, w.ir
    t0 = time.time()
    R = O.spai(w.A, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f, nthreads=os.cpu_count() or 1)
    t1 = time.time()
    pp, pc, pv = R.P_csr(w.n)
    res = O.gmres_ir(w.A, pp, pc, pv, R.d, s.u_f, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir)
    t2 = time.time()
    res2 = O.gmres_ir(w.A, pp, pc, pv, R.d, s.u_f, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "cgs2")
    t3 = time.time()
    res3 = O.gmres_ir(w.A, pp, pc, pv, R.d, s.u_f, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dcgs2")
    t4 = time.time()
    out = {
        "workload": w.name,
        "recipe": w.recipe,
        "spai": {"eps": s.eps, "alpha": s.alpha, "beta": s.beta, "maxfill": s.maxfill, "u_f": s.u_f},
        "ir": {"tau": ir.tau, "imax": ir.imax, "maxit": ir.maxit, "tol_ir": ir.tol_ir},
        "n": w.n,
        "nnz_A": w.A.nnz,
        "nnz_P": int(pp[-1]),
        "stride": int(R.J.shape[1]),
        "sha256_J_insertion_order": digest(R.J.astype(np.int32)),
        "sha256_m_insertion_order": digest(R.m.astype(np.float64)),
        "sha256_steps": digest(R.steps.astype(np.int32)),
        "max_steps": int(R.steps.max()),
        "max_len": int(R.length.max()),
        "cols_over_eps": int(((R.flags & O.FLAG_EPS) != 0).sum()),
        "its": res.its,
        "total_its": res.total,
        "status": res.status,
        "ferr": O.ferr(res.x, w.x_true),
        "nbe": O.nbe(w.A, w.b, res.x),
        "its_cgs2": res2.its,
        "ferr_cgs2": O.ferr(res2.x, w.x_true),
        "its_dcgs2": res3.its,
        "ferr_dcgs2": O.ferr(res3.x, w.x_true),
        "oracle_seconds": {"spai": t1 - t0, "gmres_ir": t2 - t1, "gmres_ir_cgs2": t3 - t2,
                           "gmres_ir_dcgs2": t4 - t3},
    }
    path = os.path.join(HERE, "convdiff512_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
