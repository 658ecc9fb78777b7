"""Write the oracle's results for the 128^3 anisotropic diffusion workload.

Calls only oracle/ (and the shared input generators): the full fixed-pattern
FP32 SPAI build on pattern(A^2) (digests of every column's values) and the
SPAI-GMRES-IR solve with modified Gram-Schmidt (the variant of the analysis in
Section 3.2) and with delayed CGS2, the two run side by side (iteration tuples,
forward and backward errors).  Output: aniso128_oracle.json next to this script.
The oracle's GMRES is single-threaded and each solve holds an n x 501 basis
(8.4 GB): about half an hour and 20 GB of memory.

    python tests/golden/make_aniso128_golden.py
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    w = W.aniso_fixed(128, "fp32")
    s, ir = w.spai, w.ir
    t0 = time.time()
    R = O.spai(w.A, w.pattern, s.eps, s.alpha, s.beta, s.maxfill, s.u_f, nthreads=os.cpu_count() or 1)
    t1 = time.time()
    print(f"build {t1 - t0:.1f} s", flush=True)
    pp, pc, pv = R.P_csr(w.n)

    def solve(ortho):
        ts = time.time()
        res = O.gmres_ir(w.A, pp, pc, pv, R.d, s.u_f, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir, ortho)
        print(f"{ortho}: {res.tuple_str()} in {time.time() - ts:.0f} s", flush=True)
        return res, time.time() - ts

    with ThreadPoolExecutor(max_workers=2) as ex:          # ctypes calls release the GIL
        (rm, tm), (rd, td) = ex.map(solve, ["mgs", "dcgs2"])
    out = {
        "workload": w.name,
        "recipe": w.recipe,
        "spai": {"eps": s.eps, "alpha": s.alpha, "beta": s.beta, "maxfill": s.maxfill, "u_f": s.u_f},
        "ir": {"tau": ir.tau, "imax": ir.imax, "maxit": ir.maxit, "tol_ir": ir.tol_ir},
        "n": w.n,
        "nnz_A": w.A.nnz,
        "nnz_P": int(pp[-1]),
        "sha256_m_insertion_order": digest(R.m.astype(np.float64)),
        "cols_over_eps": int(((R.flags & O.FLAG_EPS) != 0).sum()),
        "max_res": float(R.res.max()),
        "its": rm.its,
        "total_its": rm.total,
        "status": rm.status,
        "ferr": O.ferr(rm.x, w.x_true),
        "nbe": O.nbe(w.A, w.b, rm.x),
        "its_dcgs2": rd.its,
        "status_dcgs2": rd.status,
        "ferr_dcgs2": O.ferr(rd.x, w.x_true),
        "nbe_dcgs2": O.nbe(w.A, w.b, rd.x),
        "oracle_seconds": {"spai": t1 - t0, "gmres_ir": tm, "gmres_ir_dcgs2": td},
    }
    path = os.path.join(HERE, "aniso128_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
