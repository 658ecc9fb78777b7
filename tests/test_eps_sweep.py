"""Epsilon sweeps of the SPAI build on the paper-shaped stand-in matrices
(Section 3.1, Figures 1-2): the GPU build gives the oracle's nnz(P) and column
statistics at every epsilon in FP32 and FP64; nnz(P) falls as epsilon grows;
||I - PA||_inf stays within 2 n eps (eq. `AM1`) when every column met eps;
FP32 and FP64 builds give near-identical nnz(P) (the paper's observation that a
u_f finer than the one epsilon needs brings no advantage)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS = (0.6, 0.5, 0.4, 0.3, 0.2)


@pytest.fixture(scope="module")
def S():
    import paper_2202_10204_amd as S

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return S


@pytest.fixture(scope="module")
def h(S):
    return S.Handle()


@pytest.mark.parametrize("k", [5, 6, 2, 8])
def test_eps_sweep_matches_the_oracle(S, h, k):
    from paper_2202_10204_amd import diagnostics as D

    w = W.s0_matrix(k)
    n = w.n
    rows = D.eps_sweep(h, w.A, EPS, ("fp32", "fp64"))
    by = {(r["u_f"], r["eps"]): r for r in rows}
    for uf in ("fp32", "fp64"):
        nnz = [by[(uf, e)]["nnz_P"] for e in EPS]
        assert all(a <= b for a, b in zip(nnz, nnz[1:])), nnz      # sparser for larger eps
        for e in EPS:
            R = O.spai(w.A, None, e, -(-n // 8), 8, 63, uf)
            r = by[(uf, e)]
            assert r["nnz_P"] == int(R.P_csr(n)[0][-1])
            assert r["cols_over_eps"] == int(((R.flags & O.FLAG_EPS) != 0).sum())
            assert r["max_len"] == int(R.length.max())
            if r["cols_over_eps"] == 0:
                assert r["norm_I_minus_PA"] <= r["bound_I_minus_PA"]
            assert np.isfinite(r["kappa_inf_PA"]) and r["kappa_inf_PA"] >= 1.0
    for e in EPS:
        a, b = by[("fp32", e)]["nnz_P"], by[("fp64", e)]["nnz_P"]
        assert abs(a - b) <= 0.25 * b, (e, a, b)
