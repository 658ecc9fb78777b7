"""Right-preconditioned SPAI-GMRES-IR on the GPU (the paper's future-work
variant): the right build (Algorithm 1 on A with unit-maximum columns, P = D M)
equals the oracle's bit for bit, x0 = P b in u_f is bit-exact, P applied on the
right gives the oracle's iteration tuples and forward errors at or below
1e-12."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def S():
    import paper_2202_10204_amd as S

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return S


@pytest.fixture(scope="module")
def h(S):
    return S.Handle()


def _cases():
    return {
        "convdiff_small": W.convdiff_small(16),
        "convdiff_adaptive_48": W.convdiff_adaptive(48),
        "random_3000": W.random_system(3000, 7),
    }


CASES = _cases()


@pytest.mark.parametrize("name,uf", [(k, u) for k in CASES for u in ("fp32", "fp64", "fp16")])
def test_right_build_and_x0_match_the_oracle(S, h, name, uf):
    w = CASES[name]
    s = w.spai
    A = S.DeviceCSR.from_host(w.A)
    pat = S.DevicePattern.from_host(w.pattern) if w.pattern is not None else None
    P, warn, st = h.spai_build(A, pat, s.eps, s.alpha, s.beta, s.maxfill, uf, "right")
    R, pp, pc, pv, d = O.spai_right(w.A, w.pattern, s.eps, s.alpha, s.beta, s.maxfill, uf)
    rp_t, col_t, val_t, d_t = P.csr()
    rp, col, val, dd = rp_t.cpu().numpy(), col_t.cpu().numpy(), val_t.double().cpu().numpy(), d_t.cpu().numpy()
    assert P.view().side == 1
    assert np.array_equal(rp, pp) and np.array_equal(col, pc)
    assert np.array_equal(val, pv)
    assert np.array_equal(dd, d)
    b = torch.as_tensor(w.b, device="cuda")
    x0 = torch.zeros_like(b)
    h.precond_apply_uf(P, b, x0)
    assert np.array_equal(x0.cpu().numpy(), O.x0_right(pp, pc, pv, d, w.b, uf))
    # P w = D (M w) in FP64
    wv = np.random.default_rng(3).standard_normal(w.n)
    y = torch.zeros_like(b)
    h.precond_apply(P, torch.as_tensor(wv, device="cuda"), y)
    ref = d * (sp.csr_matrix((pv, pc, pp), shape=(w.n, w.n)) @ wv)
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("ortho", ["mgs", "dcgs2"])
def test_right_gmres_ir_matches_the_oracle(S, h, name, ortho):
    w = CASES[name]
    s, ir = w.spai, w.ir
    A = S.DeviceCSR.from_host(w.A)
    pat = S.DevicePattern.from_host(w.pattern) if w.pattern is not None else None
    P, _, _ = h.spai_build(A, pat, s.eps, s.alpha, s.beta, s.maxfill, s.u_f, "right")
    R, pp, pc, pv, d = O.spai_right(w.A, w.pattern, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    b = torch.as_tensor(w.b, device="cuda")
    x = torch.zeros_like(b)
    r = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", ortho)
    ref = O.gmres_ir(w.A, pp, pc, pv, d, s.u_f, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir, ortho, side="right")
    xg = x.cpu().numpy()
    print(name, ortho, "gpu", r["its"], "oracle", ref.its, O.ferr(xg, w.x_true))
    assert r["its"] == list(ref.its)
    assert O.ferr(xg, w.x_true) <= 1e-12
    assert np.abs(xg - ref.x).max() <= 1e-12 * np.abs(ref.x).max()


def test_right_preconditioner_is_rejected_where_unsupported(S, h):
    w = CASES["convdiff_small"]
    s, ir = w.spai, w.ir
    A = S.DeviceCSR.from_host(w.A)
    P, _, _ = h.spai_build(A, None, s.eps, 5, s.beta, s.maxfill, "fp32", "right")
    b = torch.as_tensor(w.b, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(S.SpaiError):
        h.gmres_ir_batched(A, P, [0, w.n], b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir)
    with pytest.raises(S.SpaiError):
        h.gmres_ir(A, P, b, x, 1e-4, 10, 100, W.TOL_IR32, "fp64", "mgs", "fp32")
