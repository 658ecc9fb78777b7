"""The precision sets of Tables 4 and 5 on the GPU: (u_f, u, u_r) = (half, single,
double) and (single, single, double), on the paper-shaped stand-ins of the
matrices those tables use, with the paper's protocol (identity start, beta 8,
alpha = ceil(n / beta), tau = 1e-4 for working precision single).

The build is bit-exact against the oracle (nnz(P) compared); the solve in
working precision single is compared with the oracle's binary32 GMRES-IR step
by step (each refinement step started on the GPU from the oracle's iterate,
its GMRES count compared exactly outside near ties of the stopping test), and
the single-system entry point equals the batched one bit for bit (the former
runs as a batch of one)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [(k, uf, e) for k in (5, 6, 8, 4) for uf in ("fp16", "fp32") for e in W.S0_SHAPES[k][5]]


@pytest.fixture(scope="module")
def S():
    import paper_2202_10204_amd as S

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return S


@pytest.fixture(scope="module")
def h(S):
    return S.Handle()


@pytest.fixture(scope="module")
def mats():
    return {k: W.s0_matrix(k) for k in (4, 5, 6, 8)}


# Near ties of the GMRES stopping test in binary32.  Started from the same
# iterate x_i, both sides form bit-identical r_i (binary64 evaluation of binary32
# data, terms in CSR order) and P r_i (row sums in column order); inside GMRES
# only the order of the binary32 inner-product sums differs (a workgroup tree on
# the GPU, sequential in the oracle).  The Givens estimates |g_{j+1}| / beta0 of
# the two sides then differ by a few hundred binary32 roundings at most over the
# <= 2205 iterations these systems allow, so a count can differ only where the
# oracle's estimate at the stopping iteration (gest) or at the one before it
# (gprev) lies within DELTA32 = 2^-10 (~ 16k u) of tau, relative.
DELTA32 = 2.0 ** -10


@pytest.mark.parametrize("k,uf,eps", CASES)
def test_single_working_precision_step_by_step(S, h, mats, k, uf, eps):
    """Refinement step i of the GPU's binary32 GMRES-IR, started from the oracle's
    iterate x_i (warm start), takes the oracle's GMRES count for that step
    exactly, unless the oracle's stopping test was a near tie (then within
    one); x0 = P b in u_f equals the oracle's; the GPU's whole solve converges."""
    w = mats[k]
    n, ir = w.n, w.ir
    A = S.DeviceCSR.from_host(w.A)
    P, warn, st = h.spai_build(A, None, eps, -(-n // 8), 8, 63, uf)
    R = O.spai(w.A, None, eps, -(-n // 8), 8, 63, uf)
    pp, pc, pv = R.P_csr(n)
    assert st["nnz"] == int(pp[-1])
    b = torch.as_tensor(w.b, device="cuda")
    ref = O.gmres_ir(w.A, pp, pc, pv, R.d, uf, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "mgs", "fp32")
    x0 = torch.zeros_like(b)
    h.precond_apply_uf(P, b, x0)
    assert np.array_equal(x0.cpu().numpy().astype(np.float32).astype(np.float64), ref.xhist[0])
    near, counts = 0, []
    for i, ki in enumerate(ref.its):
        xi = torch.as_tensor(ref.xhist[i], device="cuda").clone()
        r = h.gmres_ir(A, P, b, xi, ir.tau, 1, ir.maxit, ir.tol_ir, "fp64", "mgs", "fp32", x_given=True)
        margin = min(abs(ref.gest[i] - ir.tau), abs(ref.gprev[i] - ir.tau)) / ir.tau
        counts.append((r["its"][0], ki, float(margin)))
        if margin >= DELTA32:
            assert r["its"] == [ki], (i, r["its"], ki, margin)
        else:
            near += 1
            assert r["steps"] == 1 and abs(r["its"][0] - ki) <= 1, (i, r["its"], ki, margin)
    print(w.name, uf, eps, "(gpu, oracle, margin) per step:", counts, "near ties:", near)
    assert near <= 1
    x = torch.zeros_like(b)
    full = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "fp64", "mgs", "fp32")
    xg = x.cpu().numpy()
    assert np.array_equal(xg.astype(np.float32).astype(np.float64), xg)     # x in binary32
    assert full["status"] & S.W_MAXIT == 0 and ref.status & O.IR_MAXIT == 0
    assert O.ferr(xg, w.x_true) <= 2.0 ** -20
    assert O.ferr(ref.x, w.x_true) <= 2.0 ** -20


def test_single_working_precision_batched_equals_single(S, h, mats):
    """All four systems as one batch give each system's single-call result bit for bit."""
    ws = [mats[k] for k in (5, 6, 8, 4)]
    ptr = np.cumsum([0] + [w.n for w in ws])
    rows, cols, vals = [], [], []
    nnz = 0
    for w, o in zip(ws, ptr):
        rows.append(w.A.rowptr[:-1].astype(np.int64) + nnz)
        cols.append(w.A.col + o)
        vals.append(w.A.val)
        nnz += w.A.nnz
    Ab = W.CSR(int(ptr[-1]), np.concatenate(rows + [np.array([nnz])]).astype(np.int32),
               np.concatenate(cols).astype(np.int32), np.concatenate(vals))
    bb = np.concatenate([w.b for w in ws])
    A = S.DeviceCSR.from_host(Ab)
    P, _, _ = h.spai_build_batched(A, ptr, None, 0.3, 4096, 8, 63, "fp16")
    b = torch.as_tensor(bb, device="cuda")
    x = torch.zeros_like(b)
    ir = ws[0].ir
    rc, st = h.gmres_ir_batched(A, P, ptr, b, x, ir.tau, ir.imax, 2205, ir.tol_ir, "fp64", "fp32")
    xb = x.cpu().numpy()
    for q, w in enumerate(ws):
        Aq = S.DeviceCSR.from_host(w.A)
        Pq, _, _ = h.spai_build(Aq, None, 0.3, 4096, 8, 63, "fp16")
        bq = torch.as_tensor(w.b, device="cuda")
        xq = torch.zeros_like(bq)
        r = h.gmres_ir(Aq, Pq, bq, xq, ir.tau, ir.imax, 2205, ir.tol_ir, "fp64", "mgs", "fp32")
        assert r["its"] == st[q]["its"]
        assert np.array_equal(xq.cpu().numpy(), xb[ptr[q]:ptr[q + 1]])


def test_single_working_precision_rejects_unsupported_sets(S, h, mats):
    w = mats[5]
    A = S.DeviceCSR.from_host(w.A)
    b = torch.as_tensor(w.b, device="cuda")
    x = torch.zeros_like(b)
    P16, _, _ = h.spai_build(A, None, 0.3, 5, 8, 63, "fp16")
    P64, _, _ = h.spai_build(A, None, 0.3, 5, 8, 63, "fp64")
    with pytest.raises(S.SpaiError):
        h.gmres_ir(A, P16, b, x, 1e-4, 10, 37, W.TOL_IR32, "dd", "mgs", "fp32")      # u_r must be double
    with pytest.raises(S.SpaiError):
        h.gmres_ir(A, P64, b, x, 1e-4, 10, 37, W.TOL_IR32, "fp64", "mgs", "fp32")    # u_f finer than u
    with pytest.raises(S.SpaiError):
        h.gmres_ir(A, P16, b, x, 1e-4, 10, 37, W.TOL_IR32, "fp64", "dcgs2", "fp32")  # MGS only
