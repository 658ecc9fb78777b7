"""The C-ABI boundary on the GPU: device memory through the caller's allocator,
the statistics of a build (stored and numeric entries, recomputed columns) and
of a solve (backward and forward error of the returned x, Theorems 1-2), the
overflow policy of the 16-bit build, and the warm start of the refinement."""
import ctypes

import numpy as np
import pytest

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


def _dev(a):
    return torch.as_tensor(np.asarray(a), device="cuda")


def _solve_convdiff(S, w):
    s, ir = w.spai, w.ir
    h = S.Handle()
    A = S.DeviceCSR.from_host(w.A)
    P, _, st = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    b = _dev(w.b)
    x = torch.zeros_like(b)
    r = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", "dcgs2")
    _, _, val, _ = P.csr()
    out = (x.cpu().numpy(), val.cpu().numpy(), r["its"])
    del P
    h.close()
    return out


def test_allocations_go_through_the_callers_allocator(S):
    """With a counting allocator installed every device block of a build and a
    solve comes from it and goes back to it once the preconditioner and the
    handle are gone; the results equal those of hipMalloc'd memory bit for bit."""
    live, calls = {}, {"alloc": 0, "free": 0}

    def alloc(nbytes, device, stream, ctx):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))
        live[p] = int(nbytes)
        calls["alloc"] += 1
        return p

    def free(ptr, device, stream, ctx):
        live.pop(int(ptr))
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(int(ptr))

    fa, ff = S._ALLOC_FN(alloc), S._FREE_FN(free)
    w = W.convdiff_adaptive(64)
    S.use_torch_allocator(False)
    try:
        ref = _solve_convdiff(S, w)
        assert S.lib().spai_set_allocator(fa, ff, None) == 0
        got = _solve_convdiff(S, w)
    finally:
        S.use_torch_allocator(True)
    assert calls["alloc"] >= 5 and calls["free"] == calls["alloc"] and not live
    assert got[2] == ref[2]
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def test_build_and_solve_statistics(S, h):
    """nnz_numeric counts the stored values that are not zero (what the paper's
    tables count, Section 4); nbe and ferr of the solve equal the host's
    evaluation of Theorem 2's backward error and Theorem 1's forward error of
    the returned x (ferr bit for bit, nbe to the rounding of the residual)."""
    w = W.convdiff_adaptive(32)
    s, ir = w.spai, w.ir
    A = S.DeviceCSR.from_host(w.A)
    P, _, st = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    ref = O.spai(w.A, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    nz = sum(int(np.count_nonzero(ref.m[k, :ref.length[k]])) for k in range(w.n))
    assert st["nnz_numeric"] == nz and st["nnz"] == int(ref.length.sum()) and st["cols_fallback"] == 0
    assert P.view().u_f == S.FP32 and P.view().val_prec == S.FP32
    b, xt = _dev(w.b), _dev(w.x_true)
    x = torch.zeros_like(b)
    r = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", "dcgs2", x_true=xt)
    xg = x.cpu().numpy()
    assert r["ferr"] == O.ferr(xg, w.x_true) and r["ferr"] <= 1e-12
    assert r["nbe"] == pytest.approx(O.nbe(w.A, w.b, xg), rel=1e-12, abs=1e-300)
    r2 = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", "mgs")
    assert r2["ferr"] is None and r2["nbe"] <= 4 * 2.0 ** -53


def test_batched_solve_statistics(S, h):
    """Per-system nbe and ferr of the batched solver (FP64 and FP32 working
    precision) against the host's evaluation on each system's block."""
    B = W.random_batch(16, 200, 2000)
    A = S.DeviceCSR.from_host(B.A)
    s, ir = B.spai, B.ir
    P, _, _ = h.spai_build_batched(A, B.sys_ptr, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    b, xt = _dev(B.b), _dev(B.x_true)
    x = torch.zeros_like(b)
    rc, st = h.gmres_ir_batched(A, P, B.sys_ptr, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, x_true=xt)
    xg = x.cpu().numpy()
    for q in range(B.nsys):
        wq = B.system(q)
        r0, r1 = B.sys_ptr[q], B.sys_ptr[q + 1]
        assert st[q]["ferr"] == O.ferr(xg[r0:r1], wq.x_true) and st[q]["ferr"] <= 1e-12
        assert st[q]["nbe"] == pytest.approx(O.nbe(wq.A, wq.b, xg[r0:r1]), rel=1e-12, abs=1e-300)


def _overflow_system(n=24):
    A = np.eye(n) + np.diag(-2.0 * np.ones(n - 1), 1)
    Ai = np.linalg.inv(A)
    ptr, idx = [0], []
    for k in range(n):
        idx += list(np.nonzero(Ai[k])[0])
        ptr.append(len(idx))
    import scipy.sparse as sp

    Sm = sp.csr_matrix(A)
    Sm.sort_indices()
    csr = W.CSR(n, Sm.indptr.astype(np.int32), Sm.indices.astype(np.int32), Sm.data.copy())
    return A, csr, W.Pattern(n, np.array(ptr, np.int32), np.array(idx, np.int32))


def test_fp16_overflow_columns_are_recomputed_in_fp32(S, h):
    """Upper bidiagonal I - 2N: its SPAI on the pattern of A^-1 has entries up to
    ~2^23, beyond the FP16 range.  The overflowing columns are recomputed in
    FP32 and counted, P is stored in FP32 while x0 still rounds D b to FP16,
    and everything equals the oracle's policy bit for bit; the solves converge."""
    Ad, Acsr, pat = _overflow_system()
    n = Acsr.n
    A = S.DeviceCSR.from_host(Acsr)
    P, warn, st = h.spai_build(A, S.DevicePattern.from_host(pat), 0.5, 0, 8, 63, "fp16")
    ref = O.spai(Acsr, pat, 0.5, 0, 8, 63, "fp16")
    fb = (ref.flags & O.FLAG_FALLBACK) != 0
    assert fb.sum() >= 4 and st["cols_fallback"] == int(fb.sum()) and st["cols_nonfinite"] == 0
    assert warn & S.W_NONFINITE == 0
    v = P.view()
    assert v.val_prec == S.FP32 and v.u_f == S.FP16
    cols = P.columns()
    L = ref.length
    J, M = cols["J"].cpu().numpy(), cols["m"].cpu().numpy()
    for k in range(n):
        assert np.array_equal(J[k, :L[k]], ref.J[k, :L[k]]) and np.array_equal(M[k, :L[k]], ref.m[k, :L[k]]), k
    assert np.array_equal((cols["flags"].cpu().numpy() & 16) != 0, fb)
    pp, pc, pv = ref.P_csr(n)
    rng = np.random.default_rng(5)
    x_true = np.round(rng.uniform(-1, 1, n) * 2 ** 10) / 2 ** 10
    bh = Ad @ x_true
    b = _dev(bh)
    x0 = torch.zeros_like(b)
    h.precond_apply_uf(P, b, x0)
    assert np.array_equal(x0.cpu().numpy(), O.x0(pp, pc, pv, ref.d, bh, "fp16"))
    x = torch.zeros_like(b)
    r = h.gmres_ir(A, P, b, x, 1e-8, 10, n, W.TOL_IR, "dd", "mgs")
    oref = O.gmres_ir(Acsr, pp, pc, pv, ref.d, "fp16", bh, 1e-8, 10, n, W.TOL_IR)
    assert r["its"] == oref.its and O.ferr(x.cpu().numpy(), x_true) <= 1e-12
    x32 = torch.zeros_like(b)
    r32 = h.gmres_ir(A, P, b, x32, 1e-4, 10, n, W.TOL_IR32, "fp64", "mgs", "fp32")
    o32 = O.gmres_ir(Acsr, pp, pc, pv, ref.d, "fp16", bh, 1e-4, 10, n, W.TOL_IR32, "mgs", "fp32")
    assert np.array_equal(o32.xhist[0].astype(np.float32).astype(np.float64), o32.xhist[0])
    assert r32["status"] & S.W_MAXIT == 0 and O.ferr(x32.cpu().numpy(), x_true) <= 2.0 ** -20
    assert r32["its"][0] == o32.its[0]


def test_warm_start(S, h):
    """x_given: refinement from the exact solution takes no step and returns x
    unchanged; a solve split after its first step (the second call starting
    from the first one's x) repeats the whole solve's steps and its x bit for
    bit."""
    w = W.convdiff_adaptive(32)
    s, ir = w.spai, w.ir
    A = S.DeviceCSR.from_host(w.A)
    P, _, _ = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    b = _dev(w.b)
    x = _dev(w.x_true).clone()
    r = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", "dcgs2", x_given=True)
    assert r["steps"] == 0 and np.array_equal(x.cpu().numpy(), w.x_true)
    for ortho in ("mgs", "dcgs2"):
        xf = torch.zeros_like(b)
        full = h.gmres_ir(A, P, b, xf, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", ortho)
        xs = torch.zeros_like(b)
        one = h.gmres_ir(A, P, b, xs, ir.tau, 1, ir.maxit, ir.tol_ir, "dd", ortho)
        rest = h.gmres_ir(A, P, b, xs, ir.tau, ir.imax - 1, ir.maxit, ir.tol_ir, "dd", ortho, x_given=True)
        assert one["its"] + rest["its"] == full["its"], (ortho, one["its"], rest["its"], full["its"])
        assert np.array_equal(xs.cpu().numpy(), xf.cpu().numpy())
