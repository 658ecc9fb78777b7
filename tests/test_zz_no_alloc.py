"""spai_gmres_ir_noalloc: the allocation-free solve, called through the C ABI,
gives spai_gmres_ir's result bit for bit, on two calls in a row (the second
with a smaller system, so the shared device array holds the first call's
data), allocates nothing through the caller's allocator, and rejects a
problem whose workspace exceeds its fixed array."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def S():
    import paper_2202_10204_amd as S

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return S


def _params(S, ir, ortho):
    return S._IrParams(S.PREC["dd"], float(ir.tau), int(ir.imax), int(ir.maxit), float(ir.tol_ir),
                       S.ORTHO[ortho], S.FP64, 0, 0, None)


def _both(S, h, w, ortho):
    s, ir = w.spai, w.ir
    A = S.DeviceCSR.from_host(w.A)
    pat = S.DevicePattern.from_host(w.pattern) if w.pattern is not None else None
    P, _, _ = h.spai_build(A, pat, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    b = torch.as_tensor(w.b, device="cuda")
    xa = torch.zeros_like(b)
    ref = h.gmres_ir(A, P, b, xa, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", ortho)
    xn = torch.full_like(b, float("nan"))
    st = S._IrStats()
    csr = A.c()
    prm = _params(S, ir, ortho)
    rc = S.lib().spai_gmres_ir_noalloc(h._raw, ctypes.byref(csr), P.raw, ctypes.c_void_p(b.data_ptr()),
                                       ctypes.c_void_p(xn.data_ptr()), ctypes.byref(prm), ctypes.byref(st))
    assert rc >= 0, S.last_error()
    got = S._ir_dict(st, rc)
    return ref, got, xa.cpu().numpy(), xn.cpu().numpy()


@pytest.mark.parametrize("ortho", ["dcgs2", "mgs"])
def test_noalloc_equals_the_allocating_solve(S, ortho):
    calls = {"alloc": 0}

    def alloc(nbytes, device, stream, ctx):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))

    def free(ptr, device, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    fa, ff = S._ALLOC_FN(alloc), S._FREE_FN(free)
    h = S.Handle()
    try:
        for N in (32, 20):                    # second call smaller: the array keeps the first call's data
            w = W.convdiff_small(N)
            ref, got, xa, xn = _both(S, h, w, ortho)
            assert got["its"] == ref["its"] and got["status"] == ref["status"], (N, got["its"], ref["its"])
            assert np.array_equal(xn, xa), N
            assert got["nbe"] == ref["nbe"]
        # the solve itself takes no device memory: count allocations around one call
        w = W.convdiff_small(20)
        A = S.DeviceCSR.from_host(w.A)
        P, _, _ = h.spai_build(A, S.DevicePattern.from_host(w.pattern), w.spai.eps, w.spai.alpha, w.spai.beta,
                               w.spai.maxfill, w.spai.u_f)
        b = torch.as_tensor(w.b, device="cuda")
        x = torch.zeros_like(b)
        st = S._IrStats()
        csr = A.c()
        prm = _params(S, w.ir, ortho)
        assert S.lib().spai_set_allocator(fa, ff, None) == 0
        rc = S.lib().spai_gmres_ir_noalloc(h._raw, ctypes.byref(csr), P.raw, ctypes.c_void_p(b.data_ptr()),
                                           ctypes.c_void_p(x.data_ptr()), ctypes.byref(prm), ctypes.byref(st))
        assert rc >= 0 and calls["alloc"] == 0
    finally:
        S.use_torch_allocator(True)
        h.close()


def test_noalloc_rejects_a_workspace_beyond_its_array(S):
    """The 160x160 system with a 500-vector basis needs about 110 MB: rejected
    with SPAI_E_ARG and a message that gives the size; x is left untouched."""
    h = S.Handle()
    w = W.convdiff_adaptive(160)
    s, ir = w.spai, w.ir
    A = S.DeviceCSR.from_host(w.A)
    P, _, _ = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    b = torch.as_tensor(w.b, device="cuda")
    x = torch.full_like(b, 3.0)
    st = S._IrStats()
    csr = A.c()
    prm = _params(S, ir, "dcgs2")
    rc = S.lib().spai_gmres_ir_noalloc(h._raw, ctypes.byref(csr), P.raw, ctypes.c_void_p(b.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()), ctypes.byref(prm), ctypes.byref(st))
    assert rc == S.E_ARG and "allocation-free" in S.last_error() and "bytes" in S.last_error()
    assert torch.all(x == 3.0)
    prm32 = S._IrParams(S.PREC["fp64"], 1e-4, 10, 100, W.TOL_IR32, S.ORTHO["mgs"], S.FP32, 0, 0, None)
    w2 = W.convdiff_small(16)
    A2 = S.DeviceCSR.from_host(w2.A)
    P2, _, _ = h.spai_build(A2, None, 0.3, 4, 8, 20, "fp16")
    b2 = torch.as_tensor(w2.b, device="cuda")
    x2 = torch.zeros_like(b2)
    csr2 = A2.c()
    rc = S.lib().spai_gmres_ir_noalloc(h._raw, ctypes.byref(csr2), P2.raw, ctypes.c_void_p(b2.data_ptr()),
                                       ctypes.c_void_p(x2.data_ptr()), ctypes.byref(prm32), ctypes.byref(st))
    assert rc == S.E_ARG
    h.close()
