"""Synthetic input generators: sizes, structure, determinism, exact right-hand sides."""
import numpy as np
import pytest

import workloads as W


def test_convdiff_small_shape():
    w = W.convdiff_small()
    assert w.n == 1024 and w.A.nnz == 4992
    assert w.pattern.nnz == 4992 and w.spai.alpha == 0


def test_convdiff_full_shape():
    w = W.convdiff_adaptive(512)
    assert w.n == 262144 and w.A.nnz == 1_308_672
    assert w.spai.eps == 0.3 and w.spai.maxfill == 20 and w.spai.beta == 8


def test_aniso_small_pattern_is_A_squared():
    w = W.aniso_fixed(10)
    A = w.A
    assert A.nnz == 7 * 1000 - 6 * 100
    assert np.diff(w.pattern.ptr).max() == 25
    S = A.to_scipy()
    S2 = (abs(S) @ abs(S)).tocsr()
    assert w.pattern.nnz == S2.nnz


def test_generators_are_deterministic():
    a, b = W.convdiff_adaptive(32), W.convdiff_adaptive(32)
    assert np.array_equal(a.A.val, b.A.val) and np.array_equal(a.b, b.b)
    c, d = W.random_system(400, 3), W.random_system(400, 3)
    assert np.array_equal(c.A.col, d.A.col) and np.array_equal(c.x_true, d.x_true)


@pytest.mark.parametrize("make", [W.convdiff_small, lambda: W.convdiff_adaptive(40),
                                  lambda: W.aniso_fixed(9), lambda: W.random_system(700, 1)])
def test_structure(make):
    w = make()
    A = w.A
    rows = np.repeat(np.arange(A.n), A.row_nnz())
    assert np.all(np.diff(A.col)[np.diff(rows) == 0] > 0)        # sorted, unique columns
    assert np.all(A.val != 0.0)                                   # no stored zeros
    diag = A.to_scipy().diagonal()
    assert np.all(diag != 0.0)                                    # nonzero diagonal (Section 4)
    assert np.all(np.abs(w.x_true) <= 1.0)


def test_random_banded_band_and_dominance():
    w = W.random_system(2000, 7)
    A = w.A
    rows = np.repeat(np.arange(A.n), A.row_nnz())
    assert np.all(np.abs(A.col - rows) <= 32)
    nnz = A.row_nnz()
    assert nnz.min() >= 4 and nnz.max() <= 12
    S = A.to_scipy()
    d = np.abs(S.diagonal())
    off = np.asarray(abs(S).sum(1)).ravel() - d
    assert np.all(d >= 1.1 * off * (1 - 1e-6))


def test_s0_shapes_follow_the_table():
    """The paper-shaped stand-ins have the n and nnz of Table tab:mats, a nonzero
    diagonal, kappa_inf within 10x of the listed one, and an exact right-hand
    side; the matrices of the single-working-precision tables are exact in FP32
    (A, x_true and b)."""
    for k, (name, n, nnz, kappa, pset, eps) in enumerate(W.S0_SHAPES):
        if n > 1200:
            continue   # the 2205 case takes several seconds of dense algebra
        w = W.s0_matrix(k)
        assert w.n == n and w.A.nnz == nnz, name
        S = w.A.to_scipy()
        assert np.all(S.diagonal() != 0.0)
        assert 0.1 <= W.kappa_inf(w.A) / kappa <= 10.0, name
        r = np.asarray(S @ w.x_true) - w.b
        assert np.abs(r).max() == 0.0
        if pset == "hsd":
            for v in (w.A.val, w.x_true, w.b):
                assert np.array_equal(v.astype(np.float32).astype(np.float64), v), name


def test_serving_trace_mix():
    tr = W.serving_trace(200.0, 2.0)
    assert 300 <= len(tr) <= 500
    assert all(a.t < b.t for a, b in zip(tr, tr[1:]))
    kinds = {a.kind for a in tr}
    assert kinds == {"convdiff", "aniso", "random"}
    for a in tr:
        lo, hi = {"convdiff": (32, 512), "aniso": (10, 128), "random": (1000, 20000)}[a.kind]
        assert lo <= a.size <= hi
        assert a.u_f in ("fp16", "fp32")
    assert tr == W.serving_trace(200.0, 2.0)
    w = W.serving_request(tr[0])
    assert w.spai.u_f == tr[0].u_f
    r = np.asarray(w.A.to_scipy() @ w.x_true) - w.b
    assert np.abs(r).max() == 0.0
