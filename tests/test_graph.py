"""DCGS2 Arnoldi chunks replayed as HIP graphs: the kernels take the step index
from the device solver state, so one captured chunk serves every chunk of
every refinement step.  The graph replays must give the stream launches'
results bit for bit (solution, iteration tuple), over many replays with the
solver's own eager work (residuals, back-substitution, update, flag copies)
between them, on two calls in a row, and for both preconditioning sides."""
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


def _solve(S, h, w, side, graph):
    s, ir = w.spai, w.ir
    A = S.DeviceCSR.from_host(w.A)
    pat = S.DevicePattern.from_host(w.pattern) if w.pattern is not None else None
    P, _, _ = h.spai_build(A, pat, s.eps, s.alpha, s.beta, s.maxfill, s.u_f, side)
    b = torch.as_tensor(w.b, device="cuda")
    x = torch.zeros_like(b)
    r = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", "dcgs2", graph=graph)
    return x.cpu().numpy(), r


@pytest.mark.parametrize("name", ["convdiff_adaptive_48", "random_3000", "convdiff_small_16"])
@pytest.mark.parametrize("side", ["left", "right"])
def test_graph_replay_equals_stream_launches(S, h, name, side):
    w = {"convdiff_adaptive_48": lambda: W.convdiff_adaptive(48), "random_3000": lambda: W.random_system(3000, 7),
         "convdiff_small_16": lambda: W.convdiff_small(16)}[name]()
    x0, r0 = _solve(S, h, w, side, False)
    for rep in range(2):
        x1, r1 = _solve(S, h, w, side, True)
        print(name, side, rep, r0["its"], r1["its"], flush=True)
        assert r1["its"] == r0["its"] and r1["status"] == r0["status"]
        assert np.array_equal(x1, x0), float(np.abs(x1 - x0).max())
    assert O.ferr(x0, w.x_true) <= 1e-12


def test_graph_replay_at_full_size(S, h):
    """The benchmark system (262,144 unknowns, ~150 chunk replays): same bits as
    the stream launches and the oracle's tuple."""
    import json
    import os

    w = W.convdiff_adaptive(512)
    x0, r0 = _solve(S, h, w, "left", False)
    x1, r1 = _solve(S, h, w, "left", True)
    assert r1["its"] == r0["its"]
    assert np.array_equal(x1, x0)
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "convdiff512_oracle.json")))
    assert r1["its"] == golden["its"]
    assert O.ferr(x1, w.x_true) <= 1e-12


@pytest.mark.parametrize("blocks", [8, 2])
def test_graph_replay_with_more_rows_per_thread(S, h, blocks, monkeypatch):
    """The pipelined launch for more than 2 rows per thread (4 and 16 here: the
    128x128 system on 8 or 2 blocks) replayed from graphs, taking its step from
    the solver state: same bits as its stream launches."""
    monkeypatch.setenv("SPAI_ARNOLDI_BLOCKS", str(blocks))
    w = W.convdiff_adaptive(128)
    x0, r0 = _solve(S, h, w, "left", False)
    x1, r1 = _solve(S, h, w, "left", True)
    assert r1["its"] == r0["its"] and r1["status"] == r0["status"] == 0
    assert np.array_equal(x1, x0), float(np.abs(x1 - x0).max())
    assert O.ferr(x1, w.x_true) <= 1e-12


def test_graph_option_is_ignored_by_other_orthogonalisations(S, h):
    w = W.convdiff_adaptive(48)
    s, ir = w.spai, w.ir
    A = S.DeviceCSR.from_host(w.A)
    P, _, _ = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    b = torch.as_tensor(w.b, device="cuda")
    for ortho in ("mgs", "cgs2"):
        xs = []
        for graph in (False, True):
            x = torch.zeros_like(b)
            r = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", ortho, graph=graph)
            xs.append((x.cpu().numpy(), r["its"]))
        assert xs[0][1] == xs[1][1] and np.array_equal(xs[0][0], xs[1][0]), ortho
