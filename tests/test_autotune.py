"""The column-kernel autotuner: configuration table, bins, cache (host), and on
the GPU that every configuration the tuner may pick gives the same bits."""
import ctypes
import json

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def S():
    import paper_2202_10204_amd as S

    return S


def test_configuration_table_on_the_host(S):
    cfgs = [S.column_config(c) for c in range(1, S.KCFG_COUNT + 1)]
    assert [c["maxp"] for c in cfgs] == [7, 15, 20, 20, 31, 63, 20, 20, 31]
    for c in cfgs:
        assert c["maxp"] == c["lanes"] - 1
        assert c["problems_per_wave"] == 64 // c["lanes"]
        assert c["maxm"] >= c["maxp"] and c["lds_bytes_per_problem"] > 0
    # the two 20-index shapes differ in shadow rows only; the register shapes
    # mirror them and take less LDS (A-bar leaves it)
    assert cfgs[2]["maxm"] < cfgs[3]["maxm"]
    for r, l in ((6, 2), (7, 3), (8, 4)):
        assert cfgs[r]["maxm"] == cfgs[l]["maxm"] and cfgs[r]["lanes"] == cfgs[l]["lanes"]
        assert cfgs[r]["lds_bytes_per_problem"] < cfgs[l]["lds_bytes_per_problem"]
    for bad in (0, S.KCFG_COUNT + 1, -1):
        with pytest.raises(S.SpaiError):
            S.column_config(bad)


def test_bad_kernel_cfg_and_tuning_arguments_are_rejected_before_device_work(S):
    L = S.lib()
    fake_handle = ctypes.c_void_p(1)
    A = S._Csr(4, 4, 8, 8, 8)
    out = ctypes.c_void_p()
    for kc in (-1, S.KCFG_COUNT + 1):
        prm = S._BuildParams(0.3, 1, 8, 20, S.FP32, 0, 0, kc)
        assert L.spai_build(fake_handle, ctypes.byref(A), None, ctypes.byref(prm), ctypes.byref(out), None) == S.E_ARG
        assert "kernel_cfg" in S.last_error()
    prm = S._BuildParams(0.3, 1, 8, 20, S.FP32, 0, 0, 0)
    ns = (ctypes.c_double * (2 * S.KCFG_COUNT))()
    assert L.spai_tune_build(fake_handle, ctypes.byref(A), None, ctypes.byref(prm), 0, 3, ns) == S.E_ARG
    assert L.spai_tune_build(fake_handle, ctypes.byref(A), None, ctypes.byref(prm), 64, 0, ns) == S.E_ARG
    assert L.spai_tune_build(fake_handle, ctypes.byref(A), None, ctypes.byref(prm), 64, 3, None) == S.E_ARG


def test_bins_and_choice(S):
    from paper_2202_10204_amd import autotune as T

    small, big = W.convdiff_adaptive(48), W.convdiff_adaptive(96)
    fixed = W.convdiff_small(16)
    k1 = T.bin_key(small.A, None, 288, 8, 20, "fp32")
    assert k1 == "left/fp32/adaptive-b8/p20/q8/n4096"
    assert T.bin_key(big.A, None, 288, 8, 20, "fp32") != k1                    # n bucket
    assert T.bin_key(small.A, None, 288, 8, 20, "fp16") != k1
    assert T.bin_key(small.A, None, 288, 8, 20, "fp32", "right") != k1
    assert T.bin_key(fixed.A, fixed.pattern, 0, 8, 5, "fp32").startswith("left/fp32/fixed/p5/")
    # the initial pattern's longest column counts when it exceeds the fill cap
    assert "/p5/" in T.bin_key(fixed.A, fixed.pattern, 0, 8, 1, "fp32")
    assert T.pick({(4, 0): 2.0, (3, 0): 1.5, (3, 1): 1.7}) == (3, 0)
    assert T.pick({(4, 0): 1.5, (3, 1): 1.5, (3, 0): 1.5}) == (3, 0)       # ties: smaller cfg, recompute
    with pytest.raises(ValueError):
        T.pick({})


def test_cache_round_trip_without_a_device(S, tmp_path, monkeypatch):
    from paper_2202_10204_amd import autotune as T

    w = W.convdiff_adaptive(48)
    calls = []

    class FakeHandle:
        def tune_build(self, *a):
            calls.append(a)
            return {(3, 0): 900.0, (3, 1): 950.0, (4, 0): 880.0, (4, 1): 990.0, (5, 0): 1400.0}

    monkeypatch.setattr(T, "gpu_arch", lambda: "gfx950")
    cache = str(tmp_path / "tune.json")
    s = w.spai
    c1 = T.tune(FakeHandle(), None, None, w.A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp32", cache=cache)
    assert (c1["kernel_cfg"], c1["qr_update"], c1["cached"]) == (4, 0, False)
    c2 = T.tune(FakeHandle(), None, None, w.A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp32", cache=cache)
    assert c2["cached"] and c2["kernel_cfg"] == 4 and len(calls) == 1
    data = json.load(open(cache))
    assert list(data) == ["gfx950"] and c1["bin"] in data["gfx950"]
    assert data["gfx950"][c1["bin"]]["candidates"]["5/0"] == 1400.0
    T.tune(FakeHandle(), None, None, w.A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp32", cache=cache, retune=True)
    assert len(calls) == 2


# ---------------------------------------------------------------------------- GPU


torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def h(S):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return S.Handle()


def _csr(P):
    rp, col, val, d = P.csr()
    return rp.cpu().numpy(), col.cpu().numpy(), val.double().cpu().numpy(), d.cpu().numpy()


CASES = {
    "convdiff_adaptive_48": (W.convdiff_adaptive(48), "fp32"),
    "random_3000_fp16": (W.random_system(3000, 7), "fp16"),
    "convdiff_fixed_16": (W.convdiff_small(16), "fp32"),
    "aniso_fixed_12_fp16": (W.aniso_fixed(12, "fp16"), "fp16"),     # pattern(A^2): the 32-lane shapes
    "aniso_fixed_12_bf16": (W.aniso_fixed(12, "bf16"), "bf16"),
}


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(CASES))
def test_every_eligible_configuration_gives_the_same_bits(S, h, name):
    w, uf = CASES[name]
    s = w.spai
    A = S.DeviceCSR.from_host(w.A)
    pat = S.DevicePattern.from_host(w.pattern) if w.pattern is not None else None
    P0, warn0, st0 = h.spai_build(A, pat, s.eps, s.alpha, s.beta, s.maxfill, uf)
    ref = _csr(P0)
    times = h.tune_build(A, pat, s.eps, s.alpha, s.beta, s.maxfill, uf, sample=1024, reps=1)
    pmax = max(int(s.maxfill), int((w.pattern.ptr[1:] - w.pattern.ptr[:-1]).max()) if w.pattern is not None else 1)
    eligible = [c for c in range(1, S.KCFG_COUNT + 1) if S.column_config(c)["maxp"] >= pmax]
    assert sorted(times) == sorted((c, u) for c in eligible for u in (0, 1))
    assert all(t > 0 for t in times.values())
    for c in eligible:
        for u in (0, 1):
            P, warn, st = h.spai_build(A, pat, s.eps, s.alpha, s.beta, s.maxfill, uf, qr_update=bool(u),
                                       kernel_cfg=c)
            got = _csr(P)
            assert warn == warn0 and st["nnz"] == st0["nnz"], (c, u)
            for x, y in zip(got, ref):
                assert np.array_equal(x, y), (name, c, u)
    small = [c for c in range(1, S.KCFG_COUNT + 1) if S.column_config(c)["maxp"] < pmax]
    for c in small:
        with pytest.raises(S.SpaiError):
            h.spai_build(A, pat, s.eps, s.alpha, s.beta, s.maxfill, uf, kernel_cfg=c)


@pytest.mark.gpu
def test_tuned_build_uses_and_caches_the_choice(S, h, tmp_path):
    from paper_2202_10204_amd import autotune as T

    w = W.convdiff_adaptive(48)
    s = w.spai
    A = S.DeviceCSR.from_host(w.A)
    cache = str(tmp_path / "tune.json")
    P, warn, st, c = T.build(h, A, None, w.A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp32", cache=cache,
                             sample=2048, reps=2)
    assert not c["cached"] and c["arch"].startswith("gfx")
    assert S.column_config(c["kernel_cfg"])["maxp"] >= s.maxfill
    P0, _, _ = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp32")
    for x, y in zip(_csr(P), _csr(P0)):
        assert np.array_equal(x, y)
    P2, _, _, c2 = T.build(h, A, None, w.A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp32", cache=cache)
    assert c2["cached"] and c2["kernel_cfg"] == c["kernel_cfg"]
