"""The library's request loop (spai_serve_*): continuous batching of independent
solves, admission by device footprint, and results that do not depend on what
else is in flight.

Every request is solved alone (submitted, then waited for, one at a time) and
again in a mix (all submitted at once, so several batches and the device lane
run together): the solutions must be bit-identical, the GMRES tuples equal,
and equal to the oracle's for requests checked against it.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BATCH_MAX_N = 3000

# families and sizes of the stream at small sizes: three batch keys (adaptive
# FP32, adaptive FP16, fixed pattern FP32/FP16) and two systems above
# BATCH_MAX_N for the device lane
ARRIVALS = [
    W.Arrival(0.0, "random", 1200, "fp32", 0),
    W.Arrival(0.0, "random", 1500, "fp16", 1),
    W.Arrival(0.0, "random", 2600, "fp32", 2),
    W.Arrival(0.0, "convdiff", 32, "fp32", 3),
    W.Arrival(0.0, "convdiff", 36, "fp16", 4),
    W.Arrival(0.0, "aniso", 10, "fp32", 5),
    W.Arrival(0.0, "aniso", 11, "fp16", 6),
    W.Arrival(0.0, "convdiff", 56, "fp32", 7),
    W.Arrival(0.0, "aniso", 15, "fp32", 8),
    W.Arrival(0.0, "random", 1800, "fp32", 9),
]


@pytest.fixture(scope="module")
def S():
    import paper_2202_10204_amd as S

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return S


@pytest.fixture(scope="module")
def systems():
    return [W.serving_request(a) for a in ARRIVALS]


def _args(w, ortho="mgs"):
    s, ir = w.spai, w.ir
    build = {"eps": s.eps, "alpha": s.alpha, "beta": s.beta, "maxfill": s.maxfill, "u_f": s.u_f}
    irp = {"tau": ir.tau, "imax": ir.imax, "maxit": ir.maxit, "tol_ir": ir.tol_ir, "u_r": "dd", "ortho": ortho}
    return w.A, w.b, w.pattern, build, irp


def _ortho(k):
    return "dcgs2" if k == 8 else "mgs"


@pytest.fixture(scope="module")
def alone(S, systems):
    srv = S.Server(batch_lanes=3, batch_max_n=BATCH_MAX_N, hbm_budget=8 << 30, lane_workspace=512 << 20)
    out = []
    for k, w in enumerate(systems):
        rid = srv.submit(*_args(w, _ortho(k)))
        out.append(srv.wait(rid))
    srv.close()
    return out


def test_alone_results_are_valid(systems, alone):
    for k, (w, (rc, x, rec)) in enumerate(zip(systems, alone)):
        print(k, w.name, w.n, rec["lane"], rec["its"], rc, flush=True)
        assert rc >= 0, rec["error"]
        assert rec["batch_size"] == 1
        assert (rec["lane"] == -1) == (w.n > BATCH_MAX_N)
        if w.spai.u_f == "fp32":
            assert O.ferr(x, w.x_true) <= 1e-12, (k, w.name)


def test_mix_equals_alone_bitwise(S, systems, alone):
    srv = S.Server(batch_lanes=3, batch_max_n=BATCH_MAX_N, hbm_budget=8 << 30, lane_workspace=512 << 20)
    ids = [srv.submit(*_args(w, _ortho(k))) for k, w in enumerate(systems)]
    mix = [srv.wait(i) for i in ids]
    srv.close()
    batched = 0
    for k, ((rc_a, x_a, rec_a), (rc_m, x_m, rec_m)) in enumerate(zip(alone, mix)):
        assert rc_m == rc_a, (k, rec_m["error"])
        assert rec_m["its"] == rec_a["its"], k
        assert np.array_equal(x_m, x_a), (k, float(np.abs(x_m - x_a).max()))
        assert rec_m["t_submit"] <= rec_m["t_admit"] <= rec_m["t_done"]
        batched = max(batched, rec_m["batch_size"])
    # the three FP32 adaptive systems of the batch lanes share parameters: at least two ran together
    assert batched >= 2


@pytest.mark.parametrize("k", [0, 5, 7, 8])
def test_served_tuples_equal_the_oracle(systems, alone, k):
    w = systems[k]
    s, ir = w.spai, w.ir
    R = O.spai(w.A, w.pattern, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    pp, pc, pv = R.P_csr(w.n)
    res = O.gmres_ir(w.A, pp, pc, pv, R.d, s.u_f, w.b, ir.tau, ir.imax, min(ir.maxit, w.n), ir.tol_ir,
                     _ortho(k))
    rc, x, rec = alone[k]
    assert rec["its"] == list(res.its), (rec["its"], res.its)
    assert rec["nnz_p"] == int(pp[-1])
    assert np.abs(x - res.x).max() <= 1e-12 * np.abs(res.x).max()


UNIT_SLACK = 16 << 20   # per unit of work, beside the footprints (the library's allowance for small buffers)


def test_admission_respects_the_budget(S, systems, alone):
    """An arena that holds about two units of work at a time: the units in
    flight (a batch = its footprints + one lane workspace, a device-lane request
    = its footprint) never exceed it together, some requests had to wait, and
    the results are still those of the requests alone."""
    fps = [S.serve_footprint(*_args(w, _ortho(k))) for k, w in enumerate(systems)]
    lanes, lane_ws = 2, 64 << 20
    budget = 2 * (lane_ws + UNIT_SLACK) + int(max(fps) * 1.5)
    srv = S.Server(batch_lanes=lanes, batch_max_n=BATCH_MAX_N, hbm_budget=budget, lane_workspace=lane_ws)
    ids = [srv.submit(*_args(w, _ortho(k))) for k, w in enumerate(systems)]
    recs = []
    for k, i in enumerate(ids):
        rc, x, rec = srv.wait(i)
        assert rc == alone[k][0]
        assert np.array_equal(x, alone[k][1]), k
        assert np.array_equal(rec["its"], alone[k][2]["its"]), k
        assert rec["footprint"] == fps[k]
        recs.append(rec)
    srv.close()
    units = {}
    for r in recs:
        key = (r["lane"], r["t_admit"])
        u = units.setdefault(key, {"t_admit": r["t_admit"], "t_done": r["t_done"], "size": UNIT_SLACK +
                                   (lane_ws if r["lane"] >= 0 else 0)})
        u["size"] += r["footprint"]
    for u in units.values():
        held = sum(v["size"] for v in units.values() if v["t_admit"] <= u["t_admit"] < v["t_done"])
        assert held <= budget, (held, budget)
    assert any(r["t_admit"] > r["t_submit"] + 1e-3 for r in recs)     # somebody waited for a lane or memory


def test_bad_requests_are_rejected(S, systems):
    srv = S.Server(batch_lanes=1, batch_max_n=BATCH_MAX_N, hbm_budget=512 << 20, lane_workspace=128 << 20)
    w = systems[0]
    A, b, pat, build, irp = _args(w)
    with pytest.raises(S.SpaiError):
        srv.submit(A, b, pat, dict(build, maxfill=0), irp)
    with pytest.raises(S.SpaiError):
        srv.submit(A, b, pat, build, dict(irp, imax=0))
    # a request that can never fit the budget (64^3 unknowns with a 500-vector basis: about 1.2 GB)
    big = W.serving_request(W.Arrival(0.0, "aniso", 64, "fp32", 99))
    with pytest.raises(S.SpaiError):
        srv.submit(*_args(big))
    srv.close()


def test_device_lane_serves_smallest_first(S):
    """With an age limit the device lane takes the smallest waiting system first:
    submitted behind a running solve, a small system overtakes a larger one that
    arrived before it; in arrival order it does not."""
    import time

    ws = [W.serving_request(W.Arrival(0.0, "convdiff", side, "fp32", 200 + q)) for q, side in
          enumerate((400, 300, 100))]
    for age, expect_small_first in ((60000, True), (0, False)):
        srv = S.Server(batch_lanes=1, batch_max_n=1000, hbm_budget=16 << 30, lane_workspace=256 << 20,
                       sjf_age_ms=age)
        ids = [srv.submit(*_args(ws[0]))]
        time.sleep(0.02)                      # the first one is on the device lane by now
        ids += [srv.submit(*_args(w)) for w in ws[1:]]
        recs = [srv.wait(i)[2] for i in ids]
        srv.close()
        assert all(r["lane"] == -1 for r in recs)
        assert recs[0]["t_admit"] <= min(recs[1]["t_admit"], recs[2]["t_admit"])
        assert (recs[2]["t_admit"] < recs[1]["t_admit"]) == expect_small_first, (age, recs)


def test_second_waiter_for_one_request_is_rejected(S):
    """A request is waited for once: a second concurrent wait (or one after the
    first collected it) fails cleanly instead of racing for the result."""
    import threading
    import time

    w = W.serving_request(W.Arrival(0.0, "convdiff", 300, "fp32", 300))
    srv = S.Server(batch_lanes=1, batch_max_n=1000, hbm_budget=8 << 30, lane_workspace=256 << 20)
    rid = srv.submit(*_args(w))
    got = {}
    t = threading.Thread(target=lambda: got.update(r=srv.wait(rid)))
    t.start()
    time.sleep(0.05)
    assert S.lib().spai_serve_wait(srv._raw, int(rid), None, None) == S.E_ARG
    t.join()
    with pytest.raises(S.SpaiError):
        srv.wait(rid)
    srv.close()
    rc, x, rec = got["r"]
    assert rc >= 0 and O.ferr(x, w.x_true) <= 1e-12


def test_right_preconditioned_and_single_precision_requests(S):
    """Requests with a right preconditioner (device lane, right-preconditioned
    GMRES) and with working precision single (batch lane, binary32 solver) give
    the direct library calls' results bit for bit."""
    h = S.Handle()
    w = W.serving_request(W.Arrival(0.0, "random", 1500, "fp32", 400))
    s, ir = w.spai, w.ir
    A_h, b_h = w.A, w.b
    build = {"eps": s.eps, "alpha": s.alpha, "beta": s.beta, "maxfill": s.maxfill, "u_f": "fp32"}
    srv = S.Server(batch_lanes=2, batch_max_n=BATCH_MAX_N, hbm_budget=8 << 30, lane_workspace=512 << 20)
    cases = {
        "right": (dict(build, side="right"), {"tau": ir.tau, "imax": ir.imax, "maxit": ir.maxit, "tol_ir": ir.tol_ir,
                                               "u_r": "dd", "ortho": "dcgs2"}),
        "single": (dict(build, u_f="fp16"), {"tau": 1e-4, "imax": ir.imax, "maxit": ir.maxit, "tol_ir": W.TOL_IR32,
                                              "u_r": "fp64", "u": "fp32"}),
    }
    ids = {k: srv.submit(A_h, b_h, None, bp, irp) for k, (bp, irp) in cases.items()}
    got = {k: srv.wait(i) for k, i in ids.items()}
    srv.close()
    A = S.DeviceCSR.from_host(A_h)
    b = torch.as_tensor(b_h, device="cuda")
    for k, (bp, irp) in cases.items():
        rc, x, rec = got[k]
        assert rc >= 0, rec["error"]
        assert (rec["lane"] == -1) == (k == "right")
        P, _, _ = h.spai_build(A, None, bp["eps"], bp["alpha"], bp["beta"], bp["maxfill"], bp["u_f"],
                               bp.get("side", "left"))
        xd = torch.zeros_like(b)
        r = h.gmres_ir(A, P, b, xd, irp["tau"], irp["imax"], irp["maxit"], irp["tol_ir"], irp["u_r"],
                       irp.get("ortho", "mgs"), irp.get("u", "fp64"))
        assert rec["its"] == r["its"], (k, rec["its"], r["its"])
        assert np.array_equal(x, xd.cpu().numpy()), k


def test_wait_while_another_thread_submits(S):
    """One thread waits for a request while another submits two hundred more
    (the server's request table grows and rehashes meanwhile): every request
    completes with a valid result."""
    import threading

    w = W.serving_request(W.Arrival(0.0, "random", 1000, "fp32", 500))
    srv = S.Server(batch_lanes=2, batch_max_n=BATCH_MAX_N, hbm_budget=8 << 30, lane_workspace=512 << 20)
    first = srv.submit(*_args(w))
    got = {}
    t = threading.Thread(target=lambda: got.update(r=srv.wait(first)))
    t.start()
    ids = [srv.submit(*_args(w)) for _ in range(200)]
    t.join()
    rc, x, rec = got["r"]
    assert rc >= 0 and O.ferr(x, w.x_true) <= 1e-12
    for rid in ids:
        rc2, x2, rec2 = srv.wait(rid)
        assert rc2 >= 0 and rec2["its"] == rec["its"] and np.array_equal(x2, x)
    srv.close()


def test_reserved_cus_let_batches_run_beside_a_device_lane_solve(S):
    """With 8 CUs of every XCD reserved for the device lane, a large system's
    solve runs on those 64 CUs (its Arnoldi grid sized to them) while batches of
    small systems run on the other 192: batches start and finish inside the
    large solve.  Every result equals the one the same server gives the request
    alone, bit for bit, and the large solve reaches ferr <= 1e-12."""
    import threading
    import time

    big = W.serving_request(W.Arrival(0.0, "convdiff", 320, "fp32", 700))
    pool = [W.serving_request(W.Arrival(0.0, "random", 1000 + 37 * i, "fp32", 701 + i)) for i in range(40)]

    def server():
        return S.Server(batch_lanes=3, batch_max_n=BATCH_MAX_N, batch_max_systems=2, hbm_budget=8 << 30,
                        lane_workspace=256 << 20, device_lane_cus=8)

    srv = server()
    got = {}
    ib = srv.submit(*_args(big, "dcgs2"))
    t = threading.Thread(target=lambda: got.update(r=srv.wait(ib)))
    t.start()
    sent = []
    while t.is_alive() and len(sent) < 400:
        w = pool[len(sent) % len(pool)]
        sent.append((w, srv.submit(*_args(w))))
        time.sleep(0.002)
    t.join()
    mix = [(w, srv.wait(i)) for w, i in sent]
    srv.close()
    rc, xb, recb = got["r"]
    assert rc >= 0 and recb["lane"] == -1 and recb["cus"] == 64, recb
    assert O.ferr(xb, big.x_true) <= 1e-12
    inside = [r for _, (_, _, r) in mix if recb["t_solve"] < r["t_solve"] and r["t_done"] < recb["t_done"]]
    print("large solve", recb["t_solve"], recb["t_done"], "small requests sent", len(sent),
          "finished inside it", len(inside), flush=True)
    assert inside and all(r["cus"] == 192 and r["lane"] >= 0 for r in inside)
    srv = server()
    rc_a, xb_a, recb_a = srv.wait(srv.submit(*_args(big, "dcgs2")))
    assert rc_a == rc and recb_a["its"] == recb["its"] and np.array_equal(xb_a, xb)
    alone = {}
    for w, (rc_m, x_m, rec_m) in mix:
        if w.name not in alone:
            alone[w.name] = srv.wait(srv.submit(*_args(w)))
        rc_s, x_s, rec_s = alone[w.name]
        assert rc_m == rc_s and rec_m["its"] == rec_s["its"] and np.array_equal(x_m, x_s), w.name
    srv.close()
