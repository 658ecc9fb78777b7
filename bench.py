#!/usr/bin/env python3
"""Benchmark of the SPAI-GMRES-IR hot path on one MI355X.

Workload: 2D convection-diffusion on a 512 x 512 grid (n = 262,144,
nnz = 1,308,672), Peclet 100, diffusion coefficients log-uniform in [1e-2, 1],
adaptive SPAI from the identity pattern (eps = 0.3, beta = 8, at most 20
entries per column) in FP32, then GMRES-IR with an FP64 working precision, a
double-double residual and tau = 1e-8, to a forward error <= 1e-12 against the
exactly known solution.  Synthetic seeded data; the inputs are resident in HBM
before the timed region starts.

One step = one pass of the whole hot path: the SPAI build (Algorithm 1 on
A^T D, all 262,144 columns) and the SPAI-GMRES-IR solve (Algorithm 3).
`value` = steps per second = full solves per second; the JSON line also
carries SPAI columns/s, GMRES-IR solves/s, p50/p99 step times, the all-FP64
forms of the same method, the roofline of the dominant kernel (HIP events on
the library's stream) and the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SPAI cols/s + GMRES-IR solves/s at 1e-12 fwd err, mixed vs FP64; p50/p99"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs), q))


def arnoldi_bytes_per_solve(its, n, ortho):
    """Algorithmic HBM bytes of the Arnoldi iterations of one solve, the bytes the
    chosen kernel streams by design, and the number of launches that do work.

    Algorithmic: Arnoldi iteration j (0-based) reads y = P A v_j (8n) and the
    basis vectors v_0 .. v_j (8n(j+1)) once each and writes v_{j+1} (8n):
    8n(j+3), whatever the orthogonalisation.  By design, MGS streams exactly
    that; CGS2 reads the basis four times (8n(4(j+1)+2)); delayed CGS2 launch j
    reads V_{j-1}, u_j and y, then V_{j-1} again, and writes v_j and u_{j+1}
    (8n(2j+4)), and one more launch per refinement step (pass 1 only) completes
    the last column."""
    alg, design, launches = 0, 0, 0
    for k in its:
        for j in range(k):
            alg += 8 * n * (j + 3)
            if ortho == "mgs":
                design += 8 * n * (j + 3)
            elif ortho == "cgs2":
                design += 8 * n * (4 * (j + 1) + 2)
            else:
                design += 8 * n * (2 * j + 4)
            launches += 1
        if ortho == "dcgs2":
            design += 8 * n * (k + 2)
            launches += 1
    return alg, design, launches


def profiled_traffic(kernel_file, sources):
    """HBM bytes per launch from a committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary,
    or None when the summary is missing or the kernel sources changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", kernel_file)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    hsh = hashlib.sha256()
    for src in sources:
        hsh.update(open(os.path.join(ROOT, src), "rb").read())
    if kv.get("source_sha256") != hsh.hexdigest():
        return None
    return float(kv["traffic_bytes_per_launch"])


def run_form(S, h, w, A, b, x, u_f, u_r, steps, warmup, timed_kernels=(), ortho="dcgs2"):
    """Build + solve `steps` times after `warmup` untimed steps; per-step times in ms."""
    import torch

    s, ir = w.spai, w.ir
    for _ in range(warmup):
        P, _, _ = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, u_f)
        h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, u_r, ortho)
        del P
    for kc, every in timed_kernels:
        h.timing_enable(kc, every)
    stream = torch.cuda.current_stream()
    rec = []
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        P, warn, bst = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, u_f)
        e1.record(stream)
        st = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, u_r, ortho)
        e2.record(stream)
        e2.synchronize()
        rec.append((e0.elapsed_time(e1), e1.elapsed_time(e2), st, bst, warn))
        del P
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t_wall) * 1e3
    timings = {kc: h.timing_read(kc) for kc, _ in timed_kernels}
    for kc, _ in timed_kernels:
        h.timing_enable(kc, 0)
    return rec, wall, timings


def cpu_baseline(w, its_oracle, threads):
    """The oracle timed on a bounded sample of the same workload.

    SPAI: the full oracle build (all columns, `threads` threads, static column
    blocks).  GMRES-IR: the oracle's first refinement step stopped after k = 30,
    60 and 90 Arnoldi iterations; the cost c0 + c1 k + c2 k^2 fitted through
    these three points is summed over the oracle's own iteration tuple for this
    workload (stored by tests/golden/make_convdiff512_golden.py)."""
    import numpy as np

    import oracle as O

    s, ir = w.spai, w.ir
    t0 = time.perf_counter()
    R = O.spai(w.A, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f, nthreads=threads)
    t_build = time.perf_counter() - t0
    pp, pc, pv = R.P_csr(w.n)
    ks, ts = [30, 60, 90], []
    for k in ks:
        t0 = time.perf_counter()
        O.gmres_ir(w.A, pp, pc, pv, R.d, s.u_f, w.b, 0.0, 1, k, 0.0)
        ts.append(time.perf_counter() - t0)
    c = np.linalg.solve(np.array([[1, k, k * k] for k in ks], float), np.array(ts))
    t_solve = float(sum(c[0] + c[1] * k + c[2] * k * k for k in its_oracle))
    total = t_build + t_solve
    return {
        "value": 1.0 / total,
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"full oracle SPAI build ({w.n} columns, {t_build:.2f} s on {threads} threads) + "
                   f"oracle GMRES-IR (MGS) first step cut at k=30/60/90 Arnoldi iterations "
                   f"({', '.join(f'{t:.2f}' for t in ts)} s), quadratic cost fit summed over the oracle's "
                   f"tuple {sum(its_oracle)}({', '.join(map(str, its_oracle))}) -> {t_solve:.1f} s per solve"),
        "spai_cols_per_s": w.n / t_build,
        "est_seconds_per_solve": total,
    }


def run_batch(S, W, args):
    """4096 independent systems (sizes log-uniform in [200, 20000]): the batched
    SPAI build and the batched GMRES-IR (one persistent launch), timed with HIP
    events; every system must reach 1e-12."""
    import numpy as np
    import torch

    B = W.random_batch(4096)
    log(f"workload {B.name} systems={B.nsys} n={B.n} nnz={B.A.nnz}")
    h = S.Handle()
    A = S.DeviceCSR.from_host(B.A)
    b = torch.as_tensor(B.b, device="cuda")
    s, ir = B.spai, B.ir
    stream = torch.cuda.current_stream()
    rec = []
    for k in range(args.warmup + args.steps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        x = torch.zeros_like(b)
        e0.record(stream)
        P, warn, bst = h.spai_build_batched(A, B.sys_ptr, None, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
        e1.record(stream)
        rc, st = h.gmres_ir_batched(A, P, B.sys_ptr, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir)
        e2.record(stream)
        e2.synchronize()
        if k >= args.warmup:
            rec.append((e0.elapsed_time(e1), e1.elapsed_time(e2)))
        del P
    xh = x.cpu().numpy()
    ferr = max(float(np.abs(xh[B.sys_ptr[q]:B.sys_ptr[q + 1]] - B.x_true[B.sys_ptr[q]:B.sys_ptr[q + 1]]).max() /
                     np.abs(B.x_true[B.sys_ptr[q]:B.sys_ptr[q + 1]]).max()) for q in range(B.nsys))
    fails = sum(1 for q in range(B.nsys) if st[q]["status"] != 0)
    step_ms = [a + c for a, c in rec]
    its = np.array([q["total_its"] for q in st])
    out = {
        "metric": METRIC, "value": B.nsys * 1000.0 / float(np.mean(step_ms)), "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64+dd", "data": "synthetic",
        "config": {"workload": B.name, "systems": B.nsys, "n_total": B.n, "nnz_A": B.A.nnz, "spai": "adaptive identity start",
                   "eps": s.eps, "beta": s.beta, "maxfill": s.maxfill, "u_f": s.u_f, "u": "fp64", "u_r": "dd",
                   "tau": ir.tau, "arnoldi": "mgs", "parallelism": "single GPU, one workgroup per system"},
        "spai_cols_per_s": B.n * 1000.0 / float(np.mean([a for a, _ in rec])),
        "spai_ms": float(np.mean([a for a, _ in rec])),
        "gmres_ir_solves_per_s": B.nsys * 1000.0 / float(np.mean([c for _, c in rec])),
        "gmres_ir_ms": float(np.mean([c for _, c in rec])),
        "p50_ms": percentile(step_ms, 50), "p99_ms": percentile(step_ms, 99),
        "its_mean": float(its.mean()), "its_max": int(its.max()), "max_ferr": ferr, "failed_systems": fails,
        "nnz_P": int(bst["nnz"]),
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--grid", type=int, default=512, help="grid side (512 is the benchmark workload)")
    ap.add_argument("--workload", default="convdiff", choices=["convdiff", "batch"],
                    help="convdiff: the benchmark line (default); batch: 4096 independent random banded systems "
                         "(a separate measurement of the batched entry points, printed as its own JSON line)")
    ap.add_argument("--ortho", default="dcgs2", choices=["mgs", "cgs2", "dcgs2"],
                    help="Arnoldi orthogonalisation (all three give the oracle's iteration tuple)")
    ap.add_argument("--profile-run", action="store_true",
                    help="one untimed build + solve of the mixed form and a 256 MiB device copy "
                         "(the reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE); for profiler runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each system is solved on one "
              "device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2202_10204_amd as S
    import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "batch":
        run_batch(S, W, args)
        return
    w = W.convdiff_adaptive(args.grid)
    n = w.n
    log(f"workload {w.name} n={n} nnz={w.A.nnz}")
    h = S.Handle()
    A = S.DeviceCSR.from_host(w.A)
    b = torch.as_tensor(w.b, device="cuda")
    x = torch.zeros_like(b)

    if args.profile_run:
        s, ir = w.spai, w.ir
        P, _, bst = h.spai_build(A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp32")
        st = h.gmres_ir(A, P, b, x, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "dd", args.ortho)
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": w.name, "its": st["its"], "nnz_P": bst["nnz"], "copy_bytes": 256 << 20}),
              flush=True)
        return

    kernels = [("columns", 1), ("mgs", 1), ("spmv_a", 3), ("apply_p", 3), ("residual", 1), ("update", 1)]
    rec, wall, timings = run_form(S, h, w, A, b, x, "fp32", "dd", args.steps, args.warmup, kernels, args.ortho)
    log(f"mixed form: {[(round(a, 1), round(c, 1)) for a, c, *_ in rec]} ms (build, solve)")
    step_ms = [a + c for a, c, *_ in rec]
    build_ms = [a for a, *_ in rec]
    solve_ms = [c for _, c, *_ in rec]
    st = rec[-1][2]
    bst = rec[-1][3]
    xh = x.cpu().numpy()
    ferr = float(np.abs(xh - w.x_true).max() / np.abs(w.x_true).max())
    r = torch.zeros_like(b)
    h.residual(A, b, x, r, "dd")
    anorm = float(np.add.reduceat(np.abs(w.A.val), w.A.rowptr[:-1]).max())
    nbe = float(r.abs().max().item() / (anorm * np.abs(xh).max() + np.abs(w.b).max()))
    mean_ms = float(np.mean(step_ms))

    # FP64 forms of the same method: u_f = FP64 (P stored in FP64) with the DD
    # residual, and additionally u_r = FP64 (the all-FP64 form)
    forms = {}
    for name, uf, ur in (("fp64_spai_dd_residual", "fp64", "dd"), ("all_fp64", "fp64", "fp64")):
        if args.fp64_steps <= 0:
            break
        x64 = torch.zeros_like(b)
        r64, wall64, _ = run_form(S, h, w, A, b, x64, uf, ur, args.fp64_steps, 0, (), args.ortho)
        ms64 = float(np.mean([a + c for a, c, *_ in r64]))
        xe = x64.cpu().numpy()
        forms[name] = {
            "ms_per_step": ms64,
            "value": 1000.0 / ms64,
            "spai_ms": float(np.mean([a for a, *_ in r64])),
            "gmres_ir_ms": float(np.mean([c for _, c, *_ in r64])),
            "its": r64[-1][2]["its"],
            "ferr": float(np.abs(xe - w.x_true).max() / np.abs(w.x_true).max()),
            "speedup_of_mixed": ms64 / mean_ms,
        }
        log(f"{name}: {ms64:.1f} ms/step its={r64[-1][2]['its']}")

    # roofline of the dominant kernel class (sampled launch durations)
    per_class = {}
    for kc, (cnt, ms) in timings.items():
        every = dict(kernels)[kc]
        per_class[kc] = {"launches_timed": cnt, "avg_ms": (ms / cnt) if cnt else None,
                         "est_total_ms_per_step": (ms * every / args.steps) if cnt else 0.0}
    dom = max(per_class, key=lambda k: per_class[k]["est_total_ms_per_step"])
    roof = None
    if dom == "mgs" and per_class["mgs"]["avg_ms"]:
        # every launch is timed; launches enqueued past convergence (no-ops) count
        # in the time but not in the bytes, so the figure is conservative
        tot_bytes, design_bytes, real = arnoldi_bytes_per_solve(st["its"], n, args.ortho)
        cnt, ms = timings["mgs"]
        secs = ms * 1e-3 / args.steps
        achieved = tot_bytes / secs / 1e9
        kname = {"mgs": "k_arnoldi", "cgs2": "k_arnoldi_cgs2", "dcgs2": "k_arnoldi_dcgs2"}[args.ortho]
        traffic = profiled_traffic(f"{kname}_convdiff512_traffic.txt",
                                   ["paper_2202_10204_amd/csrc/gmres_ir.hip", "paper_2202_10204_amd/csrc/common.hpp"])
        roof = {"bound": "hbm", "kernel": kname, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_unit": "bytes/launch",
                "bytes_per_launch": tot_bytes / real, "design_bytes_per_launch": design_bytes / real,
                "design_rate_GBs": design_bytes / secs / 1e9, "avg_launch_us": ms * 1e3 / cnt,
                "launches_per_step": cnt / args.steps, "real_launches_per_step": real}
    elif per_class[dom]["avg_ms"]:
        roof = {"bound": "hbm", "kernel": dom, "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": None, "traffic": None, "avg_launch_us": per_class[dom]["avg_ms"] * 1e3}

    out = {
        "metric": METRIC,
        "value": 1000.0 / mean_ms,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mean_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64+dd",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "nnz_A": w.A.nnz, "spai": "adaptive identity start",
                   "eps": w.spai.eps, "beta": w.spai.beta, "maxfill": w.spai.maxfill, "u_f": "fp32",
                   "u": "fp64", "u_r": "dd", "tau": w.ir.tau, "arnoldi": args.ortho, "parallelism": "single GPU"},
        "spai_cols_per_s": n / (float(np.mean(build_ms)) * 1e-3),
        "spai_ms": float(np.mean(build_ms)),
        "gmres_ir_solves_per_s": 1000.0 / float(np.mean(solve_ms)),
        "gmres_ir_ms": float(np.mean(solve_ms)),
        "p50_ms": percentile(step_ms, 50),
        "p99_ms": percentile(step_ms, 99),
        "wall_ms_timed_region": wall,
        "its": f"{st['total_its']}({', '.join(map(str, st['its']))})",
        "ferr": ferr,
        "nbe": nbe,
        "nnz_P": int(bst["nnz"]),
        "fp64_forms": forms,
        "kernels": per_class,
        "roofline": roof,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline and args.grid == 512:
        golden = os.path.join(ROOT, "tests", "golden", "convdiff512_oracle.json")
        its_oracle = json.load(open(golden))["its"]
        threads = min(len(os.sched_getaffinity(0)), 16)
        log(f"cpu baseline on {threads} threads")
        out["cpu_baseline"] = cpu_baseline(w, its_oracle, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
