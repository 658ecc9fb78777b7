"""Autotuner for the column kernel of the SPAI build (Algorithm 1's per-column solver).

The library carries several column-kernel configurations (lanes of a wavefront
per column problem, shadow rows, gathered entries and augmentation candidates
staged in LDS; `column_config`).  Every configuration gives the same bits: a
column that outgrows one is recomputed from scratch by a larger one, with the
same arithmetic.  So the choice, and the choice of updating each column's QR
across augmentation steps or refactoring it, are questions of speed only, and
their answer depends on the GPU and on the problem's shape (fill cap, adaptive
or fixed pattern, row lengths of A, size).

`tune` times every configuration able to hold the pattern, with and without the
QR update, on a strided sample of the columns (the library's spai_tune_build:
the build's own preprocessing, then the column phase over the sample, deferred
columns included), and keeps the fastest in a JSON cache keyed by GPU
architecture and problem bin.  `build` looks the bin up (tuning it on a miss)
and runs spai_build with the chosen configuration.
"""
from __future__ import annotations

import json
import math
import os
import tempfile
from typing import Optional

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2202_10204_amd", "autotune.json")


def gpu_arch() -> str:
    """gfx name of device 0 (e.g. gfx950), without feature suffixes."""
    import torch

    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _pow2_bucket(v: int) -> int:
    return 1 << max(0, math.ceil(math.log2(max(int(v), 1))))


def bin_key(A, pattern, alpha: int, beta: int, maxfill: int, u_f: str, side: str = "left") -> str:
    """Problem bin of a build: what selects the eligible configurations (the
    pattern bound max(maxfill, longest initial column)) and what moves their
    relative speed (adaptive or fixed pattern, beta, u_f, the longest row of A
    in powers of two, n in powers of four).  A and pattern are host arrays
    (workloads.CSR / Pattern)."""
    n = int(A.n)
    rows = A.rowptr[1:] - A.rowptr[:-1]
    q = int(rows.max()) if n else 0
    pinit = int((pattern.ptr[1:] - pattern.ptr[:-1]).max()) if pattern is not None and n else 1
    pmax = max(int(maxfill), pinit)
    mode = "fixed" if alpha == 0 else f"adaptive-b{int(beta)}"
    nb = 4 ** max(0, math.ceil(math.log(max(n, 1), 4)))
    return f"{side}/{u_f}/{mode}/p{pmax}/q{_pow2_bucket(q)}/n{nb}"


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, data: dict) -> None:
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".autotune.", suffix=".json")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(times: dict) -> tuple:
    """Fastest (kernel_cfg, qr_update) of {(cfg, qr_update): ns per column}; on a
    tie the smaller configuration, then the recompute."""
    if not times:
        raise ValueError("no configuration holds this pattern")
    return min(times, key=lambda k: (times[k], k[0], k[1]))


def tune(h, A_dev, pattern_dev, A, pattern, eps: float, alpha: int, beta: int, maxfill: int, u_f: str = "fp32",
         side: str = "left", cache: Optional[str] = DEFAULT_CACHE, sample: int = 262144, reps: int = 3,
         retune: bool = False) -> dict:
    """The cached choice for this problem's bin, measured on a miss (or when
    retune).  Returns {"kernel_cfg", "qr_update", "ns_per_col", "candidates",
    "sample", "arch", "bin"}; cache None keeps nothing on disk."""
    arch = gpu_arch()
    key = bin_key(A, pattern, alpha, beta, maxfill, u_f, side)
    data = load_cache(cache) if cache else {}
    hit = data.get(arch, {}).get(key)
    if hit is not None and not retune:
        return dict(hit, arch=arch, bin=key, cached=True)
    times = h.tune_build(A_dev, pattern_dev, eps, alpha, beta, maxfill, u_f, side, sample, reps)
    cfg, inc = pick(times)
    entry = {"kernel_cfg": int(cfg), "qr_update": int(inc), "ns_per_col": float(times[(cfg, inc)]),
             "candidates": {f"{c}/{u}": float(t) for (c, u), t in sorted(times.items())},
             "sample": int(min(sample, A.n))}
    if cache:
        data = load_cache(cache)
        data.setdefault(arch, {})[key] = entry
        save_cache(cache, data)
    return dict(entry, arch=arch, bin=key, cached=False)


def build(h, A_dev, pattern_dev, A, pattern, eps: float, alpha: int, beta: int, maxfill: int, u_f: str = "fp32",
          side: str = "left", cache: Optional[str] = DEFAULT_CACHE, **kw):
    """spai_build with the tuned configuration; returns (Precond, warnings, stats, choice)."""
    c = tune(h, A_dev, pattern_dev, A, pattern, eps, alpha, beta, maxfill, u_f, side, cache, **kw)
    P, warn, st = h.spai_build(A_dev, pattern_dev, eps, alpha, beta, maxfill, u_f, side,
                               qr_update=bool(c["qr_update"]), kernel_cfg=c["kernel_cfg"])
    return P, warn, st, c
