"""Python binding of libspai (SPAI-GMRES-IR on MI355X).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libspai.so``; PyTorch provides device memory and the stream.  The names
follow the C ABI in ``include/spai.h``.

The library must have been built (``python -m paper_2202_10204_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np
import torch  # imported before libspai so both share torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspai.so")

FP64, FP32, FP16, BF16, DD = 0, 1, 2, 3, 4
PREC = {"fp64": FP64, "fp32": FP32, "fp16": FP16, "bf16": BF16, "dd": DD}

OK, E_ARG, E_OOM, E_HIP, E_INTERNAL = 0, -1, -2, -3, -4
W_EPS, W_RANKDEF, W_NONFINITE, W_MAXIT, W_NOCONV = 1, 2, 4, 8, 16

# kernel classes for sampled launch timing
KERNELS = {"columns": 0, "spmv_a": 1, "apply_p": 2, "mgs": 3, "residual": 4, "update": 5}

_c_i32, _c_i64, _c_f64, _p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class _Csr(ctypes.Structure):
    _fields_ = [("n", _c_i32), ("nnz", _c_i32), ("rowptr", _p), ("col", _p), ("val", _p)]


class _Pattern(ctypes.Structure):
    _fields_ = [("n", _c_i32), ("nnz", _c_i32), ("ptr", _p), ("idx", _p)]


class _BuildParams(ctypes.Structure):
    _fields_ = [("eps", _c_f64), ("alpha", _c_i32), ("beta", _c_i32), ("maxfill", _c_i32),
                ("u_f", ctypes.c_int), ("side", _c_i32), ("qr_update", _c_i32), ("kernel_cfg", _c_i32)]


class _ColumnConfig(ctypes.Structure):
    _fields_ = [("lanes", _c_i32), ("maxp", _c_i32), ("maxm", _c_i32), ("emax", _c_i32), ("cmax", _c_i32),
                ("problems_per_wave", _c_i32), ("lds_bytes_per_problem", _c_i32)]


KCFG_COUNT = 9


SIDE = {"left": 0, "right": 1}


class _BuildStats(ctypes.Structure):
    _fields_ = [("nnz", _c_i64), ("max_len", _c_i32), ("max_steps", _c_i32), ("max_shadow", _c_i32),
                ("cols_over_eps", _c_i32), ("cols_rankdef", _c_i32), ("cols_nonfinite", _c_i32),
                ("cols_deferred", _c_i32), ("max_res", _c_f64), ("nnz_numeric", _c_i64),
                ("cols_fallback", _c_i32), ("pad", _c_i32)]


class _View(ctypes.Structure):
    _fields_ = [("n", _c_i32), ("nnz", _c_i64), ("rowptr", _p), ("col", _p), ("val", _p),
                ("val_prec", ctypes.c_int), ("d", _p), ("stride", _c_i32), ("j_ins", _p),
                ("m_ins", _p), ("len", _p), ("steps", _p), ("res", _p), ("flags", _p), ("side", _c_i32),
                ("u_f", ctypes.c_int)]


class _IrParams(ctypes.Structure):
    _fields_ = [("u_r", ctypes.c_int), ("tau", _c_f64), ("imax", _c_i32), ("maxit", _c_i32),
                ("tol_ir", _c_f64), ("ortho", _c_i32), ("u", ctypes.c_int), ("graph", _c_i32),
                ("x_given", _c_i32), ("x_true", _p)]


ORTHO = {"mgs": 0, "cgs2": 1, "dcgs2": 2}


class _IrStats(ctypes.Structure):
    _fields_ = [("steps", _c_i32), ("its", _c_i32 * 32), ("total_its", _c_i32), ("status", _c_i32),
                ("gest", _c_f64 * 32), ("dnorm", _c_f64 * 32), ("nbe", _c_f64), ("ferr", _c_f64)]


def _ir_dict(st, status) -> dict:
    k = st.steps
    return {"steps": k, "its": list(st.its[:k]), "total_its": st.total_its, "status": status,
            "gest": list(st.gest[:k]), "dnorm": list(st.dnorm[:k]), "nbe": st.nbe,
            "ferr": None if st.ferr < 0 else st.ferr}


class _ServeParams(ctypes.Structure):
    _fields_ = [("batch_lanes", _c_i32), ("batch_max_n", _c_i32), ("batch_max_systems", _c_i32), ("sjf_age_ms", _c_i32),
                ("hbm_budget", _c_i64), ("lane_workspace", _c_i64), ("device_lane_cus", _c_i32), ("pad", _c_i32)]


class _ServeRequest(ctypes.Structure):
    _fields_ = [("n", _c_i32), ("nnz", _c_i32), ("rowptr", _p), ("col", _p), ("val", _p), ("b", _p),
                ("jnnz", _c_i32), ("jptr", _p), ("jidx", _p), ("build", _BuildParams), ("ir", _IrParams)]


class _ServeResult(ctypes.Structure):
    _fields_ = [("rc", _c_i32), ("lane", _c_i32), ("batch_size", _c_i32), ("cus", _c_i32),
                ("footprint", _c_i64), ("nnz_p", _c_i64), ("t_submit", _c_f64), ("t_admit", _c_f64),
                ("t_solve", _c_f64), ("t_done", _c_f64), ("ir", _IrStats)]


class SpaiError(RuntimeError):
    pass


_lib = None

# Device memory of the library comes from torch's caching allocator
# (spai_set_allocator): one owner for all device memory of the process.
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p)


def _torch_alloc(nbytes, device, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))
    except Exception:          # out of memory: the library reports SPAI_E_OOM
        return None


def _torch_free(ptr, device, stream, ctx):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:          # interpreter shutdown
        pass


_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)
allocator = "hip"              # "torch" once use_torch_allocator() is in force


def use_torch_allocator(enable: bool = True):
    """Route the library's device allocations through torch's caching allocator
    (enable) or back to hipMalloc/hipFree.  Installed when the library loads."""
    global allocator
    L = lib()
    if enable:
        _check(L.spai_set_allocator(_TORCH_ALLOC, _TORCH_FREE, None), "spai_set_allocator")
        allocator = "torch"
    else:
        _check(L.spai_set_allocator(_ALLOC_FN(), _FREE_FN(), None), "spai_set_allocator")   # NULL pair
        allocator = "hip"


def lib():
    """Load libspai.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SpaiError(f"{LIB_PATH} is missing: build the HIP library first "
                            "(python -m paper_2202_10204_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.spai_last_error.restype = ctypes.c_char_p
        L.spai_last_error.argtypes = []
        L.spai_create.argtypes = [P(_p)]
        L.spai_destroy.argtypes = [_p]
        L.spai_set_stream.argtypes = [_p, _p]
        L.spai_build.argtypes = [_p, P(_Csr), P(_Pattern), P(_BuildParams), P(_p), P(_BuildStats)]
        L.spai_tune_build.argtypes = [_p, P(_Csr), P(_Pattern), P(_BuildParams), _c_i32, _c_i32, P(_c_f64)]
        L.spai_column_config_get.argtypes = [_c_i32, P(_ColumnConfig)]
        L.spai_precond_import.argtypes = [_p, _c_i32, _c_i64, _p, _p, _p, ctypes.c_int, _p, P(_p)]
        L.spai_precond_view_get.argtypes = [_p, P(_View)]
        L.spai_precond_destroy.argtypes = [_p]
        L.spai_gmres_ir.argtypes = [_p, P(_Csr), _p, _p, _p, P(_IrParams), P(_IrStats)]
        L.spai_gmres_ir_noalloc.argtypes = [_p, P(_Csr), _p, _p, _p, P(_IrParams), P(_IrStats)]
        L.spai_residual.argtypes = [_p, P(_Csr), _p, _p, _p, ctypes.c_int]
        L.spai_precond_apply.argtypes = [_p, _p, _p, _p]
        L.spai_precond_apply_uf.argtypes = [_p, _p, _p, _p]
        L.spai_spmv.argtypes = [_p, P(_Csr), _p, _p]
        L.spai_build_batched.argtypes = [_p, P(_Csr), _c_i32, P(_c_i32), P(_Pattern), P(_BuildParams), P(_p),
                                         P(_BuildStats)]
        L.spai_gmres_ir_batched.argtypes = [_p, P(_Csr), _p, _c_i32, P(_c_i32), _p, _p, P(_IrParams), P(_IrStats)]
        L.spai_serve_footprint.argtypes = [P(_ServeRequest), P(_c_i64)]
        L.spai_serve_create.argtypes = [P(_ServeParams), P(_p)]
        L.spai_serve_submit.argtypes = [_p, P(_ServeRequest), P(_c_i64)]
        L.spai_serve_wait.argtypes = [_p, _c_i64, _p, P(_ServeResult)]
        L.spai_serve_destroy.argtypes = [_p]
        L.spai_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, _p]
        L.spai_timing_enable.argtypes = [_p, ctypes.c_int, ctypes.c_int]
        L.spai_timing_read.argtypes = [_p, ctypes.c_int, P(_c_i64), P(_c_f64)]
        for name in ("spai_timing_enable", "spai_timing_read", "spai_create", "spai_destroy", "spai_set_stream", "spai_build", "spai_precond_import",
                     "spai_precond_view_get", "spai_precond_destroy", "spai_gmres_ir", "spai_residual",
                     "spai_precond_apply", "spai_precond_apply_uf", "spai_spmv", "spai_build_batched",
                     "spai_gmres_ir_batched", "spai_serve_footprint", "spai_serve_create", "spai_serve_submit",
                     "spai_serve_wait", "spai_serve_destroy", "spai_set_allocator", "spai_gmres_ir_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
        use_torch_allocator(True)
    return _lib


def last_error() -> str:
    return lib().spai_last_error().decode()


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise SpaiError(f"{what} failed ({rc}): {last_error()}")
    return rc


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# device-resident inputs
# ---------------------------------------------------------------------------

def _check_structure(n: int, ptr, idx, what: str):
    """Host check of a compressed structure before it is copied to the device:
    ptr runs from 0 to len(idx) without decreasing, every index in [0, n)."""
    ptr = np.ascontiguousarray(ptr, dtype=np.int32)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    if n <= 0 or ptr.shape != (n + 1,) or ptr[0] != 0 or ptr[-1] != idx.size:
        raise SpaiError(f"{what} pointers must hold n + 1 = {n + 1} values from 0 to {idx.size}")
    if np.any(np.diff(ptr) < 0):
        raise SpaiError(f"{what} pointers decrease")
    if idx.size and (idx.min() < 0 or idx.max() >= n):
        raise SpaiError(f"{what} index outside [0, n)")
    return ptr, idx


@dataclasses.dataclass
class DeviceCSR:
    """CSR matrix on the device (int32 indices, FP64 values)."""

    n: int
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor

    @classmethod
    def from_host(cls, A, device="cuda") -> "DeviceCSR":
        rp, ci = _check_structure(int(A.n), A.rowptr, A.col, "matrix row")
        return cls(int(A.n), torch.as_tensor(rp, device=device), torch.as_tensor(ci, device=device),
                   torch.as_tensor(np.asarray(A.val, np.float64), device=device))

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    def c(self) -> _Csr:
        return _Csr(self.n, self.nnz, self.rowptr.data_ptr(), self.col.data_ptr(), self.val.data_ptr())


@dataclasses.dataclass
class DevicePattern:
    n: int
    ptr: torch.Tensor
    idx: torch.Tensor

    @classmethod
    def from_host(cls, pat, device="cuda") -> "DevicePattern":
        pp, pi = _check_structure(int(pat.n), pat.ptr, pat.idx, "pattern column")
        return cls(int(pat.n), torch.as_tensor(pp, device=device), torch.as_tensor(pi, device=device))

    def c(self) -> _Pattern:
        return _Pattern(self.n, int(self.idx.numel()), self.ptr.data_ptr(), self.idx.data_ptr())


# ---------------------------------------------------------------------------
# preconditioner object
# ---------------------------------------------------------------------------

_VAL_DTYPE = {FP64: torch.float64, FP32: torch.float32, FP16: torch.float16, BF16: torch.bfloat16}


def _copy_from_device_ptr(ptr: int, numel: int, dtype: torch.dtype, device) -> torch.Tensor:
    """Copy `numel` elements at a device address owned by the library into a new tensor."""
    out = torch.empty(numel, dtype=dtype, device=device)
    if numel:
        nbytes = numel * out.element_size()
        _hip_memcpy_d2d(out.data_ptr(), ptr, nbytes)
    return out


_hip = None


def _hip_memcpy_d2d(dst: int, src: int, nbytes: int):
    """Device-to-device copy through the HIP runtime torch has loaded."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so.7", mode=ctypes.RTLD_GLOBAL)
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [_p, _p, ctypes.c_size_t, ctypes.c_int]
    torch.cuda.current_stream().synchronize()
    rc = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3)  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise SpaiError(f"hipMemcpy failed ({rc})")


class Precond:
    """P = M^T D owned by the library (freed with the object)."""

    def __init__(self, handle: "Handle", raw: int, stats: Optional[dict] = None):
        self._h = handle
        self._raw = ctypes.c_void_p(raw)
        self.stats = stats or {}

    @property
    def raw(self):
        return self._raw

    def view(self) -> _View:
        v = _View()
        _check(lib().spai_precond_view_get(self._raw, ctypes.byref(v)), "spai_precond_view_get")
        return v

    def csr(self, device="cuda"):
        """Copies of (rowptr, col, val as stored, d)."""
        v = self.view()
        n, nnz = v.n, v.nnz
        rowptr = _copy_from_device_ptr(v.rowptr, n + 1, torch.int32, device)
        col = _copy_from_device_ptr(v.col, nnz, torch.int32, device)
        val = _copy_from_device_ptr(v.val, nnz, _VAL_DTYPE[v.val_prec], device)
        d = _copy_from_device_ptr(v.d, n, torch.float64, device)
        return rowptr, col, val, d

    def columns(self, device="cuda") -> dict:
        """Per-column build results: J_k in insertion order, m-bar, len, steps, res, flags."""
        v = self.view()
        if not v.j_ins:
            raise SpaiError("preconditioner was imported: no per-column build data")
        n, s = v.n, v.stride
        return {
            "stride": s,
            "J": _copy_from_device_ptr(v.j_ins, n * s, torch.int32, device).view(n, s),
            "m": _copy_from_device_ptr(v.m_ins, n * s, torch.float64, device).view(n, s),
            "len": _copy_from_device_ptr(v.len, n, torch.int32, device),
            "steps": _copy_from_device_ptr(v.steps, n, torch.int32, device),
            "res": _copy_from_device_ptr(v.res, n, torch.float64, device),
            "flags": _copy_from_device_ptr(v.flags, n, torch.int32, device),
        }

    def __del__(self):
        try:
            if self._raw and self._raw.value:
                lib().spai_precond_destroy(self._raw)
                self._raw = ctypes.c_void_p(0)
        except Exception:
            pass


# ---------------------------------------------------------------------------
# handle
# ---------------------------------------------------------------------------

class Handle:
    """Library handle bound to the current device and torch's current stream."""

    def __init__(self, stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise SpaiError("no GPU available: libspai runs on the device only")
        L = lib()
        raw = ctypes.c_void_p()
        _check(L.spai_create(ctypes.byref(raw)), "spai_create")
        self._raw = raw
        self.set_stream(stream or torch.cuda.current_stream())

    def set_stream(self, stream: torch.cuda.Stream):
        self.stream = stream
        _check(lib().spai_set_stream(self._raw, ctypes.c_void_p(stream.cuda_stream)), "spai_set_stream")

    def close(self):
        if getattr(self, "_raw", None) is not None and self._raw.value:
            lib().spai_destroy(self._raw)
            self._raw = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- Algorithm 1 ---------------------------------------------------------
    def spai_build(self, A: DeviceCSR, pattern: Optional[DevicePattern], eps: float, alpha: int, beta: int,
                   maxfill: int, u_f: str = "fp32", side: str = "left", qr_update: bool = False,
                   kernel_cfg: int = 0):
        """Returns (Precond, warnings, stats dict).  side = "left" (P = M^T D, Algorithm 3)
        or "right" (P = D M with A P ~ I; the solve then preconditions on the right);
        qr_update: update each column's QR across augmentation steps (same results);
        kernel_cfg: column-kernel configuration 1..KCFG_COUNT, 0 = the library's rule
        (same results)."""
        prm = _BuildParams(float(eps), int(alpha), int(beta), int(maxfill), PREC[u_f], SIDE[side],
                           int(bool(qr_update)), int(kernel_cfg))
        st = _BuildStats()
        out = ctypes.c_void_p()
        csr = A.c()
        pat = pattern.c() if pattern is not None else None
        rc = _check(lib().spai_build(self._raw, ctypes.byref(csr), ctypes.byref(pat) if pat else None,
                                     ctypes.byref(prm), ctypes.byref(out), ctypes.byref(st)), "spai_build")
        stats = {f: getattr(st, f) for f, _ in _BuildStats._fields_}
        return Precond(self, out.value, stats), rc, stats

    def tune_build(self, A: DeviceCSR, pattern: Optional[DevicePattern], eps: float, alpha: int, beta: int,
                   maxfill: int, u_f: str = "fp32", side: str = "left", sample: int = 262144, reps: int = 3):
        """Time every column-kernel configuration that holds the pattern, with and
        without the QR update, on a strided sample of columns (spai_tune_build).
        Returns {(kernel_cfg, qr_update): ns per column}."""
        prm = _BuildParams(float(eps), int(alpha), int(beta), int(maxfill), PREC[u_f], SIDE[side], 0, 0)
        out = (_c_f64 * (2 * KCFG_COUNT))()
        csr = A.c()
        pat = pattern.c() if pattern is not None else None
        _check(lib().spai_tune_build(self._raw, ctypes.byref(csr), ctypes.byref(pat) if pat else None,
                                     ctypes.byref(prm), int(sample), int(reps), out), "spai_tune_build")
        return {(1 + q // 2, q % 2): out[q] for q in range(2 * KCFG_COUNT) if out[q] >= 0.0}

    def precond_import(self, n: int, rowptr: torch.Tensor, col: torch.Tensor, val_f64: torch.Tensor,
                       val_prec: str, d: torch.Tensor) -> Precond:
        out = ctypes.c_void_p()
        _check(lib().spai_precond_import(self._raw, int(n), int(col.numel()), _ptr(rowptr), _ptr(col),
                                         _ptr(val_f64), PREC[val_prec], _ptr(d), ctypes.byref(out)),
               "spai_precond_import")
        return Precond(self, out.value)

    # -- Algorithm 3 ---------------------------------------------------------
    def gmres_ir(self, A: DeviceCSR, P: Precond, b: torch.Tensor, x: torch.Tensor, tau: float, imax: int,
                 maxit: int, tol_ir: float, u_r: str = "dd", ortho: str = "mgs", u: str = "fp64",
                 graph: bool = False, x_given: bool = False, x_true: Optional[torch.Tensor] = None):
        """graph: replay each chunk of DCGS2 Arnoldi steps as one HIP graph (same results);
        x_given: x holds the first iterate (warm start instead of x0 = P b);
        x_true: exact solution on the device, for the forward error in the result."""
        prm = _IrParams(PREC[u_r], float(tau), int(imax), int(maxit), float(tol_ir), ORTHO[ortho], PREC[u],
                        int(bool(graph)), int(bool(x_given)), _ptr(x_true))
        st = _IrStats()
        csr = A.c()
        rc = _check(lib().spai_gmres_ir(self._raw, ctypes.byref(csr), P.raw, _ptr(b), _ptr(x),
                                        ctypes.byref(prm), ctypes.byref(st)), "spai_gmres_ir")
        return _ir_dict(st, rc)

    # -- batches of independent systems (block-diagonal A, host sys_ptr) ------
    def spai_build_batched(self, A: DeviceCSR, sys_ptr, pattern: Optional[DevicePattern], eps: float, alpha: int,
                           beta: int, maxfill: int, u_f: str = "fp32", qr_update: bool = False,
                           kernel_cfg: int = 0):
        """Returns (Precond of the whole batch, warnings, stats dict)."""
        sp = (_c_i32 * len(sys_ptr))(*[int(v) for v in sys_ptr])
        prm = _BuildParams(float(eps), int(alpha), int(beta), int(maxfill), PREC[u_f], 0, int(bool(qr_update)),
                           int(kernel_cfg))
        st = _BuildStats()
        out = ctypes.c_void_p()
        csr = A.c()
        pat = pattern.c() if pattern is not None else None
        rc = _check(lib().spai_build_batched(self._raw, ctypes.byref(csr), len(sys_ptr) - 1, sp,
                                             ctypes.byref(pat) if pat else None, ctypes.byref(prm),
                                             ctypes.byref(out), ctypes.byref(st)), "spai_build_batched")
        stats = {f: getattr(st, f) for f, _ in _BuildStats._fields_}
        return Precond(self, out.value, stats), rc, stats

    def gmres_ir_batched(self, A: DeviceCSR, P: Precond, sys_ptr, b: torch.Tensor, x: torch.Tensor, tau: float,
                         imax: int, maxit: int, tol_ir: float, u_r: str = "dd", u: str = "fp64",
                         x_given: bool = False, x_true: Optional[torch.Tensor] = None):
        """Returns (warning bits of all systems, list of per-system stats dicts)."""
        nsys = len(sys_ptr) - 1
        sp = (_c_i32 * len(sys_ptr))(*[int(v) for v in sys_ptr])
        prm = _IrParams(PREC[u_r], float(tau), int(imax), int(maxit), float(tol_ir), ORTHO["mgs"], PREC[u], 0,
                        int(bool(x_given)), _ptr(x_true))
        st = (_IrStats * nsys)()
        csr = A.c()
        rc = _check(lib().spai_gmres_ir_batched(self._raw, ctypes.byref(csr), P.raw, nsys, sp, _ptr(b), _ptr(x),
                                                ctypes.byref(prm), st), "spai_gmres_ir_batched")
        return rc, [_ir_dict(st[q], st[q].status) for q in range(nsys)]

    # -- measurement ---------------------------------------------------------
    def timing_enable(self, kernel: str, sample_every: int = 1):
        _check(lib().spai_timing_enable(self._raw, KERNELS[kernel], int(sample_every)), "spai_timing_enable")

    def timing_read(self, kernel: str):
        """(launches timed, summed duration in ms) since enabling or the last read."""
        n = _c_i64()
        ms = _c_f64()
        _check(lib().spai_timing_read(self._raw, KERNELS[kernel], ctypes.byref(n), ctypes.byref(ms)),
               "spai_timing_read")
        return int(n.value), float(ms.value)

    # -- building blocks -----------------------------------------------------
    def residual(self, A: DeviceCSR, b, x, r, u_r: str = "dd"):
        csr = A.c()
        _check(lib().spai_residual(self._raw, ctypes.byref(csr), _ptr(b), _ptr(x), _ptr(r), PREC[u_r]),
               "spai_residual")

    def precond_apply(self, P: Precond, w, y):
        _check(lib().spai_precond_apply(self._raw, P.raw, _ptr(w), _ptr(y)), "spai_precond_apply")

    def precond_apply_uf(self, P: Precond, b, x0):
        _check(lib().spai_precond_apply_uf(self._raw, P.raw, _ptr(b), _ptr(x0)), "spai_precond_apply_uf")

    def spmv(self, A: DeviceCSR, x, y):
        csr = A.c()
        _check(lib().spai_spmv(self._raw, ctypes.byref(csr), _ptr(x), _ptr(y)), "spai_spmv")


# ---------------------------------------------------------------------------
# serving: the library's request loop (host arrays in, host solution out)
# ---------------------------------------------------------------------------

def _serve_request(A, b, pattern, build: dict, ir: dict):
    """Marshal one request; returns (struct, arrays kept alive while it is used)."""
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    av = np.ascontiguousarray(A.val, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    keep = [rp, ci, av, bb]
    jp = ji = None
    if pattern is not None:
        jp = np.ascontiguousarray(pattern.ptr, dtype=np.int32)
        ji = np.ascontiguousarray(pattern.idx, dtype=np.int32)
        keep += [jp, ji]
    bp = _BuildParams(float(build["eps"]), int(build["alpha"]), int(build["beta"]), int(build["maxfill"]),
                      PREC[build["u_f"]], SIDE[build.get("side", "left")], int(bool(build.get("qr_update", 0))),
                      int(build.get("kernel_cfg", 0)))
    ip = _IrParams(PREC[ir.get("u_r", "dd")], float(ir["tau"]), int(ir["imax"]), int(ir["maxit"]),
                   float(ir["tol_ir"]), ORTHO[ir.get("ortho", "mgs")], PREC[ir.get("u", "fp64")],
                   int(bool(ir.get("graph", 0))))
    r = _ServeRequest(int(A.n), int(ci.size), rp.ctypes.data, ci.ctypes.data, av.ctypes.data, bb.ctypes.data,
                      int(ji.size) if ji is not None else 0, jp.ctypes.data if jp is not None else None,
                      ji.ctypes.data if ji is not None else None, bp, ip)
    return r, keep


def column_config(cfg: int) -> dict:
    """Shape of column-kernel configuration cfg (1..KCFG_COUNT); host only."""
    c = _ColumnConfig()
    _check(lib().spai_column_config_get(int(cfg), ctypes.byref(c)), "spai_column_config_get")
    return {f: getattr(c, f) for f, _ in _ColumnConfig._fields_}


def serve_footprint(A, b, pattern, build: dict, ir: dict) -> int:
    """Device bytes admission reserves for a request (host only)."""
    r, keep = _serve_request(A, b, pattern, build, ir)
    out = _c_i64()
    _check(lib().spai_serve_footprint(ctypes.byref(r), ctypes.byref(out)), "spai_serve_footprint")
    return int(out.value)


class Server:
    """The library's request loop on the current device (see spai_serve_* in include/spai.h)."""

    def __init__(self, batch_lanes: int = 3, batch_max_n: int = 20000, batch_max_systems: int = 1024,
                 hbm_budget: int = 64 << 30, lane_workspace: int = 0, sjf_age_ms: int = 0,
                 device_lane_cus: int = 0):
        """device_lane_cus: CUs per XCD reserved for the device lane's solves (batches
        run on the others and keep running beside such a solve); 0 = none."""
        if not torch.cuda.is_available():
            raise SpaiError("no GPU available: libspai runs on the device only")
        prm = _ServeParams(int(batch_lanes), int(batch_max_n), int(batch_max_systems), int(sjf_age_ms),
                           int(hbm_budget), int(lane_workspace), int(device_lane_cus), 0)
        raw = ctypes.c_void_p()
        _check(lib().spai_serve_create(ctypes.byref(prm), ctypes.byref(raw)), "spai_serve_create")
        self._raw = raw
        self._n = {}

    def submit(self, A, b, pattern, build: dict, ir: dict) -> int:
        """Queue one system (host CSR ``A`` with rowptr/col/val, host ``b``, optional
        host pattern with ptr/idx); returns its id."""
        r, keep = _serve_request(A, b, pattern, build, ir)
        rid = _c_i64()
        _check(lib().spai_serve_submit(self._raw, ctypes.byref(r), ctypes.byref(rid)), "spai_serve_submit")
        self._n[rid.value] = int(A.n)
        return int(rid.value)

    def wait(self, rid: int):
        """Block until request ``rid`` is done; returns (rc, x or None, record dict)."""
        n = self._n.pop(rid, None)
        if n is None:
            raise SpaiError(f"spai_serve_wait: unknown or already collected request {rid}")
        x = np.empty(n, np.float64)
        res = _ServeResult()
        rc = lib().spai_serve_wait(self._raw, int(rid), x.ctypes.data, ctypes.byref(res))
        k = res.ir.steps
        rec = {"rc": res.rc, "lane": res.lane, "batch_size": res.batch_size, "footprint": res.footprint,
               "nnz_p": res.nnz_p, "t_submit": res.t_submit, "t_admit": res.t_admit, "t_solve": res.t_solve,
               "t_done": res.t_done, "cus": res.cus,
               "steps": k, "its": list(res.ir.its[:k]), "total_its": res.ir.total_its, "status": res.ir.status,
               "nbe": res.ir.nbe, "error": last_error() if rc < 0 else ""}
        return rc, (x if rc >= 0 else None), rec

    def close(self):
        if getattr(self, "_raw", None) is not None and self._raw.value:
            lib().spai_serve_destroy(self._raw)
            self._raw = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
