"""Thin ctypes binding of the C-ABI library ``libsbs.so`` (include/sbs.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels (the factorisation runs in the library's host code, as in the
paper).  PyTorch provides device memory and the stream handle.  There is no
fallback: if the library is missing or fails to load, every call raises.

The function names are those of the C ABI.  Tensors are torch CUDA tensors;
right-hand sides are C-contiguous (n, m) tensors, which is exactly the
interleaved layout (unknown i of system j at flat index i*m + j).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch  # loads the HIP runtime first, so the library binds to the same one

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbs.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SBS_TRI, SBS_PENTA, SBS_TRI_PERIODIC = 3, 5, 13
SBS_F64, SBS_F32 = 0, 1
SERVE_F32_REFINED, SERVE_F32_FP64_SWEEP = 0, 1  # sbs_server_set_fp32_mode
VARIANT_AUTO, VARIANT_RESIDENT, VARIANT_CHUNKED, VARIANT_STREAM, VARIANT_PARTITION = 0, 1, 2, 3, 4

STATUS = {0: "SBS_OK", 1: "SBS_ERR_INVALID_ARG", 2: "SBS_ERR_ZERO_PIVOT", 3: "SBS_ERR_NONFINITE",
          4: "SBS_ERR_DEVICE", 5: "SBS_ERR_NO_MEMORY", 6: "SBS_ERR_BUDGET", 7: "SBS_ERR_NOT_FOUND",
          8: "SBS_ERR_TIMEOUT", 9: "SBS_ERR_SHUTDOWN"}


class SbsError(RuntimeError):
    def __init__(self, status: int, what: str, bad_row: int = -1):
        self.status = status
        self.name = STATUS.get(status, str(status))
        self.bad_row = bad_row
        msg = f"{what}: {self.name}"
        if bad_row >= 0:
            msg += f" (row {bad_row})"
        super().__init__(msg)


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("in_flight", ctypes.c_uint64),
                ("bytes_reserved", ctypes.c_uint64), ("budget_bytes", ctypes.c_uint64),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("unknowns", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsbs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "sbs_status_str": ([i32], ctypes.c_char_p),
        "sbs_version": ([], ctypes.c_char_p),
        "sbs_factor_shared_lhs": ([i32, i64, vp, P(vp), P(i64)], i32),
        "sbs_factor_uniform": ([i32, i64, vp, P(vp), P(i64)], i32),
        "sbs_solve_batch": ([vp, vp, i64, i32, vp], i32),
        "sbs_solve_batch_variant": ([vp, vp, i64, i32, i32, vp], i32),
        "sbs_auto_variant": ([vp, i64, i32, P(i32)], i32),
        "sbs_solve_batch_partition": ([vp, vp, i64, i32, i32, i32, i32, i32, i32, vp], i32),
        "sbs_partition_shape": ([vp, i64, i32, vp, P(i32), P(i32), P(i32), P(i32)], i32),
        "sbs_solve_batch_refined": ([vp, vp, vp, i64, i32, vp, sz, vp], i32),
        "sbs_refined_workspace_bytes": ([vp, i64], sz),
        "sbs_solve_batch_refined_noalloc": ([vp, vp, vp, i64, i32, vp], i32),
        "sbs_refined_static_scratch_bytes": ([], sz),
        "sbs_cn_step": ([vp, vp, i64, i32, i32, vp], i32),
        "sbs_transpose": ([vp, vp, i64, i64, i32, vp], i32),
        "sbs_adi_step": ([vp, vp, vp, vp, i64, i64, vp], i32),
        "sbs_release": ([vp], i32),
        "sbs_handle_info": ([vp, P(i32), P(i64), P(i64)], i32),
        "sbs_server_create": ([sz, i32, i32, P(vp)], i32),
        "sbs_server_register": ([vp, vp, P(i32)], i32),
        "sbs_server_submit": ([vp, i32, vp, i64, i32, P(ctypes.c_uint64)], i32),
        "sbs_server_wait": ([vp, ctypes.c_uint64, i64, P(vp), P(ctypes.c_double)], i32),
        "sbs_server_release": ([vp, ctypes.c_uint64], i32),
        "sbs_server_fetch": ([vp, ctypes.c_uint64, vp, vp], i32),
        "sbs_server_stats_get": ([vp, P(ServerStats)], i32),
        "sbs_server_set_fp32_mode": ([vp, i32], i32),
        "sbs_server_replay": ([vp, i64, P(i32), P(vp), P(i64), P(i32), P(ctypes.c_double), P(ctypes.c_double),
                               P(ctypes.c_double)], i32),
        "sbs_server_destroy": ([vp], i32),
        "sbs_probe_linear": ([i32, vp, vp, i64, i32, i32, vp], i32),
        "sbs_probe_blocks": ([vp, i64, i64, i32, i32, i32, i32, vp], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)  # AttributeError if the library lacks a declared entry point
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def declared_symbols() -> list[str]:
    """Every function name declared in the headers under include/."""
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if f.endswith(".h"):
            text = open(os.path.join(INCLUDE, f)).read()
            names.update(re.findall(r"^\s*(?:const\s+)?[\w\s\*]+?\b(sbs_\w+)\s*\(", text, re.M))
    return sorted(names)


def _check(st: int, what: str, bad_row: int = -1) -> None:
    if st != 0:
        raise SbsError(st, what, bad_row)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return SBS_F64
    if t.dtype == torch.float32:
        return SBS_F32
    raise TypeError("right-hand sides must be float64 or float32")


def _rhs(t: torch.Tensor, n: int) -> int:
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("right-hand sides must be a contiguous CUDA tensor")
    if t.dim() != 2 or t.shape[0] != n:
        raise ValueError(f"right-hand sides must have shape ({n}, m)")
    return t.data_ptr()


# ---------------------------------------------------------------- C-ABI calls
def sbs_status_str(status: int) -> str:
    return lib().sbs_status_str(status).decode()


def sbs_version() -> str:
    return lib().sbs_version().decode()


def sbs_factor_shared_lhs(kind: int, bands) -> int:
    """Factor once (host, FP64) and upload; returns the handle (an int)."""
    B = np.ascontiguousarray(np.asarray(bands, dtype=np.float64))
    nb = 3 if kind == SBS_TRI_PERIODIC else kind
    if B.ndim != 2 or B.shape[0] != nb:
        raise ValueError(f"bands must have shape ({nb}, n)")
    h = ctypes.c_void_p()
    bad = ctypes.c_int64(-1)
    st = lib().sbs_factor_shared_lhs(kind, B.shape[1], B.ctypes.data, ctypes.byref(h), ctypes.byref(bad))
    _check(st, "sbs_factor_shared_lhs", bad.value)
    return h.value


def sbs_factor_uniform(kind: int, n: int, coeffs) -> int:
    """Factor a matrix with constant bands (one coefficient per band)."""
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    nb = 3 if kind == SBS_TRI_PERIODIC else kind
    if c.shape != (nb,):
        raise ValueError(f"coeffs must have {nb} entries")
    h = ctypes.c_void_p()
    bad = ctypes.c_int64(-1)
    _check(lib().sbs_factor_uniform(kind, n, c.ctypes.data, ctypes.byref(h), ctypes.byref(bad)),
           "sbs_factor_uniform", bad.value)
    return h.value


def sbs_release(h: int) -> None:
    _check(lib().sbs_release(h), "sbs_release")


def sbs_handle_info(h: int):
    k, n, b = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().sbs_handle_info(h, ctypes.byref(k), ctypes.byref(n), ctypes.byref(b)), "sbs_handle_info")
    return k.value, n.value, b.value


def sbs_solve_batch(h: int, rhs: torch.Tensor, stream=None) -> torch.Tensor:
    """Solve in place; rhs is a contiguous CUDA (n, m) float64/float32 tensor."""
    _, n, _ = sbs_handle_info(h)
    p = _rhs(rhs, n)
    _check(lib().sbs_solve_batch(h, p, rhs.shape[1], _dtype_code(rhs), _stream(stream)), "sbs_solve_batch")
    return rhs


def sbs_solve_batch_variant(h: int, rhs: torch.Tensor, variant: int, stream=None, n: int = None) -> torch.Tensor:
    """`n`: the handle's row count when the caller knows it (saves a query)."""
    if n is None:
        _, n, _ = sbs_handle_info(h)
    p = _rhs(rhs, n)
    _check(lib().sbs_solve_batch_variant(h, p, rhs.shape[1], _dtype_code(rhs), variant, _stream(stream)),
           "sbs_solve_batch_variant")
    return rhs


def sbs_auto_variant(h: int, m: int, dtype: int = SBS_F64) -> int:
    """The SBS_VARIANT_* that SBS_VARIANT_AUTO runs for m systems."""
    v = ctypes.c_int32()
    _check(lib().sbs_auto_variant(h, m, dtype, ctypes.byref(v)), "sbs_auto_variant")
    return v.value


def sbs_solve_batch_partition(h: int, rhs: torch.Tensor, form: int, lb: int, vec: int, S: int, flags: int = 0,
                              stream=None) -> torch.Tensor:
    """In-place partitioned solve with an explicit shape (form 0 pair, 1 separator)."""
    _, n, _ = sbs_handle_info(h)
    p = _rhs(rhs, n)
    _check(lib().sbs_solve_batch_partition(h, p, rhs.shape[1], _dtype_code(rhs), form, lb, vec, S, flags,
                                           _stream(stream)), "sbs_solve_batch_partition")
    return rhs


def sbs_partition_shape(h: int, rhs: torch.Tensor):
    """(form, lb, vec, S) of the partitioned shape AUTO runs for rhs, or None."""
    _, n, _ = sbs_handle_info(h)
    out = [ctypes.c_int32() for _ in range(4)]
    st = lib().sbs_partition_shape(h, rhs.shape[1], _dtype_code(rhs), rhs.data_ptr(), *[ctypes.byref(o) for o in out])
    if st == 7:
        return None
    _check(st, "sbs_partition_shape")
    return tuple(o.value for o in out)


def sbs_refined_workspace_bytes(h: int, m: int) -> int:
    return int(lib().sbs_refined_workspace_bytes(h, m))


def sbs_solve_batch_refined(h: int, b: torch.Tensor, x: torch.Tensor | None = None, sweeps: int = 2,
                            work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """FP32 right-hand sides b (n, m) -> FP64 solution x (n, m)."""
    _, n, _ = sbs_handle_info(h)
    if b.dtype != torch.float32:
        raise TypeError("b must be float32")
    p = _rhs(b, n)
    m = b.shape[1]
    if x is None:
        x = torch.empty((n, m), dtype=torch.float64, device=b.device)
    if x.dtype != torch.float64 or x.shape != b.shape:
        raise TypeError("x must be float64 with the shape of b")
    need = sbs_refined_workspace_bytes(h, m)
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=b.device)
    _check(lib().sbs_solve_batch_refined(h, p, _rhs(x, n), m, sweeps, work.data_ptr(),
                                         work.numel() * work.element_size(), _stream(stream)),
           "sbs_solve_batch_refined")
    return x


def sbs_refined_static_scratch_bytes() -> int:
    return int(lib().sbs_refined_static_scratch_bytes())


def sbs_solve_batch_refined_noalloc(h: int, b: torch.Tensor, x: torch.Tensor, sweeps: int = 2,
                                    stream=None) -> torch.Tensor:
    """sbs_solve_batch_refined with the library's static scratch: the caller
    passes b (n, m) FP32 and x (n, m) FP64, nothing is allocated."""
    _, n, _ = sbs_handle_info(h)
    if b.dtype != torch.float32 or x.dtype != torch.float64 or x.shape != b.shape:
        raise TypeError("b must be float32 and x float64 of the same shape")
    _check(lib().sbs_solve_batch_refined_noalloc(h, _rhs(b, n), _rhs(x, n), b.shape[1], sweeps, _stream(stream)),
           "sbs_solve_batch_refined_noalloc")
    return x


def sbs_cn_step(h: int, c: torch.Tensor, steps: int = 1, stream=None) -> torch.Tensor:
    """Crank-Nicolson steps in place: c <- A^{-1} (2I - A) c, `steps` times."""
    _, n, _ = sbs_handle_info(h)
    p = _rhs(c, n)
    _check(lib().sbs_cn_step(h, p, c.shape[1], _dtype_code(c), steps, _stream(stream)), "sbs_cn_step")
    return c


def sbs_transpose(src: torch.Tensor, dst: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    if src.dim() != 2 or not (src.is_cuda and src.is_contiguous()):
        raise ValueError("src must be a contiguous 2-D CUDA tensor")
    rows, cols = src.shape
    if dst is None:
        dst = torch.empty((cols, rows), dtype=src.dtype, device=src.device)
    if dst.shape != (cols, rows) or dst.dtype != src.dtype or not dst.is_contiguous():
        raise ValueError("dst must be a contiguous (cols, rows) tensor of src's dtype")
    _check(lib().sbs_transpose(src.data_ptr(), dst.data_ptr(), rows, cols, _dtype_code(src), _stream(stream)),
           "sbs_transpose")
    return dst


def sbs_adi_step(hy: int, hx: int, grid: torch.Tensor, work: torch.Tensor, stream=None) -> torch.Tensor:
    if grid.dtype != torch.float64 or grid.dim() != 2 or not grid.is_contiguous():
        raise ValueError("grid must be a contiguous (ny, nx) float64 tensor")
    ny, nx = grid.shape
    if work.numel() < ny * nx or work.dtype != torch.float64:
        raise ValueError("work must hold ny*nx float64 values")
    _check(lib().sbs_adi_step(hy, hx, grid.data_ptr(), work.data_ptr(), ny, nx, _stream(stream)), "sbs_adi_step")
    return grid


def sbs_server_replay(srv, lhs_ids, rhs_ptrs, m, dtype, arrival_us=None):
    """sbs_server_replay over numpy arrays (one entry per request): returns
    (status, latency_us array, elapsed seconds).  srv is the server pointer
    (ctypes.c_void_p); rhs_ptrs are device addresses."""
    import numpy as np
    n = len(lhs_ids)
    ids = np.ascontiguousarray(lhs_ids, dtype=np.int32)
    ptrs = (ctypes.c_void_p * max(n, 1))(*[int(p) for p in rhs_ptrs])
    ms = np.ascontiguousarray(m, dtype=np.int64)
    dts = np.ascontiguousarray(dtype, dtype=np.int32)
    arr = None if arrival_us is None else np.ascontiguousarray(arrival_us, dtype=np.float64)
    lat = np.empty(max(n, 1), dtype=np.float64)
    el = ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib().sbs_server_replay(
        srv, n, ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ptrs,
        ms.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), dts.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        None if arr is None else arr.ctypes.data_as(dp), lat.ctypes.data_as(dp), ctypes.byref(el))
    return st, lat[:n], el.value


class SharedLhs:
    """Owns a factored shared matrix (releases it when closed)."""

    def __init__(self, kind: int, bands):
        self.kind = kind
        self.handle = sbs_factor_shared_lhs(kind, bands)
        _, self.n, self.device_bytes = sbs_handle_info(self.handle)

    def solve(self, rhs: torch.Tensor, variant: int = VARIANT_AUTO, stream=None) -> torch.Tensor:
        return sbs_solve_batch_variant(self.handle, rhs, variant, stream, n=self.n)

    def cn_step(self, c: torch.Tensor, steps: int = 1, stream=None) -> torch.Tensor:
        return sbs_cn_step(self.handle, c, steps, stream)

    def solve_refined(self, b: torch.Tensor, sweeps: int = 2, **kw) -> torch.Tensor:
        return sbs_solve_batch_refined(self.handle, b, sweeps=sweeps, **kw)

    def close(self) -> None:
        if self.handle:
            sbs_release(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
