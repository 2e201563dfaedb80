"""Oracle for shared-LHS batched tridiagonal / pentadiagonal solves.

TEST INFRASTRUCTURE ONLY.  Plain serial FP64 CPU implementation of what the
GPU library computes (arXiv:1909.04539, Sections 3.1 and 4.1), written in C
(``sbs_oracle.c``, compiled with gcc -O2 -ffp-contract=off) with a numpy twin
(``twin.py``).  Only the tests, the smoke check and the benchmark's CPU-baseline
leg may import this package.  It imports nothing from the GPU library and
shares no code with it.

Interface: bands are given as one float64 array of shape (bands, n), band-major
and row-aligned -- band k, entry i is the coefficient in row i (tri: a, b, c;
penta: a, b, c, d, e), exactly as the library's factor call takes them.  RHS
arrays are interleaved: shape (n, m), unknown i of system j at [i, j].
Kinds: 3 tridiagonal, 5 pentadiagonal, TRI_PERIODIC (13) tridiagonal with
periodic wrap (Section 3.3; three bands, a_0 and c_{n-1} are the corners).

Parity pins: none of these functions is trusted on its own; ``tests/
test_oracle_pins.py`` checks them against dense LU, closed forms, banded LAPACK,
a manufactured solution, the DST-I diagonalisation and the numpy twin.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .twin import PivotError  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

TRI_PERIODIC = 13

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
             "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        lib.oracle_tri_factor.argtypes = [i64, dp, dp, dp, dp, dp]
        lib.oracle_tri_factor.restype = i64
        lib.oracle_tri_solve.argtypes = [i64, i64, i64, dp, dp, dp, dp]
        lib.oracle_tri_solve.restype = i64
        lib.oracle_penta_factor.argtypes = [i64, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
        lib.oracle_penta_factor.restype = i64
        lib.oracle_penta_solve.argtypes = [i64, i64, i64, dp, dp, dp, dp, dp, dp]
        lib.oracle_penta_solve.restype = i64
        lib.oracle_tri_periodic_solve.argtypes = [i64, i64, i64, dp, dp, dp, dp]
        lib.oracle_tri_periodic_solve.restype = i64
        lib.oracle_cn_steps.argtypes = [ctypes.c_int, i64, i64, dp, dp, ctypes.c_int]
        lib.oracle_cn_steps.restype = i64
        lib.oracle_adi_step.argtypes = [i64, i64, dp, dp, dp, dp, dp, dp, dp]
        lib.oracle_adi_step.restype = i64
        lib.oracle_tri_solve_mt.argtypes = [i64, i64, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_tri_solve_mt.restype = i64
        lib.oracle_penta_solve_mt.argtypes = [i64, i64, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        lib.oracle_penta_solve_mt.restype = i64
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _bands(bands, kind: int):
    nb = 3 if kind == TRI_PERIODIC else kind
    B = np.ascontiguousarray(np.asarray(bands, dtype=np.float64))
    if B.ndim != 2 or B.shape[0] != nb:
        raise ValueError(f"bands must have shape ({nb}, n)")
    return [np.ascontiguousarray(B[k]) for k in range(nb)]


def _raise(bad: int) -> None:
    if bad >= 0:
        raise PivotError(int(bad))


def tri_factor(bands):
    """Return (den, chat) of the Section 3.1 pre-factorisation."""
    a, b, c = _bands(bands, 3)
    n = len(b)
    den, chat = np.zeros(n), np.zeros(n)
    _raise(_load().oracle_tri_factor(n, _p(a), _p(b), _p(c), _p(den), _p(chat)))
    return den, chat


def penta_factor(bands):
    """Return dict(alpha, beta, gamma, delta, eps) of the Section 4.1 A = L R."""
    a, b, c, d, e = _bands(bands, 5)
    n = len(c)
    out = {k: np.zeros(n) for k in ("alpha", "beta", "gamma", "delta", "eps")}
    _raise(_load().oracle_penta_factor(n, _p(a), _p(b), _p(c), _p(d), _p(e),
                                       *(_p(out[k]) for k in ("alpha", "beta", "gamma", "delta", "eps"))))
    return out


def solve(kind: int, bands, rhs) -> np.ndarray:
    """x = A^{-1} rhs for every interleaved column; rhs shape (n, m).  Serial."""
    X = np.array(rhs, dtype=np.float64, order="C", copy=True)
    if X.ndim == 1:
        X = X[:, None]
    n, m = X.shape
    if kind == 3:
        a, b, c = _bands(bands, 3)
        _raise(_load().oracle_tri_solve(n, m, m, _p(a), _p(b), _p(c), _p(X)))
    elif kind == 5:
        a, b, c, d, e = _bands(bands, 5)
        _raise(_load().oracle_penta_solve(n, m, m, _p(a), _p(b), _p(c), _p(d), _p(e), _p(X)))
    elif kind == TRI_PERIODIC:
        if n < 3:
            raise ValueError("a periodic system needs n >= 3")
        a, b, c = _bands(bands, kind)
        _raise(_load().oracle_tri_periodic_solve(n, m, m, _p(a), _p(b), _p(c), _p(X)))
    else:
        raise ValueError("kind must be 3 (tri), 5 (penta) or 13 (periodic tri)")
    return X


def solve_inplace_mt(kind: int, bands, X: np.ndarray, nthreads: int = 0) -> None:
    """Same arithmetic as solve(), column blocks spread over OpenMP threads."""
    assert X.dtype == np.float64 and X.flags.c_contiguous and X.ndim == 2
    n, m = X.shape
    if kind == 3:
        a, b, c = _bands(bands, 3)
        _raise(_load().oracle_tri_solve_mt(n, m, _p(a), _p(b), _p(c), _p(X), nthreads))
    else:
        a, b, c, d, e = _bands(bands, 5)
        _raise(_load().oracle_penta_solve_mt(n, m, _p(a), _p(b), _p(c), _p(d), _p(e), _p(X), nthreads))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def adi_step(bands_y, bands_x, grid) -> np.ndarray:
    """One ADI step on a row-major (ny, nx) grid: tri solve along y for every
    column, then along x for every row (rows walked directly, no transpose)."""
    G = np.array(grid, dtype=np.float64, order="C", copy=True)
    ny, nx = G.shape
    ay, by, cy = _bands(bands_y, 3)
    ax, bx, cx = _bands(bands_x, 3)
    if len(by) != ny or len(bx) != nx:
        raise ValueError("band lengths must match the grid")
    _raise(_load().oracle_adi_step(ny, nx, _p(ay), _p(by), _p(cy), _p(ax), _p(bx), _p(cx), _p(G)))
    return G


def cn_steps(kind: int, bands, C, steps: int = 1) -> np.ndarray:
    """Crank-Nicolson steps A C^{n+1} = (2I - A) C^n (Sections 3.2, 4.2)."""
    X = np.array(C, dtype=np.float64, order="C", copy=True)
    n, m = X.shape
    B = np.ascontiguousarray(np.stack(_bands(bands, kind)))
    if kind == TRI_PERIODIC and n < 3:
        raise ValueError("a periodic system needs n >= 3")
    _raise(_load().oracle_cn_steps(kind, n, m, _p(B), _p(X), steps))
    return X


def twin_cn_steps(kind: int, bands, C, steps: int = 1) -> np.ndarray:
    from . import twin
    return twin.cn_steps(kind, np.stack(_bands(bands, kind)), C, steps)


def refine_reference(kind: int, bands, b32: np.ndarray) -> np.ndarray:
    """Reference for the mixed-precision form: the FP64 solve of the exact
    FP64 promotion of the stored FP32 right-hand sides."""
    return solve(kind, bands, np.asarray(b32, dtype=np.float32).astype(np.float64))


def twin_solve(kind: int, bands, rhs) -> np.ndarray:
    """The numpy twin of solve() (bit-identical by construction)."""
    from . import twin
    X = np.asarray(rhs, dtype=np.float64)
    if kind == 3:
        return twin.tri_solve(*_bands(bands, 3), X)
    if kind == TRI_PERIODIC:
        return twin.tri_periodic_solve(*_bands(bands, kind), X)
    return twin.penta_solve(*_bands(bands, 5), X)
