"""Seeded synthetic inputs for the shared-LHS batched solver workloads.

This module only draws numbers and lays them out; it holds none of the
solver's arithmetic and imports neither the GPU library nor the oracle, so
both sides of every parity test can take their inputs from it.

Layouts
-------
* bands: float64 array of shape (kind, n), band-major and row-aligned (band k,
  entry i is the coefficient of row i).  Tri: (a, b, c) with row i reading
  a_i x_{i-1} + b_i x_i + c_i x_{i+1}; penta: (a, b, c, d, e) with row i
  reading a_i x_{i-2} + b_i x_{i-1} + c_i x_i + d_i x_{i+1} + e_i x_{i+2}.
  Entries that fall outside the matrix are set to 0 here (the solvers ignore
  them either way).
* rhs: C-ordered (n, m) array; row-major order *is* the interleaved layout of
  the paper's Section 2 (unknown i of system j at flat index i*m + j).

Workloads (all seed 0 by default, numpy PCG64 ``default_rng``, draws in the
order written):
  0  tridiagonal FP64, n=256, m=1024, strictly diagonally dominant
  1  pentadiagonal FP64, n=1024, m=65536, 1-D hyperdiffusion Crank--Nicolson
     matrix (Section 4.2) with s=0.5 and truncated ends; rhs = A x_true
  2  2-D ADI step, 2048 x 2048 FP64 grid, A = I + r(-1, 2, -1), r = 0.5
     (Section 3.2's diffusion matrix), smooth field of 8 Fourier modes + noise
  3  mixed precision: tridiagonal n=512, m=2^20, weaker dominance, rhs stored
     as FP32
  4  serving trace: 64 shared matrices, Poisson arrivals, 1e5 requests
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TRI, PENTA = 3, 5

FULL_SIZES = {
    0: dict(n=256, m=1024),
    1: dict(n=1024, m=65536),
    2: dict(n=2048, m=2048),
    3: dict(n=512, m=1 << 20),
}


def tri_dominant_bands(rng: np.random.Generator, n: int, margin=(1.0, 2.0)) -> np.ndarray:
    """a, c ~ U[-1, 1]; a_0 = c_{n-1} = 0 (outside the matrix); then
    b = |a| + |c| + U[margin] so every row is strictly diagonally dominant."""
    a = rng.uniform(-1.0, 1.0, n)
    c = rng.uniform(-1.0, 1.0, n)
    a[0] = 0.0
    c[n - 1] = 0.0
    b = np.abs(a) + np.abs(c) + rng.uniform(margin[0], margin[1], n)
    return np.stack([a, b, c])


def hyperdiffusion_bands(n: int, s: float) -> np.ndarray:
    """Crank--Nicolson matrix of the 1-D hyperdiffusion step (Section 4.2):
    bands (s, -4s, 1+6s, -4s, s), out-of-range stencil entries dropped."""
    B = np.empty((PENTA, n))
    B[0], B[1], B[2], B[3], B[4] = s, -4.0 * s, 1.0 + 6.0 * s, -4.0 * s, s
    zero_outside(B)
    return B


def diffusion_bands(n: int, r: float) -> np.ndarray:
    """Crank--Nicolson matrix of the 1-D diffusion step (Section 3.2):
    bands (-r, 1+2r, -r), Dirichlet-truncated (no wrap-around)."""
    B = np.empty((TRI, n))
    B[0], B[1], B[2] = -r, 1.0 + 2.0 * r, -r
    zero_outside(B)
    return B


def zero_outside(B: np.ndarray) -> np.ndarray:
    """Set the coefficients that lie outside an n x n banded matrix to 0."""
    kind, n = B.shape
    if kind == TRI:
        B[0, 0] = 0.0
        B[2, n - 1] = 0.0
    else:
        B[0, :2] = 0.0
        B[1, :1] = 0.0
        B[3, n - 1:] = 0.0
        B[4, max(n - 2, 0):] = 0.0
    return B


def banded_matvec(B: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A x for a manufactured right-hand side (input construction only).
    Row sums are accumulated left to right over the band columns."""
    kind, n = B.shape
    h = kind // 2
    y = np.zeros_like(x, dtype=np.float64)
    for k in range(kind):
        off = k - h                        # column offset of band k
        lo, hi = max(0, -off), min(n, n - off)
        if hi <= lo:
            continue
        y[lo:hi] += B[k, lo:hi, None] * x[lo + off:hi + off]
    return y


def uniform_rows(rng: np.random.Generator, n: int, m: int, dtype=np.float64,
                 block_rows: int = 32) -> np.ndarray:
    """U[-1, 1] values of a C-ordered (n, m) array, drawn row block by row
    block (the same stream as one (n, m) draw) and stored as ``dtype``."""
    out = np.empty((n, m), dtype=dtype)
    for r0 in range(0, n, block_rows):
        r1 = min(n, r0 + block_rows)
        out[r0:r1] = rng.uniform(-1.0, 1.0, (r1 - r0, m))
    return out


@dataclass
class Workload:
    name: str
    kind: int
    bands: np.ndarray
    rhs: np.ndarray
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.bands.shape[1]

    @property
    def m(self) -> int:
        return self.rhs.shape[1]


def config0(seed: int = 0, n: int = 256, m: int = 1024) -> Workload:
    rng = np.random.default_rng(seed)
    B = tri_dominant_bands(rng, n, (1.0, 2.0))
    rhs = uniform_rows(rng, n, m)
    return Workload(f"tri_f64_n{n}_m{m}", TRI, B, rhs)


def config1(seed: int = 0, n: int = 1024, m: int = 65536, s: float = 0.5) -> Workload:
    rng = np.random.default_rng(seed)
    B = hyperdiffusion_bands(n, s)
    x_true = rng.standard_normal((n, m))
    rhs = banded_matvec(B, x_true)
    return Workload(f"penta_f64_n{n}_m{m}", PENTA, B, rhs, {"x_true": x_true})


def adi_field(rng: np.random.Generator, ny: int, nx: int, modes: int = 8) -> np.ndarray:
    """Sum of ``modes`` random Fourier modes plus 1e-3 Gaussian noise on a
    row-major (ny, nx) grid, F[y, x]."""
    k = rng.integers(1, 17, modes)
    l = rng.integers(1, 17, modes)
    A = rng.uniform(0.5, 1.5, modes)
    phi = rng.uniform(0.0, 2.0 * math.pi, modes)
    xs = np.arange(nx, dtype=np.float64)[None, :]
    ys = np.arange(ny, dtype=np.float64)[:, None]
    F = np.zeros((ny, nx))
    for q in range(modes):
        F += A[q] * np.sin(2.0 * math.pi * (k[q] * xs / nx + l[q] * ys / ny) + phi[q])
    F += 1e-3 * rng.standard_normal((ny, nx))
    return F


def config2(seed: int = 0, ny: int = 2048, nx: int = 2048, r: float = 0.5) -> Workload:
    rng = np.random.default_rng(seed)
    F = adi_field(rng, ny, nx)
    return Workload(f"adi_f64_{ny}x{nx}", TRI, diffusion_bands(ny, r), F,
                    {"bands_x": diffusion_bands(nx, r), "r": r})


def config3(seed: int = 0, n: int = 512, m: int = 1 << 20) -> Workload:
    rng = np.random.default_rng(seed)
    B = tri_dominant_bands(rng, n, (0.05, 0.5))
    b32 = uniform_rows(rng, n, m, dtype=np.float32)
    return Workload(f"tri_refine_f32in_n{n}_m{m}", TRI, B, b32)


def make_config(k: int, seed: int = 0, **sizes) -> Workload:
    return {0: config0, 1: config1, 2: config2, 3: config3}[k](seed=seed, **sizes)


# ---------------------------------------------------------------------------
# Serving trace (workload 4)

@dataclass
class Lhs:
    kind: int
    bands: np.ndarray

    @property
    def n(self) -> int:
        return self.bands.shape[1]


@dataclass
class Request:
    rid: int
    t_arrival: float          # seconds from the start of the trace
    lhs: int
    m: int
    fp32: bool


def serving_lhs_set(seed: int = 0, count: int = 64, n_lo: int = 64, n_hi: int = 8192):
    """``count`` shared matrices: the first half tridiagonal (workload-0
    recipe), the rest pentadiagonal hyperdiffusion with s ~ U[0.1, 1];
    n log-uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng([seed, 4, 0])
    out = []
    for q in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        if q < count // 2:
            out.append(Lhs(TRI, tri_dominant_bands(rng, n, (1.0, 2.0))))
        else:
            out.append(Lhs(PENTA, hyperdiffusion_bands(n, float(rng.uniform(0.1, 1.0)))))
    return out


def serving_trace(rate_hz: float, count: int = 100_000, seed: int = 0, n_lhs: int = 64,
                  m_max: int = 4096):
    """Poisson arrivals at ``rate_hz``; lhs uniform; m log-uniform in
    [1, m_max]; FP32 or FP64 with probability 1/2 each."""
    rng = np.random.default_rng([seed, 4, 1])
    gaps = rng.exponential(1.0 / rate_hz, count)
    t = np.cumsum(gaps) - gaps[0]
    lhs = rng.integers(0, n_lhs, count)
    m = np.rint(np.exp(rng.uniform(0.0, math.log(m_max), count))).astype(np.int64)
    m = np.maximum(m, 1)
    fp32 = rng.random(count) < 0.5
    return [Request(i, float(t[i]), int(lhs[i]), int(m[i]), bool(fp32[i])) for i in range(count)]


def request_rhs(req: Request, n: int, seed: int = 0) -> np.ndarray:
    """The request's right-hand sides, U[-1, 1], interleaved (n, m)."""
    rng = np.random.default_rng([seed, 4, 2, req.rid])
    x = rng.uniform(-1.0, 1.0, (n, req.m))
    return x.astype(np.float32) if req.fp32 else x
