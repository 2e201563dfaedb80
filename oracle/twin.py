"""Numpy twin of the C oracle (TEST INFRASTRUCTURE ONLY).

A second, independent transcription of the same recurrences as
``sbs_oracle.c``: each row of the interleaved (n, m) array is one numpy
expression, evaluated with the same IEEE operations in the same order (a
product, then a difference, then a true division; numpy never fuses a
multiply into an add).  The C oracle and this twin must therefore agree bit
for bit, which pins each against transcription slips in the other.

Band convention and out-of-matrix coefficients are as in the C file:
tridiagonal row i is a_i x_{i-1} + b_i x_i + c_i x_{i+1}; pentadiagonal row i
is a_i x_{i-2} + b_i x_{i-1} + c_i x_i + d_i x_{i+1} + e_i x_{i+2}.
"""
from __future__ import annotations

import numpy as np


class PivotError(ArithmeticError):
    """A zero or non-finite pivot at ``row`` (0-based)."""

    def __init__(self, row: int):
        super().__init__(f"zero or non-finite pivot at row {row}")
        self.row = row


def _check(p: float, i: int) -> None:
    if not (np.isfinite(p) and p != 0.0):
        raise PivotError(i)


def tri_factor(a, b, c):
    """Section 3.1 pre-factorisation: returns (den, chat) with
    den_0 = b_0, den_i = b_i - a_i chat_{i-1}, chat_i = c_i / den_i and
    chat_{n-1} = 0 (c_{n-1} is outside the matrix)."""
    n = len(b)
    den = np.zeros(n)
    chat = np.zeros(n)
    den[0] = b[0]
    _check(den[0], 0)
    chat[0] = c[0] / den[0] if n > 1 else 0.0
    for i in range(1, n):
        den[i] = b[i] - a[i] * chat[i - 1]
        _check(den[i], i)
        chat[i] = c[i] / den[i] if i < n - 1 else 0.0
    return den, chat


def tri_solve(a, b, c, d):
    """Section 3.1 forward and backward sweeps over interleaved d (n, m)."""
    den, chat = tri_factor(a, b, c)
    x = np.array(d, dtype=np.float64, copy=True)
    n = x.shape[0]
    x[0] = x[0] / den[0]
    for i in range(1, n):
        x[i] = (x[i] - a[i] * x[i - 1]) / den[i]
    for i in range(n - 2, -1, -1):
        x[i] = x[i] - chat[i] * x[i + 1]
    return x


def penta_factor(a, b, c, d, e):
    """Section 4.1 factorisation A = L R with all out-of-matrix terms 0.
    Returns a dict of the five factor vectors."""
    n = len(c)
    al, be, ga, de, ep = (np.zeros(n) for _ in range(5))
    for i in range(n):
        ai = a[i] if i >= 2 else 0.0
        bi = b[i] if i >= 1 else 0.0
        di = d[i] if i <= n - 2 else 0.0
        ei = e[i] if i <= n - 3 else 0.0
        gm2 = ga[i - 2] if i >= 2 else 0.0
        gm1 = ga[i - 1] if i >= 1 else 0.0
        dm2 = de[i - 2] if i >= 2 else 0.0
        dm1 = de[i - 1] if i >= 1 else 0.0
        be[i] = bi - ai * gm2
        al[i] = c[i] - ai * dm2 - be[i] * gm1
        _check(al[i], i)
        ga[i] = (di - be[i] * dm1) / al[i]
        de[i] = ei / al[i]
        ep[i] = ai
    return {"alpha": al, "beta": be, "gamma": ga, "delta": de, "eps": ep}


def penta_solve(a, b, c, d, e, f):
    """Section 4.1: L g = f forward, then R x = g backward, interleaved (n, m)."""
    F = penta_factor(a, b, c, d, e)
    al, be, ga, de, ep = F["alpha"], F["beta"], F["gamma"], F["delta"], F["eps"]
    x = np.array(f, dtype=np.float64, copy=True)
    n = x.shape[0]
    zero = np.zeros_like(x[0])
    for i in range(n):
        g2 = x[i - 2] if i >= 2 else zero
        g1 = x[i - 1] if i >= 1 else zero
        x[i] = (x[i] - ep[i] * g2 - be[i] * g1) / al[i]
    for i in range(n - 1, -1, -1):
        x1 = x[i + 1] if i + 1 < n else zero
        x2 = x[i + 2] if i + 2 < n else zero
        x[i] = x[i] - ga[i] * x1 - de[i] * x2
    return x


def tri_periodic_solve(a, b, c, d):
    """Section 3.3: periodic tridiagonal (corners a_0 top-right, c_{n-1}
    bottom-left) by Sherman-Morrison.  A = A' + u v^T with
    u = (-b_0, 0.., c_{n-1}), v = (1, 0.., -a_0/b_0); A' is tridiagonal with
    A'_00 = 2 b_0 and A'_{n-1,n-1} = b_{n-1} + a_0 c_{n-1} / b_0; then
    y = A'^{-1} d, z = A'^{-1} u and x = y - ((v.y) / (1 + v.z)) z.
    Raises PivotError(n) when 1 + v.z is zero or not finite."""
    n = len(b)
    if n < 3:
        raise ValueError("a periodic system needs n >= 3")
    vlast = -a[0] / b[0]
    bp = np.array(b, dtype=np.float64, copy=True)
    bp[0] = b[0] + b[0]
    bp[n - 1] = b[n - 1] + a[0] * c[n - 1] / b[0]
    u = np.zeros((n, 1))
    u[0, 0] = -b[0]
    u[n - 1, 0] = c[n - 1]
    z = tri_solve(a, bp, c, u)[:, 0]
    vz1 = 1.0 + (z[0] + vlast * z[n - 1])
    _check(vz1, n)
    y = tri_solve(a, bp, c, d)
    s = (y[0] + vlast * y[n - 1]) / vz1
    return y - s * z[:, None]


def cn_steps(kind, bands, C, steps=1):
    """Sections 3.2 / 4.2: Crank-Nicolson steps A C^{n+1} = (2I - A) C^n with
    f_i = 2 C_i - (A C)_i summed over the bands left to right (terms outside
    the matrix zero; wrapped for kind 13), then the solve."""
    B = np.asarray(bands, dtype=np.float64)
    nb = B.shape[0]
    h = nb // 2
    X = np.array(C, dtype=np.float64, copy=True)
    n = X.shape[0]
    for _ in range(steps):
        F = np.empty_like(X)
        for i in range(n):
            ac = np.zeros_like(X[0])
            for k in range(nb):
                col = i + k - h
                if kind == 13:
                    col %= n
                elif col < 0 or col >= n:
                    continue
                ac = ac + B[k, i] * X[col]
            F[i] = 2.0 * X[i] - ac
        if kind == 3:
            X = tri_solve(*B, F)
        elif kind == 5:
            X = penta_solve(*B, F)
        else:
            X = tri_periodic_solve(*B, F)
    return X
