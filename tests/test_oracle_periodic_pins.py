"""Pins for the periodic tridiagonal oracle (Section 3.3, Sherman-Morrison),
CPU only.  The oracle is checked against a dense solve of the periodic matrix
built entry by entry, the FFT diagonalisation of circulant matrices (the
paper's constant-coefficient Crank-Nicolson benchmark is circulant), the
plain tridiagonal oracle when the corners vanish, the backward error and its
numpy twin; planted mistakes in a copy of the algorithm must fail the dense
pin."""
import numpy as np
import pytest

import oracle
from oracle import twin

P = oracle.TRI_PERIODIC


def dense_periodic(B):
    """Row i: a_i at column (i-1) mod n, b_i at i, c_i at (i+1) mod n."""
    a, b, c = B
    n = len(b)
    A = np.zeros((n, n))
    for i in range(n):
        A[i, (i - 1) % n] += a[i]
        A[i, i] += b[i]
        A[i, (i + 1) % n] += c[i]
    return A


def colrel(x, ref):
    num = np.max(np.abs(x - ref), axis=0)
    den = np.maximum(np.max(np.abs(ref), axis=0), np.finfo(float).tiny)
    return float(np.max(num / den))


def random_periodic(rng, n, margin=(1.0, 2.0)):
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    b = np.abs(a) + np.abs(c) + rng.uniform(*margin, n)
    return np.stack([a, b, c])


@pytest.mark.parametrize("n", list(range(3, 21)) + [31, 64, 100])
def test_periodic_matches_dense_lu(n):
    rng = np.random.default_rng(700 + n)
    B = random_periodic(rng, n)
    d = rng.uniform(-1, 1, (n, 5))
    ref = np.linalg.solve(dense_periodic(B), d)
    assert colrel(oracle.solve(P, B, d), ref) <= 1e-14


@pytest.mark.parametrize("n", [3, 8, 64, 257])
@pytest.mark.parametrize("abc", [(-0.1, 1.2, -0.1), (-1.0, 3.0, -1.0), (-50.0, 101.0, -50.0), (0.3, -2.0, 0.9)])
def test_circulant_matches_fft_diagonalisation(n, abc):
    # Constant bands make the periodic matrix circulant: its eigenvectors are
    # the Fourier modes, with eigenvalue b + c e^{2 pi i k/n} + a e^{-2 pi i k/n}.
    a, b, c = abc
    B = np.stack([np.full(n, a), np.full(n, b), np.full(n, c)])
    d = np.random.default_rng(n).uniform(-1, 1, (n, 6))
    k = np.arange(n)
    lam = b + c * np.exp(2j * np.pi * k / n) + a * np.exp(-2j * np.pi * k / n)
    ref = np.real(np.fft.ifft(np.fft.fft(d, axis=0) / lam[:, None], axis=0))
    kappa = np.max(np.abs(lam)) / np.min(np.abs(lam))
    assert colrel(oracle.solve(P, B, d), ref) <= 20 * kappa * np.finfo(float).eps


def test_paper_crank_nicolson_bands_are_circulant():
    # The benchmark matrix of Section 3.2: a = c = -sigma, b = 1 + 2 sigma.
    n, sigma = 128, 0.5 * 1e-3 * 128 ** 2
    B = np.stack([np.full(n, -sigma), np.full(n, 1 + 2 * sigma), np.full(n, -sigma)])
    x_true = np.random.default_rng(1).standard_normal((n, 4))
    d = dense_periodic(B) @ x_true
    assert colrel(oracle.solve(P, B, d), x_true) <= 1e-13


@pytest.mark.parametrize("n", [3, 10, 64])
def test_without_corners_equals_plain_tridiagonal(n):
    rng = np.random.default_rng(n)
    B = random_periodic(rng, n)
    B[0, 0] = 0.0
    B[2, n - 1] = 0.0
    d = rng.uniform(-1, 1, (n, 3))
    assert colrel(oracle.solve(P, B, d), oracle.solve(3, B, d)) <= 1e-15


@pytest.mark.parametrize("n", [3, 33, 500])
def test_backward_error(n):
    rng = np.random.default_rng(n + 1)
    B = random_periodic(rng, n, (0.05, 0.5))
    d = rng.uniform(-1, 1, (n, 8))
    x = oracle.solve(P, B, d)
    A = dense_periodic(B)
    r = np.max(np.abs(d - A @ x), axis=0)
    scale = np.max(np.sum(np.abs(A), axis=1)) * np.max(np.abs(x), axis=0) + np.max(np.abs(d), axis=0)
    assert np.max(r / scale) <= 1e-15


@pytest.mark.parametrize("n,m", [(3, 1), (7, 5), (130, 33)])
def test_c_oracle_and_twin_bit_identical(n, m):
    rng = np.random.default_rng(n * m)
    B = random_periodic(rng, n)
    d = rng.uniform(-1, 1, (n, m))
    assert np.array_equal(oracle.solve(P, B, d), oracle.twin_solve(P, B, d))


def test_rejects_short_and_reports_bad_pivot():
    with pytest.raises(ValueError):
        oracle.solve(P, np.ones((3, 2)), np.ones((2, 1)))
    B = random_periodic(np.random.default_rng(3), 6)
    B[1, 0] = 0.0                                     # A'_00 = 2 b_0 = 0
    with pytest.raises(oracle.PivotError) as e:
        oracle.solve(P, B, np.ones((6, 1)))
    assert e.value.row == 0


# ---------------------------------------------------------------- planted mistakes
def _mut_periodic(a, b, c, d, which):
    n = len(b)
    vlast = -a[0] / b[0]
    bp = np.array(b, dtype=float)
    if which != "no_end_terms":                       # A' keeps b on its diagonal ends
        bp[0] = b[0] + b[0]
        bp[n - 1] = b[n - 1] + a[0] * c[n - 1] / b[0]
    u = np.zeros((n, 1))
    u[0, 0] = -b[0]
    u[n - 1, 0] = c[n - 1]
    z = twin.tri_solve(a, bp, c, u)[:, 0]
    y = twin.tri_solve(a, bp, c, d)
    if which == "drop_vlast":                         # v . w taken as w_0 alone
        vz1, vy = 1.0 + z[0], y[0]
    else:
        vz1, vy = 1.0 + (z[0] + vlast * z[n - 1]), y[0] + vlast * y[n - 1]
    s = vy / vz1
    return y + s * z[:, None] if which == "sign" else y - s * z[:, None]


@pytest.mark.parametrize("which", ["no_end_terms", "drop_vlast", "sign"])
def test_dense_pin_catches_periodic_mistakes(which):
    rng = np.random.default_rng(11)
    B = random_periodic(rng, 12)
    d = rng.uniform(-1, 1, (12, 4))
    ref = np.linalg.solve(dense_periodic(B), d)
    assert colrel(_mut_periodic(*B, d, "none"), ref) <= 1e-14
    assert colrel(_mut_periodic(*B, d, which), ref) > 1e-6
