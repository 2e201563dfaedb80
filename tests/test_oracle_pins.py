"""Pins for the oracle (CPU only).

The oracle is trusted only after it agrees with things that are fixed by the
paper or by mathematics and that do not re-type its own formulas: dense LU
with partial pivoting, closed-form inverses and factors, banded LAPACK,
manufactured solutions, the DST-I diagonalisation of the ADI operator, and its
independent numpy twin.  The last test plants typical transcription mistakes
in a copy of the twin and checks that these pins catch every one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.fft
import scipy.linalg

import oracle
from oracle import twin
from paper_1909_04539_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(B):
    """Dense n x n matrix from row-aligned bands (row i, column i + k - kind//2)."""
    kind, n = B.shape
    h = kind // 2
    A = np.zeros((n, n))
    for k in range(kind):
        for i in range(n):
            j = i + k - h
            if 0 <= j < n:
                A[i, j] = B[k, i]
    return A


def colrel(x, ref):
    """max over systems j of ||x_j - ref_j||_inf / ||ref_j||_inf."""
    num = np.max(np.abs(x - ref), axis=0)
    den = np.maximum(np.max(np.abs(ref), axis=0), np.finfo(float).tiny)
    return float(np.max(num / den))


def random_penta_dominant(rng, n):
    B = rng.uniform(-1, 1, (5, n))
    B[2] = np.sum(np.abs(np.delete(B, 2, axis=0)), axis=0) + rng.uniform(1, 2, n)
    return W.zero_outside(B)


def random_tri_dominant(rng, n):
    return W.tri_dominant_bands(rng, n, (1.0, 2.0))


# ---------------------------------------------------------------- P1 dense LU
@pytest.mark.parametrize("n", list(range(1, 17)) + [23, 31, 32, 47, 64])
def test_tri_matches_dense_lu(n):
    rng = np.random.default_rng(100 + n)
    B = random_tri_dominant(rng, n)
    m = int(rng.integers(1, 9))
    d = rng.uniform(-1, 1, (n, m))
    ref = np.linalg.solve(dense(B), d)
    assert colrel(oracle.solve(3, B, d), ref) <= 1e-14


@pytest.mark.parametrize("n", list(range(1, 17)) + [23, 31, 32, 47, 64])
def test_penta_matches_dense_lu(n):
    rng = np.random.default_rng(200 + n)
    B = random_penta_dominant(rng, n)
    m = int(rng.integers(1, 9))
    f = rng.uniform(-1, 1, (n, m))
    ref = np.linalg.solve(dense(B), f)
    assert colrel(oracle.solve(5, B, f), ref) <= 1e-14


@pytest.mark.parametrize("n", [5, 16, 64])
def test_penta_spd_hyperdiffusion_matches_dense_lu(n):
    # Not diagonally dominant (|1+6s| < 10|s| for s = 0.5): SPD only.
    B = W.hyperdiffusion_bands(n, 0.5)
    rng = np.random.default_rng(n)
    f = rng.standard_normal((n, 3))
    A = dense(B)
    assert np.all(np.linalg.eigvalsh(A) > 0)
    ref = np.linalg.solve(A, f)
    assert colrel(oracle.solve(5, B, f), ref) <= 1e-13


# ---------------------------------------------------------------- P2 residual
@pytest.mark.parametrize("kind,n", [(3, 200), (5, 200), (3, 1), (5, 2), (5, 3)])
def test_backward_error(kind, n):
    rng = np.random.default_rng(7 * n + kind)
    B = random_tri_dominant(rng, n) if kind == 3 else random_penta_dominant(rng, n)
    d = rng.uniform(-1, 1, (n, 16))
    x = oracle.solve(kind, B, d)
    A = dense(B)
    r = d - A @ x
    eta = np.max(np.abs(r), axis=0) / (np.linalg.norm(A, np.inf) * np.max(np.abs(x), axis=0)
                                       + np.max(np.abs(d), axis=0))
    assert float(np.max(eta)) <= 2e-16 * 8


# ---------------------------------------------------------------- P3 special cases
def test_single_unknown():
    d = np.array([[3.0, -6.0, 1.5]])
    assert np.array_equal(oracle.solve(3, np.array([[9.0], [2.0], [7.0]]), d), d / 2.0)
    assert np.array_equal(oracle.solve(5, np.array([[9.0], [9.0], [4.0], [7.0], [7.0]]), d), d / 4.0)


def test_diagonal_matrix_is_elementwise_division():
    rng = np.random.default_rng(3)
    n = 20
    diag = rng.uniform(1, 3, n)
    d = rng.uniform(-1, 1, (n, 5))
    Bt = np.stack([np.zeros(n), diag, np.zeros(n)])
    Bp = np.stack([np.zeros(n), np.zeros(n), diag, np.zeros(n), np.zeros(n)])
    assert np.array_equal(oracle.solve(3, Bt, d), d / diag[:, None])
    assert np.array_equal(oracle.solve(5, Bp, d), d / diag[:, None])


def test_zero_pivot_reports_row():
    B = W.diffusion_bands(8, 0.5)
    B[1, 0] = 0.0
    with pytest.raises(oracle.PivotError) as e:
        oracle.solve(3, B, np.ones((8, 2)))
    assert e.value.row == 0
    # den_3 = b_3 - a_3 chat_2 forced to zero
    B = W.diffusion_bands(8, 0.5)
    den, chat = oracle.tri_factor(B)
    B[1, 3] = B[0, 3] * chat[2]
    with pytest.raises(oracle.PivotError) as e:
        oracle.tri_factor(B)
    assert e.value.row == 3
    P = W.hyperdiffusion_bands(9, 0.5)
    P[2, 0] = np.nan
    with pytest.raises(oracle.PivotError) as e:
        oracle.penta_factor(P)
    assert e.value.row == 0


def test_out_of_matrix_coefficients_are_ignored():
    rng = np.random.default_rng(11)
    for kind, n in [(3, 7), (5, 9), (5, 3), (5, 2), (3, 1)]:
        B = random_tri_dominant(rng, n) if kind == 3 else random_penta_dominant(rng, n)
        junk = B.copy()
        if kind == 3:
            junk[0, 0], junk[2, n - 1] = 1e300, -7.0
        else:
            junk[0, :2], junk[1, 0] = 5e200, -3.0
            junk[3, n - 1] = 9.0
            junk[4, max(n - 2, 0):] = 4.0
        d = rng.uniform(-1, 1, (n, 3))
        assert np.array_equal(oracle.solve(kind, B, d), oracle.solve(kind, junk, d))


# ---------------------------------------------------------------- P4 / P5 closed forms
@pytest.mark.parametrize("n", [1, 2, 3, 8, 17, 32])
def test_tri_inverse_closed_form(n):
    # T = tridiag(-1, 2, -1): (T^-1)_{ij} = (min(i,j)+1)(n - max(i,j)) / (n+1), 0-based.
    B = np.stack([-np.ones(n), 2 * np.ones(n), -np.ones(n)])
    W.zero_outside(B)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    Tinv = (np.minimum(i, j) + 1) * (n - np.maximum(i, j)) / (n + 1)
    X = oracle.solve(3, B, np.eye(n))
    kappa = 4 * (n + 1) ** 2 / math.pi ** 2 + 1
    assert colrel(X, Tinv) <= 1e-15 * kappa * 4


@pytest.mark.parametrize("n", [2, 5, 40])
def test_tri_factor_closed_form(n):
    B = np.stack([-np.ones(n), 2 * np.ones(n), -np.ones(n)])
    W.zero_outside(B)
    den, chat = oracle.tri_factor(B)
    k = np.arange(n)
    assert np.allclose(den, (k + 2) / (k + 1), rtol=4e-16 * n, atol=0)
    assert np.allclose(chat[:-1], -(k[:-1] + 1) / (k[:-1] + 2), rtol=4e-16 * n, atol=0)
    assert chat[-1] == 0.0


def test_penta_inverse_of_T_squared():
    # A = T^2 (bands 1,-4,6,-4,1 with corner entries 5) has A^-1 = (T^-1)^2.
    n = 12
    T = dense(W.zero_outside(np.stack([-np.ones(n), 2 * np.ones(n), -np.ones(n)])))
    A = T @ T
    B = np.zeros((5, n))
    for k in range(5):
        for i in range(n):
            j = i + k - 2
            if 0 <= j < n:
                B[k, i] = A[i, j]
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    Tinv = (np.minimum(i, j) + 1) * (n - np.maximum(i, j)) / (n + 1)
    X = oracle.solve(5, B, np.eye(n))
    assert colrel(X, Tinv @ Tinv) <= 1e-11


# ---------------------------------------------------------------- P6 / P7 structure
@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 100])
def test_penta_with_outer_bands_zero_is_tri_bit_exact(n):
    rng = np.random.default_rng(n)
    T = random_tri_dominant(rng, n)
    P = np.stack([np.zeros(n), T[0], T[1], T[2], np.zeros(n)])
    d = rng.uniform(-1, 1, (n, 6))
    assert np.array_equal(oracle.solve(5, P, d), oracle.solve(3, T, d))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 33])
def test_penta_LR_reconstructs_A(n):
    rng = np.random.default_rng(50 + n)
    B = random_penta_dominant(rng, n)
    F = oracle.penta_factor(B)
    L, R = np.diag(F["alpha"]), np.eye(n)
    for i in range(n):
        if i >= 1:
            L[i, i - 1] = F["beta"][i]
        if i >= 2:
            L[i, i - 2] = F["eps"][i]
        if i + 1 < n:
            R[i, i + 1] = F["gamma"][i]
        if i + 2 < n:
            R[i, i + 2] = F["delta"][i]
    A = dense(B)
    assert np.max(np.abs(L @ R - A)) <= 4 * np.finfo(float).eps * np.max(np.abs(A)) * 4
    # gamma_{n-1}, delta_{n-2}, delta_{n-1} are not entries of R: they are zero.
    assert F["gamma"][-1] == 0.0 and F["delta"][-1] == 0.0
    if n >= 2:
        assert F["delta"][-2] == 0.0


# ---------------------------------------------------------------- P8 banded LAPACK
def lapack_banded(B, rhs):
    kind, n = B.shape
    h = kind // 2
    ab = np.zeros((kind, n))
    for k in range(kind):
        off = k - h
        for i in range(n):
            j = i + off
            if 0 <= j < n:
                ab[h - off, j] = B[k, i]
    return scipy.linalg.solve_banded((h, h), ab, rhs)


@pytest.mark.parametrize("k,sizes", [(0, {}), (1, {"m": 4096}), (3, {"m": 8192})])
def test_configs_match_banded_lapack(k, sizes):
    wl = W.make_config(k, **sizes)
    rhs = wl.rhs.astype(np.float64)
    x = oracle.solve(wl.kind, wl.bands, rhs)
    assert colrel(x, lapack_banded(wl.bands, rhs)) <= 1e-14


def test_config1_full_size_matches_banded_lapack_and_manufactured_solution():
    wl = W.config1()
    x = oracle.solve(5, wl.bands, wl.rhs)
    cols = np.random.default_rng(0).choice(wl.m, 2048, replace=False)
    assert colrel(x[:, cols], lapack_banded(wl.bands, wl.rhs[:, cols])) <= 1e-14
    # P9: rhs = A x_true; kappa_2(A) ~ 9, so the forward error is a few ulps.
    assert colrel(x, wl.extra["x_true"]) <= 1e-13


def test_spd_configs_match_cholesky_banded():
    wl = W.config1(m=512)
    B = wl.bands
    n = wl.n
    ab = np.zeros((3, n))          # upper form for solveh_banded
    ab[2] = B[2]
    ab[1, 1:] = B[3, :-1]
    ab[0, 2:] = B[4, :-2]
    ref = scipy.linalg.solveh_banded(ab, wl.rhs)
    assert colrel(oracle.solve(5, B, wl.rhs), ref) <= 1e-14


# ---------------------------------------------------------------- P10 ADI closed form
@pytest.mark.parametrize("ny,nx", [(64, 64), (48, 80), (2048, 2048)])
def test_adi_step_matches_dst_diagonalisation(ny, nx):
    r = 0.5
    rng = np.random.default_rng(ny + nx)
    F = W.adi_field(rng, ny, nx)
    U = oracle.adi_step(W.diffusion_bands(ny, r), W.diffusion_bands(nx, r), F)
    # A = I + rT is diagonalised by DST-I: lambda_k = 1 + 4r sin^2((k+1)pi/(2(n+1))).
    ly = 1 + 4 * r * np.sin((np.arange(ny) + 1) * math.pi / (2 * (ny + 1))) ** 2
    lx = 1 + 4 * r * np.sin((np.arange(nx) + 1) * math.pi / (2 * (nx + 1))) ** 2
    C = scipy.fft.dstn(F, type=1)
    ref = scipy.fft.idstn(C / (ly[:, None] * lx[None, :]), type=1)
    assert np.max(np.abs(U - ref)) / np.max(np.abs(ref)) <= 1e-14


# ---------------------------------------------------------------- P11 twin
@pytest.mark.parametrize("kind,n,m", [(3, 1, 3), (3, 2, 5), (3, 256, 64), (5, 1, 2), (5, 2, 3),
                                      (5, 3, 4), (5, 1024, 33)])
def test_c_oracle_and_numpy_twin_bit_identical(kind, n, m):
    rng = np.random.default_rng(kind * 1000 + n)
    B = random_tri_dominant(rng, n) if kind == 3 else W.hyperdiffusion_bands(n, 0.5)
    d = rng.uniform(-1, 1, (n, m))
    assert np.array_equal(oracle.solve(kind, B, d), oracle.twin_solve(kind, B, d))


def test_twin_factors_bit_identical():
    rng = np.random.default_rng(5)
    B = random_penta_dominant(rng, 50)
    Fc, Ft = oracle.penta_factor(B), twin.penta_factor(*B)
    for k in Fc:
        assert np.array_equal(Fc[k], Ft[k])
    T = random_tri_dominant(rng, 50)
    for u, v in zip(oracle.tri_factor(T), twin.tri_factor(*T)):
        assert np.array_equal(u, v)


def test_multithreaded_driver_is_identical_to_serial():
    wl = W.config0(m=333)
    X = wl.rhs.copy()
    oracle.solve_inplace_mt(3, wl.bands, X, nthreads=4)
    assert np.array_equal(X, oracle.solve(3, wl.bands, wl.rhs))
    wl = W.config1(m=257, n=100)
    X = wl.rhs.copy()
    oracle.solve_inplace_mt(5, wl.bands, X, nthreads=3)
    assert np.array_equal(X, oracle.solve(5, wl.bands, wl.rhs))


def test_refine_reference_uses_exact_fp64_promotion():
    wl = W.config3(n=64, m=16)
    x = oracle.refine_reference(3, wl.bands, wl.rhs)
    assert np.array_equal(x, oracle.solve(3, wl.bands, wl.rhs.astype(np.float64)))


# ---------------------------------------------------------------- generator recipes vs paper
def test_generator_matrices_match_paper_recipes():
    g = json.load(open(os.path.join(GOLDEN, "paper_matrices.json")))
    for sig, coeffs in g["diffusion"].items():
        B = W.diffusion_bands(6, float(sig))
        assert np.array_equal(B[:, 2], coeffs)
        assert B[0, 0] == 0 and B[2, -1] == 0
    for sig, coeffs in g["hyperdiffusion"].items():
        B = W.hyperdiffusion_bands(7, float(sig))
        assert np.array_equal(B[:, 3], coeffs)


def test_generator_row_blocks_equal_one_draw():
    a = W.uniform_rows(np.random.default_rng(1), 37, 11, block_rows=5)
    b = np.random.default_rng(1).uniform(-1, 1, (37, 11))
    assert np.array_equal(a, b)


def test_config0_is_strictly_dominant():
    B = W.config0().bands
    assert np.all(B[1] > np.abs(B[0]) + np.abs(B[2]))


# ---------------------------------------------------------------- pins catch planted mistakes
def _mut_tri(a, b, c, d, which):
    den, chat = twin.tri_factor(a, b, c)
    x = np.array(d, dtype=float)
    n = len(b)
    x[0] = x[0] / den[0]
    for i in range(1, n):
        if which == "sign":
            x[i] = (x[i] + a[i] * x[i - 1]) / den[i]
        else:
            x[i] = (x[i] - a[i] * x[i - 1]) / den[i]
    for i in range(n - 2, -1, -1):
        if which == "paper_typo":          # x_i = dhat_i - a_i chat_i, as printed
            x[i] = x[i] - a[i] * chat[i]
        elif which == "index":
            x[i] = x[i] - chat[i + 1 if i + 1 < n - 1 else i] * x[i + 1]
        else:
            x[i] = x[i] - chat[i] * x[i + 1]
    return x


def _mut_penta(a, b, c, d, e, f, which):
    F = twin.penta_factor(a, b, c, d, e)
    al, be, ga, de, ep = F["alpha"], F["beta"], F["gamma"], F["delta"], F["eps"]
    if which == "transposed":             # use the super-diagonals as sub-diagonals
        F = twin.penta_factor(e, d, c, b, a)
        al, be, ga, de, ep = F["alpha"], F["beta"], F["gamma"], F["delta"], F["eps"]
    x = np.array(f, dtype=float)
    n = len(c)
    z = np.zeros_like(x[0])
    for i in range(n):
        g2 = x[i - 2] if i >= 2 else z
        g1 = x[i - 1] if i >= 1 else z
        if which == "drop_eps":
            x[i] = (x[i] - be[i] * g1) / al[i]
        else:
            x[i] = (x[i] - ep[i] * g2 - be[i] * g1) / al[i]
    for i in range(n - 1, -1, -1):
        x1 = x[i + 1] if i + 1 < n else z
        x2 = x[i + 2] if i + 2 < n else z
        if which == "drop_delta":
            x[i] = x[i] - ga[i] * x1
        else:
            x[i] = x[i] - ga[i] * x1 - de[i] * x2
    return x


@pytest.mark.parametrize("which", ["sign", "paper_typo", "index"])
def test_dense_lu_pin_catches_tri_mistakes(which):
    rng = np.random.default_rng(9)
    B = random_tri_dominant(rng, 12)
    d = rng.uniform(-1, 1, (12, 4))
    ref = np.linalg.solve(dense(B), d)
    assert colrel(_mut_tri(*B, d, "none"), ref) <= 1e-14
    assert colrel(_mut_tri(*B, d, which), ref) > 1e-6


@pytest.mark.parametrize("which", ["drop_eps", "drop_delta", "transposed"])
def test_dense_lu_pin_catches_penta_mistakes(which):
    rng = np.random.default_rng(10)
    B = random_penta_dominant(rng, 12)
    f = rng.uniform(-1, 1, (12, 4))
    ref = np.linalg.solve(dense(B), f)
    assert colrel(_mut_penta(*B, f, "none"), ref) <= 1e-14
    assert colrel(_mut_penta(*B, f, which), ref) > 1e-6
