"""Pins for the Crank-Nicolson step oracle (Sections 3.2 and 4.2), CPU only:
A C^{n+1} = (2I - A) C^n.  Checked against dense linear algebra, against the
explicit stencils the paper prints for its two benchmark schemes, against the
Fourier amplification factors of the periodic constant-coefficient scheme, and
against the non-increasing norm of a symmetric scheme; planted mistakes must
fail the dense pin."""
import numpy as np
import pytest

import oracle

PER = oracle.TRI_PERIODIC


def dense(kind, B):
    nb, n = B.shape
    h = nb // 2
    A = np.zeros((n, n))
    for k in range(nb):
        for i in range(n):
            j = i + k - h
            if kind == PER:
                A[i, j % n] += B[k, i]
            elif 0 <= j < n:
                A[i, j] = B[k, i]
    return A


def colrel(x, ref):
    num = np.max(np.abs(x - ref), axis=0)
    den = np.maximum(np.max(np.abs(ref), axis=0), np.finfo(float).tiny)
    return float(np.max(num / den))


def random_bands(kind, n, seed):
    rng = np.random.default_rng(seed)
    nb = 5 if kind == 5 else 3
    B = rng.uniform(-1, 1, (nb, n))
    B[nb // 2] = np.sum(np.abs(np.delete(B, nb // 2, axis=0)), axis=0) + rng.uniform(1, 2, n)
    return B


def dense_steps(kind, B, C, steps):
    A = dense(kind, B)
    E = 2 * np.eye(len(A)) - A
    X = C.copy()
    for _ in range(steps):
        X = np.linalg.solve(A, E @ X)
    return X


@pytest.mark.parametrize("kind", [3, 5, PER])
@pytest.mark.parametrize("n", [3, 4, 9, 40])
@pytest.mark.parametrize("steps", [1, 3])
def test_cn_matches_dense(kind, n, steps):
    B = random_bands(kind, n, n + kind)
    C = np.random.default_rng(n).uniform(-1, 1, (n, 5))
    assert colrel(oracle.cn_steps(kind, B, C, steps), dense_steps(kind, B, C, steps)) <= 1e-13


def _paper_rhs(kind, s, C):
    """The explicit halves printed for the benchmark schemes, periodic in i."""
    r = lambda k: np.roll(C, -k, axis=0)          # r(k)[i] = C[i + k]
    if kind == PER:
        return s * r(-1) + (1 - 2 * s) * C + s * r(1)
    return -s * r(-2) + 4 * s * r(-1) + (1 - 6 * s) * C + 4 * s * r(1) - s * r(2)


@pytest.mark.parametrize("s", [0.01, 0.5, 40.0])
def test_explicit_half_equals_printed_diffusion_stencil(s):
    n = 64
    B = np.stack([np.full(n, -s), np.full(n, 1 + 2 * s), np.full(n, -s)])
    C = np.random.default_rng(1).uniform(-1, 1, (n, 3))
    ref = np.linalg.solve(dense(PER, B), _paper_rhs(PER, s, C))
    assert colrel(oracle.cn_steps(PER, B, C, 1), ref) <= 1e-13


@pytest.mark.parametrize("s", [0.01, 0.5, 5.0])
def test_explicit_half_equals_printed_hyperdiffusion_stencil(s):
    # Interior rows of the pentadiagonal scheme (no wrap in this library's
    # pentadiagonal kind): compare rows away from the ends after one step of
    # an input that vanishes near both ends, where truncation changes nothing.
    n = 80
    B = np.stack([np.full(n, s), np.full(n, -4 * s), np.full(n, 1 + 6 * s), np.full(n, -4 * s), np.full(n, s)])
    C = np.zeros((n, 2))
    C[10:70] = np.random.default_rng(2).uniform(-1, 1, (60, 2))
    f_paper = _paper_rhs(5, s, C)
    f = 2 * C - dense(5, B) @ C
    assert np.max(np.abs(f - f_paper)) <= 1e-13 * (1 + 16 * s)
    ref = np.linalg.solve(dense(5, B), f_paper)
    assert colrel(oracle.cn_steps(5, B, C, 1), ref) <= 1e-12


@pytest.mark.parametrize("n", [8, 64, 256])
@pytest.mark.parametrize("s", [0.1, 2.0])
def test_periodic_diffusion_amplification_factors(n, s):
    # Fourier mode k of the periodic scheme is multiplied each step by
    # (1 - 2s(1 - cos t_k)) / (1 + 2s(1 - cos t_k)), t_k = 2 pi k / n.
    B = np.stack([np.full(n, -s), np.full(n, 1 + 2 * s), np.full(n, -s)])
    C = np.random.default_rng(n).uniform(-1, 1, (n, 4))
    steps = 5
    t = 2 * np.pi * np.arange(n) / n
    g = (1 - 2 * s * (1 - np.cos(t))) / (1 + 2 * s * (1 - np.cos(t)))
    ref = np.real(np.fft.ifft(np.fft.fft(C, axis=0) * (g ** steps)[:, None], axis=0))
    assert colrel(oracle.cn_steps(PER, B, C, steps), ref) <= 1e-12


def test_symmetric_scheme_never_grows():
    # Symmetric A with eigenvalues >= 1: (2I - A) A^{-1} has eigenvalues in
    # (-1, 1], so every column's 2-norm is non-increasing (unconditional
    # stability of Crank-Nicolson).
    n, s = 100, 3.0
    B = np.stack([np.full(n, s), np.full(n, -4 * s), np.full(n, 1 + 6 * s), np.full(n, -4 * s), np.full(n, s)])
    C = np.random.default_rng(4).uniform(-1, 1, (n, 6))
    prev = np.linalg.norm(C, axis=0)
    for _ in range(10):
        C = oracle.cn_steps(5, B, C, 1)
        cur = np.linalg.norm(C, axis=0)
        assert np.all(cur <= prev * (1 + 1e-14))
        prev = cur


@pytest.mark.parametrize("kind", [3, 5, PER])
def test_c_oracle_and_twin_bit_identical(kind):
    B = random_bands(kind, 37, 5)
    C = np.random.default_rng(6).uniform(-1, 1, (37, 9))
    assert np.array_equal(oracle.cn_steps(kind, B, C, 2), oracle.twin_cn_steps(kind, B, C, 2))


# ---------------------------------------------------------------- planted mistakes
def _mut_cn(kind, B, C, which):
    A = dense(kind, B)
    if which == "no_wrap":                         # explicit half without the periodic corners
        A_e = dense(3, B)
    else:
        A_e = A
    n = len(A)
    E = {"none": 2 * np.eye(n) - A_e, "no_wrap": 2 * np.eye(n) - A_e,
         "sign": 2 * np.eye(n) + A_e, "no_two": np.eye(n) - A_e}[which]
    return np.linalg.solve(A, E @ C)


@pytest.mark.parametrize("which", ["sign", "no_two", "no_wrap"])
def test_dense_pin_catches_cn_mistakes(which):
    B = random_bands(PER, 12, 8)
    C = np.random.default_rng(9).uniform(-1, 1, (12, 3))
    ref = oracle.cn_steps(PER, B, C, 1)
    assert colrel(_mut_cn(PER, B, C, "none"), ref) <= 1e-13
    assert colrel(_mut_cn(PER, B, C, which), ref) > 1e-6
