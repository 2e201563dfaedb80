"""C-ABI boundary checks that need no GPU: the library loads, exports every
entry point the header declares, and rejects bad arguments before touching
the device."""
import ctypes
import subprocess

import numpy as np
import pytest

from paper_1909_04539_amd import sbs, workloads as W


@pytest.fixture(scope="module")
def L():
    return sbs.lib()


def test_every_declared_symbol_is_exported(L):
    declared = sbs.declared_symbols()
    assert len(declared) >= 18
    out = subprocess.run(["nm", "-D", "--defined-only", sbs.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert getattr(L, s) is not None


def test_status_strings(L):
    for code in range(10):
        assert sbs.sbs_status_str(code)
    assert sbs.sbs_status_str(2) == "zero or non-finite pivot"
    assert sbs.sbs_status_str(99) == "unknown status"
    assert "gfx950" in sbs.sbs_version()


def _factor(L, kind, n, bands):
    h = ctypes.c_void_p(123)
    bad = ctypes.c_int64(7)
    B = None if bands is None else np.ascontiguousarray(bands, dtype=np.float64)
    st = L.sbs_factor_shared_lhs(kind, n, None if B is None else B.ctypes.data, ctypes.byref(h),
                                 ctypes.byref(bad))
    return st, h.value, bad.value


def test_factor_rejects_bad_arguments(L):
    B = W.diffusion_bands(8, 0.5)
    assert _factor(L, 4, 8, B)[0] == 1
    assert _factor(L, 3, 0, B)[0] == 1
    assert _factor(L, 3, -5, B)[0] == 1
    assert _factor(L, 3, 8, None)[0] == 1
    st, h, bad = _factor(L, 3, 8, B * np.nan)
    assert st == 3 and h is None and bad == 0
    assert L.sbs_factor_shared_lhs(3, 8, B.ctypes.data, None, None) == 1


def test_factor_reports_nonfinite_row(L):
    P = W.hyperdiffusion_bands(12, 0.5)
    P[3, 6] = np.inf
    st, h, bad = _factor(L, 5, 12, P)
    assert (st, h, bad) == (3, None, 6)
    # an infinite coefficient outside the matrix is ignored (it is not read)
    P = W.hyperdiffusion_bands(12, 0.5)
    P[0, 0] = np.inf
    P[4, 11] = np.nan
    st, _, bad = _factor(L, 5, 12, P)
    assert st != 3 and bad == -1


def test_factor_reports_zero_pivot_row_before_any_device_work(L):
    B = W.diffusion_bands(8, 0.5)
    B[1, 0] = 0.0
    assert _factor(L, 3, 8, B)[::2] == (2, 0)
    # den_2 = b_2 - a_2 chat_1 forced to zero
    B = np.stack([-np.ones(6), 2 * np.ones(6), -np.ones(6)])
    B[1, 2] = -(2.0 / 3.0) * -1.0   # chat_1 = -2/3 for T, so b_2 = a_2 chat_1 makes den_2 = 0
    st, h, bad = _factor(L, 3, 6, B)
    assert (st, h, bad) == (2, None, 2)
    P = W.hyperdiffusion_bands(9, 0.5)
    P[2, 0] = 0.0
    assert _factor(L, 5, 9, P)[::2] == (2, 0)


def test_null_handle_calls(L):
    assert L.sbs_release(None) == 0
    assert L.sbs_solve_batch(None, None, 10, 0, None) == 1
    assert L.sbs_solve_batch_variant(None, None, 10, 0, 0, None) == 1
    assert L.sbs_handle_info(None, None, None, None) == 1
    assert L.sbs_refined_workspace_bytes(None, 10) == 0
    assert L.sbs_solve_batch_refined(None, None, None, 10, 2, None, 0, None) == 1
    assert L.sbs_adi_step(None, None, None, None, 4, 4, None) == 1


def test_transpose_argument_checks(L):
    assert L.sbs_transpose(None, None, 0, 5, 0, None) == 0      # empty: nothing to do
    assert L.sbs_transpose(None, None, 3, 5, 0, None) == 1
    assert L.sbs_transpose(None, None, -1, 5, 0, None) == 1
    assert L.sbs_transpose(None, None, 3, 5, 7, None) == 1
    buf = ctypes.create_string_buffer(1024)
    p = ctypes.addressof(buf)
    assert L.sbs_transpose(p, p + 8, 4, 4, 0, None) == 1        # overlapping


def test_server_argument_checks(L):
    out = ctypes.c_void_p()
    assert L.sbs_server_create(0, 4, 0, ctypes.byref(out)) == 1
    assert L.sbs_server_create(1 << 20, 99, 0, ctypes.byref(out)) == 1
    assert L.sbs_server_create(1 << 20, 4, 0, None) == 1
    t = ctypes.c_uint64()
    assert L.sbs_server_submit(None, 0, None, 1, 0, ctypes.byref(t)) == 1
    assert L.sbs_server_wait(None, 1, 0, None, None) == 1
    assert L.sbs_server_release(None, 1) == 1
    assert L.sbs_server_destroy(None) == 0


def test_periodic_factor_errors_without_device(L):
    # Periodic tridiagonal handles (Section 3.3): n >= 3, corners must be
    # finite, b_0 = 0 breaks the splitting at row 0, and the singular periodic
    # Laplacian (rows sum to zero) makes 1 + v.z vanish: reported as row n.
    ring = lambda n, b: np.stack([np.full(n, -1.0), np.full(n, b), np.full(n, -1.0)])
    assert _factor(L, 13, 2, ring(2, 4.0))[0] == 1
    B = ring(6, 4.0)
    B[0, 0] = np.nan                                   # corner a_0
    assert _factor(L, 13, 6, B)[0] == 3 and _factor(L, 13, 6, B)[2] == 0
    B = ring(6, 4.0)
    B[1, 0] = 0.0
    st, h, bad = _factor(L, 13, 6, B)
    assert st == 2 and h is None and bad == 0
    for n in (3, 4, 5, 8, 64):
        st, h, bad = _factor(L, 13, n, ring(n, 2.0))
        assert st == 2 and h is None and bad == n


def test_uniform_factor_errors_without_device(L):
    def fac(kind, n, coeffs):
        h = ctypes.c_void_p(5)
        bad = ctypes.c_int64(7)
        c = None if coeffs is None else np.ascontiguousarray(coeffs, dtype=np.float64)
        st = L.sbs_factor_uniform(kind, n, None if c is None else c.ctypes.data, ctypes.byref(h), ctypes.byref(bad))
        return st, h.value, bad.value
    assert fac(3, 10, None)[0] == 1
    assert fac(4, 10, [1.0, 2.0, 3.0, 4.0])[0] == 1
    assert fac(3, 0, [1.0, 2.0, 3.0])[0] == 1
    assert fac(13, 2, [-1.0, 4.0, -1.0])[0] == 1
    assert fac(3, 10, [1.0, np.inf, 1.0])[0:3:2] == (3, 0)
    st, h, bad = fac(3, 10, [1.0, 0.0, 1.0])             # b_0 = 0
    assert st == 2 and h is None and bad == 0
    st, h, bad = fac(13, 16, [-1.0, 2.0, -1.0])          # periodic Laplacian: singular
    assert st == 2 and h is None and bad == 16


def test_factor_rejects_n_beyond_32_bit_rows(L):
    # The kernels index rows with 32-bit integers: n > INT32_MAX is an
    # argument error, reported before the bands are read (the 3-entry arrays
    # passed here would be far too short for such n).
    big = 2 ** 31
    for kind in (3, 5, 13):
        coeffs = np.ones(3 if kind != 5 else 5)
        st, h, bad = _factor(L, kind, big, coeffs)
        assert (st, h, bad) == (1, None, -1)
        h2 = ctypes.c_void_p(9)
        c = np.ascontiguousarray(coeffs)
        assert L.sbs_factor_uniform(kind, big, c.ctypes.data, ctypes.byref(h2), None) == 1
        assert h2.value is None


def test_probe_argument_checks(L):
    # the measurement probes reject shapes whose accesses would leave the array
    buf = ctypes.create_string_buffer(4096 + 16)
    p = (ctypes.addressof(buf) + 15) // 16 * 16
    assert L.sbs_probe_linear(3, p, p, 4096, 4, 1, None) == 1       # mode
    assert L.sbs_probe_linear(0, p, p, 4000 + 8, 4, 1, None) == 1   # not a multiple of 16
    assert L.sbs_probe_linear(0, p, p, 4096, 3, 1, None) == 1       # unroll
    assert L.sbs_probe_linear(0, None, p, 4096, 4, 1, None) == 1
    assert L.sbs_probe_blocks(p, 100, 64, 64, 1, 32, 1, None) == 1   # n not whole blocks
    assert L.sbs_probe_blocks(p, 128, 100, 64, 1, 32, 1, None) == 1  # m not whole groups
    assert L.sbs_probe_blocks(p, 1024, 64, 16, 1, 32, 1, None) == 1  # 2048 threads
    assert L.sbs_probe_blocks(p, 128, 64, 64, 2, 33, 1, None) == 1   # S not whole pairs
    assert L.sbs_probe_blocks(None, 128, 64, 64, 1, 32, 1, None) == 1
