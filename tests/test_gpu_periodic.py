"""GPU parity of periodic tridiagonal solves (Section 3.3) against the
periodic oracle, FP64 within 1e-12 per column: the sweep variants (the
Sherman-Morrison correction folded into the two sweeps) and the partitioned
variant (the wrap as one more interface pair); plus the entry points that
reject periodic handles and a periodic ADI step."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1909_04539_amd import sbs

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
P = sbs.SBS_TRI_PERIODIC


def colrel(x, ref):
    num = np.max(np.abs(x - ref), axis=0)
    den = np.maximum(np.max(np.abs(ref), axis=0), np.finfo(float).tiny)
    return float(np.max(num / den))


def ring_bands(n, seed, margin=(1.0, 2.0)):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    b = np.abs(a) + np.abs(c) + rng.uniform(*margin, n)
    return np.stack([a, b, c])


def chunked_fits(n, elem=8):
    # checkpoints (one value per 32-row chunk per lane) + two factor chunks of 32 rows
    row = 8 * elem
    return ((n + 31) // 32) * 64 * elem + 2 * 32 * row <= 160 * 1024


def partition_available(n, m=1):
    """Periodic plans: n a whole number P >= 2 of blocks of 16, 32 or 64 rows,
    and either at most 90 interface unknowns in the pair form (2 per block:
    the wrap adds one pair) or, in the separator form, at most 64 blocks
    (one separator each) whose factors, spikes and separator inverse fit in
    the LDS with room for one system (the ring bands here differ per row), or
    -- with the plan read from global memory, blocks of 32 rows with two
    systems per lane (m even) or of 64 rows -- whose separator inverse and
    buffers for one workgroup of at most 512 threads fit there."""
    r16 = lambda v: -(-v // 16) * 16
    for lb in (16, 32, 64):
        P = n // lb
        if n % lb or P < 2:
            continue
        if 2 * P <= 90:
            return True
        blob = r16(P * lb * 32) + r16(P * lb * 16) + r16(P * 3 * 8) + r16(P * P * 8) + r16(P * 4)
        if P <= 64 and blob + r16(P * 8) + 2 * r16((P + 1) * 8) <= 160 * 1024:
            return True
    for lb, vec in ((32, 2), (64, 1)):
        P = n // lb
        if n % lb or P < 2 or P > 64 or (vec == 2 and m % 2) or vec > m:
            continue
        for S in (64, 32, 16, 8, 4, 2, 1):
            if S >= vec and S % vec == 0 and (S // vec) * P <= 512 and \
                    r16(P * P * 8) + 3 * r16(S * (P + 1) * 8) <= 160 * 1024:
                return True
    return False


def gpu_solve(B, rhs, variant=sbs.VARIANT_AUTO, dtype=torch.float64):
    with sbs.SharedLhs(P, B) as lhs:
        x = torch.from_numpy(np.ascontiguousarray(rhs)).to(DEV, dtype)
        lhs.solve(x, variant)
        torch.cuda.synchronize()
        return x.cpu().numpy().astype(np.float64)


SHAPES = [(3, 1), (3, 64), (4, 7), (7, 130), (32, 64), (33, 65), (64, 100), (65, 1000), (96, 33), (200, 4097),
          (1024, 2000), (2048, 129), (4096, 300), (20000, 70)]


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("variant", [sbs.VARIANT_AUTO, sbs.VARIANT_RESIDENT, sbs.VARIANT_CHUNKED,
                                     sbs.VARIANT_STREAM, sbs.VARIANT_PARTITION])
def test_periodic_parity(n, m, variant):
    if variant == sbs.VARIANT_RESIDENT and n > 64:
        pytest.skip("resident needs n <= 64")
    if variant == sbs.VARIANT_CHUNKED and not chunked_fits(n):
        pytest.skip("checkpoints exceed the chunked variant's LDS")
    print(f"case periodic n={n} m={m} variant={variant}", flush=True)
    B = ring_bands(n, n + m)
    if variant == sbs.VARIANT_PARTITION and not partition_available(n, m):
        with pytest.raises(sbs.SbsError) as e:
            gpu_solve(B, np.zeros((n, m)), variant)
        assert e.value.status == 1
        return
    rhs = np.random.default_rng(m).uniform(-1, 1, (n, m))
    got = gpu_solve(B, rhs, variant)
    ref = oracle.solve(oracle.TRI_PERIODIC, B, rhs)
    assert colrel(got, ref) <= 1e-12


def test_periodic_variants_agree_bit_for_bit():
    B = ring_bands(60, 1)
    rhs = np.random.default_rng(2).uniform(-1, 1, (60, 190))
    outs = [gpu_solve(B, rhs, v) for v in (sbs.VARIANT_RESIDENT, sbs.VARIANT_CHUNKED, sbs.VARIANT_STREAM)]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


def test_paper_crank_nicolson_periodic_bands():
    # Section 3.2: a = c = -sigma, b = 1 + 2 sigma on a periodic grid.
    n, m = 512, 4096
    sigma = 0.5 * (1.0 / n) ** -2 * 1e-6
    B = np.stack([np.full(n, -sigma), np.full(n, 1 + 2 * sigma), np.full(n, -sigma)])
    rhs = np.random.default_rng(5).uniform(-1, 1, (n, m))
    assert colrel(gpu_solve(B, rhs), oracle.solve(oracle.TRI_PERIODIC, B, rhs)) <= 1e-12


@pytest.mark.parametrize("n,m", [(16, 64), (300, 1000), (3000, 129)])
def test_periodic_fp32_plain_solve(n, m):
    B = ring_bands(n, 3 + n)
    rhs = np.random.default_rng(n).uniform(-1, 1, (n, m)).astype(np.float32)
    got = gpu_solve(B, rhs, dtype=torch.float32)
    ref = oracle.solve(oracle.TRI_PERIODIC, B, rhs.astype(np.float64))
    assert colrel(got, ref) <= 1e-5


def test_periodic_auto_variant_and_rejections():
    B = ring_bands(300, 9)
    with sbs.SharedLhs(P, ring_bands(1024, 9)) as whole:
        assert sbs.sbs_auto_variant(whole.handle, 1000) == sbs.VARIANT_PARTITION
    with sbs.SharedLhs(P, B) as lhs:
        assert sbs.sbs_auto_variant(lhs.handle, 1000) == sbs.VARIANT_CHUNKED   # 300 rows: no whole blocks
        x = torch.zeros((300, 64), dtype=torch.float64, device=DEV)
        with pytest.raises(sbs.SbsError):
            lhs.solve(x, sbs.VARIANT_PARTITION)
        with pytest.raises(sbs.SbsError):
            lhs.solve_refined(torch.zeros((300, 64), dtype=torch.float32, device=DEV))
        L = sbs.lib()
        srv = ctypes.c_void_p()
        assert L.sbs_server_create(1 << 24, 1, 0, ctypes.byref(srv)) == 0
        i = ctypes.c_int32()
        assert L.sbs_server_register(srv, lhs.handle, ctypes.byref(i)) == 1   # invalid argument
        assert L.sbs_server_destroy(srv) == 0
        _, n, dev_bytes = sbs.sbs_handle_info(lhs.handle)
        assert n == 300 and dev_bytes <= 320 * (64 + 32 + 64)


def test_periodic_adi_step():
    # Periodic in x, bounded in y; reference: oracle solves along y for every
    # column, then along x for every row (rows passed as interleaved columns).
    ny, nx = 96, 130
    By = np.stack([np.r_[0.0, np.full(ny - 1, -0.5)], np.full(ny, 2.0), np.r_[np.full(ny - 1, -0.5), 0.0]])
    Bx = ring_bands(nx, 4)
    g = np.random.default_rng(6).uniform(-1, 1, (ny, nx))
    ref = oracle.solve(3, By, g)
    ref = oracle.solve(oracle.TRI_PERIODIC, Bx, np.ascontiguousarray(ref.T)).T
    with sbs.SharedLhs(3, By) as hy, sbs.SharedLhs(P, Bx) as hx:
        G = torch.from_numpy(g.copy()).to(DEV)
        work = torch.empty_like(G)
        sbs.sbs_adi_step(hy.handle, hx.handle, G, work)
        torch.cuda.synchronize()
        assert colrel(G.cpu().numpy(), ref) <= 1e-12
