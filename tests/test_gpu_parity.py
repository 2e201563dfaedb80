"""GPU parity: the HIP path through the C ABI against the oracle.

Bar: FP64 results within 1e-12 of the oracle, measured per system as
||x_gpu - x_oracle||_inf / ||x_oracle||_inf and maximised over systems.  The
GPU multiplies by stored reciprocals and fuses multiply-adds, so the two
differ by a few units of roundoff times the condition number (well below
1e-13 for every matrix here).  Layout transforms are compared bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1909_04539_amd import sbs, workloads as W

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
DEV = "cuda:0"


def colrel(x, ref):
    num = np.max(np.abs(x - ref), axis=0)
    den = np.maximum(np.max(np.abs(ref), axis=0), np.finfo(float).tiny)
    return float(np.max(num / den))


def bands_for(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == 3:
        return W.tri_dominant_bands(rng, n)
    B = rng.uniform(-1, 1, (5, n))
    B[2] = np.sum(np.abs(np.delete(B, 2, axis=0)), axis=0) + rng.uniform(1, 2, n)
    return W.zero_outside(B)


def chunked_fits(kind, n, elem=8):
    """The chunked variant keeps per-chunk checkpoints plus two factor chunks
    in one workgroup's LDS, at most 160 KiB (the whole LDS of a CU)."""
    K = (n + 31) // 32
    S = 1 if kind == 3 else 2
    row = (4 if kind == 3 else 8) * elem
    return K * S * 64 * elem + 2 * 32 * row <= 160 * 1024


def partition_available(kind, n, elem=8, m=1 << 20, cus=256):
    """Mirror of the library's rule (for matrices whose blocks all differ):
    some block length lb in (16, 32, 64) with P = ceil(n/lb) <= 64 blocks, at
    most 90 interface unknowns 2h(P-1), and for some S systems per workgroup
    (64, 32, 16; 8 and 4 only while a batch of m leaves CUs idle) at most
    512 (lb 64, FP64) or 1024 threads and block factors + spikes + interface
    inverse + block map + interface values (and, for FP64 pentadiagonal
    matrices, the interface unknowns beside them) within 160 KiB of LDS."""
    h = kind // 2
    row = (4 if kind == 3 else 8) * elem
    r16 = lambda v: -(-v // 16) * 16
    for lb in (16, 32, 64):
        P = -(-n // lb)
        Nr = 2 * h * (P - 1)
        if P > 64 or Nr > 90:
            continue
        maxt = 512 if (lb == 64 and elem == 8) else 1024
        S = 64
        while S >= 4:
            if S < 16 and -(-m // (2 * S)) >= cus:
                break
            if S * P <= maxt:
                lds = (r16(P * lb * row) + r16(P * lb * 2 * h * elem) + r16(Nr * Nr * elem) + r16(P * 4)
                       + r16(S * (Nr + 1) * elem) * (2 if elem == 8 and kind == 5 else 1))
                if lds <= 160 * 1024:
                    return True
            S //= 2
    return False


def separator_available(kind, n, elem=8, m=1 << 20):
    """Mirror of the library's rule for the separator form (matrices whose
    blocks all differ): some block length lb in (16, 32, 64) with
    P = ceil(n/lb) <= 64 blocks and at most 128 separator unknowns h(P-1),
    whose block factors + spikes + separator band rows + inverse of the
    separator system + block map, with the published block tops and the
    separator right-hand sides (and, in FP64, the separators) of one
    system per workgroup, fit in 160 KiB of LDS."""
    h = kind // 2
    row = (4 if kind == 3 else 8) * elem
    r16 = lambda v: -(-v // 16) * 16
    for lb in (16, 32, 64):
        P = -(-n // lb)
        Nr = h * (P - 1)
        if P > 64 or Nr > 128:
            continue
        blob = (r16(P * lb * row) + r16(P * lb * 2 * h * elem) + r16(P * h * (2 * h + 1) * elem)
                + r16(Nr * Nr * elem) + r16(P * 4))
        if blob + r16(P * h * elem) + r16((Nr + 1) * elem) * (2 if elem == 8 else 1) <= 160 * 1024:
            return True
    return False


def separator_in_memory_available(kind, n, elem=8, m=1 << 20):
    """Mirror of the library's rule for the separator form with its plan
    read from global memory (taken where the whole plan does not fit the
    LDS): blocks of 32 rows with two systems per lane (m even) or of 64 rows
    with one, P = ceil(n/lb) <= 64 blocks, at most 128 separator unknowns,
    a workgroup of (S / vec) * P threads within the shape's limit (512 for
    FP64, 1024 for FP32), and S^{-1} plus the separator buffers (two for
    FP32; three for FP64, or two where the separators overwrite their
    right-hand sides: whole waves, one matrix-core tile per wave) within
    160 KiB of LDS."""
    h = kind // 2
    r16 = lambda v: -(-v // 16) * 16
    maxt = 512 if elem == 8 else 1024
    for lb, vec in ((32, 2), (64, 1)):
        if vec == 2 and m % 2:
            continue
        P = -(-n // lb)
        Nr = h * (P - 1)
        if P > 64 or Nr > 128:
            continue
        for S in (64, 32, 16, 8, 4, 2, 1):
            if S < vec or S % vec or S > m:
                continue
            threads = (S // vec) * P
            if threads > maxt:
                continue
            sinv, red = r16(Nr * Nr * elem), r16(S * (Nr + 1) * elem)
            if sinv + red * (3 if elem == 8 else 2) <= 160 * 1024:
                return True
            tiles = -(-Nr // 16) * -(-S // 16)
            if elem == 8 and sinv + 2 * red <= 160 * 1024 and threads % 64 == 0 and tiles <= threads // 64:
                return True
    return False


def gpu_solve(kind, B, rhs, variant=sbs.VARIANT_AUTO, dtype=torch.float64):
    with sbs.SharedLhs(kind, B) as lhs:
        x = torch.from_numpy(np.ascontiguousarray(rhs)).to(DEV, dtype)
        lhs.solve(x, variant)
        torch.cuda.synchronize()
        return x.cpu().numpy().astype(np.float64)


SHAPES = [(1, 1), (2, 3), (3, 64), (4, 5), (5, 65), (8, 1), (31, 63), (32, 64), (33, 127), (63, 130),
          (64, 1), (65, 200), (100, 129), (256, 1024), (1000, 77), (1025, 64), (2048, 65)]


@pytest.mark.parametrize("kind", [3, 5])
@pytest.mark.parametrize("variant", [sbs.VARIANT_AUTO, sbs.VARIANT_RESIDENT, sbs.VARIANT_CHUNKED,
                                     sbs.VARIANT_STREAM, sbs.VARIANT_PARTITION])
@pytest.mark.parametrize("n,m", SHAPES)
def test_fp64_matches_oracle(kind, variant, n, m):
    if variant == sbs.VARIANT_RESIDENT and n > 64:
        pytest.skip("resident variant holds at most 64 rows")
    print(f"case kind={kind} variant={variant} n={n} m={m}", flush=True)
    B = bands_for(kind, n, 1000 * kind + n)
    rhs = np.random.default_rng(n * 7 + m).uniform(-1, 1, (n, m))
    if (variant == sbs.VARIANT_CHUNKED and not chunked_fits(kind, n)) or \
            (variant == sbs.VARIANT_PARTITION and not partition_available(kind, n, m=m)
             and not separator_available(kind, n, m=m) and not separator_in_memory_available(kind, n, m=m)):
        with pytest.raises(sbs.SbsError) as e:
            gpu_solve(kind, B, rhs, variant)
        assert e.value.status == 1
        return
    got = gpu_solve(kind, B, rhs, variant)
    assert colrel(got, oracle.solve(kind, B, rhs)) <= TOL64


@pytest.mark.parametrize("n", [900, 1000])
def test_penta_interface_forms(n):
    # FP64 pentadiagonal plans with 64-row blocks: 15 blocks give workgroups
    # of 15 x 32 = 480 threads, not whole waves, so the interface unknowns
    # come from per-lane dot products; 16 blocks give 512 threads and the
    # matrix-core product.  Both against the oracle.
    m = 4096
    assert partition_available(5, n, m=m)
    B = bands_for(5, n, 77 + n)
    rhs = np.random.default_rng(n).uniform(-1, 1, (n, m))
    got = gpu_solve(5, B, rhs, sbs.VARIANT_PARTITION)
    assert colrel(got, oracle.solve(5, B, rhs)) <= TOL64


@pytest.mark.parametrize("n", [900, 1000, 1024])
@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_penta_partition_tiny_batches(n, m):
    # a workgroup of 4 systems x 15 or 16 blocks with most of its systems
    # missing: per-lane form at 60 threads, matrix-core form at 64
    B = bands_for(5, n, 5 * n + m)
    rhs = np.random.default_rng(m).uniform(-1, 1, (n, m))
    got = gpu_solve(5, B, rhs, sbs.VARIANT_PARTITION)
    assert colrel(got, oracle.solve(5, B, rhs)) <= TOL64


def test_partition_plan_rule():
    # penta n = 2048 needs 31 blocks of 64 rows: 120 interface unknowns, over the
    # pair form's limit; the separator form has 62, but with every block
    # different its 32 block factors and spikes exceed the LDS
    assert not partition_available(5, 2048) and partition_available(5, 1024) and partition_available(3, 2048)
    assert not separator_available(5, 2048) and separator_available(5, 1024) and separator_available(3, 2048)
    assert separator_available(3, 3000, elem=4) and not partition_available(3, 3000, elem=4)
    # with the plan read from global memory the separator form reaches
    # penta n = 2048 (and 3000 with 64-row blocks), not 5000
    assert separator_in_memory_available(5, 2048) and separator_in_memory_available(5, 3000, m=33)
    assert not separator_in_memory_available(5, 5000)


@pytest.mark.parametrize("kind", [3, 5])
@pytest.mark.parametrize("n", [1, 40, 64, 65, 700, 1024, 1500, 2048, 3000, 5000])
def test_auto_variant_query(kind, n):
    # what AUTO runs: partitioned when a plan exists, else resident / chunked / stream
    # (for 1000 systems AUTO never takes the separator form with its plan in
    # memory: its shape with the most workgroups has runs of 16 or 32 bytes)
    with sbs.SharedLhs(kind, bands_for(kind, n, n)) as lhs:
        for dtype, elem in ((sbs.SBS_F64, 8), (sbs.SBS_F32, 4)):
            if partition_available(kind, n, elem, m=1000) or separator_available(kind, n, elem, m=1000):
                want = sbs.VARIANT_PARTITION
            elif n <= 64:
                want = sbs.VARIANT_RESIDENT
            else:
                want = sbs.VARIANT_CHUNKED if chunked_fits(kind, n, elem) else sbs.VARIANT_STREAM
            assert sbs.sbs_auto_variant(lhs.handle, 1000, dtype) == want
        with pytest.raises(sbs.SbsError):
            sbs.sbs_auto_variant(lhs.handle, 0)


@pytest.mark.parametrize("kind", [3, 5])
@pytest.mark.parametrize("n,m", [(64, 4096), (65, 33), (129, 1000), (500, 17), (1024, 3000), (2048, 130)])
def test_partition_fp32(kind, n, m):
    if not partition_available(kind, n, elem=4, m=m) and not separator_available(kind, n, elem=4, m=m) \
            and not separator_in_memory_available(kind, n, elem=4, m=m):
        pytest.skip("no partition plan")
    B = bands_for(kind, n, 9 + n)
    rhs = np.random.default_rng(n + m).uniform(-1, 1, (n, m)).astype(np.float32)
    got = gpu_solve(kind, B, rhs, sbs.VARIANT_PARTITION, dtype=torch.float32)
    ref = oracle.solve(kind, B, rhs.astype(np.float64))
    assert colrel(got, ref) <= 2e-5


def test_variants_agree_bit_for_bit():
    # The sweep variants run the same recurrences in the same order.
    for kind in (3, 5):
        B = bands_for(kind, 60, kind)
        rhs = np.random.default_rng(kind).uniform(-1, 1, (60, 190))
        outs = [gpu_solve(kind, B, rhs, v) for v in (1, 2, 3)]
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])


@pytest.mark.parametrize("kind", [3, 5])
@pytest.mark.parametrize("n,m", [(7, 3), (64, 64), (300, 100), (1024, 257)])
def test_fp32_plain_solve_accuracy(kind, n, m):
    B = bands_for(kind, n, 5 + n)
    rhs = np.random.default_rng(n).uniform(-1, 1, (n, m)).astype(np.float32)
    got = gpu_solve(kind, B, rhs, dtype=torch.float32)
    ref = oracle.solve(kind, B, rhs.astype(np.float64))
    assert colrel(got, ref) <= 2e-5      # FP32 arithmetic, well-conditioned matrices


def test_config0_full():
    wl = W.config0()
    got = gpu_solve(3, wl.bands, wl.rhs)
    assert colrel(got, oracle.solve(3, wl.bands, wl.rhs)) <= TOL64


def test_config1_full_size_sampled_columns():
    wl = W.config1()
    with sbs.SharedLhs(5, wl.bands) as lhs:
        x = torch.from_numpy(wl.rhs).to(DEV)
        lhs.solve(x)
        torch.cuda.synchronize()
        cols = np.unique(np.concatenate([[0, 63, 64, 65, wl.m - 64, wl.m - 1],
                                         np.random.default_rng(1).choice(wl.m, 500, replace=False)]))
        got = x[:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    ref = oracle.solve(5, wl.bands, wl.rhs[:, cols])
    assert colrel(got, ref) <= TOL64
    # manufactured solution: rhs = A x_true
    assert colrel(got, wl.extra["x_true"][:, cols]) <= 1e-12


def test_full_size_random_bands_sampled_columns():
    # the headline's size with random diagonally dominant bands: every block
    # of the partition plan is stored (no two alike), right-hand sides drawn
    # on the device; sampled columns (wave and group edges, the last one)
    # against the oracle
    n, m = 1024, 65536
    B = bands_for(5, n, 11)
    g = torch.Generator(device=DEV)
    g.manual_seed(12)
    x = torch.rand((n, m), dtype=torch.float64, device=DEV, generator=g) * 2 - 1
    cols = np.unique(np.concatenate([[0, 31, 32, 63, 64, m - 33, m - 32, m - 1],
                                     np.random.default_rng(3).choice(m, 200, replace=False)]))
    idx = torch.from_numpy(cols).to(DEV)
    rhs_cols = x[:, idx].cpu().numpy()
    with sbs.SharedLhs(5, B) as lhs:
        assert sbs.sbs_auto_variant(lhs.handle, m) == sbs.VARIANT_PARTITION
        lhs.solve(x)
        torch.cuda.synchronize()
    got = x[:, idx].cpu().numpy()
    del x
    assert colrel(got, oracle.solve(5, B, rhs_cols)) <= TOL64


def test_handle_storage_is_independent_of_batch_size():
    for kind, n in ((3, 1000), (5, 1000), (5, 3)):
        B = bands_for(kind, n, 3)
        with sbs.SharedLhs(kind, B) as lhs:
            rows = (n + 63) // 64 * 64
            # FP64 factor + FP32 shadow + original bands, per padded row ...
            per_row = {3: 32 + 16 + 64, 5: 64 + 32 + 64}[kind]
            # ... plus up to three pair-form and three separator plans (block
            # factors and spikes in FP64 and FP32, an interface inverse of at
            # most 90 x 90 or 128 x 128 in both precisions, a block map of at
            # most 64 ints, each blob 256-byte aligned) and, for the 32- and
            # 64-row separator plans, the mixed-precision kernel's copy (FP32
            # coefficients and spikes, FP64 band rows, FP32 inverse)
            plan_row = {3: (32 + 16) * 3 // 2, 5: (64 + 32) * 3 // 2}[kind]
            rec_row = {3: 5 * 4 + 3 * 8, 5: 9 * 4 + 5 * 8}[kind]
            bound = (rows * (per_row + 6 * plan_row + 2 * rec_row) + 3 * 90 * 90 * 12 + 3 * 128 * 128 * 12
                     + 2 * 128 * 128 * 4 + 16 * 2048)
            assert rows * per_row <= lhs.device_bytes <= bound, (kind, n, lhs.device_bytes, bound)
    # Shared LHS storage against one copy per system (the storage counts
    # closing Sections 3.1 and 4.1): 3N + MN vs 4MN, 5N + MN vs 6MN.
    M, N = 65536, 1024
    assert round(100 * (1 - (3 * N + M * N) / (4 * M * N))) == 75
    assert round(100 * (1 - (5 * N + M * N) / (6 * M * N))) == 83


def test_zero_m_is_a_noop_and_bad_variant_is_rejected():
    B = bands_for(5, 100, 1)
    with sbs.SharedLhs(5, B) as lhs:
        x = torch.zeros((100, 0), dtype=torch.float64, device=DEV)
        lhs.solve(x)
        y = torch.zeros((100, 4), dtype=torch.float64, device=DEV)
        with pytest.raises(sbs.SbsError) as e:
            lhs.solve(y, sbs.VARIANT_RESIDENT)
        assert e.value.status == 1
        with pytest.raises(sbs.SbsError):
            lhs.solve(y, 9)


def test_factor_errors_on_gpu():
    P = W.hyperdiffusion_bands(50, 0.5)
    P[2, 17] = 0.0
    P[1, 17] = 0.0
    P[0, 17] = 0.0
    with pytest.raises(sbs.SbsError) as e:
        sbs.SharedLhs(5, P)
    assert e.value.status == 2 and e.value.bad_row == 17


# ----------------------------------------------------------------- mixed precision
# n = 512 tri and 300 tri / penta: the one-wave-per-block kernel (32-row
# blocks; 64-row blocks for penta 512, whose 32-row edges exceed the LDS);
# 700 penta: the pair-form kernel; 1 and 2 rows: one block
@pytest.mark.parametrize("kind,n,m", [(3, 512, 4096), (3, 1, 5), (3, 33, 70), (5, 700, 300), (5, 2, 64),
                                      (5, 512, 256), (5, 300, 130), (3, 300, 65)])
def test_refined_matches_fp64_oracle(kind, n, m):
    if kind == 3:
        wl = W.config3(n=n, m=m)
        B, b32 = wl.bands, wl.rhs
    else:
        B = W.hyperdiffusion_bands(n, 0.5)
        b32 = np.random.default_rng(n).uniform(-1, 1, (n, m)).astype(np.float32)
    ref = oracle.refine_reference(kind, B, b32)
    with sbs.SharedLhs(kind, B) as lhs:
        b = torch.from_numpy(b32).to(DEV)
        errs = []
        for sweeps in (0, 1, 2):
            x = lhs.solve_refined(b, sweeps=sweeps)
            torch.cuda.synchronize()
            errs.append(colrel(x.cpu().numpy(), ref))
    print(f"refinement errors kind={kind} n={n} m={m}: {errs}", flush=True)
    assert errs[0] <= 1e-4
    assert errs[2] <= TOL64
    assert errs[2] <= errs[0]


def test_refined_config3_full_size_sampled_columns():
    wl = W.config3()
    cols = np.unique(np.concatenate([[0, 1, 63, 64, wl.m - 1],
                                     np.random.default_rng(2).choice(wl.m, 300, replace=False)]))
    with sbs.SharedLhs(3, wl.bands) as lhs:
        b = torch.from_numpy(wl.rhs).to(DEV)
        x = lhs.solve_refined(b, sweeps=2)
        torch.cuda.synchronize()
        got = x[:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
        del x, b
    ref = oracle.refine_reference(3, wl.bands, wl.rhs[:, cols])
    assert colrel(got, ref) <= TOL64


# ----------------------------------------------------------------- layout
@pytest.mark.parametrize("rows,cols", [(1, 1), (3, 5), (64, 64), (65, 130), (1, 200), (257, 3), (2048, 2048)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_transpose_is_bit_exact(rows, cols, dtype):
    idx = torch.arange(rows * cols, dtype=torch.int64)
    src = idx.to(dtype).reshape(rows, cols).to(DEV)
    dst = sbs.sbs_transpose(src)
    torch.cuda.synchronize()
    want = idx.reshape(rows, cols).t().contiguous().to(dtype)
    got = dst.cpu()
    assert torch.equal(got.view(torch.int64 if dtype == torch.float64 else torch.int32),
                       want.view(torch.int64 if dtype == torch.float64 else torch.int32))


def test_transpose_keeps_nan_payloads_and_signed_zeros():
    bits = torch.tensor([0x7ff8000000000001, -0x8000000000000000, 0x7ff0000000000000, 1, 0x000fffffffffffff,
                         -0x0008000000000000], dtype=torch.int64)
    src = bits.repeat(70).reshape(20, 21).view(torch.float64).to(DEV)
    got = sbs.sbs_transpose(src).cpu().view(torch.int64)
    assert torch.equal(got, bits.repeat(70).reshape(20, 21).t().contiguous())


@pytest.mark.parametrize("ny,nx", [(64, 64), (48, 80), (2048, 2048)])
def test_adi_step_matches_oracle(ny, nx):
    wl = W.config2(ny=ny, nx=nx)
    ref = oracle.adi_step(wl.bands, wl.extra["bands_x"], wl.rhs)
    hy = sbs.SharedLhs(3, wl.bands)
    hx = sbs.SharedLhs(3, wl.extra["bands_x"])
    g = torch.from_numpy(wl.rhs).to(DEV)
    work = torch.empty_like(g)
    sbs.sbs_adi_step(hy.handle, hx.handle, g, work)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    hy.close()
    hx.close()
    assert colrel(got, ref) <= TOL64          # per column
    assert colrel(got.T, ref.T) <= TOL64      # per row


@pytest.mark.parametrize("kind,coeffs", [(3, [-0.5, 2.0, -0.5]), (5, [0.5, -2.0, 4.0, -2.0, 0.5]),
                                         (13, [-0.3, 1.6, -0.3])])
@pytest.mark.parametrize("n", [5, 64, 1024, 3000])
def test_uniform_factor_equals_general_factor(kind, coeffs, n):
    # the uniform entry point is the general one on the expanded bands
    B = np.stack([np.full(n, c) for c in coeffs])
    if kind != 13:
        B = W.zero_outside(B)
    rhs = np.random.default_rng(n).uniform(-1, 1, (n, 130))
    hu = sbs.sbs_factor_uniform(kind, n, coeffs)
    try:
        outs = []
        for h in (hu, None):
            with (sbs.SharedLhs(kind, B) if h is None else _Borrowed(h)) as lhs:
                x = torch.from_numpy(rhs).to(DEV)
                lhs.solve(x)
                torch.cuda.synchronize()
                outs.append(x.cpu().numpy())
                assert sbs.sbs_handle_info(lhs.handle)[1] == n
        assert np.array_equal(outs[0], outs[1])
        ref_kind = oracle.TRI_PERIODIC if kind == 13 else kind
        assert colrel(outs[0], oracle.solve(ref_kind, B, rhs)) <= TOL64
    finally:
        sbs.sbs_release(hu)


class _Borrowed:
    """A handle used like SharedLhs without being released on exit."""

    def __init__(self, h):
        self.handle = h

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        return False

    def solve(self, rhs, variant=sbs.VARIANT_AUTO):
        return sbs.sbs_solve_batch_variant(self.handle, rhs, variant)


@pytest.mark.parametrize("ny,nx", [(64, 1024), (300, 1000), (130, 900), (100, 65)])
def test_adi_step_with_pentadiagonal_rows(ny, nx):
    # a pentadiagonal x-matrix: its row-layout partition uses the matrix-core
    # interface step (1024 rows: 16 blocks) or the per-lane one (900: 15);
    # against the oracle's solves along y and then along x
    By = W.diffusion_bands(ny, 0.5)
    Bx = bands_for(5, nx, nx + 1)
    g = np.random.default_rng(ny * nx).uniform(-1, 1, (ny, nx))
    with sbs.SharedLhs(3, By) as hy, sbs.SharedLhs(5, Bx) as hx:
        G = torch.from_numpy(g.copy()).to(DEV)
        work = torch.empty_like(G)
        sbs.sbs_adi_step(hy.handle, hx.handle, G, work)
        torch.cuda.synchronize()
        got = G.cpu().numpy()
    ref = oracle.solve(5, Bx, np.ascontiguousarray(oracle.solve(3, By, g).T)).T
    assert colrel(got.T, ref.T) <= TOL64


@pytest.mark.parametrize("ny,nx", [(64, 2048), (333, 1024), (1000, 96), (257, 64), (100, 65), (40, 1001)])
def test_adi_rows_equal_the_transposed_path(ny, nx):
    # The x-direction solve reads the grid's rows in place when the x-matrix
    # has a partition plan (pair form); it must give the bits of transpose,
    # interleaved solve, transpose back where the interleaved solve takes the
    # pair form too (the same plan and arithmetic), else agree to 1e-13.
    By = W.diffusion_bands(ny, 0.5)
    Bx = bands_for(3, nx, nx)
    g = np.random.default_rng(ny + nx).uniform(-1, 1, (ny, nx))
    with sbs.SharedLhs(3, By) as hy, sbs.SharedLhs(3, Bx) as hx:
        assert sbs.sbs_auto_variant(hx.handle, ny) == sbs.VARIANT_PARTITION
        G = torch.from_numpy(g.copy()).to(DEV)
        work = torch.empty_like(G)
        sbs.sbs_adi_step(hy.handle, hx.handle, G, work)
        R = torch.from_numpy(g.copy()).to(DEV)
        hy.solve(R)
        T = sbs.sbs_transpose(R)
        form = sbs.sbs_partition_shape(hx.handle, T)[0]
        hx.solve(T)
        R = sbs.sbs_transpose(T)
        torch.cuda.synchronize()
        if form == 0:
            assert torch.equal(G, R)
        else:
            assert colrel(G.cpu().numpy(), R.cpu().numpy()) <= 1e-13
        ref = oracle.adi_step(By, Bx, g)
        assert colrel(G.cpu().numpy(), ref) <= TOL64


@pytest.mark.parametrize("n", [1024, 2048])
def test_auto_on_the_ill_conditioned_laplacian(n):
    # T = tridiag(-1, 2, -1), condition number ~ 4e5 (n = 1024) and 1.7e6
    # (n = 2048): whatever variant AUTO picks stays within the bar.
    B = W.zero_outside(np.stack([-np.ones(n), np.full(n, 2.0), -np.ones(n)]))
    rhs = np.random.default_rng(n).uniform(-1, 1, (n, 300))
    got = gpu_solve(3, B, rhs)
    assert colrel(got, oracle.solve(3, B, rhs)) <= TOL64


@pytest.mark.parametrize("n", [256, 1000, 2048])
def test_auto_with_tiny_block_pivots(n):
    # a = c = 1, b = 3 but b = 1e-12 at the start of every 16-row block after
    # the first: well conditioned, global pivots of order one, but every
    # block of a partition plan starts with a 1e-12 pivot.  The plans are
    # dropped at factor time and AUTO runs the sweeps.
    B = np.stack([np.ones(n), np.full(n, 3.0), np.ones(n)])
    B[1, 16::16] = 1e-12
    B = W.zero_outside(B)
    rhs = np.random.default_rng(n + 1).uniform(-1, 1, (n, 257))
    with sbs.SharedLhs(3, B) as lhs:
        assert sbs.sbs_auto_variant(lhs.handle, 257) != sbs.VARIANT_PARTITION
    got = gpu_solve(3, B, rhs)
    assert colrel(got, oracle.solve(3, B, rhs)) <= TOL64
