"""GPU parity of the separator-partitioned solve (the partitioned variant's
form for plain solves of interleaved right-hand sides): every shape the
library builds -- block length, one or two systems per lane, systems per
workgroup, group order, staggered starts and the plan read from global
memory -- against the oracle, on
matrices whose blocks all differ, with ragged last blocks, partial last
groups and odd batch sizes; periodic matrices; FP32; and the choice AUTO
makes for the benchmark's shapes."""
import numpy as np
import pytest
import torch

import oracle
from paper_1909_04539_amd import sbs, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL64 = 1e-12


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


def shape_run(h, rhs_np, lb, vec, S, flags, dtype=torch.float64):
    """Solve with one separator shape; None if the library has no such shape."""
    x = torch.from_numpy(np.ascontiguousarray(rhs_np)).to(DEV, dtype)
    try:
        sbs.sbs_solve_batch_partition(h.handle, x, 1, lb, vec, S, flags)
    except sbs.SbsError as e:
        assert e.status == 1
        return None
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.float64)


SHAPES = [(lb, vec, S) for lb in (16, 32, 64) for vec in (1, 2) for S in (64, 32, 16, 8, 2)]


@pytest.mark.parametrize("kind,n,m", [(3, 100, 130), (3, 1000, 77), (3, 1024, 256), (3, 2900, 64),
                                      (5, 100, 129), (5, 1000, 66), (5, 1024, 192), (5, 1400, 64),
                                      (5, 33, 7), (3, 17, 1)])
def test_every_shape_matches_oracle(kind, n, m):
    B = bands_for(kind, n, 300 + n)
    rhs = np.random.default_rng(n + m).uniform(-1, 1, (n, m))
    ref = oracle.solve(kind, B, rhs)
    ran = 0
    with sbs.SharedLhs(kind, B) as h:
        for lb, vec, S in SHAPES:
            # flags: chiplet order, staggered start, plan read from global memory
            for flags in (0, 1, 4 | (1 << 8), 16):
                print(f"case kind={kind} n={n} m={m} lb={lb} vec={vec} S={S} flags={flags}", flush=True)
                got = shape_run(h, rhs, lb, vec, S, flags)
                if got is None:
                    if flags == 0:
                        break  # no such shape (the other flags add none but 16's)
                    continue
                assert colrel(got, ref) <= TOL64, (lb, vec, S, flags, colrel(got, ref))
                ran += 1
    assert ran > 0


def test_two_systems_per_lane_needs_even_m_and_pair_alignment():
    n, m = 1024, 64
    B = bands_for(5, n, 5)
    with sbs.SharedLhs(5, B) as h:
        odd = torch.rand((n, m + 1), dtype=torch.float64, device=DEV)
        with pytest.raises(sbs.SbsError):
            sbs.sbs_solve_batch_partition(h.handle, odd, 1, 32, 2, 32, 2)
        # a view starting one element in: 8-byte aligned, not 16
        buf = torch.rand(n * m + 1, dtype=torch.float64, device=DEV)
        view = buf[1:].view(n, m)
        with pytest.raises(sbs.SbsError):
            sbs.sbs_solve_batch_partition(h.handle, view, 1, 32, 2, 32, 2)
        # AUTO still solves it (one system per lane)
        ref = oracle.solve(5, B, view.cpu().numpy())
        h.solve(view)
        torch.cuda.synchronize()
        assert colrel(view.cpu().numpy(), ref) <= TOL64


@pytest.mark.parametrize("n", [64, 512, 1024, 2048])
def test_periodic_shapes_match_periodic_oracle(n):
    rng = np.random.default_rng(n)
    a, c = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    B = np.stack([a, np.abs(a) + np.abs(c) + rng.uniform(1, 2, n), c])
    m = 96
    rhs = rng.uniform(-1, 1, (n, m))
    ref = oracle.solve(oracle.TRI_PERIODIC, B, rhs)
    ran = 0
    with sbs.SharedLhs(sbs.SBS_TRI_PERIODIC, B) as h:
        for lb, vec, S in SHAPES:
            got = shape_run(h, rhs, lb, vec, S, 2)
            if got is not None:
                assert colrel(got, ref) <= TOL64, (lb, vec, S)
                ran += 1
    assert ran > 0


@pytest.mark.parametrize("kind,n", [(3, 512), (5, 1024)])
def test_fp32_shapes(kind, n):
    # FP32 storage and arithmetic with the FP32 rounding of the FP64 plan:
    # within the same bound as the FP32 sweeps (a few hundred ulps of FP32
    # for these well-conditioned matrices)
    B = bands_for(kind, n, 9 + n)
    m = 256
    rhs = np.random.default_rng(n).uniform(-1, 1, (n, m)).astype(np.float32)
    ref = oracle.solve(kind, B, rhs.astype(np.float64))
    ran = 0
    with sbs.SharedLhs(kind, B) as h:
        for lb, vec, S in SHAPES:
            got = shape_run(h, rhs, lb, vec, S, 2, torch.float32)
            if got is not None:
                assert colrel(got, ref) <= 2e-5, (lb, vec, S, colrel(got, ref))
                ran += 1
    assert ran > 0


def test_constant_bands_full_size_sampled():
    # the benchmark's matrix and size: AUTO takes the separator form with
    # two systems per lane, and sampled columns (wave edges, group edges,
    # the last columns) match the oracle
    wl = W.config1()
    with sbs.SharedLhs(5, wl.bands) as h:
        x = torch.from_numpy(wl.rhs).to(DEV)
        shape = sbs.sbs_partition_shape(h.handle, x)
        print(f"AUTO shape for n=1024 m=65536: {shape}", flush=True)
        assert shape is not None and shape[0] == 1 and shape[2] == 2
        h.solve(x)
        torch.cuda.synchronize()
        cols = np.unique(np.r_[0, 1, 31, 32, 33, 63, 64, 65, 4095, 4096, 65534, 65535,
                               np.random.default_rng(1).integers(0, 65536, 200)])
        got = x[:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    ref = oracle.solve(5, wl.bands, wl.rhs[:, cols])
    assert colrel(got, ref) <= TOL64
    # manufactured solution: the right-hand side is A x_true
    assert colrel(got, wl.extra["x_true"][:, cols]) <= 1e-13


@pytest.mark.parametrize("kind,n,m", [(5, 2048, 640), (5, 3000, 130), (3, 4000, 96), (5, 1500, 64)])
def test_long_systems_read_the_plan_from_memory(kind, n, m):
    # systems whose plan (random bands: every block distinct) does not fit
    # the LDS: the factor rows, spikes and separator rows are read from
    # global memory, S^{-1} alone is in LDS (and, for the longest S^{-1},
    # the separators overwrite their right-hand sides)
    B = bands_for(kind, n, 77 + n)
    rhs = np.random.default_rng(n).uniform(-1, 1, (n, m))
    ref = oracle.solve(kind, B, rhs)
    ran = 0
    with sbs.SharedLhs(kind, B) as h:
        for lb, vec, S in [(32, 2, 16), (32, 2, 8), (64, 1, 16), (64, 1, 8), (64, 1, 4)]:
            print(f"case kind={kind} n={n} m={m} lb={lb} vec={vec} S={S}", flush=True)
            got = shape_run(h, rhs, lb, vec, S, 0)
            if got is not None:
                assert colrel(got, ref) <= TOL64, (lb, vec, S, colrel(got, ref))
                ran += 1
        # and whatever AUTO takes
        x = torch.from_numpy(rhs).to(DEV)
        print(f"AUTO shape: {sbs.sbs_partition_shape(h.handle, x)}", flush=True)
        h.solve(x)
        torch.cuda.synchronize()
        assert colrel(x.cpu().numpy(), ref) <= TOL64
    assert ran > 0


LONG = [(32, 2, 16), (32, 2, 8), (64, 1, 16), (64, 1, 8), (64, 1, 4)]


@pytest.mark.parametrize("kind,n,m,bands,shapes,flags", [
    (5, 1024, 1024, "hyper", [(32, 2, 32)], 0), (5, 1024, 514, "hyper", [(64, 1, 32)], 0),
    (5, 1024, 1000, "random", [(32, 2, 32)], 1), (3, 1000, 258, "random", [(32, 2, 32)], 0),
    (5, 2048, 640, "random", LONG, 16), (5, 3000, 130, "random", LONG, 16),
    (3, 1024, 256, "slow", [(32, 2, 32)], 0)])
def test_windowed_separator_product_equals_every_column(kind, n, m, bands, shapes, flags):
    # The plan drops entries of S^{-1} at most 2^-60 / Nr of their row's
    # largest, and each 16-row tile of the product reads only the columns
    # that hold the rest: bit for bit the product over every column (flags
    # bit 6), and within the parity bar of the oracle.  "slow": the
    # (-1, 2.01, -1) matrix, whose window is every column.
    if bands == "hyper":
        B = W.hyperdiffusion_bands(n, 0.5)
    elif bands == "slow":
        B = W.zero_outside(np.stack([-np.ones(n), np.full(n, 2.01), -np.ones(n)]))
    else:
        B = bands_for(kind, n, 900 + n)
    rhs = np.random.default_rng(n + m).uniform(-1, 1, (n, m))
    ref = oracle.solve(kind, B, rhs)
    ran = 0
    with sbs.SharedLhs(kind, B) as h:
        for lb, vec, S in shapes:
            print(f"case kind={kind} n={n} m={m} {bands} lb={lb} vec={vec} S={S} flags={flags}", flush=True)
            win = shape_run(h, rhs, lb, vec, S, flags)
            if win is None:
                continue
            print(f"case kind={kind} n={n} m={m} {bands} lb={lb} vec={vec} S={S} flags={flags | 64}", flush=True)
            full = shape_run(h, rhs, lb, vec, S, flags | 64)
            assert full is not None
            assert np.array_equal(win, full), (lb, vec, S)
            assert colrel(win, ref) <= TOL64, (lb, vec, S, colrel(win, ref))
            ran += 1
    assert ran > 0


@pytest.mark.parametrize("kind,n,m,bands,want", [
    (3, 2048, 2048, "adi", (1, 32, 2, 16)), (5, 1024, 2048, "hyper", (1, 32, 2, 16)),
    (5, 1024, 65536, "random", None), (5, 1024, 65536, "hyper", (1, 32, 2, 32)),
    (3, 256, 1024, "random", (0, 16, 1, 16)), (5, 512, 4096, "hyper", (1, 16, 1, 16)),
    (5, 384, 2048, "hyper", (1, 16, 1, 16)), (3, 1024, 4096, "random", (0, 32, 1, 16))])
def test_auto_shape_for_latency_bound_batches(kind, n, m, bands, want):
    # Where the pair form would take 64-row blocks of at most 16 systems
    # (128-byte runs: too few systems to fill the chip), AUTO takes the
    # separator form with 32-row blocks, two systems per lane and 16 per
    # workgroup; for pentadiagonal matrices, where it would take 32-row pair
    # blocks of at most 16 systems, 16-row separator blocks with one system
    # per lane.  Pair shapes with 256-byte runs, other pair shapes and
    # separator shapes that fill the chip stay as they were.
    if bands == "adi":
        B = W.diffusion_bands(n, 0.5)  # the ADI step's y matrix
    elif bands == "hyper":
        B = W.hyperdiffusion_bands(n, 0.5)
    else:
        B = bands_for(kind, n, 40 + n)
    with sbs.SharedLhs(kind, B) as h:
        x = torch.empty((n, m), dtype=torch.float64, device=DEV)
        got = sbs.sbs_partition_shape(h.handle, x)
        print(f"AUTO shape kind={kind} n={n} m={m} {bands}: {got}", flush=True)
        if want is None:  # a shape that fills the chip with 256-byte runs
            assert got[3] * 8 >= 256, got
        else:
            assert tuple(got) == want
        if m <= 2048:
            rhs = np.random.default_rng(n).uniform(-1, 1, (n, m))
            x.copy_(torch.from_numpy(rhs))
            h.solve(x)
            torch.cuda.synchronize()
            cols = np.r_[0, 1, 15, 16, 17, m // 2, m - 2, m - 1]
            ref = oracle.solve(kind, B, rhs[:, cols])
            assert colrel(x[:, torch.from_numpy(cols).to(DEV)].cpu().numpy(), ref) <= TOL64
