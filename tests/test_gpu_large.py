"""GPU parity at batch sizes whose 32- or 64-row chunks span more than 2 GiB,
so that the sweeps address rows through one buffer resource per row instead
of 31-bit offsets; the batch widths leave a ragged last wave.  Right-hand
sides are drawn on the device; sampled columns (first, last, around wave and
middle boundaries) are checked against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1909_04539_amd import sbs, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def colrel(x, ref):
    num = np.max(np.abs(x - ref), axis=0)
    den = np.maximum(np.max(np.abs(ref), axis=0), np.finfo(float).tiny)
    return float(np.max(num / den))


def sample_cols(m):
    return np.unique(np.array([0, 1, 63, 64, 65, m // 2 - 1, m // 2, m - 65, m - 64, m - 2, m - 1]))


def random_rhs(n, m, dtype, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    return torch.rand((n, m), dtype=dtype, device=DEV, generator=g) * 2 - 1


def tri_bands(n, seed, periodic=False):
    rng = np.random.default_rng(seed)
    a, c = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    B = np.stack([a, np.abs(a) + np.abs(c) + rng.uniform(1, 2, n), c])
    return B if periodic else W.zero_outside(B)


def check(kind, B, x_dev, rhs_cols, cols, ref_fn=None, tol=1e-12):
    got = x_dev[:, torch.from_numpy(cols).to(DEV)].double().cpu().numpy()
    ref = (ref_fn or (lambda b: oracle.solve(kind, B, b)))(rhs_cols)
    assert colrel(got, ref) <= tol


@pytest.mark.parametrize("variant", [sbs.VARIANT_CHUNKED, sbs.VARIANT_STREAM, sbs.VARIANT_AUTO])
def test_fp64_chunks_past_2gib(variant):
    n, m = 65, (1 << 23) + 3            # 32 rows x m x 8 B > 2 GiB
    print(f"case n={n} m={m} variant={variant}", flush=True)
    B = tri_bands(n, 1)
    x = random_rhs(n, m, torch.float64, 2)
    cols = sample_cols(m)
    rhs_cols = x[:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    with sbs.SharedLhs(3, B) as lhs:
        lhs.solve(x, variant)
        torch.cuda.synchronize()
    check(3, B, x, rhs_cols, cols)
    del x
    torch.cuda.empty_cache()


def test_fp64_resident_chunk_past_2gib():
    n, m = 40, (1 << 22) + 5            # one 64-row chunk x m x 8 B > 2 GiB
    B = tri_bands(n, 3)
    x = random_rhs(n, m, torch.float64, 4)
    cols = sample_cols(m)
    rhs_cols = x[:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    with sbs.SharedLhs(3, B) as lhs:
        lhs.solve(x, sbs.VARIANT_RESIDENT)
        torch.cuda.synchronize()
    check(3, B, x, rhs_cols, cols)
    del x
    torch.cuda.empty_cache()


def test_fp32_chunks_past_2gib():
    n, m = 65, (1 << 24) + 7            # 32 rows x m x 4 B > 2 GiB
    B = tri_bands(n, 5)
    x = random_rhs(n, m, torch.float32, 6)
    cols = sample_cols(m)
    rhs_cols = x[:, torch.from_numpy(cols).to(DEV)].double().cpu().numpy()
    with sbs.SharedLhs(3, B) as lhs:
        lhs.solve(x, sbs.VARIANT_CHUNKED)
        torch.cuda.synchronize()
    check(3, B, x, rhs_cols, cols, tol=1e-5)
    del x
    torch.cuda.empty_cache()


def test_cn_step_chunks_past_2gib():
    # periodic, 65 rows: no partition plan, so the Crank-Nicolson sweep kernel
    n, m = 65, (1 << 23) + 3
    B = tri_bands(n, 7, periodic=True)
    x = random_rhs(n, m, torch.float64, 8)
    cols = sample_cols(m)
    rhs_cols = x[:, torch.from_numpy(cols).to(DEV)].cpu().numpy()
    with sbs.SharedLhs(sbs.SBS_TRI_PERIODIC, B) as lhs:
        assert sbs.sbs_auto_variant(lhs.handle, m) != sbs.VARIANT_PARTITION
        lhs.cn_step(x, 2)
        torch.cuda.synchronize()
    check(13, B, x, rhs_cols, cols, ref_fn=lambda b: oracle.cn_steps(oracle.TRI_PERIODIC, B, b, 2))
    del x
    torch.cuda.empty_cache()
