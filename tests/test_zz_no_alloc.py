"""The allocation-free mixed-precision entry point against the one that takes a
workspace: the same kernels, so the same bits, on two calls in a row (the
second smaller), through the C ABI.  Also its size limit and that it does not
need the caller's scratch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1909_04539_amd import sbs, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(kind, n, seed):
    rng = np.random.default_rng(seed)
    if kind == 3:
        return W.tri_dominant_bands(rng, n)
    B = rng.uniform(-1, 1, (5, n))
    B[2] = np.sum(np.abs(np.delete(B, 2, axis=0)), axis=0) + rng.uniform(1, 2, n)
    return W.zero_outside(B)


@pytest.mark.parametrize("kind,n,ms", [(3, 2000, (3000, 700)), (5, 1500, (2048, 77)), (3, 256, (5000, 64))])
def test_noalloc_matches_workspace_entry_point(kind, n, ms):
    bands = _case(kind, n, 7 + n)
    h = sbs.SharedLhs(kind, bands)
    L = sbs.lib()
    st = torch.cuda.current_stream().cuda_stream
    print(f"kind {kind} n {n} m {ms}: fused={sbs.sbs_auto_variant(h.handle, ms[0]) == sbs.VARIANT_PARTITION}",
          flush=True)
    g = torch.Generator(device=DEV)
    g.manual_seed(n)
    for m in ms:
        b = (torch.rand((n, m), generator=g, device=DEV, dtype=torch.float64) * 2 - 1).float()
        need = sbs.sbs_refined_workspace_bytes(h.handle, m)
        work = torch.empty(need, dtype=torch.uint8, device=DEV)
        x_ref = torch.empty((n, m), dtype=torch.float64, device=DEV)
        assert L.sbs_solve_batch_refined(h.handle, b.data_ptr(), x_ref.data_ptr(), m, 2, work.data_ptr(),
                                         need, st) == 0
        x = torch.full((n, m), float("nan"), dtype=torch.float64, device=DEV)
        assert L.sbs_solve_batch_refined_noalloc(h.handle, b.data_ptr(), x.data_ptr(), m, 2, st) == 0
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref), (kind, n, m)
        # and against the oracle of the promoted FP32 right-hand sides
        cols = np.unique(np.r_[0, m - 1, np.random.default_rng(m).integers(0, m, 24)])
        ref = oracle.refine_reference(kind, bands, b.cpu().numpy()[:, cols])
        got = x.cpu().numpy()[:, cols]
        err = np.max(np.max(np.abs(got - ref), axis=0) / np.max(np.abs(ref), axis=0))
        assert err <= 1e-12, err
    h.close()


def test_noalloc_rejects_requests_beyond_its_scratch():
    n = 4000  # tridiagonal, beyond any fused plan: the multi-pass form needs n*m floats
    h = sbs.SharedLhs(3, _case(3, n, 3))
    cap = sbs.sbs_refined_static_scratch_bytes()
    m = cap // (4 * n) + 64
    assert sbs.sbs_refined_workspace_bytes(h.handle, m) > cap
    b = torch.zeros((n, m), dtype=torch.float32, device=DEV)
    x = torch.zeros((n, m), dtype=torch.float64, device=DEV)
    st = sbs.lib().sbs_solve_batch_refined_noalloc(h.handle, b.data_ptr(), x.data_ptr(), m, 2,
                                                   torch.cuda.current_stream().cuda_stream)
    assert st == 1  # SBS_ERR_INVALID_ARG, nothing queued
    torch.cuda.synchronize()
    assert not torch.any(x)
    h.close()
