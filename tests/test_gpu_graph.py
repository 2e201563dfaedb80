"""Solves captured in a HIP graph (torch.cuda.CUDAGraph is hipGraph on ROCm):
the entry points launch kernels only (no allocation, no memset), so a caller
can capture them.  Each graph is replayed several times with eager work and
synchronisation between the replays, and every replay is compared bit for
bit with the eager result."""
import numpy as np
import pytest
import torch

from paper_1909_04539_amd import sbs, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def replays_match(step, x, rhs, want, times=3):
    for _ in range(3):  # warm: first launches set kernel attributes
        x.copy_(rhs)
        step(x)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    x.copy_(rhs)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step(x)
    for _ in range(times):
        x.copy_(rhs)                 # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, want)
        x.mul_(0.5)                  # more eager work on the same buffer
        torch.cuda.synchronize()


@pytest.mark.parametrize("kind,n,m", [(3, 256, 1024), (5, 1024, 4096), (3, 3000, 300)])
def test_solve_in_a_graph(kind, n, m):
    rng = np.random.default_rng(n + m)
    B = W.tri_dominant_bands(rng, n) if kind == 3 else W.hyperdiffusion_bands(n, 0.5)
    rhs = torch.from_numpy(rng.uniform(-1, 1, (n, m))).to(DEV)
    with sbs.SharedLhs(kind, B) as lhs:
        want = rhs.clone()
        lhs.solve(want)
        torch.cuda.synchronize()
        replays_match(lambda y: lhs.solve(y), torch.empty_like(rhs), rhs, want)


def test_cn_step_in_a_graph():
    n, m = 512, 2048
    B = np.stack([np.full(n, -0.3), np.full(n, 1.6), np.full(n, -0.3)])
    rhs = torch.from_numpy(np.random.default_rng(4).uniform(-1, 1, (n, m))).to(DEV)
    with sbs.SharedLhs(sbs.SBS_TRI_PERIODIC, B) as lhs:
        want = rhs.clone()
        lhs.cn_step(want, 2)
        torch.cuda.synchronize()
        replays_match(lambda y: lhs.cn_step(y, 2), torch.empty_like(rhs), rhs, want)
