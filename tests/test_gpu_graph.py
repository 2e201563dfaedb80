"""Solves, refined solves, Crank-Nicolson and ADI steps captured in a HIP graph
(torch.cuda.CUDAGraph is hipGraph on ROCm):
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


def test_refined_solve_in_a_graph():
    wl = W.config3(n=512, m=4096)
    b = torch.from_numpy(wl.rhs).to(DEV)
    with sbs.SharedLhs(3, wl.bands) as lhs:
        work = torch.empty(sbs.sbs_refined_workspace_bytes(lhs.handle, wl.m), dtype=torch.uint8, device=DEV)
        want = torch.empty((wl.n, wl.m), dtype=torch.float64, device=DEV)
        lhs.solve_refined(b, sweeps=2, x=want, work=work)
        torch.cuda.synchronize()
        x = torch.empty_like(want)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            lhs.solve_refined(b, sweeps=2, x=x, work=work)
        for _ in range(3):
            x.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(x, want)


def test_adi_step_in_a_graph():
    ny, nx = 256, 1024
    By, Bx = W.diffusion_bands(ny, 0.5), W.diffusion_bands(nx, 0.3)
    g0 = torch.from_numpy(np.random.default_rng(6).uniform(-1, 1, (ny, nx))).to(DEV)
    with sbs.SharedLhs(3, By) as hy, sbs.SharedLhs(3, Bx) as hx:
        work = torch.empty_like(g0)
        want = g0.clone()
        sbs.sbs_adi_step(hy.handle, hx.handle, want, work)
        torch.cuda.synchronize()
        replays_match(lambda y: sbs.sbs_adi_step(hy.handle, hx.handle, y, work), torch.empty_like(g0), g0, want)


def test_cn_step_in_a_graph():
    n, m = 512, 2048
    B = np.stack([np.full(n, -0.3), np.full(n, 1.6), np.full(n, -0.3)])
    rhs = torch.from_numpy(np.random.default_rng(4).uniform(-1, 1, (n, m))).to(DEV)
    with sbs.SharedLhs(sbs.SBS_TRI_PERIODIC, B) as lhs:
        want = rhs.clone()
        lhs.cn_step(want, 2)
        torch.cuda.synchronize()
        replays_match(lambda y: lhs.cn_step(y, 2), torch.empty_like(rhs), rhs, want)
