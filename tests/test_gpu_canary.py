"""Guard bands: no kernel reads its way into a fault or writes outside the
arrays it was given.  Every device array a call writes is placed inside a
larger buffer whose guard elements before and after it hold a sentinel bit
pattern; after the call (and a synchronisation) the guards must be
bit-identical, and the result must still match the oracle.  Shapes are
ragged on purpose: m not a multiple of the wave, the workgroup's systems or
two, n not a multiple of any block length."""
import numpy as np
import pytest
import torch

import oracle
from paper_1909_04539_amd import sbs, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GUARD = 4096          # elements on each side (an even count keeps 16-byte alignment)
SENTINEL = 0x7FF4DEADBEEF0A5A  # a NaN payload no kernel computes


def guarded(values, dtype=torch.float64):
    """A device tensor holding `values` with GUARD sentinel elements on each
    side; returns (buffer, view)."""
    n, m = values.shape
    itype = torch.int64 if dtype == torch.float64 else torch.int32
    sent = SENTINEL if dtype == torch.float64 else 0x7FA5A5A5
    buf = torch.full((2 * GUARD + n * m,), sent, dtype=itype, device=DEV).view(dtype)
    view = buf[GUARD:GUARD + n * m].view(n, m)
    view.copy_(torch.from_numpy(np.ascontiguousarray(values)).to(DEV, dtype))
    return buf, view


def guards_intact(buf, count):
    itype = torch.int64 if buf.dtype == torch.float64 else torch.int32
    sent = SENTINEL if buf.dtype == torch.float64 else 0x7FA5A5A5
    raw = buf.view(itype)
    torch.cuda.synchronize()
    return bool(torch.all(raw[:GUARD] == sent)) and bool(torch.all(raw[GUARD + count:] == sent))


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


CASES = [(3, 37, 65), (5, 37, 130), (3, 250, 97), (5, 1000, 99), (5, 1003, 66), (3, 3001, 70), (5, 5000, 33)]


@pytest.mark.parametrize("kind,n,m", CASES)
@pytest.mark.parametrize("variant", [sbs.VARIANT_AUTO, sbs.VARIANT_RESIDENT, sbs.VARIANT_CHUNKED,
                                     sbs.VARIANT_STREAM, sbs.VARIANT_PARTITION])
def test_solve_variants_stay_inside(kind, n, m, variant):
    B = bands_for(kind, n, n + m)
    rhs = np.random.default_rng(n * m).uniform(-1, 1, (n, m))
    with sbs.SharedLhs(kind, B) as h:
        buf, x = guarded(rhs)
        try:
            sbs.sbs_solve_batch_variant(h.handle, x, variant)
        except sbs.SbsError as e:
            assert e.status == 1  # variant not available for this size
            assert guards_intact(buf, n * m)
            return
        assert guards_intact(buf, n * m), (kind, n, m, variant)
        assert colrel(x.cpu().numpy(), oracle.solve(kind, B, rhs)) <= 1e-12


@pytest.mark.parametrize("kind,n,m", [(3, 1000, 99), (5, 1000, 130), (5, 1024, 66), (3, 100, 7)])
def test_every_partition_shape_stays_inside(kind, n, m):
    B = bands_for(kind, n, 2 * n + m)
    rhs = np.random.default_rng(m).uniform(-1, 1, (n, m))
    ref = oracle.solve(kind, B, rhs)
    ran = 0
    with sbs.SharedLhs(kind, B) as h:
        for form in (0, 1):
            for lb in (16, 32, 64):
                for vec in ((1,) if form == 0 else (1, 2)):
                    for S in (64, 32, 16, 8, 2):
                        for flags in ((0,) if form == 0 else (0, 1, 4 | (1 << 8))):
                            buf, x = guarded(rhs)
                            try:
                                sbs.sbs_solve_batch_partition(h.handle, x, form, lb, vec, S, flags)
                            except sbs.SbsError:
                                assert guards_intact(buf, n * m)
                                continue
                            assert guards_intact(buf, n * m), (form, lb, vec, S, flags)
                            assert colrel(x.cpu().numpy(), ref) <= 1e-12, (form, lb, vec, S, flags)
                            ran += 1
    assert ran > 0


@pytest.mark.parametrize("kind,n,m", [(3, 300, 65), (5, 1000, 99), (13, 512, 70), (5, 3000, 33)])
def test_crank_nicolson_stays_inside(kind, n, m):
    if kind == 13:
        rng = np.random.default_rng(n)
        a, c = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        B = np.stack([a, np.abs(a) + np.abs(c) + rng.uniform(1, 2, n), c])
    else:
        B = bands_for(kind, n, n)
    C = np.random.default_rng(m).uniform(-1, 1, (n, m))
    with sbs.SharedLhs(kind, B) as h:
        buf, c = guarded(C)
        h.cn_step(c, 2)
        assert guards_intact(buf, n * m)
        assert colrel(c.cpu().numpy(), oracle.cn_steps(kind, B, C, 2)) <= 1e-12


@pytest.mark.parametrize("kind,n,m", [(3, 512, 1000), (3, 2000, 130), (5, 1000, 77), (5, 3000, 66)])
def test_refined_stays_inside(kind, n, m):
    B = bands_for(kind, n, n + 1)
    b_np = np.random.default_rng(m).uniform(-1, 1, (n, m)).astype(np.float32)
    with sbs.SharedLhs(kind, B) as h:
        bbuf, b = guarded(b_np, torch.float32)
        xbuf, x = guarded(np.zeros((n, m)))
        need = sbs.sbs_refined_workspace_bytes(h.handle, m)
        wbuf, work = guarded(np.zeros((1, max(1, need // 8) + 1)))
        sbs.sbs_solve_batch_refined(h.handle, b, x=x, sweeps=2, work=work.view(torch.uint8).view(-1))
        assert guards_intact(bbuf, n * m) and guards_intact(xbuf, n * m)
        assert guards_intact(wbuf, work.numel())
        assert torch.equal(b.cpu(), torch.from_numpy(b_np))  # read only
        ref = oracle.refine_reference(kind, B, b_np)
        assert colrel(x.cpu().numpy(), ref) <= 1e-12
        # the allocation-free form, same guards
        xbuf2, x2 = guarded(np.zeros((n, m)))
        sbs.sbs_solve_batch_refined_noalloc(h.handle, b, x2)
        assert guards_intact(xbuf2, n * m) and torch.equal(x2, x)


@pytest.mark.parametrize("ny,nx", [(100, 77), (257, 1000), (2048, 130)])
def test_transpose_and_adi_stay_inside(ny, nx):
    G = np.random.default_rng(ny).uniform(-1, 1, (ny, nx))
    sbuf, src = guarded(G)
    dbuf, dst = guarded(np.zeros((nx, ny)))
    sbs.sbs_transpose(src, dst)
    assert guards_intact(sbuf, ny * nx) and guards_intact(dbuf, ny * nx)
    assert torch.equal(dst.cpu(), torch.from_numpy(G.T.copy()))
    By, Bx = W.diffusion_bands(ny, 0.5), W.diffusion_bands(nx, 0.5)
    with sbs.SharedLhs(3, By) as hy, sbs.SharedLhs(3, Bx) as hx:
        gbuf, g = guarded(G)
        wbuf, work = guarded(np.zeros((ny, nx)))
        sbs.sbs_adi_step(hy.handle, hx.handle, g, work)
        assert guards_intact(gbuf, ny * nx) and guards_intact(wbuf, ny * nx)
        assert colrel(g.cpu().numpy(), oracle.adi_step(By, Bx, G)) <= 1e-12
