"""GPU tests of the serving loop: every request's result is the same whether
it is solved alone (plain or mixed-precision entry point) or served in a mix
of overlapping requests, admission follows the HBM budget, and requests that
arrive while others run are admitted and overlap them."""
import ctypes
import threading
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1909_04539_amd import sbs, workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


class Server:
    def __init__(self, budget, streams=4, batch=0):
        self.L = sbs.lib()
        self.p = ctypes.c_void_p()
        st = self.L.sbs_server_create(budget, streams, batch, ctypes.byref(self.p))
        assert st == 0, st

    def register(self, h):
        i = ctypes.c_int32()
        assert self.L.sbs_server_register(self.p, h, ctypes.byref(i)) == 0
        return i.value

    def set_fp32_mode(self, mode):
        return self.L.sbs_server_set_fp32_mode(self.p, mode)

    def submit(self, lhs, t):
        tk = ctypes.c_uint64()
        st = self.L.sbs_server_submit(self.p, lhs, t.data_ptr(), t.shape[1],
                                      sbs.SBS_F64 if t.dtype == torch.float64 else sbs.SBS_F32, ctypes.byref(tk))
        return st, tk.value

    def wait(self, tk, timeout_us=-1):
        x = ctypes.c_void_p()
        lat = ctypes.c_double()
        st = self.L.sbs_server_wait(self.p, tk, timeout_us, ctypes.byref(x), ctypes.byref(lat))
        return st, x.value, lat.value

    def fetch(self, tk, n, m):
        out = torch.empty((n, m), dtype=torch.float64, device=DEV)
        st = self.L.sbs_server_fetch(self.p, tk, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        assert st == 0, st
        return out

    def release(self, tk):
        return self.L.sbs_server_release(self.p, tk)

    def stats(self):
        s = sbs.ServerStats()
        assert self.L.sbs_server_stats_get(self.p, ctypes.byref(s)) == 0
        return s

    def close(self):
        assert self.L.sbs_server_destroy(self.p) == 0


def make_lhs_set(count, n_lo, n_hi, seed=0):
    lhss = W.serving_lhs_set(seed=seed, count=count, n_lo=n_lo, n_hi=n_hi)
    return lhss, [sbs.SharedLhs(l.kind, l.bands) for l in lhss]


def alone(h, kind, rhs, variant=sbs.VARIANT_STREAM):
    """The request solved on its own through the plain entry points.  The
    serving tiles run the per-system sweeps (chunked or stream, which give
    identical bits), so that is the variant to compare bit for bit; AUTO may
    pick the partitioned variant, whose rounding differs."""
    if rhs.dtype == torch.float64:
        x = rhs.clone()
        sbs.sbs_solve_batch_variant(h.handle, x, variant)
        return x
    return h.solve_refined(rhs, sweeps=2)


def oracle_of(lhs, rhs_np):
    """The oracle's answer for one request: the FP64 solve of an FP64
    request, or of the exact FP64 promotion of an FP32 request's stored
    right-hand sides (the reference of the mixed-precision form)."""
    if rhs_np.dtype == np.float32:
        return oracle.refine_reference(lhs.kind, lhs.bands, rhs_np)
    return oracle.solve(lhs.kind, lhs.bands, rhs_np)


def col_err(got, ref):
    """max over systems of ||got_j - ref_j||_inf / ||ref_j||_inf"""
    return float(np.max(np.max(np.abs(got - ref), axis=0) / np.maximum(np.max(np.abs(ref), axis=0), 1e-300)))


def serve_all(srv, ids, trace, rhs, lhss):
    """Submit every request at once, then wait for each and fetch its FP64
    result to the host."""
    tickets = []
    for r, t in zip(trace, rhs):
        st, tk = srv.submit(ids[r.lhs], t)
        assert st == 0
        tickets.append(tk)
    out = []
    for r, tk in zip(trace, tickets):
        st, ptr, lat = srv.wait(tk)
        assert st == 0 and ptr
        got = srv.fetch(tk, lhss[r.lhs].n, r.m)
        torch.cuda.synchronize()
        out.append(got.cpu().numpy())
        assert srv.release(tk) == 0
    return out


def test_every_served_result_matches_the_oracle_alone_and_in_the_mix():
    # 16 matrices of 40..1500 rows plus one tridiagonal and one
    # pentadiagonal matrix above 4096 rows; 1200 overlapping requests, FP32
    # and FP64, submitted at once.
    lhss, hs = make_lhs_set(16, 40, 1500)
    rng = np.random.default_rng(99)
    for kind, n in ((3, 5000), (5, 6000)):
        B = W.tri_dominant_bands(rng, n) if kind == 3 else W.hyperdiffusion_bands(n, 0.7)
        lhss.append(W.Lhs(kind, B))
        hs.append(sbs.SharedLhs(kind, B))
    srv = Server(budget=4 << 30, streams=4)
    ids = [srv.register(h.handle) for h in hs]
    trace = W.serving_trace(rate_hz=1e6, count=1200, n_lhs=len(hs), m_max=300)
    rhs_np = [W.request_rhs(r, lhss[r.lhs].n) for r in trace]
    rhs = [torch.from_numpy(x).to(DEV) for x in rhs_np]
    assert any(lhss[r.lhs].n > 4096 and r.fp32 for r in trace)
    assert any(lhss[r.lhs].n > 4096 and not r.fp32 for r in trace)
    torch.cuda.synchronize()
    mix = serve_all(srv, ids, trace, rhs, lhss)
    s = srv.stats()
    print(f"served {s.completed} requests in {s.launches} launches; p50 {s.p50_us:.0f} us p99 {s.p99_us:.0f} us",
          flush=True)
    assert s.completed == len(trace) and s.launches < len(trace)   # requests were coalesced
    # 1. every served result against the oracle, at the stated tolerance
    worst = 0.0
    for k, r in enumerate(trace):
        err = col_err(mix[k], oracle_of(lhss[r.lhs], rhs_np[k]))
        assert err <= 1e-12, (k, r, err)
        worst = max(worst, err)
    print(f"largest error against the oracle over {len(trace)} served requests: {worst:.2e}", flush=True)
    # 2. the same request served alone gives the same bits as in the mix
    for k, r in enumerate(trace):
        alone_srv = serve_all(srv, ids, [r], [rhs[k]], lhss)[0]
        assert np.array_equal(alone_srv, mix[k]), (k, r)
    # 3. FP64 requests: the same bits as the plain entry point's per-system
    # sweep alone (AUTO may pick the partitioned variant: 1e-12 of it)
    for k, r in enumerate(trace):
        if r.fp32:
            continue
        ref = alone(hs[r.lhs], lhss[r.lhs].kind, rhs[k])
        torch.cuda.synchronize()
        assert np.array_equal(ref.cpu().numpy(), mix[k]), (k, r)
    srv.close()
    for h in hs:
        h.close()


def test_fp32_requests_as_one_fp64_sweep():
    # The server's second mode for FP32 requests: one FP64 sweep of the
    # stored FP32 values.  Every result against the oracle of the FP64
    # promotion at 1e-12, the same bits alone and in the mix, and the same
    # bits as the plain entry point's FP64 sweep of the promoted values;
    # requests submitted before the switch keep the refined form.
    lhss, hs = make_lhs_set(8, 40, 1500, seed=5)
    rng = np.random.default_rng(98)
    for kind, n in ((3, 5000), (5, 6000)):  # long enough to stream instead of checkpointing
        B = W.tri_dominant_bands(rng, n) if kind == 3 else W.hyperdiffusion_bands(n, 0.7)
        lhss.append(W.Lhs(kind, B))
        hs.append(sbs.SharedLhs(kind, B))
    srv = Server(budget=4 << 30, streams=4)
    assert srv.set_fp32_mode(7) == 1
    ids = [srv.register(h.handle) for h in hs]
    trace = W.serving_trace(rate_hz=1e6, count=400, n_lhs=len(hs), m_max=200, seed=3)
    rhs_np = [W.request_rhs(r, lhss[r.lhs].n) for r in trace]
    rhs = [torch.from_numpy(x).to(DEV) for x in rhs_np]
    assert any(lhss[r.lhs].n > 4096 and r.fp32 for r in trace)
    torch.cuda.synchronize()
    assert srv.set_fp32_mode(sbs.SERVE_F32_FP64_SWEEP) == 0
    mix = serve_all(srv, ids, trace, rhs, lhss)
    for k, r in enumerate(trace):
        err = col_err(mix[k], oracle_of(lhss[r.lhs], rhs_np[k]))
        assert err <= 1e-12, (k, r, err)
        if r.fp32:
            assert err <= 1e-13, (k, r, err)  # no FP32 arithmetic on the way
            x = rhs[k].double()
            sbs.sbs_solve_batch_variant(hs[r.lhs].handle, x, sbs.VARIANT_STREAM)
            torch.cuda.synchronize()
            assert np.array_equal(x.cpu().numpy(), mix[k]), (k, r)
    for k in range(0, len(trace), 7):
        assert np.array_equal(serve_all(srv, ids, [trace[k]], [rhs[k]], lhss)[0], mix[k]), k
    # back to the refined form: a request submitted now is refined again
    k = next(i for i, r in enumerate(trace) if r.fp32)
    assert srv.set_fp32_mode(sbs.SERVE_F32_REFINED) == 0
    again = serve_all(srv, ids, [trace[k]], [rhs[k]], lhss)[0]
    ref = alone(hs[trace[k].lhs], lhss[trace[k].lhs].kind, rhs[k])
    torch.cuda.synchronize()
    assert col_err(again, ref.cpu().numpy()) <= 1e-12
    srv.close()
    for h in hs:
        h.close()


def test_native_replay_of_a_trace():
    # the load generator the benchmark uses: 500 requests submitted at their
    # Poisson arrival times from a native thread, each waited for and
    # released by another; every latency is filled in and nothing stays
    # reserved
    lhss, hs = make_lhs_set(6, 40, 900, seed=2)
    srv = Server(budget=2 << 30, streams=4)
    ids = [srv.register(h.handle) for h in hs]
    trace = W.serving_trace(rate_hz=2e4, count=500, n_lhs=len(hs), m_max=256, seed=8)
    rhs = [torch.from_numpy(W.request_rhs(r, lhss[r.lhs].n)).to(DEV) for r in trace]
    torch.cuda.synchronize()
    st, lat, el = sbs.sbs_server_replay(
        srv.p, [ids[r.lhs] for r in trace], [t.data_ptr() for t in rhs], [r.m for r in trace],
        [sbs.SBS_F32 if r.fp32 else sbs.SBS_F64 for r in trace], [r.t_arrival * 1e6 for r in trace])
    assert st == 0, st
    assert np.all(lat >= 0) and el >= trace[-1].t_arrival
    s = srv.stats()
    assert s.completed == len(trace) and s.bytes_reserved == 0 and s.in_flight == 0
    srv.close()
    for h in hs:
        h.close()


def test_budget_admission_queueing_and_rejection():
    lhss, hs = make_lhs_set(2, 200, 200)
    n = lhss[0].n
    per = n * 64 * 8                                  # one FP64 request of m = 64
    srv = Server(budget=3 * per, streams=2)
    i0 = srv.register(hs[0].handle)
    big = torch.zeros((n, 1000), dtype=torch.float64, device=DEV)
    assert srv.submit(i0, big)[0] == 6                # larger than the whole budget
    rhs = [torch.rand((n, 64), dtype=torch.float64, device=DEV) for _ in range(8)]
    tks = [srv.submit(i0, t)[1] for t in rhs]
    # at most three fit; nobody releases, so the rest must queue
    for tk in tks[:3]:
        assert srv.wait(tk, 10_000_000)[0] == 0
    assert srv.wait(tks[3], 200_000)[0] == 8          # still queued: budget is held
    s = srv.stats()
    assert s.bytes_reserved <= 3 * per and s.queued >= 1 and s.rejected == 1
    for tk in tks[:3]:
        assert srv.release(tk) == 0
    for t, tk in zip(rhs[3:], tks[3:]):
        st, ptr, _ = srv.wait(tk, 10_000_000)
        assert st == 0
        assert torch.equal(srv.fetch(tk, n, 64), alone(hs[0], 3, t))
        assert srv.release(tk) == 0
    assert srv.release(tks[0]) == 7                   # already released
    srv.close()
    for h in hs:
        h.close()


def test_arrivals_during_running_work_are_admitted_and_overlap():
    # A long request keeps the GPU busy; short requests submitted afterwards
    # from another thread finish before it does.
    B = W.hyperdiffusion_bands(8192, 0.5)
    hl = sbs.SharedLhs(5, B)
    hs = sbs.SharedLhs(3, W.diffusion_bands(64, 0.5))
    srv = Server(budget=8 << 30, streams=4)
    il, ish = srv.register(hl.handle), srv.register(hs.handle)
    long_rhs = torch.rand((8192, 4096), dtype=torch.float32, device=DEV)
    short = [torch.rand((64, 8), dtype=torch.float64, device=DEV) for _ in range(20)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, tl = srv.submit(il, long_rhs)
    assert st == 0
    time.sleep(0.002)
    done_short = []

    def client():
        for t in short:
            s2, tk = srv.submit(ish, t)
            assert s2 == 0
            assert srv.wait(tk, 30_000_000)[0] == 0
            done_short.append((tk, time.perf_counter()))

    th = threading.Thread(target=client)
    th.start()
    th.join()
    st_long, _, lat_long = srv.wait(tl, 60_000_000)
    assert st_long == 0
    t_long_done = t0 + lat_long * 1e-6
    # short requests submitted after the long one finished while it still ran
    assert len(done_short) == len(short)
    first_short = min(t for _, t in done_short)
    print(f"long request {lat_long/1e3:.1f} ms; first short done at {(first_short - t0)*1e3:.1f} ms", flush=True)
    assert first_short < t_long_done
    assert srv.stats().launches >= 2
    for tk, _ in done_short:
        srv.release(tk)
    srv.release(tl)
    srv.close()
    hl.close()
    hs.close()


def test_small_request_completes_before_its_launch_ends():
    # One launch holding a large and a small request: with per-request
    # completion the small one is reported done before the large one.
    big_b = W.hyperdiffusion_bands(4096, 0.5)
    hb = sbs.SharedLhs(5, big_b)
    hsm = sbs.SharedLhs(3, W.diffusion_bands(64, 0.5))
    srv = Server(budget=4 << 30, streams=1)
    ib, ism = srv.register(hb.handle), srv.register(hsm.handle)
    big = torch.rand((4096, 65536), dtype=torch.float64, device=DEV)
    small = torch.rand((64, 64), dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    st1, tb = srv.submit(ib, big)
    st2, ts = srv.submit(ism, small)
    assert st1 == 0 and st2 == 0
    st, _, lat_s = srv.wait(ts, 60_000_000)
    assert st == 0
    st, _, lat_b = srv.wait(tb, 60_000_000)
    assert st == 0
    assert lat_s < lat_b
    assert torch.equal(srv.fetch(ts, 64, 64), alone(hsm, 3, small))
    srv.release(ts)
    srv.release(tb)
    srv.close()
    hb.close()
    hsm.close()
