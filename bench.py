"""Benchmark: shared-LHS batched solves on one MI355X.

Headline (the JSON line's `value`): right-hand-side unknowns solved per
second for the pentadiagonal FP64 workload -- n = 1024 unknowns, m = 65536
systems sharing one matrix (1-D hyperdiffusion Crank--Nicolson step, s = 0.5)
-- one in-place solve per step, inputs resident in HBM.  Beside it: the
roofline of the kernel that runs it (algorithmic 16 B per unknown against 8 TB/s),
the oracle timed on the host cores, and the other workloads (long
pentadiagonal systems with random bands, tridiagonal
n=256 batch, 2-D ADI step, mixed-precision refinement, serving).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--only headline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1909_04539_amd", "csrc")
# source file of each kernel the headline may run
KERNEL_SOURCE = {"k_sep": os.path.join(CSRC, "sep.hip"), "k_part": os.path.join(CSRC, "kernels.hip"),
                 "k_sweep": os.path.join(CSRC, "kernels.hip")}
VARIANTS = {"auto": 0, "resident": 1, "chunked": 2, "stream": 3, "partition": 4}
# kernel that runs each variant of the headline solve
KERNEL_OF = {1: "k_sweep", 2: "k_sweep", 3: "k_sweep", 4: "k_part"}


def traffic_file(kernel):
    return os.path.join(ROOT, "profiles", f"{kernel}_penta_f64_n1024_m65536.json")


def measured_traffic(kernel):
    """HBM bytes per launch of the headline kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by the copy calibration),
    or None if the kernel source has changed since they were taken."""
    import hashlib
    try:
        rec = json.load(open(traffic_file(kernel)))
        sha = hashlib.sha256(open(KERNEL_SOURCE[kernel], "rb").read()).hexdigest()
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    return round(rec["traffic_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(step, K, W, torch):
    """W untimed steps, then K timed steps bracketed by synchronisation; HIP
    events on the launch stream give the device time of the same region."""
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(K):
        step()
    e1.record(s)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / K
    dev = e0.elapsed_time(e1) * 1e-3 / K
    return wall, dev


def host_cpu():
    """The host the oracle runs on: usable cores and the CPU model (the
    `model name` field that lscpu also prints)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "model": model}


def _median_host(fn, X, src, reps=5):
    """Median wall time of `reps` runs of fn(X), X restored from src before
    each (untimed)."""
    ts = []
    for _ in range(reps):
        X[...] = src
        t = time.perf_counter()
        fn(X)
        ts.append(time.perf_counter() - t)
    return sorted(ts)[reps // 2]


def cpu_baseline(kind, bands, rhs_sample, target_s=10.0):
    """The oracle (C, OpenMP over column blocks) on a bounded sample: the
    median of 5 timed solves on all host cores and on one thread, after
    repeated solves for about `target_s` seconds."""
    import oracle
    threads = oracle.max_threads()
    X = rhs_sample.copy()
    n, m = X.shape
    reps, t0 = 0, time.perf_counter()
    while True:                                   # warm the caches and the thread team
        X[...] = rhs_sample
        oracle.solve_inplace_mt(kind, bands, X, threads)
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= 1000:
            break
    per = _median_host(lambda Y: oracle.solve_inplace_mt(kind, bands, Y, threads), X, rhs_sample)
    one = _median_host(lambda Y: oracle.solve_inplace_mt(kind, bands, Y, 1), X, rhs_sample)
    return {"value": n * m / per, "unit": "unknowns/s", "cores": threads, "kind": "oracle",
            "value_1_thread": n * m / one, "host": host_cpu(),
            "sample": f"n={n}, m={m} columns of the same workload (seeded); median of 5 timed solves "
                      f"(input restored untimed) after {reps} warm-up solves over {el:.1f} s; "
                      f"value_1_thread: median of 5 on one thread"}


def cpu_other_configs(W):
    """The oracle on the other workloads (medians of 5, inputs restored
    untimed): the tridiagonal n=256 batch (whole), the ADI step at 2048^2
    (whole, serial: columns then rows), and the mixed-precision workload's
    reference (the FP64 solve of the promoted FP32 right-hand sides) on its
    first 65536 of 2^20 columns."""
    import oracle
    threads = oracle.max_threads()
    out = {"cores": threads, "host": host_cpu()}
    wl = W.config0()
    X = wl.rhs.copy()
    t = _median_host(lambda Y: oracle.solve_inplace_mt(3, wl.bands, Y, threads), X, wl.rhs)
    t1 = _median_host(lambda Y: oracle.solve_inplace_mt(3, wl.bands, Y, 1), X, wl.rhs)
    out["tri_f64_n256_m1024"] = {"unknowns_per_s": wl.n * wl.m / t, "unknowns_per_s_1_thread": wl.n * wl.m / t1,
                                 "us_per_solve": t * 1e6}
    wl = W.config2()
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.adi_step(wl.bands, wl.extra["bands_x"], wl.rhs)
        ts.append(time.perf_counter() - t0)
    t = sorted(ts)[2]
    out["adi_f64_2048x2048"] = {"points_per_s": wl.n * wl.m / t, "ms_per_step": t * 1e3, "threads": 1}
    wl = W.config3()
    src = np.ascontiguousarray(wl.rhs[:, :65536].astype(np.float64))
    X = src.copy()
    t = _median_host(lambda Y: oracle.solve_inplace_mt(3, wl.bands, Y, threads), X, src)
    out["refined_reference_n512"] = {"unknowns_per_s": src.size / t, "sample": "first 65536 of 2^20 columns"}
    return out


def bench_headline(args, torch, sbs, W):
    wl = W.config1()
    n, m = wl.n, wl.m
    rhs = torch.from_numpy(wl.rhs).to("cuda:0")
    lhs = sbs.SharedLhs(5, wl.bands)
    variant = VARIANTS[args.variant]
    ran = variant if variant else sbs.sbs_auto_variant(lhs.handle, m)
    kernel = KERNEL_OF[ran]
    shape = None
    if ran == VARIANTS["partition"]:
        shape = sbs.sbs_partition_shape(lhs.handle, rhs)       # (form, lb, vec, S)
        kernel = "k_sep" if shape and shape[0] == 1 else "k_part"
    step = lambda: lhs.solve(rhs, variant)
    wall, dev = timed_steps(step, args.steps, args.warmup, torch)
    # the kernel alone, two more ways: the median of 20 back-to-back launches
    # each bracketed by its own events, and the median of 20 launches with
    # the right-hand side restored from a pristine copy (untimed) before each,
    # so that every launch solves the same input (the copy leaves part of the
    # input written back to memory only during the solve, which costs it
    # some bandwidth)
    b2b, _ = _event_median(step, 20, 3, torch)
    pristine = rhs.clone()
    med, mn = _event_median(step, 20, 3, torch, restore=lambda: rhs.copy_(pristine))
    del pristine
    unknowns = n * m
    # roofline over the timed region: the average device time per launch of
    # the K timed steps, the figure a kernel trace of this run averages
    achieved = 16.0 * unknowns / dev / 1e9
    res = {
        "wall_s": wall, "dev_s": dev, "unknowns": unknowns,
        "variant": {v: k for k, v in VARIANTS.items()}[ran], "kernel": kernel,
        "shape": None if shape is None else {"form": ["pair", "separator"][shape[0]], "lb": shape[1],
                                             "systems_per_lane": shape[2], "systems_per_workgroup": shape[3]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(kernel),
                     "kernel": kernel, "kernel_us_mean_of_timed_steps": round(dev * 1e6, 2),
                     "kernel_us_median_back_to_back": round(b2b * 1e6, 2),
                     "kernel_us_median_restored": round(med * 1e6, 2), "kernel_us_min_restored": round(mn * 1e6, 2),
                     "frac_restored": round(16.0 * unknowns / med / 1e9 / HBM_PEAK_GBS, 4),
                     "timing": "achieved = algorithmic bytes / mean kernel time of the K timed steps (HIP events "
                               "on the launch stream around the timed region); also the median of 20 back-to-back "
                               "launches and of 20 launches each after an untimed restore of the input"},
        "cpu_sample": wl.rhs[:, :8192].copy(), "bands": wl.bands,
    }
    lhs.close()
    del rhs
    return res


def bench_penta_general(args, torch, sbs, W):
    """The headline's size with a general matrix: random diagonally dominant
    bands, so no two partition blocks share a stored copy."""
    n, m = 1024, 65536
    rng = np.random.default_rng(11)
    B = rng.uniform(-1, 1, (5, n))
    B[2] = np.sum(np.abs(np.delete(B, 2, axis=0)), axis=0) + rng.uniform(1, 2, n)
    B = W.zero_outside(B)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(12)
    rhs = torch.rand((n, m), dtype=torch.float64, device="cuda:0", generator=g)
    lhs = sbs.SharedLhs(5, B)
    ran = sbs.sbs_auto_variant(lhs.handle, m)
    wall, dev = timed_steps(lambda: lhs.solve(rhs), 20, 3, torch)
    lhs.close()
    u = n * m
    return {"workload": "penta_f64_n1024_m65536_random_bands", "variant": {v: k for k, v in VARIANTS.items()}[ran],
            "unknowns_per_s": u / dev, "us_per_solve": dev * 1e6, "hbm_frac_16B": round(16 * u / dev / 1e9 / HBM_PEAK_GBS, 4)}


def bench_penta_large(args, torch, sbs, W):
    """Pentadiagonal systems of 2048 rows with random diagonally dominant
    bands (every block of a partition plan distinct): what AUTO runs (the
    separator form with its plan read from global memory, 16 systems per
    workgroup), beside the chunked sweep (24 B per unknown moved, of 16 B
    algorithmic)."""
    n, m = 2048, 65536
    rng = np.random.default_rng(21)
    B = rng.uniform(-1, 1, (5, n))
    B[2] = np.sum(np.abs(np.delete(B, 2, axis=0)), axis=0) + rng.uniform(1, 2, n)
    B = W.zero_outside(B)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(22)
    rhs = torch.rand((n, m), dtype=torch.float64, device="cuda:0", generator=g)
    lhs = sbs.SharedLhs(5, B)
    ran = sbs.sbs_auto_variant(lhs.handle, m)
    shape = sbs.sbs_partition_shape(lhs.handle, rhs) if ran == VARIANTS["partition"] else None
    wall, dev = timed_steps(lambda: lhs.solve(rhs), 10, 2, torch)
    wall, dev_chunked = timed_steps(lambda: lhs.solve(rhs, VARIANTS["chunked"]), 10, 2, torch)
    lhs.close()
    u = n * m
    return {"workload": "penta_f64_n2048_m65536_random_bands", "variant": {v: k for k, v in VARIANTS.items()}[ran],
            "shape": None if shape is None else {"form": ["pair", "separator"][shape[0]], "block_rows": shape[1],
                                                 "systems_per_lane": shape[2], "systems_per_workgroup": shape[3]},
            "unknowns_per_s": u / dev, "us_per_solve": dev * 1e6,
            "hbm_frac_16B": round(16 * u / dev / 1e9 / HBM_PEAK_GBS, 4),
            "chunked_us_per_solve": dev_chunked * 1e6}


def bench_periodic_and_cn(args, torch, sbs, W):
    """Periodic tridiagonal solves (Section 3.3) and Crank-Nicolson steps of
    the paper's two benchmark schemes (Sections 3.2, 4.2) at the headline's
    size: diffusion on a periodic grid, a = c = -s, b = 1 + 2s, and
    hyperdiffusion with truncated ends, s = 0.5.  One step is one solve or
    one Crank-Nicolson step (explicit half fused) of all m systems."""
    n, m = 1024, 65536
    s = 0.5
    g = torch.Generator(device="cuda:0")
    g.manual_seed(13)
    c = torch.rand((n, m), dtype=torch.float64, device="cuda:0", generator=g)
    ring = np.stack([np.full(n, -s), np.full(n, 1 + 2 * s), np.full(n, -s)])
    out = {}
    hp = sbs.SharedLhs(sbs.SBS_TRI_PERIODIC, ring)
    hh = sbs.SharedLhs(5, W.hyperdiffusion_bands(n, s))
    u = n * m
    for name, fn in (("tri_periodic_solve", lambda: hp.solve(c)),
                     ("cn_step_periodic_diffusion", lambda: hp.cn_step(c)),
                     ("cn_step_hyperdiffusion", lambda: hh.cn_step(c))):
        wall, dev = timed_steps(fn, 20, 3, torch)
        out[name] = {"us_per_step": round(dev * 1e6, 1), "unknowns_per_s": u / dev,
                     "hbm_frac_16B": round(16 * u / dev / 1e9 / HBM_PEAK_GBS, 4)}
    out["workload"] = "n1024_m65536_f64"
    out["variant"] = {v: k for k, v in VARIANTS.items()}[sbs.sbs_auto_variant(hp.handle, m)]
    hp.close()
    hh.close()
    return out


def mall_flush(torch):
    """A function that overwrites 1 GiB of device memory (more than the
    256 MB last-level cache and the L2s together), for cold-cache timing."""
    junk = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0")
    return lambda: junk.fill_(1.0)


def bench_tri256(args, torch, sbs, W):
    """Back-to-back calls from Python, the kernel alone (per-launch events,
    warm and with the caches flushed before each launch), and the same
    solves replayed from a HIP graph (50 solves per replay), which leaves out
    the host's cost per call."""
    wl = W.config0()
    rhs = torch.from_numpy(wl.rhs).to("cuda:0")
    lhs = sbs.SharedLhs(3, wl.bands)
    wall, dev = timed_steps(lambda: lhs.solve(rhs), 200, 20, torch)
    pristine = rhs.clone()
    warm, _ = _event_median(lambda: lhs.solve(rhs), 50, 5, torch, restore=lambda: rhs.copy_(pristine))
    flush = mall_flush(torch)
    cold, _ = _event_median(lambda: lhs.solve(rhs), 20, 3, torch,
                            restore=lambda: (rhs.copy_(pristine), flush()))
    del flush
    x = rhs.clone()
    per_graph = 50
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        for _ in range(per_graph):
            lhs.solve(x)
    _, gdev = timed_steps(lambda: g.replay(), 10, 2, torch)
    lhs.close()
    u = wl.n * wl.m
    return {"workload": "tri_f64_n256_m1024", "unknowns_per_s": u / dev, "us_per_solve": dev * 1e6,
            "hbm_frac_16B": round(16 * u / dev / 1e9 / HBM_PEAK_GBS, 4),
            "us_kernel_median_warm": warm * 1e6, "us_kernel_median_cold": cold * 1e6,
            "us_per_solve_graph": gdev / per_graph * 1e6,
            "bound": "latency: back-to-back calls from Python cost about 10 us of host work each; "
                     "us_per_solve_graph is the device's own time per solve; cold = 1 GiB written "
                     "between the input's restore and the launch (median of 20)"}


def bench_adi(args, torch, sbs, W):
    wl = W.config2()
    g = torch.from_numpy(wl.rhs).to("cuda:0")
    work = torch.empty_like(g)
    hy, hx = sbs.SharedLhs(3, wl.bands), sbs.SharedLhs(3, wl.extra["bands_x"])
    step = lambda: sbs.sbs_adi_step(hy.handle, hx.handle, g, work)
    wall, dev = timed_steps(step, 20, 3, torch)
    pristine = g.clone()
    warm, _ = _event_median(step, 20, 3, torch, restore=lambda: g.copy_(pristine))
    flush = mall_flush(torch)
    cold, _ = _event_median(step, 20, 3, torch, restore=lambda: (g.copy_(pristine), flush()))
    del flush
    hy.close()
    hx.close()
    pts = wl.n * wl.m
    return {"workload": "adi_f64_2048x2048", "points_per_s": pts / dev, "unknowns_per_s": 2 * pts / dev,
            "ms_per_step": dev * 1e3, "hbm_frac_32B_per_point": round(32 * pts / dev / 1e9 / HBM_PEAK_GBS, 4),
            "us_median_warm": warm * 1e6, "us_median_cold": cold * 1e6,
            "bound": "latency: 2048 systems per solve do not fill the chip; cold = 1 GiB written between "
                     "the grid's restore and the step (median of 20)"}


def bench_refined(args, torch, sbs, W):
    wl = W.config3()
    n, m = wl.n, wl.m
    b = torch.from_numpy(wl.rhs).to("cuda:0")
    x = torch.empty((n, m), dtype=torch.float64, device="cuda:0")
    lhs = sbs.SharedLhs(3, wl.bands)
    work = torch.empty(sbs.sbs_refined_workspace_bytes(lhs.handle, m), dtype=torch.uint8, device="cuda:0")
    step = lambda: lhs.solve_refined(b, sweeps=2, x=x, work=work)
    wall, dev = timed_steps(step, 20, 3, torch)
    u = n * m
    out = {"workload": "tri_refine_f32in_f64out_n512_m1048576", "unknowns_per_s": u / dev, "ms_per_solve": dev * 1e3,
           "hbm_frac_12B_io_min": round(12 * u / dev / 1e9 / HBM_PEAK_GBS, 4)}
    # plain FP64 on the same shape, for comparison
    x.copy_(b)
    wall, dev64 = timed_steps(lambda: lhs.solve(x), 20, 3, torch)
    out["plain_f64_unknowns_per_s"] = u / dev64
    out["plain_f64_hbm_frac_16B"] = round(16 * u / dev64 / 1e9 / HBM_PEAK_GBS, 4)
    # accuracy on sampled columns against the FP64 oracle of double(b32)
    import oracle
    # (err_k: after k correction rounds; the bench's solve uses two)
    cols = np.random.default_rng(3).choice(m, 64, replace=False)
    ref = oracle.refine_reference(3, wl.bands, wl.rhs[:, cols])
    for k in (0, 1, 2):
        xs = lhs.solve_refined(b, sweeps=k, x=x, work=work)[:, torch.from_numpy(cols).cuda()].cpu().numpy()
        out[f"err{k}_max_col_rel_vs_oracle"] = float(np.max(np.max(np.abs(xs - ref), axis=0) /
                                                            np.max(np.abs(ref), axis=0)))
    out["max_col_rel_err_vs_oracle"] = out["err2_max_col_rel_vs_oracle"]
    lhs.close()
    return out


class _Server:
    """Minimal client of the C-ABI serving loop (argument marshalling only)."""

    def __init__(self, sbs, budget, streams=4):
        import ctypes
        self.ct, self.L = ctypes, sbs.lib()
        self.p = ctypes.c_void_p()
        st = self.L.sbs_server_create(budget, streams, 0, ctypes.byref(self.p))
        if st:
            raise RuntimeError(f"sbs_server_create: {st}")

    def register(self, h):
        i = self.ct.c_int32()
        assert self.L.sbs_server_register(self.p, h, self.ct.byref(i)) == 0
        return i.value

    def set_fp32_mode(self, mode):
        assert self.L.sbs_server_set_fp32_mode(self.p, mode) == 0

    def submit(self, lhs, ptr, m, dtype):
        tk = self.ct.c_uint64()
        st = self.L.sbs_server_submit(self.p, lhs, ptr, m, dtype, self.ct.byref(tk))
        if st:
            raise RuntimeError(f"sbs_server_submit: {st}")
        return tk.value

    def wait_release(self, tk):
        x, lat = self.ct.c_void_p(), self.ct.c_double()
        st = self.L.sbs_server_wait(self.p, tk, -1, self.ct.byref(x), self.ct.byref(lat))
        self.L.sbs_server_release(self.p, tk)
        return st, lat.value

    def stats(self, sbs):
        s = sbs.ServerStats()
        self.L.sbs_server_stats_get(self.p, self.ct.byref(s))
        return s

    def close(self):
        self.L.sbs_server_destroy(self.p)


def serving_cpu_oracle(lhss, trace, pool64_host, offs, loads, budget_s):
    """The oracle serving the same requests on the host cores, one request
    at a time in arrival order (FIFO): each request's service time is
    measured (the C oracle, OpenMP over column blocks; FP32 requests are
    solved in FP64 from their promoted values, the reference of the mixed
    precision form), on the longest prefix of the trace that fits in
    `budget_s` seconds of service.  Arrivals keep the trace's shape, rescaled
    to each offered load of the host's own saturation rate, and latencies
    (arrival to completion, queueing included) follow from the measured
    service times: completion_k = max(arrival_k, completion_{k-1}) + S_k."""
    import oracle
    threads = oracle.max_threads()
    serv = []
    unknowns = 0.0
    t_all = time.perf_counter()
    for k, r in enumerate(trace):
        L = lhss[r.lhs]
        X = pool64_host[offs[k]:offs[k] + L.n * r.m].reshape(L.n, r.m)
        X = (X.astype(np.float32).astype(np.float64) if r.fp32 else X.copy())
        t = time.perf_counter()
        oracle.solve_inplace_mt(L.kind, L.bands, X, threads)
        serv.append(time.perf_counter() - t)
        unknowns += L.n * r.m
        if time.perf_counter() - t_all >= budget_s:
            break
    S = np.array(serv)
    count = len(S)
    lam_sat = count / S.sum()
    gaps = np.array([r.t_arrival for r in trace[:count]])          # unit-rate Poisson arrivals
    out = {"requests": count, "cores": threads, "saturation_req_per_s": lam_sat,
           "unknowns_per_s_at_saturation": unknowns / S.sum(), "loads": {}}
    for rho in loads:
        arr = gaps / (rho * lam_sat)
        done = 0.0
        lat = np.empty(count)
        for k in range(count):
            done = max(arr[k], done) + S[k]
            lat[k] = done - arr[k]
        out["loads"][str(rho)] = {"p50_us": float(np.percentile(lat, 50) * 1e6),
                                  "p99_us": float(np.percentile(lat, 99) * 1e6)}
    return out


def bench_serving(args, torch, sbs, W):
    """Serving form: 64 shared matrices (half tridiagonal, half
    pentadiagonal, n log-uniform 64..8192), 1e5 requests with m
    log-uniform 1..4096, FP32 or FP64, HBM budget 200 GB.  Right-hand sides
    are read-only slices of a resident random pool (inputs pre-staged,
    untimed).  A closed-loop run gives the saturation rate; then Poisson
    arrivals at 0.5, 0.8 and 0.95 of it, each reporting p50 / p99 latency
    (submit to completion, queueing included) and throughput.  The 0.8
    arrivals are replayed through a plain FP64 FIFO (one sbs_solve_batch per
    request, no coalescing), and the oracle serves the same requests on the
    host cores.  Requests reach the server through its native trace replay
    (sbs_server_replay: one thread submits at the arrival times, another
    waits for and releases each request), so the rates are the server's and
    not a Python client's."""
    count = args.serve_requests
    loads = (0.5, 0.8, 0.95)
    lhss = W.serving_lhs_set()
    hs = [sbs.SharedLhs(l.kind, l.bands) for l in lhss]
    pool_elems = 1 << 28
    g = torch.Generator(device="cuda:0")
    g.manual_seed(4)
    pool64 = torch.rand(pool_elems, dtype=torch.float64, device="cuda:0", generator=g) * 2 - 1
    pool32 = pool64.to(torch.float32)
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(200e9, free - 16e9))
    srv = _Server(sbs, budget)
    ids = [srv.register(h.handle) for h in hs]
    trace = W.serving_trace(rate_hz=1.0, count=count)       # arrival shape; rescaled below
    rng = np.random.default_rng(7)
    offs = []
    for r in trace:
        nm = lhss[r.lhs].n * r.m
        offs.append(int(rng.integers(0, pool_elems - nm + 1)) // 64 * 64)
    ptr = [(pool32 if r.fp32 else pool64).data_ptr() + o * (4 if r.fp32 else 8) for r, o in zip(trace, offs)]
    dt = [sbs.SBS_F32 if r.fp32 else sbs.SBS_F64 for r in trace]
    unknowns = float(sum(lhss[r.lhs].n * r.m for r in trace))
    torch.cuda.synchronize()

    ids_all = np.array([ids[r.lhs] for r in trace], dtype=np.int32)
    ptr_all = np.array(ptr, dtype=np.uint64)
    m_all = np.array([r.m for r in trace], dtype=np.int64)
    dt_all = np.array(dt, dtype=np.int32)

    def run(arrivals, reqs=count, ks=None):
        # requests ks (default: the first reqs of the trace) in order, through
        # the library's native replay (submitting thread + waiting thread), so
        # that no interpreter sits between the arrivals and the server
        ks = np.arange(reqs) if ks is None else np.asarray(ks)
        arr = None if arrivals is None else np.asarray(arrivals, dtype=np.float64)[:len(ks)] * 1e6
        st, lat, elapsed = sbs.sbs_server_replay(srv.p, ids_all[ks], ptr_all[ks], m_all[ks], dt_all[ks], arr)
        if st:
            raise RuntimeError(f"sbs_server_replay: {st}")
        return elapsed, lat

    pct = lambda a, q: float(np.percentile(a, q))
    run(None, min(count, 20000))                # warm-up pass
    make, _ = run(None)
    lam_sat = count / make
    base_gaps = np.array([r.t_arrival for r in trace])       # arrivals of a unit-rate Poisson process
    res = {"workload": f"serving_64lhs_{count}req", "requests": count, "unknowns": unknowns,
           "saturation_req_per_s": lam_sat, "saturation_unknowns_per_s": unknowns / make, "loads": {}}
    launches0 = srv.stats(sbs).launches
    for rho in loads:
        log(f"  serving at {rho} of saturation")
        span, lat = run(base_gaps / (rho * lam_sat))
        res["loads"][str(rho)] = {"offered_req_per_s": rho * lam_sat, "p50_us": pct(lat, 50), "p99_us": pct(lat, 99),
                                  "max_us": float(lat.max()), "unknowns_per_s": unknowns / span}
    res["launches_per_run"] = (srv.stats(sbs).launches - launches0) / len(loads)
    # Closed loop per precision (up to 2e4 requests of each), and FP32
    # requests served as one FP64 sweep of their stored values (the server's
    # second mode): the mix at saturation and at 0.8 of that saturation.
    sub = {p: [k for k in range(count) if trace[k].fp32 == p][:20000] for p in (False, True)}
    usub = {p: float(sum(lhss[trace[k].lhs].n * trace[k].m for k in sub[p])) for p in sub}
    per = {}
    for p, name in ((False, "fp64_requests"), (True, "fp32_requests_refined")):
        span, _ = run(None, ks=sub[p])
        per[name] = {"requests": len(sub[p]), "unknowns_per_s": usub[p] / span}
    srv.set_fp32_mode(1)
    log("  FP32 requests as one FP64 sweep")
    span, _ = run(None, ks=sub[True])
    per["fp32_requests_fp64_sweep"] = {"requests": len(sub[True]), "unknowns_per_s": usub[True] / span}
    res["closed_loop_per_precision"] = per
    make2, _ = run(None)
    lam2 = count / make2
    span, lat = run(base_gaps / (0.8 * lam2))
    res["fp32_as_fp64_sweep"] = {"saturation_unknowns_per_s": unknowns / make2,
                                 "0.8": {"offered_req_per_s": 0.8 * lam2, "p50_us": pct(lat, 50),
                                         "p99_us": pct(lat, 99), "unknowns_per_s": unknowns / span}}
    srv.set_fp32_mode(0)
    srv.close()

    # Plain FP64 FIFO on the 0.8 arrivals: one solve per request, in order.
    log("  plain FP64 FIFO at 0.8")
    arrivals = base_gaps / (0.8 * lam_sat)
    stream = torch.cuda.current_stream()
    lat_f = np.zeros(count)
    t0 = time.perf_counter()
    for k, r in enumerate(trace):
        while time.perf_counter() - t0 < arrivals[k]:
            pass
        h = hs[r.lhs]
        x = pool64[offs[k]:offs[k] + h.n * r.m].view(h.n, r.m)
        sbs.sbs_solve_batch(h.handle, x)
        stream.synchronize()
        lat_f[k] = (time.perf_counter() - t0 - arrivals[k]) * 1e6
    fifo_span = time.perf_counter() - t0
    res["fifo_f64_at_0.8"] = {"p50_us": pct(lat_f, 50), "p99_us": pct(lat_f, 99),
                              "unknowns_per_s": unknowns / fifo_span}
    for h in hs:
        h.close()
    log("  oracle serving on the host")
    res["cpu_oracle"] = serving_cpu_oracle(lhss, trace, pool64.cpu().numpy(), offs, loads, args.cpu_seconds)
    del pool32, pool64
    res["note"] = ("requests submitted and released by the server's native trace replay; "
                   "latency = submit to completion incl. queueing; rhs device-resident; FP32 requests get the "
                   "mixed-precision solve with 2 corrections (FP64 result); the FIFO baseline solves every "
                   "request in FP64 on one stream without coalescing; cpu_oracle: the oracle on the host cores, "
                   "FIFO, on a prefix of the same trace at the same loads of its own saturation rate; "
                   "closed_loop_per_precision: up to 2e4 requests of one precision each, closed loop; "
                   "fp32_as_fp64_sweep: the same trace with FP32 requests solved by one FP64 sweep of their "
                   "stored values (sbs_server_set_fp32_mode), saturation and 0.8 of it")
    return res


def _event_median(launch, reps, warm, torch, restore=None):
    """Median (and min) device time of `launch` over `reps` runs, each
    bracketed by its own pair of HIP events on the current stream; all runs
    are queued back to back (the host is far ahead of the device), so the
    events measure the kernel alone.  `restore`, if given, runs untimed
    before every run (e.g. the pristine right-hand side copied back)."""
    s = torch.cuda.current_stream()
    for _ in range(warm):
        if restore:
            restore()
        launch()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        if restore:
            restore()
        e0.record(s)
        launch()
        e1.record(s)
    torch.cuda.synchronize()
    t = sorted(e0.elapsed_time(e1) * 1e-3 for e0, e1 in ev)
    return t[len(t) // 2], t[0]


def stream_ceiling(torch, sbs, reps=20):
    """The hand-written streaming probes (libsbs, include/sbs_probe.h):
    a linear copy of 1 GiB (best of the unroll / occupancy settings tried),
    read-only and write-only sweeps, and the partitioned solve's own access
    pattern on the headline's (1024, 65536) FP64 array with no arithmetic.
    Returns (records, best copy GB/s of read + write)."""
    import ctypes
    L = sbs.lib()
    st = torch.cuda.current_stream().cuda_stream
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0").uniform_()
    b = torch.empty_like(a)
    out = []

    def lin(mode, unroll, wgs):
        def go():
            r = L.sbs_probe_linear(mode, a.data_ptr(), b.data_ptr(), nbytes, unroll, wgs, st)
            assert r == 0, r
        med, mn = _event_median(go, reps, 3, torch)
        moved = nbytes * (2 if mode == 0 else 1)
        return {"probe": ["copy", "read", "write"][mode], "unroll": unroll, "wg_per_cu": wgs,
                "us_median": med * 1e6, "GBps": moved / med / 1e9, "GBps_best": moved / mn / 1e9}

    for unroll in (1, 2, 4, 8):
        for wgs in (2, 4, 8):
            out.append(lin(0, unroll, wgs))
    best = max((r for r in out if r["probe"] == "copy"), key=lambda r: r["GBps"])
    out.append(lin(1, best["unroll"], best["wg_per_cu"]))
    out.append(lin(2, best["unroll"], best["wg_per_cu"]))
    med, mn = _event_median(lambda: b.copy_(a), reps, 3, torch)
    out.append({"probe": "torch_copy_", "us_median": med * 1e6, "GBps": 2 * nbytes / med / 1e9})
    del a, b
    # the partitioned solve's access pattern: (lb, vec, S, workgroups per CU)
    n, m = 1024, 65536
    x = torch.empty((n, m), dtype=torch.float64, device="cuda:0").uniform_()
    for lb, vec, S, wgs in ((64, 1, 32, 1), (64, 1, 16, 2), (64, 2, 32, 1), (64, 2, 32, 2), (32, 1, 32, 1),
                            (32, 2, 32, 1), (32, 2, 32, 2), (32, 1, 16, 2), (16, 2, 32, 1), (16, 1, 16, 1),
                            (16, 2, 16, 2)):
        def go():
            r = L.sbs_probe_blocks(x.data_ptr(), n, m, lb, vec, S, wgs, st)
            assert r == 0, (lb, vec, S, wgs, r)
        med, mn = _event_median(go, reps, 3, torch)
        out.append({"probe": "solve_pattern", "n": n, "m": m, "lb": lb, "vec": vec, "S": S, "wg_per_cu": wgs,
                    "us_median": med * 1e6, "GBps": 16 * n * m / med / 1e9, "GBps_best": 16 * n * m / mn / 1e9})
    del x
    return out, best["GBps"]


def copy_probe(args):
    """Streaming probes: each record on its own JSON line."""
    import torch
    from paper_1909_04539_amd import sbs
    recs, _ = stream_ceiling(torch, sbs)
    for r in recs:
        print(json.dumps(r), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--variant", default="auto", choices=list(VARIANTS))
    ap.add_argument("--only", default="", help="'headline' skips the other workloads")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--serve-requests", type=int, default=100000)
    ap.add_argument("--probe", default="", choices=["", "copy"], help="run a calibration probe instead")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the batched solve shards over systems with no exchange "
              "; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.probe == "copy":
        copy_probe(args)
        return
    import torch
    from paper_1909_04539_amd import sbs, workloads as W
    sbs.lib()
    log("headline: penta f64 n=1024 m=65536")
    h = bench_headline(args, torch, sbs, W)
    extra = {}
    if args.only == "serving":
        print(json.dumps(bench_serving(args, torch, sbs, W)), flush=True)
        return
    if args.only != "headline":
        for name, fn in (("penta_general", bench_penta_general), ("periodic_and_cn", bench_periodic_and_cn),
                         ("penta_n2048_m65536", bench_penta_large), ("tri_n256_m1024", bench_tri256),
                         ("adi_2048", bench_adi), ("refined_n512_m1M", bench_refined), ("serving", bench_serving)):
            log(f"workload {name}")
            try:
                extra[name] = fn(args, torch, sbs, W)
            except Exception as e:  # report, do not hide
                extra[name] = {"error": repr(e)}
    log("cpu baseline (oracle)")
    cpu = cpu_baseline(5, h["bands"], h["cpu_sample"], args.cpu_seconds)
    if args.only != "headline":
        log("oracle on the other workloads")
        cpu["other_workloads"] = cpu_other_configs(W)
    line = {
        "metric": "RHS unknowns solved/s (pentadiagonal FP64, shared LHS)",
        "value": h["unknowns"] / h["wall_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["wall_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded): rhs = A x_true, x_true ~ N(0,1)",
        "config": {"workload": "penta_f64_n1024_m65536_shared_lhs", "n": 1024, "m": 65536,
                   "matrix": "I + s(1,-4,6,-4,1), s=0.5, truncated ends", "variant": h["variant"],
                   "shape": h["shape"]},
        "roofline": h["roofline"],
        "cpu_baseline": cpu,
        "kernel_ms": h["dev_s"] * 1e3,
        "other_workloads": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
