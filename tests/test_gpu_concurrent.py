"""Concurrent solves: the factored handle is read-only after factoring, so
several host threads may solve with it at once, each on its own stream (the
C ABI's thread-safety statement).  Six threads share two handles and run
plain solves and Crank-Nicolson steps on their own right-hand sides; every
result is checked against the oracle (FP64, 1e-12 per column)."""
import threading

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


def test_threads_share_handles_on_their_own_streams():
    n3, n5 = 700, 1024
    B3 = W.tri_dominant_bands(np.random.default_rng(1), n3)
    B5 = W.hyperdiffusion_bands(n5, 0.4)
    jobs = []  # (kind, bands, rhs, op)
    for t in range(6):
        kind, B = (3, B3) if t % 2 == 0 else (5, B5)
        m = [4096, 333, 8192, 65, 2048, 1000][t]
        rhs = np.random.default_rng(10 + t).uniform(-1, 1, (B.shape[1], m))
        jobs.append((kind, B, rhs, "cn" if t >= 4 else "solve"))
    handles = {3: sbs.SharedLhs(3, B3), 5: sbs.SharedLhs(5, B5)}
    results, errors = [None] * len(jobs), []
    barrier = threading.Barrier(len(jobs), timeout=60)

    def work(i):
        try:
            kind, B, rhs, op = jobs[i]
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                x = torch.from_numpy(rhs).to(DEV)
                barrier.wait()
                for _ in range(3):  # three rounds, so launches from the threads interleave
                    y = x.clone()
                    if op == "solve":
                        handles[kind].solve(y)
                    else:
                        handles[kind].cn_step(y, 2)
                s.synchronize()
                results[i] = y.cpu().numpy()
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(jobs))]
    for th in threads:
        th.start()
    for th in threads:
        th.join(120)
    assert not any(th.is_alive() for th in threads)
    for h in handles.values():
        h.close()
    assert not errors, errors
    for (kind, B, rhs, op), got in zip(jobs, results):
        ref = oracle.solve(kind, B, rhs) if op == "solve" else oracle.cn_steps(kind, B, rhs, 2)
        assert colrel(got, ref) <= 1e-12, (kind, rhs.shape, op)
