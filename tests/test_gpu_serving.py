"""Serving form: results of every query are the same alone and in the mix
(bit-exact), equal the oracle's, and admission pushes back when the device
budget is exhausted."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2105_10312_amd import capart, workload

pytestmark = pytest.mark.gpu
FIELDS = ("status", "verdict", "verdict_1g", "pidx", "sizes", "aidx", "maxU", "sumU", "n_evals", "alloc", "R",
          "R_1g")
THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    e = capart.Engine(0)
    yield e
    e.close()


def queries(n_q, seed=5):
    return workload.config_c5(seed=seed, n_queries=n_q)


def wait(srv, ticket, n, timeout=30.0):
    t0 = time.time()
    while True:
        r = srv.poll(ticket, n)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {ticket} not complete")
        time.sleep(0.0002)


def test_alone_equals_mix_equals_oracle(eng):
    ts = queries(400)
    srv = capart.Server(eng.ctx, K=4, mode="BF_INA", max_tasks=64, max_M=108)
    say("serving: 40 queries alone")
    alone = {}
    for q in range(40):
        task = ts.set(q)
        tk = srv.submit(task)
        assert tk is not None
        alone[q] = wait(srv, tk, len(task["T"]))
    say("serving: 400 queries replayed at 20k q/s (Poisson)")
    rng = np.random.default_rng(1)
    arrival = np.cumsum(rng.exponential(1e6 / 20000.0, ts.n_sets))
    mix, stats = srv.replay(ts, arrival)
    say("stats", stats)
    assert stats["completed"] == ts.n_sets and stats["p50_us"] <= stats["p99_us"]
    assert stats["batches"] >= 1
    off = ts["set_offset"]
    for q, r in alone.items():
        for f in FIELDS:
            if f in ("alloc", "R", "R_1g"):
                m = mix[f][off[q]:off[q + 1]]
            elif f == "sizes":
                m = mix[f][q:q + 1]
            else:
                m = mix[f][q:q + 1]
            assert np.array_equal(np.asarray(r[f]).ravel(), np.asarray(m).ravel()), (q, f)
    idx = np.arange(0, ts.n_sets, 4)
    small = [int(i) for i in idx if ts.sizes()[i] <= 24][:60]
    sub = workload.subset(ts, small)
    want = oracle.solve(sub, 4, "BF_INA", nthreads=THREADS)
    task_idx = np.concatenate([np.arange(off[s], off[s + 1]) for s in small])
    for f in FIELDS:
        g = mix[f][task_idx] if f in ("alloc", "R", "R_1g") else mix[f][small]
        assert np.array_equal(g, want[f]), f
    srv.close()


def test_burst_is_batched_and_overlaps(eng):
    ts = queries(2000, seed=6)
    srv = capart.Server(eng.ctx, K=4, mode="BF_INA", max_tasks=64, max_M=108, streams=4)
    arrival = np.zeros(ts.n_sets)  # everything at once
    out, stats = srv.replay(ts, arrival, collect=True)
    say("burst stats", stats)
    assert stats["completed"] == ts.n_sets
    assert stats["mean_batch"] > 1.0  # queries that arrive together share launches
    ref = capart.capart_solve(eng.ctx, ts, 4, "BF_INA", max_tasks=64, max_M=108)
    for f in FIELDS:
        assert np.array_equal(out[f], ref[f]), f
    srv.close()


def test_admission_pushes_back_when_budget_is_full(eng):
    ts = queries(300, seed=7)
    # room for only a few queries
    srv = capart.Server(eng.ctx, K=4, mode="BF_INA", max_tasks=64, max_M=108, max_queries=8, streams=1,
                        device_bytes=8 << 20)
    tickets, rejected = [], 0
    for q in range(40):
        tk = srv.submit(ts.set(q))
        if tk is None:
            rejected += 1
        else:
            tickets.append((q, tk))
    assert rejected > 0 and len(tickets) <= 8
    for q, tk in tickets:
        wait(srv, tk, len(ts["T"][ts["set_offset"][q]:ts["set_offset"][q + 1]]))
    # space is free again
    assert srv.submit(ts.set(100)) is not None
    assert srv.stats()["rejected"] >= rejected
    srv.close()
