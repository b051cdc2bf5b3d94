"""Batched form (persistent, work-item queue, autotuned, HIP-graph-captured):
bit-exact against the plain GPU path and the oracle, identical under every
tuning choice, and identical across repeated graph replays."""
import os
import sys

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


def host(out, S, N, K):
    r = {}
    for f in FIELDS:
        a = out[f].cpu().numpy()
        r[f] = a[:S * K].reshape(S, K) if f == "sizes" else a[:N if f in ("alloc", "R", "R_1g") else S]
    return r


def plain(eng, ts, K, mode, max_tasks, max_M):
    import torch
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, K)
    capart.capart_solve_async(eng.ctx, dev, K, mode, out, max_tasks=max_tasks, max_M=max_M)
    torch.cuda.synchronize()
    return host(out, ts.n_sets, ts.n_tasks, K)


def batched(eng, ts, K, mode, max_tasks, max_M, **kw):
    import torch
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, K)
    plan = capart.Plan(eng.ctx, dev, K, mode, out, max_tasks, max_M, **kw)
    plan.run()
    torch.cuda.synchronize()
    res = host(out, ts.n_sets, ts.n_tasks, K)
    info = plan.info()
    plan.close()
    return res, info


def same(a, b, label):
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f"{label}: {f}"


@pytest.mark.parametrize("mode", ["BF_INA", "SMS_ACT"])
def test_batched_matches_plain_and_oracle(eng, mode):
    ts = workload.config_c2(n_sets=6000 if mode == "BF_INA" else 1500)
    say(f"batched {mode}: {ts.n_sets} sets")
    p = plain(eng, ts, 4, mode, 10, 80)
    b, info = batched(eng, ts, 4, mode, 10, 80)
    say("plan", info)
    same(b, p, f"batched vs plain {mode}")
    # a persistent grid over work items, or the direct schedule (no items)
    assert (info["n_items"] > 0) != (info["blocks"] == 0) and info["total_evals"] == 4263 * ts.n_sets
    idx = np.arange(0, ts.n_sets, max(1, ts.n_sets // 150))
    sub = workload.subset(ts, idx)
    want = oracle.solve(sub, 4, mode, nthreads=THREADS)
    task_idx = np.concatenate([np.arange(ts["set_offset"][s], ts["set_offset"][s + 1]) for s in idx])
    for f in FIELDS:
        g = b[f][task_idx] if f in ("alloc", "R", "R_1g") else b[f][idx]
        assert np.array_equal(g, want[f]), f


def test_every_tuning_choice_gives_identical_bytes(eng):
    ts = workload.config_c2(seed=5, n_sets=3000)
    ref, _ = batched(eng, ts, 4, "BF_ACT", 10, 80, autotune=False)
    for threads in (64, 128, 256):
        for form in (1, 2):
            for item_evals, bpc in ((512, 1), (4096, 4), (65536, 8)):
                capart.capart_set_tuning(eng.ctx, threads, 0, form)
                got, info = batched(eng, ts, 4, "BF_ACT", 10, 80, autotune=False, item_evals=item_evals,
                                    blocks_per_cu=bpc)
                same(got, ref, f"threads={threads} form={form} item={item_evals} bpc={bpc}")
    capart.capart_set_tuning(eng.ctx, 0, 0, 0)


def test_direct_schedule_matches_plain(eng):
    """The plan's direct schedule (one block per set chunk) gives the plain
    path's bytes, with and without graph capture, on even and uneven batches."""
    for ts, mt, mm in ((workload.config_c2(seed=8, n_sets=3000), 10, 80),
                       (workload.config_c3(seed=9, n_sets=3000), 32, 108)):
        ref = plain(eng, ts, 4, "SMS_INA", mt, mm)
        for graph in (False, True):
            got, info = batched(eng, ts, 4, "SMS_INA", mt, mm, autotune=False, blocks_per_cu=-1, use_graph=graph)
            assert info["blocks"] == 0
            same(got, ref, f"direct graph={graph}")


def test_three_size_classes_match_plain(eng):
    """Sets of 2..64 tasks (frontier, memo and 64-bit-mask classes, each with
    its own launch and queue) in the batched form give the plain path's bytes,
    and sampled sets the oracle's."""
    ts = workload.config_c5(seed=10, n_queries=3000)
    say("mixed sizes: 3000 sets, n 2..64")
    ref = plain(eng, ts, 4, "BF_ACT", 64, 108)
    for bpc in (4, -1):
        got, info = batched(eng, ts, 4, "BF_ACT", 64, 108, autotune=False, blocks_per_cu=bpc)
        same(got, ref, f"mixed sizes bpc={bpc}")
    rng = np.random.default_rng(13)
    n = ts.sizes()
    idx = np.sort(np.concatenate([rng.choice(np.nonzero(n <= 14)[0], 20, replace=False),
                                  rng.choice(np.nonzero((n > 14) & (n <= 32))[0], 8, replace=False),
                                  rng.choice(np.nonzero(n > 32)[0], 4, replace=False)]))
    sub = workload.subset(ts, idx)
    want = oracle.solve(sub, 4, "BF_ACT", nthreads=THREADS)
    task_idx = np.concatenate([np.arange(ts["set_offset"][s], ts["set_offset"][s + 1]) for s in idx])
    for f in FIELDS:
        g = ref[f][task_idx] if f in ("alloc", "R", "R_1g") else ref[f][idx]
        assert np.array_equal(g, want[f]), f


def test_graph_replays_are_identical(eng):
    import torch
    ts = workload.config_c2(seed=6, n_sets=4000)
    ref = plain(eng, ts, 4, "BF_INA", 10, 80)
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, 4)
    plan = capart.Plan(eng.ctx, dev, 4, "BF_INA", out, 10, 80, autotune=False, use_graph=True)
    assert plan.info()["use_graph"] == 1
    for rep in range(4):
        for t in out.values():
            t.fill_(0x55 if t.dtype != torch.uint64 else 0)  # scribble between replays
        x = torch.randn(1 << 20, device="cuda")
        _ = (x * 2).sum().item()  # eager work on the same device between replays
        plain(eng, workload.config_c2(seed=7, n_sets=300), 4, "BF_INA", 10, 80)
        plan.run()
        torch.cuda.synchronize()
        same(host(out, ts.n_sets, ts.n_tasks, 4), ref, f"replay {rep}")
    plan.close()


def test_uneven_batch_c3(eng):
    ts = workload.config_c3(n_sets=20000)
    say("uneven c3 batch: 20000 sets, n in 4..32, M in {16,48,80,108}")
    p = plain(eng, ts, 4, "BF_INA", 32, 108)
    b, info = batched(eng, ts, 4, "BF_INA", 32, 108)
    say("plan", info)
    same(b, p, "c3 batched vs plain")
    rng = np.random.default_rng(12)
    small = [s for s in rng.permutation(ts.n_sets) if ts["M"][s] <= 48 and ts.sizes()[s] <= 20][:120]
    idx = np.sort(np.concatenate([small, rng.choice(ts.n_sets, 12, replace=False)]))
    sub = workload.subset(ts, idx)
    want = oracle.solve(sub, 4, "BF_INA", nthreads=THREADS)
    task_idx = np.concatenate([np.arange(ts["set_offset"][s], ts["set_offset"][s + 1]) for s in idx])
    for f in FIELDS:
        g = b[f][task_idx] if f in ("alloc", "R", "R_1g") else b[f][idx]
        assert np.array_equal(g, want[f]), f


def test_plan_rejects_exhaustive_and_bad_arguments(eng):
    ts = workload.config_c1(n_sets=10)
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, 3)
    with pytest.raises(capart.CapartError):
        capart.Plan(eng.ctx, dev, 3, "EXH", out, 5, 8)
    with pytest.raises(capart.CapartError):
        capart.Plan(eng.ctx, dev, 9, "BF_INA", out, 5, 8)
