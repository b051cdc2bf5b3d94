"""Admissible partition sizes on the GPU (through the C ABI): bit-exact with
the oracle on every evaluation path (exhaustive forms, frontier, test memo,
the three loop forms, wide sets, batched plans, the server); excluded
partitionings carry "none" debug keys; Algorithm 1 refuses a restriction."""
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
MIG_LIKE = tuple(range(4, 256, 4)) + (1, 2)   # 1, 2 and multiples of 4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    e = capart.Engine(0)
    yield e
    e.close()


def same(got, want, label):
    for f in FIELDS:
        g, w = np.asarray(got[f]).ravel(), np.asarray(want[f]).ravel()
        assert g.shape == w.shape and np.array_equal(g, w), f"{label}: field {f} differs"


def mixed():
    c2 = workload.subset(workload.config_c2(n_sets=2000), np.arange(150))
    c3 = workload.subset(workload.config_c3(n_sets=2000), np.arange(150))
    c5 = workload.config_c5(seed=101, n_queries=300)
    wide = workload.subset(c5, np.nonzero((c5.sizes() > 32) & (c5["M"] <= 48))[0][:10])
    return workload.concat([c2, c3, wide])


@pytest.mark.parametrize("adm", [(1, 2, 4), (3, 5), (1, 2, 3, 6)])
def test_exhaustive_matches_oracle(eng, adm):
    ts = workload.config_c1(n_sets=100)
    want = oracle.solve(ts, 3, "EXH", admissible=adm)
    for exh_form in (1, 2):
        capart.capart_set_tuning(eng.ctx, exh_form=exh_form)
        same(eng.solve(ts, 3, "EXH", admissible=adm), want, f"EXH {adm} form {exh_form}")
    capart.capart_set_tuning(eng.ctx)


@pytest.mark.parametrize("mode", ["BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_heuristic_paths_match_oracle(eng, mode):
    ts = mixed()
    say(f"admissible {mode}: {ts.n_sets} sets")
    want = oracle.solve(ts, 4, mode, nthreads=THREADS, admissible=MIG_LIKE)
    ref = None
    for tune in ({}, {"loop_form": 2}, {"loop_form": 3}, {"frontier": 2, "memo": -1}, {"wide_chunk": -1},
                 {"wide_chunk": 3}):
        capart.capart_set_tuning(eng.ctx, **tune)
        got = eng.solve(ts, 4, mode, debug=True, admissible=MIG_LIKE)
        same(got, want, f"{mode} {tune}")
        if ref is None:
            ref = got
        assert np.array_equal(got["dbg_key"], ref["dbg_key"]), (mode, tune)
    capart.capart_set_tuning(eng.ctx)
    # excluded partitionings carry "none" keys
    for s in range(0, ts.n_sets, 37):
        M = int(ts["M"][s])
        parts = oracle.enumerate_partitionings(M, 4)
        ok = np.isin(parts, (0,) + MIG_LIKE).all(axis=1)
        keys = ref["dbg_key"][ref["dbg_offset"][s]:ref["dbg_offset"][s] + len(parts)]
        assert (keys[~ok] == np.uint64(2**64 - 1)).all()


def test_batched_plans_match_plain(eng):
    import torch
    ts = mixed()
    dev = capart.device_tasksets(ts)
    want = eng.solve(ts, 4, "BF_INA", admissible=MIG_LIKE)
    for bpc in (4, -1):
        out = capart.device_results(ts.n_sets, ts.n_tasks, 4)
        plan = capart.Plan(eng.ctx, dev, 4, "BF_INA", out, 64, 108, autotune=False, blocks_per_cu=bpc,
                           admissible=MIG_LIKE)
        plan.run()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        plan.close()
        for f in FIELDS:
            w = np.asarray(want[f]).ravel()
            assert np.array_equal(got[f].ravel()[:w.size], w), (bpc, f)


def test_alg1_refuses_a_restriction(eng):
    ts = workload.config_c1(n_sets=2)
    st, _keep = capart.make_tasksets(capart._host_ts(ts))
    opt = capart.make_options(1, "BF_INA", 0, admissible=(1, 2))
    out = {name: np.zeros(16, dt) for name, dt, shape in capart.ALG1_FIELDS}
    res = capart.capart_alg1_results(*[capart._ptr(out[f[0]]) for f in capart.ALG1_FIELDS])
    rc = capart.load_library().capart_alg1(eng.ctx, capart.C.byref(st), capart.C.byref(opt), capart.C.byref(res))
    assert rc == capart.CAPART_E_INVAL


@pytest.mark.parametrize("mode,policy", [("BF_INA", "FP_DM"), ("SMS_ACT", "EDF")])
def test_server_matches_oracle(eng, mode, policy):
    """A server whose configuration restricts the part sizes: every query of a
    serving mix (narrow, memo-class and wide queries, replayed at 20k q/s)
    gets the plain path's results under the same restriction, which the
    tests above check against the oracle; a sample against the oracle
    directly."""
    c5 = workload.config_c5(seed=103, n_queries=400)
    pick = [i for i in range(c5.n_sets) if c5.sizes()[i] <= 24 or c5["M"][i] <= 48][:200]
    ts = workload.subset(c5, pick)
    srv = capart.Server(eng.ctx, K=4, mode=mode, max_tasks=64, max_M=108, policy=policy, admissible=MIG_LIKE)
    try:
        rng = np.random.default_rng(104)
        arrival = np.cumsum(rng.exponential(1e6 / 20000.0, ts.n_sets))
        say(f"server admissible {mode} {policy}: {ts.n_sets} queries")
        got, stats = srv.replay(ts, arrival)
        assert stats["completed"] == ts.n_sets
    finally:
        srv.close()
    same(got, eng.solve(ts, 4, mode, admissible=MIG_LIKE, policy=policy), f"server {mode} {policy}")
    small = [i for i in range(ts.n_sets) if ts.sizes()[i] <= 16][:40]
    sub = workload.subset(ts, small)
    want = oracle.solve(sub, 4, mode, nthreads=THREADS, admissible=MIG_LIKE, policy=policy)
    off = ts["set_offset"]
    task_idx = np.concatenate([np.arange(off[s], off[s + 1]) for s in small])
    for f in FIELDS:
        g = got[f][task_idx] if f in ("alloc", "R", "R_1g") else (got[f][small] if f != "sizes" else got[f][small])
        assert np.array_equal(np.asarray(g).ravel(), np.asarray(want[f]).ravel()), f"oracle sample: {f}"
