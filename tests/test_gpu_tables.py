"""Explicit per-task time tables on the GPU (through the C ABI).

Tables that restate the parametric model give the parametric results bit for
bit; general tables (saturating memory-intensive profiles) give the oracle's
results bit for bit in every allocation mode, for Algorithm 1, on the host and
device entry points and through the batched plans; tables outside the
contract get the oracle's status; a server created with room for tables
takes them, others and the one-set calls refuse them."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from brute import exec_time
from paper_2105_10312_amd import capart, workload

pytestmark = pytest.mark.gpu

FIELDS = ("status", "verdict", "verdict_1g", "pidx", "sizes", "aidx", "maxU", "sumU", "n_evals", "alloc", "R",
          "R_1g")
A1_FIELDS = ("status", "verdict", "nparts", "sizes", "alloc", "R", "tried", "merged")
THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    e = capart.Engine(0)
    yield e
    e.close()


def model_tables(ts):
    """Tables that restate the parametric model, from brute.py's own time model."""
    out = workload.TaskSets({k: v.copy() for k, v in ts.items()})
    sizes, Ms = ts.sizes(), ts["M"].astype(np.int64)
    out["table_offset"] = np.concatenate([[0], np.cumsum(sizes * Ms)[:-1]]).astype(np.int64)
    cn, cc = [], []
    for s in range(ts.n_sets):
        a, b, M = int(ts["set_offset"][s]), int(ts["set_offset"][s + 1]), int(Ms[s])
        for i in range(a, b):
            for m in range(1, M + 1):
                args = (int(ts["C_seq"][i]), int(ts["C_par"][i]), int(ts["k_permille"][i]), m)
                cn.append(exec_time(*args, False))
                cc.append(exec_time(*args, True))
    out["Cn_table"] = np.array(cn, np.int64)
    out["Cc_table"] = np.array(cc, np.int64)
    return out


def tables_only(ts):
    """The same batch without the parametric fields (they are not read)."""
    return workload.TaskSets({k: v for k, v in ts.items() if k not in ("C_seq", "C_par", "k_permille")})


def same(got, want, fields, label):
    for f in fields:
        g, w = np.asarray(got[f]).ravel(), np.asarray(want[f]).ravel()
        assert g.shape == w.shape and np.array_equal(g, w), f"{label}: field {f} differs"


def alg1_oracle(ts, mode):
    S, N = ts.n_sets, ts.n_tasks
    off = ts["set_offset"]
    out = dict(status=np.zeros(S, np.int32), verdict=np.zeros(S, np.uint8), nparts=np.zeros(S, np.int32),
               sizes=np.zeros(N, np.int32), alloc=np.full(N, -1, np.int8), R=np.full(N, -1, np.int64),
               tried=np.zeros(S, np.int64), merged=np.zeros(S, np.int64))
    for s in range(S):
        r = oracle.alg1(ts.set(s), mode)
        a, b = int(off[s]), int(off[s + 1])
        out["verdict"][s], out["tried"][s], out["merged"][s] = r["verdict"], r["tried"], r["merged"]
        if r["verdict"]:
            out["nparts"][s] = r["k"]
            out["sizes"][a:a + r["k"]] = r["sizes"]
            out["alloc"][a:b] = r["alloc"]
            out["R"][a:b] = r["R"]
    return out


def test_model_tables_give_the_parametric_results(eng):
    c1 = workload.config_c1(n_sets=60)
    c2 = workload.subset(workload.config_c2(n_sets=2000), np.arange(200))
    c5 = workload.subset(workload.config_c5(n_queries=400), np.arange(120))
    for ts, K, modes in ((c1, 3, ("EXH", "BF_INA")), (c2, 4, ("BF_INA", "SMS_ACT")), (c5, 4, ("BF_ACT", "SMS_INA"))):
        tt = tables_only(model_tables(ts))
        for mode in modes:
            say(f"model tables {mode}: {ts.n_sets} sets")
            same(eng.solve(tt, K, mode), eng.solve(ts, K, mode), FIELDS, f"model tables {mode}")
    f4 = workload.config_paper_fig4(sets_per_point=3)
    tt = tables_only(model_tables(f4))
    for mode in ("BF_INA", "SMS_ACT"):
        same(eng.alg1(tt, mode), eng.alg1(f4, mode), A1_FIELDS, f"model tables alg1 {mode}")


@pytest.mark.parametrize("mode", ["EXH", "BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_general_tables_match_oracle(eng, mode):
    if mode == "EXH":
        ts = workload.with_time_tables(workload.config_c1(n_sets=100), seed=91)
        K = 3
    else:
        c2 = workload.subset(workload.config_c2(n_sets=2000), np.arange(300))
        c3 = workload.subset(workload.config_c3(n_sets=2000), np.arange(150))
        c5 = workload.config_c5(seed=92, n_queries=300)
        wide = workload.subset(c5, np.nonzero((c5.sizes() > 32) & (c5["M"] <= 48))[0][:12])
        ts = workload.with_time_tables(workload.concat([c2, c3, wide]), seed=93)
        K = 4
    tt = tables_only(ts)
    say(f"general tables {mode}: {tt.n_sets} sets")
    want = oracle.solve(tt, K, mode, nthreads=THREADS)
    assert (want["status"] == oracle.OK).all()
    same(eng.solve(tt, K, mode), want, FIELDS, f"general tables {mode}")


def test_general_tables_alg1_match_oracle(eng):
    f4 = workload.with_time_tables(workload.config_paper_fig4(sets_per_point=4), seed=94)
    tt = tables_only(f4)
    for mode in ("BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"):
        say(f"general tables alg1 {mode}: {tt.n_sets} sets")
        same(eng.alg1(tt, mode), alg1_oracle(tt, mode), A1_FIELDS, f"alg1 tables {mode}")


def test_device_entry_points_with_tables(eng):
    import torch
    ts = tables_only(workload.with_time_tables(workload.subset(workload.config_c2(n_sets=1000), np.arange(120)),
                                               seed=95))
    dev = capart.device_tasksets(ts)
    assert "Cn_table" in dev
    out = capart.device_results(ts.n_sets, ts.n_tasks, 4)
    capart.capart_solve_async(eng.ctx, dev, 4, "SMS_INA", out, max_tasks=10, max_M=80)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    want = eng.solve(ts, 4, "SMS_INA")
    for f in FIELDS:
        n = np.asarray(want[f]).size
        assert np.array_equal(got[f].ravel()[:n], np.asarray(want[f]).ravel()), f
    a1 = capart.device_alg1_results(ts.n_sets, ts.n_tasks)
    capart.capart_alg1_async(eng.ctx, dev, "BF_INA", a1, max_tasks=10, max_M=80)
    torch.cuda.synchronize()
    want = eng.alg1(ts, "BF_INA")
    for f in A1_FIELDS:
        n = np.asarray(want[f]).size
        assert np.array_equal(a1[f].cpu().numpy().ravel()[:n], np.asarray(want[f]).ravel()), f


def test_tables_outside_the_contract(eng):
    ts = workload.with_time_tables(workload.config_c1(n_sets=6), seed=96)
    M = int(ts["M"][0])
    t = tables_only(workload.TaskSets({k: v.copy() for k, v in ts.items()}))
    t["Cn_table"][1] = t["Cn_table"][0] + 1
    a2 = int(t["table_offset"][2])
    t["Cn_table"][a2 + M - 1] = 1
    t["Cc_table"][a2 + M - 1] = 1
    got = eng.solve(t, 3, "BF_INA")
    want = oracle.solve(t, 3, "BF_INA")
    same(got, want, FIELDS, "invalid tables")
    assert got["status"][0] == capart.CAPART_E_RANGE and got["status"][2] == capart.CAPART_E_RANGE


@pytest.mark.parametrize("mode", ["BF_INA", "SMS_ACT"])
def test_batched_plans_with_tables(eng, mode):
    """The batched form (autotuned plan, HIP graph, three replays with eager
    work between them) on general tables: the plain path's results, which the
    tests above check against the oracle, on every replay; a sample against
    the oracle directly."""
    import torch
    c2 = workload.subset(workload.config_c2(n_sets=3000), np.arange(2000))
    c3 = workload.subset(workload.config_c3(n_sets=3000), np.arange(1500))
    ts = tables_only(workload.with_time_tables(workload.concat([c2, c3]), seed=98))
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, 4)
    plan = capart.Plan(eng.ctx, dev, 4, mode, out, 32, 108)
    want = eng.solve(ts, 4, mode)
    for rep in range(3):
        plan.run()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        for f in FIELDS:
            n = np.asarray(want[f]).size
            assert np.array_equal(got[f].ravel()[:n], np.asarray(want[f]).ravel()), (f, rep)
        torch.zeros(1 << 20, device="cuda").sum().item()
    pick = np.arange(0, ts.n_sets, 50)
    sub = workload.subset(ts, pick)
    ref = oracle.solve(sub, 4, mode, nthreads=THREADS)
    mine = eng.solve(sub, 4, mode)
    same(mine, ref, FIELDS, f"tables sample {mode}")
    plan.close()
    say(f"batched tables {mode}: {int(want['verdict'].sum())} of {ts.n_sets} schedulable")


def query_fields(r, q, off, K):
    """Query q's results out of a batch result dict."""
    a, b = int(off[q]), int(off[q + 1])
    return {f: (np.asarray(r[f]).reshape(-1, K)[q] if f == "sizes" else
                (np.asarray(r[f])[a:b] if f in ("alloc", "R", "R_1g") else np.asarray(r[f])[q:q + 1]))
            for f in FIELDS}


@pytest.mark.parametrize("mode,policy", [("BF_INA", "FP_DM"), ("SMS_ACT", "FP_DM"), ("BF_ACT", "EDF")])
def test_server_with_tables(eng, mode, policy):
    """A server created with room for tables: queries with general tables and
    parametric queries submitted in alternating runs of each kind (a batch
    holds one kind), then the tables batch replayed at 20k q/s; every query
    gets the oracle's results, and a query whose table leaves the contract
    gets E_RANGE without disturbing the others."""
    c5 = workload.config_c5(seed=71, n_queries=700)
    pick = [i for i in range(c5.n_sets) if c5.sizes()[i] <= 24 and c5["M"][i] >= 2][:150]
    ts = workload.subset(c5, pick)
    tt = tables_only(workload.with_time_tables(ts, seed=72))
    bad = 7
    a = int(tt["table_offset"][bad])
    tt["Cn_table"][a + 1] = tt["Cn_table"][a] + 1  # increasing in m
    off, K = ts["set_offset"], 4
    say(f"server tables {mode} {policy}: oracle on {ts.n_sets} queries, both kinds")
    want_t = oracle.solve(tt, K, mode, nthreads=THREADS, policy=policy)
    want_p = oracle.solve(ts, K, mode, nthreads=THREADS, policy=policy)
    assert want_t["status"][bad] == capart.CAPART_E_RANGE
    assert (np.delete(want_t["status"], bad) == oracle.OK).all()
    srv = capart.Server(eng.ctx, K=K, mode=mode, max_tasks=24, max_M=108, policy=policy, tables=True)
    try:
        rng = np.random.default_rng(73)
        kind, left, tickets = True, 0, []
        for q in range(ts.n_sets):
            if left == 0:
                kind, left = not kind, int(rng.integers(1, 8))
            left -= 1
            tk = srv.submit(tt.set(q) if kind else ts.set(q))
            assert tk is not None
            tickets.append((q, kind, tk))
        say(f"server tables: {len(tickets)} queries submitted, {srv.stats()['batches']} batches so far")
        for q, kind, tk in tickets:
            got = wait(srv, tk, int(off[q + 1] - off[q]))
            want = query_fields(want_t if kind else want_p, q, off, K)
            same(got, want, FIELDS, f"query {q} ({'tables' if kind else 'parametric'})")
        arrival = np.cumsum(rng.exponential(1e6 / 20000.0, tt.n_sets))
        mix, stats = srv.replay(tt, arrival)
        say("server tables replay", stats)
        same(mix, want_t, FIELDS, f"replay {mode} {policy}")
    finally:
        srv.close()


def wait(srv, ticket, n, timeout=30.0):
    t0 = time.time()
    while True:
        r = srv.poll(ticket, n)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {ticket} not complete")
        time.sleep(0.0002)


def test_paths_without_tables_refuse_them(eng):
    """A server created without room for tables, and the one-set calls."""
    ts = tables_only(workload.with_time_tables(workload.config_c1(n_sets=4), seed=97))
    srv = capart.Server(eng.ctx, K=3, mode="BF_INA", max_tasks=5, max_M=8)
    try:
        with pytest.raises(capart.CapartError):
            srv.replay(ts, np.zeros(ts.n_sets))
        with pytest.raises(capart.CapartError):
            srv.submit(ts.set(0))
    finally:
        srv.close()
    task = ts.set(1)
    n, M = len(task["T"]), int(task["M"])
    with pytest.raises(capart.CapartError):
        eng.test_triple(task, [M], np.zeros(n, np.int8))
    with pytest.raises(capart.CapartError):
        eng.allocate(task, [M], 3, "BF_INA")
