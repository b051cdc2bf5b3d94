"""EDF per-partition policy on the GPU (through the C ABI): bit-exact with the
oracle's EDF in every allocation mode and on every evaluation path (loop
forms, feasibility frontier, test memo, wide-set wave path, exhaustive forms,
batched plans, device entry points, Algorithm 1), over the random input
domain and at the test's stated limits."""
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2105_10312_amd import capart, workload
from test_gpu_random_domain import random_batch

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


def same(got, want, fields, label):
    for f in fields:
        g, w = np.asarray(got[f]).ravel(), np.asarray(want[f]).ravel()
        if not (g.shape == w.shape and np.array_equal(g, w)):
            bad = np.nonzero(g != w)[0][:3] if g.shape == w.shape else []
            raise AssertionError(f"{label}: field {f} differs at {list(bad)}")


def mixed():
    """Implicit (C2), constrained (C3) and wide (C5, 33..64 tasks) sets."""
    c2 = workload.subset(workload.config_c2(n_sets=2000), np.arange(100))
    c3 = workload.subset(workload.config_c3(n_sets=2000), np.arange(60))
    c5 = workload.config_c5(seed=101, n_queries=300)
    wide = workload.subset(c5, np.nonzero((c5.sizes() > 32) & (c5["M"] <= 48))[0][:6])
    return workload.concat([c2, c3, wide])


def limit_sets():
    """Sets at the EDF test's stated limits, as one-unit partitions with
    sequential times (k = 1000): a busy period that takes the utilisation
    bound, deadline counts either side of the limit (density at most 1
    deciding first), utilisation exactly 1 (implicit, and constrained but
    still schedulable), just above 1, a single task meeting or missing its
    deadline, and three constrained-deadline sets beyond the deadline limit
    that the fixed-priority fallback decides (schedulable, a true miss, and
    the fallback's pessimism)."""
    cases = [
        ([9_999, 5_000], [10_000, 1_000_000_000], [10_000, 1_000_000_000]),
        ([10_000, 5_000], [10_000, 1_000_000_000], [10_000, 1_000_000_000]),
        ([1, 50_000], [2, 1 << 30], [2, 1 << 30]),
        ([1, 200_000], [2, 1 << 30], [2, 1 << 30]),
        ([1, 3, 3], [4, 6, 12], [4, 6, 12]),
        ([1, 3, 3], [4, 6, 12], [3, 6, 12]),
        ([2, 3, 4], [4, 6, 12], [4, 6, 12]),
        ([7], [100], [7]),
        ([7], [100], [6]),
        ([1, 300_000], [4, 1 << 30], [1, 600_000]),
        ([1, 200_000], [2, 1 << 30], [2, 399_998]),
        ([1, 200_000], [2, 1 << 30], [2, 399_999]),
    ]
    off = np.concatenate([[0], np.cumsum([len(c[0]) for c in cases])]).astype(np.int64)
    cat = lambda i, dt: np.concatenate([np.asarray(c[i], dt) for c in cases])
    N = int(off[-1])
    return workload.TaskSets(set_offset=off, M=np.ones(len(cases), np.int32), T=cat(1, np.int64),
                             D=cat(2, np.int64), C_seq=cat(0, np.int64), C_par=np.zeros(N, np.int64),
                             k_permille=np.full(N, 1000, np.int32), type=np.zeros(N, np.uint8))


@pytest.mark.parametrize("mode", ["BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_heuristic_paths_match_oracle(eng, mode):
    ts = mixed()
    say(f"EDF {mode}: {ts.n_sets} sets")
    want = oracle.solve(ts, 4, mode, nthreads=THREADS, policy="EDF")
    fp = oracle.solve(ts, 4, mode, nthreads=THREADS)
    assert (want["verdict_1g"] >= fp["verdict_1g"]).all()
    for tune in ({}, {"loop_form": 2}, {"loop_form": 3}, {"frontier": 2, "memo": -1}, {"wide_chunk": -1}):
        capart.capart_set_tuning(eng.ctx, **tune)
        same(eng.solve(ts, 4, mode, policy="EDF"), want, FIELDS, f"EDF {mode} {tune}")
    capart.capart_set_tuning(eng.ctx)
    # the FP results on the same context are untouched
    same(eng.solve(ts, 4, mode), fp, FIELDS, f"FP {mode}")


def test_exhaustive_matches_oracle(eng):
    ts = workload.config_c1(n_sets=100)
    small = random_batch(7001, 60, 3, 7, 12, 10 ** 9)
    for batch, K in ((ts, 3), (small, 3)):
        want = oracle.solve(batch, K, "EXH", policy="EDF")
        for exh_form in (1, 2):
            capart.capart_set_tuning(eng.ctx, exh_form=exh_form)
            same(eng.solve(batch, K, "EXH", policy="EDF"), want, FIELDS, f"EDF EXH form {exh_form}")
    capart.capart_set_tuning(eng.ctx)


@pytest.mark.parametrize("K", [1, 3, 8])
def test_random_domain_matches_oracle(eng, K):
    ts = random_batch(5000 + K, 150, K, 64, 255, 40000)
    for mode in ("BF_INA", "SMS_ACT"):
        say(f"EDF random domain {mode} K={K}")
        want = oracle.solve(ts, K, mode, nthreads=THREADS, policy="EDF")
        same(eng.solve(ts, K, mode, policy="EDF"), want, FIELDS, f"EDF random {mode} K={K}")


def test_limits_match_oracle(eng):
    ts = limit_sets()
    want = oracle.solve(ts, 1, "BF_INA", policy="EDF")
    got = eng.solve(ts, 1, "BF_INA", policy="EDF")
    same(got, want, FIELDS, "EDF limits")
    assert list(got["verdict_1g"]) == [1, 0, 1, 1, 1, 1, 0, 1, 0, 1, 0, 0]


def test_alg1_matches_oracle(eng):
    f4 = workload.config_paper_fig4(sets_per_point=3)
    c3 = workload.subset(workload.config_c3(n_sets=2000), np.arange(60))
    for ts in (f4, c3):
        off = ts["set_offset"]
        for mode in ("BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"):
            say(f"EDF alg1 {mode}: {ts.n_sets} sets")
            got = eng.alg1(ts, mode, policy="EDF")
            for s in range(ts.n_sets):
                w = oracle.alg1(ts.set(s), mode, policy="EDF")
                a, b = int(off[s]), int(off[s + 1])
                assert int(got["verdict"][s]) == w["verdict"], (mode, s)
                assert int(got["tried"][s]) == w["tried"] and int(got["merged"][s]) == w["merged"], (mode, s)
                if w["verdict"]:
                    assert int(got["nparts"][s]) == w["k"]
                    assert np.array_equal(got["sizes"][a:a + w["k"]], w["sizes"]), (mode, s)
                    assert np.array_equal(got["alloc"][a:b], w["alloc"]), (mode, s)
                    assert np.array_equal(got["R"][a:b], w["R"]), (mode, s)


def test_batched_plans_and_device_entry(eng):
    import torch
    ts = workload.concat([workload.subset(workload.config_c2(n_sets=2000), np.arange(100)),
                          workload.subset(workload.config_c3(n_sets=2000), np.arange(60))])
    want = eng.solve(ts, 4, "BF_INA", policy="EDF")
    dev = capart.device_tasksets(ts)
    for bpc in (8, -1):
        out = capart.device_results(ts.n_sets, ts.n_tasks, 4)
        plan = capart.Plan(eng.ctx, dev, 4, "BF_INA", out, 32, 108, autotune=False, blocks_per_cu=bpc,
                           policy="EDF")
        plan.run()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items()}
        plan.close()
        for f in FIELDS:
            w = np.asarray(want[f]).ravel()
            assert np.array_equal(got[f].ravel()[:w.size], w), (bpc, f)
    out = capart.device_results(ts.n_sets, ts.n_tasks, 4)
    capart.capart_solve_async(eng.ctx, dev, 4, "BF_INA", out, max_tasks=32, max_M=108, policy="EDF")
    torch.cuda.synchronize()
    for f in FIELDS:
        w = np.asarray(want[f]).ravel()
        assert np.array_equal(out[f].cpu().numpy().ravel()[:w.size], w), f


def test_unknown_policy_is_rejected(eng):
    ts = workload.config_c1(n_sets=2)
    with pytest.raises(capart.CapartError):
        eng.solve(ts, 3, "BF_INA", policy=7)


def test_server_matches_solve(eng):
    """Queries served under EDF (continuous batching over several streams)
    give the batch solve's results bit for bit."""
    c5 = workload.config_c5(seed=103, n_queries=150)
    want = eng.solve(c5, 4, "BF_INA", policy="EDF")
    srv = capart.Server(eng.ctx, K=4, mode="BF_INA", max_tasks=64, max_M=108, policy="EDF")
    rng = np.random.default_rng(3)
    arrival = np.cumsum(rng.exponential(1e6 / 5000.0, c5.n_sets))
    say(f"EDF serving: {c5.n_sets} queries")
    mix, stats = srv.replay(c5, arrival)
    srv.close()
    assert stats["completed"] == c5.n_sets
    same(mix, want, FIELDS, "EDF server")


def test_tables_and_admissible_sizes_under_edf(eng):
    from test_gpu_tables import tables_only
    c2 = workload.subset(workload.config_c2(n_sets=2000), np.arange(100))
    c3 = workload.subset(workload.config_c3(n_sets=2000), np.arange(40))
    tt = tables_only(workload.with_time_tables(workload.concat([c2, c3]), seed=98))
    adm = (1, 2) + tuple(range(4, 256, 4))
    for mode in ("BF_INA", "SMS_ACT"):
        say(f"EDF tables + admissible {mode}: {tt.n_sets} sets")
        want = oracle.solve(tt, 4, mode, nthreads=THREADS, admissible=adm, policy="EDF")
        same(eng.solve(tt, 4, mode, admissible=adm, policy="EDF"), want, FIELDS, f"EDF tables {mode}")
    f4 = tables_only(workload.with_time_tables(workload.config_paper_fig4(sets_per_point=2), seed=99))
    off = f4["set_offset"]
    got = eng.alg1(f4, "BF_ACT", policy="EDF")
    for s in range(f4.n_sets):
        w = oracle.alg1(f4.set(s), "BF_ACT", policy="EDF")
        a, b = int(off[s]), int(off[s + 1])
        assert int(got["verdict"][s]) == w["verdict"] and int(got["tried"][s]) == w["tried"], s
        if w["verdict"]:
            assert np.array_equal(got["sizes"][a:a + w["k"]], w["sizes"]), s
            assert np.array_equal(got["alloc"][a:b], w["alloc"]) and np.array_equal(got["R"][a:b], w["R"]), s


def test_response_report_around_the_largest_deadline(eng):
    """Where the density bound decides, the reported response time is
    min(D_i, H) with H the busy period, and the kernels stop iterating H at
    the partition's largest deadline: sets whose busy period ends well
    before, just before, at and after the largest deadline (chosen triple
    and whole GPU) give the oracle's R and R_1g."""
    from test_gpu_alg1 import as_batch
    tasks = []
    # light: busy period far below every deadline
    tasks.append(dict(M=4, T=[1000, 2000, 4000], D=[1000, 2000, 4000], C_seq=[5, 5, 5], C_par=[20, 40, 80],
                      k_permille=[1000, 1000, 1000], type=[0, 0, 1]))
    # heavy: utilisation near 1 on the chosen part, busy period past the largest deadline
    tasks.append(dict(M=2, T=[10, 15, 35], D=[10, 15, 35], C_seq=[2, 3, 4], C_par=[4, 6, 12],
                      k_permille=[1000, 1000, 1000], type=[0, 0, 0]))
    rng = np.random.default_rng(55)
    for _ in range(120):
        n = int(rng.integers(2, 9))
        T = rng.integers(20, 400, n)
        u = rng.dirichlet(np.ones(n)) * float(rng.uniform(0.3, 1.8))
        Cp = np.maximum(1, (u * T * rng.uniform(0.5, 1.0, n)).astype(np.int64))
        Cs = np.maximum(0, (u * T).astype(np.int64) - Cp)
        tasks.append(dict(M=int(rng.integers(1, 7)), T=T, D=T, C_seq=Cs, C_par=Cp,
                          k_permille=rng.choice([1000, 1200, 2300], n), type=rng.integers(0, 2, n)))
    ts = as_batch(tasks)
    for K, mode in ((1, "BF_INA"), (3, "BF_INA"), (3, "SMS_ACT"), (2, "EXH")):
        want = oracle.solve(ts, K, mode, policy="EDF")
        got = eng.solve(ts, K, mode, policy="EDF")
        same(got, want, FIELDS, f"EDF report K={K} {mode}")
        say(f"EDF report K={K} {mode}: {int(got['verdict'].sum())} of {ts.n_sets} schedulable, "
            f"{int((got['R'] > 0).sum())} response times")
