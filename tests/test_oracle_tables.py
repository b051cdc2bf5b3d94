"""The oracle with explicit per-task time tables (Cn[m], Cc[m] for m = 1..M)
instead of the parametric model, pinned three ways: tables written from the
parametric model (by the independent Python model in brute.py) change no
result; on tiny sets with general tables (saturating memory-intensive
profiles) the exhaustive optimum, the whole-GPU baseline and Algorithm 1's
partitions agree with discrete-time simulation; and tables outside the
contract are rejected."""
import numpy as np
import pytest

import oracle
from brute import best_exhaustive, exec_time, partition_feasible, whole_gpu
from paper_2105_10312_amd import workload

FIELDS = ("status", "verdict", "verdict_1g", "pidx", "sizes", "aidx", "maxU", "sumU", "n_evals", "alloc", "R",
          "R_1g")


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


def tiny_sets(seed, count, nmax=4, Mmax=6):
    rng = np.random.default_rng(seed)
    n = rng.integers(1, nmax + 1, count)
    M = rng.integers(1, Mmax + 1, count)
    U = rng.uniform(0.4, 1.0, count) * np.minimum(M, n) * 0.9
    return workload.gen_sets(seed, n, U, M, tmin=10, tmax=60)


@pytest.mark.parametrize("mode,K", [("EXH", 3), ("BF_INA", 4), ("SMS_ACT", 4)])
def test_model_tables_change_nothing(mode, K):
    ts = workload.config_c1(n_sets=40) if mode == "EXH" else workload.subset(workload.config_c2(n_sets=200),
                                                                             np.arange(40))
    want = oracle.solve(ts, K, mode)
    got = oracle.solve(model_tables(ts), K, mode)
    for f in FIELDS:
        assert np.array_equal(got[f], want[f]), f


def test_model_tables_change_nothing_alg1():
    ts = workload.config_paper_fig4(sets_per_point=1, U_points=[10, 30, 42, 44, 46])
    tt = model_tables(ts)
    for mode in ("BF_INA", "SMS_ACT"):
        for s in range(ts.n_sets):
            a, b = oracle.alg1(ts.set(s), mode), oracle.alg1(tt.set(s), mode)
            for f in ("verdict", "k", "tried", "merged"):
                assert a[f] == b[f]
            for f in ("sizes", "alloc", "R"):
                assert np.array_equal(a[f], b[f])


def test_general_tables_exhaustive_matches_brute_force():
    ts = workload.with_time_tables(tiny_sets(71, 60), seed=72)
    got = oracle.solve(ts, 3, "EXH")
    for s in range(ts.n_sets):
        task = ts.set(s)
        found, mx, sm, pidx, aidx, sizes, alloc = best_exhaustive(task, 3)
        assert bool(got["verdict"][s]) == found, s
        if found:
            assert (int(got["maxU"][s]), int(got["sumU"][s]), int(got["pidx"][s]), int(got["aidx"][s])) == \
                (mx, sm, pidx, aidx), s
        ok1g, R1g = whole_gpu(task)
        assert bool(got["verdict_1g"][s]) == ok1g
        a = int(ts["set_offset"][s])
        assert list(got["R_1g"][a:a + len(task["T"])]) == R1g


def test_general_tables_alg1_partitions_simulate_feasible():
    ts = workload.with_time_tables(tiny_sets(73, 80, nmax=5, Mmax=8), seed=74)
    seen = 0
    for s in range(ts.n_sets):
        task = ts.set(s)
        for mode in ("BF_INA", "SMS_INA", "BF_ACT"):
            r = oracle.alg1(task, mode)
            if not r["verdict"]:
                continue
            seen += 1
            assert int(np.sum(r["sizes"])) <= task["M"]
            for p, m in enumerate(r["sizes"]):
                mem = [i for i in range(len(task["T"])) if r["alloc"][i] == p]
                assert partition_feasible(task, mem, int(m))[0]
    assert seen > 20


def test_tables_outside_the_contract_are_rejected():
    ts = workload.with_time_tables(workload.config_c1(n_sets=6), seed=75)
    base = oracle.solve(ts, 3, "BF_INA")["status"]
    assert (base == oracle.OK).all()
    M = int(ts["M"][0])
    bad = []
    t = workload.TaskSets({k: v.copy() for k, v in ts.items()})
    t["Cn_table"][1] = t["Cn_table"][0] + 1                  # rises from m = 1 to 2
    bad.append(t)
    t = workload.TaskSets({k: v.copy() for k, v in ts.items()})
    t["Cc_table"][2] = t["Cn_table"][2] - 1                  # faster in conflict
    bad.append(t)
    t = workload.TaskSets({k: v.copy() for k, v in ts.items()})
    t["Cn_table"][M - 1] = 1                                 # super-linear speed-up
    t["Cc_table"][M - 1] = 1
    bad.append(t)
    t = workload.TaskSets({k: v.copy() for k, v in ts.items()})
    t["Cn_table"][:M] = 1 << 31                              # too large
    t["Cc_table"][:M] = 1 << 31
    bad.append(t)
    for t in bad:
        st = oracle.solve(t, 3, "BF_INA")["status"]
        assert st[0] == oracle.E_RANGE and (st[1:] == oracle.OK).all()
