"""The necessary condition by which the engine skips partitionings without
evaluating them (every schedulable partition has utilisation at most 1; a
task on a part of at most m_1 units needs at least its utilisation on m_1
units; at most one task of each type per part escapes conflict), restated on
the host with the oracle's execution times, is sound: every partitioning it
rules out has no schedulable allocation in the oracle's exhaustive search,
under both policies.  It fires on a good share of the partitionings of
loaded sets, so the check is not vacuous."""
import numpy as np
import pytest

import oracle
from paper_2105_10312_amd import workload

Q = 1 << 32


def ceil_term(C, T):
    return (1 << 32) + 1 if C > T else -((-C * Q) // T)


def ruled_out(task, m1, k):
    n = len(task["T"])
    T = [int(x) for x in task["T"]]
    un = [ceil_term(oracle.exec_time(task, i, m1, False), T[i]) for i in range(n)]
    uc = [ceil_term(oracle.exec_time(task, i, m1, True), T[i]) for i in range(n)]
    sav = [max(0, uc[i] - un[i]) for i in range(n)]
    mem = sorted((sav[i] for i in range(n) if int(task["type"][i]) == 1), reverse=True)
    cmp_ = sorted((sav[i] for i in range(n) if int(task["type"][i]) == 0), reverse=True)
    return sum(uc) - sum(mem[:k]) - sum(cmp_[:k]) >= n + k * Q


@pytest.mark.parametrize("policy", ["FP_DM", "EDF"])
def test_ruled_out_partitionings_have_no_schedulable_allocation(policy):
    rng = np.random.default_rng(17 if policy == "FP_DM" else 18)
    fired = checked = 0
    for _ in range(160):
        n = int(rng.integers(2, 7))
        M = int(rng.integers(2, 11))
        T = rng.integers(10, 80, n)
        D = np.array([int(rng.integers(max(1, t * 2 // 3), t + 1)) for t in T])
        C1 = np.maximum(1, (T * rng.uniform(0.2, 1.6, n)).astype(np.int64))
        Cs = (C1 * rng.uniform(0.0, 0.3, n)).astype(np.int64)
        ty = rng.integers(0, 2, n)
        task = dict(M=M, T=T, D=D, C_seq=Cs, C_par=C1 - Cs, k_permille=np.where(ty == 1, 2300, 1200), type=ty)
        for row in oracle.enumerate_partitionings(M, 4):
            sz = [int(x) for x in row if x > 0]
            if not ruled_out(task, sz[0], len(sz)):
                continue
            fired += 1
            ts = workload.TaskSets(set_offset=np.array([0, n], np.int64), M=np.array([M], np.int32),
                                   T=np.asarray(T, np.int64), D=np.asarray(D, np.int64),
                                   C_seq=np.asarray(Cs, np.int64), C_par=np.asarray(C1 - Cs, np.int64),
                                   k_permille=np.asarray(task["k_permille"], np.int32),
                                   type=np.asarray(ty, np.uint8))
            if policy == "FP_DM":
                assert not oracle.best_on_partitioning(task, sz, "EXH")[0], (task, sz)
            else:
                r = oracle.solve(ts, len(sz), "EXH", flags=oracle.FLAG_NO_LEMMA1, admissible=tuple(sorted(set(sz))),
                                 policy="EDF")
                # no schedulable partitioning made of these sizes at all, so none is this one
                assert not (r["verdict"][0] and sorted(r["sizes"][0][r["sizes"][0] > 0].tolist()) == sorted(sz)), \
                    (task, sz)
            checked += 1
    assert fired >= 100 and checked == fired
