"""The oracle's memoised exhaustive search (FLAG_EXH_FAST: every allocation
of every partitioning scored from a table of (task subset, size) tests)
against the plain exhaustive search, which decodes and tests every triple
directly: identical results, field by field, on random small sets (both
policies, admissible sizes, K up to 4) and on sets of the exhaustive stress
shape (12 tasks) with few parts."""
import numpy as np
import pytest

import oracle
from paper_2105_10312_amd import workload

FIELDS = ("status", "verdict", "verdict_1g", "pidx", "sizes", "aidx", "maxU", "sumU", "n_evals", "alloc", "R",
          "R_1g")


def same(a, b, label):
    for f in FIELDS:
        assert np.array_equal(np.asarray(a[f]), np.asarray(b[f])), (label, f)


def random_batch(seed, count, nmax, Mmax):
    rng = np.random.default_rng(seed)
    sets = []
    for _ in range(count):
        n = int(rng.integers(1, nmax + 1))
        M = int(rng.integers(1, Mmax + 1))
        T = rng.integers(8, 60, n)
        D = np.array([int(rng.integers(max(1, t // 2), t + 1)) for t in T])
        C1 = np.maximum(1, (T * rng.uniform(0.05, 0.9, n)).astype(np.int64))
        Cs = (C1 * rng.uniform(0.0, 0.5, n)).astype(np.int64)
        ty = rng.integers(0, 2, n)
        sets.append(dict(M=M, T=T, D=D, C_seq=Cs, C_par=C1 - Cs, k_permille=np.where(ty == 1, 2300, 1200), type=ty))
    off = np.concatenate([[0], np.cumsum([len(s["T"]) for s in sets])]).astype(np.int64)
    cat = lambda key, dt: np.concatenate([np.asarray(s[key], dt) for s in sets])
    return workload.TaskSets(set_offset=off, M=np.array([s["M"] for s in sets], np.int32), T=cat("T", np.int64),
                             D=cat("D", np.int64), C_seq=cat("C_seq", np.int64), C_par=cat("C_par", np.int64),
                             k_permille=cat("k_permille", np.int32), type=cat("type", np.uint8))


@pytest.mark.parametrize("K", [1, 2, 3, 4])
@pytest.mark.parametrize("policy", ["FP_DM", "EDF"])
def test_memo_search_equals_plain_search_on_small_sets(K, policy):
    ts = random_batch(100 + K, 120, 7 if K <= 3 else 6, 9)
    plain = oracle.solve(ts, K, "EXH", nthreads=8, policy=policy)
    fast = oracle.solve(ts, K, "EXH", flags=oracle.FLAG_EXH_FAST, nthreads=8, policy=policy)
    same(fast, plain, f"K={K} {policy}")
    assert plain["verdict"].sum() > 10 and (plain["verdict"] == 0).sum() > 5


def test_memo_search_with_admissible_sizes_and_without_lemma1():
    ts = random_batch(7, 100, 6, 8)
    for adm in ((1, 2, 4, 8), (3, 5)):
        plain = oracle.solve(ts, 3, "EXH", admissible=adm)
        fast = oracle.solve(ts, 3, "EXH", flags=oracle.FLAG_EXH_FAST, admissible=adm)
        same(fast, plain, f"admissible {adm}")
    nl = oracle.FLAG_NO_LEMMA1
    same(oracle.solve(ts, 3, "EXH", flags=nl | oracle.FLAG_EXH_FAST), oracle.solve(ts, 3, "EXH", flags=nl), "no L1")


def test_memo_search_on_twelve_task_sets():
    """Sets of the exhaustive stress config (12 tasks on 48 units) with at most
    two parts, and the same sets on 8 units with at most three parts."""
    c4 = workload.subset(workload.config_c4(n_sets=100), np.arange(24))
    same(oracle.solve(c4, 2, "EXH", flags=oracle.FLAG_EXH_FAST, nthreads=8), oracle.solve(c4, 2, "EXH", nthreads=8),
         "n=12 M=48 K=2")
    assert plain_k2_has_both(c4)
    # on 8 units, with the times scaled by 1/4 so that most sets fit
    small = workload.subset(c4, np.arange(8))
    small["M"] = np.full(8, 8, np.int32)
    small["C_seq"] = small["C_seq"] // 4
    small["C_par"] = np.maximum(1, small["C_par"] // 4)
    want = oracle.solve(small, 3, "EXH", nthreads=8)
    same(oracle.solve(small, 3, "EXH", flags=oracle.FLAG_EXH_FAST, nthreads=8), want, "n=12 M=8 K=3")
    assert want["verdict"].sum() >= 4


def plain_k2_has_both(ts):
    v = oracle.solve(ts, 2, "EXH", nthreads=8)["verdict"]
    return v.sum() >= 3 and (v == 0).sum() >= 3
