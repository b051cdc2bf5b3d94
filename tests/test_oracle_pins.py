"""Pins for the CPU oracle: worked examples, closed forms, brute force and
invariants.  None of these re-types the oracle's own code: the expected values
come from hand derivations (tests/golden), textbook results, a discrete-time
schedule simulation, direct set-partition enumeration or mathematical
properties of the method."""
import itertools
import json
import os
import random
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import brute
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def as_task(d):
    return {"M": int(d["M"]), "T": np.array(d["T"], np.int64), "D": np.array(d["D"], np.int64),
            "C_seq": np.array(d["C_seq"], np.int64), "C_par": np.array(d["C_par"], np.int64),
            "k_permille": np.array(d["k_permille"], np.int32), "type": np.array(d["type"], np.uint8)}


def as_batch(tasks):
    off = np.zeros(len(tasks) + 1, np.int64)
    off[1:] = np.cumsum([len(t["T"]) for t in tasks])
    b = {"set_offset": off, "M": np.array([t["M"] for t in tasks], np.int32)}
    for key, dt in (("T", np.int64), ("D", np.int64), ("C_seq", np.int64), ("C_par", np.int64),
                    ("k_permille", np.int32), ("type", np.uint8)):
        b[key] = np.concatenate([np.asarray(t[key], dt) for t in tasks]) if tasks else np.zeros(0, dt)
    return b


def rand_task(rng, n, M, tmax=30, kchoices=(1000, 1200, 2300)):
    T = [rng.randint(2, tmax) for _ in range(n)]
    D = [rng.randint(1, t) for t in T]
    Cs = [rng.randint(0, 4) for _ in range(n)]
    Cp = [rng.randint(0 if Cs[i] > 0 else 1, 3 * M) for i in range(n)]
    return as_task(dict(M=M, T=T, D=D, C_seq=Cs, C_par=Cp,
                        k_permille=[rng.choice(kchoices) for _ in range(n)],
                        type=[rng.randint(0, 1) for _ in range(n)]))


# ---- worked examples ---------------------------------------------------------

def test_w1_worked_example():
    w = load("w1_worked_example.json")
    t = as_task(w["set"])
    assert [oracle.m_min(t, i) for i in range(3)] == w["m_min"]
    assert [oracle.u1(t, i) for i in range(3)] == w["u1"]
    assert not oracle.lemma1_reject(t)
    f, R, _, _ = oracle.eval_triple(t, [8], [0, 0, 0])
    assert f == w["whole_gpu"]["schedulable"] and R.tolist() == w["whole_gpu"]["R"]
    r = oracle.solve(as_batch([t]), w["K"], "EXH")
    e = w["exhaustive"]
    assert int(r["verdict"][0]) == e["verdict"] and int(r["pidx"][0]) == e["pidx"]
    assert r["sizes"][0].tolist() == e["sizes"] and r["alloc"].tolist() == e["alloc"]
    assert int(r["aidx"][0]) == e["aidx"] and r["R"].tolist() == e["R"]
    assert int(r["maxU"][0]) == e["maxU"] and int(r["sumU"][0]) == e["sumU"]
    assert r["R_1g"].tolist() == w["whole_gpu"]["R"] and int(r["verdict_1g"][0]) == 0
    for pidx, v in w["exhaustive_feasible_on"].items():
        f, R, mx, sm = oracle.eval_triple(t, v["sizes"], v["alloc"])
        assert f and R.tolist() == v["R"] and mx == max(v["U"]) and sm == sum(v["U"])


def test_w1_heuristic_traces():
    w = load("w1_worked_example.json")
    t = as_task(w["set"])
    parts = oracle.enumerate_partitionings(8, 3)
    for mode, want in (("BF_INA", w["heuristic_ina_feasible_pidx"]), ("SMS_INA", w["heuristic_ina_feasible_pidx"]),
                       ("BF_ACT", w["heuristic_act_feasible_pidx"]), ("SMS_ACT", w["heuristic_act_feasible_pidx"])):
        got = []
        for p, row in enumerate(parts):
            sz = [x for x in row if x > 0]
            if oracle.heuristic(t, sz, mode) is not None:
                got.append(p)
        assert got == want, mode
    assert oracle.heuristic(t, [5, 3], "BF_INA") is None
    assert oracle.heuristic(t, [6, 2], "BF_INA").tolist() == [0, 0, 1]
    assert oracle.heuristic(t, [3, 3, 2], "BF_INA").tolist() == [0, 1, 2]
    # ACT forbids every pair of the example (each pair needs m_min_i + m_min_j units)
    for i, j in itertools.combinations(range(3), 2):
        assert oracle.forbidden(t, i, j)
    for mode in ("BF_INA", "SMS_INA", "BF_ACT", "SMS_ACT"):
        r = oracle.solve(as_batch([t]), 3, mode)
        assert int(r["pidx"][0]) == 9 and r["alloc"].tolist() == [0, 1, 2]


def test_w5_bf_and_sms_rank_differently():
    """A fixed partitioning on which the two orders of H(pi) place a task on
    different parts (hand-derived, tests/golden/w5_bf_vs_sms.json): BF's lower
    merged utilisation puts b beside a, SMS's fewest units puts b alone."""
    w = load("w5_bf_vs_sms.json")
    t = as_task(w["set"])
    for mode, alloc in w["alloc"].items():
        assert oracle.heuristic(t, w["partitioning"], mode).tolist() == alloc, mode
    for mode in ("BF_INA", "SMS_INA"):
        f, R, mx, sm = oracle.eval_triple(t, w["partitioning"], w["alloc"][mode])
        assert f and R.tolist() == w["R"][mode] and [mx, sm] == w["key"][mode], mode
        r = oracle.solve(as_batch([t]), 2, mode, admissible=tuple(w["admissible"]))
        assert int(r["verdict"][0]) == 1 and int(r["pidx"][0]) == w["pidx"] and int(r["n_evals"][0]) == w["n_evals"]
        assert r["alloc"].tolist() == w["alloc"][mode] and r["R"].tolist() == w["R"][mode], mode
        assert [int(r["maxU"][0]), int(r["sumU"][0])] == w["key"][mode], mode
        assert r["R_1g"].tolist() == w["R_1g"]
    assert oracle.forbidden(t, 0, 1)


def test_w2_rta_textbook():
    w = load("w2_rta_textbook.json")
    t = as_task(w["set"])
    f, R, _, _ = oracle.eval_triple(t, [1], [0, 0, 0])
    assert f and R.tolist() == w["R"]


def test_w3_conflict_example():
    w = load("w3_conflict_example.json")
    for case, top_type, want in (("A", 1, w["Cn4"]), ("B", 0, w["Cc4"])):
        types = [0] * 9 + [1]
        D = [1000] * 10
        top = 9 if top_type == 1 else 0
        D[top] = 500
        t = as_task(dict(M=4, T=[1000] * 10, D=D, C_seq=[10] * 10, C_par=[40] * 10, k_permille=[1500] * 10,
                         type=types))
        f, R, _, _ = oracle.eval_triple(t, [4], [0] * 10)
        assert R[top] == want, case
    assert oracle.exec_time(t, 0, 4, False) == w["Cn4"] and oracle.exec_time(t, 0, 4, True) == w["Cc4"]


# ---- closed forms --------------------------------------------------------------

def test_time_model_closed_form():
    rng = random.Random(7)
    for _ in range(300):
        cs, cp = rng.randint(0, 10**6), rng.randint(0, 10**7)
        if cs + cp == 0:
            cp = 1
        k = rng.choice([1000, 1001, 1200, 2300, 999999])
        t = as_task(dict(M=255, T=[2**31 - 1], D=[2**31 - 1], C_seq=[cs], C_par=[cp], k_permille=[k], type=[0]))
        prev_n = prev_c = None
        for m in (1, 2, 3, 7, 8, 64, 80, 107, 108, 255):
            cn = oracle.exec_time(t, 0, m, False)
            cc = oracle.exec_time(t, 0, m, True)
            exact_n = Fraction(cs) + Fraction(cp, m)
            assert cn - 1 < exact_n <= cn  # ceiling of a/m + b
            assert cc - 1 < Fraction(k * cn, 1000) <= cc
            if prev_n is not None:
                assert cn <= prev_n and cc <= prev_c  # no timing anomalies
            prev_n, prev_c = cn, cc
        t1000 = dict(t, k_permille=np.array([1000], np.int32))
        assert oracle.exec_time(t1000, 0, 5, True) == oracle.exec_time(t1000, 0, 5, False)


def test_lemma2_closed_form():
    rng = random.Random(11)
    for _ in range(2000):
        M = rng.randint(1, 120)
        T = rng.randint(1, 5000)
        D = rng.randint(1, T)
        cs = rng.randint(0, 2 * D)
        cp = rng.randint(0, 50 * D)
        if cs + cp == 0:
            cs = 1
        t = as_task(dict(M=M, T=[T], D=[D], C_seq=[cs], C_par=[cp], k_permille=[1200], type=[0]))
        if cp == 0:
            want = 1 if cs <= D else oracle.M_INF
        elif D > cs:
            want = -(-cp // (D - cs))
            if want > M:
                want = oracle.M_INF
        else:
            want = oracle.M_INF
        assert oracle.m_min(t, 0) == want


def _partition_count_gf(M, K):
    # coefficient of x^M in prod_{j=1..K} 1/(1-x^j): partitions into parts <= K,
    # conjugate to partitions into at most K parts
    c = [1] + [0] * M
    for j in range(1, K + 1):
        for s in range(j, M + 1):
            c[s] += c[s - j]
    return c[M]


@pytest.mark.parametrize("M,K,want", [(8, 3, 10), (16, 4, 64), (48, 4, 1033), (80, 4, 4263), (108, 4, 10018)])
def test_enumeration_counts(M, K, want):
    assert oracle.count_partitionings(M, K) == want == _partition_count_gf(M, K)


@pytest.mark.parametrize("M,K", [(1, 1), (1, 4), (5, 8), (8, 3), (12, 2), (30, 4), (40, 6)])
def test_enumeration_order(M, K):
    tab = oracle.enumerate_partitionings(M, K)
    assert len(tab) == _partition_count_gf(M, K)
    rows = [tuple(int(x) for x in r) for r in tab]
    assert rows == sorted(rows, reverse=True) and len(set(rows)) == len(rows)
    for r in rows:
        nz = [x for x in r if x > 0]
        assert sum(nz) == M and list(nz) == sorted(nz, reverse=True) and len(nz) <= K
        assert all(x == 0 for x in r[len(nz):])
    assert rows[0][0] == M


def test_w1_enumeration_listing():
    want = [(8,), (7, 1), (6, 2), (6, 1, 1), (5, 3), (5, 2, 1), (4, 4), (4, 3, 1), (4, 2, 2), (3, 3, 2)]
    got = [tuple(int(x) for x in r if x > 0) for r in oracle.enumerate_partitionings(8, 3)]
    assert got == want == brute.integer_partitions_desc(8, 3)


# ---- brute force ---------------------------------------------------------------

def test_rta_vs_simulation():
    rng = random.Random(3)
    for _ in range(400):
        n = rng.randint(1, 5)
        M = rng.randint(1, 6)
        t = rand_task(rng, n, M, tmax=25)
        m = rng.randint(1, M)
        f, R, _, _ = oracle.eval_triple(t, [m], [0] * n, early_exit=False)
        members = list(range(n))
        C = []
        for i in members:
            same = sum(1 for j in members if t["type"][j] == t["type"][i])
            C.append(brute.exec_time(int(t["C_seq"][i]), int(t["C_par"][i]), int(t["k_permille"][i]), m, same >= 2))
        order = sorted(members, key=lambda i: (int(t["D"][i]), int(t["T"][i]), i))
        prio = [order.index(i) for i in members]
        sim = brute.simulate_fp(C, [int(x) for x in t["T"]], [int(x) for x in t["D"]], prio)
        assert R.tolist() == sim
        assert f == all(r >= 0 for r in sim)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(0, 2**32 - 1))
def test_exhaustive_vs_bruteforce(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 4)
    M = rng.randint(1, 6)
    K = rng.randint(1, 3)
    t = rand_task(rng, n, M, tmax=20)
    r = oracle.solve(as_batch([t]), K, "EXH", flags=oracle.FLAG_NO_LEMMA1 if seed % 2 else 0)
    found, mx, sm, pidx, aidx, sizes, alloc = brute.best_exhaustive(t, K)
    assert bool(r["verdict"][0]) == found
    if found:
        assert (int(r["maxU"][0]), int(r["sumU"][0]), int(r["pidx"][0]), int(r["aidx"][0])) == (mx, sm, pidx, aidx)
        assert [x for x in r["sizes"][0].tolist() if x > 0] == list(sizes)
        assert r["alloc"].tolist() == alloc
        # response times of the chosen triple, by simulation per partition
        for p, m in enumerate(sizes):
            mem = [i for i in range(n) if alloc[i] == p]
            C = []
            for i in mem:
                same = sum(1 for j in mem if t["type"][j] == t["type"][i])
                C.append(brute.exec_time(int(t["C_seq"][i]), int(t["C_par"][i]), int(t["k_permille"][i]), m,
                                         same >= 2))
            order = sorted(mem, key=lambda i: (int(t["D"][i]), int(t["T"][i]), i))
            sim = brute.simulate_fp(C, [int(t["T"][i]) for i in mem], [int(t["D"][i]) for i in mem],
                                    [order.index(i) for i in mem])
            assert [int(r["R"][i]) for i in mem] == sim
    else:
        assert int(r["pidx"][0]) == -1 and all(x == -1 for x in r["alloc"].tolist())
    ok1g, R1g = brute.whole_gpu(t)
    assert bool(r["verdict_1g"][0]) == ok1g and r["R_1g"].tolist() == R1g


# ---- invariants -----------------------------------------------------------------

def _rand_batch(seed, nsets, nmax, Mmax, tmax=40):
    rng = random.Random(seed)
    return [rand_task(rng, rng.randint(1, nmax), rng.randint(1, Mmax), tmax=tmax) for _ in range(nsets)]


@pytest.mark.parametrize("mode", ["EXH", "BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_I1_single_partition_is_whole_gpu(mode):
    tasks = _rand_batch(21, 60, 5, 8)
    r = oracle.solve(as_batch(tasks), 1, mode)
    if mode.endswith("ACT"):
        # forbidden pairs may keep ACT from co-locating tasks that the whole GPU
        # schedules; it never accepts a set the whole GPU rejects
        assert (r["verdict"] <= r["verdict_1g"]).all()
        assert (r["verdict"] < r["verdict_1g"]).any()
    else:
        assert (r["verdict"] == r["verdict_1g"]).all()
    feas = np.repeat(r["verdict"].astype(bool), [len(t["T"]) for t in tasks])
    assert (r["R"][feas] == r["R_1g"][feas]).all()


def test_I2_no_interference_is_classical_rta():
    rng = random.Random(5)
    for _ in range(200):
        n, M = rng.randint(1, 5), rng.randint(1, 6)
        t = rand_task(rng, n, M, tmax=25, kchoices=(1000,))
        m = rng.randint(1, M)
        C = [brute.exec_time(int(t["C_seq"][i]), int(t["C_par"][i]), 1000, m, False) for i in range(n)]
        order = sorted(range(n), key=lambda i: (int(t["D"][i]), int(t["T"][i]), i))
        sim = brute.simulate_fp(C, [int(x) for x in t["T"]], [int(x) for x in t["D"]],
                                [order.index(i) for i in range(n)])
        _, R, _, _ = oracle.eval_triple(t, [m], [0] * n)
        assert R.tolist() == sim


@pytest.mark.parametrize("mode", ["EXH"])
def test_I3_verdict_monotone_in_M(mode):
    tasks = _rand_batch(31, 40, 4, 6)
    for t in tasks:
        prev, prev1 = 0, 0
        for M in range(1, 9):
            r = oracle.solve(as_batch([dict(t, M=M)]), 3, mode)
            assert int(r["verdict"][0]) >= prev and int(r["verdict_1g"][0]) >= prev1
            prev, prev1 = int(r["verdict"][0]), int(r["verdict_1g"][0])


def test_I3_fixed_triple_monotone_in_sizes():
    rng = random.Random(41)
    for _ in range(300):
        n, M = rng.randint(1, 6), 20
        t = rand_task(rng, n, M, tmax=40)
        k = rng.randint(1, 3)
        sizes = [rng.randint(1, 6) for _ in range(k)]
        alloc = [rng.randrange(k) for _ in range(n)]
        f0 = oracle.eval_triple(t, sizes, alloc)[0]
        bigger = [s + rng.randint(0, 3) for s in sizes]
        f1 = oracle.eval_triple(t, bigger, alloc)[0]
        assert f1 >= f0


def test_I4_relabel_equal_size_parts():
    rng = random.Random(43)
    for _ in range(300):
        n = rng.randint(1, 6)
        t = rand_task(rng, n, 20, tmax=40)
        sizes = [4, 4, 2]
        alloc = [rng.randrange(3) for _ in range(n)]
        swapped = [{0: 1, 1: 0}.get(a, a) for a in alloc]
        a = oracle.eval_triple(t, sizes, alloc)
        b = oracle.eval_triple(t, sizes, swapped)
        assert a[0] == b[0] and (not a[0] or (a[2], a[3]) == (b[2], b[3]))


@pytest.mark.parametrize("mode", ["EXH", "BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_I5_lemma1_never_changes_result(mode):
    tasks = _rand_batch(51, 80, 5, 6, tmax=30)
    a = oracle.solve(as_batch(tasks), 3, mode)
    b = oracle.solve(as_batch(tasks), 3, mode, flags=oracle.FLAG_NO_LEMMA1)
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    # and Lemma 1 fires on some of these sets
    assert any(oracle.lemma1_reject(t) for t in tasks)


def test_lemma1_rejects_only_infeasible():
    rng = random.Random(53)
    hits = 0
    for _ in range(300):
        t = rand_task(rng, rng.randint(1, 4), rng.randint(1, 5), tmax=15)
        if oracle.lemma1_reject(t):
            hits += 1
            assert not brute.best_exhaustive(t, 3)[0]
            # the exact utilisation really exceeds M
            u = sum(Fraction(int(t["C_seq"][i]) + int(t["C_par"][i]), int(t["T"][i])) for i in range(len(t["T"])))
            assert u > t["M"]
    assert hits > 0


def test_I6_permuting_tasks_keeps_exh_verdict_and_key():
    rng = random.Random(61)
    for _ in range(60):
        n = rng.randint(2, 5)
        t = rand_task(rng, n, rng.randint(2, 6), tmax=30)
        perm = list(range(n))
        rng.shuffle(perm)
        tp = dict(t)
        for key in ("T", "D", "C_seq", "C_par", "k_permille", "type"):
            tp[key] = t[key][perm]
        a = oracle.solve(as_batch([t]), 3, "EXH")
        b = oracle.solve(as_batch([tp]), 3, "EXH")
        assert a["verdict"][0] == b["verdict"][0]
        assert (a["maxU"][0], a["sumU"][0]) == (b["maxU"][0], b["sumU"][0])


def test_I7_feasibility_monotone_in_m_so_binary_search_equals_scan():
    rng = random.Random(71)
    for _ in range(300):
        n = rng.randint(1, 5)
        t = rand_task(rng, n, 32, tmax=60)
        feas = [oracle.eval_triple(t, [m], [0] * n, early_exit=True)[0] for m in range(1, 33)]
        # monotone: once feasible, stays feasible
        first = feas.index(True) if True in feas else None
        if first is not None:
            assert all(feas[first:])
            lo, hi = 1, 32  # binary search for the least feasible m
            while lo < hi:
                mid = (lo + hi) // 2
                if feas[mid - 1]:
                    hi = mid
                else:
                    lo = mid + 1
            assert lo == first + 1


# ---- heuristic self-consistency -------------------------------------------------

@pytest.mark.parametrize("mode", ["BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_heuristic_consistency(mode):
    rng = random.Random(81)
    for _ in range(120):
        n = rng.randint(1, 5)
        M = rng.randint(2, 8)
        t = rand_task(rng, n, M, tmax=40)
        parts = oracle.enumerate_partitionings(M, 3)
        for row in parts:
            sz = [int(x) for x in row if x > 0]
            al = oracle.heuristic(t, sz, mode)
            exh = oracle.best_on_partitioning(t, sz, "EXH")[0]
            if al is None:
                continue
            assert exh  # heuristic-feasible implies exhaustive-feasible
            f, _, _, _ = oracle.eval_triple(t, sz, al.tolist(), early_exit=True)
            assert f
            # brute force: every partition passes the simulation
            for p, m in enumerate(sz):
                assert brute.partition_feasible(t, [i for i in range(n) if al[i] == p], m)[0]
            if mode.endswith("ACT"):
                for i, j in itertools.combinations(range(n), 2):
                    if al[i] == al[j]:
                        assert not oracle.forbidden(t, i, j)


def test_forbidden_pairs_definition():
    # a pair is forbidden iff no size in [max(mi,mj), mi+mj-1] (capped at M)
    # schedules the two tasks together (Definition 3, Algorithm 2)
    rng = random.Random(91)
    for _ in range(200):
        M = rng.randint(2, 10)
        t = rand_task(rng, 2, M, tmax=30)
        mi, mj = oracle.m_min(t, 0), oracle.m_min(t, 1)
        if mi >= oracle.M_INF or mj >= oracle.M_INF:
            assert oracle.forbidden(t, 0, 1)
            continue
        ok = any(brute.partition_feasible(t, [0, 1], m)[0] for m in range(max(mi, mj), min(mi + mj - 1, M) + 1))
        assert oracle.forbidden(t, 0, 1) == (not ok)


# ---- validation ---------------------------------------------------------------------

def test_validation_codes():
    good = dict(M=8, T=[100], D=[100], C_seq=[1], C_par=[10], k_permille=[1200], type=[0])
    cases = [
        (dict(good, M=0), oracle.E_INVAL), (dict(good, M=256), oracle.E_INVAL),
        (dict(good, T=[0], D=[0]), oracle.E_RANGE), (dict(good, D=[101]), oracle.E_RANGE),
        (dict(good, D=[0]), oracle.E_RANGE), (dict(good, T=[2**31], D=[5]), oracle.E_RANGE),
        (dict(good, C_seq=[-1]), oracle.E_RANGE), (dict(good, C_seq=[0], C_par=[0]), oracle.E_RANGE),
        (dict(good, C_par=[2**31]), oracle.E_RANGE), (dict(good, k_permille=[999]), oracle.E_RANGE),
        (dict(good, k_permille=[1000001]), oracle.E_RANGE), (dict(good, type=[2]), oracle.E_RANGE),
        (good, oracle.OK),
    ]
    for d, want in cases:
        r = oracle.solve(as_batch([as_task(d)]), 3, "BF_INA")
        assert int(r["status"][0]) == want, d
        if want != oracle.OK:
            assert r["alloc"].tolist() == [-1] and r["R"].tolist() == [-1] and int(r["n_evals"][0]) == 0
    big = as_task(dict(M=8, T=[100] * 65, D=[100] * 65, C_seq=[1] * 65, C_par=[1] * 65, k_permille=[1200] * 65,
                       type=[0] * 65))
    assert int(oracle.solve(as_batch([big]), 3, "BF_INA")["status"][0]) == oracle.E_INVAL
    # exhaustive needs k^n < 2^62
    ex = as_task(dict(M=8, T=[100] * 40, D=[100] * 40, C_seq=[1] * 40, C_par=[1] * 40, k_permille=[1200] * 40,
                      type=[0] * 40))
    assert int(oracle.solve(as_batch([ex]), 3, "EXH")["status"][0]) == oracle.E_INVAL
