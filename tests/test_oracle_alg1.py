"""Pins of the oracle's Algorithm 1 (free partition sizes): the hand-derived
merge example and the paper's worked set at M = 7 and 8, soundness by
discrete-time simulation of every partition returned (Lemma 3), structural
properties, and agreement with the exhaustive search over fixed partitionings
(a schedulable Algorithm 1 result is a feasible triple)."""
import json
import os

import numpy as np
import pytest

import oracle
from brute import partition_feasible, simulate_fp, task_time

GOLD = os.path.join(os.path.dirname(__file__), "golden")
MODES = ("BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT")


def load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def test_merge_example():
    g = load("w4_alg1_merge_example.json")
    for case in g["cases"]:
        task = dict(g["tasks"], M=case["M"])
        for mode in MODES:
            r = oracle.alg1(task, mode)
            assert r["verdict"] == case["verdict"], (case["M"], mode)
            if case["verdict"]:
                assert list(r["sizes"]) == case["sizes"]
                assert list(r["alloc"]) == case["alloc"]
                assert list(r["R"]) == case["R"]
                assert r["tried"] == case["tried"] and r["merged"] == case["merged"]


def test_orders_merge_different_partners():
    """A set on which order > (lower utilisation of the union) and order >>
    (fewer units of the valid merge) merge the operand with different partners
    (hand-derived, tests/golden/w6_alg1_orders.json)."""
    g = load("w6_alg1_orders.json")
    for variant in ("INA", "ACT"):  # ACT forbids no pair of this set beforehand
        for order in ("BF", "SMS"):
            want = g[f"{order}_INA"]
            r = oracle.alg1(g["set"], f"{order}_{variant}")
            assert r["verdict"] == want["verdict"] and list(r["sizes"]) == want["sizes"], order
            assert list(r["alloc"]) == want["alloc"] and list(r["R"]) == want["R"], order
            assert r["tried"] == want["tried"] and r["merged"] == want["merged"], order


def test_scheduled_workload():
    """The scheduled workload of Figs. 5 and 7 (hand-derived,
    tests/golden/w7_alg1_workload.json): two compute tasks that must share
    one unit are both in conflict (the worst load); on two units they stay
    apart (the best load)."""
    g = load("w7_alg1_workload.json")
    for case in g["cases"]:
        task = dict(g["set"], M=case["M"])
        for mode in MODES:
            r = oracle.alg1(task, mode)
            assert r["verdict"] == 1 and list(r["sizes"]) == case["sizes"], (case["M"], mode)
            assert r["workload"] == case["workload"], (case["M"], mode)
    assert g["best"] == g["cases"][1]["workload"] and g["worst"] == g["cases"][0]["workload"]


def test_workload_lies_between_the_bounds():
    """On random sets: best (no task in conflict) <= workload <= worst (every
    task in conflict), with equality to best exactly when no final partition
    holds two tasks of one type."""
    checked = 0
    for task in random_sets(61, 300):
        for mode in ("BF_INA", "SMS_ACT"):
            r = oracle.alg1(task, mode)
            if not r["verdict"]:
                assert r["workload"] == 0
                continue
            n = len(task["T"])
            ceil_q32 = lambda c, t: -((-c * (1 << 32)) // t)
            best = sum(ceil_q32(oracle.exec_time(task, i, 1, False), int(task["T"][i])) for i in range(n))
            worst = sum(ceil_q32(oracle.exec_time(task, i, 1, True), int(task["T"][i])) for i in range(n))
            assert best <= r["workload"] <= worst
            types = np.asarray(task["type"])
            clash = any(np.bincount(types[r["alloc"] == p], minlength=2).max() >= 2 for p in range(r["k"]))
            assert (r["workload"] == best) == (not clash or best == worst)
            checked += 1
    assert checked >= 100


def test_worked_example_m7_m8():
    w1 = load("w1_worked_example.json")
    g = load("w4_alg1_merge_example.json")["w1_cases"]
    task = {k: w1["tasks"][k] for k in ("T", "D", "C_seq", "C_par", "k_permille", "type")} \
        if "tasks" in w1 else None
    if task is None:
        task = dict(T=[100, 150, 200], D=[100, 150, 200], C_seq=[10, 5, 20], C_par=[200, 300, 240],
                    k_permille=[1200, 2300, 1200], type=[0, 1, 0])
    for mode in MODES:
        r8 = oracle.alg1(dict(task, M=8), mode)
        assert r8["verdict"] == 1 and list(r8["sizes"]) == g["M8"]["sizes"]
        assert list(r8["alloc"]) == g["M8"]["alloc"] and list(r8["R"]) == g["M8"]["R"]
        r7 = oracle.alg1(dict(task, M=7), mode)
        assert r7["verdict"] == 0
        assert r7["tried"] == (g["M7"]["tried_ACT"] if mode.endswith("ACT") else g["M7"]["tried_INA"])


def random_sets(seed, count, nmax=5, Mmax=8):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(1, nmax + 1))
        T = rng.integers(8, 40, n)
        C1 = np.maximum(1, (T * rng.uniform(0.1, 1.2, n)).astype(int))
        Cs = (C1 * rng.uniform(0.0, 0.4, n)).astype(int)
        Cp = np.maximum(C1 - Cs, 0)
        Cp[(Cs + Cp) == 0] = 1
        D = np.maximum(1, (T * rng.uniform(0.6, 1.0, n)).astype(int))
        ty = rng.integers(0, 2, n)
        k = np.where(ty == 1, 2300, 1200)
        yield dict(M=int(rng.integers(1, Mmax + 1)), T=T, D=D, C_seq=Cs, C_par=Cp, k_permille=k, type=ty)


@pytest.mark.parametrize("mode", MODES)
def test_soundness_by_simulation(mode):
    """Lemma 3: on success the sizes sum to at most M and every partition is
    schedulable on its own units; checked by simulating each partition from a
    synchronous release (response times equal too)."""
    succ = 0
    for task in random_sets(71, 400):
        r = oracle.alg1(task, mode)
        n = len(task["T"])
        if not r["verdict"]:
            assert r["k"] == 0 and (r["alloc"] == -1).all()
            continue
        succ += 1
        assert r["sizes"].sum() <= task["M"]
        assert r["k"] == n - r["merged"]
        assert sorted(set(r["alloc"].tolist())) == list(range(r["k"]))
        for p in range(r["k"]):
            members = [i for i in range(n) if r["alloc"][i] == p]
            ok, _ = partition_feasible(task, members, int(r["sizes"][p]))
            assert ok, (task, r, p)
            for i in members:
                assert r["sizes"][p] >= oracle.m_min(task, i)
    assert succ > 40


@pytest.mark.parametrize("mode", ["BF_ACT", "SMS_ACT"])
def test_act_never_colocates_forbidden_pairs(mode):
    for task in random_sets(72, 300):
        r = oracle.alg1(task, mode)
        if not r["verdict"]:
            continue
        n = len(task["T"])
        for i in range(n):
            for j in range(i + 1, n):
                if r["alloc"][i] == r["alloc"][j]:
                    assert not oracle.forbidden(task, i, j)


def test_init_partitions_when_they_fit():
    """When the Lemma 2 sizes already fit (Pi <= M) nothing is merged: one
    partition per task, ordered by decreasing utilisation."""
    seen = 0
    for task in random_sets(73, 300):
        n = len(task["T"])
        mm = [oracle.m_min(task, i) for i in range(n)]
        if max(mm) > task["M"] or sum(mm) > task["M"] or oracle.lemma1_reject(task):
            continue
        seen += 1
        for mode in MODES:
            r = oracle.alg1(task, mode)
            assert r["verdict"] == 1 and r["k"] == n and r["tried"] == 0
            assert sorted(r["sizes"].tolist()) == sorted(mm)
            for i in range(n):
                assert r["sizes"][r["alloc"][i]] == mm[i]
    assert seen > 20


@pytest.mark.parametrize("mode", MODES)
def test_success_implies_exhaustive_feasible(mode):
    """A schedulable result of Algorithm 1 is a feasible (partitioning,
    allocation) pair once its unused units join a part; so the exhaustive
    search over fixed partitionings with as many parts finds one too."""
    checked = 0
    for task in random_sets(74, 200, nmax=4, Mmax=7):
        r = oracle.alg1(task, mode)
        if not r["verdict"]:
            continue
        ts = {k: np.asarray(v) for k, v in task.items() if k != "M"}
        n = len(task["T"])
        batch = dict(set_offset=np.array([0, n], np.int64), M=np.array([task["M"]], np.int32),
                     T=np.asarray(task["T"], np.int64), D=np.asarray(task["D"], np.int64),
                     C_seq=np.asarray(task["C_seq"], np.int64), C_par=np.asarray(task["C_par"], np.int64),
                     k_permille=np.asarray(task["k_permille"], np.int32), type=np.asarray(task["type"], np.uint8))
        del ts
        want = oracle.solve(batch, max(1, r["k"]), "EXH")
        assert want["verdict"][0] == 1, (task, r)
        checked += 1
    assert checked > 20


def paper_sets_200(seed, points, per_point=1):
    """The paper's 200-task sets (Figs. 6-8: n = 200, M = 68)."""
    from paper_2105_10312_amd import workload
    ts = workload.config_paper_fig4(seed=seed, n=200, sets_per_point=per_point, U_points=points)
    return [ts.set(s) for s in range(ts.n_sets)]


@pytest.mark.parametrize("mode", MODES)
def test_soundness_at_200_tasks(mode):
    """Lemma 3 on a 200-task set of the paper's generator: the sizes fit in M,
    every task sits in one partition, each partition is at least its members'
    Lemma 2 sizes, and a discrete-time simulation of every partition from a
    synchronous release meets every deadline with the response times given;
    with ACT no forbidden pair shares a partition.  A set at a higher
    utilisation fails, and then no partition is reported."""
    task = paper_sets_200(62, [36])[0]
    n = len(task["T"])
    r = oracle.alg1(task, mode)
    assert r["verdict"] == 1
    assert r["k"] == n - r["merged"] and r["sizes"].sum() <= task["M"]
    assert sorted(set(r["alloc"].tolist())) == list(range(r["k"]))
    for p in range(r["k"]):
        members = [i for i in range(n) if r["alloc"][i] == p]
        m = int(r["sizes"][p])
        assert all(m >= oracle.m_min(task, i) for i in members)
        C = [task_time(task, i, m, sum(1 for j in members if task["type"][j] == task["type"][i]) >= 2)
             for i in members]
        T = [int(task["T"][i]) for i in members]
        D = [int(task["D"][i]) for i in members]
        order = sorted(range(len(members)), key=lambda a: (D[a], T[a], members[a]))
        prio = [order.index(a) for a in range(len(members))]
        resp = simulate_fp(C, T, D, prio)
        assert resp == [int(r["R"][i]) for i in members], (p, members)
        if mode.endswith("ACT"):
            for x in range(len(members)):
                for y in range(x + 1, len(members)):
                    assert not oracle.forbidden(task, members[x], members[y])
    bad = oracle.alg1(paper_sets_200(62, [50])[0], mode)
    assert bad["verdict"] == 0 and bad["k"] == 0 and (bad["alloc"] == -1).all() and (bad["R"] == -1).all()
    assert bad["workload"] == 0


def test_oracle_limits_at_200_tasks():
    """Sets of more than 64 tasks take Algorithm 1 only, with M <= 127
    (partition indices are int8)."""
    task = paper_sets_200(63, [30])[0]
    with pytest.raises(ValueError):
        oracle.alg1(dict(task, M=128), "BF_INA")
    with pytest.raises(ValueError):
        oracle.best_on_partitioning(task, [34, 34], "BF_INA")
    with pytest.raises(ValueError):
        oracle.forbidden(task, 0, 200)
