"""Exhaustive allocation on the GPU: plain enumeration (form 1) and subset
tables with pruned depth-first search (form 2) against the oracle, and the
exhaustive-search stress workload (n=12, M=48, K=4) on sampled partitionings."""
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
    capart.capart_set_tuning(e.ctx, 0, 0, 0, 0)
    e.close()


def solve_form(eng, ts, K, form, debug=False):
    capart.capart_set_tuning(eng.ctx, 0, 0, 0, form)
    try:
        return eng.solve(ts, K, "EXH", debug=debug)
    finally:
        capart.capart_set_tuning(eng.ctx, 0, 0, 0, 0)


@pytest.mark.parametrize("form", [1, 2])
def test_c1_both_forms(eng, form):
    ts = workload.config_c1()
    got = solve_form(eng, ts, 3, form)
    want = oracle.solve(ts, 3, "EXH", nthreads=THREADS)
    for f in FIELDS:
        assert np.array_equal(got[f], want[f]), (form, f)


def small_sets(n, M, n_sets, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    U = rng.uniform(0.5, 0.4 * M, n_sets)
    return workload.gen_sets(seed, np.full(n_sets, n), U, np.full(n_sets, M), tmin=1e3, tmax=1e6)


def test_forms_agree_and_match_oracle_n8(eng):
    ts = small_sets(8, 24, 60, seed=31)
    a = solve_form(eng, ts, 4, 1, debug=True)
    b = solve_form(eng, ts, 4, 2, debug=True)
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f
    assert np.array_equal(a["dbg_key"], b["dbg_key"])
    sub = workload.subset(ts, np.arange(3))
    want = oracle.solve(sub, 4, "EXH", nthreads=THREADS)
    for f in FIELDS:
        g = a[f][:3] if f not in ("alloc", "R", "R_1g") else a[f][:sub.n_tasks]
        assert np.array_equal(g, want[f]), f


def test_symmetric_sets_equal_parts(eng):
    # identical tasks and equal-size parts: many relabellings share a key, the
    # smallest allocation index must win
    t = dict(M=12, T=np.full(6, 100), D=np.full(6, 100), C_seq=np.full(6, 5), C_par=np.full(6, 60),
             k_permille=np.full(6, 1500), type=np.array([0, 1, 0, 1, 0, 1]))
    off = np.array([0, 6])
    ts = workload.TaskSets(set_offset=off, M=np.array([12], np.int32))
    for key, dt in (("T", np.int64), ("D", np.int64), ("C_seq", np.int64), ("C_par", np.int64),
                    ("k_permille", np.int32), ("type", np.uint8)):
        ts[key] = np.asarray(t[key], dt)
    want = oracle.solve(ts, 4, "EXH")
    for form in (1, 2):
        got = solve_form(eng, ts, 4, form, debug=True)
        for f in FIELDS:
            assert np.array_equal(got[f], want[f]), (form, f)


def test_c4_stress_sampled(eng):
    """The exhaustive stress workload (n=12, M=48, K=4) on 48 sets through the
    subset-table search; per-partitioning keys of sampled (set, partitioning)
    pairs compared with the oracle's plain enumeration of all k^12 maps."""
    full = workload.config_c4()
    ts = workload.subset(full, np.arange(48))
    say("c4: 48 sets, n=12, M=48, K=4")
    got = solve_form(eng, ts, 4, 2, debug=True)
    assert (got["status"] == 0).all() and (got["n_evals"] == 1033).all()
    parts = oracle.enumerate_partitionings(48, 4)
    nparts = (parts > 0).sum(1)
    smallest = np.where(parts > 0, parts, 99).min(1)
    rng = np.random.default_rng(4)
    checked = 0
    for s in rng.choice(ts.n_sets, 6, replace=False):
        task = ts.set(int(s))
        if oracle.lemma1_reject(task):
            continue
        # balanced partitionings are the ones most often schedulable
        cand = np.nonzero((nparts <= 3) & (smallest >= 6))[0]
        picks = list(rng.choice(cand, 3, replace=False))
        if s % 2 == 0:
            picks.append(int(rng.choice(np.nonzero((nparts == 4) & (smallest >= 6))[0])))
        for p in picks:
            sz = [int(x) for x in parts[p] if x > 0]
            f, al, mx, sm, ai = oracle.best_on_partitioning(task, sz, "EXH")
            k = got["dbg_key"][got["dbg_offset"][s] + p]
            if f:
                assert (int(k[0]), int(k[1]), int(k[2])) == (mx, sm, ai), (s, p)
            else:
                assert int(k[2]) == 2**64 - 1, (s, p)
            checked += 1
    assert checked >= 6
    # the exhaustive optimum is never worse than the heuristic's (same set)
    heur = eng.solve(ts, 4, "BF_INA")
    assert (got["verdict"] >= heur["verdict"]).all()
    both = (got["verdict"] == 1) & (heur["verdict"] == 1)
    g = [(int(a), int(b)) for a, b in zip(got["maxU"][both], got["sumU"][both])]
    h = [(int(a), int(b)) for a, b in zip(heur["maxU"][both], heur["sumU"][both])]
    assert all(x <= y for x, y in zip(g, h))


def test_c4_full_selection_matches_memo_oracle(eng):
    """The whole exhaustive search of 16 sets of the stress workload (every
    allocation of all 1,033 partitionings of 48 units into at most 4 parts)
    against the oracle's memoised exhaustive search, stored by
    tests/golden/make_c4_exhaustive.py: every output field, bit for bit,
    through the subset-table search (form 2) and, on two sets, through plain
    enumeration (form 1)."""
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden", "c4_exhaustive_16sets.json")) as f:
        g = json.load(f)
    idx = np.array(g["generator"]["indices"])
    ts = workload.subset(workload.config_c4(n_sets=g["generator"]["n_sets"]), idx)
    want = {f: np.array(g[f]) for f in FIELDS}
    assert want["verdict"].sum() >= 8
    say(f"c4 full selection: {ts.n_sets} sets, form 2")
    got = solve_form(eng, ts, g["K"], 2)
    for f in FIELDS:
        assert np.array_equal(np.asarray(got[f]).reshape(want[f].shape), want[f]), ("form 2", f)
    two = workload.subset(ts, np.array([int(np.argmax(want["verdict"])), 0]))
    say("c4 full selection: 2 sets, form 1")
    got1 = solve_form(eng, two, g["K"], 1)
    want2 = solve_form(eng, two, g["K"], 2)
    for f in FIELDS:
        assert np.array_equal(got1[f], want2[f]), ("form 1", f)
