"""Parity of the HIP engine (through the C ABI) with the CPU oracle.

Integer method, so the bar is bit-exact equality of every output field:
status, verdict, verdict_1g, pidx, sizes, aidx, maxU, sumU, n_evals, alloc,
R and R_1g; per-partitioning debug keys are compared where noted."""
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


def assert_same(got, want, ts, label=""):
    off = ts["set_offset"]
    for f in FIELDS:
        g, w = np.asarray(got[f]), np.asarray(want[f])
        if g.shape != w.shape or not np.array_equal(g, w):
            bad = np.argwhere(g.reshape(w.shape) != w)[:5] if g.size == w.size else None
            detail = ""
            if bad is not None and len(bad):
                i = int(bad[0][0])
                if f in ("alloc", "R", "R_1g"):
                    s = int(np.searchsorted(off, i, side="right") - 1)
                    detail = f" first mismatch at task {i} (set {s}): got {g.ravel()[i]} want {w.ravel()[i]}"
                else:
                    detail = f" first mismatch at set {i}: got {g.reshape(w.shape)[i]} want {w[i]}"
            raise AssertionError(f"{label}: field {f} differs;{detail}")


def as_batch(tasks):
    off = np.zeros(len(tasks) + 1, np.int64)
    off[1:] = np.cumsum([len(t["T"]) for t in tasks])
    b = workload.TaskSets(set_offset=off, M=np.array([t["M"] for t in tasks], np.int32))
    for key, dt in (("T", np.int64), ("D", np.int64), ("C_seq", np.int64), ("C_par", np.int64),
                    ("k_permille", np.int32), ("type", np.uint8)):
        b[key] = np.concatenate([np.asarray(t[key], dt) for t in tasks])
    return b


# ---- config 1: exhaustive, in full -------------------------------------------------

def test_c1_exhaustive_full(eng):
    ts = workload.config_c1()
    say("c1 exhaustive: 100 sets n=5 M=8 K=3")
    got = eng.solve(ts, 3, "EXH")
    want = oracle.solve(ts, 3, "EXH", nthreads=THREADS)
    assert_same(got, want, ts, "c1 EXH")
    assert want["verdict"].sum() > 10 and (want["verdict"] == 0).sum() > 0


def test_c1_per_partitioning_debug_keys(eng):
    ts = workload.config_c1(seed=11, n_sets=40)
    got = eng.solve(ts, 3, "EXH", debug=True)
    parts = oracle.enumerate_partitionings(8, 3)
    keys = got["dbg_key"]
    for s in range(ts.n_sets):
        task = ts.set(s)
        lem = oracle.lemma1_reject(task)
        for p, row in enumerate(parts):
            sz = [int(x) for x in row if x > 0]
            f, al, mx, sm, ai = oracle.best_on_partitioning(task, sz, "EXH")
            k = keys[got["dbg_offset"][s] + p]
            if f and not lem:
                assert (int(k[0]), int(k[1]), int(k[2])) == (mx, sm, ai), (s, p)
            else:
                assert int(k[2]) == 2**64 - 1, (s, p)


# ---- config 2: heuristic allocation, seeded subsets -----------------------------------

@pytest.mark.parametrize("mode,nsets", [("BF_INA", 400), ("BF_ACT", 400), ("SMS_INA", 120), ("SMS_ACT", 200)])
def test_c2_heuristic_subset(eng, mode, nsets):
    full = workload.config_c2(n_sets=2000)
    rng = np.random.default_rng(7)
    ts = workload.subset(full, np.sort(rng.choice(full.n_sets, nsets, replace=False)))
    say(f"c2 {mode}: {nsets} sets n=10 M=80 K=4")
    got = eng.solve(ts, 4, mode)
    want = oracle.solve(ts, 4, mode, nthreads=THREADS)
    assert_same(got, want, ts, f"c2 {mode}")
    assert want["verdict"].mean() > 0.05


def test_c2_per_partitioning_debug_sample(eng):
    full = workload.config_c2(n_sets=50)
    ts = workload.subset(full, np.arange(4))
    got = eng.solve(ts, 4, "BF_INA", debug=True)
    parts = oracle.enumerate_partitionings(80, 4)
    rng = np.random.default_rng(3)
    for s in range(ts.n_sets):
        task = ts.set(s)
        lem = oracle.lemma1_reject(task)
        for p in rng.choice(len(parts), 150, replace=False):
            sz = [int(x) for x in parts[p] if x > 0]
            f, al, mx, sm, ai = oracle.best_on_partitioning(task, sz, "BF_INA")
            k = got["dbg_key"][got["dbg_offset"][s] + p]
            if f and not lem:
                assert (int(k[0]), int(k[1]), int(k[2])) == (mx, sm, 0), (s, p)
            else:
                assert int(k[2]) == 2**64 - 1, (s, p)


# ---- config 3 shape: uneven sets, constrained deadlines ------------------------------

def test_c3_uneven_subset(eng):
    full = workload.config_c3(n_sets=3000)
    rng = np.random.default_rng(9)
    # small M and n keep the oracle quick; the full mix is covered on samples below
    idx = [s for s in rng.permutation(full.n_sets) if full["M"][s] <= 48 and full.sizes()[s] <= 16][:250]
    ts = workload.subset(full, np.sort(idx))
    say("c3 BF_INA: 250 uneven sets")
    got = eng.solve(ts, 4, "BF_INA")
    want = oracle.solve(ts, 4, "BF_INA", nthreads=THREADS)
    assert_same(got, want, ts, "c3 BF_INA")


def test_c3_mixed_sizes_sample(eng):
    full = workload.config_c3(n_sets=400)
    rng = np.random.default_rng(10)
    idx = np.sort(rng.choice(full.n_sets, 24, replace=False))
    ts = workload.subset(full, idx)
    say("c3 BF_INA: 24 sets, all sizes")
    got = eng.solve(ts, 4, "BF_INA")
    want = oracle.solve(ts, 4, "BF_INA", nthreads=THREADS)
    assert_same(got, want, ts, "c3 mixed")


# ---- edge cases ------------------------------------------------------------------------

def edge_sets():
    rng = np.random.default_rng(123)
    t = []

    def mk(M, T, D, Cs, Cp, k, ty):
        return dict(M=M, T=np.array(T), D=np.array(D), C_seq=np.array(Cs), C_par=np.array(Cp),
                    k_permille=np.array(k), type=np.array(ty))

    t.append(mk(1, [10], [10], [3], [4], [1200], [0]))                      # n=1, M=1
    t.append(mk(1, [10], [10], [10], [1], [1200], [0]))                     # n=1, misses
    t.append(mk(5, [1, 50], [1, 50], [1, 0], [0, 5], [1000, 1000], [0, 1]))  # T=1 task: utilisation 1
    t.append(mk(6, [20, 20, 20], [20, 20, 20], [5, 5, 5], [30, 30, 30], [2300] * 3, [1, 1, 1]))  # all memory
    t.append(mk(6, [20, 20, 20], [20, 20, 20], [5, 5, 5], [30, 30, 30], [1200] * 3, [0, 0, 0]))  # all compute
    t.append(mk(4, [9, 9, 9, 9], [9, 9, 9, 9], [2, 2, 2, 2], [4, 4, 4, 4], [1000] * 4, [0, 1, 0, 1]))  # ties
    t.append(mk(8, [40, 40], [12, 12], [12, 0], [0, 96], [1200, 1200], [0, 1]))  # D = C exactly
    t.append(mk(8, [100] * 6, [100] * 6, [1] * 6, [800] * 6, [1200] * 6, [0, 1] * 3))  # Lemma 1 rejects
    t.append(mk(10, [2**31 - 1] * 3, [2**31 - 1] * 3, [2**30, 5, 7], [2**30 - 1, 9, 11], [1000000, 1200, 2300],
                [0, 0, 1]))                                                  # extreme values
    t.append(mk(3, [7, 11, 13], [5, 11, 13], [1, 1, 1], [2, 3, 4], [1500, 1500, 1500], [0, 1, 0]))
    return t


@pytest.mark.parametrize("mode", ["EXH", "BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
@pytest.mark.parametrize("K", [1, 2, 3])
def test_edge_cases(eng, mode, K):
    ts = as_batch(edge_sets())
    say(f"edge cases {mode} K={K}")
    got = eng.solve(ts, K, mode)
    want = oracle.solve(ts, K, mode, nthreads=THREADS)
    assert_same(got, want, ts, f"edge {mode} K={K}")


def large_sets():
    """Maximum sizes: n=64 tasks on 108 units, n=32 on 255 units, light enough
    that many partitionings are schedulable (deep heuristic paths)."""
    rng = np.random.default_rng(321)
    out = []
    for n, M, ulo, uhi, one_type in ((64, 108, 0.01, 0.08, True), (64, 108, 0.02, 0.12, False),
                                     (32, 255, 0.05, 0.4, False), (64, 128, 0.01, 0.1, False)):
        T = rng.integers(5000, 200000, n)
        C1 = np.maximum(1, (T * rng.uniform(ulo, uhi, n)).astype(np.int64))
        Cs = (C1 * rng.uniform(0.02, 0.1, n)).astype(np.int64)
        ty = np.zeros(n, np.int64) if one_type else rng.integers(0, 2, n)
        k = np.full(n, 1000) if one_type else np.where(ty == 1, 2300, 1200)
        D = np.maximum(Cs + (C1 - Cs + M - 1) // M, (T * rng.uniform(0.5, 1.0, n)).astype(np.int64))
        out.append(dict(M=M, T=T, D=np.minimum(D, T), C_seq=Cs, C_par=C1 - Cs, k_permille=k, type=ty))
    return out


@pytest.mark.parametrize("mode", ["BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_large_sets(eng, mode):
    ts = as_batch(large_sets())
    say(f"large sets {mode} K=3")
    got = eng.solve(ts, 3, mode)
    want = oracle.solve(ts, 3, mode, nthreads=THREADS)
    assert_same(got, want, ts, f"large {mode}")


def test_invalid_sets_are_reported_and_skipped(eng):
    good = dict(M=8, T=np.array([100, 200]), D=np.array([100, 150]), C_seq=np.array([5, 5]),
                C_par=np.array([100, 200]), k_permille=np.array([1200, 2300]), type=np.array([0, 1]))
    bad = [dict(good, M=0), dict(good, D=np.array([101, 150])), dict(good, type=np.array([0, 3])),
           dict(good, C_seq=np.array([0, 0]), C_par=np.array([0, 5])), dict(good, k_permille=np.array([999, 1000]))]
    sets = [good] + bad + [good]
    ts = as_batch(sets)
    for mode in ("EXH", "BF_INA"):
        got = eng.solve(ts, 3, mode)
        want = oracle.solve(ts, 3, mode)
        assert_same(got, want, ts, f"invalid {mode}")
        assert got["status"].tolist() == [0, -1, -2, -2, -2, -2, 0]


def test_k8_partitionings(eng):
    full = workload.config_c2(seed=21, n_sets=60)
    sets = []
    for s in range(30):
        d = full.set(s)
        d["M"] = 12
        sets.append(d)
    ts = as_batch(sets)
    for mode in ("BF_INA", "SMS_ACT"):
        got = eng.solve(ts, 8, mode)
        want = oracle.solve(ts, 8, mode, nthreads=THREADS)
        assert_same(got, want, ts, f"K=8 {mode}")


# ---- flags, launch forms, entry points ---------------------------------------------------

def test_flags_and_per_set_launch(eng):
    ts = workload.subset(workload.config_c2(n_sets=300), np.arange(60))
    base = eng.solve(ts, 4, "BF_INA")
    nol1 = eng.solve(ts, 4, "BF_INA", flags=capart.CAPART_FLAG_NO_LEMMA1)
    per = eng.solve(ts, 4, "BF_INA", flags=capart.CAPART_FLAG_PER_SET_LAUNCH)
    for f in FIELDS:
        assert np.array_equal(base[f], nol1[f]), f
        assert np.array_equal(base[f], per[f]), f
    skip = eng.solve(ts, 4, "BF_INA", flags=capart.CAPART_FLAG_SKIP_1G)
    assert (skip["R_1g"] == -1).all() and (skip["verdict_1g"] == 0).all()
    assert np.array_equal(skip["R"], base["R"]) and np.array_equal(skip["pidx"], base["pidx"])


@pytest.mark.parametrize("policy", ["FP_DM", "EDF"])
@pytest.mark.parametrize("mode", ["EXH", "BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_per_set_launch_matches_oracle(eng, mode, policy):
    """The plain one-launch-sequence-per-set path against the oracle, field by
    field: exhaustive on the n=5, M=8 sets, the heuristics on n=10, M=80 sets
    and on uneven sets with constrained deadlines."""
    if mode == "EXH":
        batches = [(workload.config_c1(n_sets=40, seed=21), 3)]
    else:
        c3 = workload.config_c3(n_sets=400, seed=22)
        small = np.nonzero(c3.sizes() <= 20)[0][:30]
        batches = [(workload.subset(workload.config_c2(n_sets=300, seed=23), np.arange(30)), 4),
                   (workload.subset(c3, small), 4)]
    for ts, K in batches:
        say(f"per-set launch {mode} {policy}: {ts.n_sets} sets")
        got = eng.solve(ts, K, mode, flags=capart.CAPART_FLAG_PER_SET_LAUNCH, policy=policy)
        want = oracle.solve(ts, K, mode, nthreads=THREADS, policy=policy)
        assert_same(got, want, ts, f"per-set {mode} {policy}")


def test_golden_bf_and_sms_rank_differently(eng):
    """The hand-derived partitioning on which BF and SMS place a task on
    different parts: the one-partitioning allocation and the solve restricted
    to that partitioning by admissible sizes."""
    import json
    with open(os.path.join(os.path.dirname(__file__), "golden", "w5_bf_vs_sms.json")) as f:
        w = json.load(f)
    task = dict(w["set"])
    ts = as_batch([task])
    for mode, alloc in w["alloc"].items():
        found, al, mx, sm = eng.allocate(task, w["partitioning"], 2, mode)[:4]
        assert found and al.tolist() == alloc, mode
        got = eng.solve(ts, 2, mode, admissible=tuple(w["admissible"]))
        assert int(got["pidx"][0]) == w["pidx"] and got["alloc"].tolist() == alloc, mode
        assert got["R_1g"].tolist() == w["R_1g"] and int(got["n_evals"][0]) == w["n_evals"]
        if mode in w["key"]:
            assert [mx, sm] == w["key"][mode] and got["R"].tolist() == w["R"][mode], mode
            assert [int(got["maxU"][0]), int(got["sumU"][0])] == w["key"][mode], mode


def test_async_device_path_matches_host_path(eng):
    import torch
    ts = workload.subset(workload.config_c2(n_sets=500), np.arange(200))
    host = eng.solve(ts, 4, "BF_INA")
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, 4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        capart.capart_solve_async(eng.ctx, dev, 4, "BF_INA", out, stream=stream, max_tasks=10, max_M=80)
    stream.synchronize()
    for f in FIELDS:
        g = out[f].cpu().numpy()
        w = host[f].ravel()
        assert np.array_equal(g[:w.size], w), f


def test_test_triple_matches_oracle(eng):
    rng = np.random.default_rng(5)
    full = workload.config_c2(seed=33, n_sets=80)
    for s in range(80):
        task = full.set(s)
        k = int(rng.integers(1, 5))
        sizes = np.sort(rng.integers(1, 30, k))[::-1].copy()
        sizes = np.maximum(1, (sizes * 80 // max(1, sizes.sum()))).astype(np.int32)
        alloc = rng.integers(0, k, len(task["T"])).astype(np.int8)
        f, R, mx, sm = eng.test_triple(task, sizes, alloc)
        wf, wR, wmx, wsm = oracle.eval_triple(task, sizes, alloc, early_exit=False)
        assert f == wf and R.tolist() == wR.tolist(), s
        if f:
            assert (mx, sm) == (wmx, wsm)


def test_allocate_matches_oracle(eng):
    full = workload.config_c2(seed=34, n_sets=30)
    parts = oracle.enumerate_partitionings(80, 4)
    rng = np.random.default_rng(6)
    for s in range(12):
        task = full.set(s)
        for p in rng.choice(len(parts), 4, replace=False):
            sz = [int(x) for x in parts[p] if x > 0]
            for mode in ("BF_INA", "SMS_ACT"):
                got = eng.allocate(task, sz, 4, mode)
                want = oracle.best_on_partitioning(task, sz, mode)
                if oracle.lemma1_reject(task):
                    assert not got[0]
                    continue
                assert got[0] == want[0], (s, p, mode)
                if want[0]:
                    assert got[1].tolist() == want[1].tolist() and got[2:4] == want[2:4]
    task = workload.config_c1().set(3)
    for sz in ([8], [5, 3], [3, 3, 2]):
        got = eng.allocate(task, sz, 3, "EXH")
        want = oracle.best_on_partitioning(task, sz, "EXH")
        assert got[0] == want[0] and (not want[0] or (got[1].tolist() == want[1].tolist() and got[2:] == want[2:]))


# ---- the benchmark's configuration at full size, sampled -----------------------------------

def test_c2_full_size_sampled(eng):
    """All 100,000 sets of the n=10, M=80 workload in one device launch, as the
    benchmark runs it; 300 sampled sets compared with the oracle, and
    properties that hold at any size checked on every set."""
    import torch
    ts = workload.config_c2()
    say("c2 full: 100000 sets, device path")
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, 4)
    capart.capart_solve_async(eng.ctx, dev, 4, "BF_INA", out, max_tasks=10, max_M=80)
    torch.cuda.synchronize()
    got = {f: out[f].cpu().numpy() for f in FIELDS}
    got["sizes"] = got["sizes"].reshape(-1, 4)
    assert (got["status"] == 0).all() and (got["n_evals"] == 4263).all()
    v = got["verdict"].astype(bool)
    assert (got["verdict_1g"] <= got["verdict"]).all()  # the whole GPU is partitioning 0
    assert (got["pidx"][v] >= 0).all() and (got["pidx"][~v] == -1).all()
    assert (got["sizes"][v].sum(1) == 80).all()
    assert (got["maxU"][v] <= 2**32 + 10).all()
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(ts.n_sets, 300, replace=False))
    sub = workload.subset(ts, idx)
    want = oracle.solve(sub, 4, "BF_INA", nthreads=THREADS)
    task_idx = np.concatenate([np.arange(ts["set_offset"][s], ts["set_offset"][s + 1]) for s in idx])
    gsub = {f: (got[f][task_idx] if f in ("alloc", "R", "R_1g") else got[f][idx]) for f in FIELDS}
    assert_same(gsub, want, sub, "c2 full sampled")


@pytest.mark.parametrize("mode", ["BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_frontier_and_direct_tests_agree(eng, mode):
    """Frontier lookups and direct response-time tests give identical results,
    per partitioning (debug keys) and per set."""
    parts = [workload.subset(workload.config_c2(seed=41, n_sets=400), np.arange(150)),
             workload.subset(workload.config_c3(seed=42, n_sets=600), np.arange(200))]
    for ts in parts:
        for K in (4, 8):
            capart.capart_set_tuning(eng.ctx, frontier=1)
            a = eng.solve(ts, K, mode, debug=True)
            capart.capart_set_tuning(eng.ctx, frontier=2, memo=-1)
            b = eng.solve(ts, K, mode, debug=True)
            capart.capart_set_tuning(eng.ctx)
            for f in FIELDS + ("dbg_key",):
                assert np.array_equal(a[f], b[f]), (mode, K, f)
    ts = parts[0]
    want = oracle.solve(ts, 4, mode, nthreads=THREADS)
    capart.capart_set_tuning(eng.ctx, frontier=1)
    got = eng.solve(ts, 4, mode)
    capart.capart_set_tuning(eng.ctx)
    assert_same(got, want, ts, f"frontier {mode}")


def memo_sets():
    """Sets above the frontier limit (the test memo's range): C3's uneven sets
    of 15..32 tasks, a few light ones on which most partitionings are
    schedulable (deep heuristic paths, many distinct subsets), and serving
    queries of 33..64 tasks."""
    c3 = workload.config_c3(seed=43, n_sets=2500)
    n = c3.sizes()
    pick = np.nonzero((n >= 15) & (c3["M"] <= 48))[0][:60]
    rng = np.random.default_rng(44)
    light = workload.gen_sets(45, rng.integers(15, 33, 8), rng.uniform(1.0, 4.0, 8), np.full(8, 24),
                              tmin=1e3, tmax=1e5)
    # 33..64 tasks (64-bit rank masks, two-word memo entries)
    c5 = workload.config_c5(seed=46, n_queries=600)
    n5 = c5.sizes()
    wide = np.nonzero((n5 > 32) & (c5["M"] <= 48))[0][:10]
    return workload.concat([workload.subset(c3, pick), light, workload.subset(c5, wide)])


@pytest.mark.parametrize("mode", ["BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_memo_matches_direct_tests(eng, mode):
    """The per-set test memo (default size, and a 256-entry table that fills
    up and falls back to direct tests), in both loop forms that use it, gives
    the same key on every partitioning as direct tests, and the oracle's
    results per set."""
    ts = memo_sets()
    say(f"memo {mode}: {ts.n_sets} sets, n 15..64")
    capart.capart_set_tuning(eng.ctx, memo=-1)
    ref = eng.solve(ts, 4, mode, debug=True)
    for memo in (0, 8):
        for form in (1, 3):  # nested loops; state machine with packed tests
            capart.capart_set_tuning(eng.ctx, loop_form=form, memo=memo)
            got = eng.solve(ts, 4, mode, debug=True)
            for f in FIELDS + ("dbg_key",):
                assert np.array_equal(got[f], ref[f]), (mode, memo, form, f)
    capart.capart_set_tuning(eng.ctx)
    idx = np.arange(0, ts.n_sets, 6)
    sub = workload.subset(ts, idx)
    want = oracle.solve(sub, 4, mode, nthreads=THREADS)
    got = eng.solve(sub, 4, mode)
    assert_same(got, want, sub, f"memo {mode}")


def wide_sets():
    """Sets of 33..64 tasks (the wide-set launch): serving queries on the
    smaller budgets, a few with constrained deadlines, a few light ones."""
    c5 = workload.config_c5(seed=47, n_queries=1500)
    n5 = c5.sizes()
    pick = np.nonzero((n5 > 32) & (c5["M"] <= 48))[0][:14]
    rng = np.random.default_rng(48)
    cons = workload.gen_sets(49, rng.integers(33, 65, 4), rng.uniform(2.0, 8.0, 4), np.array([16, 48, 16, 48]),
                             tmin=1e3, tmax=1e5, deadline="constrained")
    light = workload.gen_sets(50, rng.integers(33, 65, 4), rng.uniform(1.0, 3.0, 4), np.full(4, 16),
                              tmin=1e3, tmax=1e5)
    return workload.concat([workload.subset(c5, pick), cons, light])


@pytest.mark.parametrize("mode", ["BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT"])
def test_wide_wave_path_matches_lane_path(eng, mode):
    """Sets above 32 tasks: the wave-per-partitioning launch (default chunk,
    and chunks of 1 and 7 partitionings, which leave waves idle and do not
    divide P) gives the same key on every partitioning and the same results
    as one lane per partitioning, for K = 4 and K = 8; the final kernel's
    wave replay of the chosen partitioning gives the allocation; the oracle
    agrees on the sets of 16 units."""
    ts = wide_sets()
    for K in (4, 8):
        sub = ts if K == 4 else workload.subset(ts, np.nonzero(ts["M"] <= 16)[0])
        say(f"wide {mode} K={K}: {sub.n_sets} sets, n 33..64")
        capart.capart_set_tuning(eng.ctx, wide_chunk=-1)
        ref = eng.solve(sub, K, mode, debug=True)
        for wc in (0, 1, 7):
            capart.capart_set_tuning(eng.ctx, wide_chunk=wc)
            got = eng.solve(sub, K, mode, debug=True)
            for f in FIELDS + ("dbg_key",):
                assert np.array_equal(got[f], ref[f]), (mode, K, wc, f)
        capart.capart_set_tuning(eng.ctx)
    small = workload.subset(ts, np.nonzero(ts["M"] <= 16)[0][:6])
    want = oracle.solve(small, 4, mode, nthreads=THREADS)
    assert_same(eng.solve(small, 4, mode), want, small, f"wide {mode}")
