"""Parity of the GPU Algorithm 1 (free partition sizes, through the C ABI)
with the CPU oracle's Algorithm 1.

Integer method: every output is compared bit for bit (status, verdict,
number of partitions, their sizes in par_list order, task -> partition,
response times, merges tried and accepted, scheduled workload)."""
import json
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2105_10312_amd import capart, workload

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
MODES = ("BF_INA", "BF_ACT", "SMS_INA", "SMS_ACT")
FIELDS = ("status", "verdict", "nparts", "sizes", "alloc", "R", "tried", "merged", "workload")
THREADS = min(16, os.cpu_count() or 1)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    e = capart.Engine(0)
    yield e
    e.close()


def as_batch(tasks):
    off = np.zeros(len(tasks) + 1, np.int64)
    off[1:] = np.cumsum([len(t["T"]) for t in tasks])
    b = workload.TaskSets(set_offset=off, M=np.array([t["M"] for t in tasks], np.int32))
    for key, dt in (("T", np.int64), ("D", np.int64), ("C_seq", np.int64), ("C_par", np.int64),
                    ("k_permille", np.int32), ("type", np.uint8)):
        b[key] = np.concatenate([np.asarray(t[key], dt) for t in tasks])
    return b


def oracle_batch(ts, mode, no_lemma1=False):
    """The oracle's Algorithm 1 on every set, laid out like the C-ABI results."""
    S, N = ts.n_sets, ts.n_tasks
    off = ts["set_offset"]
    flags = oracle.FLAG_NO_LEMMA1 if no_lemma1 else 0
    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(lambda s: oracle.alg1(ts.set(s), mode, flags), range(S)))
    out = dict(status=np.zeros(S, np.int32), verdict=np.zeros(S, np.uint8), nparts=np.zeros(S, np.int32),
               sizes=np.zeros(N, np.int32), alloc=np.full(N, -1, np.int8), R=np.full(N, -1, np.int64),
               tried=np.zeros(S, np.int64), merged=np.zeros(S, np.int64), workload=np.zeros(S, np.uint64))
    for s, r in enumerate(res):
        a = int(off[s])
        out["verdict"][s] = r["verdict"]
        out["tried"][s] = r["tried"]
        out["merged"][s] = r["merged"]
        out["workload"][s] = r["workload"]
        if r["verdict"]:
            out["nparts"][s] = r["k"]
            out["sizes"][a:a + r["k"]] = r["sizes"]
            out["alloc"][a:int(off[s + 1])] = r["alloc"]
            out["R"][a:int(off[s + 1])] = r["R"]
    return out


def assert_same(got, want, ts, label):
    off = ts["set_offset"]
    for f in FIELDS:
        g, w = np.asarray(got[f]), np.asarray(want[f])
        if g.shape != w.shape or not np.array_equal(g, w):
            detail = ""
            if g.shape == w.shape:
                i = int(np.argwhere(g != w)[0][0])
                where = f"task {i} (set {int(np.searchsorted(off, i, side='right') - 1)})" \
                    if f in ("sizes", "alloc", "R") else f"set {i}"
                detail = f" first mismatch at {where}: got {g[i]} want {w[i]}"
            raise AssertionError(f"{label}: field {f} differs;{detail}")


def run_both(eng, ts, mode, label, no_lemma1=False):
    flags = capart.CAPART_FLAG_NO_LEMMA1 if no_lemma1 else 0
    say(f"[alg1] {label} {mode}: {ts.n_sets} sets, {ts.n_tasks} tasks")
    got = eng.alg1(ts, mode, flags)
    want = oracle_batch(ts, mode, no_lemma1)
    assert_same(got, want, ts, f"{label} {mode}")
    return got


def random_tiny(seed, count, nmax=6, Mmax=10):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(1, nmax + 1))
        T = rng.integers(8, 60, n)
        C1 = np.maximum(1, (T * rng.uniform(0.1, 1.5, n)).astype(np.int64))
        Cs = (C1 * rng.uniform(0.0, 0.4, n)).astype(np.int64)
        Cp = np.maximum(C1 - Cs, 0)
        Cp[(Cs + Cp) == 0] = 1
        D = np.maximum(1, (T * rng.uniform(0.6, 1.0, n)).astype(np.int64))
        ty = rng.integers(0, 2, n)
        k = np.where(ty == 1, 2300, 1200)
        out.append(dict(M=int(rng.integers(1, Mmax + 1)), T=T, D=D, C_seq=Cs, C_par=Cp, k_permille=k, type=ty))
    return out


def test_golden_merge_example(eng):
    with open(os.path.join(HERE, "golden", "w4_alg1_merge_example.json")) as f:
        g = json.load(f)
    tasks = [dict(g["tasks"], M=c["M"]) for c in g["cases"]]
    w1 = dict(T=[100, 150, 200], D=[100, 150, 200], C_seq=[10, 5, 20], C_par=[200, 300, 240],
              k_permille=[1200, 2300, 1200], type=[0, 1, 0])
    tasks += [dict(w1, M=7), dict(w1, M=8)]
    ts = as_batch(tasks)
    for mode in MODES:
        got = run_both(eng, ts, mode, "golden")
        # the hand-derived values themselves
        for s, c in enumerate(g["cases"]):
            assert got["verdict"][s] == c["verdict"]
            if c["verdict"]:
                a = int(ts["set_offset"][s])
                assert list(got["sizes"][a:a + got["nparts"][s]]) == c["sizes"]
                assert list(got["alloc"][a:a + 2]) == c["alloc"] and list(got["R"][a:a + 2]) == c["R"]
        a = int(ts["set_offset"][4])
        assert list(got["sizes"][a:a + 3]) == g["w1_cases"]["M8"]["sizes"]


def test_golden_orders_merge_different_partners(eng):
    """The hand-derived set on which orders > and >> merge different partners."""
    with open(os.path.join(HERE, "golden", "w6_alg1_orders.json")) as f:
        g = json.load(f)
    ts = as_batch([g["set"]])
    for mode in MODES:
        got = run_both(eng, ts, mode, "w6")
        want = g["BF_INA" if mode.startswith("BF") else "SMS_INA"]
        assert int(got["verdict"][0]) == want["verdict"]
        assert list(got["sizes"][:got["nparts"][0]]) == want["sizes"], mode
        assert list(got["alloc"]) == want["alloc"] and list(got["R"]) == want["R"], mode
        assert int(got["tried"][0]) == want["tried"] and int(got["merged"][0]) == want["merged"], mode


@pytest.mark.parametrize("mode", MODES)
def test_random_tiny_sets(eng, mode):
    ts = as_batch(random_tiny(11, 3000))
    run_both(eng, ts, mode, "tiny")
    run_both(eng, ts, mode, "tiny no-lemma1", no_lemma1=True)


@pytest.mark.parametrize("mode", MODES)
def test_paper_fig4_workload(eng, mode):
    ts = workload.config_paper_fig4(sets_per_point=20)
    got = run_both(eng, ts, mode, "fig4")
    rate = got["verdict"].reshape(-1, 20).mean(axis=1)
    say(f"[alg1] fig4 {mode} schedulability by U=2..68: {np.round(rate, 2).tolist()}")
    assert rate[:10].min() == 1.0  # light sets (U <= 20 on 68 units) are all placed


@pytest.mark.parametrize("mode", MODES)
def test_other_workloads(eng, mode):
    c2 = workload.subset(workload.config_c2(n_sets=2000), np.arange(600))
    run_both(eng, c2, mode, "c2")
    c3 = workload.subset(workload.config_c3(n_sets=3000), np.arange(800))
    run_both(eng, c3, mode, "c3")
    c5 = workload.config_c5(n_queries=600)
    run_both(eng, c5, mode, "c5")


def test_edge_cases(eng):
    rng = np.random.default_rng(5)
    tasks = []
    # one task: fits alone or not at all
    tasks.append(dict(M=4, T=[100], D=[100], C_seq=[10], C_par=[100], k_permille=[1200], type=[0]))
    tasks.append(dict(M=1, T=[100], D=[100], C_seq=[10], C_par=[100], k_permille=[1200], type=[0]))
    # 64 tasks on 128 units (n * M at the LDS table limit), light and heavy
    for U in (4.0, 40.0, 90.0):
        g = workload.gen_sets(int(U), [64], [U], [128], tmin=50, tmax=4000, deadline=0.75, fsplit="paper")
        tasks.append(g.set(0))
    # maximal conflict inflation: k = 1000x makes the ">" rank sum exceed the u32 table
    for _ in range(40):
        n = int(rng.integers(2, 9))
        T = rng.integers(50, 400, n)
        Cs = rng.integers(0, 5, n)
        Cp = rng.integers(1, 200, n)
        ty = rng.integers(0, 2, n)
        k = rng.choice([1000, 1000000, 250000], n)
        tasks.append(dict(M=int(rng.integers(2, 40)), T=T, D=T, C_seq=Cs, C_par=Cp, k_permille=k, type=ty))
    # same-type pairs only (every merge is in conflict), different types only
    for ty in (0, 1):
        tasks.append(dict(M=12, T=[100] * 6, D=[90] * 6, C_seq=[5] * 6, C_par=[150] * 6,
                          k_permille=[1200 + 1100 * ty] * 6, type=[ty] * 6))
    # a task that no size within M schedules (Lemma 2 fails)
    tasks.append(dict(M=3, T=[100, 100], D=[20, 100], C_seq=[19, 1], C_par=[100, 10], k_permille=[1200, 1200],
                      type=[0, 1]))
    ts = as_batch(tasks)
    for mode in MODES:
        run_both(eng, ts, mode, "edge")
        run_both(eng, ts, mode, "edge no-lemma1", no_lemma1=True)


def test_invalid_sets_report_status(eng):
    good = dict(M=8, T=[100, 200], D=[100, 200], C_seq=[10, 10], C_par=[100, 400], k_permille=[1200, 2300],
                type=[0, 1])
    bad_range = dict(good, D=[100, 300])          # D > T
    bad_k = dict(good, k_permille=[999, 1200])    # k below 1000
    ts = as_batch([good, bad_range, good, bad_k])
    got = eng.alg1(ts, "SMS_INA")
    want_status = capart.capart_validate(ts, 1, "SMS_INA")
    assert list(got["status"]) == list(want_status)
    assert list(got["status"][[1, 3]]) == [capart.CAPART_E_RANGE] * 2
    for s in (1, 3):
        a, b = int(ts["set_offset"][s]), int(ts["set_offset"][s + 1])
        assert got["verdict"][s] == 0 and got["nparts"][s] == 0
        assert (got["alloc"][a:b] == -1).all() and (got["R"][a:b] == -1).all()
    ok = oracle_batch(workload.subset(ts, [0]), "SMS_INA")
    assert got["verdict"][0] == ok["verdict"][0] and got["verdict"][2] == ok["verdict"][0]


def test_exhaustive_mode_rejected(eng):
    ts = as_batch([dict(M=8, T=[100], D=[100], C_seq=[10], C_par=[100], k_permille=[1200], type=[0])])
    with pytest.raises(capart.CapartError):
        eng.alg1(ts, "EXH")


def test_async_matches_host(eng):
    import torch
    ts = workload.config_paper_fig4(sets_per_point=10)
    dev = capart.device_tasksets(ts)
    out = capart.device_alg1_results(ts.n_sets, ts.n_tasks)
    s = torch.cuda.Stream()
    for mode in MODES:
        capart.capart_alg1_async(eng.ctx, dev, mode, out, stream=s, max_tasks=50, max_M=68)
        s.synchronize()
        got = {k: v.cpu().numpy()[:(ts.n_sets if k in ("status", "verdict", "nparts", "tried", "merged")
                                    else ts.n_tasks)] for k, v in out.items()}
        assert_same(got, eng.alg1(ts, mode), ts, f"async {mode}")
    torch.cuda.synchronize()


def test_count_work_writes_same_results(eng):
    ts = workload.config_paper_fig4(sets_per_point=5)
    dev = capart.device_tasksets(ts)
    for mode in ("BF_INA", "SMS_ACT"):
        out = capart.device_alg1_results(ts.n_sets, ts.n_tasks)
        work = capart.capart_alg1_count_work(eng.ctx, dev, mode, out, 50, 68)
        got = {k: v.cpu().numpy()[:(ts.n_sets if k in ("status", "verdict", "nparts", "tried", "merged")
                                    else ts.n_tasks)] for k, v in out.items()}
        assert_same(got, eng.alg1(ts, mode), ts, f"count_work {mode}")
        # every merge tried runs at least one exact test
        assert work["tests"] >= int(got["tried"].sum()) > 0
        assert work["terms"] >= work["tests"]
