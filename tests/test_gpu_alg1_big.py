"""Parity of the GPU Algorithm 1 on sets of more than 64 tasks (one block of
256 threads per set, fixed priority) with the CPU oracle's Algorithm 1: the
paper's 200-task sets (Figs. 6-8: n = 200, M = 68), mixed batches in which
small sets run through the same path, the limits of the path, explicit time
tables, and the batch the bench times, sampled.

Integer method: every output is compared bit for bit (status, verdict,
number of partitions, their sizes in par_list order, task -> partition,
response times, merges tried and accepted, scheduled workload)."""
import numpy as np
import pytest

from paper_2105_10312_amd import capart, workload
from test_gpu_alg1 import MODES, as_batch, assert_same, oracle_batch, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    e = capart.Engine(0)
    yield e
    e.close()


def paper_200(seed, points, per_point):
    return workload.config_paper_fig4(seed=seed, n=200, sets_per_point=per_point, U_points=points)


def check(eng, ts, mode, label, no_lemma1=False):
    flags = capart.CAPART_FLAG_NO_LEMMA1 if no_lemma1 else 0
    say(f"[alg1-big] {label} {mode}: {ts.n_sets} sets, {ts.n_tasks} tasks")
    got = eng.alg1(ts, mode, flags)
    assert_same(got, oracle_batch(ts, mode, no_lemma1), ts, f"{label} {mode}")
    return got


@pytest.mark.parametrize("mode", MODES)
def test_paper_200_task_sets(eng, mode):
    """Utilisations across the schedulability edge of the 200-task experiment
    (the analysis-time range of Fig. 8 is U = 35..45), and past Lemma 1."""
    ts = paper_200(81, [10, 20, 30, 34, 36, 38, 40, 42, 44, 50, 70], 4)
    got = check(eng, ts, mode, "fig6")
    rate = got["verdict"].reshape(-1, 4).mean(axis=1)
    say(f"[alg1-big] {mode} schedulability by U: {np.round(rate, 2).tolist()}")
    assert rate[:3].min() == 1.0 and rate[-1] == 0.0
    check(eng, workload.subset(ts, np.arange(16, 44)), mode, "fig6 no-lemma1", no_lemma1=True)


@pytest.mark.parametrize("mode", MODES)
def test_mixed_sizes_share_the_path(eng, mode):
    """A batch with one set above 64 tasks runs every set through the block
    path: sets of 1..64 tasks give the oracle's results there too, and the
    same as through the one-wave path."""
    rng = np.random.default_rng(7)
    sizes = [1, 2, 9, 31, 32, 33, 63, 64, 65, 100, 128, 129, 191, 200, 255, 256]
    Ms = [68 if n * 68 <= capart.CAPART_ALG1_BIG_MAX_NM else capart.CAPART_ALG1_BIG_MAX_NM // n for n in sizes]
    U = [float(rng.uniform(0.2, 0.7)) * min(0.8 * n, m) for n, m in zip(sizes, Ms)]
    ts = workload.gen_sets(17, sizes, U, Ms, tmin=50, tmax=4000, deadline=0.75, fsplit="paper")
    got = check(eng, ts, mode, "mixed")
    small = workload.subset(ts, np.arange(8))
    assert_same({k: v[:(8 if k in ("status", "verdict", "nparts", "tried", "merged", "workload")
                     else small.n_tasks)] for k, v in got.items()},
                eng.alg1(small, mode), small, f"wave path {mode}")


def test_limits(eng):
    """n = 256 at the n * M limit (M = 56), M = 127 with 65 tasks, one set
    beyond the n * M limit (status E_INVAL, failure outputs, the others
    unaffected), and the call-level refusals: EDF, and max_M above 127."""
    base = workload.gen_sets(23, [256, 256, 65, 200, 120], [8.0, 30.0, 40.0, 20.0, 30.0], [56, 56, 127, 68, 120],
                             tmin=50, tmax=4000, deadline=0.75, fsplit="paper")
    inside = workload.subset(base, np.arange(4))
    a = int(base["set_offset"][4])
    for mode in MODES:
        want = check(eng, inside, mode, "limits")
        got = eng.alg1(base, mode)
        assert list(got["status"]) == [0, 0, 0, 0, capart.CAPART_E_INVAL]
        assert (got["alloc"][a:] == -1).all() and (got["R"][a:] == -1).all() and got["verdict"][4] == 0
        assert got["nparts"][4] == 0 and (got["sizes"][a:] == 0).all()
        for f in ("verdict", "nparts", "tried", "merged", "workload"):
            assert np.array_equal(got[f][:4], want[f]), f
        for f in ("sizes", "alloc", "R"):
            assert np.array_equal(got[f][:a], want[f]), f
    ts = paper_200(5, [30], 2)
    with pytest.raises(capart.CapartError):
        eng.alg1(ts, "BF_INA", policy="EDF")
    with pytest.raises(capart.CapartError):
        capart.capart_alg1(eng.ctx, ts, "BF_INA", max_M=128)
    with pytest.raises(capart.CapartError):
        capart.capart_alg1(eng.ctx, ts, "BF_INA", max_tasks=257)


def test_conflict_extremes(eng):
    """Inflation factors up to 1000x (times saturate at 2^31 in the tables and
    are recomputed in 64 bits for the utilisations) and one type only."""
    rng = np.random.default_rng(9)
    tasks = []
    for _ in range(12):
        n = int(rng.integers(65, 160))
        T = rng.integers(50, 4000, n)
        Cs = rng.integers(0, 5, n)
        Cp = rng.integers(1, 60, n)
        ty = rng.integers(0, 2, n)
        k = rng.choice([1000, 1000000, 250000, 2300], n)
        M = min(int(rng.integers(20, 90)), capart.CAPART_ALG1_BIG_MAX_NM // n)
        tasks.append(dict(M=M, T=T, D=T, C_seq=Cs, C_par=Cp, k_permille=k, type=ty))
    for ty in (0, 1):
        n = 100
        tasks.append(dict(M=60, T=[1000] * n, D=[900] * n, C_seq=[5] * n, C_par=[120] * n,
                          k_permille=[1200 + 1100 * ty] * n, type=[ty] * n))
    ts = as_batch(tasks)
    for mode in MODES:
        check(eng, ts, mode, "extremes")


def test_time_tables(eng):
    """Explicit per-task time tables on 200-task sets."""
    ts = workload.with_time_tables(paper_200(33, [20, 34, 38, 42], 2), seed=34)
    for mode in ("BF_INA", "SMS_ACT"):
        want = oracle_batch(ts, mode)
        assert_same(eng.alg1(ts, mode), want, ts, f"tables {mode}")


def test_async_and_counted_work(eng):
    import torch
    ts = paper_200(41, [36, 40], 8)
    dev = capart.device_tasksets(ts)
    for mode in ("BF_ACT", "SMS_INA"):
        out = capart.device_alg1_results(ts.n_sets, ts.n_tasks)
        s = torch.cuda.Stream()
        capart.capart_alg1_async(eng.ctx, dev, mode, out, stream=s, max_tasks=200, max_M=68)
        s.synchronize()
        want = eng.alg1(ts, mode)
        got = {k: v.cpu().numpy()[:(ts.n_sets if k in ("status", "verdict", "nparts", "tried", "merged",
                                                        "workload") else ts.n_tasks)] for k, v in out.items()}
        assert_same(got, want, ts, f"async {mode}")
        out2 = capart.device_alg1_results(ts.n_sets, ts.n_tasks)
        work = capart.capart_alg1_count_work(eng.ctx, dev, mode, out2, 200, 68)
        got2 = {k: v.cpu().numpy()[:(ts.n_sets if k in ("status", "verdict", "nparts", "tried", "merged",
                                                         "workload") else ts.n_tasks)] for k, v in out2.items()}
        assert_same(got2, want, ts, f"count_work {mode}")
        assert work["tests"] >= int(want["tried"].sum()) > 0 and work["terms"] >= work["tests"]
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", MODES)
def test_bench_batch_sampled(eng, mode):
    """The batch the bench times for the 200-task experiment (34 utilisation
    points x 100 sets, one launch), every 17th set checked against the
    oracle."""
    import torch
    ts = workload.config_paper_fig4(n=200)
    dev = capart.device_tasksets(ts)
    out = capart.device_alg1_results(ts.n_sets, ts.n_tasks)
    capart.capart_alg1_async(eng.ctx, dev, mode, out, max_tasks=200, max_M=68)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    pick = np.arange(0, ts.n_sets, 17)
    sub = workload.subset(ts, pick)
    want = oracle_batch(sub, mode)
    off = ts["set_offset"]
    sel_t = np.concatenate([np.arange(off[s], off[s + 1]) for s in pick])
    per_set = ("status", "verdict", "nparts", "tried", "merged", "workload")
    mine = {k: (got[k][pick] if k in per_set else got[k][sel_t]) for k in got}
    assert_same(mine, want, sub, f"bench batch {mode}")
    say(f"[alg1-big] bench batch {mode}: {int(got['verdict'][:ts.n_sets].sum())} of {ts.n_sets} schedulable")
