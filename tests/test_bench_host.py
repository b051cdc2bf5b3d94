"""Host-side pieces of the benchmark: the exact Lemma 1 pruned-set count it
reports, checked against the oracle's per-set Lemma 1 test, and the refusal of
more than one GPU."""
import os
import subprocess
import sys

import numpy as np

import oracle
from paper_2105_10312_amd import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_lemma1_pruned_count_matches_oracle():
    rng = np.random.default_rng(1)
    U = rng.uniform(4, 12, 400)
    ts = workload.gen_sets(3, np.full(400, 6), U, np.full(400, 8), tmin=1e3, tmax=1e6)
    want = sum(oracle.lemma1_reject(ts.set(i)) for i in range(ts.n_sets))
    assert 0 < want < ts.n_sets
    assert bench.lemma1_pruned(ts) == want


def test_lemma1_pruned_count_with_time_tables():
    # the table profiles keep Cn(1) = C_seq + C_par, so Lemma 1 decides alike
    rng = np.random.default_rng(2)
    U = rng.uniform(4, 12, 300)
    ts = workload.gen_sets(4, np.full(300, 6), U, np.full(300, 8), tmin=1e3, tmax=1e6)
    want = sum(oracle.lemma1_reject(ts.set(i)) for i in range(ts.n_sets))
    tt = workload.with_time_tables(ts)
    for key in ("C_seq", "C_par", "k_permille"):
        del tt[key]
    assert 0 < want < ts.n_sets
    assert bench.lemma1_pruned(tt) == want


def test_lemma1_pruned_count_large_ratios():
    # C/T ratios far above M: the per-term clamp must keep the sum exact
    ts = workload.TaskSets(set_offset=np.array([0, 2, 3, 5]), M=np.array([4, 255, 1], np.int32))
    ts["T"] = np.array([1, 7, 2**31 - 1, 3, 5], np.int64)
    ts["D"] = ts["T"].copy()
    ts["C_seq"] = np.array([2**30, 1, 2**30, 1, 1], np.int64)
    ts["C_par"] = np.array([2**30 - 1, 1, 2**30, 1, 4], np.int64)
    ts["k_permille"] = np.full(5, 1000, np.int32)
    ts["type"] = np.zeros(5, np.uint8)
    want = sum(oracle.lemma1_reject(ts.set(i)) for i in range(ts.n_sets))
    assert bench.lemma1_pruned(ts) == want == 2


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
