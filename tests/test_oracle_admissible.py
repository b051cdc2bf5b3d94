"""The oracle with admissible partition sizes (MIG-like restrictions),
pinned against brute force over the allowed partitionings, against the
unrestricted search (an empty restriction changes nothing, a restriction
never helps), and on a restriction that leaves exactly one partitioning."""
import numpy as np
import pytest

import oracle
from brute import best_exhaustive
from paper_2105_10312_amd import workload

FIELDS = ("status", "verdict", "verdict_1g", "pidx", "sizes", "aidx", "maxU", "sumU", "n_evals", "alloc", "R",
          "R_1g")


def tiny(seed, count):
    rng = np.random.default_rng(seed)
    n = rng.integers(1, 5, count)
    M = rng.integers(2, 8, count)
    U = rng.uniform(0.4, 1.0, count) * np.minimum(M, n) * 0.9
    return workload.gen_sets(seed, n, U, M, tmin=10, tmax=60)


def test_every_size_admissible_changes_nothing():
    ts = workload.config_c1(n_sets=50)
    for mode in ("EXH", "BF_INA", "SMS_ACT"):
        a = oracle.solve(ts, 3, mode)
        b = oracle.solve(ts, 3, mode, admissible=range(1, 256))
        for f in FIELDS:
            assert np.array_equal(a[f], b[f]), (mode, f)


@pytest.mark.parametrize("adm", [(1, 2, 4), (2, 3), (1, 3, 5, 7), (4,)])
def test_restricted_exhaustive_matches_brute_force(adm):
    ts = tiny(61, 50)
    got = oracle.solve(ts, 3, "EXH", admissible=adm)
    for s in range(ts.n_sets):
        found, mx, sm, pidx, aidx, sizes, alloc = best_exhaustive(ts.set(s), 3, admissible=set(adm))
        assert bool(got["verdict"][s]) == found, (adm, s)
        if found:
            assert (int(got["maxU"][s]), int(got["sumU"][s]), int(got["pidx"][s]), int(got["aidx"][s])) == \
                (mx, sm, pidx, aidx)


def test_restriction_never_helps():
    ts = workload.subset(workload.config_c2(n_sets=300), np.arange(100))
    for mode in ("BF_INA", "SMS_INA"):
        free = oracle.solve(ts, 4, mode)
        mig = oracle.solve(ts, 4, mode, admissible=(10, 20, 30, 40, 70, 80))
        assert np.array_equal(free["n_evals"], mig["n_evals"])
        assert np.array_equal(free["verdict_1g"], mig["verdict_1g"])
        assert not (mig["verdict"].astype(bool) & ~free["verdict"].astype(bool)).any()
        both = (mig["verdict"] == 1) & (free["verdict"] == 1)
        key_free = list(zip(free["maxU"][both], free["sumU"][both]))
        key_mig = list(zip(mig["maxU"][both], mig["sumU"][both]))
        assert all(f <= g for f, g in zip(key_free, key_mig))
        # every chosen partitioning uses admissible sizes only
        sz = mig["sizes"][mig["verdict"] == 1]
        assert np.isin(sz[sz > 0], (10, 20, 30, 40, 70, 80)).all()


def test_one_admissible_partitioning():
    # M = 8, K = 3: only (5, 3) uses sizes {3, 5}; it is number 4 in the canonical order
    ts = workload.config_c1(n_sets=40)
    got = oracle.solve(ts, 3, "EXH", admissible=(3, 5))
    ok = got["verdict"] == 1
    assert ok.any() and (got["pidx"][ok] == 4).all() and (got["pidx"][~ok] == -1).all()
    assert (got["sizes"][ok] == [5, 3, 0]).all()
