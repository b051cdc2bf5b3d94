"""Seeded input generators: determinism (byte hashes) and the recipe's
properties (UUniFast sums, deadlines, discard rule, types and factors)."""
import hashlib

import numpy as np

from paper_2105_10312_amd import workload as w

KEYS = ("set_offset", "M", "T", "D", "C_seq", "C_par", "k_permille", "type")


def digest(ts):
    return hashlib.sha256(b"".join(np.ascontiguousarray(ts[k]).tobytes() for k in KEYS)).hexdigest()[:16]


def test_deterministic_per_seed():
    assert digest(w.config_c1()) == digest(w.config_c1())
    assert digest(w.config_c2(n_sets=300)) == digest(w.config_c2(n_sets=300))
    assert digest(w.config_c2(seed=2, n_sets=300)) != digest(w.config_c2(seed=3, n_sets=300))


def test_uunifast_sums_and_bounds():
    rng = np.random.Generator(np.random.PCG64(1))
    U = rng.uniform(0.5, 16, 500)
    for n in (1, 2, 5, 10, 32):
        u = w.uunifast(rng, n, U)
        assert u.shape == (500, n) and (u >= 0).all()
        assert np.allclose(u.sum(1), U)


def _check(ts, n=None, M=None, implicit=True):
    off = ts["set_offset"]
    assert off[0] == 0 and (np.diff(off) >= 1).all() and off[-1] == ts.n_tasks
    T, D, Cs, Cp = ts["T"], ts["D"], ts["C_seq"], ts["C_par"]
    assert (T >= 1).all() and (T < 2**31).all() and (D >= 1).all() and (D <= T).all()
    assert (Cs >= 0).all() and (Cp >= 0).all() and (Cs + Cp >= 1).all()
    if implicit:
        assert (D == T).all()
    ty = ts["type"]
    assert set(np.unique(ty)) <= {0, 1}
    assert ((ts["k_permille"] == 2300) == (ty == 1)).all() and ((ts["k_permille"] == 1200) == (ty == 0)).all()
    Ms = np.repeat(ts["M"], np.diff(off)).astype(np.int64)
    assert (Cs + (Cp + Ms - 1) // Ms <= D).all()  # discard rule: every task fits the whole GPU
    if n is not None:
        assert (np.diff(off) == n).all()
    if M is not None:
        assert (ts["M"] == M).all()


def test_config_recipes():
    c1 = w.config_c1()
    _check(c1, n=5, M=8)
    # U stepped 0.5 .. 4.0 round-robin: one-unit utilisation sums track it
    u = np.add.reduceat((c1["C_seq"] + c1["C_par"]) / c1["T"], c1["set_offset"][:-1])
    target = 0.5 * (1 + np.arange(100) % 8)
    assert np.allclose(u, target, rtol=0.02, atol=0.02)
    _check(w.config_c2(n_sets=2000), n=10, M=80)
    c3 = w.config_c3(n_sets=2000)
    _check(c3, implicit=False)
    sz = np.diff(c3["set_offset"])
    assert sz.min() >= 4 and sz.max() <= 32 and set(np.unique(c3["M"])) == {16, 48, 80, 108}
    assert (c3["D"] < c3["T"]).mean() > 0.5
    _check(w.config_c4(n_sets=200), n=12, M=48)
    c5 = w.config_c5(n_queries=500)
    _check(c5)
    sz = np.diff(c5["set_offset"])
    assert sz.min() >= 2 and sz.max() <= 64
    # memory-intensive with probability one half
    ty = w.config_c2(n_sets=5000)["type"]
    assert abs(ty.mean() - 0.5) < 0.02


def test_subset_and_concat_roundtrip():
    ts = w.config_c2(n_sets=50)
    a, b = w.subset(ts, np.arange(20)), w.subset(ts, np.arange(20, 50))
    c = w.concat([a, b])
    for k in KEYS:
        assert np.array_equal(c[k], ts[k])


def test_paper_fig4_recipe():
    """The paper's own experiment: n = 50, M = 68, U = 2..68 step 2 with the
    sets ordered by point, D = 0.75 T, periods 50..4000, the type-dependent
    sequential share b = 0.02 a (compute) or 0.1 a (memory) of C1 = a + b."""
    ts = w.config_paper_fig4(sets_per_point=20)
    _check(ts, n=50, M=68, implicit=False)
    assert ts.n_sets == 34 * 20
    assert (ts["D"] == np.floor(0.75 * ts["T"]).astype(np.int64)).all()
    assert ts["T"].min() >= 50 and ts["T"].max() <= 4000
    C1 = ts["C_seq"] + ts["C_par"]
    share = np.where(ts["type"] == 1, 0.1 / 1.1, 0.02 / 1.02)
    assert (np.abs(ts["C_seq"] - np.rint(share * C1)) <= 0.5).all()
    u = np.add.reduceat(C1 / ts["T"], ts["set_offset"][:-1]).reshape(34, 20).mean(axis=1)
    assert np.allclose(u, np.arange(2, 69, 2), rtol=0.03)
    a = w.config_paper_fig4(sets_per_point=20)
    for key in ("T", "D", "C_seq", "C_par", "k_permille", "type"):
        assert np.array_equal(a[key], ts[key])
