"""Seeded synthetic task-set generators (input data only).

This module draws the integer task sets that both the CPU oracle and the HIP
engine consume.  It performs none of the method's arithmetic: no execution
time under interference, no schedulability test, no partitioning.  The one
formula it evaluates is the whole-GPU execution time of a lone task, used only
to shape inputs (to reject a draw whose task could not meet its deadline even
alone on the whole GPU, and to draw a constrained deadline above it).

Recipe (paper, Section "Task set generation"): total utilisation U is split over
the n tasks with UUniFast (Bini & Buttazzo); each task's period is drawn, its
one-compute-unit execution time is u*T, a share of that time does not scale
with compute units; each task is memory- or compute-intensive with probability
prm = 50 %, and its interference factor is 2.3 (memory) or 1.2 (compute) when
it shares a partition with another task of its type.  Sets whose tasks are
infeasible on the whole GPU are discarded and redrawn (UUniFast-Discard).

Concrete distributions used here (the paper's period list is not given):
  * T  = round(exp(Uniform(ln Tmin, ln Tmax))) microseconds;
  * C1 = max(1, round(u*T)) is the time on one compute unit, f ~ U[0.05, 0.5],
    C_seq = round(f*C1), C_par = C1 - C_seq (C(m) = C_seq + ceil(C_par/m));
  * memory intensity mi ~ U{0..999} per-mille; type = memory iff mi >= 500;
    k = 2300 per-mille (memory) or 1200 (compute);
  * D = T (implicit deadlines) or D ~ U{Cw..T} with Cw the whole-GPU time
    (constrained deadlines).

All arrays are structure-of-arrays numpy arrays:
  set_offset int64[S+1], M int32[S], T, D, C_seq, C_par int64[N],
  k_permille int32[N], type uint8[N]  (0 = compute, 1 = memory).
"""
from __future__ import annotations

import numpy as np

TYPE_COMPUTE = 0
TYPE_MEMORY = 1
K_COMPUTE = 1200
K_MEMORY = 2300

__all__ = [
    "TaskSets", "uunifast", "gen_sets", "config_c1", "config_c2", "config_c3",
    "config_c4", "config_c5_query_sizes", "config_paper_fig4", "with_time_tables", "concat", "subset",
    "TYPE_COMPUTE",
    "TYPE_MEMORY",
]


class TaskSets(dict):
    """dict of SoA arrays with a few helpers (n_sets, n_tasks, set(i))."""

    @property
    def n_sets(self) -> int:
        return int(self["M"].shape[0])

    @property
    def n_tasks(self) -> int:
        return int(self["T"].shape[0])

    def sizes(self) -> np.ndarray:
        return np.diff(self["set_offset"])

    def set(self, s: int) -> dict:
        a, b = int(self["set_offset"][s]), int(self["set_offset"][s + 1])
        one = {k: self[k][a:b] for k in ("T", "D", "C_seq", "C_par", "k_permille", "type") if k in self} | {
            "M": int(self["M"][s])}
        if "Cn_table" in self:
            t0, t1 = int(self["table_offset"][s]), int(self["table_offset"][s]) + (b - a) * int(self["M"][s])
            one["Cn_table"] = self["Cn_table"][t0:t1]
            one["Cc_table"] = self["Cc_table"][t0:t1]
        return one


def uunifast(rng: np.random.Generator, n: int, U: np.ndarray) -> np.ndarray:
    """UUniFast (Bini & Buttazzo 2005), vectorised over sets of equal size n.

    Returns u[len(U), n] with rows summing to U."""
    U = np.asarray(U, dtype=np.float64)
    out = np.empty((U.shape[0], n), dtype=np.float64)
    sum_u = U.copy()
    for i in range(1, n):
        r = rng.random(U.shape[0])
        nxt = sum_u * r ** (1.0 / (n - i))
        out[:, i - 1] = sum_u - nxt
        sum_u = nxt
    out[:, n - 1] = sum_u
    return out


def _whole_gpu_time(c_seq, c_par, M):
    # input-shaping bound only: a lone task's time on all M compute units
    return c_seq + (c_par + M - 1) // M


def _draw_group(rng, n, U, M, tmin, tmax, deadline, fsplit):
    """Draw len(U) sets of n tasks; returns dict of [S, n] arrays."""
    S = U.shape[0]
    u = uunifast(rng, n, U)
    T = np.rint(np.exp(rng.uniform(np.log(tmin), np.log(tmax), size=(S, n)))).astype(np.int64)
    T = np.clip(T, 1, (1 << 31) - 1)
    C1 = np.maximum(1, np.rint(u * T)).astype(np.int64)
    if fsplit == "uniform":
        f = rng.uniform(0.05, 0.5, size=(S, n))
    else:
        f = None
    mi = rng.integers(0, 1000, size=(S, n))
    typ = (mi >= 500).astype(np.uint8)
    if fsplit == "paper":
        # paper mode: b = 0.02 a (compute) or 0.1 a (memory) with C1 = a + b
        f = np.where(typ == TYPE_MEMORY, 0.1 / 1.1, 0.02 / 1.02)
    c_seq = np.rint(f * C1).astype(np.int64)
    c_par = C1 - c_seq
    k = np.where(typ == TYPE_MEMORY, K_MEMORY, K_COMPUTE).astype(np.int32)
    Mcol = np.asarray(M, dtype=np.int64)[:, None]
    cw = _whole_gpu_time(c_seq, c_par, Mcol)
    if deadline == "implicit":
        D = T.copy()
    elif deadline == "constrained":
        lo = np.minimum(cw, T)
        D = lo + np.floor(rng.random((S, n)) * (T - lo + 1)).astype(np.int64)
        D = np.minimum(D, T)
    elif isinstance(deadline, float):
        D = np.maximum(1, np.floor(deadline * T)).astype(np.int64)
    else:
        raise ValueError(deadline)
    ok = np.all((cw <= D) & (C1 < (1 << 31)), axis=1)
    return dict(T=T, D=D, C_seq=c_seq, C_par=c_par, k_permille=k, type=typ), ok


def gen_sets(seed: int, n: np.ndarray, U: np.ndarray, M: np.ndarray, *, tmin: float, tmax: float,
             deadline="implicit", fsplit="uniform", max_rounds: int = 10000) -> TaskSets:
    """Generate task sets; set s has n[s] tasks, utilisation U[s] and budget M[s].

    Sets failing the discard rule are redrawn (same generator stream) until
    all are accepted.  Deterministic in (seed, n, U, M, options)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = np.asarray(n, dtype=np.int64)
    U = np.asarray(U, dtype=np.float64)
    M = np.asarray(M, dtype=np.int32)
    S = n.shape[0]
    off = np.zeros(S + 1, dtype=np.int64)
    off[1:] = np.cumsum(n)
    N = int(off[-1])
    keys = (("T", np.int64), ("D", np.int64), ("C_seq", np.int64), ("C_par", np.int64), ("k_permille", np.int32),
            ("type", np.uint8))
    out = TaskSets(set_offset=off, M=M.copy())
    for key, dt in keys:
        out[key] = np.zeros(N, dtype=dt)
    for nv in np.unique(n):
        idx = np.nonzero(n == nv)[0]
        pending = idx
        for _ in range(max_rounds):
            if pending.size == 0:
                break
            g, ok = _draw_group(rng, int(nv), U[pending], M[pending], tmin, tmax, deadline, fsplit)
            acc = pending[ok]
            # task positions of the accepted sets, row-major [set, task]
            pos = (off[acc][:, None] + np.arange(int(nv))[None, :]).ravel()
            for key, dt in keys:
                out[key][pos] = g[key][ok].ravel().astype(dt)
            pending = pending[~ok]
        if pending.size:
            raise RuntimeError(f"discard loop did not converge for n={nv}")
    return out


def concat(parts: list) -> TaskSets:
    """Concatenate several TaskSets into one batch."""
    off = [np.zeros(1, np.int64)]
    base = 0
    for p in parts:
        off.append(p["set_offset"][1:] + base)
        base += p.n_tasks
    out = TaskSets(set_offset=np.concatenate(off), M=np.concatenate([p["M"] for p in parts]))
    for key in ("T", "D", "C_seq", "C_par", "k_permille", "type"):
        out[key] = np.concatenate([p[key] for p in parts])
    return out


def subset(ts: TaskSets, idx) -> TaskSets:
    """Select sets by index (order kept as given)."""
    idx = np.asarray(idx, dtype=np.int64)
    sz = ts.sizes()[idx]
    off = np.zeros(idx.shape[0] + 1, np.int64)
    off[1:] = np.cumsum(sz)
    take = np.concatenate([np.arange(ts["set_offset"][s], ts["set_offset"][s + 1]) for s in idx]) \
        if idx.size else np.zeros(0, np.int64)
    out = TaskSets(set_offset=off, M=ts["M"][idx].copy())
    for key in ("T", "D", "C_seq", "C_par", "k_permille", "type"):
        if key in ts:
            out[key] = ts[key][take].copy()
    if "Cn_table" in ts:
        lens = sz * ts["M"][idx].astype(np.int64)
        out["table_offset"] = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
        rows = [np.arange(ts["table_offset"][s], ts["table_offset"][s] + ln) for s, ln in zip(idx, lens)]
        tk = np.concatenate(rows) if rows else np.zeros(0, np.int64)
        out["Cn_table"] = ts["Cn_table"][tk].copy()
        out["Cc_table"] = ts["Cc_table"][tk].copy()
    return out


# --- the five workloads -------------------------------------------------------

def config_c1(seed: int = 1, n_sets: int = 100) -> TaskSets:
    """100 sets, n=5, M=8 (<=3 parts, exhaustive); U = 0.5..4.0 round-robin;
    T log-uniform 1e4..1e6 us; D = T."""
    s = np.arange(n_sets)
    U = 0.5 * (1 + (s % 8))
    return gen_sets(seed, np.full(n_sets, 5), U, np.full(n_sets, 8), tmin=1e4, tmax=1e6)


def config_c2(seed: int = 2, n_sets: int = 100_000) -> TaskSets:
    """100,000 sets, n=10, M=80 (<=4 parts, heuristic allocation);
    U ~ U(1,16); T log-uniform 1e3..1e6 us; D = T."""
    rng = np.random.Generator(np.random.PCG64(seed + 1_000_003))
    U = rng.uniform(1.0, 16.0, size=n_sets)
    return gen_sets(seed, np.full(n_sets, 10), U, np.full(n_sets, 80), tmin=1e3, tmax=1e6)


def config_c3(seed: int = 3, n_sets: int = 1_000_000) -> TaskSets:
    """1e6 uneven sets: n ~ U{4..32}, M from {16,48,80,108}; U ~ U(1,16);
    T as C2; constrained D ~ U{Cw..T}."""
    rng = np.random.Generator(np.random.PCG64(seed + 1_000_003))
    n = rng.integers(4, 33, size=n_sets)
    M = rng.choice(np.array([16, 48, 80, 108]), size=n_sets)
    U = rng.uniform(1.0, 16.0, size=n_sets)
    return gen_sets(seed, n, U, M, tmin=1e3, tmax=1e6, deadline="constrained")


def config_c4(seed: int = 4, n_sets: int = 1000) -> TaskSets:
    """1,000 sets, n=12, M=48 (<=4 parts, exhaustive); U, T as C2; D = T."""
    rng = np.random.Generator(np.random.PCG64(seed + 1_000_003))
    U = rng.uniform(1.0, 16.0, size=n_sets)
    return gen_sets(seed, np.full(n_sets, 12), U, np.full(n_sets, 48), tmin=1e3, tmax=1e6)


def config_c5_query_sizes(seed: int, n_queries: int):
    """Serving queries: n = round(exp(U(ln 2, ln 64))), M from {16,48,80,108},
    U ~ U(1, min(16, n * u_safe(M))) where u_safe(M) = 1 / (0.5 + 0.5 / M) is
    the one-task utilisation that still fits the whole GPU at the largest
    sequential fraction (0.5): above it a query of few tasks could almost
    never pass the discard rule."""
    rng = np.random.Generator(np.random.PCG64(seed + 1_000_003))
    n = np.rint(np.exp(rng.uniform(np.log(2), np.log(64), size=n_queries))).astype(np.int64)
    M = rng.choice(np.array([16, 48, 80, 108]), size=n_queries)
    u_safe = 1.0 / (0.5 + 0.5 / M)
    U = rng.uniform(1.0, np.minimum(16.0, n * u_safe), size=n_queries)
    return n, U, M


def config_c5(seed: int = 5, n_queries: int = 1000) -> TaskSets:
    n, U, M = config_c5_query_sizes(seed, n_queries)
    return gen_sets(seed, n, U, M, tmin=1e3, tmax=1e6)


def config_paper_fig4(seed: int = 6, n: int = 50, M: int = 68, sets_per_point: int = 100,
                      U_points=None) -> TaskSets:
    """The paper's own experiment (Section "Task set generation", Fig. 4):
    n = 50 tasks, M = 68 compute units, utilisation U = 2, 4, .., 68 with
    100 sets per point (sets ordered by point), periods 50..4000 us
    (log-uniform here: the paper's period list is not given), D = 0.75 T,
    C_seq = 0.02/1.02 (compute) or 0.1/1.1 (memory) of the one-unit time,
    k = 1.2 / 2.3, prm = 50 %."""
    if U_points is None:
        U_points = np.arange(2, M + 1, 2, dtype=np.float64)
    U = np.repeat(np.asarray(U_points, np.float64), sets_per_point)
    S = U.shape[0]
    return gen_sets(seed, np.full(S, n), U, np.full(S, M), tmin=50, tmax=4000, deadline=0.75, fsplit="paper")


def with_time_tables(ts: TaskSets, seed: int = 7) -> TaskSets:
    """The same sets with explicit per-task time tables Cn[m], Cc[m] for
    m = 1..M (input profiles, as measured kernels would give; laid out per set
    as [task][m] from table_offset[s]).  Shapes: a compute-intensive task keeps
    speeding up with more units (C_seq + ceil(C_par/m)); a memory-intensive
    one stops beyond a saturation size m_sat ~ U{2..M} (Section "Task model",
    Definition 1); in conflict a task pays an extra delay that shrinks with m
    but more slowly (its own saturation size m_c ~ U{1..M}, share 0.1..1.5 of
    its time there).  Every table is non-increasing in m, the conflict table
    is never below the other, and m Cn(m) >= Cn(1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = ts.sizes()
    Ms = ts["M"].astype(np.int64)
    lens = sizes * Ms
    out = TaskSets({k: v.copy() for k, v in ts.items()})
    out["table_offset"] = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    total = int(lens.sum())
    Cn = np.zeros(total, np.int64)
    Cc = np.zeros(total, np.int64)
    for s in range(ts.n_sets):
        a, b, M = int(ts["set_offset"][s]), int(ts["set_offset"][s + 1]), int(Ms[s])
        m = np.arange(1, M + 1, dtype=np.int64)[None, :]
        n = b - a
        cs = ts["C_seq"][a:b, None]
        cp = ts["C_par"][a:b, None]
        mem = ts["type"][a:b, None] == TYPE_MEMORY
        msat = np.where(mem, rng.integers(2, M + 1, (n, 1)) if M >= 2 else 1, M)
        cn = cs + (cp + np.minimum(m, msat) - 1) // np.minimum(m, msat)
        mc = rng.integers(1, M + 1, (n, 1))
        share = rng.uniform(0.1, 1.5, (n, 1))
        extra = np.ceil(share * (cs + (cp + np.minimum(m, mc) - 1) // np.minimum(m, mc))).astype(np.int64)
        cc = cn + extra
        t0 = int(out["table_offset"][s])
        Cn[t0:t0 + n * M] = cn.ravel()
        Cc[t0:t0 + n * M] = cc.ravel()
    out["Cn_table"] = Cn
    out["Cc_table"] = Cc
    return out
