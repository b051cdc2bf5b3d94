"""Independent brute-force checkers used to pin the oracle on tiny inputs.

Nothing here shares code with the oracle or the engine:
  * ``simulate_fp`` runs a discrete-time preemptive fixed-priority schedule
    of one partition from a synchronous release (critical instant, valid for
    D <= T) and reports each task's first-job response time or -1 on a miss;
  * ``best_exhaustive`` enumerates set partitions of the tasks into blocks
    and every assignment of those blocks to the parts of every integer
    partition of M, and keeps the triples whose every partition passes the
    simulation; it reports the optimum (maxU, sumU) and, from that optimum,
    the lowest (partitioning index, allocation index) under the ordering
    conventions (descending-lexicographic partitionings, base-k allocation
    index with task 0 most significant).
"""
from __future__ import annotations

import itertools
from fractions import Fraction


def ceil_div(a: int, b: int) -> int:
    return -((-a) // b)


def exec_time(c_seq: int, c_par: int, k: int, m: int, conflict: bool) -> int:
    """Execution time on m compute units: (C_seq + C_par/m), inflated by k/1000
    on conflict; rounded up to whole microseconds at each step."""
    base = Fraction(c_seq) + Fraction(c_par, m)
    base = int(-(-base.numerator // base.denominator))
    if conflict:
        v = Fraction(k * base, 1000)
        return int(-(-v.numerator // v.denominator))
    return base


def task_time(task, i: int, m: int, conflict: bool) -> int:
    """Task i's time on m units: its explicit table entry if the task set has
    tables ("Cn_table"/"Cc_table", [i*M + m-1]), else the parametric model."""
    if task.get("Cn_table") is not None:
        tab = task["Cc_table"] if conflict else task["Cn_table"]
        return int(tab[i * int(task["M"]) + m - 1])
    return exec_time(int(task["C_seq"][i]), int(task["C_par"][i]), int(task["k_permille"][i]), m, conflict)


def simulate_fp(C, T, D, prio):
    """Discrete-time preemptive FP simulation; prio[i] smaller = higher.

    Returns first-job response times (or -1 where the first job misses)."""
    n = len(C)
    horizon = max(D) if n else 0
    remaining = {}  # (task, job) -> remaining work
    resp = [-1] * n
    order = sorted(range(n), key=lambda i: prio[i])
    for t in range(horizon + 1):
        for i in range(n):
            if t % T[i] == 0:
                remaining[(i, t // T[i])] = C[i]
        # pick the highest-priority pending job (earliest job of that task)
        run = None
        for i in order:
            jobs = sorted(j for (ti, j) in remaining if ti == i and remaining[(ti, j)] > 0)
            if jobs:
                run = (i, jobs[0])
                break
        if run is None:
            continue
        remaining[run] -= 1
        if remaining[run] == 0:
            i, j = run
            if j == 0:
                resp[i] = t + 1
    return [r if (r != -1 and r <= D[i]) else -1 for i, r in enumerate(resp)]


def partition_feasible(task, members, m):
    """(feasible, U) of one partition of size m holding task indices `members`."""
    if not members:
        return True, 0
    types = [int(task["type"][i]) for i in members]
    C = []
    for i in members:
        same = sum(1 for j in members if int(task["type"][j]) == int(task["type"][i]))
        C.append(task_time(task, i, m, same >= 2))
    T = [int(task["T"][i]) for i in members]
    D = [int(task["D"][i]) for i in members]
    keyed = sorted(range(len(members)), key=lambda a: (D[a], T[a], members[a]))
    prio = [0] * len(members)
    for r, a in enumerate(keyed):
        prio[a] = r
    resp = simulate_fp(C, T, D, prio)
    if any(r < 0 for r in resp):
        return False, None
    U = sum(ceil_div(C[a] << 32, T[a]) for a in range(len(members)))
    del types
    return True, U


def integer_partitions_desc(M: int, K: int):
    """All partitions of M into <= K positive parts, sorted descending-lex."""
    out = []

    def rec(rem, mx, cur):
        if rem == 0:
            out.append(tuple(cur))
            return
        if len(cur) == K:
            return
        for x in range(1, min(rem, mx) + 1):
            rec(rem - x, x, cur + [x])

    rec(M, M, [])
    out.sort(reverse=True)
    return out


def set_partitions(items):
    """All set partitions of a list into non-empty blocks."""
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for p in set_partitions(rest):
        for i in range(len(p)):
            yield p[:i] + [[first] + p[i]] + p[i + 1:]
        yield [[first]] + p


def best_exhaustive(task, K: int, admissible=None):
    """Brute-force optimum: returns (found, maxU, sumU, pidx, aidx, sizes, alloc).
    admissible: allowed part sizes (None: every size); other partitionings keep
    their index but are skipped."""
    n = len(task["T"])
    M = int(task["M"])
    parts = integer_partitions_desc(M, K)
    best = None
    for pidx, sizes in enumerate(parts):
        if admissible is not None and any(x not in admissible for x in sizes):
            continue
        k = len(sizes)
        for blocks in set_partitions(list(range(n))):
            if len(blocks) > k:
                continue
            # place the blocks on distinct parts (remaining parts empty)
            for slots in itertools.permutations(range(k), len(blocks)):
                alloc = [0] * n
                for b, p in zip(blocks, slots):
                    for i in b:
                        alloc[i] = p
                ok = True
                Us = []
                for p in range(k):
                    mem = [i for i in range(n) if alloc[i] == p]
                    f, U = partition_feasible(task, mem, sizes[p])
                    if not f:
                        ok = False
                        break
                    Us.append(U)
                if not ok:
                    continue
                aidx = 0
                for i in range(n):
                    aidx = aidx * k + alloc[i]
                key = (max(Us), sum(Us), pidx, aidx)
                if best is None or key < best[0]:
                    best = (key, sizes, alloc)
    if best is None:
        return (False, None, None, -1, -1, None, None)
    (mx, sm, pidx, aidx), sizes, alloc = best
    return (True, mx, sm, pidx, aidx, sizes, alloc)


def whole_gpu(task):
    """1G baseline by simulation: (schedulable, R list with -1 for misses)."""
    n = len(task["T"])
    M = int(task["M"])
    mem = list(range(n))
    C = []
    for i in mem:
        same = sum(1 for j in mem if int(task["type"][j]) == int(task["type"][i]))
        C.append(task_time(task, i, M, same >= 2))
    T = [int(x) for x in task["T"]]
    D = [int(x) for x in task["D"]]
    keyed = sorted(range(n), key=lambda a: (D[a], T[a], a))
    prio = [0] * n
    for r, a in enumerate(keyed):
        prio[a] = r
    resp = simulate_fp(C, T, D, prio)
    return all(r >= 0 for r in resp), resp


def simulate_long(C, T, D, policy, horizon):
    """Unit-step preemptive schedule of one server from a synchronous release
    with periodic arrivals over [0, horizon), for long horizons (per-task job
    queues, O(n) per step).  policy "EDF": earliest absolute deadline first,
    ties to the lower task index; "DM": fixed priority by (D, T, index).
    Returns (first missed absolute deadline or None, first-job completion
    times (None if not completed), the first instant t > 0 by which all work
    released before t is done (the synchronous busy period) or None)."""
    from collections import deque
    n = len(C)
    queues = [deque() for _ in range(n)]  # [absolute deadline, remaining]
    dm = sorted(range(n), key=lambda i: (D[i], T[i], i))
    first_done = [None] * n
    jobs_done = [0] * n
    idle = None
    for t in range(horizon):
        if idle is None and t > 0 and not any(queues):
            idle = t  # all work released before t is done
        for i in range(n):
            if t % T[i] == 0:
                queues[i].append([t + D[i], C[i]])
        for i in range(n):
            if queues[i] and queues[i][0][0] <= t:
                return queues[i][0][0], first_done, idle
        if policy == "EDF":
            run = None
            for i in range(n):
                if queues[i] and (run is None or queues[i][0][0] < queues[run][0][0]):
                    run = i
        else:
            run = next((i for i in dm if queues[i]), None)
        if run is None:
            continue
        job = queues[run][0]
        job[1] -= 1
        if job[1] == 0:
            queues[run].popleft()
            if jobs_done[run] == 0:
                first_done[run] = t + 1
            jobs_done[run] += 1
    return None, first_done, idle
