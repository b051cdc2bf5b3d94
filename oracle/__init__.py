"""CPU oracle for contention-aware GPU partitioning (arXiv 2105.10312).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the engine.  The arithmetic lives in
``capart_oracle.c`` (plain C, 128-bit intermediates, no SIMD intrinsics);
this module compiles it with gcc and marshals numpy arrays through ctypes.

Modes: EXH (exhaustive allocation), BF_INA, BF_ACT, SMS_INA, SMS_ACT
(heuristic allocation over each fixed partitioning).  FLAG_EXH_FAST gives the
exhaustive mode through a memo of partition tests ("oracle_fast": the same
search, every allocation of every partitioning, scored from a table of
(task subset, size) tests; checked against the plain search).  Per-partition policy:
FP_DM (fixed priority, deadline monotonic, exact response times) or EDF
(processor-demand test).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "capart_oracle.c")
LIB = os.path.join(HERE, "liboracle_capart.so")

EXH, BF_INA, BF_ACT, SMS_INA, SMS_ACT = 0, 1, 2, 3, 4
MODES = {"EXH": EXH, "BF_INA": BF_INA, "BF_ACT": BF_ACT, "SMS_INA": SMS_INA, "SMS_ACT": SMS_ACT}
FLAG_NO_LEMMA1 = 1
FLAG_EDF = 2
FLAG_EXH_FAST = 4  # exhaustive mode scored through a memo of partition tests (sets of at most 16 tasks)
POLICIES = {"FP_DM": 0, "EDF": FLAG_EDF}
EDF_BP_STEPS, EDF_ND_CAP = 4096, 65536
OK, E_INVAL, E_RANGE = 0, -1, -2
M_INF = 1000000

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (gcc -O2, no SIMD intrinsics) into liboracle_capart.so."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-Wno-unused-parameter", "-o", tmp, SRC, "-lpthread"])
        os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C")
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C")
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C")
        set_args = [C.c_int, C.c_int, i64p, i64p, i64p, i64p, i32p, u8p]
        lib.or_solve_batch.restype = C.c_int
        lib.or_solve_batch.argtypes = [C.c_int64, i64p, i32p, i64p, i64p, i64p, i64p, i32p, u8p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_int, C.c_int, C.c_int, C.c_int,
                                       i32p, u8p, u8p, i32p, i32p, i64p, u64p, u64p, i64p,
                                       i8p, i64p, i64p, C.c_void_p]
        lib.or_count_partitionings.restype = C.c_int64
        lib.or_count_partitionings.argtypes = [C.c_int, C.c_int]
        lib.or_enumerate_partitionings.restype = C.c_int64
        lib.or_enumerate_partitionings.argtypes = [C.c_int, C.c_int, np.ctypeslib.ndpointer(np.intc, flags="C"),
                                                   C.c_int64]
        lib.or_eval_triple_ex.restype = C.c_int
        lib.or_eval_triple_ex.argtypes = set_args + [i32p, C.c_int, i8p, C.c_int, i64p,
                                                     C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.c_void_p]
        lib.or_heuristic_ex.restype = C.c_int
        lib.or_heuristic_ex.argtypes = set_args + [i32p, C.c_int, C.c_int, i8p]
        lib.or_best_on_partitioning.restype = C.c_int
        lib.or_best_on_partitioning.argtypes = set_args + [i32p, C.c_int, C.c_int, i8p,
                                                           C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                                           C.POINTER(C.c_int64)]
        lib.or_m_min_ex.restype = C.c_int
        lib.or_m_min_ex.argtypes = set_args + [C.c_int]
        lib.or_forbidden_ex.restype = C.c_int
        lib.or_forbidden_ex.argtypes = set_args + [C.c_int, C.c_int]
        lib.or_lemma1_reject_ex.restype = C.c_int
        lib.or_lemma1_reject_ex.argtypes = set_args
        lib.or_u1_ex.restype = C.c_uint64
        lib.or_u1_ex.argtypes = set_args + [C.c_int]
        lib.or_alg1_ex.restype = C.c_int
        lib.or_alg1_ex.argtypes = set_args + [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, i32p, i8p, i64p,
                                              C.c_void_p]
        lib.or_time.restype = C.c_int64
        lib.or_time.argtypes = [i64p, i64p, i32p, C.c_int, C.c_int, C.c_int]
        _lib = lib
    return _lib


def _set_arrays(ts: dict):
    """T, D, C_seq, C_par, k, type; with explicit time tables ("Cn_table" and
    "Cc_table") the parametric fields may be absent (zeros are passed)."""
    N = len(ts["T"])
    z64, z32 = np.zeros(N, np.int64), np.zeros(N, np.int32)
    return (np.ascontiguousarray(ts["T"], np.int64), np.ascontiguousarray(ts["D"], np.int64),
            np.ascontiguousarray(ts.get("C_seq", z64), np.int64), np.ascontiguousarray(ts.get("C_par", z64), np.int64),
            np.ascontiguousarray(ts.get("k_permille", z32), np.int32), np.ascontiguousarray(ts["type"], np.uint8))


def _tables(ts: dict):
    """(table_offset, Cn_table, Cc_table) arrays, or Nones for the parametric model."""
    if ts.get("Cn_table") is None:
        return None, None, None
    return (np.ascontiguousarray(ts["table_offset"], np.int64), np.ascontiguousarray(ts["Cn_table"], np.int64),
            np.ascontiguousarray(ts["Cc_table"], np.int64))


def _one(task: dict):
    arrs = _set_arrays(task)
    return (len(arrs[0]), int(task["M"])) + arrs


def admissible_mask(sizes) -> np.ndarray:
    """4-word mask with bit m set for every admissible partition size m."""
    mask = np.zeros(4, np.uint64)
    for m in sizes:
        mask[int(m) // 64] |= np.uint64(1) << np.uint64(int(m) % 64)
    return mask


def solve(ts: dict, K: int, mode="BF_INA", flags: int = 0, nthreads: int = 1, counters: bool = False,
          admissible=None, policy: str = "FP_DM") -> dict:
    """Solve every set of a SoA batch; returns a dict of numpy result arrays.
    admissible: allowed partition sizes (an iterable of sizes), None = every size.
    policy: per-partition scheduling, "FP_DM" (fixed priority, deadline
    monotonic, exact response times) or "EDF" (processor-demand test)."""
    lib = _load()
    flags = int(flags) | POLICIES[policy]
    mode = MODES[mode] if isinstance(mode, str) else int(mode)
    off = np.ascontiguousarray(ts["set_offset"], np.int64)
    M = np.ascontiguousarray(ts["M"], np.int32)
    S = M.shape[0]
    N = int(off[-1]) if S else 0
    T, D, Cs, Cp, k, ty = _set_arrays(ts)
    out = dict(status=np.zeros(S, np.int32), verdict=np.zeros(S, np.uint8), verdict_1g=np.zeros(S, np.uint8),
               pidx=np.zeros(S, np.int32), sizes=np.zeros(S * K, np.int32), aidx=np.zeros(S, np.int64),
               maxU=np.zeros(S, np.uint64), sumU=np.zeros(S, np.uint64), n_evals=np.zeros(S, np.int64),
               alloc=np.zeros(N, np.int8), R=np.zeros(N, np.int64), R_1g=np.zeros(N, np.int64))
    cnt = np.zeros(S * 3, np.int64) if counters else None
    to, cn, cc = _tables(ts)
    adm = admissible_mask(admissible) if admissible is not None else None
    rc = lib.or_solve_batch(S, off, M, T, D, Cs, Cp, k, ty,
                            to.ctypes.data if to is not None else None, cn.ctypes.data if cn is not None else None,
                            cc.ctypes.data if cc is not None else None, adm.ctypes.data if adm is not None else None,
                            K, mode, flags, nthreads,
                            out["status"], out["verdict"], out["verdict_1g"], out["pidx"], out["sizes"],
                            out["aidx"], out["maxU"], out["sumU"], out["n_evals"], out["alloc"], out["R"],
                            out["R_1g"], cnt.ctypes.data if cnt is not None else None)
    if rc != OK:
        raise ValueError(f"oracle rejected batch: {rc}")
    out["sizes"] = out["sizes"].reshape(S, K)
    if counters:
        out["counters"] = cnt.reshape(S, 3)
    return out


def count_partitionings(M: int, K: int) -> int:
    return int(_load().or_count_partitionings(M, K))


def enumerate_partitionings(M: int, K: int) -> np.ndarray:
    P = count_partitionings(M, K)
    buf = np.zeros(max(P, 1) * K, np.intc)
    _load().or_enumerate_partitionings(M, K, buf, P)
    return buf[:P * K].reshape(P, K).astype(np.int32)


def eval_triple(task: dict, sizes, alloc, early_exit: bool = False, counters: bool = False):
    """Evaluate one (set, partitioning, allocation); returns (feasible, R, maxU, sumU[, counters])."""
    lib = _load()
    sz = np.ascontiguousarray(sizes, np.int32)
    al = np.ascontiguousarray(alloc, np.int8)
    n = len(task["T"])
    R = np.zeros(n, np.int64)
    mx, sm = C.c_uint64(0), C.c_uint64(0)
    cnt = np.zeros(3, np.int64)
    f = lib.or_eval_triple_ex(*_one(task), sz, len(sz), al, int(early_exit), R, C.byref(mx), C.byref(sm),
                              cnt.ctypes.data)
    res = (bool(f), R, int(mx.value), int(sm.value))
    return res + (cnt,) if counters else res


def heuristic(task: dict, sizes, mode="BF_INA"):
    """H(pi) on one fixed partitioning; returns alloc (int8[n]) or None."""
    lib = _load()
    mode = MODES[mode] if isinstance(mode, str) else int(mode)
    sz = np.ascontiguousarray(sizes, np.int32)
    al = np.zeros(len(task["T"]), np.int8)
    ok = lib.or_heuristic_ex(*_one(task), sz, len(sz), mode, al)
    return al if ok else None


def best_on_partitioning(task: dict, sizes, mode="EXH"):
    """Best allocation on one partitioning: (found, alloc, maxU, sumU, aidx)."""
    lib = _load()
    mode = MODES[mode] if isinstance(mode, str) else int(mode)
    sz = np.ascontiguousarray(sizes, np.int32)
    al = np.zeros(len(task["T"]), np.int8)
    mx, sm, ai = C.c_uint64(0), C.c_uint64(0), C.c_int64(-1)
    f = lib.or_best_on_partitioning(*_one(task), sz, len(sz), mode, al, C.byref(mx), C.byref(sm), C.byref(ai))
    if f < 0:
        raise ValueError("set outside the oracle's limits")
    return bool(f), al, int(mx.value), int(sm.value), int(ai.value)


def alg1(task: dict, mode="BF_INA", flags: int = 0, policy: str = "FP_DM") -> dict:
    """The paper's Algorithm 1 with free partition sizes on one set.

    mode: BF_* = order ">" (Definition 5), SMS_* = order ">>" (Definition 4);
    *_ACT fills the forbidden list beforehand.  Returns verdict, the final
    partitions in par_list order (sizes), task -> partition (alloc), response
    times R, the numbers of merges tried and accepted, and (on success) the
    scheduled workload: the Q32 sum of every task's one-unit utilisation in the
    conflict state its partition gives it (Figs. 5 and 7; 0 on failure)."""
    lib = _load()
    flags = int(flags) | POLICIES[policy]
    mode = MODES[mode] if isinstance(mode, str) else int(mode)
    if mode == MODES["EXH"]:
        raise ValueError("Algorithm 1 takes a heuristic order (BF_* or SMS_*)")
    n = len(task["T"])
    k = C.c_int32(0)
    sizes = np.zeros(n, np.int32)
    al = np.zeros(n, np.int8)
    R = np.zeros(n, np.int64)
    st = np.zeros(3, np.int64)
    cn = np.ascontiguousarray(task["Cn_table"], np.int64) if task.get("Cn_table") is not None else None
    cc = np.ascontiguousarray(task["Cc_table"], np.int64) if cn is not None else None
    ok = lib.or_alg1_ex(*_one(task), cn.ctypes.data if cn is not None else None,
                        cc.ctypes.data if cc is not None else None, mode, int(flags), C.byref(k), sizes, al, R,
                        st.ctypes.data)
    if ok < 0:
        raise ValueError("set outside the oracle's limits")
    return dict(verdict=int(ok), k=int(k.value), sizes=sizes[:k.value].copy(), alloc=al, R=R,
                tried=int(st[0]), merged=int(st[1]), workload=int(np.uint64(st[2].view(np.uint64))))


def m_min(task: dict, i: int) -> int:
    return int(_load().or_m_min_ex(*_one(task), i))


def forbidden(task: dict, i: int, j: int) -> bool:
    f = _load().or_forbidden_ex(*_one(task), i, j)
    if f < 0:
        raise ValueError("set or task index outside the oracle's limits")
    return bool(f)


def lemma1_reject(task: dict) -> bool:
    return bool(_load().or_lemma1_reject_ex(*_one(task)))


def u1(task: dict, i: int) -> int:
    return int(_load().or_u1_ex(*_one(task), i))


def exec_time(task: dict, i: int, m: int, conflict: bool) -> int:
    a = _set_arrays(task)
    return int(_load().or_time(a[2], a[3], a[4], i, m, int(conflict)))
