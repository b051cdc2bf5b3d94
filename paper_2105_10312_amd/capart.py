"""Thin ctypes binding of libcapart (the gfx950 engine's C ABI).

Argument marshalling only: every step of the method runs in the HIP kernels
behind ``include/capart.h``.  Functions keep the C names.  Host-pointer calls
take numpy arrays; ``capart_solve_async`` takes torch tensors that live on the
GPU (torch is used for device memory and streams, nothing else).  There is no
CPU fallback: if ``libcapart.so`` is missing the import of the library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcapart.so")

CAPART_OK, CAPART_E_INVAL, CAPART_E_RANGE, CAPART_E_NOMEM = 0, -1, -2, -3
CAPART_E_DEVICE, CAPART_E_AGAIN, CAPART_E_STATE = -4, -5, -6
CAPART_EXHAUSTIVE, CAPART_HEUR_BF_INA, CAPART_HEUR_BF_ACT = 0, 1, 2
CAPART_HEUR_SMS_INA, CAPART_HEUR_SMS_ACT = 3, 4
CAPART_POLICY_FP_DM = 0
CAPART_POLICY_EDF = 1
POLICIES = {"FP_DM": CAPART_POLICY_FP_DM, "EDF": CAPART_POLICY_EDF}
CAPART_FLAG_SKIP_1G, CAPART_FLAG_NO_LEMMA1, CAPART_FLAG_PER_SET_LAUNCH = 1, 2, 4
CAPART_SERVER_TABLES = 8
CAPART_ALG1_MAX_TASKS, CAPART_ALG1_BIG_MAX_M, CAPART_ALG1_BIG_MAX_NM = 256, 127, 14336
MODES = {"EXH": CAPART_EXHAUSTIVE, "BF_INA": CAPART_HEUR_BF_INA, "BF_ACT": CAPART_HEUR_BF_ACT,
         "SMS_INA": CAPART_HEUR_SMS_INA, "SMS_ACT": CAPART_HEUR_SMS_ACT}
EXPORTS = ["capart_create", "capart_destroy", "capart_last_error", "capart_build_hash", "capart_measure_valu",
           "capart_count_partitionings", "capart_solve_async_noalloc",
           "capart_enumerate_partitionings", "capart_validate", "capart_test_triple", "capart_allocate",
           "capart_solve", "capart_solve_async", "capart_set_tuning", "capart_get_tuning", "capart_timing_enable",
           "capart_timing_read", "capart_plan_batch", "capart_run_batch", "capart_plan_get_info",
           "capart_plan_destroy", "capart_server_create", "capart_server_submit", "capart_server_poll",
           "capart_server_stats_get", "capart_server_replay", "capart_server_destroy", "capart_count_work",
           "capart_alg1", "capart_alg1_async", "capart_alg1_count_work"]

_vp = C.c_void_p


class capart_tasksets(C.Structure):
    _fields_ = [("n_sets", C.c_int64), ("n_tasks_total", C.c_int64), ("max_tasks", C.c_int32),
                ("max_M", C.c_int32), ("set_offset", _vp), ("M", _vp), ("T", _vp), ("D", _vp),
                ("C_seq", _vp), ("C_par", _vp), ("k_permille", _vp), ("type", _vp),
                ("table_offset", _vp), ("Cn_table", _vp), ("Cc_table", _vp), ("table_len", C.c_int64)]


class capart_options(C.Structure):
    _fields_ = [("K", C.c_int32), ("policy", C.c_int32), ("alloc_mode", C.c_int32), ("flags", C.c_uint32),
                ("admissible", C.c_uint64 * 4)]


class capart_results(C.Structure):
    _fields_ = [("status", _vp), ("verdict", _vp), ("verdict_1g", _vp), ("pidx", _vp), ("sizes", _vp),
                ("aidx", _vp), ("maxU", _vp), ("sumU", _vp), ("n_evals", _vp), ("alloc", _vp), ("R", _vp),
                ("R_1g", _vp), ("dbg_key", _vp), ("dbg_offset", _vp)]


class capart_alg1_results(C.Structure):
    _fields_ = [("status", _vp), ("verdict", _vp), ("nparts", _vp), ("sizes", _vp), ("alloc", _vp), ("R", _vp),
                ("tried", _vp), ("merged", _vp), ("workload", _vp)]


ALG1_FIELDS = [("status", np.int32, "S"), ("verdict", np.uint8, "S"), ("nparts", np.int32, "S"),
               ("sizes", np.int32, "N"), ("alloc", np.int8, "N"), ("R", np.int64, "N"),
               ("tried", np.int64, "S"), ("merged", np.int64, "S"), ("workload", np.uint64, "S")]


class capart_tuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("chunk", C.c_int32), ("loop_form", C.c_int32), ("exh_form", C.c_int32),
                ("frontier", C.c_int32), ("memo", C.c_int32), ("wide_chunk", C.c_int32),
                ("reserved", C.c_int32)]


class capart_plan_config(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("blocks_per_cu", C.c_int32), ("item_evals", C.c_int32),
                ("use_graph", C.c_int32)]


class capart_plan_info(C.Structure):
    _fields_ = [("n_sets", C.c_int64), ("n_items", C.c_int64), ("total_evals", C.c_int64), ("threads", C.c_int32),
                ("loop_form", C.c_int32), ("blocks", C.c_int32), ("item_evals", C.c_int32),
                ("candidates_tried", C.c_int32), ("use_graph", C.c_int32), ("tune_ms", C.c_double)]


class capart_server_config(C.Structure):
    _fields_ = [("K", C.c_int32), ("alloc_mode", C.c_int32), ("flags", C.c_uint32), ("max_tasks", C.c_int32),
                ("max_M", C.c_int32), ("max_queries", C.c_int32), ("device_bytes", C.c_int64),
                ("streams", C.c_int32), ("max_batch", C.c_int32), ("policy", C.c_int32),
                ("admissible", C.c_uint64 * 4)]


class capart_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("batches", C.c_int64), ("evals", C.c_int64), ("p50_us", C.c_double), ("p99_us", C.c_double),
                ("mean_us", C.c_double), ("max_us", C.c_double), ("elapsed_s", C.c_double),
                ("queries_per_s", C.c_double), ("evals_per_s", C.c_double), ("mean_batch", C.c_double)]


class CapartError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"capart error {code}: {msg}")
        self.code = code


_lib = None


def load_library():
    """Load libcapart.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # torch ships its own HIP runtime with the same soname; loading torch
        # first makes libcapart bind to that one copy, so that torch's device
        # memory and streams belong to the runtime that launches the kernels
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(LIB_PATH)
        lib.capart_build_hash.argtypes = []
        lib.capart_build_hash.restype = C.c_char_p
        built = lib.capart_build_hash().decode()
        from . import build as _build
        if os.path.isdir(_build.CSRC) and built != _build.source_hash():
            raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {built}, sources "
                               f"{_build.source_hash()}): rebuild it with __graft_entry__.build()")
        P = C.POINTER
        lib.capart_create.argtypes = [C.c_int, P(_vp)]
        lib.capart_destroy.argtypes = [_vp]
        lib.capart_last_error.argtypes = [_vp]
        lib.capart_last_error.restype = C.c_char_p
        lib.capart_count_partitionings.argtypes = [C.c_int32, C.c_int32, P(C.c_int64)]
        lib.capart_measure_valu.argtypes = [_vp, P(C.c_double), P(C.c_double)]
        lib.capart_enumerate_partitionings.argtypes = [C.c_int32, C.c_int32, _vp, C.c_int64, P(C.c_int64)]
        lib.capart_validate.argtypes = [P(capart_tasksets), P(capart_options), _vp]
        lib.capart_test_triple.argtypes = [_vp, P(capart_tasksets), _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp]
        lib.capart_allocate.argtypes = [_vp, P(capart_tasksets), _vp, C.c_int32, P(capart_options), _vp, _vp,
                                        _vp, _vp, _vp]
        lib.capart_solve.argtypes = [_vp, P(capart_tasksets), P(capart_options), P(capart_results)]
        lib.capart_solve_async.argtypes = [_vp, P(capart_tasksets), P(capart_options), P(capart_results), _vp]
        lib.capart_solve_async_noalloc.argtypes = [_vp, P(capart_tasksets), P(capart_options), P(capart_results),
                                                   _vp]
        lib.capart_alg1.argtypes = [_vp, P(capart_tasksets), P(capart_options), P(capart_alg1_results)]
        lib.capart_alg1_async.argtypes = [_vp, P(capart_tasksets), P(capart_options), P(capart_alg1_results),
                                          _vp]
        lib.capart_alg1_count_work.argtypes = [_vp, P(capart_tasksets), P(capart_options),
                                               P(capart_alg1_results), _vp, _vp]
        lib.capart_set_tuning.argtypes = [_vp, P(capart_tuning)]
        lib.capart_get_tuning.argtypes = [_vp, P(capart_tuning)]
        lib.capart_timing_enable.argtypes = [_vp, C.c_int]
        lib.capart_plan_batch.argtypes = [_vp, P(capart_tasksets), P(capart_options), P(capart_results),
                                          P(capart_plan_config), P(_vp)]
        lib.capart_run_batch.argtypes = [_vp, _vp]
        lib.capart_plan_get_info.argtypes = [_vp, P(capart_plan_info)]
        lib.capart_plan_destroy.argtypes = [_vp]
        lib.capart_server_create.argtypes = [_vp, P(capart_server_config), P(_vp)]
        lib.capart_server_submit.argtypes = [_vp, P(capart_tasksets), P(C.c_uint64)]
        lib.capart_server_poll.argtypes = [_vp, C.c_uint64, P(capart_results), P(C.c_int32)]
        lib.capart_server_stats_get.argtypes = [_vp, P(capart_server_stats), C.c_int32]
        lib.capart_server_replay.argtypes = [_vp, P(capart_tasksets), _vp, P(capart_results),
                                             P(capart_server_stats)]
        lib.capart_server_destroy.argtypes = [_vp]
        lib.capart_count_work.argtypes = [_vp, P(capart_tasksets), P(capart_options), P(capart_results), _vp, _vp]
        lib.capart_timing_read.argtypes = [_vp, _vp, _vp]
        for name in EXPORTS:
            if name not in ("capart_last_error", "capart_build_hash"):
                getattr(lib, name).restype = C.c_int32
        _lib = lib
    return _lib


def _check(rc, ctx=None):
    if rc != CAPART_OK:
        msg = load_library().capart_last_error(ctx)
        raise CapartError(rc, msg.decode() if msg else "")
    return rc


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


def _mode(mode):
    return MODES[mode] if isinstance(mode, str) else int(mode)


def admissible_mask(sizes) -> list:
    """The 4-word mask of the admissible partition sizes (None or empty: every size)."""
    w = [0, 0, 0, 0]
    for m in (sizes if sizes is not None else ()):
        w[int(m) // 64] |= 1 << (int(m) % 64)
    return w


def make_options(K: int, mode="BF_INA", flags: int = 0, admissible=None, policy="FP_DM") -> capart_options:
    """policy: "FP_DM" (fixed priority, deadline monotonic) or "EDF", or the C constant."""
    pol = POLICIES[policy] if isinstance(policy, str) else int(policy)
    return capart_options(int(K), pol, _mode(mode), int(flags),
                          (C.c_uint64 * 4)(*admissible_mask(admissible)))


def make_tasksets(ts: dict, max_tasks: int | None = None, max_M: int | None = None, tasks_cap: int = 64) -> tuple:
    """capart_tasksets over numpy (host) or torch (device) arrays; returns (struct, keep-alive).
    Without max_tasks the bound is the largest set, capped at tasks_cap (256 for
    the Algorithm 1 calls)."""
    off = ts["set_offset"]
    S = int(ts["M"].shape[0])
    if max_tasks is None:
        sizes = np.diff(np.asarray(off.cpu() if hasattr(off, "cpu") else off))
        max_tasks = int(min(tasks_cap, max(1, sizes.max() if S else 1)))
    if max_M is None:
        Mh = ts["M"].cpu().numpy() if hasattr(ts["M"], "cpu") else ts["M"]
        max_M = int(min(255, max(1, Mh.max() if S else 1)))
    N = int(ts["T"].shape[0])
    tab = ts.get("Cn_table") is not None
    st = capart_tasksets(S, N, int(max_tasks), int(max_M), _ptr(off), _ptr(ts["M"]), _ptr(ts["T"]),
                         _ptr(ts["D"]), _ptr(ts.get("C_seq")), _ptr(ts.get("C_par")), _ptr(ts.get("k_permille")),
                         _ptr(ts["type"]), _ptr(ts["table_offset"]) if tab else None,
                         _ptr(ts["Cn_table"]) if tab else None, _ptr(ts["Cc_table"]) if tab else None,
                         int(ts["Cn_table"].shape[0]) if tab else 0)
    return st, ts


def _host_ts(ts: dict) -> dict:
    """SoA arrays with the boundary's dtypes; explicit time tables ("table_offset",
    "Cn_table", "Cc_table") are kept when present, and then the parametric
    fields may be absent."""
    h = {"set_offset": np.ascontiguousarray(ts["set_offset"], np.int64),
         "M": np.ascontiguousarray(ts["M"], np.int32),
         "T": np.ascontiguousarray(ts["T"], np.int64), "D": np.ascontiguousarray(ts["D"], np.int64),
         "type": np.ascontiguousarray(ts["type"], np.uint8)}
    for key, dt in (("C_seq", np.int64), ("C_par", np.int64), ("k_permille", np.int32)):
        if ts.get(key) is not None:
            h[key] = np.ascontiguousarray(ts[key], dt)
    if ts.get("Cn_table") is not None:
        for key in ("table_offset", "Cn_table", "Cc_table"):
            h[key] = np.ascontiguousarray(ts[key], np.int64)
    return h


# ---- C-ABI mirrors ---------------------------------------------------------------

def capart_create(device: int = 0):
    lib = load_library()
    h = _vp()
    _check(lib.capart_create(int(device), C.byref(h)), None)
    return h


def capart_destroy(ctx) -> None:
    _check(load_library().capart_destroy(ctx))


def capart_last_error(ctx=None) -> str:
    return load_library().capart_last_error(ctx).decode()


def capart_count_partitionings(M: int, K: int) -> int:
    c = C.c_int64(0)
    _check(load_library().capart_count_partitionings(int(M), int(K), C.byref(c)))
    return int(c.value)


def capart_enumerate_partitionings(M: int, K: int) -> np.ndarray:
    P = capart_count_partitionings(M, K)
    buf = np.zeros((max(P, 1), K), np.int32)
    c = C.c_int64(0)
    _check(load_library().capart_enumerate_partitionings(int(M), int(K), buf.ctypes.data, P, C.byref(c)))
    return buf[:P]


def capart_validate(ts: dict, K: int, mode="BF_INA", flags: int = 0, max_tasks=None, max_M=None) -> np.ndarray:
    h = _host_ts(ts)
    st, _keep = make_tasksets(h, max_tasks, max_M)
    opt = make_options(K, mode, flags)
    out = np.zeros(st.n_sets, np.int32)
    _check(load_library().capart_validate(C.byref(st), C.byref(opt), out.ctypes.data))
    return out


def _one_set(task: dict) -> dict:
    """One set as a host batch; a task dict with "Cn_table" and "Cc_table"
    (n * M entries each, task-major) brings explicit time tables."""
    n = len(task["T"])
    one = {"set_offset": np.array([0, n]), "M": np.array([int(task["M"])]), "T": task["T"], "D": task["D"],
           "type": task["type"]}
    for key in ("C_seq", "C_par", "k_permille"):
        if task.get(key) is not None:
            one[key] = task[key]
    if task.get("Cn_table") is not None:
        one.update(table_offset=np.zeros(1, np.int64), Cn_table=task["Cn_table"], Cc_table=task["Cc_table"])
    return _host_ts(one)


def capart_test_triple(ctx, task: dict, sizes, alloc):
    """One triple of one set on the device: (feasible, R[n], maxU, sumU)."""
    h = _one_set(task)
    st, _keep = make_tasksets(h)
    sz = np.ascontiguousarray(sizes, np.int32)
    al = np.ascontiguousarray(alloc, np.int8)
    n = len(al)
    feas = np.zeros(1, np.uint8)
    R = np.zeros(n, np.int64)
    mx = np.zeros(1, np.uint64)
    sm = np.zeros(1, np.uint64)
    _check(load_library().capart_test_triple(ctx, C.byref(st), sz.ctypes.data, len(sz), al.ctypes.data,
                                             feas.ctypes.data, R.ctypes.data, mx.ctypes.data, sm.ctypes.data), ctx)
    return bool(feas[0]), R, int(mx[0]), int(sm[0])


def capart_measure_valu(ctx) -> tuple:
    """(full-rate 32-bit VALU lane-operations per second, best kernel ms) measured on the device."""
    ops, ms = C.c_double(0.0), C.c_double(0.0)
    _check(load_library().capart_measure_valu(ctx, C.byref(ops), C.byref(ms)), ctx)
    return ops.value, ms.value


def capart_allocate(ctx, task: dict, sizes, K: int, mode="BF_INA", policy="FP_DM"):
    """Best allocation on one partitioning: (found, alloc[n], maxU, sumU, aidx)."""
    h = _one_set(task)
    st, _keep = make_tasksets(h)
    sz = np.ascontiguousarray(sizes, np.int32)
    opt = make_options(K, mode, policy=policy)
    n = len(task["T"])
    al = np.zeros(n, np.int8)
    found = np.zeros(1, np.uint8)
    mx = np.zeros(1, np.uint64)
    sm = np.zeros(1, np.uint64)
    ai = np.zeros(1, np.int64)
    _check(load_library().capart_allocate(ctx, C.byref(st), sz.ctypes.data, len(sz), C.byref(opt), al.ctypes.data,
                                          found.ctypes.data, mx.ctypes.data, sm.ctypes.data, ai.ctypes.data), ctx)
    return bool(found[0]), al, int(mx[0]), int(sm[0]), int(ai[0])


RESULT_FIELDS = (("status", np.int32, "S"), ("verdict", np.uint8, "S"), ("verdict_1g", np.uint8, "S"),
                 ("pidx", np.int32, "S"), ("sizes", np.int32, "SK"), ("aidx", np.int64, "S"),
                 ("maxU", np.uint64, "S"), ("sumU", np.uint64, "S"), ("n_evals", np.int64, "S"),
                 ("alloc", np.int8, "N"), ("R", np.int64, "N"), ("R_1g", np.int64, "N"))


def dbg_offsets(M, K: int) -> np.ndarray:
    """Prefix sums of P(M_s, K): start of each set's per-partitioning debug keys."""
    M = np.asarray(M)
    cnt = np.array([capart_count_partitionings(int(m), K) if 1 <= m <= 255 else 0 for m in M], np.int64)
    off = np.zeros(len(M) + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    return off


def capart_solve(ctx, ts: dict, K: int, mode="BF_INA", flags: int = 0, debug: bool = False, max_tasks=None,
                 max_M=None, admissible=None, policy="FP_DM") -> dict:
    """Solve a host batch (synchronous); returns a dict of numpy result arrays.
    admissible: the allowed partition sizes (None: every size); policy:
    per-partition scheduling ("FP_DM" or "EDF")."""
    h = _host_ts(ts)
    st, _keep = make_tasksets(h, max_tasks, max_M)
    opt = make_options(K, mode, flags, admissible, policy)
    S, N = st.n_sets, st.n_tasks_total
    out = {}
    for name, dt, shape in RESULT_FIELDS:
        size = S if shape == "S" else (S * K if shape == "SK" else N)
        out[name] = np.zeros(max(size, 1), dt)
    dbg = dboff = None
    if debug:
        dboff = dbg_offsets(h["M"], K)
        dbg = np.zeros(max(3 * int(dboff[-1]), 3), np.uint64)
    res = capart_results(*[_ptr(out[f[0]]) for f in RESULT_FIELDS], _ptr(dbg), _ptr(dboff))
    _check(load_library().capart_solve(ctx, C.byref(st), C.byref(opt), C.byref(res)), ctx)
    for name, dt, shape in RESULT_FIELDS:
        size = S if shape == "S" else (S * K if shape == "SK" else N)
        out[name] = out[name][:size]
    out["sizes"] = out["sizes"].reshape(S, K)
    if debug:
        out["dbg_key"] = dbg[:3 * int(dboff[-1])].reshape(-1, 3)
        out["dbg_offset"] = dboff
    return out


def device_results(S: int, N: int, K: int, device="cuda"):
    """Allocate result tensors on the GPU for capart_solve_async."""
    import torch
    tmap = {np.int32: torch.int32, np.uint8: torch.uint8, np.int64: torch.int64, np.uint64: torch.uint64,
            np.int8: torch.int8}
    out = {}
    for name, dt, shape in RESULT_FIELDS:
        size = S if shape == "S" else (S * K if shape == "SK" else N)
        out[name] = torch.empty(max(size, 1), dtype=tmap[dt], device=device)
    return out


def device_tasksets(ts: dict, device="cuda") -> dict:
    """Copy a host batch to GPU tensors (SoA, same dtypes)."""
    import torch
    h = _host_ts(ts)
    return {k: torch.from_numpy(v).to(device) for k, v in h.items()}


def capart_solve_async(ctx, dev_ts: dict, K: int, mode, dev_out: dict, stream=None, flags: int = 0,
                       max_tasks=None, max_M=None, dbg_key=None, dbg_offset=None, admissible=None,
                       policy="FP_DM") -> None:
    """Solve a batch resident in GPU memory; results land in dev_out (torch tensors) on `stream`."""
    import torch
    if max_tasks is None or max_M is None:
        raise ValueError("device batches need declared max_tasks and max_M bounds")
    st, _keep = make_tasksets(dev_ts, max_tasks, max_M)
    opt = make_options(K, mode, flags, admissible, policy)
    res = capart_results(*[_ptr(dev_out[f[0]]) for f in RESULT_FIELDS], _ptr(dbg_key), _ptr(dbg_offset))
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(load_library().capart_solve_async(ctx, C.byref(st), C.byref(opt), C.byref(res),
                                             C.c_void_p(stream.cuda_stream)), ctx)


def capart_solve_async_noalloc(ctx, dev_ts: dict, K: int, mode, dev_out: dict, stream=None, flags: int = 0,
                               max_tasks=None, max_M=None, admissible=None, policy="FP_DM") -> None:
    """capart_solve_async without any device allocation (the library's per-GPU
    scratch array holds the workspace); raises CapartError (E_RANGE) for a
    batch whose workspace exceeds CAPART_NOALLOC_SCRATCH_BYTES."""
    import torch
    if max_tasks is None or max_M is None:
        raise ValueError("device batches need declared max_tasks and max_M bounds")
    st, _keep = make_tasksets(dev_ts, max_tasks, max_M)
    opt = make_options(K, mode, flags, admissible, policy)
    res = capart_results(*[_ptr(dev_out[f[0]]) for f in RESULT_FIELDS], None, None)
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(load_library().capart_solve_async_noalloc(ctx, C.byref(st), C.byref(opt), C.byref(res),
                                                     C.c_void_p(stream.cuda_stream)), ctx)


def capart_alg1(ctx, ts: dict, mode="BF_INA", flags: int = 0, max_tasks=None, max_M=None, policy="FP_DM") -> dict:
    """Algorithm 1 (free partition sizes) over a host batch (synchronous); numpy results.
    sizes[set_offset[s] : set_offset[s] + nparts[s]] are set s's partitions in par_list order."""
    h = _host_ts(ts)
    st, _keep = make_tasksets(h, max_tasks, max_M, tasks_cap=256)
    opt = make_options(1, mode, flags, policy=policy)
    S, N = st.n_sets, st.n_tasks_total
    out = {name: np.zeros(max(S if shape == "S" else N, 1), dt) for name, dt, shape in ALG1_FIELDS}
    res = capart_alg1_results(*[_ptr(out[f[0]]) for f in ALG1_FIELDS])
    _check(load_library().capart_alg1(ctx, C.byref(st), C.byref(opt), C.byref(res)), ctx)
    return {name: out[name][:(S if shape == "S" else N)] for name, dt, shape in ALG1_FIELDS}


def device_alg1_results(S: int, N: int, device="cuda") -> dict:
    """Result tensors on the GPU for capart_alg1_async."""
    import torch
    tmap = {np.int32: torch.int32, np.uint8: torch.uint8, np.int64: torch.int64, np.int8: torch.int8,
            np.uint64: torch.uint64}
    return {name: torch.empty(max(S if shape == "S" else N, 1), dtype=tmap[dt], device=device)
            for name, dt, shape in ALG1_FIELDS}


def capart_alg1_async(ctx, dev_ts: dict, mode, dev_out: dict, stream=None, flags: int = 0, max_tasks=None,
                      max_M=None, policy="FP_DM") -> None:
    """Algorithm 1 over a batch resident in GPU memory; results land in dev_out on `stream`."""
    import torch
    if max_tasks is None or max_M is None:
        raise ValueError("device batches need declared max_tasks and max_M bounds")
    st, _keep = make_tasksets(dev_ts, max_tasks, max_M)
    opt = make_options(1, mode, flags, policy=policy)
    res = capart_alg1_results(*[_ptr(dev_out[f[0]]) for f in ALG1_FIELDS])
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(load_library().capart_alg1_async(ctx, C.byref(st), C.byref(opt), C.byref(res),
                                            C.c_void_p(stream.cuda_stream)), ctx)


def capart_alg1_count_work(ctx, dev_ts: dict, mode, dev_out: dict, max_tasks: int, max_M: int, stream=None,
                           flags: int = 0, policy="FP_DM") -> dict:
    """Counted work of Algorithm 1 on a device batch: response-time terms and exact tests."""
    import torch
    st, _keep = make_tasksets(dev_ts, max_tasks, max_M)
    opt = make_options(1, mode, flags, policy=policy)
    res = capart_alg1_results(*[_ptr(dev_out[f[0]]) for f in ALG1_FIELDS])
    if stream is None:
        stream = torch.cuda.current_stream()
    counts = np.zeros(2, np.int64)
    _check(load_library().capart_alg1_count_work(ctx, C.byref(st), C.byref(opt), C.byref(res),
                                                 C.c_void_p(stream.cuda_stream), counts.ctypes.data), ctx)
    return {"terms": int(counts[0]), "tests": int(counts[1])}


def capart_set_tuning(ctx, threads: int = 0, chunk: int = 0, loop_form: int = 0, exh_form: int = 0,
                      frontier: int = 0, memo: int = 0, wide_chunk: int = 0) -> None:
    t = capart_tuning(int(threads), int(chunk), int(loop_form), int(exh_form), int(frontier), int(memo),
                      int(wide_chunk))
    _check(load_library().capart_set_tuning(ctx, C.byref(t)), ctx)


def capart_get_tuning(ctx) -> dict:
    t = capart_tuning()
    _check(load_library().capart_get_tuning(ctx, C.byref(t)), ctx)
    return {"threads": t.threads, "chunk": t.chunk, "loop_form": t.loop_form, "exh_form": t.exh_form,
            "frontier": t.frontier, "memo": t.memo, "wide_chunk": t.wide_chunk}


def capart_timing_enable(ctx, enable: bool = True) -> None:
    _check(load_library().capart_timing_enable(ctx, int(bool(enable))), ctx)


def capart_timing_read(ctx):
    """Summed kernel milliseconds since the last read: ({prep, eval, final}, {launch counts})."""
    ms = np.zeros(3, np.float64)
    n = np.zeros(3, np.int64)
    _check(load_library().capart_timing_read(ctx, ms.ctypes.data, n.ctypes.data), ctx)
    names = ("prep", "eval", "final")
    return dict(zip(names, ms.tolist())), dict(zip(names, n.tolist()))


def capart_count_work(ctx, dev_ts: dict, K: int, mode, dev_out: dict, max_tasks: int, max_M: int, stream=None,
                      flags: int = 0, admissible=None, policy="FP_DM") -> dict:
    """Exact algorithmic work of one heuristic solve (counting kernel variant)."""
    import torch
    st, _keep = make_tasksets(dev_ts, max_tasks, max_M)
    opt = make_options(K, mode, flags, admissible, policy)
    res = capart_results(*[_ptr(dev_out[f[0]]) for f in RESULT_FIELDS], None, None)
    if stream is None:
        stream = torch.cuda.current_stream()
    cnt = np.zeros(3, np.int64)
    _check(load_library().capart_count_work(ctx, C.byref(st), C.byref(opt), C.byref(res),
                                            C.c_void_p(stream.cuda_stream), cnt.ctypes.data), ctx)
    return {"terms": int(cnt[0]), "tests": int(cnt[1]), "lookups": int(cnt[2])}


class Plan:
    """Batched form: a persistent, optionally graph-captured launch bound to one
    device batch and its device result tensors (keeps them alive)."""

    def __init__(self, ctx, dev_ts: dict, K: int, mode, dev_out: dict, max_tasks: int, max_M: int, flags: int = 0,
                 autotune: bool = True, blocks_per_cu: int = 0, item_evals: int = 0, use_graph: bool = True,
                 dbg_key=None, dbg_offset=None, admissible=None, policy="FP_DM"):
        self.ctx = ctx
        self._st, self._keep = make_tasksets(dev_ts, max_tasks, max_M)
        self._opt = make_options(K, mode, flags, admissible, policy)
        self._out = dev_out
        self._res = capart_results(*[_ptr(dev_out[f[0]]) for f in RESULT_FIELDS], _ptr(dbg_key), _ptr(dbg_offset))
        self._dbg = (dbg_key, dbg_offset)
        cfg = capart_plan_config(int(bool(autotune)), int(blocks_per_cu), int(item_evals), int(bool(use_graph)))
        h = _vp()
        _check(load_library().capart_plan_batch(ctx, C.byref(self._st), C.byref(self._opt), C.byref(self._res),
                                                C.byref(cfg), C.byref(h)), ctx)
        self.handle = h

    def run(self, stream=None) -> None:
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        _check(load_library().capart_run_batch(self.handle, C.c_void_p(stream.cuda_stream)), self.ctx)

    def info(self) -> dict:
        i = capart_plan_info()
        _check(load_library().capart_plan_get_info(self.handle, C.byref(i)), self.ctx)
        return {f[0]: getattr(i, f[0]) for f in capart_plan_info._fields_}

    def close(self) -> None:
        if getattr(self, "handle", None):
            _check(load_library().capart_plan_destroy(self.handle), self.ctx)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stats_dict(st) -> dict:
    return {f[0]: getattr(st, f[0]) for f in capart_server_stats._fields_}


def host_results(S: int, N: int, K: int) -> dict:
    out = {}
    for name, dt, shape in RESULT_FIELDS:
        size = S if shape == "S" else (S * K if shape == "SK" else N)
        out[name] = np.zeros(max(size, 1), dt)
    return out


class Server:
    """Serving form: admission-controlled, device-resident query state,
    continuous batching over several streams (see capart_server_* in capart.h)."""

    def __init__(self, ctx, K: int = 4, mode="BF_INA", flags: int = 0, max_tasks: int = 64, max_M: int = 108,
                 max_queries: int = 0, device_bytes: int = 0, streams: int = 0, max_batch: int = 0,
                 policy="FP_DM", tables: bool = False, admissible=None):
        self.ctx = ctx
        self.K = int(K)
        pol = POLICIES[policy] if isinstance(policy, str) else int(policy)
        if tables:
            flags = int(flags) | CAPART_SERVER_TABLES
        cfg = capart_server_config(int(K), _mode(mode), int(flags), int(max_tasks), int(max_M), int(max_queries),
                                   int(device_bytes), int(streams), int(max_batch), pol,
                                   (C.c_uint64 * 4)(*admissible_mask(admissible)))
        h = _vp()
        _check(load_library().capart_server_create(ctx, C.byref(cfg), C.byref(h)), ctx)
        self.handle = h

    def submit(self, task: dict):
        """Returns a ticket, or None when the server pushes back (E_AGAIN)."""
        hts = _one_set(task)
        st, _keep = make_tasksets(hts)
        t = C.c_uint64(0)
        rc = load_library().capart_server_submit(self.handle, C.byref(st), C.byref(t))
        if rc == CAPART_E_AGAIN:
            return None
        _check(rc, self.ctx)
        return int(t.value)

    def poll(self, ticket: int, n: int):
        """Returns a dict of one query's results, or None if not complete yet."""
        out = host_results(1, n, self.K)
        res = capart_results(*[_ptr(out[f[0]]) for f in RESULT_FIELDS], None, None)
        done = C.c_int32(0)
        _check(load_library().capart_server_poll(self.handle, C.c_uint64(ticket), C.byref(res), C.byref(done)),
               self.ctx)
        if not done.value:
            return None
        out["sizes"] = out["sizes"][:self.K].reshape(1, self.K)
        for name, dt, shape in RESULT_FIELDS:
            if shape == "N":
                out[name] = out[name][:n]
        return out

    def stats(self, reset: bool = False) -> dict:
        st = capart_server_stats()
        _check(load_library().capart_server_stats_get(self.handle, C.byref(st), int(bool(reset))), self.ctx)
        return _stats_dict(st)

    def replay(self, ts: dict, arrival_us, collect: bool = True):
        """Open-loop replay of a host batch at the given arrival times (us)."""
        h = _host_ts(ts)
        st, _keep = make_tasksets(h)
        arr = np.ascontiguousarray(arrival_us, np.float64)
        S, N = st.n_sets, st.n_tasks_total
        out = host_results(S, N, self.K) if collect else None
        res = capart_results(*[_ptr(out[f[0]]) for f in RESULT_FIELDS], None, None) if collect else None
        stats = capart_server_stats()
        _check(load_library().capart_server_replay(self.handle, C.byref(st), arr.ctypes.data,
                                                   C.byref(res) if collect else None, C.byref(stats)), self.ctx)
        if collect:
            for name, dt, shape in RESULT_FIELDS:
                size = S if shape == "S" else (S * self.K if shape == "SK" else N)
                out[name] = out[name][:size]
            out["sizes"] = out["sizes"].reshape(S, self.K)
        return out, _stats_dict(stats)

    def close(self) -> None:
        if getattr(self, "handle", None):
            _check(load_library().capart_server_destroy(self.handle), self.ctx)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Engine:
    """Owns one context on one device."""

    def __init__(self, device: int = 0):
        self.ctx = capart_create(device)

    def close(self):
        if self.ctx is not None:
            capart_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, ts, K, mode="BF_INA", flags=0, debug=False, admissible=None, policy="FP_DM"):
        return capart_solve(self.ctx, ts, K, mode, flags, debug, admissible=admissible, policy=policy)

    def alg1(self, ts, mode="BF_INA", flags=0, policy="FP_DM"):
        return capart_alg1(self.ctx, ts, mode, flags, policy=policy)

    def test_triple(self, task, sizes, alloc):
        return capart_test_triple(self.ctx, task, sizes, alloc)

    def allocate(self, task, sizes, K, mode="BF_INA"):
        return capart_allocate(self.ctx, task, sizes, K, mode)
