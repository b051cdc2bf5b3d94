"""The no-allocation entry point (capart_solve_async_noalloc) against
capart_solve_async on the same device batches, field by field: two calls in a
row, the second on a smaller batch, so the shared per-GPU scratch array is
reused with the first call's contents still in it; every mode family, both
policies; and the workspace limit, which is refused before any launch."""
import numpy as np
import pytest

from paper_2105_10312_amd import capart, workload

pytestmark = pytest.mark.gpu
FIELDS = ("status", "verdict", "verdict_1g", "pidx", "sizes", "aidx", "maxU", "sumU", "n_evals", "alloc", "R",
          "R_1g")


@pytest.fixture(scope="module")
def eng():
    e = capart.Engine(0)
    yield e
    e.close()


def run(eng, ts, K, mode, policy, noalloc, max_tasks, max_M):
    import torch
    dev = capart.device_tasksets(ts)
    out = capart.device_results(ts.n_sets, ts.n_tasks, K)
    for v in out.values():
        v.fill_(-7 if v.dtype.is_signed else 7)  # stale values must be overwritten
    fn = capart.capart_solve_async_noalloc if noalloc else capart.capart_solve_async
    fn(eng.ctx, dev, K, mode, out, max_tasks=max_tasks, max_M=max_M, policy=policy)
    torch.cuda.synchronize()
    return {f: out[f].cpu().numpy() for f in FIELDS}


@pytest.mark.parametrize("mode,policy", [("BF_INA", "FP_DM"), ("SMS_ACT", "FP_DM"), ("BF_INA", "EDF"),
                                         ("EXH", "FP_DM")])
def test_noalloc_matches_solve_async_twice(eng, mode, policy):
    if mode == "EXH":
        big, small, K, mt, mM = (workload.config_c1(n_sets=100, seed=41), workload.config_c1(n_sets=30, seed=42),
                                 3, 5, 8)
    else:
        c3 = workload.config_c3(n_sets=3000, seed=43)
        big = workload.subset(c3, np.arange(1500))
        small = workload.subset(workload.config_c2(n_sets=400, seed=44), np.arange(200))
        K, mt, mM = 4, 32, 108
    for ts in (big, small):
        print(f"noalloc {mode} {policy}: {ts.n_sets} sets", flush=True)
        want = run(eng, ts, K, mode, policy, False, mt, mM)
        got = run(eng, ts, K, mode, policy, True, mt, mM)
        for f in FIELDS:
            assert np.array_equal(got[f], want[f]), (ts.n_sets, f)
        assert (want["status"] == 0).all()


def test_noalloc_refuses_a_batch_beyond_its_workspace(eng):
    # 2,000,000 one-task sets need about 2,000,000 x (41 + 44 + 32) bytes of workspace
    S = 2_000_000
    ts = workload.TaskSets(set_offset=np.arange(S + 1, dtype=np.int64), M=np.full(S, 1, np.int32),
                           T=np.full(S, 100, np.int64), D=np.full(S, 100, np.int64),
                           C_seq=np.full(S, 1, np.int64), C_par=np.zeros(S, np.int64),
                           k_permille=np.full(S, 1000, np.int32), type=np.zeros(S, np.uint8))
    dev = capart.device_tasksets(ts)
    out = capart.device_results(S, S, 1)
    with pytest.raises(capart.CapartError) as ei:
        capart.capart_solve_async_noalloc(eng.ctx, dev, 1, "BF_INA", out, max_tasks=1, max_M=1)
    assert ei.value.code == capart.CAPART_E_RANGE and "no-allocation limit" in str(ei.value)
