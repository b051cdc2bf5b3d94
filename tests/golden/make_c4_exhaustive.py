"""Writes c4_exhaustive_16sets.json: the exhaustive search's full result for
the first 16 sets of the exhaustive stress workload (12 tasks, 48 units, at
most 4 parts: every allocation of all 1,033 partitionings), computed by the
oracle's memoised exhaustive search, which tests/test_oracle_fast.py checks
against the plain search.  Calls only the oracle and the input generator.

    python tests/golden/make_c4_exhaustive.py [threads]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2105_10312_amd import workload  # noqa: E402

N_SETS, K = 16, 4


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    ts = workload.subset(workload.config_c4(n_sets=1000), np.arange(N_SETS))
    t0 = time.time()
    r = oracle.solve(ts, K, "EXH", flags=oracle.FLAG_EXH_FAST, nthreads=threads)
    dt = time.time() - t0
    out = {"_source": "oracle.solve(config_c4(n_sets=1000)[0:16], K=4, EXH, FLAG_EXH_FAST); written by "
                      "tests/golden/make_c4_exhaustive.py",
           "generator": {"config": "config_c4", "n_sets": 1000, "indices": list(range(N_SETS))},
           "K": K, "seconds": round(dt, 1), "threads": threads}
    for f in ("status", "verdict", "verdict_1g", "pidx", "aidx", "maxU", "sumU", "n_evals", "alloc", "R", "R_1g"):
        out[f] = [int(x) for x in np.asarray(r[f]).ravel()]
    out["sizes"] = [[int(x) for x in row] for row in r["sizes"]]
    with open(os.path.join(HERE, "c4_exhaustive_16sets.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"{N_SETS} sets in {dt:.1f} s, {sum(out['verdict'])} schedulable")


if __name__ == "__main__":
    main()
