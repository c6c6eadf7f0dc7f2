"""Write learned16384_counts.json: the oracle's weak-pseudo-manifold count of
every instance of the 16384-instance learned-scheduler workload (n = 5..8,
m = n + 4, upper-bound property applied), for the full-size GPU parity test.

Only the oracle and the seeded input generator run here.  About 15 minutes
on 8 host threads.  Usage:  python tests/golden/make_learned_counts.py
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import oracle as O  # noqa: E402
import wpm_inputs as W  # noqa: E402

COUNT = 16384


def main():
    t0 = time.time()
    insts = W.learned(O.kdim_of, count=COUNT)

    def one(inst):
        F = O.facets_of(inst)
        return O.count_wpm(inst.n, F, O.default_max_facets(inst.n, inst.m))

    threads = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as ex:
        counts = list(ex.map(one, insts, chunksize=16))
    arr = np.array(counts, dtype=np.int64)
    out = {
        "workload": "learned-scheduler batch: 16384 lambda = [I_n | 4 uniform], n = 5..8, m = n + 4",
        "source": "oracle.count_wpm (backtracking enumerator), upper-bound property when m = n + 4",
        "instances": COUNT,
        "total": int(arr.sum()),
        "counts_sha256_int64le": hashlib.sha256(arr.astype("<i8").tobytes()).hexdigest(),
        "counts": counts,
    }
    with open(os.path.join(HERE, "learned16384_counts.json"), "w") as f:
        json.dump(out, f)
    print(f"total {out['total']} in {time.time() - t0:.0f} s with {threads} threads")


if __name__ == "__main__":
    main()
