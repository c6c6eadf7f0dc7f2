"""Write <workload>_counts.json: the oracle's weak-pseudo-manifold count of
every instance of a batched synthetic workload, for the full-size GPU parity
tests and the benchmark's oracle check.

Workloads (wpm_inputs recipes; the upper-bound property of Section 4.2 is
applied when m = n + 4, as Algorithm 4.4 does, and for the 7-subsets of [11]
as well, since m = n + 4 there too):
  batch    4096 instances, n = 4..7, 12 <= k <= 32   -> batch4096_counts.json
  stress   64 random 0.75-dense subsets of the 7-subsets of [11],
           32 <= k <= 40                              -> stress64_counts.json
  learned  16384 instances, n = 5..8, k <= 36         -> learned16384_counts.json

Only the oracle and the seeded input generator run here: instances are
selected with the oracle's own kernel dimension, and each count comes from
the oracle's backtracking enumerator (no kernel, no sweep).
Usage:  python tests/golden/make_counts.py batch|stress|learned [threads]
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

WORKLOADS = {
    "batch": (4096, lambda c: W.batch(O.kdim_of, count=c),
              "batch: 4096 lambda = [I_n | 4 uniform], n = 4..7, m = n + 4, 12 <= k <= 32"),
    "stress": (64, lambda c: W.stress(O.kdim_of, count=c),
               "stress: 64 random 0.75-dense subsets of the 7-subsets of [11], 32 <= k <= 40"),
    "learned": (16384, lambda c: W.learned(O.kdim_of, count=c),
                "learned-scheduler batch: 16384 lambda = [I_n | 4 uniform], n = 5..8, m = n + 4"),
}


def main():
    name = sys.argv[1]
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else min(16, os.cpu_count() or 1)
    count, gen, desc = WORKLOADS[name]
    t0 = time.time()
    insts = gen(count)
    print(f"selected {len(insts)} instances in {time.time() - t0:.0f} s", flush=True)
    ks = [O.kdim_of(i) for i in insts]

    def one(inst):
        F = O.facets_of(inst)
        t = time.time()
        c = O.count_wpm(inst.n, F, O.default_max_facets(inst.n, inst.m))
        return c, time.time() - t

    # largest kernels first, so the slowest searches do not end the run alone
    order = sorted(range(len(insts)), key=lambda i: -ks[i])
    counts = [0] * len(insts)
    secs = [0.0] * len(insts)
    with ThreadPoolExecutor(threads) as ex:
        for i, (c, s) in zip(order, ex.map(one, [insts[i] for i in order])):
            counts[i], secs[i] = c, s
    arr = np.array(counts, dtype=np.int64)
    out = {
        "workload": desc,
        "source": "oracle.count_wpm (backtracking enumerator), upper-bound property when m = n + 4",
        "instances": len(insts),
        "total": int(arr.sum()),
        "counts_sha256_int64le": hashlib.sha256(arr.astype("<i8").tobytes()).hexdigest(),
        "k": ks,
        "counts": counts,
        "oracle_seconds_single_thread": [round(s, 3) for s in secs],
    }
    path = os.path.join(HERE, f"{name}{len(insts)}_counts.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"{path}: total {out['total']} in {time.time() - t0:.0f} s with {threads} threads")


if __name__ == "__main__":
    main()
