#!/usr/bin/env python3
"""Writes rmat22_df.json: the oracle's results on the 4M-vertex R-MAT
workload (scale 22, edge factor 16, the benchmark's seed), static Leiden and
then one DF update of 1e-3 |E| undirected updates (the first batch of a
two-batch stream), in the deterministic (synchronous) schedule.

Calls only the oracle and the seeded input generators.  Memberships are
stored as SHA-256 digests of their little-endian uint32 bytes.  Takes a few
minutes of single-threaded CPU time.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2410_15451_amd import inputs  # noqa: E402

SCALE, FRAC = 22, 1e-3


def digest(C):
    return hashlib.sha256(np.ascontiguousarray(C, dtype="<u4").tobytes()).hexdigest()


def main():
    t = time.time()
    g = inputs.rmat(SCALE, seed=inputs.BASE_SEED + 2)
    C0, q0, st0 = oracle.static(g)
    nb = inputs.batch_size_for(g.nnz, FRAC)
    (dels, ins), _ = inputs.random_batch_stream(g.n, g.undirected_keys(), nb, 2, seed=inputs.BASE_SEED + 2 + 1000)
    gt, dw = oracle.apply_batch(g, dels, ins)
    C1, _, q1, st1 = oracle.update(gt, dw, ins, oracle.initial_state(g, C0), "df")
    out = {
        "workload": "R-MAT scale %d, seed BASE_SEED + 2; DF update of %g |E| (first batch of a 2-batch stream, "
                    "seed BASE_SEED + 1002)" % (SCALE, FRAC),
        "n": g.n, "nnz": g.nnz, "batch_undirected_updates": nb,
        "static": {"q": q0, "passes": st0["passes"], "iters": st0["iters"], "membership_sha256": digest(C0),
                   "communities": int(len(np.unique(C0)))},
        "df": {"nnz": gt.nnz, "q": q1, "passes": st1["passes"], "iters": st1["iters"],
               "affected": st1["affected"], "membership_sha256": digest(C1)},
    }
    with open(os.path.join(HERE, "rmat22_df.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote rmat22_df.json in %.0f s" % (time.time() - t))


if __name__ == "__main__":
    main()
