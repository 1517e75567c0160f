"""The stored goldens agree with the oracle as it stands (CPU).

tests/golden/*.json hold oracle results written by the committed scripts beside
them; the GPU tests compare against those files.  Re-running the cheapest few
recorded solves here catches a later change to the oracle's arithmetic that was
not followed by regenerating the goldens.
"""
import hashlib
import json
import os

import numpy as np

import oracle as O
from paper_2108_10591_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def cheapest(runs, cost, count):
    return sorted(runs.items(), key=lambda kv: cost(kv[1]))[:count]


def test_batch_golden_matches_oracle():
    g = json.load(open(os.path.join(GOLDEN, "batch_oracle.json")))
    B = W.batch(g["workload"])
    tol = W.BATCHES[g["workload"]]["tol"]
    for k, r in cheapest(g["runs"], lambda r: r["n"] * r["iters"], 3):
        R = O.solve(B.systems[int(k)], tol=tol, maxit=10_000, variant="pbicgsafe")
        assert (R.iters, R.status) == (r["iters"], r["status"]), k
        assert sha(R.hist) == r["hist_sha256"] and sha(R.x) == r["x_sha256"], k


def test_varcoef_golden_matches_oracle():
    g = json.load(open(os.path.join(GOLDEN, "varcoef_oracle.json")))
    p = g["problems"]
    B, _ = W.varcoef_problems(p["count"], p["N"], seed=p["seed"])
    for k, r in cheapest(g["runs"], lambda r: r["iters"], 2):
        R = O.solve(B.systems[int(k)], **g["solve"])
        assert (R.iters, R.status) == (r["iters"], r["status"]), k
        assert sha(R.hist) == r["hist_sha256"] and sha(R.x) == r["x_sha256"], k
