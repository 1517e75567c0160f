"""Write the oracle's full solves of the two large workloads to full_size_oracle.json.

Calls only the CPU oracle and the seeded input generators; run from the repository
root:  python tests/golden/make_full_size.py
Each record holds the iteration count, status, the whole residual history, a
SHA-256 of the solution's bytes and a few sampled entries.
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2108_10591_amd import workloads  # noqa: E402

SAMPLES = [0, 1, 17, 4095, 65536, 123457, 999999]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_oracle.json")


def solve_one(key):
    name, variant = key.split("/")
    A = workloads.workload(name)
    tol = workloads.WORKLOADS[name]["tol"]
    t = time.time()
    R = oracle.solve(A, tol=tol, maxit=10_000, variant=variant, rr_m=100)
    print(f"{name} {variant}: {R.iters} iterations, status {R.status}, "
          f"{time.time() - t:.0f} s", flush=True)
    return key, {
        "tol": tol, "iters": R.iters, "status": R.status,
        "hist": [float(h) for h in R.hist],
        "x_sha256": hashlib.sha256(np.ascontiguousarray(R.x).tobytes()).hexdigest(),
        "x_samples": {str(i): float(R.x[i]) for i in SAMPLES if i < A.n},
        "x_minus_1_inf": float(np.abs(R.x - 1.0).max()),
        "seconds": round(time.time() - t, 1),
    }


def main():
    out = {"source": "oracle/oracle.c via oracle.solve (FP64, inner products rounded once from "
                     "their exact value); x0 = 0, b = A*1, maxit 10000, rr_m 100",
           "runs": {}}
    keys = [f"{name}/{variant}" for name in ("cd3d_128", "rand_band_1m")
            for variant in ("pbicgsafe", "ssbicgsafe2", "pbicgsafe_rr", "pbicgstab")]
    # independent solves in parallel processes (each holds one matrix)
    with ProcessPoolExecutor(max_workers=4) as ex:
        for key, rec in ex.map(solve_one, keys):
            out["runs"][key] = rec
    with open(OUT, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
