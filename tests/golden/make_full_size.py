"""Write the oracle's full solves of the two large workloads to full_size_oracle.json.

Calls only the CPU oracle and the seeded input generators; run from the repository
root:  python tests/golden/make_full_size.py [--only-missing]
Each record holds the iteration count, status, the whole residual history, a
SHA-256 of the solution's bytes and a few sampled entries.  Keys are
"workload/variant" for FP64 solves and "workload/variant@p<precision>" for the
mixed-precision ones (precision 1: FP32 values in every product; 2: FP32 values
in the Krylov products, FP64 residual statements; 3: as 2, with p, u, z held as
FP32 numbers).  --only-missing keeps the
records already in the file and adds the others.
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
    variant, _, prec = variant.partition("@p")
    A = workloads.workload(name)
    tol = workloads.WORKLOADS[name]["tol"]
    t = time.time()
    R = oracle.solve(A, tol=tol, maxit=10_000, variant=variant, rr_m=100,
                     precision=int(prec) if prec else 0)
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


KEYS = [f"{name}/{variant}" for name in ("cd3d_128", "rand_band_1m")
        for variant in ("pbicgsafe", "ssbicgsafe2", "pbicgsafe_rr", "pbicgstab",
                        "pbicgsafe@p1", "pbicgsafe_rr@p2", "pbicgsafe_rr@p3")]


def main():
    out = {"source": "oracle/oracle.c via oracle.solve (FP64 arithmetic, inner products rounded "
                     "once from their exact value; @p1/@p2: the matrix values rounded to FP32 in "
                     "every product / in the Krylov products / and p, u, z held in FP32); x0 = 0, b = A*1, "
                     "maxit 10000, rr_m 100",
           "runs": {}}
    keys = KEYS
    if "--only-missing" in sys.argv and os.path.exists(OUT):
        out["runs"] = json.load(open(OUT))["runs"]
        keys = [k for k in KEYS if k not in out["runs"]]
    # independent solves in parallel processes (each holds one matrix; the oracle's
    # OpenMP threads are shared among them)
    with ProcessPoolExecutor(max_workers=2) as ex:
        for key, rec in ex.map(solve_one, keys):
            out["runs"][key] = rec
    with open(OUT, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
