"""Write the oracle's solves of every system of the 512-system batch to batch_oracle.json.

Calls only the CPU oracle and the seeded input generators; run from the repository
root:  python tests/golden/make_batch.py
A batched solve must give each system exactly what solving it alone gives, so each
record is one independent oracle solve (p-BiCGSafe, FP64, x0 = 0, b = A*1, tol 1e-8):
iteration count, status, a SHA-256 of the residual history and of the solution's
bytes, and a few sampled entries.  Systems are solved in parallel processes.
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_oracle.json")
NAME = "cd2d_batch_512"


def solve_one(k):
    import oracle
    from paper_2108_10591_amd import workloads
    A = workloads.batch(NAME).systems[k]
    tol = workloads.BATCHES[NAME]["tol"]
    R = oracle.solve(A, tol=tol, maxit=10_000, variant="pbicgsafe")
    return k, {"n": A.n, "iters": R.iters, "status": R.status,
               "hist_sha256": hashlib.sha256(np.ascontiguousarray(R.hist).tobytes()).hexdigest(),
               "x_sha256": hashlib.sha256(np.ascontiguousarray(R.x).tobytes()).hexdigest(),
               "x_samples": {str(i): float(R.x[i]) for i in (0, A.n // 2, A.n - 1)},
               "x_minus_1_inf": float(np.abs(R.x - 1.0).max())}


def main():
    from paper_2108_10591_amd import workloads
    nsys = workloads.batch(NAME).nsys
    t = time.time()
    runs = {}
    with ProcessPoolExecutor(max_workers=3) as ex:
        for k, rec in ex.map(solve_one, range(nsys)):
            runs[str(k)] = rec
            if k % 32 == 0:
                print(f"system {k}: n={rec['n']} iters={rec['iters']} status={rec['status']} "
                      f"({time.time() - t:.0f} s)", flush=True)
    out = {"source": "oracle/oracle.c via oracle.solve (FP64, inner products rounded once "
                     "from their exact value), "
                     "each system alone; p-BiCGSafe, x0 = 0, b = A*1, tol 1e-8, maxit 10000",
           "workload": NAME, "runs": runs}
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"done in {time.time() - t:.0f} s", flush=True)


if __name__ == "__main__":
    main()
