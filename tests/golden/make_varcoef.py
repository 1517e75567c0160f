"""Write the oracle's solves of 16 high-contrast variable-coefficient problems to
varcoef_oracle.json.

Calls only the CPU oracle and the seeded input generators; run from the repository
root:  python tests/golden/make_varcoef.py
These are the learned-initial-guess problems (128 x 128, diffusion exp(g) with g a
Gaussian random field, convection up to 30): p-BiCGSafe-rr (m = 50) to 1e-10 ||b||
takes a thousand iterations and more, and late in such a solve inner products such
as (r0*, r_i) cancel to a tiny fraction of their terms.  There the value of an
inner product summed to about twice double precision can depend on the summation
order, and one differing bit changes the rest of the solve.  Each record holds the
iteration count, status and SHA-256 digests of the residual history and of the
solution's bytes.  Problems are solved in parallel processes.
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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "varcoef_oracle.json")
COUNT, N, SEED = 16, 128, 7
SOLVE = dict(tol=1e-10, maxit=20_000, variant="pbicgsafe_rr", rr_m=50, norm_ref=1)


def solve_one(k):
    import oracle
    from paper_2108_10591_amd import workloads
    B, _ = workloads.varcoef_problems(COUNT, N, seed=SEED)
    A = B.systems[k]
    R = oracle.solve(A, **SOLVE)
    return k, {"n": A.n, "iters": R.iters, "status": R.status,
               "hist_sha256": hashlib.sha256(np.ascontiguousarray(R.hist).tobytes()).hexdigest(),
               "x_sha256": hashlib.sha256(np.ascontiguousarray(R.x).tobytes()).hexdigest()}


def main():
    t = time.time()
    runs = {}
    with ProcessPoolExecutor(max_workers=6) as ex:
        for k, rec in ex.map(solve_one, range(COUNT)):
            runs[str(k)] = rec
            print(f"problem {k}: iters={rec['iters']} status={rec['status']} ({time.time() - t:.0f} s)",
                  flush=True)
    out = {"source": "oracle/oracle.c via oracle.solve (FP64, inner products rounded once from "
                     "their exact value), each problem alone; x0 = 0",
           "problems": {"count": COUNT, "N": N, "seed": SEED}, "solve": SOLVE, "runs": runs}
    with open(OUT, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
