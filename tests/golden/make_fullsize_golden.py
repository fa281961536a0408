"""Writes tests/golden/q100_oracle.json: the FP64 oracle's converged solve of
the 100^3 elasticity workload (3,060,300 DOF, sigma 2.0, body load + noise).
Calls only the oracle and the input generator. Takes minutes."""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import build_workload  # noqa: E402


def main():
    prob, b = build_workload("q1_100")
    A = (prob.row_ptr, prob.col, prob.val)
    t0 = time.time()
    st, L, alpha, restarts, mp = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    res = oracle.pcg(A, L, U, b, rtol=1e-8, history=True)
    x = res["x"]
    idx = np.arange(0, prob.n, 9973)
    out = dict(
        what="FP64 oracle: IC(0) with the global shift rule, then PCG to rtol 1e-8 (true residual checked) "
             "on the 100^3 Q1 elasticity workload, seeds 1003 / 2003",
        n=prob.n, nnz=prob.nnz, alpha=alpha, restarts=restarts, min_pivot=mp, status=res["status"],
        iters=res["iters"], replacements=res["replacements"], relres=res["relres"],
        true_relres=res["true_relres"], x_norm=float(np.linalg.norm(x)),
        sample_index=idx.tolist(), x_sample=x[idx].tolist(),
        relres_history_every_50=res["hist"][::50].tolist(), seconds=time.time() - t0)
    with open(os.path.join(HERE, "q100_oracle.json"), "w") as f:
        json.dump(out, f)
    print(json.dumps({k: out[k] for k in ("iters", "alpha", "true_relres", "seconds")}))


if __name__ == "__main__":
    main()
