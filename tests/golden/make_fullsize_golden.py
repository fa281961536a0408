"""Writes tests/golden/q1_100_oracle.json: FP64 oracle solves of the 100^3
elasticity workload (3,060,300 DOF, sigma 2.0, seed 1003), for the full-size
GPU parity tests and the benchmark's error-against-oracle figure.

Calls only the oracle and the input generator. Content, per right-hand side
(the body load + noise of seed 2003, and load cases 0 and 1 of the sixteen
traction columns of seed 2004):
  * the converged solve (rtol 1e-8, true residual checked): status, k0,
    relative and true residual, the recurrence residual of every step;
  * x sampled every 997th entry at k0 - 1, k0 and k0 + 1 steps (the last two
    of runs with rtol 0 and max_iter fixed), so that a GPU solve stopping
    within one step of the oracle is compared with the oracle at its own
    step count.
The factor (IC(0) with the global shift rule) is computed once; the solves run
in forked worker processes that share it. Takes about ten minutes on 8 cores.
"""

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from synth import WORKLOADS, build_workload, traction_loads  # noqa: E402

OUT = os.path.join(HERE, "q1_100_oracle.json")
STRIDE = 997
TRACTION_COLUMNS = (0, 1)

_S = {}  # matrix, factor and right-hand sides, inherited by the forked workers


def _solve(job):
    name, k = job
    A, L, U = _S["A"], _S["L"], _S["U"]
    b = _S["rhs"][name]
    if k is None:
        r = oracle.pcg(A, L, U, b, rtol=1e-8, history=True)
    else:
        r = oracle.pcg(A, L, U, b, rtol=0.0, max_iter=k, max_replace=0)
    return name, k, r


def main():
    t0 = time.time()
    prob, b = build_workload("q1_100")
    A = (prob.row_ptr, prob.col, prob.val)
    st, L, alpha, restarts, minpiv = oracle.ic0_shifted(*A)
    assert st == oracle.OK
    U = oracle.transpose(*L)
    seed_t = WORKLOADS["q1_150_loads16"]["seed_b"]
    B = traction_loads(100, max(TRACTION_COLUMNS) + 1, seed_t)
    rhs = {"body": b}
    for c in TRACTION_COLUMNS:
        rhs[f"traction{c}"] = np.ascontiguousarray(B[:, c])
    _S.update(A=A, L=L, U=U, rhs=rhs)
    idx = np.arange(0, prob.n, STRIDE)
    ctx = mp.get_context("fork")
    with ctx.Pool(len(rhs)) as pool:
        conv = {name: r for name, _, r in pool.map(_solve, [(name, None) for name in rhs])}
    jobs = []
    for name, r in conv.items():
        assert r["status"] == oracle.OK and r["replacements"] == 0, (name, r["status"])
        jobs += [(name, r["iters"] - 1), (name, r["iters"] + 1)]
    with ctx.Pool(min(8, len(jobs))) as pool:
        near = pool.map(_solve, jobs)
    cases = {}
    for name, r in conv.items():
        k0 = r["iters"]
        xs = {str(k0): r["x"][idx].tolist()}
        for nm, k, rk in near:
            if nm == name:
                assert rk["iters"] == k and rk["status"] == oracle.MAXITER
                xs[str(k)] = rk["x"][idx].tolist()
        cases[name] = dict(
            status=r["status"], iters=k0, replacements=r["replacements"], relres=r["relres"],
            true_relres=r["true_relres"], x_norm=float(np.linalg.norm(r["x"])),
            relres_history=r["hist"].tolist(), x_sample_at=xs)
    out = dict(
        what="FP64 oracle on the 100^3 Q1 elasticity workload (sigma 2.0, seed 1003): IC(0) with the global "
             "shift rule, then PCG to rtol 1e-8 (true residual checked) from x0 = 0; x sampled every "
             f"{STRIDE}th entry at the converged step count k0 and at k0 - 1, k0 + 1 (runs with rtol 0)",
        rhs={"body": "body load (0,0,-1) + N(0, 0.1^2) noise, seed 2003",
             **{f"traction{c}": f"load case {c} of traction_loads(100, 16, {seed_t})" for c in TRACTION_COLUMNS}},
        n=prob.n, nnz=prob.nnz, alpha=alpha, restarts=restarts, min_pivot=minpiv,
        sample_stride=STRIDE, sample_index=idx.tolist(), cases=cases, seconds=time.time() - t0)
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(json.dumps({k: (v["iters"], v["true_relres"]) for k, v in cases.items()}), f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
