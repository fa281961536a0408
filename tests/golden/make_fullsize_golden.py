"""Writes tests/golden/q1_<E>_oracle.json and q1_<E>_oracle_x.npz: FP64 oracle
solves of a full-size elasticity workload, for the full-size GPU parity tests
and the benchmark's error-against-oracle figures:
  * E = 100 (default): 3,060,300 DOF, sigma 2.0, seed 1003; the body load +
    noise of seed 2003 and load cases 0 and 1 of the sixteen traction columns
    of seed 2004;
  * E = 150 (argument "150"): 10,260,450 DOF, sigma 1.5, seed 1004; load cases
    0 and 1 of its sixteen traction columns (seed 2004).

Calls only the oracle and the input generator. Per right-hand side:
  * JSON: the converged solve (rtol 1e-8, true residual checked): status, k0,
    relative and true residual, the recurrence residual of every step;
  * NPZ: x sampled every 997th entry after every step k0 - W .. k0 + W
    (W = 8; one run with rtol 0 that goes past k0 records them), so a GPU
    solve that stops near k0 is compared with the oracle at its own step
    count.
The factor (IC(0) with the global shift rule) is computed once; the solves run
in forked worker processes that share it, one thread each. Takes about 15
minutes (E = 100) and about an hour (E = 150) on 8 cores.
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

STRIDE = 997
TRACTION_COLUMNS = (0, 1)
W = 8
# per workload: the generator's name, whether the body-load column is solved,
# and the recording window K_LO .. K_HI (the run goes to K_HI steps; every
# k0 +- W must fall inside, asserted)
CASES = {100: dict(name="q1_100", body=True, k_lo=760, k_hi=850),
         150: dict(name="q1_150_loads16", body=False, k_lo=960, k_hi=1080)}
E_RUN = int(sys.argv[1]) if len(sys.argv) > 1 else 100
CFG = CASES[E_RUN]
OUT = os.path.join(HERE, f"q1_{E_RUN}_oracle.json")
OUT_X = os.path.join(HERE, f"q1_{E_RUN}_oracle_x.npz")
K_LO, K_HI = CFG["k_lo"], CFG["k_hi"]

_S = {}  # matrix, factor and right-hand sides, inherited by the forked workers


def _solve(job):
    name, record = job
    oracle.set_threads(1)
    A, L, U = _S["A"], _S["L"], _S["U"]
    b = _S["rhs"][name]
    if not record:
        return name, record, oracle.pcg(A, L, U, b, rtol=1e-8, history=True)
    return name, record, oracle.pcg(A, L, U, b, rtol=0.0, max_iter=K_HI, max_replace=0,
                                    snap=(_S["idx"], K_LO, K_HI))


def main():
    t0 = time.time()
    prob, b = build_workload(CFG["name"])
    A = (prob.row_ptr, prob.col, prob.val)
    st, L, alpha, restarts, minpiv = oracle.ic0_shifted(*A)
    assert st == oracle.OK
    U = oracle.transpose(*L)
    seed_t = WORKLOADS["q1_150_loads16"]["seed_b"]
    B = traction_loads(E_RUN, max(TRACTION_COLUMNS) + 1, seed_t)
    rhs = {"body": b} if CFG["body"] else {}
    for c in TRACTION_COLUMNS:
        rhs[f"traction{c}"] = np.ascontiguousarray(B[:, c])
    idx = np.arange(0, prob.n, STRIDE)
    _S.update(A=A, L=L, U=U, rhs=rhs, idx=idx)
    jobs = [(name, rec) for name in rhs for rec in (False, True)]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        res = pool.map(_solve, jobs)
    conv = {name: r for name, rec, r in res if not rec}
    recd = {name: r for name, rec, r in res if rec}
    cases, xw = {}, {}
    for name, r in conv.items():
        assert r["status"] == oracle.OK and r["replacements"] == 0, (name, r["status"])
        k0 = r["iters"]
        assert K_LO <= k0 - W and k0 + W <= K_HI, (name, k0)
        snap = recd[name]["x_snap"]
        win = snap[k0 - W - K_LO:k0 + W - K_LO + 1]
        assert np.isfinite(win).all()
        # the recording run is the same iteration: it passes k0 with the same iterate
        assert np.array_equal(win[W], r["x"][idx])
        xw[name] = win
        cases[name] = dict(
            status=r["status"], iters=k0, replacements=r["replacements"], relres=r["relres"],
            true_relres=r["true_relres"], x_norm=float(np.linalg.norm(r["x"])),
            relres_history=r["hist"].tolist(), x_window_steps=[k0 - W, k0 + W])
    out = dict(
        what=f"FP64 oracle on the {E_RUN}^3 Q1 elasticity workload ({CFG['name']}): IC(0) with the global "
             "shift rule, then PCG to rtol 1e-8 (true residual checked) from x0 = 0; the iterates on every "
             f"{STRIDE}th entry after steps k0 - {W} .. k0 + {W} are in q1_100_oracle_x.npz (key = case name, "
             "row = step - (k0 - W))",
        rhs={**({"body": "body load (0,0,-1) + N(0, 0.1^2) noise, seed 2003"} if CFG["body"] else {}),
             **{f"traction{c}": f"load case {c} of traction_loads({E_RUN}, 16, {seed_t})" for c in TRACTION_COLUMNS}},
        n=prob.n, nnz=prob.nnz, alpha=alpha, restarts=restarts, min_pivot=minpiv,
        sample_stride=STRIDE, sample_index=idx.tolist(), window=W, cases=cases, seconds=time.time() - t0)
    np.savez(OUT_X, **xw)
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(json.dumps({k: (v["iters"], v["true_relres"]) for k, v in cases.items()}), f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
