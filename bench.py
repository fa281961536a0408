"""Benchmark of the IC(0)-PCG path on one MI355X.

Workload: clamped Q1 linear-elasticity box of 100^3 unit hexahedra
(3,060,300 DOF, 242,991,882 stored entries), lognormal Young's modulus with
sigma = 2.0, nu = 0.3. IC(0) is computed in FP64 on the GPU; PCG runs to a
relative residual of 1e-8 with a true-residual check.

A timed step is one multi-RHS solve of 16 load cases (body load plus a
seeded random traction on the top face) with the IC(0) factor applied in
FP32 and FP64 recurrences. The value is solved right-hand sides per second
over the timed steps (inputs resident in HBM). Reported beside it:
single-RHS solves in FP64, FP32-L and BF16-L, and the multicolour node order
(the right-hand sides permuted in and the solutions back inside the timing)
and the block multicolour order (4^3-node mesh blocks) for one FP64 solve and
one 16-RHS step each, with the factors (P-time) and the ordering time
separately.

One JSON line on stdout; progress on stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--E", type=int, default=100, help="elements per box edge")
    ap.add_argument("--sigma", type=float, default=2.0)
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--skip-cpu", action="store_true", help="omit the CPU oracle baseline")
    ap.add_argument("--skip-single", action="store_true", help="omit the single-RHS variants")
    ap.add_argument("--skip-150", action="store_true", help="omit the 150^3 inference workload")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--kernels-only", action="store_true",
                    help="factor, then only the per-kernel launches at the headline shape and a copy of known "
                         "size (the target of the rocprofv3 counter passes)")
    return ap.parse_args()


def grouped_pattern(rp, ci, gmax=3):
    """Rows grouped as the row-group SpMV reads them (consecutive rows with
    identical column lists, runs cut into pieces of gmax): returns (number of
    groups, column indices stored once per group)."""
    lens = np.diff(rp)
    n = lens.shape[0]
    same = np.zeros(n, bool)
    cand = np.nonzero(lens[1:] == lens[:-1])[0] + 1
    if cand.size:
        starts = rp[cand]
        ln = lens[cand]
        idx = np.repeat(starts - rp[0], ln) + (np.arange(ln.sum()) - np.repeat(np.cumsum(ln) - ln, ln))
        eq = ci[idx] == ci[idx - np.repeat(ln, ln)]
        ok = np.logical_and.reduceat(eq, np.cumsum(ln) - ln) if eq.size else np.zeros(0, bool)
        same[cand] = ok
    begin = ~same
    run_start = np.maximum.accumulate(np.where(begin, np.arange(n), 0))
    leader = begin | (((np.arange(n) - run_start) % gmax) == 0)
    return int(leader.sum()), int(lens[leader].sum())


def kernel_bytes(n, nnzA, nnzL, nsn, R, vbytes, rbytes, obytes, ngroups, grouped_cols):
    """Algorithmic bytes per launch (int32 columns, each vector row read
    once): the row-group SpMV reads A's values, the column indices once per
    row group, one 16-byte record per group (offset, first row, length and
    size), x, and writes y; a triangular solve reads its factor (value + 4 B
    column), one 16-byte schedule record per supernode, the right-hand side,
    and writes the solution."""
    spmv = 8 * nnzA + 4 * grouped_cols + 16 * ngroups + 16 * n * R
    trsv = (vbytes + 4) * nnzL + 16 * nsn + (rbytes + obytes) * n * R
    return spmv, trsv


def rz_extra_bytes(n, R):
    """What the backward solve of a PCG step reads beyond the solve itself: r
    (FP64) for r^T z."""
    return 8 * n * R


def xr_extra_bytes(n, R):
    """What the forward solve of a PCG step moves beyond the solve itself when
    it applies the previous step's update x += alpha p, r -= alpha w (FP32 /
    BF16 factors on several columns): w, x and p read, r and x written (FP64;
    r is the solve's right-hand side, already counted)."""
    return 40 * n * R


def rearm_extra_bytes(n, R):
    """What the backward solve of a PCG step writes beyond the solve itself
    where it forms r^T z (FP32 / BF16 factors on 2-16 columns): y re-armed as
    pending once read (FP32)."""
    return 4 * n * R


def step_fuses_rz(R):
    """Whether the library's PCG step at this width forms r^T z in the
    backward solve, which then also re-arms y (its default for FP32 / BF16
    factors on 2-16 columns; ICPCG_FUSE_RZ=0 turns it off)."""
    return R > 1 and os.environ.get("ICPCG_FUSE_RZ", "1") != "0"


def step_fuses_xr(R):
    """Whether the library's PCG step at this width applies the x, r update
    in the forward solve (its default for FP32 / BF16 factors on 2-16
    columns; ICPCG_FUSE_XR=0 turns it off)."""
    return R > 1 and os.environ.get("ICPCG_FUSE_XR", "1") != "0"


def recorded_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, if the kernel
    source is unchanged since the counters were taken (else None)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "q1_100_R16_hbm_counters.md")
    try:
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        rec = json.loads(m.group(1))[kernel]
        src = open(os.path.join(ROOT, rec["src"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["src_sha256"]:
            return None
        return rec["hbm_bytes"]
    except (OSError, KeyError, AttributeError, ValueError):
        return None


def time_kernels(ctx, M, P, R, reps, torch):
    """Average duration of one SpMV (the row-group kernel the solver uses) and
    one forward and one backward solve launch at block width R, with events on
    the stream the library launches on. The backward solve is the launch a PCG
    step makes: it also reads r and forms r^T z per column (fused into the
    solve for FP32 / BF16 factors on 2-16 columns, with its one-block
    finalize; else the separate pass). The three are launched in a PCG step's
    order (SpMV, forward, backward) and timed each time, so every launch meets
    the cache state the step leaves (the SpMV streams A and x through the
    caches between two solves)."""
    n = M.n
    X = torch.randn(n, R, dtype=torch.float64, device="cuda")
    W = torch.empty_like(X)
    Rf = torch.randn(n, R, dtype=torch.float64, device="cuda")
    Yf = P.trsv(Rf)
    s = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    # the trsv entry point fills the output with the pending pattern first; time
    # the fill alone and subtract it so the figure is the solve kernel's
    Yf.fill_(float("nan"))
    torch.cuda.synchronize()
    fill = 0.0
    for _ in range(reps):
        e0, e1 = ev(), ev()
        e0.record(s)
        Yf.fill_(float("nan"))
        e1.record(s)
        e1.synchronize()
        fill += e0.elapsed_time(e1)
    fill = fill / reps * 1e-3

    Zb = torch.empty_like(Yf)
    rz = torch.empty(R, dtype=torch.float64, device="cuda")

    def step():
        M.spmv(X, out=W)
        Y = P.trsv(Rf)
        P.trsv_rz(Y, Rf, Zb, rz)

    step()
    torch.cuda.synchronize()
    tot = [0.0, 0.0, 0.0]
    for _ in range(reps):
        e = [ev() for _ in range(4)]
        e[0].record(s)
        M.spmv(X, out=W)
        e[1].record(s)
        Y = P.trsv(Rf)
        e[2].record(s)
        P.trsv_rz(Y, Rf, Zb, rz)
        e[3].record(s)
        e[3].synchronize()
        for k in range(3):
            tot[k] += e[k].elapsed_time(e[k + 1])
    ms = [t / reps * 1e-3 for t in tot]
    return {"spmv": ms[0], "trsv_L": max(1e-9, ms[1] - fill), "trsv_U_rz": max(1e-9, ms[2] - fill)}


def cpu_baseline(prob, b, k_target, iters=24):
    """The FP64 oracle on the host, two legs on the same matrix: (i) one
    thread: full IC(0), then `iters` PCG iterations; (ii) the row-parallel
    loops (SpMV rows, vector updates) on every core the process may use,
    inner products and triangular solves sequential: `iters` iterations. CG
    time is extrapolated to the GPU's FP64 iteration count; the reported value
    is the faster leg (the multi-core one)."""
    import oracle
    A = (prob.row_ptr, prob.col, prob.val)
    nproc = os.cpu_count()
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        share = nproc
    threads = int(os.environ.get("OMP_NUM_THREADS", share) or share)
    default = oracle.set_threads(0)
    try:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        st, L, alpha, _, _ = oracle.ic0_shifted(*A)
        t_fac = time.perf_counter() - t0
        U = oracle.transpose(*L)
        t0 = time.perf_counter()
        oracle.pcg(A, L, U, b, rtol=0.0, max_iter=iters, max_replace=0)
        t_it1 = (time.perf_counter() - t0) / iters
        used = oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.pcg(A, L, U, b, rtol=0.0, max_iter=iters, max_replace=0)
        t_itm = (time.perf_counter() - t0) / iters
    finally:
        oracle.set_threads(default)
    per1, perm_ = t_it1 * k_target, t_itm * k_target
    sample = (f"oracle on the full {prob.n}-DOF matrix: IC(0) single thread {t_fac:.1f} s (alpha={alpha}); "
              f"{iters} FP64 PCG iterations per leg, CG time extrapolated to {k_target} iterations: one thread "
              f"{t_it1:.3f} s/iteration = {per1:.1f} s per right-hand side; {used} threads (SpMV rows and vector "
              f"updates parallel, inner products and triangular solves sequential; host nproc {nproc}, "
              f"affinity {share}) {t_itm:.3f} s/iteration = {perm_:.1f} s per right-hand side; factor time "
              f"excluded from the rate")
    return dict(value=1.0 / perm_, unit="RHS/s", cores=used, kind="oracle", sample=sample,
                single_thread=dict(value=1.0 / per1, unit="RHS/s", cores=1, s_per_iter=t_it1),
                multi_thread=dict(value=1.0 / perm_, unit="RHS/s", cores=used, s_per_iter=t_itm),
                nproc=nproc, factor_s=t_fac)


def errors_vs_oracle(E, sigma, n, rtol, singles, outs, torch):
    """Relative error, on the stored sample of entries, of this run's solutions
    against the FP64 oracle's (tests/golden/q1_100_oracle.json, written by a
    script that calls only the oracle): the single-RHS body-load solves (FP64
    at the oracle's own step count when the GPU stopped within one step of it,
    FP32-L and BF16-L against the oracle's converged x), and load cases 0 and 1
    of the 16-column steps against the oracle's converged solves of those
    columns. None for other workloads."""
    if (E, sigma, rtol) != (100, 2.0, 1e-8):
        return None
    g = load_golden(100)
    if g is None or g["n"] != n:
        return None
    out = {}
    for name, (X, info) in singles.items():
        if name in ("fp64", "fp32_L", "bf16_L"):
            out[name] = golden_rel(g, X, "body", torch, info["iters"] if name == "fp64" else None)
            if name == "fp64":
                out["fp64_iters_minus_oracle"] = info["iters"] - g["cases"]["body"]["iters"]
    for name, (X, infos) in outs.items():
        if name.startswith("multi16") and X.dim() == 2:
            for c in (0, 1):
                out[f"{name}_col{c}"] = golden_rel(g, X[:, c].contiguous(), f"traction{c}", torch)
    out["oracle_iters"] = {k: v["iters"] for k, v in g["cases"].items()}
    out["note"] = ("relative 2-norm error on every 997th entry; FP64 runs at equal step count, reduced-precision "
                   "factors against the oracle's converged FP64 solution")
    return out

def load_golden(E):
    """The stored FP64 oracle solves of the E^3 workload (tests/golden, written
    by a script that calls only the oracle), or None."""
    base = os.path.join(ROOT, "tests", "golden", f"q1_{E}_oracle")
    try:
        g = json.load(open(base + ".json"))
        with np.load(base + "_x.npz") as z:
            g["x"] = {k: z[k] for k in z.files}
    except OSError:
        return None
    return g


def golden_rel(g, x, case, torch, k=None):
    """Relative error of x on the stored sample against the oracle's x after k
    steps (default: the oracle's converged count); None outside the window."""
    c = g["cases"][case]
    k = c["iters"] if k is None else k
    lo, hi = c["x_window_steps"]
    if not lo <= k <= hi:
        return None
    idx = torch.as_tensor(g["sample_index"], dtype=torch.long, device="cuda")
    ref = torch.as_tensor(g["x"][case][k - lo], dtype=torch.float64, device="cuda")
    return float(torch.linalg.norm(x[idx] - ref) / torch.linalg.norm(ref))


def inference_150(ctx, torch, rtol):
    """The 150^3 inference workload (10,260,450 DOF, 820M stored entries,
    sigma 1.5; 16 traction load cases): IC(0) on the GPU (P-time), one FP64
    solve of load case 0 (the comparison: 16 such sequential solves), then one
    16-RHS step with the factor applied in FP32 at the autotuned width, steps
    replayed as a hipGraph; load cases 0 and 1 against the stored FP64 oracle
    solves when present (FP64 at its own step count, the batch's columns
    against the oracle's converged x)."""
    import paper_2412_07127_amd as pkg
    from synth import build_workload
    t = time.perf_counter()
    prob, B = build_workload("q1_150_loads16")
    log(f"inference workload: generated E=150 n={prob.n} nnz={prob.nnz} ({time.perf_counter() - t:.1f} s)")
    A = pkg.CSR.from_numpy(prob.row_ptr, prob.col, prob.val, "cuda")
    M = ctx.matrix(A)
    torch.cuda.synchronize()
    t = time.perf_counter()
    L, finfo = ctx.factor(A)
    torch.cuda.synchronize()
    p_time = time.perf_counter() - t
    P64 = ctx.prec(L, "f64")
    P32 = ctx.prec(L, "f32")
    del L
    Bt = torch.from_numpy(B).cuda()
    b0 = Bt[:, 0].contiguous()
    ctx.solve(M, P64, b0, rtol=rtol, max_iter=5)  # code objects and workspace, untimed
    log("inference workload: one FP64 solve of load case 0 ...")
    torch.cuda.synchronize()
    t = time.perf_counter()
    x0, i0 = ctx.solve(M, P64, b0, rtol=rtol)
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t
    log(f"inference workload: FP64 {t64:.3f} s, {i0[0]['iters']} it; autotune and one 16-RHS step ...")
    tune = ctx.autotune(M, P32, 16)
    ctx.solve(M, P32, Bt, rtol=rtol, use_graph=True, max_iter=5)
    torch.cuda.synchronize()
    t = time.perf_counter()
    X, info = ctx.solve(M, P32, Bt, rtol=rtol, use_graph=True)
    torch.cuda.synchronize()
    t16 = time.perf_counter() - t
    iters = [i["iters"] for i in info]
    out = dict(workload="Q1 elasticity 150^3 elements, sigma=1.5, 16 traction load cases", n=prob.n,
               nnz_A=prob.nnz, p_time_s=round(p_time, 4), alpha=finfo["alpha"],
               fp64_single_s=round(t64, 4), fp64_single_iters=i0[0]["iters"],
               step16_s=round(t16, 4), per_rhs_s=round(t16 / 16, 4), rhs_per_s=round(16 / t16, 4),
               iters_min=min(iters), iters_max=max(iters), true_relres_max=max(i["true_relres"] for i in info),
               block_width=tune["block_width"],
               speedup_vs_16_sequential_fp64=round(16 * t64 / t16, 3))
    g = load_golden(150)
    if g is not None and g["n"] == prob.n:
        out["err_vs_oracle"] = dict(
            fp64_col0=golden_rel(g, x0, "traction0", torch, i0[0]["iters"]),
            fp64_col0_iters_minus_oracle=i0[0]["iters"] - g["cases"]["traction0"]["iters"],
            step16_col0=golden_rel(g, X[:, 0].contiguous(), "traction0", torch),
            step16_col1=golden_rel(g, X[:, 1].contiguous(), "traction1", torch))
    log(f"inference workload: {out}")
    del A, M, P64, P32, Bt, X, x0
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: multi-GPU runs are not part of this build "
              "(the multi-RHS path shards by columns; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2412_07127_amd as pkg
    from synth import WORKLOADS, body_load, node_blocks, q1_elasticity, traction_loads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    E, sigma = args.E, args.sigma
    t0 = time.perf_counter()
    # the named workload of this size, if any (its seeds), else seeds from E
    w = next((v for v in WORKLOADS.values() if (v["E"], v["sigma"]) == (E, sigma)), None)
    prob = q1_elasticity(E, sigma, w["seed_A"] if w else 1000 + E)
    b = body_load(E, 0.1, w["seed_b"] if w else 2000 + E)
    B = traction_loads(E, args.nrhs, WORKLOADS["q1_150_loads16"]["seed_b"])
    log(f"generated E={E}: n={prob.n} nnz={prob.nnz} ({time.perf_counter() - t0:.1f} s)")

    A = pkg.CSR.from_numpy(prob.row_ptr, prob.col, prob.val, "cuda")
    ctx = pkg.Context()
    M = ctx.matrix(A)  # row-group analysis, once (as the solver uses it)
    torch.cuda.synchronize()

    def timed_factor(Am):
        ctx.factor(Am)  # the first call loads code objects
        torch.cuda.synchronize()
        t = time.perf_counter()
        Lx, fi = ctx.factor(Am)
        torch.cuda.synchronize()
        return Lx, fi, time.perf_counter() - t

    # natural order: IC(0) in FP64 (P-time)
    Lf, finfo, p_time = timed_factor(A)
    log(f"factor: {p_time:.3f} s alpha={finfo['alpha']} restarts={finfo['restarts']} levels={finfo['nlevels']}")
    t0 = time.perf_counter()
    P64 = ctx.prec(Lf, "f64")
    P32 = ctx.prec(Lf, "f32")
    torch.cuda.synchronize()
    prec_time = (time.perf_counter() - t0) / 2
    pinfo = P32.info()
    log(f"prec setup {prec_time:.3f} s; schedule {pinfo}")

    # multicolour node order: colouring, P A P^T, IC(0) of the permuted matrix
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm, ncol = ctx.color_order(A, seed=0)
    Ac = ctx.permute(A, perm)
    torch.cuda.synchronize()
    order_time = time.perf_counter() - t0
    Mc = ctx.matrix(Ac)
    Lc, finfo_c, p_time_c = timed_factor(Ac)
    Pc64 = ctx.prec(Lc, "f64")
    Pc32 = ctx.prec(Lc, "f32")
    pinfo_c = Pc32.info()
    log(f"multicolour: {ncol} colours, ordering {order_time:.3f} s, factor {p_time_c:.3f} s, "
        f"alpha={finfo_c['alpha']}, supernode levels {pinfo_c['nsn_levels_L']}")
    # block multicolour order: mesh blocks of 4^3 nodes (the partition is input
    # structure, made outside the timing), coloured first fit in block order
    blk, nblk = node_blocks(E, 4)
    blk_t = torch.from_numpy(blk).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm_b, ncol_b = ctx.block_color_order(A, blk_t, nblk)
    Ab = ctx.permute(A, perm_b)
    torch.cuda.synchronize()
    order_time_b = time.perf_counter() - t0
    Mb = ctx.matrix(Ab)
    Lb, finfo_b, p_time_b = timed_factor(Ab)
    Pb64 = ctx.prec(Lb, "f64")
    Pb32 = ctx.prec(Lb, "f32")
    pinfo_b = Pb64.info()
    log(f"block multicolour: {ncol_b} colours over {nblk} blocks, ordering {order_time_b:.3f} s, factor "
        f"{p_time_b:.3f} s, alpha={finfo_b['alpha']}, supernode levels {pinfo_b['nsn_levels_L']}")
    del Lf, Lc, Lb, blk_t
    perms = {"natural": None, "colour": perm, "block": perm_b}

    bt = torch.from_numpy(b).cuda()
    Bt = torch.from_numpy(B).cuda()
    variants = {}

    if args.kernels_only:
        R = args.nrhs if args.nrhs in (1, 2, 4, 8, 16) else 16
        kt = time_kernels(ctx, M, P32, R, args.kernel_reps, torch)
        # eager steps of the headline solve, so that the step's own launches
        # (the forward solve with the x, r update among them) are counted too:
        # 7 iterations take 8 steps with the update in the forward solve (the
        # first step's forward solve has no update to apply)
        ctx.solve(M, P32, Bt, rtol=0.0, max_iter=7, max_replace=0, block_width=R)
        torch.cuda.synchronize()
        # calibration for counter scaling: one plain device copy of 2^30 bytes each way
        src = torch.empty(2 ** 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"kernels_only": True, "R": R, "ms": {k_: v * 1e3 for k_, v in kt.items()},
                          "copy_bytes_each_way": src.numel() * 8}), flush=True)
        return

    def solve_in(order, Mx, Px, rhs, graph=False):
        """One solve of the original system: in a reordered system the right-
        hand sides are permuted in and the solution back (inside the timing).
        graph: the steps between two convergence polls replay a captured hipGraph."""
        pm = perms[order]
        if pm is None:
            return ctx.solve(Mx, Px, rhs, rtol=args.rtol, use_graph=graph)
        Xp, info = ctx.solve(Mx, Px, ctx.permute_rows(pm, rhs), rtol=args.rtol, use_graph=graph)
        return ctx.permute_rows(pm, Xp, inverse=True), info

    def run_single(order, Mx, Px, name):
        log(f"{name}: one solve ...")
        torch.cuda.synchronize()
        t = time.perf_counter()
        X, info = solve_in(order, Mx, Px, bt)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        i = info[0]
        singles[name] = (X, i)
        variants[name] = dict(cg_s=dt, iters=i["iters"], status=i["status"], true_relres=i["true_relres"],
                              replacements=i["replacements"], ms_per_iter=1e3 * dt / max(1, i["iters"]))
        log(f"{name}: {dt:.3f} s, {i['iters']} it, true relres {i['true_relres']:.2e}, status {i['status']}")
        return X

    singles = {}
    if not args.skip_single:
        x64 = run_single("natural", M, P64, "fp64")
        x32 = run_single("natural", M, P32, "fp32_L")
        Pb = ctx.prec(P64.L, "bf16")
        xb = run_single("natural", M, Pb, "bf16_L")
        xc = run_single("colour", Mc, Pc64, "fp64_multicolour")
        xk = run_single("block", Mb, Pb64, "fp64_block_multicolour")
        nx = torch.linalg.norm(x64).item()
        for name, xx in (("fp32_L", x32), ("bf16_L", xb), ("fp64_multicolour", xc), ("fp64_block_multicolour", xk)):
            variants[name]["rel_diff_vs_fp64_gpu"] = torch.linalg.norm(xx - x64).item() / nx
        del Pb

    tunes = {}

    def multi(order, Mx, Px, name, steps, warmup):
        log(f"{name}: autotune, {warmup} warm-up and {steps} timed steps ...")
        tunes[name] = ctx.autotune(Mx, Px, args.nrhs)  # the width choice is setup, outside the timing
        for _ in range(warmup):
            solve_in(order, Mx, Px, Bt, graph=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = None
        for _ in range(steps):
            X, infos = solve_in(order, Mx, Px, Bt, graph=True)
        torch.cuda.synchronize()
        total = time.perf_counter() - t
        step_s = total / steps
        iters = [i["iters"] for i in infos]
        tr = [i["true_relres"] for i in infos]
        variants[name] = dict(step_s=step_s, per_rhs_s=step_s / args.nrhs, rhs_per_s=args.nrhs * steps / total,
                              iters_max=max(iters), iters_min=min(iters), true_relres_max=max(tr),
                              statuses=sorted(set(i["status"] for i in infos)))
        log(f"{name}: {step_s:.3f} s/step ({args.nrhs} RHS), iters {min(iters)}..{max(iters)}, "
            f"max true relres {max(tr):.2e}")
        outs[name] = (X, infos)
        return total, step_s

    outs = {}

    # multicolour order, 16 load cases (reported beside the headline)
    if not args.skip_single:
        multi("colour", Mc, Pc32, "multi16_fp32_L_multicolour", 1, 0)
        multi("block", Mb, Pb32, "multi16_fp32_L_block_multicolour", 1, 1)
    # headline: natural order, 16 load cases, FP32 factor, FP64 recurrences
    total, step_s = multi("natural", M, P32, "multi16_fp32_L", args.steps, args.warmup)
    value = args.nrhs * args.steps / total
    err = errors_vs_oracle(E, sigma, prob.n, args.rtol, singles, outs, torch)
    if err:
        log(f"error against the stored FP64 oracle solutions: {err}")

    # per-kernel live timing at the headline's launch shape
    R = args.nrhs if args.nrhs in (1, 2, 4, 8, 16) else 16
    # the block multicolour order's kernels first, the headline's last (their
    # dispatches are then the last ones of a profiled run)
    log(f"per-kernel timing at width {R} ...")
    kt_b = time_kernels(ctx, Mb, Pb32, R, args.kernel_reps, torch) if not args.skip_single else None
    kt = time_kernels(ctx, M, P32, R, args.kernel_reps, torch)
    n, nnzA, nnzL = prob.n, prob.nnz, pinfo["nnz"]
    ngroups, gcols = grouped_pattern(prob.row_ptr, prob.col)
    nsnL, nsnU = pinfo["nsupernodes_L"], pinfo["nsupernodes_U"]
    spmv_b, trsvL_b = kernel_bytes(n, nnzA, nnzL, nsnL, R, 4, 8, 4, ngroups, gcols)
    _, trsvU_b = kernel_bytes(n, nnzA, nnzL, nsnU, R, 4, 4, 4, ngroups, gcols)
    trsvU_b += rz_extra_bytes(n, R)
    # the step's forward solve also applies the previous step's x, r update
    # where the library fuses it (the standalone launch is the plain solve)
    fxr = step_fuses_xr(R)
    kernels = {
        "spmv": dict(s=kt["spmv"], bytes=spmv_b, gbs=spmv_b / kt["spmv"] / 1e9),
        "trsv_L": dict(s=kt["trsv_L"], bytes=trsvL_b, gbs=trsvL_b / kt["trsv_L"] / 1e9,
                       bytes_in_step=trsvL_b + (xr_extra_bytes(n, R) if fxr else 0),
                       counters="trsv_L_xr" if fxr else "trsv_L"),
        "trsv_U_rz": dict(s=kt["trsv_U_rz"], bytes=trsvU_b, gbs=trsvU_b / kt["trsv_U_rz"] / 1e9,
                          bytes_in_step=trsvU_b + (rearm_extra_bytes(n, R) if step_fuses_rz(R) else 0),
                          counters="trsv_U_rz_step" if step_fuses_rz(R) else "trsv_U_rz"),
    }
    for v in kernels.values():
        v.setdefault("bytes_in_step", v["bytes"])
    for k_, v in kernels.items():
        log(f"kernel {k_}: {v['s'] * 1e3:.3f} ms, {v['gbs']:.0f} GB/s algorithmic")
    kernels_b = None
    if kt_b is not None:
        _, trsvLb = kernel_bytes(n, nnzA, nnzL, pinfo_b["nsupernodes_L"], R, 4, 8, 4, ngroups, gcols)
        _, trsvUb = kernel_bytes(n, nnzA, nnzL, pinfo_b["nsupernodes_U"], R, 4, 4, 4, ngroups, gcols)
        trsvUb += rz_extra_bytes(n, R)
        # the SpMV of the permuted matrix is costed at the natural pattern's grouping
        kernels_b = {k_: dict(ms=round(kt_b[k_] * 1e3, 4), algorithmic_GBs=round(b_ / kt_b[k_] / 1e9, 1))
                     for k_, b_ in (("spmv", spmv_b), ("trsv_L", trsvLb), ("trsv_U_rz", trsvUb))}
        log(f"block multicolour kernels: {kernels_b}")
    # the same kernels inside the headline's PCG step: 64 eager steps of the
    # headline solve (16 columns, FP32 factor) with events at every phase
    # boundary on the library's stream (graph replay runs the same kernels)
    log("in-step phase timing: 64 eager steps of the headline solve ...")
    ctx.step_timing(True)
    ctx.solve(M, P32, Bt, rtol=0.0, max_iter=64, max_replace=0, block_width=R)
    ph = ctx.step_timing_get()
    ctx.step_timing(False)
    log(f"in-step phases (ms): {ph}")
    in_step = {"spmv": ph["spmv"] * 1e-3, "trsv_L": ph["trsv_L"] * 1e-3, "trsv_U_rz": ph["trsv_U"] * 1e-3}
    for k_ in kernels:
        kernels[k_]["in_step_s"] = in_step[k_]
    # the roofline's kernel: the largest of the three inside the step
    dom = max(kernels, key=lambda k_: kernels[k_]["in_step_s"])
    gbs_in = kernels[dom]["bytes_in_step"] / kernels[dom]["in_step_s"] / 1e9
    roof = dict(bound="hbm", kernel=dom + ("_xr" if dom == "trsv_L" and fxr else ""), achieved=round(gbs_in, 1),
                peak=PEAK_HBM_GBS, unit="GB/s", frac=round(gbs_in / PEAK_HBM_GBS, 4),
                traffic=recorded_traffic(kernels[dom].get("counters", dom)),
                algorithmic_bytes_per_launch=kernels[dom]["bytes_in_step"],
                launch_ms=round(kernels[dom]["in_step_s"] * 1e3, 4),
                timing="mean of 64 in-step launches (events at the step's phase boundaries)")

    # the learned correction at this scale: one forward (inference) and one
    # loss + gradient pass (a training step's work) over nnz(L) edges
    gnn = None
    if not args.skip_single:
        log("learned correction at this size: one forward, one loss + gradient ...")
        from paper_2412_07127_amd import gnn as G
        g = G.GNNGraph(ctx, A, P64)
        theta = G.init_params(0, zero_output=False)
        z = G.rademacher(prob.n, torch.Generator().manual_seed(0))
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        grad = torch.zeros_like(theta)
        Lp = g.forward(theta)
        g.loss_grad(theta, z, loss, grad)
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.forward(theta, out=Lp)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t
        t = time.perf_counter()
        g.loss_grad(theta, z, loss, grad)
        torch.cuda.synchronize()
        t_lg = time.perf_counter() - t
        gnn = dict(params=G.num_params(), edges=int(P64.L.nnz), forward_ms=round(1e3 * t_fwd, 2),
                   loss_grad_ms=round(1e3 * t_lg, 2), loss=float(loss.item()))
        log(f"gnn: forward {1e3 * t_fwd:.1f} ms, loss+gradient {1e3 * t_lg:.1f} ms over {gnn['edges']} edges")
        del g, Lp, grad
        torch.cuda.empty_cache()

    cpu = None
    if not args.skip_cpu:
        k64 = variants.get("fp64", {}).get("iters", 800)
        log("CPU oracle baseline ...")
        cpu = cpu_baseline(prob, b, k64)
        log(f"cpu baseline: {cpu['sample']}")
        cpu = {k_: cpu[k_] for k_ in ("value", "unit", "cores", "kind", "sample", "single_thread", "multi_thread",
                                      "nproc", "factor_s")}

    inf150 = None
    if not args.skip_150:
        inf150 = inference_150(ctx, torch, args.rtol)

    fp64 = variants.get("fp64")
    out = {
        "metric": "PCG time-to-1e-8 residual & HBM GB/s at 3.06M DOF: FP64 vs mixed/multi-RHS",
        "value": round(value, 4),
        "unit": "RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 recurrences + f32 factor",
        "data": "synthetic",
        "config": {
            "workload": (f"Q1 elasticity {E}^3 elements, {n} DOF, nnz {nnzA}, sigma={sigma}; "
                         f"{args.nrhs} load cases per step; IC(0) FP64 on GPU (natural order), factor applied "
                         f"in FP32; rtol {args.rtol} (true residual); steps replayed as a captured hipGraph"),
            "nrhs": args.nrhs, "block_width": R, "n": n, "nnz_A": nnzA, "nnz_L": nnzL, "hip_graph": True,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "p_time_s": round(p_time, 4),
        "p_time_multicolour_s": round(p_time_c, 4),
        "ordering_s": round(order_time, 4),
        "autotune": {k: dict(block_width=v["block_width"], ms_per_rhs_step=round(v["ms_per_rhs"], 4),
                             ms_per_step_by_width={str(w): round(t, 4) for w, t in v["ms_per_step"].items()})
                     for k, v in tunes.items()},
        "p_time_block_multicolour_s": round(p_time_b, 4),
        "ordering_block_multicolour_s": round(order_time_b, 4),
        "block_multicolour": dict(block_nodes=64, blocks=nblk, colours=ncol_b, alpha=finfo_b["alpha"],
                                  supernode_levels=pinfo_b["nsn_levels_L"], kernels=kernels_b),
        "prec_setup_s": round(prec_time, 4),
        "factor": dict(alpha=finfo["alpha"], restarts=finfo["restarts"], row_levels=finfo["nlevels"],
                       supernode_levels_L=pinfo["nsn_levels_L"], supernode_levels_U=pinfo["nsn_levels_U"]),
        "factor_multicolour": dict(alpha=finfo_c["alpha"], restarts=finfo_c["restarts"],
                                   row_levels=finfo_c["nlevels"], supernode_levels_L=pinfo_c["nsn_levels_L"],
                                   supernode_levels_U=pinfo_c["nsn_levels_U"]),
        "variants": variants,
        "gnn_correction": gnn,
        "kernels": {k_: dict(ms_in_step=round(v["in_step_s"] * 1e3, 4),
                             algorithmic_GBs_in_step=round(v["bytes_in_step"] / v["in_step_s"] / 1e9, 1),
                             frac_hbm_peak_in_step=round(v["bytes_in_step"] / v["in_step_s"] / 1e9 / PEAK_HBM_GBS, 4),
                             bytes_in_step=v["bytes_in_step"],
                             ms_standalone=round(v["s"] * 1e3, 4), algorithmic_GBs_standalone=round(v["gbs"], 1),
                             bytes=v["bytes"])
                    for k_, v in kernels.items()},
        "step_fuses_xr": fxr,
        "step_phases_ms": {k_: round(v, 4) for k_, v in ph.items() if k_ != "steps"},
        "err_vs_oracle": err,
        "inference_150": inf150,
    }
    if fp64:
        out["speedup_per_rhs_vs_fp64_single"] = round(fp64["cg_s"] / (step_s / args.nrhs), 3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
