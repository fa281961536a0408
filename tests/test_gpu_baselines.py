"""Table 1's baselines on the GPU PCG loop (Jacobi, no preconditioner)
against the oracle, and the None / Jacobi / IC(0) iteration structure."""

import numpy as np
import pytest
import torch

import oracle
import paper_2412_07127_amd as pkg
from gpu_common import named_matrix, oracle_factor, relerr, rounding_bars, workload_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


def to_gpu(A):
    return pkg.CSR.from_numpy(*A, device="cuda")


@pytest.mark.parametrize("key", ["w:q1_8", "lap7", "q1e4s2.0"])
@pytest.mark.parametrize("kind", ["jacobi", "none"])
def test_baseline_matches_oracle(ctx, key, kind):
    """The GPU solve against the oracle: x after the GPU's k steps, and the
    stopping step, within the bars the iteration's own rounding sensitivity
    gives (gpu_common.rounding_bars: 10x what a one-ulp change of every entry
    of A does to the oracle's x at the same k; twice the shift it causes in
    the stopping step). These baselines take 3-25x the iterations of IC(0)
    (40-800 here), over which rounding differences grow."""
    A_h = named_matrix(key)
    A = to_gpu(A_h)
    P = ctx.prec_simple(A, kind)
    assert P.info()["kind"] == {"jacobi": 1, "none": 2}[kind]
    n = len(A_h[0]) - 1
    b = np.random.default_rng(4).standard_normal(n)
    X, info = ctx.solve(A, P, torch.from_numpy(b).cuda(), rtol=1e-8, max_iter=20 * n)
    ref = oracle.pcg_simple(A_h, b, kind, rtol=1e-8, max_iter=20 * n)
    k = info[0]["iters"]
    assert info[0]["status"] == 0 and ref["status"] == oracle.OK
    assert info[0]["true_relres"] <= 1e-8
    same_k = oracle.pcg_simple(A_h, b, kind, rtol=0.0, max_iter=k, max_replace=0)
    err = relerr(X.cpu().numpy(), same_k["x"])
    xbar, kbar = rounding_bars(A_h, b, k, kind)
    print(f"{key} {kind}: gpu {k} oracle {ref['iters']} iterations (bar {kbar}); equal-k difference {err:.2e} "
          f"(bar {xbar:.2e})")
    assert abs(k - ref["iters"]) <= kbar
    assert err <= xbar


@pytest.mark.parametrize("kind", ["jacobi", "none"])
def test_baseline_multi_rhs_and_graph(ctx, kind):
    """Four columns at once, eager and graph-replayed (bitwise equal), each
    against the oracle at equal k within the column's derived bar."""
    A_h = named_matrix("w:q1_8")
    A = ctx.matrix(to_gpu(A_h))
    P = ctx.prec_simple(A.A, kind)
    n = A.n
    B = np.random.default_rng(8).standard_normal((n, 4))
    Bt = torch.from_numpy(B).cuda()
    X, info = ctx.solve(A, P, Bt, rtol=1e-8, block_width=4, max_iter=20 * n)
    Xg, infog = ctx.solve(A, P, Bt, rtol=1e-8, block_width=4, max_iter=20 * n, use_graph=True)
    assert torch.equal(X, Xg) and info == infog
    rows = []
    for c in range(4):
        k = info[c]["iters"]
        ref = oracle.pcg_simple(A_h, B[:, c], kind, rtol=0.0, max_iter=k, max_replace=0)
        err = relerr(X[:, c].cpu().numpy(), ref["x"])
        xbar, _ = rounding_bars(A_h, B[:, c], k, kind)
        rows.append((k, err, xbar))
    print(f"{kind}: (iterations, equal-k difference, bar) per column {rows}")
    for k, err, xbar in rows:
        assert err <= xbar


def test_table1_iteration_structure(ctx):
    """None > Jacobi > IC(0) in iterations on the 8^3 and 40^3 elasticity workloads."""
    for name in ("q1_8", "q1_40"):
        prob, b = workload_problem(name)
        A = to_gpu((prob.row_ptr, prob.col, prob.val))
        Lf, _ = ctx.factor(A)
        its = {}
        for kind, P in (("none", ctx.prec_simple(A, "none")), ("jacobi", ctx.prec_simple(A, "jacobi")),
                        ("ic0", ctx.prec(Lf, "f64"))):
            _, info = ctx.solve(A, P, torch.from_numpy(b).cuda(), rtol=1e-8, max_iter=20 * prob.n)
            assert info[0]["status"] == 0
            its[kind] = info[0]["iters"]
        print(f"{name}: iterations {its}")
        assert its["none"] > its["jacobi"] > its["ic0"]


def test_factor_calls_reject_baselines(ctx):
    A = to_gpu(named_matrix("lap7"))
    P = ctx.prec_simple(A, "jacobi")
    st = ctx.lib.icpcg_prec_transpose(ctx.h, P.h, None, None, None)
    assert st == pkg._lib.E_INVALID
    st = ctx.lib.icpcg_prec_update_values(ctx.h, P.h, None)
    assert st == pkg._lib.E_INVALID
    # Jacobi needs a positive diagonal
    rp, ci, v = named_matrix("lap7")
    v = v.copy()
    v[rp[3]:rp[4]][ci[rp[3]:rp[4]] == 3] = -1.0
    with pytest.raises(pkg.IcpcgError) as ei:
        ctx.prec_simple(to_gpu((rp, ci, v)), "jacobi")
    assert ei.value.status == pkg._lib.E_INVALID
