"""Fill-in dropout (Eq. 10) on the GPU against the oracle, PCG with the
thinned factor, and the shape of the paper's Table 3 on a synthetic matrix."""

import numpy as np
import pytest
import torch

import oracle
import paper_2412_07127_amd as pkg
from paper_2412_07127_amd import gnn as GG
from gpu_common import oracle_factor, random_lower_pattern, relerr, workload_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


def to_gpu(A):
    return pkg.CSR.from_numpy(*A, device="cuda")


@pytest.mark.parametrize("key", ["w:q1_8", "q1e4s2.0", "random"])
@pytest.mark.parametrize("eps", [0.0, 1e-3, 1e-2, 0.1])
def test_dropout_bit_exact(ctx, key, eps):
    if key == "random":
        L = random_lower_pattern(700, 0.05, 9)
        rows = np.repeat(np.arange(700), np.diff(L[0]))
        off = L[1] != rows
        L[2][off & (np.random.default_rng(1).random(L[2].size) < 0.05)] = 0.0  # exact zeros off the diagonal
    else:
        L = oracle_factor(key)[1]
    D = ctx.dropout(to_gpu(L), eps)
    rp, ci, v = oracle.dropout(L, eps)
    assert np.array_equal(D.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(D.col.cpu().numpy(), ci)
    assert np.array_equal(D.val.cpu().numpy().view(np.uint64), v.view(np.uint64))


def test_pcg_with_thinned_factor_matches_oracle(ctx):
    A_h, L, U, _ = oracle_factor("w:q1_8")
    Ld = oracle.dropout(L, 0.05 * np.abs(L[2]).max())
    print(f"kept {len(Ld[1])} of {len(L[1])} entries")
    assert len(Ld[1]) < len(L[1])
    Ud = oracle.transpose(*Ld)
    b = workload_problem("q1_8")[1]
    P = ctx.prec(ctx.dropout(to_gpu(L), 0.05 * np.abs(L[2]).max()), "f64")
    X, info = ctx.solve(to_gpu(A_h), P, torch.from_numpy(b).cuda(), rtol=1e-8)
    ref = oracle.pcg(A_h, Ld, Ud, b, rtol=1e-8)
    k = info[0]["iters"]
    assert info[0]["status"] == 0 and abs(k - ref["iters"]) <= 1
    same_k = oracle.pcg(A_h, Ld, Ud, b, rtol=0.0, max_iter=k, max_replace=0)
    assert relerr(X.cpu().numpy(), same_k["x"]) <= 1e-10


def test_table3_shape(ctx):
    """nnz, iterations and triangular-solve time against the threshold, with
    eps in the network's scaled units (|l| <= eps sqrt(s), s the spread of
    tril(A)), on the 40^3 workload."""
    prob, b = workload_problem("q1_40")
    A = to_gpu((prob.row_ptr, prob.col, prob.val))
    Lf, _ = ctx.factor(A)
    P0 = ctx.prec(Lf, "f64")
    s = GG.GNNGraph(ctx, A, P0).inputs()[2]
    bt = torch.from_numpy(b).cuda()
    rows = []
    for eps in (0.0, 0.001, 0.01, 0.02, 0.05):
        Ld = ctx.dropout(Lf, eps * np.sqrt(s))
        P = ctx.prec(Ld, "f64")
        _, info = ctx.solve(A, P, bt, rtol=1e-8)
        assert info[0]["status"] == 0
        R = torch.randn(prob.n, dtype=torch.float64, device="cuda")
        for _ in range(3):
            P.apply(R)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            P.apply(R)
        e1.record()
        torch.cuda.synchronize()
        rows.append((eps, Ld.nnz, info[0]["iters"], e0.elapsed_time(e1) / 10))
    print("eps, nnz(L), iterations, L^-T L^-1 apply ms:")
    for r in rows:
        print(f"  {r[0]:<6} {r[1]:>10} {r[2]:>5} {r[3]:.3f}")
    nnz = [r[1] for r in rows]
    assert all(a >= b_ for a, b_ in zip(nnz, nnz[1:]))
