"""The stop test of supplementary Algorithm 1 with the true-residual check and
residual replacement, on the GPU against the oracle.

Three cases force the replacement branch deterministically:
  * the worked example of tests/test_oracle.py (A = L = I, b = 3/4, x_0 = 2^53),
    whose every step is exact, so statuses, counts and x must agree bit for bit;
  * the 8^3 workload with a tolerance (1e-14) below what FP64 attains in
    b - A x (about 2e-14): the recurrence converges, the true residual does not,
    and each allowed replacement is used;
  * a two-column block where one column converged and waits for its
    replacement while the last active column stops on a non-finite r^T z, so
    the step ends before its p update: the replaced column must still follow
    its own one-column iteration.
"""

import os

import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import paper_2412_07127_amd as pkg
from gpu_common import relerr
from synth import build_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


@pytest.fixture(scope="module")
def ctx_sep_xr():
    """A context whose PCG steps update x and r in their own pass."""
    torch.cuda.set_device(0)
    old = os.environ.get("ICPCG_FUSE_XR")
    os.environ["ICPCG_FUSE_XR"] = "0"
    try:
        c = pkg.Context()
    finally:
        if old is None:
            del os.environ["ICPCG_FUSE_XR"]
        else:
            os.environ["ICPCG_FUSE_XR"] = old
    return c


def _csr_np(M):
    M = sp.csr_matrix(M)
    M.sort_indices()
    return M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float64)


@pytest.mark.parametrize("n", [1, 2])
@pytest.mark.parametrize("mr", [0, 1, 3])
def test_replacement_worked_example(ctx, n, mr):
    I = _csr_np(sp.identity(n))
    U = oracle.transpose(*I)
    b = np.full(n, 0.75)
    x0 = np.full(n, 2.0 ** 53)
    ref = oracle.pcg(I, I, U, b, x0=x0, rtol=1e-8, max_replace=mr, max_iter=50)
    A = pkg.CSR.from_numpy(*I)
    P = ctx.prec(A, "f64")
    # the same case in both columns of a two-column block, and alone
    for R in (1, 2):
        B = torch.from_numpy(np.repeat(b[:, None], R, 1) if R > 1 else b).cuda()
        X0 = torch.from_numpy(np.repeat(x0[:, None], R, 1) if R > 1 else x0).cuda()
        X, info = ctx.solve(A, P, B, X0=X0, rtol=1e-8, max_replace=mr, max_iter=50, block_width=R)
        Xh = X.cpu().numpy().reshape(n, R)
        for c in range(R):
            assert info[c]["status"] == ref["status"]
            assert info[c]["iters"] == ref["iters"] and info[c]["replacements"] == ref["replacements"]
            assert np.array_equal(Xh[:, c], ref["x"])
            assert info[c]["true_relres"] == ref["true_relres"]
    assert ref["replacements"] == min(mr, 1)


@pytest.fixture(scope="module")
def q8():
    prob, b = build_workload("q1_8")
    Ah = (prob.row_ptr, prob.col, prob.val)
    st, L, alpha, _, _ = oracle.ic0_shifted(*Ah)
    return Ah, L, oracle.transpose(*L), b


@pytest.mark.parametrize("mr", [0, 1])
def test_replacement_below_attainable_accuracy(ctx, q8, mr):
    Ah, L, U, b = q8
    ref = oracle.pcg(Ah, L, U, b, rtol=1e-14, max_replace=mr, max_iter=2000)
    P = ctx.prec(pkg.CSR.from_numpy(*L), "f64")
    X, info = ctx.solve(pkg.CSR.from_numpy(*Ah), P, torch.from_numpy(b).cuda(), rtol=1e-14, max_replace=mr,
                        max_iter=2000)
    i = info[0]
    e = relerr(X.cpu().numpy(), ref["x"])
    print(f"max_replace {mr}: gpu {i['iters']} it, {i['replacements']} repl, true relres {i['true_relres']:.2e}; "
          f"oracle {ref['iters']} it, {ref['replacements']} repl, {ref['true_relres']:.2e}; |dx|/|x| {e:.1e}")
    assert ref["status"] == oracle.TRUE_RESIDUAL and ref["replacements"] == mr
    assert i["status"] == ref["status"] and i["replacements"] == ref["replacements"]
    assert abs(i["iters"] - ref["iters"]) <= 1
    assert e <= 1e-10


def _breakdown_block(L8, A8, dtype):
    """blockdiag(A_8, T) with T the 96 x 96 second-difference matrix, and the
    factor blockdiag(L_8, D) with D = I except a tiny pivot t at row 70 (FP64:
    1e-200; FP32 / bfloat16: 1e-30, representable in both). Column 0 is the 8^3
    workload's load (zero on T's rows), column 1 the unit vector at T's first
    row: plain CG on T from e_1 reaches row k at step k + 1, so column 1's
    z = P^-1 r overflows at step 71, r^T z is infinite and the column stops
    there, after column 0 has converged (44-57 steps) and waits for its
    replacement."""
    n1 = A8[0].shape[0] - 1
    m, k = 96, 70
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    A = _csr_np(sp.block_diag([sp.csr_matrix((A8[2], A8[1], A8[0])), T]))
    d = np.ones(m)
    d[k] = 1e-200 if dtype == "f64" else 1e-30
    L = _csr_np(sp.block_diag([sp.csr_matrix((L8[2], L8[1], L8[0])), sp.diags(d)]))
    return A, L, n1


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_replacement_after_last_column_breaks_down(ctx, ctx_sep_xr, q8, dtype):
    Ah8, L8, _, b8 = q8
    A, L, n1 = _breakdown_block(L8, Ah8, dtype)
    U = oracle.transpose(*L)
    n = A[0].shape[0] - 1
    B = np.zeros((n, 2))
    B[:n1, 0] = b8
    B[n1, 1] = 1.0
    prec = {"f64": 0, "f32": 1, "bf16": 2}[dtype]
    refs = [oracle.pcg(A, L, U, np.ascontiguousarray(B[:, c]), rtol=1e-14, max_replace=1, max_iter=2000, prec=prec)
            for c in range(2)]
    # the designed order of events, on the oracle
    assert refs[0]["status"] == oracle.TRUE_RESIDUAL and refs[0]["replacements"] == 1
    assert refs[1]["status"] == oracle.NONFINITE and refs[1]["iters"] == 70
    P = ctx.prec(pkg.CSR.from_numpy(*L), dtype)
    X, info = ctx.solve(pkg.CSR.from_numpy(*A), P, torch.from_numpy(B).cuda(), rtol=1e-14, max_replace=1,
                        max_iter=2000, block_width=2)
    Xh = X.cpu().numpy()
    e = relerr(Xh[:, 0], refs[0]["x"])
    print(f"{dtype}: column 0 gpu {info[0]['iters']} it / {info[0]['replacements']} repl / status "
          f"{info[0]['status']}, oracle {refs[0]['iters']} / {refs[0]['replacements']}; |dx|/|x| {e:.1e}; "
          f"column 1 gpu {info[1]['iters']} it status {info[1]['status']}")
    assert info[1]["status"] == pkg._lib.E_NONFINITE and info[1]["iters"] == refs[1]["iters"]
    assert info[0]["status"] == refs[0]["status"] and info[0]["replacements"] == 1
    # FP64: the oracle's arithmetic up to summation order (iterations +-1);
    # FP32 / bfloat16 factor: the preconditioner rounds differently inside a row
    # on the two sides, which moves the step at which a 1e-14 recurrence
    # tolerance is crossed by up to two
    assert abs(info[0]["iters"] - refs[0]["iters"]) <= (1 if dtype == "f64" else 2)
    assert e <= 1e-10
    if dtype != "f64":
        # the same block with the x, r update in its own pass instead of the
        # forward solve: same statuses and counts; where both stop at the same
        # step the iterates are the same bits (||r||^2 alone is summed in
        # another order, which may move a 1e-14 stop by one step)
        X2, info2 = ctx_sep_xr.solve(pkg.CSR.from_numpy(*A), ctx_sep_xr.prec(pkg.CSR.from_numpy(*L), dtype),
                                     torch.from_numpy(B).cuda(), rtol=1e-14, max_replace=1, max_iter=2000,
                                     block_width=2)
        for c in range(2):
            assert info2[c]["status"] == info[c]["status"] and info2[c]["replacements"] == info[c]["replacements"]
            assert abs(info2[c]["iters"] - info[c]["iters"]) <= 1
            if info2[c]["iters"] == info[c]["iters"]:
                assert torch.equal(X2[:, c], X[:, c]), c
