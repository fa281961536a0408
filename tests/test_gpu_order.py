"""Multicolour ordering on the GPU (colouring, P A P^T, row permutation)
against the oracle, and IC(0)-PCG on the reordered system."""

import time

import numpy as np
import pytest
import torch

import oracle
from oracle import order as OO
import paper_2412_07127_amd as pkg
from gpu_common import named_matrix, relerr, workload_problem
from synth import node_blocks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


def to_gpu(A):
    return pkg.CSR.from_numpy(*A, device="cuda")


@pytest.mark.parametrize("key,seed", [("w:q1_8", 0), ("q1e4s2.0", 5), ("lap7", 1), ("tridiag", 3)])
def test_colour_order_bit_exact(ctx, key, seed):
    A_h = named_matrix(key)
    perm, nc = ctx.color_order(to_gpu(A_h), seed=seed)
    ref, col, nc_ref = OO.color_order(A_h, seed=seed)
    print(f"{key}: {nc} colours")
    assert nc == nc_ref
    assert np.array_equal(perm.cpu().numpy(), ref)


@pytest.mark.parametrize("key", ["w:q1_8", "q1e4s2.0", "lap7"])
def test_permute_matrix_bit_exact(ctx, key):
    A_h = named_matrix(key)
    ref_perm, _, _ = OO.color_order(A_h, seed=2)
    B = ctx.permute(to_gpu(A_h), torch.from_numpy(ref_perm).cuda())
    rp, ci, v = OO.permute(A_h, ref_perm)
    assert np.array_equal(B.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(B.col.cpu().numpy(), ci)
    assert np.array_equal(B.val.cpu().numpy(), v)


def test_permute_rows_round_trip_and_bad_perm(ctx):
    n = 1000
    perm = torch.from_numpy(np.random.default_rng(3).permutation(n).astype(np.int32)).cuda()
    for R in (1, 4):
        X = torch.randn(n, R, dtype=torch.float64, device="cuda") if R > 1 else \
            torch.randn(n, dtype=torch.float64, device="cuda")
        Y = ctx.permute_rows(perm, X)
        pl = perm.long()
        assert torch.equal(Y, X[pl])
        assert torch.equal(ctx.permute_rows(perm, Y, inverse=True), X)
    A_h = named_matrix("lap7")
    bad = torch.zeros(len(A_h[0]) - 1, dtype=torch.int32, device="cuda")
    with pytest.raises(pkg.IcpcgError) as ei:
        ctx.permute(to_gpu(A_h), bad)
    assert ei.value.status == pkg._lib.E_INVALID


def test_reordered_factor_and_solve_match_oracle(ctx):
    prob, b = workload_problem("q1_8")
    A_h = (prob.row_ptr, prob.col, prob.val)
    perm, nc = ctx.color_order(to_gpu(A_h), seed=0)
    Ap = ctx.permute(to_gpu(A_h), perm)
    Lg, finfo = ctx.factor(Ap)
    pn = perm.cpu().numpy()
    Ap_h = OO.permute(A_h, pn)
    st, L, alpha, _, _ = oracle.ic0_shifted(*Ap_h)
    assert finfo["alpha"] == alpha
    assert relerr(Lg.val.cpu().numpy(), L[2]) <= 1e-12
    P = ctx.prec(Lg, "f64")
    info = P.info()
    print(f"{nc} colours: row levels {info['nlevels_L']} (natural order: 159)")
    assert info["nlevels_L"] <= 3 * nc
    bp = ctx.permute_rows(perm, torch.from_numpy(b).cuda())
    Xp, inf = ctx.solve(Ap, P, bp, rtol=1e-8)
    U = oracle.transpose(*L)
    ref = oracle.pcg(Ap_h, L, U, b[pn], rtol=1e-8)
    k = inf[0]["iters"]
    assert inf[0]["status"] == 0 and abs(k - ref["iters"]) <= 1
    same_k = oracle.pcg(Ap_h, L, U, b[pn], rtol=0.0, max_iter=k, max_replace=0)
    assert relerr(Xp.cpu().numpy(), same_k["x"]) <= 1e-10
    x = ctx.permute_rows(perm, Xp, inverse=True).cpu().numpy()
    assert relerr(oracle.spmv(*A_h, x), b) <= 1e-8


@pytest.mark.parametrize("key,E,bs", [("w:q1_8", 8, 2), ("w:q1_8", 8, 4), ("q1e4s2.0", 4, 2), ("w:q1_40", 40, 4)])
def test_block_colour_order_bit_exact(ctx, key, E, bs):
    A_h = named_matrix(key)
    blk, nblk = node_blocks(E, bs)
    perm, nc = ctx.block_color_order(to_gpu(A_h), torch.from_numpy(blk), nblk)
    ref, col, nc_ref = OO.block_color_order(A_h, blk, nblk=nblk)
    print(f"{key} blocks of {bs}^3 nodes: {nblk} blocks, {nc} colours")
    assert nc == nc_ref
    assert np.array_equal(perm.cpu().numpy(), ref)


def test_block_colour_order_random_partition_and_bad_ids(ctx):
    A_h = named_matrix("lap7")
    n = len(A_h[0]) - 1
    blk = np.random.default_rng(4).integers(0, 17, n).astype(np.int32)
    nblk = 20  # blocks 17..19 are empty
    perm, nc = ctx.block_color_order(to_gpu(A_h), torch.from_numpy(blk), nblk)
    ref, _, nc_ref = OO.block_color_order(A_h, blk, nblk=nblk)
    assert nc == nc_ref and np.array_equal(perm.cpu().numpy(), ref)
    bad = blk.copy()
    bad[7] = nblk
    with pytest.raises(pkg.IcpcgError) as ei:
        ctx.block_color_order(to_gpu(A_h), torch.from_numpy(bad), nblk)
    assert ei.value.status == pkg._lib.E_INVALID


def test_block_reordered_factor_and_solve_match_oracle(ctx):
    prob, b = workload_problem("q1_8")
    A_h = (prob.row_ptr, prob.col, prob.val)
    blk, nblk = node_blocks(8, 2)
    perm, nc = ctx.block_color_order(to_gpu(A_h), torch.from_numpy(blk), nblk)
    Ap = ctx.permute(to_gpu(A_h), perm)
    Lg, finfo = ctx.factor(Ap)
    pn = perm.cpu().numpy()
    Ap_h = OO.permute(A_h, pn)
    st, L, alpha, _, _ = oracle.ic0_shifted(*Ap_h)
    assert finfo["alpha"] == alpha
    assert relerr(Lg.val.cpu().numpy(), L[2]) <= 1e-12
    P = ctx.prec(Lg, "f64")
    print(f"{nc} colours: supernode levels {P.info()['nsn_levels_L']}")
    bp = ctx.permute_rows(perm, torch.from_numpy(b).cuda())
    Xp, inf = ctx.solve(Ap, P, bp, rtol=1e-8)
    U = oracle.transpose(*L)
    ref = oracle.pcg(Ap_h, L, U, b[pn], rtol=1e-8)
    k = inf[0]["iters"]
    assert inf[0]["status"] == 0 and abs(k - ref["iters"]) <= 1
    same_k = oracle.pcg(Ap_h, L, U, b[pn], rtol=0.0, max_iter=k, max_replace=0)
    assert relerr(Xp.cpu().numpy(), same_k["x"]) <= 1e-10
    x = ctx.permute_rows(perm, Xp, inverse=True).cpu().numpy()
    assert relerr(oracle.spmv(*A_h, x), b) <= 1e-8


def test_reordering_iterations_and_time(ctx):
    """Natural vs multicolour vs block multicolour (4^3-node blocks) order on
    the 40^3 workload: factor levels, iterations and solve time (FP64, one
    right-hand side), as measured."""
    prob, b = workload_problem("q1_40")
    A = to_gpu((prob.row_ptr, prob.col, prob.val))
    bt = torch.from_numpy(b).cuda()
    rows = {}
    for name in ("natural", "coloured", "block4"):
        if name == "coloured":
            perm, nc = ctx.color_order(A, seed=0)
            Am = ctx.permute(A, perm)
            rhs = ctx.permute_rows(perm, bt)
        elif name == "block4":
            blk, nblk = node_blocks(40, 4)
            perm, nc = ctx.block_color_order(A, torch.from_numpy(blk), nblk)
            Am = ctx.permute(A, perm)
            rhs = ctx.permute_rows(perm, bt)
        else:
            Am, rhs, nc = A, bt, 0
        M = ctx.matrix(Am)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Lf, _ = ctx.factor(Am)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        P = ctx.prec(Lf, "f64")
        ctx.solve(M, P, rhs, rtol=1e-8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = ctx.solve(M, P, rhs, rtol=1e-8)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        assert info[0]["status"] == 0 and info[0]["true_relres"] <= 1e-8
        pi = P.info()
        rows[name] = dict(colours=nc, levels=pi["nlevels_L"], sn_levels=pi["nsn_levels_L"],
                          iters=info[0]["iters"], p_time=round(tp, 4), cg_time=round(tc, 4),
                          ms_per_iter=round(1e3 * tc / info[0]["iters"], 3))
    print("natural vs multicolour vs block multicolour:", rows)
    assert rows["coloured"]["sn_levels"] < rows["natural"]["sn_levels"]
    assert rows["block4"]["sn_levels"] < rows["natural"]["sn_levels"]
