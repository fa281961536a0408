"""Captured PCG steps (hipGraph replay) against eager launches, and the block
width autotuner, through the C ABI; columns checked against the FP64 oracle."""

import numpy as np
import pytest
import torch

import oracle
import paper_2412_07127_amd as pkg
from gpu_common import named_matrix, oracle_factor, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


def to_gpu(A):
    return pkg.CSR.from_numpy(*A, device="cuda")


def rhs(n, R, seed):
    B = np.random.default_rng(seed).standard_normal((n, R)) if R > 1 else \
        np.random.default_rng(seed).standard_normal(n)
    return torch.from_numpy(B).cuda()


def same(a, b):
    Xa, ia = a
    Xb, ib = b
    assert torch.equal(Xa, Xb)
    assert ia == ib


@pytest.mark.parametrize("key,dt,R,width", [("w:q1_8", "f64", 1, 1), ("lap7", "f32", 4, 4),
                                            ("q1e4s1.5", "bf16", 16, 16), ("w:q1_8", "f64", 5, 4)])
def test_graph_replay_matches_eager(ctx, key, dt, R, width):
    A_h, L, _, _ = oracle_factor(key)
    A = ctx.matrix(to_gpu(A_h))
    P = ctx.prec(to_gpu(L), dt)
    B = rhs(A.n, R, 5)
    kw = dict(rtol=1e-8, block_width=width, check_every=3)
    eager = ctx.solve(A, P, B, **kw)
    assert all(i["status"] == 0 for i in eager[1])
    # other launches between the replays: a product, and a solve whose graph
    # has other operands (the context then captures again)
    other = ctx.prec(to_gpu(L), "f64" if dt != "f64" else "f32")
    for rep in range(3):
        g = ctx.solve(A, P, B, use_graph=True, **kw)
        torch.cuda.synchronize()
        same(g, eager)
        A.spmv(torch.ones(A.n, dtype=torch.float64, device="cuda"))
        if rep == 1:
            ctx.solve(A, other, B, use_graph=True, **kw)
        torch.cuda.synchronize()


def test_graph_replay_stops_like_eager(ctx):
    A_h, L, _, _ = oracle_factor("w:q1_8")
    A = ctx.matrix(to_gpu(A_h))
    P = ctx.prec(to_gpu(L), "f64")
    B = rhs(A.n, 2, 9)
    kw = dict(rtol=1e-12, max_iter=7, max_replace=0, block_width=2, check_every=4)
    eager = ctx.solve(A, P, B, **kw)
    graph = ctx.solve(A, P, B, use_graph=True, **kw)
    same(graph, eager)
    assert [i["iters"] for i in graph[1]] == [7, 7]
    assert all(i["status"] == pkg._lib.E_MAXITER for i in graph[1])
    Bh = B.cpu().numpy()
    for c in range(2):
        ref = oracle.pcg(A_h, L, oracle.transpose(*L), Bh[:, c], rtol=0.0, max_iter=7, max_replace=0)
        assert relerr(graph[0][:, c].cpu().numpy(), ref["x"]) <= 1e-10


def test_autotune_and_solve(ctx):
    A_h, L, U, _ = oracle_factor("w:q1_8")
    A = ctx.matrix(to_gpu(A_h))
    P = ctx.prec(to_gpu(L), "f64")
    info = ctx.autotune(A, P, 12)
    print("autotune:", info)
    assert info["block_width"] in (1, 2, 4, 8, 16)
    assert sorted(info["ms_per_step"]) == [1, 2, 4, 8, 16]
    assert all(v > 0 for v in info["ms_per_step"].values())
    w = info["block_width"]
    assert info["ms_per_rhs"] == pytest.approx(info["ms_per_step"][w] * (-(-12 // w)) / 12)
    assert ctx.autotune(A, P, 12)["block_width"] == w  # cached
    small = ctx.autotune(A, P, 3)
    assert sorted(small["ms_per_step"]) == [1, 2, 4]
    B = rhs(A.n, 12, 21)
    X, infos = ctx.solve(A, P, B, rtol=1e-8)  # block_width 0: the tuned width
    Bh, Xh = B.cpu().numpy(), X.cpu().numpy()
    for c in range(12):
        k = infos[c]["iters"]
        ref = oracle.pcg(A_h, L, U, Bh[:, c], rtol=1e-8)
        assert infos[c]["status"] == 0 and abs(k - ref["iters"]) <= 1
        same_k = oracle.pcg(A_h, L, U, Bh[:, c], rtol=0.0, max_iter=k, max_replace=0)
        assert relerr(Xh[:, c], same_k["x"]) <= 1e-10


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_step_timing_phases(ctx, dt):
    """Per-phase timing of eager steps: every phase of each recorded step is
    measured (a positive mean; the x, r update phase is empty where the forward
    solve applies the update), the record stops at 64 steps, timed steps give
    the same result as untimed ones (the marks are events only), and
    graph-replayed steps are not recorded. With the update in the forward
    solve, the last iteration's stop test runs in the step after it: 41 steps
    for 40 iterations, queued in batches of 8 (the queued steps after the stop
    return at once and are recorded too)."""
    A_h = named_matrix("w:q1_40")
    _, L, _, _ = oracle_factor("w:q1_40")
    A = ctx.matrix(to_gpu(A_h))
    P = ctx.prec(to_gpu(L), dt)
    B = rhs(A.n, 16, 5)
    ref = ctx.solve(A, P, B, rtol=0.0, max_iter=40, max_replace=0, block_width=16)
    ctx.step_timing(True)
    try:
        got = ctx.solve(A, P, B, rtol=0.0, max_iter=40, max_replace=0, block_width=16)
        t = ctx.step_timing_get()
        print(dt, t)
        same(got, ref)
        fused_xr = dt != "f64"
        assert t["steps"] == (48 if fused_xr else 40)
        for k in ctx.STEP_PHASES:
            if fused_xr and k == "update_xr":
                assert t[k] >= 0.0
            else:
                assert t[k] > 0.0, k
        # a second, longer solve fills the record to its cap
        ctx.step_timing(True)
        ctx.solve(A, P, B, rtol=0.0, max_iter=100, max_replace=0, block_width=16)
        assert ctx.step_timing_get()["steps"] == 64
        # graph replay: nothing recorded
        ctx.step_timing(True)
        ctx.solve(A, P, B, rtol=0.0, max_iter=40, max_replace=0, block_width=16, use_graph=True)
        assert ctx.step_timing_get()["steps"] == 0
    finally:
        ctx.step_timing(False)
