"""The mixed-precision, multi-column arithmetic the headline runs, against the
oracle column by column (factor applied in FP32 or bfloat16 with FP32
accumulation, SpMV and recurrences in FP64).

The oracle emulates the same arithmetic in float (oracle.apply_f32,
oracle.pcg(prec=1|2)); the two sides round differently inside a row (the
order of the additions follows the lane layout on the GPU), so reduced
precision is compared within bounds, and every converged column is also
measured against the FP64 oracle solution.
"""

import os

import numpy as np
import pytest
import torch

import oracle
import paper_2412_07127_amd as pkg
from gpu_common import oracle_factor, relerr, stop_agrees, workload_problem
from synth import traction_loads

pytestmark = pytest.mark.gpu

PREC = {"f32": 1, "bf16": 2}
# apply parity bars (relative, per column): the factor's values are the same
# float / bfloat16 numbers on both sides and every operation is one float
# rounding, so the two results differ by the rounding of reordered sums (about
# 40 terms per row) propagated through the two solves
APPLY_TOL = {"f32": 1e-5, "bf16": 1e-4}


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


@pytest.fixture(scope="module")
def ctx_unfused():
    """A context whose backward solves never form r^T z (a separate pass does)."""
    torch.cuda.set_device(0)
    old = os.environ.get("ICPCG_FUSE_RZ")
    os.environ["ICPCG_FUSE_RZ"] = "0"
    try:
        c = pkg.Context()
    finally:
        if old is None:
            del os.environ["ICPCG_FUSE_RZ"]
        else:
            os.environ["ICPCG_FUSE_RZ"] = old
    return c


@pytest.fixture(scope="module")
def ctx_sep_xr():
    """A context whose PCG steps update x and r in their own pass (the forward
    solve does not apply them)."""
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


def to_gpu(A):
    return pkg.CSR.from_numpy(*A, device="cuda")


@pytest.mark.parametrize("key,R", [("w:q1_8", 2), ("w:q1_8", 4), ("w:q1_8", 8), ("w:q1_8", 16), ("w:q1_40", 16)])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_apply_block_reduced_precision(ctx, key, R, dt):
    _, L, U, _ = oracle_factor(key)
    n = L[0].shape[0] - 1
    P = ctx.prec(to_gpu(L), dt)
    Rh = np.random.default_rng(100 + R).standard_normal((n, R))
    _, Z = P.apply(torch.from_numpy(Rh).cuda())
    Zh = Z.double().cpu().numpy()
    cols = range(R) if n < 10000 else (0, 5, 10, 15)
    worst = 0.0
    for c in cols:
        z_emul = oracle.apply_f32(L, U, Rh[:, c], PREC[dt])
        worst = max(worst, relerr(Zh[:, c], z_emul))
    print(f"{key} R={R} {dt}: worst column |z - z_emul|/|z_emul| = {worst:.2e}")
    assert worst <= APPLY_TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("R", [1, 2, 16])
@pytest.mark.parametrize("fused", [True, False])
def test_apply_rz_matches_oracle(ctx, ctx_unfused, dt, R, fused):
    """r^T z of the step's preconditioner solve (formed by the backward solve
    for FP32 / BF16 factors on several columns) against the oracle's inner
    product of the same r with its own z."""
    c = ctx if fused else ctx_unfused
    _, L, U, _ = oracle_factor("w:q1_8")
    n = L[0].shape[0] - 1
    P = c.prec(to_gpu(L), dt)
    Rh = np.random.default_rng(7 + R).standard_normal((n, R))
    Y, Z, rz = P.apply_rz(torch.from_numpy(Rh).cuda())
    Zh = Z.double().cpu().numpy().reshape(n, R)
    rzh = rz.cpu().numpy()
    for k in range(R):
        if dt == "f64":
            _, z = oracle.apply(L, U, Rh[:, k])
            tol = 1e-12
        else:
            z = oracle.apply_f32(L, U, Rh[:, k], PREC[dt])
            tol = APPLY_TOL[dt]
        # the GPU's r^T z is its own z's inner product with r (to FP64 rounding
        # of a reordered sum) ...
        assert abs(rzh[k] - oracle.dot(Rh[:, k], Zh[:, k])) <= 1e-13 * abs(rzh[k])
        # ... and the oracle's within the apply's bound (r^T z is positive:
        # z = P^-1 r with P SPD)
        assert abs(rzh[k] - oracle.dot(Rh[:, k], z)) <= tol * abs(rzh[k])


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("R", [1, 4, 16])
def test_trsv_rz_is_apply_rz_backward_half(ctx, dt, R):
    """The backward solve with r^T z alone (the launch a PCG step makes) gives
    the Z and r^T z of apply_rz bit for bit when fed apply_rz's Y."""
    _, L, U, _ = oracle_factor("w:q1_40")
    n = L[0].shape[0] - 1
    P = ctx.prec(to_gpu(L), dt)
    Rt = torch.from_numpy(np.random.default_rng(40 + R).standard_normal((n, R) if R > 1 else n)).cuda()
    Y, Z, rz = P.apply_rz(Rt)
    Z2, rz2 = P.trsv_rz(Y, Rt)
    assert torch.equal(Z, Z2) and torch.equal(rz, rz2)


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_apply_rz_fused_equals_unfused(ctx, ctx_unfused, dt):
    """The fused form changes only where r^T z is summed: Z is bit-identical."""
    _, L, U, _ = oracle_factor("w:q1_40")
    n = L[0].shape[0] - 1
    Rt = torch.from_numpy(np.random.default_rng(3).standard_normal((n, 16))).cuda()
    outs = []
    for c in (ctx, ctx_unfused):
        P = c.prec(to_gpu(L), dt)
        outs.append(P.apply_rz(Rt))
    assert torch.equal(outs[0][1], outs[1][1])
    d = (outs[0][2] - outs[1][2]).abs() / outs[1][2].abs()
    assert float(d.max()) <= 1e-13


_ORC = {}


def _oracle_pcg(key, k, prec, **kw):
    """Oracle PCG of load case k of the 16 traction columns (cached per run)."""
    tag = (key, k, prec, tuple(sorted(kw.items())))
    if tag not in _ORC:
        prob, _ = workload_problem(key)
        Ah = (prob.row_ptr, prob.col, prob.val)
        _, L, U, _ = oracle_factor(f"w:{key}")
        B = traction_loads(_E[key], 16, 2000 + _E[key])
        _ORC[tag] = oracle.pcg(Ah, L, U, np.ascontiguousarray(B[:, k]), prec=prec, **kw)
    return _ORC[tag]


_E = {"q1_8": 8, "q1_40": 40}


def _pcg_columns(ctx, key, E, dt, cols, rtol=1e-8):
    prob, _ = workload_problem(key)
    Ah = (prob.row_ptr, prob.col, prob.val)
    _, L, U, _ = oracle_factor(f"w:{key}")
    B = traction_loads(E, 16, 2000 + E)
    P = ctx.prec(to_gpu(L), dt)
    A = to_gpu(Ah)
    X, info = ctx.solve(A, P, torch.from_numpy(B).cuda(), rtol=rtol, block_width=16)
    return Ah, L, U, B, P, A, X.cpu().numpy(), info


@pytest.mark.parametrize("key,E", [("q1_8", 8), ("q1_40", 40)])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
@pytest.mark.parametrize("fused", [True, False])
def test_multi_rhs_reduced_precision_pcg(ctx, ctx_unfused, key, E, dt, fused):
    """16 load cases at once with the factor in FP32 / BF16 (the headline's
    arithmetic, at sizes the oracle finishes in seconds). Per column:
      * the oracle's float-emulated PCG on the same column stops at an agreeing
        step (within one, or anywhere on the plateau where the oracle's own
        recurrence residual stays within 2 rtol: the two sides round the
        preconditioner's sums in different orders);
      * after 3 steps the iterates agree to the apply's bound times the growth of
        three steps;
      * the converged x is within 1e-5 of the FP64 oracle's converged x, and the
        true residual is below the tolerance."""
    c = ctx if fused else ctx_unfused
    Ah, L, U, B, P, A, Xh, info = _pcg_columns(c, key, E, dt, None)
    cols = range(16) if E == 8 else (0, 7, 15)
    prec = PREC[dt]
    worst = dict(dk=0, e3=0.0, e64=0.0)
    # three steps, every column at once
    X3, i3 = c.solve(A, P, torch.from_numpy(B).cuda(), rtol=0.0, max_iter=3, max_replace=0, block_width=16)
    X3 = X3.cpu().numpy()
    for k in cols:
        ref = _oracle_pcg(key, k, prec, rtol=1e-8, history=True)
        ref64 = _oracle_pcg(key, k, 0, rtol=1e-8)
        r3 = _oracle_pcg(key, k, prec, rtol=0.0, max_iter=3, max_replace=0)
        assert info[k]["status"] == 0 and info[k]["true_relres"] <= 1e-8
        worst["dk"] = max(worst["dk"], abs(info[k]["iters"] - ref["iters"]))
        worst["e3"] = max(worst["e3"], relerr(X3[:, k], r3["x"]))
        worst["e64"] = max(worst["e64"], relerr(Xh[:, k], ref64["x"]))
        assert stop_agrees(info[k]["iters"], ref["iters"], ref["hist"]), (k, info[k]["iters"], ref["iters"])
    print(f"{key} {dt} fused={fused}: max |dk| {worst['dk']}, 3-step |dx|/|x| {worst['e3']:.2e}, "
          f"converged vs FP64 oracle {worst['e64']:.2e}")
    assert worst["e3"] <= 10 * APPLY_TOL[dt]
    assert worst["e64"] <= 1e-5


@pytest.mark.parametrize("key,E,R", [("q1_8", 8, 2), ("q1_8", 8, 16), ("q1_40", 40, 16)])
@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_pcg_xr_in_forward_solve_equals_separate_pass(ctx, ctx_sep_xr, key, E, R, dt):
    """The forward solve that applies the previous step's x, r update forms the
    same values as the separate pass (the same fused multiply-adds), so the
    iterates are bit-identical at equal step counts; only ||r||^2 is summed in
    another order, which can move a converged stop by one step at most."""
    prob, _ = workload_problem(key)
    Ah = (prob.row_ptr, prob.col, prob.val)
    _, L, U, _ = oracle_factor(f"w:{key}")
    B = torch.from_numpy(np.ascontiguousarray(traction_loads(E, 16, 2000 + E)[:, :R])).cuda()
    for k in (1, 2, 7):
        outs = []
        for c in (ctx, ctx_sep_xr):
            P = c.prec(to_gpu(L), dt)
            outs.append(c.solve(to_gpu(Ah), P, B, rtol=0.0, max_iter=k, max_replace=0, block_width=R))
        (Xa, ia), (Xb, ib) = outs
        assert [i["iters"] for i in ia] == [i["iters"] for i in ib] == [k] * R
        assert [i["status"] for i in ia] == [i["status"] for i in ib] == [pkg._lib.E_MAXITER] * R
        assert torch.equal(Xa, Xb), k
    outs = []
    for c in (ctx, ctx_sep_xr):
        P = c.prec(to_gpu(L), dt)
        outs.append(c.solve(to_gpu(Ah), P, B, rtol=1e-8, block_width=R))
    (Xa, ia), (Xb, ib) = outs
    same = 0
    for c in range(R):
        assert ia[c]["status"] == ib[c]["status"] == 0
        assert abs(ia[c]["iters"] - ib[c]["iters"]) <= 1
        if ia[c]["iters"] == ib[c]["iters"]:
            same += 1
            assert torch.equal(Xa[:, c], Xb[:, c]), c
    print(f"{key} R={R} {dt}: {same} of {R} columns stop at the same step (bit-identical x there)")


# ------------------------------------------------------------ autograd

def test_autograd_prec_apply_matches_oracle_adjoint(ctx):
    """prec_apply(l_val, R, P) through torch.autograd: l_val.grad and R.grad
    equal the oracle's reverse-mode derivative (FP64)."""
    _, L, U, _ = oracle_factor("q1e5s2.0")
    n = L[0].shape[0] - 1
    P = ctx.prec(to_gpu(L), "f64")
    rng = np.random.default_rng(21)
    Rh = rng.standard_normal((n, 4))
    Gh = rng.standard_normal((n, 4))
    lv = torch.from_numpy(L[2]).cuda().requires_grad_(True)
    Rt = torch.from_numpy(Rh).cuda().requires_grad_(True)
    Z = pkg.prec_apply(lv, Rt, P)
    (Z * torch.from_numpy(Gh).cuda()).sum().backward()
    ref = oracle.apply_adjoint(L, U, Rh, Gh)
    assert relerr(Z.detach().cpu().numpy(), ref["Z"]) <= 1e-12
    assert relerr(lv.grad.cpu().numpy(), ref["dL"]) <= 1e-10
    assert relerr(Rt.grad.cpu().numpy(), ref["Rbar"]) <= 1e-10


def test_autograd_version_guard(ctx):
    """A backward after the preconditioner's values were replaced by another
    forward refuses to run (it would differentiate the wrong factor)."""
    _, L, U, _ = oracle_factor("w:q1_8")
    n = L[0].shape[0] - 1
    P = ctx.prec(to_gpu(L), "f64")
    lv = torch.from_numpy(L[2]).cuda().requires_grad_(True)
    Rt = torch.from_numpy(np.random.default_rng(2).standard_normal((n, 2))).cuda()
    Z1 = pkg.prec_apply(lv, Rt, P)
    Z2 = pkg.prec_apply(lv * 1.5, Rt, P)
    Z2.sum().backward()  # the latest forward is fine
    with pytest.raises(RuntimeError, match="changed between forward and backward"):
        Z1.sum().backward()
    for _ in range(3):  # fresh tensors at reused addresses do not fool the guard
        Z1 = pkg.prec_apply(lv.detach().clone().requires_grad_(True), Rt, P)
        pkg.prec_apply(lv.detach().clone(), Rt, P)
        with pytest.raises(RuntimeError):
            Z1.sum().backward()


# ------------------------------------------------- finite differences, 48^3

def test_adjoint_central_differences_q48(ctx):
    """Reverse-mode dl/dL of l = sum_k ||A z_k - r_k||^2, Z = L^-T L^-1 R, at
    48^3 (345,744 DOF, 8 seeded N(0,1) columns), against central differences
    with h = 1e-6 on 64 seeded nonzeros of L, each l evaluated on the GPU.
    Per entry: |g - fd| <= 1e-6 |g| + 10 eps |l| / h + the difference
    quotient's truncation error (bounded by comparing h and 2h)."""
    from synth import build_workload
    prob, Rh = build_workload("q1_48_block8")
    Ah = (prob.row_ptr, prob.col, prob.val)
    st, L, _, _, _ = oracle.ic0_shifted(*Ah)
    A = to_gpu(Ah)
    P = ctx.prec(to_gpu(L), "f64")
    Rt = torch.from_numpy(Rh).cuda()
    lv0 = torch.from_numpy(L[2]).cuda()

    def loss(lv):
        P.update_values(lv)
        _, Z = P.apply(Rt)
        D = ctx.spmv(A, Z) - Rt
        return float((D * D).sum())

    P.update_values(lv0)
    Y, Z = P.apply(Rt)
    G = 2.0 * ctx.spmv(A, (ctx.spmv(A, Z) - Rt).contiguous())
    _, dL = P.apply_backward(G, Y, Z)
    dL = dL.cpu().numpy()
    l0 = loss(lv0)
    q = np.random.default_rng(4000).choice(L[2].size, 64, replace=False)
    eps = np.finfo(float).eps
    worst = 0.0
    for idx in q:
        fd = []
        for h in (1e-6, 2e-6):
            lp = lv0.clone(); lp[idx] += h
            lm = lv0.clone(); lm[idx] -= h
            fd.append((loss(lp) - loss(lm)) / (2 * h))
        g = dL[idx]
        trunc = abs(fd[1] - fd[0])  # O(h^2) term: 3x its own size at h
        tol = 1e-6 * abs(g) + 10 * eps * abs(l0) / 1e-6 + trunc
        worst = max(worst, abs(g - fd[0]) / tol)
        assert abs(g - fd[0]) <= tol, (idx, g, fd)
    P.update_values(lv0)
    print(f"48^3: l = {l0:.6e}; worst |g - fd| / tolerance = {worst:.2f}")
