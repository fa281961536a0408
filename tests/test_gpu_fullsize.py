"""Full-size cases in the launch configuration the benchmark times.

The 100^3 elasticity workload (3,060,300 DOF), the 48^3 workload with an
8-column block (adjoint), and the 150^3 workload (10,260,450 DOF, 16 load
cases).
Where the oracle finishes in seconds it is compared element by element
(factor, level sets, triangular solves, the first PCG iterations, the
adjoint); converged solves are checked through the true residual computed by
the oracle's SpMV on the CPU.
"""

import json
import os
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2412_07127_amd as pkg
import gpu_common
from gpu_common import relerr
from synth import body_load, build_workload, q1_elasticity, traction_loads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


@pytest.fixture(scope="module")
def q100(ctx):
    prob, b = build_workload("q1_100")
    Ah = (prob.row_ptr, prob.col, prob.val)
    A = pkg.CSR.from_numpy(*Ah)
    Lg, finfo = ctx.factor(A)
    st, L, alpha, restarts, _ = oracle.ic0_shifted(*Ah)
    assert st == oracle.OK
    U = oracle.transpose(*L)
    return dict(prob=prob, b=b, Ah=Ah, A=A, Lg=Lg, finfo=finfo, L=L, U=U, alpha=alpha, restarts=restarts)


def true_relres(Ah, x, b):
    return relerr(oracle.spmv(*Ah, x), b)


def test_q100_factor_full_parity(q100):
    assert q100["finfo"]["alpha"] == q100["alpha"] and q100["finfo"]["restarts"] == q100["restarts"]
    g = q100["Lg"].numpy()
    L = q100["L"]
    assert np.array_equal(g[0], L[0]) and np.array_equal(g[1], L[1])
    scale = np.abs(L[2]).max()
    assert np.abs(g[2] - L[2]).max() <= 1e-12 * scale


def test_q100_levels_and_transpose(ctx, q100):
    P = ctx.prec(q100["Lg"], "f64")
    lv = {k: v.cpu().numpy() for k, v in P.levels().items()}
    L = q100["L"]
    lev, nl = oracle.levels_lower(L[0], L[1])
    levu, nlu = oracle.levels_upper(L[0], L[1])
    assert nl == nlu == 21 * 100 - 9
    assert np.array_equal(lv["level_L"], lev) and np.array_equal(lv["level_U"], levu)
    perm, lp = oracle.level_sort(lev, nl)
    assert np.array_equal(lv["perm_L"], perm) and np.array_equal(lv["level_ptr_L"], lp)
    # pattern of L^T equals the oracle's; values are the GPU factor's, transposed exactly
    U = P.transpose().numpy()
    Ug = oracle.transpose(*q100["Lg"].numpy())
    for a, b in zip(U, Ug):
        assert np.array_equal(a, b)
    assert np.array_equal(U[0], q100["U"][0]) and np.array_equal(U[1], q100["U"][1])
    info = P.info()
    assert info["nsn_levels_L"] == info["nsn_levels_U"] == 7 * 100 - 3


@pytest.mark.parametrize("R", [1, 16])
def test_q100_trsv_parity(ctx, q100, R):
    P = ctx.prec(q100["Lg"], "f64")
    n = q100["prob"].n
    Rh = np.random.default_rng(R).standard_normal((n, R))
    Y = P.trsv(torch.from_numpy(Rh).cuda()).cpu().numpy()
    Z = P.trsv(torch.from_numpy(Y).cuda(), transpose=True).cpu().numpy()
    for c in ([0] if R == 1 else [0, 7, 15]):
        y = oracle.trsv_lower(*q100["L"], Rh[:, c])
        z = oracle.trsv_upper(*q100["U"], y)
        assert relerr(Y[:, c], y) <= 1e-12
        assert relerr(Z[:, c], z) <= 1e-12


def test_q100_spmv_block16(ctx, q100):
    n = q100["prob"].n
    X = np.random.default_rng(5).standard_normal((n, 16))
    W = ctx.spmv(q100["A"], torch.from_numpy(X).cuda()).cpu().numpy()
    for c in (0, 9):
        ref = oracle.spmv(*q100["Ah"], X[:, c])
        assert np.abs(W[:, c] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_q100_pcg_first_iterations_match_oracle(ctx, q100):
    """Same x after the same number of iterations, same factor on both sides.
    The early iterates of this workload are very sensitive (a 1e-13 relative
    change of L moves x by ~2e-6 after 25 iterations), so the loop is compared
    over a few iterations with identical inputs; converged solves are judged by
    their true residual and against the stored oracle solution."""
    P = ctx.prec(pkg.CSR.from_numpy(*q100["L"]), "f64")
    b = q100["b"]
    k = 5
    X, info = ctx.solve(q100["A"], P, torch.from_numpy(b).cuda(), rtol=0.0, max_iter=k, max_replace=0)
    assert info[0]["status"] == pkg._lib.E_MAXITER and info[0]["iters"] == k
    ref = oracle.pcg(q100["Ah"], q100["L"], q100["U"], b, rtol=0.0, max_iter=k, max_replace=0)
    assert relerr(X.cpu().numpy(), ref["x"]) <= 1e-10


def load_golden(E):
    """FP64 oracle solves of the E^3 workload (written by
    tests/golden/make_fullsize_golden.py, which calls only the oracle): x on
    every 997th entry after every step k0 - 8 .. k0 + 8 around the oracle's
    converged step count k0. A missing file fails the tests that need it."""
    base = os.path.join(os.path.dirname(__file__), "golden", f"q1_{E}_oracle")
    for f in (base + ".json", base + "_x.npz"):
        assert os.path.exists(f), f"{f} is missing (tests/golden/make_fullsize_golden.py writes it)"
    g = json.load(open(base + ".json"))
    g["idx"] = np.asarray(g["sample_index"])
    with np.load(base + "_x.npz") as z:
        g["x"] = {k: z[k] for k in z.files}
    return g


@pytest.fixture(scope="module")
def golden():
    return load_golden(100)


def sample_err(x, g, case, k=None):
    """Relative error of x on the stored sample against the oracle's x after k
    steps (default: the oracle's converged count)."""
    c = g["cases"][case]
    k = c["iters"] if k is None else k
    lo, hi = c["x_window_steps"]
    assert lo <= k <= hi, f"oracle x stored after steps {lo}..{hi}, GPU stopped at {k}"
    return relerr(np.asarray(x)[g["idx"]], g["x"][case][k - lo])


def stop_agrees(k, c, rtol=1e-8):
    """gpu_common.stop_agrees against a stored oracle case (the oracle's load
    case 0 reads 1.06e-8, 1.14e-8, 1.64e-8, 1.36e-8, 1.23e-8, 1.06e-8, 9.3e-9
    over steps 799-805: a plateau on which runs that agree to 1e-11 may stop
    at any step)."""
    return gpu_common.stop_agrees(k, c["iters"], c["relres_history"], rtol)


# x of two FP64 runs of the same steps that differ only in the order of their
# additions: measured at equal step count at convergence (about 800 steps)
FP64_EQUAL_K = 1e-10
# a reduced-precision factor changes the preconditioner (about 1e-7 relative in
# each apply): both runs reach a true residual of 1e-8 with different iterates
REDUCED_VS_FP64 = 1e-5


@pytest.mark.parametrize("factor", ["gpu", "oracle"])
def test_q100_converged_solve_against_stored_oracle(ctx, q100, golden, factor):
    """FP64 solve of the body load to rtol 1e-8: iterations within one of the
    oracle's, and x at the GPU's own step count equal to the oracle's x after
    that many steps (1e-10), with the GPU's factor and with the oracle's."""
    assert golden["alpha"] == q100["alpha"] and golden["n"] == q100["prob"].n
    L = q100["Lg"] if factor == "gpu" else pkg.CSR.from_numpy(*q100["L"])
    P = ctx.prec(L, "f64")
    X, info = ctx.solve(q100["A"], P, torch.from_numpy(q100["b"]).cuda(), rtol=1e-8)
    k = info[0]["iters"]
    k0 = golden["cases"]["body"]["iters"]
    e = sample_err(X.cpu().numpy(), golden, "body", k)
    e0 = sample_err(X.cpu().numpy(), golden, "body")
    print(f"factor {factor}: gpu iters {k}, oracle {k0}; |x - x_oracle(k)|/|x_oracle(k)| = {e:.2e} "
          f"(against the oracle's converged x: {e0:.2e}); true relres {info[0]['true_relres']:.2e}")
    assert info[0]["status"] == 0 and stop_agrees(k, golden["cases"]["body"])
    assert e <= FP64_EQUAL_K


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_q100_reduced_precision_error_vs_oracle(ctx, q100, golden, dt):
    """FP32 / BF16 factor with FP64 recurrences to a true residual of 1e-8: the
    error of x against the FP64 oracle's converged solution."""
    P = ctx.prec(q100["Lg"], dt)
    X, info = ctx.solve(q100["A"], P, torch.from_numpy(q100["b"]).cuda(), rtol=1e-8)
    e = sample_err(X.cpu().numpy(), golden, "body")
    print(f"{dt}: iters {info[0]['iters']} (FP64 oracle {golden['cases']['body']['iters']}), "
          f"|x - x_oracle|/|x_oracle| = {e:.2e}")
    assert info[0]["status"] == 0 and info[0]["true_relres"] <= 1e-8
    assert e <= REDUCED_VS_FP64


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_q100_solve_true_residual(ctx, q100, dt):
    P = ctx.prec(q100["Lg"], dt)
    b = q100["b"]
    X, info = ctx.solve(q100["A"], P, torch.from_numpy(b).cuda(), rtol=1e-8)
    x = X.cpu().numpy()
    tr = true_relres(q100["Ah"], x, b)
    print(f"{dt}: iters {info[0]['iters']} true relres (oracle SpMV) {tr:.3e} "
          f"(library {info[0]['true_relres']:.3e}) replacements {info[0]['replacements']}")
    assert info[0]["status"] == 0
    assert tr <= 1e-8
    assert abs(tr - info[0]["true_relres"]) <= 1e-3 * tr + 1e-14


def test_q100_multi_rhs_16(ctx, q100, golden):
    """The headline's launch configuration: 16 load cases, FP32 factor, width
    16, steps replayed as a hipGraph. Load cases 0 and 1 against the FP64
    oracle's converged solves of those columns."""
    P = ctx.prec(q100["Lg"], "f32")
    B = traction_loads(100, 16, 2004)
    X, info = ctx.solve(q100["A"], P, torch.from_numpy(B).cuda(), rtol=1e-8, block_width=16, use_graph=True)
    Xh = X.cpu().numpy()
    assert all(i["status"] == 0 for i in info)
    for c in (0, 5, 15):
        assert true_relres(q100["Ah"], Xh[:, c], B[:, c]) <= 1e-8
    for c in (0, 1):
        e = sample_err(Xh[:, c], golden, f"traction{c}")
        print(f"load case {c}: {info[c]['iters']} iterations (FP64 oracle {golden['cases'][f'traction{c}']['iters']}),"
              f" |x - x_oracle|/|x_oracle| = {e:.2e}")
        assert e <= REDUCED_VS_FP64
    # a column of the batch is the same iteration as its own single-column
    # solve (same factor); with the factor applied in FP32 the 16-column and
    # 1-column kernels round differently (summation order inside a row and in
    # the reductions), which over ~850 iterations moves the stopping step by a
    # few, so the counts agree to 1% and the solutions to 1e-6
    x1, i1 = ctx.solve(q100["A"], P, torch.from_numpy(np.ascontiguousarray(B[:, 5])).cuda(), rtol=1e-8)
    print(f"column 5: batch {info[5]['iters']} iterations, alone {i1[0]['iters']}")
    assert abs(i1[0]["iters"] - info[5]["iters"]) <= max(2, 0.01 * info[5]["iters"])
    assert relerr(Xh[:, 5], x1.cpu().numpy()) <= 1e-6


def test_q100_multi_rhs_16_fp64_equal_k(ctx, q100, golden):
    """16 load cases with the factor in FP64: load cases 0 and 1 stop within
    one step of the oracle's solves of those columns and equal the oracle's x
    after the same number of steps."""
    P = ctx.prec(q100["Lg"], "f64")
    B = traction_loads(100, 16, 2004)
    X, info = ctx.solve(q100["A"], P, torch.from_numpy(B).cuda(), rtol=1e-8, block_width=16, use_graph=True)
    Xh = X.cpu().numpy()
    for c in (0, 1):
        k, k0 = info[c]["iters"], golden["cases"][f"traction{c}"]["iters"]
        e = sample_err(Xh[:, c], golden, f"traction{c}", k)
        print(f"load case {c}: gpu {k} iterations, oracle {k0}; |x - x_oracle(k)|/|x_oracle(k)| = {e:.2e}")
        assert info[c]["status"] == 0 and stop_agrees(k, golden["cases"][f"traction{c}"])
        assert e <= FP64_EQUAL_K


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_q48_adjoint_full_size(ctx, dt):
    prob, Rh = build_workload("q1_48_block8")   # 48^3 elements, 8 seeded N(0,1) residual columns
    Ah = (prob.row_ptr, prob.col, prob.val)
    st, L, alpha, _, _ = oracle.ic0_shifted(*Ah)
    U = oracle.transpose(*L)
    A = pkg.CSR.from_numpy(*Ah)
    P = ctx.prec(pkg.CSR.from_numpy(*L), dt)
    tdt = torch.float64 if dt == "f64" else torch.float32
    Rt = torch.from_numpy(Rh).cuda()
    Y, Z = P.apply(Rt.to(tdt))
    # loss = sum_k ||A z_k - r_k||^2  ->  G = 2 A (A Z - R)
    Zd = Z.double()
    G = 2.0 * ctx.spmv(A, (ctx.spmv(A, Zd.contiguous()) - Rt).contiguous())
    dR, dL = P.apply_backward(G, Y, Z)
    Gh = G.cpu().numpy()
    ref = oracle.apply_adjoint(L, U, Rh, Gh)
    ez = relerr(Zd.cpu().numpy(), ref["Z"])
    er = relerr(dR.double().cpu().numpy(), ref["Rbar"])
    el = relerr(dL.double().cpu().numpy(), ref["dL"])
    print(f"{dt}: Z {ez:.2e} dR {er:.2e} dL {el:.2e}")
    tol = 1e-10 if dt == "f64" else 1e-3
    assert ez <= tol and er <= tol and el <= tol


def test_q150_multi_rhs_inference_scale(ctx):
    """150^3 elements (10,260,450 DOF, 820M entries), 16 load cases, FP32 factor."""
    prob = q1_elasticity(150, 1.5, 1004)
    Ah = (prob.row_ptr, prob.col, prob.val)
    A = pkg.CSR.from_numpy(*Ah)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Lg, finfo = ctx.factor(A)
    torch.cuda.synchronize()
    t_fac = time.perf_counter() - t0
    P = ctx.prec(Lg, "f32")
    P64 = ctx.prec(Lg, "f64")
    del Lg
    B = traction_loads(150, 16, 2004)
    Bt = torch.from_numpy(B).cuda()
    M = ctx.matrix(A)
    # the comparison of the batched solve: sequential FP64 solves (one timed, x16)
    b0 = Bt[:, 0].contiguous()
    ctx.solve(M, P64, b0, rtol=1e-8, max_iter=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0, info0 = ctx.solve(M, P64, b0, rtol=1e-8)
    torch.cuda.synchronize()
    t_64 = time.perf_counter() - t0
    assert info0[0]["status"] == 0 and info0[0]["true_relres"] <= 1e-8
    del P64
    ctx.autotune(M, P, 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, info = ctx.solve(M, P, Bt, rtol=1e-8, use_graph=True)
    torch.cuda.synchronize()
    t_cg = time.perf_counter() - t0
    iters = [i["iters"] for i in info]
    print(f"q150: factor {t_fac:.2f} s alpha {finfo['alpha']}; 16 load cases {t_cg:.2f} s "
          f"({t_cg / 16:.3f} s per RHS), iters {min(iters)}..{max(iters)}; one FP64 solve "
          f"{t_64:.2f} s ({info0[0]['iters']} it), 16 sequential = {16 * t_64:.1f} s, "
          f"ratio {16 * t_64 / t_cg:.1f}x")
    assert all(i["status"] == 0 for i in info)
    Xh = X.cpu().numpy()
    for c in (0, 15):
        assert true_relres(Ah, Xh[:, c], B[:, c]) <= 1e-8
    # against the FP64 oracle's solves of load cases 0 and 1: the FP64 solve at
    # its own step count (1e-10), the batch's FP32-factor columns against the
    # oracle's converged solutions (1e-5)
    g = load_golden(150)
    assert g["alpha"] == finfo["alpha"] and g["n"] == prob.n
    k = info0[0]["iters"]
    e64 = sample_err(x0.cpu().numpy(), g, "traction0", k)
    errs = [sample_err(Xh[:, c], g, f"traction{c}") for c in (0, 1)]
    print(f"q150 against the oracle: FP64 load case 0 at step {k} (oracle {g['cases']['traction0']['iters']}): "
          f"{e64:.2e}; batch columns 0, 1: {errs[0]:.2e}, {errs[1]:.2e}")
    assert stop_agrees(k, g["cases"]["traction0"])
    assert e64 <= FP64_EQUAL_K
    assert max(errs) <= REDUCED_VS_FP64
