"""Pins of the FP64 CPU oracle against what the mathematics fixes (CPU only).

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong index or sign, a transposed operand, an off-by-one in the iteration
count) fails at least one of them.
"""

import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle
from synth import (banded_spd, dense_spd, dense_to_csr, kershaw4, laplacian7, q1_elasticity,
                   spectrum_spd, tridiagonal_spd, build_workload)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def csr_of(M, pattern=None):
    return dense_to_csr(M, pattern)


def lower_dense(lrp, lci, lv, n):
    return sp.csr_matrix((lv, lci, lrp), shape=(n, n)).toarray()


# ------------------------------------------------------------------ IC(0)

@pytest.mark.parametrize("n", [1, 2, 7, 40])
def test_ic0_tridiagonal_is_cholesky(n):
    M = tridiagonal_spd(n, seed=n)
    st, L, alpha, _, _ = oracle.ic0_shifted(*csr_of(M))
    assert st == oracle.OK and alpha == 0.0
    Ld = lower_dense(*L, n)
    C = np.linalg.cholesky(M)
    assert np.abs(Ld - C).max() <= 1e-14 * np.abs(C).max()


@pytest.mark.parametrize("n", [3, 12, 30])
def test_ic0_full_pattern_is_cholesky(n):
    M = dense_spd(n, seed=n, cond=1e3)
    st, L, alpha, _, _ = oracle.ic0_shifted(*csr_of(M, np.ones((n, n), bool)))
    assert st == oracle.OK and alpha == 0.0
    C = np.linalg.cholesky(M)
    assert np.abs(lower_dense(*L, n) - C).max() <= 1e-12 * np.abs(C).max()


def test_ic0_full_band_is_cholesky():
    n, bw = 25, 3
    M = banded_spd(n, bw, seed=1)
    pat = np.abs(np.subtract.outer(np.arange(n), np.arange(n))) <= bw
    st, L, alpha, _, _ = oracle.ic0_shifted(*csr_of(M, pat))
    assert st == oracle.OK and alpha == 0.0
    C = np.linalg.cholesky(M)
    assert np.abs(lower_dense(*L, n) - C).max() <= 1e-13 * np.abs(C).max()


def test_ic0_diagonal_is_sqrt():
    d = np.array([4.0, 9.0, 2.0, 0.25])
    st, L, _, _, mp = oracle.ic0_shifted(*csr_of(np.diag(d)))
    assert st == oracle.OK
    assert np.array_equal(L[2], np.sqrt(d))
    assert mp == 0.25


@pytest.mark.parametrize("E", [2, 3])
def test_ic0_defining_identity_on_pattern(E):
    """(L L^T)_ij = A_ij on every stored lower entry; off the pattern LL^T may differ."""
    p = q1_elasticity(E, 2.0, 21)
    st, L, alpha, _, _ = oracle.ic0_shifted(p.row_ptr, p.col, p.val)
    assert st == oracle.OK
    n = p.n
    Ld = lower_dense(*L, n)
    A = p.to_scipy().toarray() + alpha * np.diag(np.diag(p.to_scipy().toarray()))
    P = Ld @ Ld.T
    lrp, lci, _ = L
    rows = np.repeat(np.arange(n), np.diff(lrp))
    err = np.abs(P[rows, lci] - A[rows, lci])
    assert err.max() <= 1e-12 * np.abs(A).max()
    # lower triangular with positive diagonal, on exactly tril(A)'s stored pattern
    assert np.all(np.diag(Ld) > 0)
    T = sp.tril(p.to_scipy()).tocsr()
    T.sort_indices()
    assert np.array_equal(lrp, T.indptr) and np.array_equal(lci, T.indices)
    assert lci.shape[0] == (p.nnz + n) // 2


def test_ic0_kershaw_breakdown_and_shift():
    g = json.load(open(os.path.join(GOLDEN, "kershaw4.json")))
    A = np.array(g["A"], float)
    assert np.all(np.linalg.eigvalsh(A) > 0)
    C = np.linalg.cholesky(A)
    assert np.allclose(np.diag(C) ** 2, g["cholesky_pivots_squared"], rtol=1e-14)
    rp, ci, v = csr_of(A)
    lrp, lci, lv = oracle.tril(rp, ci, v)
    st, L, fr, mp = oracle.ic0(lrp, lci, lv, 0.0)
    assert st == oracle.PIVOT
    assert fr == g["ic0_fail_row"]
    assert abs(mp - g["ic0_pivots_squared"][3]) < 1e-13
    # the shift rule recovers, and the shifted factor satisfies the identity for A + alpha diag(A)
    st, L, alpha, restarts, _ = oracle.ic0_shifted(rp, ci, v)
    assert st == oracle.OK and alpha > 0 and restarts >= 1
    seq = [0.0] + [1e-3 * 2 ** k for k in range(40)]
    assert alpha == seq[restarts]
    Ld = lower_dense(*L, 4)
    As = A + alpha * np.diag(np.diag(A))
    P = Ld @ Ld.T
    for i in range(4):
        for q in range(L[0][i], L[0][i + 1]):
            j = L[1][q]
            assert abs(P[i, j] - As[i, j]) < 1e-13
    # one step earlier in the shift sequence still fails
    st_prev, *_ = oracle.ic0(lrp, lci, lv, seq[restarts - 1])
    assert st_prev == oracle.PIVOT


def test_ic0_laplacian_never_shifts():
    rp, ci, v = laplacian7(6, 5, 4)
    st, L, alpha, restarts, mp = oracle.ic0_shifted(rp, ci, v)
    assert st == oracle.OK and alpha == 0.0 and restarts == 0 and mp > 0


def test_tril_and_transpose_against_scipy():
    p = q1_elasticity(3, 1.0, 2)
    lrp, lci, lv = oracle.tril(p.row_ptr, p.col, p.val)
    T = sp.tril(p.to_scipy()).tocsr()
    T.sort_indices()
    assert np.array_equal(lrp, T.indptr) and np.array_equal(lci, T.indices)
    assert np.array_equal(lv, T.data)
    urp, uci, uv = oracle.transpose(lrp, lci, lv)
    U = T.T.tocsr()
    U.sort_indices()
    assert np.array_equal(urp, U.indptr) and np.array_equal(uci, U.indices)
    assert np.array_equal(uv, U.data)


# ------------------------------------------------------------------ levels

def q1_levels_closed_form(E):
    N1 = E + 1
    K_, J_, I_ = np.meshgrid(np.arange(E), np.arange(N1), np.arange(N1), indexing="ij")
    i = np.repeat(I_.reshape(-1), 3); j = np.repeat(J_.reshape(-1), 3); k = np.repeat(K_.reshape(-1), 3)
    d = np.tile(np.arange(3), N1 * N1 * E)
    lo = 3 * (i + 2 * j + 4 * k) + d
    up = 3 * ((E - i) + 2 * (E - j) + 4 * (E - 1 - k)) + (2 - d)
    return lo, up


@pytest.mark.parametrize("E", [1, 2, 3, 4, 5])
def test_levels_q1_closed_form(E):
    p = q1_elasticity(E, 1.0, 1)
    lrp, lci, _ = oracle.tril(p.row_ptr, p.col, p.val)
    lev, nl = oracle.levels_lower(lrp, lci)
    levu, nlu = oracle.levels_upper(lrp, lci)
    lo, up = q1_levels_closed_form(E)
    assert nl == 21 * E - 9 and nlu == 21 * E - 9
    assert np.array_equal(lev, lo)
    assert np.array_equal(levu, up)


def test_levels_properties_and_sort():
    p = q1_elasticity(4, 1.0, 1)
    lrp, lci, _ = oracle.tril(p.row_ptr, p.col, p.val)
    lev, nl = oracle.levels_lower(lrp, lci)
    levu, nlu = oracle.levels_upper(lrp, lci)
    rows = np.repeat(np.arange(p.n), np.diff(lrp))
    off = lci < rows
    # every dependency sits on a strictly lower level; the level is tight
    assert np.all(lev[lci[off]] < lev[rows[off]])
    assert np.all(levu[rows[off]] < levu[lci[off]])
    tight = np.full(p.n, -1)
    np.maximum.at(tight, rows[off], lev[lci[off]])
    assert np.array_equal(lev, tight + 1)
    perm, lp = oracle.level_sort(lev, nl)
    assert np.array_equal(perm, np.lexsort((np.arange(p.n), lev)))
    assert np.array_equal(lp, np.concatenate([[0], np.cumsum(np.bincount(lev, minlength=nl))]))


def test_levels_special_patterns():
    M = tridiagonal_spd(9)
    lrp, lci, _ = oracle.tril(*csr_of(M))
    lev, nl = oracle.levels_lower(lrp, lci)
    assert nl == 9 and np.array_equal(lev, np.arange(9))
    levu, nlu = oracle.levels_upper(lrp, lci)
    assert nlu == 9 and np.array_equal(levu, np.arange(9)[::-1])
    lrp, lci, _ = oracle.tril(*csr_of(np.diag(np.arange(1.0, 6.0))))
    assert oracle.levels_lower(lrp, lci)[1] == 1
    assert oracle.levels_upper(lrp, lci)[1] == 1


# --------------------------------------------------------- triangular solves

def test_trsv_against_scipy_solve_triangular():
    rng = np.random.default_rng(5)
    n = 30
    M = np.tril(rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.3), -1)
    M += np.diag(1.0 + rng.random(n))
    lrp, lci, lv = csr_of(M)
    r = rng.standard_normal(n)
    y = oracle.trsv_lower(lrp, lci, lv, r)
    assert np.allclose(y, sla.solve_triangular(M, r, lower=True), rtol=1e-13, atol=1e-13)
    urp, uci, uv = oracle.transpose(lrp, lci, lv)
    z = oracle.trsv_upper(urp, uci, uv, y)
    assert np.allclose(z, sla.solve_triangular(M.T, y, lower=False), rtol=1e-13, atol=1e-13)


def test_trsv_residual_on_factor():
    p = q1_elasticity(4, 2.0, 9)
    st, L, _, _, _ = oracle.ic0_shifted(p.row_ptr, p.col, p.val)
    r = np.random.default_rng(1).standard_normal(p.n)
    y = oracle.trsv_lower(*L, r)
    Ls = sp.csr_matrix((L[2], L[1], L[0]), shape=(p.n, p.n))
    assert np.linalg.norm(Ls @ y - r) / np.linalg.norm(r) < 1e-13
    U = oracle.transpose(*L)
    z = oracle.trsv_upper(*U, y)
    assert np.linalg.norm(Ls.T @ z - y) / np.linalg.norm(y) < 1e-13


def test_spmv_against_dense():
    p = q1_elasticity(3, 1.0, 4)
    x = np.random.default_rng(2).standard_normal(p.n)
    w = oracle.spmv(p.row_ptr, p.col, p.val, x)
    assert np.allclose(w, p.to_scipy().toarray() @ x, rtol=1e-13, atol=1e-12)


# --------------------------------------------------------------------- PCG

def _identity_factor(n):
    I = np.eye(n)
    L = csr_of(I)
    return L, oracle.transpose(*L)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_pcg_k_distinct_eigenvalues(k):
    """CG on A with k distinct eigenvalues reaches the solution after k products."""
    n = 50
    lam = np.linspace(1.0, 10.0, k)
    M = spectrum_spd(n, lam, seed=k)
    A = csr_of(M, np.ones((n, n), bool))
    L, U = _identity_factor(n)
    b = np.random.default_rng(k).standard_normal(n)
    res = oracle.pcg(A, L, U, b, rtol=1e-10, max_replace=0)
    assert res["status"] == oracle.OK
    assert res["iters"] == k
    assert np.allclose(res["x"], np.linalg.solve(M, b), rtol=1e-8)


def test_pcg_exact_factor_one_iteration():
    n = 40
    M = dense_spd(n, seed=3, cond=1e4)
    A = csr_of(M, np.ones((n, n), bool))
    st, L, _, _, _ = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    b = np.random.default_rng(0).standard_normal(n)
    res = oracle.pcg(A, L, U, b, rtol=1e-10)
    assert res["iters"] == 1 and res["status"] == oracle.OK
    assert np.linalg.norm(res["x"] - np.linalg.solve(M, b)) <= 1e-10 * np.linalg.norm(res["x"])


def test_pcg_zero_rhs_and_exact_start():
    p = q1_elasticity(2, 1.0, 3)
    A = (p.row_ptr, p.col, p.val)
    st, L, _, _, _ = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    res = oracle.pcg(A, L, U, np.zeros(p.n), x0=np.ones(p.n))
    assert res["iters"] == 0 and res["status"] == oracle.OK and np.all(res["x"] == 0)
    xs = np.linalg.solve(p.to_scipy().toarray(), np.ones(p.n))
    res = oracle.pcg(A, L, U, np.ones(p.n), x0=xs, rtol=1e-6)
    assert res["iters"] == 0


def test_pcg_solution_and_residual_q1_8():
    prob, b = build_workload("q1_8")
    A = (prob.row_ptr, prob.col, prob.val)
    st, L, alpha, _, _ = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    res = oracle.pcg(A, L, U, b, rtol=1e-8)
    assert res["status"] == oracle.OK and 5 < res["iters"] < 200
    D = prob.to_scipy().toarray()
    xs = np.linalg.solve(D, b)
    assert np.linalg.norm(D @ res["x"] - b) / np.linalg.norm(b) <= 1e-8
    kappa = np.linalg.cond(D)
    assert np.linalg.norm(res["x"] - xs) / np.linalg.norm(xs) <= kappa * 1e-8
    assert res["true_relres"] <= 1e-8


def test_pcg_a_norm_bound_eq6():
    """A-norm form of the CG error bound (Eq. 6) with kappa of L^-1 A L^-T."""
    p = q1_elasticity(2, 1.0, 8)
    A = (p.row_ptr, p.col, p.val)
    st, L, _, _, _ = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    n = p.n
    D = p.to_scipy().toarray()
    Ld = lower_dense(*L, n)
    Li = np.linalg.inv(Ld)
    ev = np.linalg.eigvalsh(Li @ D @ Li.T)
    kappa = ev[-1] / ev[0]
    q = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    b = np.random.default_rng(3).standard_normal(n)
    xs = np.linalg.solve(D, b)
    e0 = np.sqrt(xs @ D @ xs)
    for l in range(1, 12):
        res = oracle.pcg(A, L, U, b, rtol=0.0, max_iter=l, max_replace=0)
        assert res["status"] == oracle.MAXITER and res["iters"] == l
        e = res["x"] - xs
        assert np.sqrt(e @ D @ e) <= 2 * e0 * q ** l * (1 + 1e-8) + 1e-12


def test_pcg_failure_statuses():
    n = 4
    L, U = _identity_factor(n)
    # indefinite A: p^T A p <= 0 on the first step
    M = np.diag([1.0, -3.0, 1.0, 1.0])
    res = oracle.pcg(csr_of(M), L, U, np.ones(n))
    assert res["status"] == oracle.BREAKDOWN
    # non-finite input
    res = oracle.pcg(csr_of(np.eye(n) * 2), L, U, np.array([1.0, np.nan, 0, 0]))
    assert res["status"] == oracle.NONFINITE
    # max_iter exhausted
    p = q1_elasticity(2, 1.0, 3)
    A = (p.row_ptr, p.col, p.val)
    Lp = oracle.ic0_shifted(*A)[1]
    res = oracle.pcg(A, Lp, oracle.transpose(*Lp), np.ones(p.n), rtol=1e-30, max_iter=7)
    assert res["status"] == oracle.MAXITER and res["iters"] == 7


def test_pcg_iteration_count_convention():
    """Iterations = products A p: the listing's pre-loop step is iteration 1, so a
    2-eigenvalue problem stops at exactly 2 and max_iter=1 stops after one product."""
    n = 20
    M = spectrum_spd(n, [1.0, 4.0], seed=1)
    A = csr_of(M, np.ones((n, n), bool))
    L, U = _identity_factor(n)
    b = np.random.default_rng(9).standard_normal(n)
    r1 = oracle.pcg(A, L, U, b, rtol=0.0, max_iter=1, max_replace=0)
    # after one step of CG from 0 the iterate is the steepest-descent step alpha b
    alpha = (b @ b) / (b @ M @ b)
    assert np.allclose(r1["x"], alpha * b, rtol=1e-13)
    r2 = oracle.pcg(A, L, U, b, rtol=1e-12, max_replace=0)
    assert r2["iters"] == 2


@pytest.mark.parametrize("prec", [1, 2])
def test_pcg_reduced_precision_factor_q1_8(prec):
    prob, b = build_workload("q1_8")
    A = (prob.row_ptr, prob.col, prob.val)
    st, L, _, _, _ = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    ref = oracle.pcg(A, L, U, b, rtol=1e-8)
    res = oracle.pcg(A, L, U, b, rtol=1e-8, prec=prec)
    assert res["status"] == oracle.OK
    assert res["true_relres"] <= 1e-8
    err = np.linalg.norm(res["x"] - ref["x"]) / np.linalg.norm(ref["x"])
    assert err < 1e-6
    assert abs(res["iters"] - ref["iters"]) <= (3 if prec == 1 else 30)


def test_round_bf16_against_torch():
    import torch
    assert oracle.round_bf16(1.0) == 1.0
    assert oracle.round_bf16(1.0 + 2 ** -8) == 1.0                 # tie to even
    assert oracle.round_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6    # tie to even (up)
    x = np.random.default_rng(0).standard_normal(20000).astype(np.float32) * 1e3
    got = oracle.cast_values(x.astype(np.float64), 2)
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(got, want)
    got32 = oracle.cast_values(x.astype(np.float64), 1)
    assert np.array_equal(got32, x)


def test_apply_f32_close_to_f64():
    p = q1_elasticity(3, 1.0, 5)
    st, L, _, _, _ = oracle.ic0_shifted(p.row_ptr, p.col, p.val)
    U = oracle.transpose(*L)
    r = np.random.default_rng(0).standard_normal(p.n)
    _, z = oracle.apply(L, U, r)
    z32 = oracle.apply_f32(L, U, r, 1)
    z16 = oracle.apply_f32(L, U, r, 2)
    e32 = np.linalg.norm(z32 - z) / np.linalg.norm(z)
    e16 = np.linalg.norm(z16 - z) / np.linalg.norm(z)
    # float arithmetic leaves errors of float's unit roundoff (2^-24 = 6e-8)
    # times the solve's growth, and a BF16 factor (2^-9 = 2e-3) far more: an
    # emulation that kept FP64 anywhere, or skipped the BF16 rounding, lands
    # orders of magnitude lower
    assert 1e-8 < e32 < 1e-5
    assert 1e-4 < e16 < 1e-1
    # the result is the float solve's, widened
    for zz in (z32, z16):
        assert np.array_equal(zz.astype(np.float32).astype(np.float64), zz)


def test_apply_f32_exact_on_dyadic_factor():
    """A factor whose values are powers of two (and sums of two) with an
    integer right-hand side: every intermediate of both triangular solves is a
    short dyadic rational, exact in float, so the float-emulated apply equals
    the exact L^-T L^-1 r computed in rational arithmetic from the dense
    factor, bit for bit."""
    from fractions import Fraction
    rng = np.random.default_rng(12)
    n = 9
    Ld = np.zeros((n, n))
    for i in range(n):
        Ld[i, i] = float(2 ** int(rng.integers(0, 3)))
        for j in range(i):
            if rng.random() < 0.45:
                Ld[i, j] = float(rng.choice([-0.5, 0.25, -0.125, 0.75]))
    L = dense_to_csr(Ld)
    U = oracle.transpose(*L)
    r = rng.integers(-8, 9, n).astype(np.float64)
    F = [[Fraction(Ld[i, j]) for j in range(n)] for i in range(n)]
    y = []
    for i in range(n):
        y.append((Fraction(r[i]) - sum(F[i][j] * y[j] for j in range(i))) / F[i][i])
    z = [Fraction(0)] * n
    for i in reversed(range(n)):
        z[i] = (y[i] - sum(F[j][i] * z[j] for j in range(i + 1, n))) / F[i][i]
    # the exact result is short enough for float (checked, so the test means
    # what it says)
    exact = np.array([float(v) for v in z])
    assert all(Fraction(float(np.float32(v))) == v for v in z)
    assert np.array_equal(oracle.apply_f32(L, U, r, 1), exact)
    assert np.array_equal(oracle.apply(L, U, r)[1], exact)


# ----------------------------------------------------------------- adjoint

def test_adjoint_diagonal_closed_form():
    l = np.array([1.5, 2.0, 0.7])
    r = np.array([0.3, -1.0, 2.0])
    g = np.array([1.0, 0.5, -2.0])
    L = csr_of(np.diag(l))
    U = oracle.transpose(*L)
    out = oracle.apply_adjoint(L, U, r[:, None], g[:, None])
    assert np.allclose(out["Z"][:, 0], r / l ** 2, rtol=1e-15)
    # z_i = r_i / l_i^2  =>  dl/dl_i = -2 g_i r_i / l_i^3,  dl/dr_i = g_i / l_i^2
    assert np.allclose(out["dL"], -2 * g * r / l ** 3, rtol=1e-14)
    assert np.allclose(out["Rbar"][:, 0], g / l ** 2, rtol=1e-15)


def test_adjoint_central_differences():
    p = q1_elasticity(2, 1.0, 6)
    st, L, _, _, _ = oracle.ic0_shifted(p.row_ptr, p.col, p.val)
    lrp, lci, lv = L
    n, m = p.n, 3
    rng = np.random.default_rng(4000)
    R = rng.standard_normal((n, m))
    W = rng.standard_normal((n, m))

    def loss(vals, Rm):
        Lx = (lrp, lci, vals)
        Z = oracle.apply_adjoint(Lx, oracle.transpose(*Lx), Rm, np.zeros_like(Rm))["Z"]
        return float(np.sum(W * Z) + 0.5 * np.sum(Z * Z))

    Z = oracle.apply_adjoint(L, oracle.transpose(*L), R, np.zeros_like(R))["Z"]
    G = W + Z
    out = oracle.apply_adjoint(L, oracle.transpose(*L), R, G)
    h = 1e-6
    for q in rng.choice(lv.shape[0], 20, replace=False):
        vp = lv.copy(); vp[q] += h
        vm = lv.copy(); vm[q] -= h
        fd = (loss(vp, R) - loss(vm, R)) / (2 * h)
        assert abs(fd - out["dL"][q]) <= 1e-6 * abs(fd) + 1e-7, (q, fd, out["dL"][q])
    for (i, k) in [(0, 0), (n // 2, 1), (n - 1, 2)]:
        Rp = R.copy(); Rp[i, k] += h
        Rm = R.copy(); Rm[i, k] -= h
        fd = (loss(lv, Rp) - loss(lv, Rm)) / (2 * h)
        assert abs(fd - out["Rbar"][i, k]) <= 1e-6 * abs(fd) + 1e-7


def test_adjoint_rbar_is_apply_of_g():
    p = q1_elasticity(2, 1.0, 6)
    st, L, _, _, _ = oracle.ic0_shifted(p.row_ptr, p.col, p.val)
    U = oracle.transpose(*L)
    G = np.random.default_rng(1).standard_normal((p.n, 2))
    R = np.random.default_rng(2).standard_normal((p.n, 2))
    out = oracle.apply_adjoint(L, U, R, G)
    for k in range(2):
        _, z = oracle.apply(L, U, G[:, k])
        assert np.array_equal(out["Rbar"][:, k], z)
    # symmetric operator: <G, apply(R)> == <apply(G), R>
    assert abs(np.sum(G * out["Z"]) - np.sum(out["Rbar"] * R)) < 1e-10 * np.abs(np.sum(G * out["Z"]))


def test_dot_is_nearly_exactly_rounded():
    """The inner product matches the correctly rounded sum (math.fsum of the
    rounded products) even under heavy cancellation."""
    import math
    rng = np.random.default_rng(7)
    a = rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))
    b = rng.standard_normal(200000)
    a = np.concatenate([a, -a[:1000]]); b = np.concatenate([b, b[:1000]])
    exact = math.fsum(a * b)
    got = oracle.dot(a, b)
    assert abs(got - exact) <= 4 * np.finfo(float).eps * math.fsum(np.abs(a * b))
    assert oracle.dot(np.ones(10), np.arange(10.0)) == 45.0


# ------------------------------------------- Table 1 baselines (None, Jacobi)

@pytest.mark.parametrize("k", [1, 3, 6])
def test_plain_cg_k_distinct_eigenvalues(k):
    """Unpreconditioned CG: k distinct eigenvalues -> k products."""
    n = 40
    M = spectrum_spd(n, np.linspace(2.0, 7.0, k), seed=10 + k)
    A = csr_of(M, np.ones((n, n), bool))
    b = np.random.default_rng(k).standard_normal(n)
    res = oracle.pcg_simple(A, b, "none", rtol=1e-10, max_replace=0)
    assert res["status"] == oracle.OK and res["iters"] == k
    assert np.allclose(res["x"], np.linalg.solve(M, b), rtol=1e-8)


def test_jacobi_equals_cg_on_symmetrically_scaled_matrix():
    """Jacobi-PCG on A is CG on D^-1/2 A D^-1/2 with x = D^-1/2 x_hat, b_hat =
    D^-1/2 b: the same iterates at every k."""
    p = q1_elasticity(3, 2.0, 17)
    M = p.to_scipy().toarray()
    d = np.diag(M).copy()
    s = 1.0 / np.sqrt(d)
    Ms = M * s[:, None] * s[None, :]
    pat = M != 0
    A = csr_of(M, pat)
    As = csr_of(Ms, pat)
    b = np.random.default_rng(3).standard_normal(p.n)
    for k in (1, 4, 15):
        rj = oracle.pcg_simple(A, b, "jacobi", rtol=0.0, max_iter=k, max_replace=0)
        rn = oracle.pcg_simple(As, s * b, "none", rtol=0.0, max_iter=k, max_replace=0)
        assert rj["iters"] == rn["iters"] == k
        assert np.linalg.norm(rj["x"] - s * rn["x"]) <= 1e-10 * np.linalg.norm(rj["x"])
    full = oracle.pcg_simple(A, b, "jacobi", rtol=1e-10)
    assert full["status"] == oracle.OK
    assert np.allclose(full["x"], np.linalg.solve(M, b), rtol=1e-7, atol=1e-9 * np.abs(full["x"]).max())


def test_jacobi_on_diagonal_matrix_one_iteration():
    n = 30
    D = np.diag(np.random.default_rng(1).uniform(1, 100, n))
    A = csr_of(D, np.eye(n, dtype=bool))
    b = np.random.default_rng(2).standard_normal(n)
    res = oracle.pcg_simple(A, b, "jacobi", rtol=1e-12)
    assert res["iters"] == 1
    assert np.allclose(res["x"], b / np.diag(D), rtol=1e-14)


# ------------------------------------------------ fill-in dropout (Eq. 10)

def test_dropout_worked_example():
    # rows: [2], [0.0005 3], [-0.02 0.01 4]; eps = 0.01 keeps |l| > 0.01 and the diagonal
    L = (np.array([0, 1, 3, 6]), np.array([0, 0, 1, 0, 1, 2], np.int32),
         np.array([2.0, 0.0005, 3.0, -0.02, 0.01, 4.0]))
    rp, ci, v = oracle.dropout(L, 0.01)
    assert rp.tolist() == [0, 1, 2, 4]
    assert ci.tolist() == [0, 1, 0, 2]
    assert v.tolist() == [2.0, 3.0, -0.02, 4.0]
    # eps = 0 removes exact zeros only; a tiny diagonal is never removed
    L0 = (np.array([0, 1, 3]), np.array([0, 0, 1], np.int32), np.array([1e-30, 0.0, 1.0]))
    rp, ci, v = oracle.dropout(L0, 0.0)
    assert rp.tolist() == [0, 1, 2] and ci.tolist() == [0, 1] and v.tolist() == [1e-30, 1.0]


def test_dropout_of_ic_factor_is_a_subpattern():
    p = q1_elasticity(3, 1.5, 21)
    st, L, *_ = oracle.ic0_shifted(p.row_ptr, p.col, p.val)
    n = p.n
    for eps in (0.0, 1e-3, 1e-2, 5e-2):
        D = lower_dense(*oracle.dropout(L, eps), n)
        F = lower_dense(*L, n)
        off = ~np.eye(n, dtype=bool)
        assert np.array_equal(np.diag(D), np.diag(F))
        assert np.array_equal(D[off], np.where(np.abs(F) > eps, F, 0.0)[off])


# ------------------------------------------------- residual replacement

def _offset_case(n, max_replace):
    """A = I_n, L = I_n, b = 3/4 per entry, x_0 = 2^53 per entry. Every step is
    exact or rounds by hand: r_0 = fl(3/4 - 2^53) = -(2^53 - 1), so z = p = r_0,
    alpha = r_0^T z / p^T A p = 1 and x_1 = 2^53 + r_0 = 1 exactly, while the
    recurrence gives r_1 = r_0 - r_0 = 0: the recurrence has converged but the
    true residual b - x_1 = -1/4 per entry (relative 1/3). A replacement sets
    r = -1/4; then beta = (n/16) / fl(n (2^53 - 1)^2) ~ 2^-110 leaves
    p = fl(-1/4 + beta r_0... ) = -1/4 (the term is below half an ulp of 1/4),
    alpha = 1 and x_2 = 1 - 1/4 = 3/4 exactly, r_2 = 0 and b - x_2 = 0."""
    L, U = _identity_factor(n)
    A = csr_of(np.eye(n))
    b = np.full(n, 0.75)
    x0 = np.full(n, 2.0 ** 53)
    return oracle.pcg(A, L, U, b, x0=x0, rtol=1e-8, max_replace=max_replace, max_iter=50)


@pytest.mark.parametrize("n", [1, 4])
def test_pcg_replacement_worked_example(n):
    """Supplementary Algorithm 1 with the true-residual check: a recurrence that
    reaches zero while b - A x does not triggers exactly one replacement, after
    which one more step lands on the exact solution."""
    res = _offset_case(n, 0)
    # no replacement allowed: the recurrence stopped after 1 product, x_1 = 1
    assert res["status"] == oracle.TRUE_RESIDUAL
    assert res["iters"] == 1 and res["replacements"] == 0
    assert np.all(res["x"] == 1.0)
    assert res["relres"] == 0.0 and res["true_relres"] == pytest.approx(1.0 / 3.0, rel=1e-15)
    for mr in (1, 3):
        res = _offset_case(n, mr)
        assert res["status"] == oracle.OK
        assert res["iters"] == 2 and res["replacements"] == 1
        assert np.all(res["x"] == 0.75)
        assert res["true_relres"] == 0.0


def test_pcg_replacement_counts_against_max_iter():
    """A replacement at the iteration cap reports the cap, not success."""
    L, U = _identity_factor(2)
    res = oracle.pcg(csr_of(np.eye(2)), L, U, np.full(2, 0.75), x0=np.full(2, 2.0 ** 53), rtol=1e-8,
                     max_replace=3, max_iter=1)
    assert res["status"] == oracle.MAXITER
    assert res["iters"] == 1 and res["replacements"] == 1
    assert np.all(res["x"] == 1.0)


def test_pcg_replacement_below_attainable_accuracy():
    """A tolerance below what FP64 attains in b - A x on the 8^3 workload
    (about 2e-14 here): the recurrence residual keeps shrinking past it, the
    true residual does not, so each allowed replacement is used and the status
    says the true residual stayed above the tolerance. A replacement restarts
    the recurrence from b - A x, so the run is longer and its recurrence
    residual again ends below the tolerance. (With three replacements the
    restarted recurrences wander for hundreds of iterations and their length
    changes with the last bits of the input, so the pin stops at one.)"""
    prob, b = build_workload("q1_8")
    A = (prob.row_ptr, prob.col, prob.val)
    st, L, alpha, _, _ = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    D = prob.to_scipy().toarray()
    nb = np.linalg.norm(b)
    eps = np.finfo(float).eps
    prev = None
    for mr in (0, 1):
        res = oracle.pcg(A, L, U, b, rtol=1e-14, max_replace=mr, max_iter=2000)
        assert res["status"] == oracle.TRUE_RESIDUAL
        assert res["replacements"] == mr
        assert res["relres"] <= 1e-14 < res["true_relres"]
        tr = np.linalg.norm(b - D @ res["x"]) / nb
        assert tr == pytest.approx(res["true_relres"], rel=1e-2)
        # the attainable level: a small multiple of eps ||A|| ||x|| / ||b||
        assert tr <= 100 * eps * np.linalg.norm(D, 2) * np.linalg.norm(res["x"]) / nb
        if prev is not None:
            assert res["iters"] > prev
        prev = res["iters"]


def test_pcg_bitwise_independent_of_threads():
    """The row-parallel loops (SpMV rows, vector updates) give the same bits at
    any thread count: each output element is computed by the same sequential
    code, and the inner products stay sequential."""
    p = q1_elasticity(6, 1.0, 5)
    A = (p.row_ptr, p.col, p.val)
    st, L, _, _, _ = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    b = np.random.default_rng(3).standard_normal(p.n)
    default = oracle.set_threads(0)
    try:
        runs = []
        for t in (1, 3, 8):
            assert oracle.set_threads(t) == t
            runs.append((oracle.pcg(A, L, U, b, rtol=1e-10), oracle.spmv(*A, b)))
        for r, w in runs[1:]:
            assert np.array_equal(r["x"], runs[0][0]["x"]) and r["iters"] == runs[0][0]["iters"]
            assert np.array_equal(w, runs[0][1])
    finally:
        oracle.set_threads(default)


def test_pcg_snapshots_are_the_iterates():
    """The recorded entries at step k equal x after a run stopped at k."""
    p = q1_elasticity(5, 1.0, 9)
    A = (p.row_ptr, p.col, p.val)
    st, L, _, _, _ = oracle.ic0_shifted(*A)
    U = oracle.transpose(*L)
    b = np.random.default_rng(1).standard_normal(p.n)
    idx = np.arange(0, p.n, 7)
    r = oracle.pcg(A, L, U, b, rtol=1e-10, snap=(idx, 3, 9))
    for k in range(3, 10):
        rk = oracle.pcg(A, L, U, b, rtol=0.0, max_iter=k, max_replace=0)
        assert np.array_equal(r["x_snap"][k - 3], rk["x"][idx])
    late = oracle.pcg(A, L, U, b, rtol=1e-10, snap=(idx, r["iters"], r["iters"] + 2))
    assert np.array_equal(late["x_snap"][0], r["x"][idx]) and np.isnan(late["x_snap"][1:]).all()
