"""GPU kernels through the C ABI against the FP64 oracle, element by element
(small and mid-size cases spanning many tiles and ragged tails)."""

import numpy as np
import pytest
import torch

import oracle
import paper_2412_07127_amd as pkg
from gpu_common import workload_problem, named_matrix, oracle_factor, random_lower_pattern, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    return pkg.Context()


def to_gpu(A):
    return pkg.CSR.from_numpy(*A, device="cuda")


def cols_of(X):
    return X if X.ndim == 2 else X[:, None]


# ---------------------------------------------------------------- SpMV

@pytest.mark.parametrize("key", ["w:q1_8", "lap7", "q1e3s2.0", "tridiag"])
@pytest.mark.parametrize("R", [1, 2, 4, 8, 16])
def test_spmv(ctx, key, R):
    A = named_matrix(key)
    n = A[0].shape[0] - 1
    X = np.random.default_rng(R).standard_normal((n, R))
    W = ctx.spmv(to_gpu(A), torch.from_numpy(X).cuda()).cpu().numpy()
    for c in range(R):
        ref = oracle.spmv(*A, X[:, c])
        assert np.abs(W[:, c] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("key", ["w:q1_8", "lap7", "q1e3s2.0", "grouped_ragged"])
@pytest.mark.parametrize("R", [1, 2, 4, 8, 16])
def test_grouped_spmv(ctx, key, R):
    """Row-group SpMV (analyzed matrix) equals the oracle's row products."""
    if key == "grouped_ragged":
        # rows 0-2 share columns, 3 alone, 4-8 share (split into 3 + 2), ragged tail
        rng = np.random.default_rng(1)
        n = 301
        rows, cols = [], []
        i = 0
        while i < n:
            g = min(int(rng.integers(1, 6)), n - i)
            base = sorted(set(rng.choice(n, size=int(rng.integers(1, 12)), replace=False).tolist()) |
                          set(range(i, i + g)))
            for r in range(i, i + g):
                rows += [r] * len(base)
                cols += base
            i += g
        rp = np.zeros(n + 1, np.int64)
        np.add.at(rp, np.asarray(rows) + 1, 1)
        A = (np.cumsum(rp), np.asarray(cols, np.int32), rng.standard_normal(len(cols)))
    else:
        A = named_matrix(key)
    n = A[0].shape[0] - 1
    M = ctx.matrix(to_gpu(A))
    X = np.random.default_rng(R).standard_normal((n, R))
    W = M.spmv(torch.from_numpy(X).cuda()).cpu().numpy()
    for c in range(R):
        ref = oracle.spmv(*A, X[:, c])
        assert np.abs(W[:, c] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def long_and_empty_rows(n=700, seed=11, with_diag=False):
    """General CSR with rows longer than any prefetch window (~230 entries),
    short rows and, unless with_diag, empty rows (first, last and inside)."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        if not with_diag and i in (0, 5, 6, n // 2, n - 1):
            rows.append(np.zeros(0, np.int64))
            continue
        k = 230 if i % 97 == 3 else int(rng.integers(1, 9))
        c = set(rng.choice(n, size=k, replace=False).tolist())
        if with_diag:
            c.add(i)
        rows.append(np.array(sorted(c), np.int64))
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    return rp, ci, rng.standard_normal(len(ci))


@pytest.mark.parametrize("R", [1, 2, 4, 8, 16])
def test_spmv_long_and_empty_rows(ctx, R):
    """Plain SpMV on a raw CSR: empty rows give 0, rows past the prefetch
    window take the remainder loop."""
    A = long_and_empty_rows()
    n = A[0].shape[0] - 1
    X = np.random.default_rng(R + 7).standard_normal((n, R))
    W = ctx.spmv(to_gpu(A), torch.from_numpy(X).cuda()).cpu().numpy()
    for c in range(R):
        ref = oracle.spmv(*A, X[:, c])
        assert np.abs(W[:, c] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())
    assert np.all(W[[0, 5, 6, n // 2, n - 1]] == 0.0)


@pytest.mark.parametrize("R", [1, 4, 16])
def test_grouped_spmv_long_groups(ctx, R):
    """Row groups of 3 rows sharing ~150 columns (past the 96-entry window)."""
    rng = np.random.default_rng(3)
    n, rows = 450, []
    for g in range(0, n, 3):
        k = 150 if g % 30 == 0 else int(rng.integers(1, 20))
        c = np.array(sorted(set(rng.choice(n, size=k, replace=False).tolist()) | {g, g + 1, g + 2}), np.int64)
        rows += [c, c, c]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    A = (rp, ci, rng.standard_normal(len(ci)))
    M = ctx.matrix(to_gpu(A))
    X = np.random.default_rng(R).standard_normal((n, R))
    W = M.spmv(torch.from_numpy(X).cuda()).cpu().numpy()
    for c in range(R):
        ref = oracle.spmv(*A, X[:, c])
        assert np.abs(W[:, c] - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_solve_with_analyzed_matrix(ctx):
    prob, b = workload_problem("q1_8")
    Ah = (prob.row_ptr, prob.col, prob.val)
    M = ctx.matrix(to_gpu(Ah))
    _, L, U, _ = oracle_factor("w:q1_8")
    P = ctx.prec(to_gpu(L), "f64")
    X, info = ctx.solve(M, P, torch.from_numpy(b).cuda(), rtol=1e-8)
    ref = oracle.pcg(Ah, L, U, b, rtol=1e-8)
    assert info[0]["status"] == 0 and abs(info[0]["iters"] - ref["iters"]) <= 1
    same_k = oracle.pcg(Ah, L, U, b, rtol=0.0, max_iter=info[0]["iters"], max_replace=0)
    assert relerr(X.cpu().numpy(), same_k["x"]) <= 1e-10


# -------------------------------------------------------------- levels

LEVEL_CASES = ["w:q1_8", "q1e5s1.0", "lap7", "tridiag", "diag", "randlow", "one"]


def level_matrix(key):
    if key == "diag":
        n = 1000
        return np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.full(n, 2.0)
    if key == "randlow":
        return random_lower_pattern(3000, 0.004, 5)
    if key == "one":
        return np.array([0, 1], np.int64), np.array([0], np.int32), np.array([3.0])
    A = named_matrix(key)
    return oracle.tril(*A)


@pytest.mark.parametrize("key", LEVEL_CASES)
def test_levels_bit_exact(ctx, key):
    L = level_matrix(key)
    P = ctx.prec(to_gpu(L), "f64")
    g = {k: v.cpu().numpy() for k, v in P.levels().items()}
    lev, nl = oracle.levels_lower(L[0], L[1])
    perm, lp = oracle.level_sort(lev, nl)
    levu, nlu = oracle.levels_upper(L[0], L[1])
    permu, lpu = oracle.level_sort(levu, nlu)
    assert np.array_equal(g["level_L"], lev)
    assert np.array_equal(g["perm_L"], perm)
    assert np.array_equal(g["level_ptr_L"], lp)
    assert np.array_equal(g["level_U"], levu)
    assert np.array_equal(g["perm_U"], permu)
    assert np.array_equal(g["level_ptr_U"], lpu)
    info = P.info()
    assert info["nlevels_L"] == nl and info["nlevels_U"] == nlu
    # supernodes never lengthen the dependency chain
    assert info["nsn_levels_L"] <= nl and info["nsn_levels_U"] <= nlu


def test_supernode_levels_q1():
    """3-DOF nodes form supernodes: node-level count 7E - 3 for the Q1 grid."""
    ctx = pkg.Context()
    for E in (2, 4, 8):
        A = named_matrix(f"q1e{E}s1.0")
        L = oracle.tril(*A)
        info = ctx.prec(to_gpu(L), "f64").info()
        n = L[0].shape[0] - 1
        assert info["nsupernodes_L"] == n // 3 and info["nsupernodes_U"] == n // 3
        assert info["nsn_levels_L"] == 7 * E - 3
        assert info["nsn_levels_U"] == 7 * E - 3


@pytest.mark.parametrize("key", ["w:q1_8", "randlow", "tridiag"])
def test_transpose_exact(ctx, key):
    L = level_matrix(key)
    P = ctx.prec(to_gpu(L), "f64")
    U = P.transpose().numpy()
    Ur = oracle.transpose(*L)
    for a, b in zip(U, Ur):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------- SpTRSV

@pytest.mark.parametrize("key", ["w:q1_8", "q1e5s2.0", "lap7", "tridiag", "randlow"])
@pytest.mark.parametrize("R", [1, 4, 16])
def test_trsv_f64(ctx, key, R):
    if key == "randlow":
        L = random_lower_pattern(3000, 0.004, 5)
    else:
        _, L, _, _ = oracle_factor(key)
    U = oracle.transpose(*L)
    n = L[0].shape[0] - 1
    P = ctx.prec(to_gpu(L), "f64")
    Rh = np.random.default_rng(R + 1).standard_normal((n, R))
    Y = P.trsv(torch.from_numpy(Rh).cuda()).cpu().numpy()
    Z = P.trsv(torch.from_numpy(Y).cuda(), transpose=True).cpu().numpy()
    for c in range(R):
        y = oracle.trsv_lower(*L, Rh[:, c])
        z = oracle.trsv_upper(*U, y)
        assert relerr(Y[:, c], y) <= 1e-12
        assert relerr(Z[:, c], z) <= 1e-12


def arrow_lower(n=700, dense_from=600, seed=9):
    """Lower factor whose last rows are dense (every third column): rows of the
    forward solve and, through them, rows of the backward solve run past the
    prefetch window."""
    rng = np.random.default_rng(seed)
    rows, vals = [], []
    for i in range(n):
        if i >= dense_from:
            c = np.arange(0, i, 3)
        else:
            k = min(i, int(rng.integers(0, 5)))
            c = np.sort(rng.choice(i, size=k, replace=False)) if k else np.zeros(0, int)
        rows.append(np.concatenate([c, [i]]).astype(np.int64))
        vals.append(np.concatenate([0.02 * rng.standard_normal(len(c)), [1.0 + rng.random()]]))
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    return rp, np.concatenate(rows).astype(np.int32), np.concatenate(vals)


@pytest.mark.parametrize("R", [1, 4, 16])
def test_trsv_rows_past_window(ctx, R):
    L = arrow_lower()
    U = oracle.transpose(*L)
    assert np.diff(L[0]).max() > 64 and np.diff(U[0]).max() > 64
    n = L[0].shape[0] - 1
    P = ctx.prec(to_gpu(L), "f64")
    Rh = np.random.default_rng(R + 3).standard_normal((n, R))
    Y = P.trsv(torch.from_numpy(Rh).cuda()).cpu().numpy()
    Z = P.trsv(torch.from_numpy(Y).cuda(), transpose=True).cpu().numpy()
    for c in range(R):
        y = oracle.trsv_lower(*L, Rh[:, c])
        z = oracle.trsv_upper(*U, y)
        assert relerr(Y[:, c], y) <= 1e-12
        assert relerr(Z[:, c], z) <= 1e-12


@pytest.mark.parametrize("dt,prec", [("f32", 1), ("bf16", 2)])
def test_apply_reduced_precision(ctx, dt, prec):
    A, L, U, _ = oracle_factor("w:q1_8")
    n = L[0].shape[0] - 1
    P = ctx.prec(to_gpu(L), dt)
    r = np.random.default_rng(0).standard_normal(n)
    _, Z = P.apply(torch.from_numpy(r).cuda())
    z_emul = oracle.apply_f32(L, U, r, prec)   # float emulation of the same arithmetic
    _, z64 = oracle.apply(L, U, r)
    z = Z.double().cpu().numpy()
    e_emul = relerr(z, z_emul)
    e64 = relerr(z, z64)
    print(f"{dt}: |z-z_emul|/|z|={e_emul:.2e} |z-z_f64|/|z|={e64:.2e}")
    assert e_emul <= (1e-5 if dt == "f32" else 1e-4)
    assert e64 <= (1e-4 if dt == "f32" else 5e-2)


# ---------------------------------------------------------------- IC(0)

@pytest.mark.parametrize("key", ["w:q1_8", "q1e5s2.0", "lap7", "tridiag", "kershaw", "w:q1_40"])
def test_factor(ctx, key):
    A, L, U, alpha = oracle_factor(key)
    Lg, info = ctx.factor(to_gpu(A))
    assert info["alpha"] == alpha
    g = Lg.numpy()
    assert np.array_equal(g[0], L[0]) and np.array_equal(g[1], L[1])
    err = np.abs(g[2] - L[2]).max() / np.abs(L[2]).max()
    assert err <= 1e-12, err


# ------------------------------------------------------------------ PCG

@pytest.mark.parametrize("idx", ["q1_8", "q1_40"])
def test_solve_f64_matches_oracle(ctx, idx):
    prob, b = workload_problem(idx)
    Ah = (prob.row_ptr, prob.col, prob.val)
    A = to_gpu(Ah)
    Lg, _ = ctx.factor(A)
    P = ctx.prec(Lg, "f64")
    X, info = ctx.solve(A, P, torch.from_numpy(b).cuda(), rtol=1e-8)
    _, L, U, _ = oracle_factor(f"w:{idx}")
    ref = oracle.pcg(Ah, L, U, b, rtol=1e-8)
    k = info[0]["iters"]
    print(f"{idx}: gpu iters {k} oracle iters {ref['iters']} true relres {info[0]['true_relres']:.3e}")
    assert info[0]["status"] == pkg._lib.OK
    assert abs(k - ref["iters"]) <= 1
    assert info[0]["true_relres"] <= 1e-8
    same_k = oracle.pcg(Ah, L, U, b, rtol=0.0, max_iter=k, max_replace=0)
    assert relerr(X.cpu().numpy(), same_k["x"]) <= 1e-10


def test_multi_rhs_columns_match_oracle(ctx):
    prob, _ = workload_problem("q1_8")
    Ah = (prob.row_ptr, prob.col, prob.val)
    A = to_gpu(Ah)
    _, L, U, _ = oracle_factor("w:q1_8")
    P = ctx.prec(to_gpu(L), "f64")
    n = prob.n
    B = np.random.default_rng(11).standard_normal((n, 5))
    B[:, 3] *= 1e-3
    X, info = ctx.solve(A, P, torch.from_numpy(B).cuda(), rtol=1e-8)
    Xh = X.cpu().numpy()
    for c in range(5):
        k = info[c]["iters"]
        ref = oracle.pcg(Ah, L, U, B[:, c], rtol=1e-8)
        assert info[c]["status"] == 0 and abs(k - ref["iters"]) <= 1
        same_k = oracle.pcg(Ah, L, U, B[:, c], rtol=0.0, max_iter=k, max_replace=0)
        assert relerr(Xh[:, c], same_k["x"]) <= 1e-10


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_solve_reduced_precision(ctx, dt):
    prob, b = workload_problem("q1_40")
    Ah = (prob.row_ptr, prob.col, prob.val)
    A = to_gpu(Ah)
    Lg, _ = ctx.factor(A)
    P = ctx.prec(Lg, dt)
    X, info = ctx.solve(A, P, torch.from_numpy(b).cuda(), rtol=1e-8)
    _, L, U, _ = oracle_factor("w:q1_40")
    ref = oracle.pcg(Ah, L, U, b, rtol=1e-8)
    x = X.cpu().numpy()
    tr = relerr(oracle.spmv(*Ah, x), b)
    err = relerr(x, ref["x"])
    print(f"{dt}: iters {info[0]['iters']} (fp64 oracle {ref['iters']}), true relres {tr:.3e}, "
          f"|x - x_oracle|/|x_oracle| = {err:.3e}, replacements {info[0]['replacements']}")
    assert info[0]["status"] == 0
    assert tr <= 1e-8
    assert err <= 1e-5


# ------------------------------------------------------------- adjoint

@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_adjoint_matches_oracle(ctx, dt):
    _, L, U, _ = oracle_factor("q1e5s2.0")
    n = L[0].shape[0] - 1
    R = 8
    rng = np.random.default_rng(3000)
    Rh = rng.standard_normal((n, R))
    G = rng.standard_normal((n, R))
    ref = oracle.apply_adjoint(L, U, Rh, G)
    P = ctx.prec(to_gpu(L), dt)
    tdt = torch.float64 if dt == "f64" else torch.float32
    Y, Z = P.apply(torch.from_numpy(Rh).cuda().to(tdt))
    dR, dL = P.apply_backward(torch.from_numpy(G).cuda(), Y, Z)
    ez = relerr(Z.double().cpu().numpy(), ref["Z"])
    er = relerr(dR.double().cpu().numpy(), ref["Rbar"])
    el = relerr(dL.double().cpu().numpy(), ref["dL"])
    print(f"{dt}: Z {ez:.2e} dR {er:.2e} dL {el:.2e}")
    tol = 1e-10 if dt == "f64" else 1e-3
    assert ez <= tol and er <= tol and el <= tol


# ------------------------------------------------------------ edge cases

def test_zero_rhs_and_exact_start(ctx):
    prob, b = workload_problem("q1_8")
    A = to_gpu((prob.row_ptr, prob.col, prob.val))
    Lg, _ = ctx.factor(A)
    P = ctx.prec(Lg, "f64")
    X, info = ctx.solve(A, P, torch.zeros(prob.n, dtype=torch.float64, device="cuda"),
                        X0=torch.ones(prob.n, dtype=torch.float64, device="cuda"))
    assert info[0]["iters"] == 0 and info[0]["status"] == 0
    assert torch.count_nonzero(X).item() == 0
    Bt = torch.from_numpy(b).cuda()
    X1, info1 = ctx.solve(A, P, Bt, rtol=1e-10)
    X2, info2 = ctx.solve(A, P, Bt, X0=X1, rtol=1e-6)
    assert info2[0]["iters"] == 0 and torch.equal(X1, X2)


def test_max_iter_and_nonfinite(ctx):
    prob, b = workload_problem("q1_8")
    A = to_gpu((prob.row_ptr, prob.col, prob.val))
    Lg, _ = ctx.factor(A)
    P = ctx.prec(Lg, "f64")
    X, info = ctx.solve(A, P, torch.from_numpy(b).cuda(), rtol=1e-30, max_iter=5)
    assert info[0]["status"] == pkg._lib.E_MAXITER and info[0]["iters"] == 5
    bad = b.copy()
    bad[7] = np.nan
    X, info = ctx.solve(A, P, torch.from_numpy(bad).cuda())
    assert info[0]["status"] == pkg._lib.E_NONFINITE


def test_invalid_inputs_rejected(ctx):
    rp, ci, v = named_matrix("lap7")
    ci2 = ci.copy()
    ci2[[3, 4]] = ci2[[4, 3]]  # unsorted row
    with pytest.raises(pkg.IcpcgError) as e:
        ctx.factor(to_gpu((rp, ci2, v)))
    assert e.value.status == pkg._lib.E_INVALID
    # a factor with an entry above the diagonal is rejected
    L = oracle.tril(rp, ci, v)
    Lbad = (L[0], L[1].copy(), L[2])
    Lbad[1][L[0][5]] = 6
    with pytest.raises(pkg.IcpcgError):
        ctx.prec(to_gpu(Lbad), "f64")
    # non-positive diagonal
    Lneg = (L[0], L[1], L[2].copy())
    Lneg[2][L[0][3] - 1] = -1.0
    with pytest.raises(pkg.IcpcgError):
        ctx.prec(to_gpu(Lneg), "f64")


def test_pivot_breakdown_gives_up_with_status(ctx):
    A = named_matrix("kershaw")
    Lg, info = ctx.factor(to_gpu(A), max_restarts=0, raise_on_pivot=False)
    assert info["status"] == pkg._lib.E_PIVOT and info["alpha"] == 0.0


def test_dependency_wait_limit_reports_device_error(ctx, monkeypatch):
    """Failure handling forced from the host: a context whose dependency waits
    may not wait at all gives up every pending wait (the kernels still finish)
    and the solve reports ICPCG_E_DEVICE; other contexts are unaffected."""
    prob, b = workload_problem("q1_8")
    A = to_gpu((prob.row_ptr, prob.col, prob.val))
    Lg, _ = ctx.factor(A)
    P = ctx.prec(Lg, "f64")
    monkeypatch.setenv("ICPCG_WAIT_LIMIT_US", "0")
    ctx0 = pkg.Context()
    monkeypatch.delenv("ICPCG_WAIT_LIMIT_US")
    bt = torch.from_numpy(b).cuda()
    with pytest.raises(pkg.IcpcgError) as ei:
        ctx0.solve(A, P, bt, rtol=1e-8)
    assert ei.value.status == pkg._lib.E_DEVICE
    assert "time limit" in str(ei.value)
    X, info = ctx.solve(A, P, bt, rtol=1e-8)
    assert info[0]["status"] == 0 and info[0]["true_relres"] <= 1e-8
    ctx0.close()
