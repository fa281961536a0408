"""Pins of the GNN-correction oracle (oracle/gnn.py) against closed forms,
brute force and finite differences (CPU)."""

import itertools

import numpy as np
import pytest

import oracle
from oracle import gnn as G
from synth import dense_to_csr, q1_elasticity


def small_graph(E=2, sigma=1.0, seed=5):
    p = q1_elasticity(E, sigma, seed)
    A = (p.row_ptr, p.col, p.val)
    st, L, alpha, restarts, mp = oracle.ic0_shifted(*A)
    assert st == oracle.OK
    return A, L, G.Graph(A, L)


def dense(rp, ci, val, n):
    D = np.zeros((n, n))
    for i in range(n):
        D[i, ci[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    return D


def pattern(rp, ci, n):
    B = np.zeros((n, n), bool)
    for i in range(n):
        B[i, ci[rp[i]:rp[i + 1]]] = True
    return B


def test_param_count():
    # 27 (normalization) + 169 + 177 (block 1) + 177 + 177 (block 2) + 177 (block 3)
    assert G.num_params() == 904
    th = G.init_params(3)
    assert np.array_equal(G.pack(G.unpack(th)), th)


def test_algorithms_1_and_2_equal_dense_products():
    A, L, g = small_graph()
    n = g.n
    z = np.random.default_rng(1).choice([-1.0, 1.0], n)
    DA = dense(*A, n)
    DL = dense(*L, n)
    assert np.allclose(G.coo_matvec(g.a_rows, A[1].astype(np.int64), A[2], z), DA @ z, rtol=1e-13, atol=1e-12)
    assert np.allclose(G.coo_llt_matvec(g.r, g.c, g.Lic, z), DL @ (DL.T @ z), rtol=1e-13, atol=1e-12)


def test_hutchinson_average_over_all_probes_is_frobenius_norm():
    # Eq. 4: E_z ||M z||^2 = ||M||_F^2 for Rademacher z; the average over all
    # 2^n sign vectors is exact
    rng = np.random.default_rng(4)
    n = 7
    M = rng.standard_normal((n, n))
    Aspd = M @ M.T + n * np.eye(n)
    A = dense_to_csr(Aspd)
    Lp = dense_to_csr(np.tril(rng.standard_normal((n, n))) + 3 * np.eye(n))
    g = G.Graph(A, Lp)
    DL = dense(*Lp, n)
    acc = 0.0
    for signs in itertools.product([-1.0, 1.0], repeat=n):
        z = np.array(signs)
        d = G.coo_llt_matvec(g.r, g.c, g.Lic, z) - G.coo_matvec(g.a_rows, A[1].astype(np.int64), A[2], z)
        acc += d @ d
    fro = np.linalg.norm(DL @ DL.T - Aspd, "fro") ** 2
    assert acc / 2 ** n == pytest.approx(fro, rel=1e-12)


def test_node_features_brute_force():
    A, L, g = small_graph(E=2, sigma=1.5, seed=9)
    n = g.n
    x = G.node_features(g)
    B = pattern(A[0], A[1], n)
    D = dense(*A, n)
    off = B & ~np.eye(n, dtype=bool)
    deg = off.sum(1).astype(float)
    assert np.array_equal(x[:, 0], deg)
    for i in range(n):
        nd = deg[off[i]]
        assert x[i, 1] == nd.max() and x[i, 2] == nd.min()
        assert x[i, 3] == pytest.approx(nd.mean(), rel=1e-14)
        assert x[i, 4] == pytest.approx(((nd - nd.mean()) ** 2).mean(), rel=1e-12, abs=1e-12)
    ad = np.abs(D)
    assert np.allclose(x[:, 5], np.diag(ad) / ad.sum(1), rtol=1e-14)
    assert np.allclose(x[:, 6], np.where(off, ad, 0).max(1) / np.diag(ad), rtol=1e-14)
    ang = np.pi * np.arange(n) / n
    assert np.allclose(x[:, 7:], np.stack([np.sin(ang), np.cos(ang)], 1), rtol=0, atol=1e-15)
    # a 3-DOF node's rows of the Q1 matrix share one neighbourhood
    assert x[0, 0] == x[1, 0] == x[2, 0]


def test_zero_output_reproduces_ic():
    A, L, g = small_graph()
    th = G.init_params(7, zero_output=True)
    Lp = G.predict(g, th)
    assert np.array_equal(Lp, g.Lic)


def test_graph_normalization_standardizes():
    A, L, g = small_graph()
    th = G.init_params(7)
    _, C = G.forward(g, th, keep=True)
    h0, x = C["hs"][0], C["x"]
    assert np.allclose(h0.mean(0), 0.0, atol=1e-12)
    vx = x.var(0)
    assert np.allclose(h0.var(0), vx / (vx + G.GN_EPS), rtol=1e-12)


def test_message_passing_selectors():
    # weights that pick single features give closed forms: they fix which end of
    # an edge is the row and how the aggregation sums (undirected, diagonal once)
    A, L, g = small_graph(E=2, sigma=1.2, seed=3)
    n = g.n
    d = {name: np.zeros(shape) for name, shape in G.param_layout()}
    d["gn_gamma"][:] = 1.0  # alpha = beta = 0: h0 = x / sqrt(mean(x^2) + eps)
    f_r, f_c = 5, 6
    d["e0_W1"][0, 1 + f_r] = 1.0       # hidden 0 <- h_row[f_r]
    d["e0_W1"][1, 1 + 9 + f_c] = 1.0   # hidden 1 <- h_col[f_c]
    d["e0_w2"][0], d["e0_w2"][1] = 1.0, -2.0
    d["n0_W1"][0, 9] = 0.25            # node hidden 0 <- sum
    d["n0_W1"][1, 10] = 1.0            # node hidden 1 <- mean
    d["n0_W2"][3, 0] = 1.0
    d["n0_W2"][4, 1] = 1.0
    th = G.pack(d)
    _, C = G.forward(g, th, keep=True)
    x = C["x"]
    h0 = x / np.sqrt((x * x).mean(0) + G.GN_EPS)
    e = np.tanh(h0[g.r, f_r]) - 2.0 * np.tanh(h0[g.c, f_c])
    assert np.allclose(C["es"][0], e, rtol=1e-14, atol=1e-15)
    S = np.zeros((n, n))
    S[g.r, g.c] = e
    S = S + np.tril(S, -1).T          # symmetric, diagonal once
    s = S.sum(1)
    PL = pattern(L[0], L[1], n)
    cnt = PL.sum(1) + PL.sum(0) - 1
    h1 = C["hs"][1]
    assert np.allclose(h1[:, 3], np.tanh(0.25 * s), rtol=1e-13, atol=1e-15)
    assert np.allclose(h1[:, 4], np.tanh(s / cnt), rtol=1e-13, atol=1e-15)
    assert np.allclose(np.delete(h1, [3, 4], 1), 0.0)


def test_gradient_matches_central_differences():
    A, L, g = small_graph(E=2, sigma=1.0, seed=8)
    th = G.init_params(11, zero_output=False)
    # alpha away from 1: some features of this small graph are constant, and
    # alpha = 1 would centre them to zero, where the loss is too curved for
    # central differences
    d = G.unpack(th)
    rng = np.random.default_rng(12)
    d["gn_alpha"][:] = rng.uniform(0.3, 0.7, 9)
    d["gn_gamma"][:] = rng.uniform(0.5, 1.5, 9)
    d["gn_beta"][:] = rng.uniform(-0.2, 0.2, 9)
    z = np.random.default_rng(2).choice([-1.0, 1.0], g.n)
    x = G.node_features(g)
    f, grad = G.loss_and_grad(g, th, z, x)
    assert f == pytest.approx(G.loss(g, G.predict(g, th, x), z), rel=1e-13)
    h = 1e-6
    fd = np.empty_like(th)
    for k in range(th.size):
        tp = th.copy(); tp[k] += h
        tm = th.copy(); tm[k] -= h
        fd[k] = (G.loss(g, G.predict(g, tp, x), z) - G.loss(g, G.predict(g, tm, x), z)) / (2 * h)
    scale = np.abs(grad).max()
    err = np.abs(fd - grad)
    print(f"loss {f:.6e}, max |grad| {scale:.3e}, max |fd - grad| {err.max():.3e}")
    assert np.all(err <= 1e-6 * np.abs(grad) + 1e-7 * scale)
    # every parameter group receives gradient
    for name, shp in G.param_layout():
        assert np.abs(G.unpack(grad)[name]).max() > 0, name


def test_adam_closed_form_first_step():
    # the first bias-corrected step moves every parameter by lr * sign(grad)
    th = np.array([1.0, -2.0, 0.5])
    gr = np.array([3.0, -0.25, 1e-3])
    t1, m, v = G.adam_step(th, gr, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(t1, th - 0.01 * np.sign(gr), rtol=1e-15)


def test_edge_scale_closed_form_and_dense_brute_force():
    """The edge input scale s is the population standard deviation of the stored
    entries of tril(A) (the edges, diagonal included). Tridiagonal 2/-1 of order
    m: m entries 2 and m-1 entries -1, so with N = 2m-1 the mean is
    (m+1)/N and the variance (m (2-mu)^2 + (m-1)(1+mu)^2) / N. Dense case:
    every lower entry of a random SPD matrix, summed by plain loops. Full A
    instead of tril(A), or the sample (N-1) variance, differs in both."""
    for m in (3, 10, 41):
        T = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
        A = dense_to_csr(T)
        st, L, *_ = oracle.ic0_shifted(*A)
        g = G.Graph(A, L)
        N = 2 * m - 1
        mu = (m + 1) / N
        var = (m * (2 - mu) ** 2 + (m - 1) * (1 + mu) ** 2) / N
        assert G.edge_scale(g) == pytest.approx(np.sqrt(var), rel=1e-14)
    rng = np.random.default_rng(11)
    n = 9
    Mx = rng.standard_normal((n, n))
    D = Mx @ Mx.T + n * np.eye(n)
    A = dense_to_csr(D, np.ones((n, n), bool))
    st, L, *_ = oracle.ic0_shifted(*A)
    g = G.Graph(A, L)
    vals = [D[i, j] for i in range(n) for j in range(i + 1)]
    mean = sum(vals) / len(vals)
    var = sum((v - mean) ** 2 for v in vals) / len(vals)
    assert G.edge_scale(g) == pytest.approx(var ** 0.5, rel=1e-13)


def test_corrected_factor_scale_equivariance():
    """Eq. 2 corrects the factor in the units of the scaled matrix A / s that the
    network sees: every input of the network is invariant under A -> c A (ratios,
    degrees, a_ij / s), L_IC(c A) = sqrt(c) L_IC(A) and s(c A) = c s(A), so the
    corrected factor must scale by sqrt(c) as a factor of c A does. With c = 4
    every step scales by a power of two, so the identity is exact."""
    p = q1_elasticity(2, 1.0, 5)
    th = G.init_params(3, zero_output=False)
    outs = []
    for c in (1.0, 4.0, 3.0):
        A = (p.row_ptr, p.col, p.val * c)
        st, L, *_ = oracle.ic0_shifted(*A)
        g = G.Graph(A, L)
        outs.append(G.predict(g, th))
    assert np.array_equal(outs[1], 2.0 * outs[0])
    assert np.allclose(outs[2], np.sqrt(3.0) * outs[0], rtol=1e-12, atol=0)
    assert not np.array_equal(outs[0], G.predict(G.Graph((p.row_ptr, p.col, p.val), oracle.ic0_shifted(
        p.row_ptr, p.col, p.val)[1]), G.init_params(3, zero_output=True)))


def test_corrected_factor_constant_output_diagonal():
    """A network whose last edge layer outputs the constant c on every edge: on
    the diagonal the corrected squared pivot is the IC(0) squared pivot times
    exp(c) (the exponential, then the square root, of the correction), and off
    the diagonal the change is the same for every entry."""
    A, L, g = small_graph()
    d = G.unpack(G.init_params(4, zero_output=True).copy())
    c = 0.3
    d["e2_b2"][0] = c
    Lp = G.predict(g, G.pack(d))
    dg = g.diag
    assert np.allclose((Lp[dg] / g.Lic[dg]) ** 2, np.exp(c), rtol=1e-14, atol=0)
    off = Lp[~dg] - g.Lic[~dg]
    assert np.allclose(off, off[0], rtol=1e-12, atol=0) and off[0] > 0


def test_loss_gradient_in_L_matches_central_differences():
    """d(Eq. 5 loss)/dL on every stored entry of L, against central differences
    of the loss itself (a slip in either product of the closed form, or a
    transposed operand, fails)."""
    A, L, g = small_graph(E=2, sigma=1.5, seed=21)
    rng = np.random.default_rng(3)
    Lval = g.Lic * (1.0 + 0.1 * rng.standard_normal(g.Lic.size))
    z = rng.choice([-1.0, 1.0], g.n)
    f, dL = G.loss_and_grad_L(g, Lval, z)
    assert f == pytest.approx(G.loss(g, Lval, z), rel=1e-14)
    h = 1e-6
    for q in range(Lval.size):
        lp = Lval.copy(); lp[q] += h
        lm = Lval.copy(); lm[q] -= h
        fd = (G.loss(g, lp, z) - G.loss(g, lm, z)) / (2 * h)
        assert abs(fd - dL[q]) <= 1e-6 * abs(dL[q]) + 1e-8 * np.abs(dL).max(), q


def _iters(A, Lval, L, b):
    Lx = (L[0], L[1], Lval)
    return oracle.pcg(A, Lx, oracle.transpose(*Lx), b, rtol=1e-8)["iters"]


def _adam_on_values(Lval0, grad_fn, steps, lr, keep_diag_positive):
    th = Lval0.copy()
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    for t in range(1, steps + 1):
        gsum = grad_fn(th, t)
        th, m, v = G.adam_step(th, gsum, m, v, t, lr)
        th = np.where(keep_diag_positive, np.maximum(th, 1e-3 * np.abs(Lval0)), th)
    return th


def test_ceiling_free_factor_under_eq5():
    """How far Eq. (5) can take L at all, with no network: Adam on L's stored
    values themselves (the largest correction any network on this pattern
    could output), from L_IC, with fresh probes every step. The Eq. (5) loss
    falls by about a third, while PCG needs no fewer iterations than with
    L_IC: on these elasticity matrices Eq. (5)'s optimum on tril(A)'s pattern
    is not a better preconditioner than IC(0). (An experiment recorded as a
    test: its numbers are printed.)"""
    A, L, g = small_graph(E=4, sigma=1.5, seed=31)
    b = np.random.default_rng(4).standard_normal(g.n)
    rng = np.random.default_rng(5)
    zs_eval = [rng.choice([-1.0, 1.0], g.n) for _ in range(16)]
    mean_loss = lambda Lv: np.mean([G.loss(g, Lv, z) for z in zs_eval])

    def grad(th, t):
        zs = [rng.choice([-1.0, 1.0], g.n) for _ in range(8)]
        return sum(G.loss_and_grad_L(g, th, z)[1] for z in zs) / len(zs)

    Lopt = _adam_on_values(g.Lic, grad, steps=300, lr=2e-3 * np.abs(g.Lic).mean(), keep_diag_positive=g.diag)
    l0, l1 = mean_loss(g.Lic), mean_loss(Lopt)
    k0, k1 = _iters(A, g.Lic, L, b), _iters(A, Lopt, L, b)
    print(f"Eq. 5 loss {l0:.4e} -> {l1:.4e} ({100 * (l1 - l0) / l0:+.1f}%); PCG iterations {k0} -> {k1}")
    assert l1 < 0.85 * l0
    assert k1 >= k0 - 1


def test_ceiling_free_factor_under_solve_loss():
    """The same with the loss the preconditioner is used for:
    ||L^-T L^-1 A z - z||^2 (its gradient from the adjoint of the
    preconditioner solve). The loss falls, the iterations do not: IC(0) is
    already at this pattern's iteration floor here. (Experiment as a test.)"""
    A, L, g = small_graph(E=4, sigma=1.5, seed=31)
    b = np.random.default_rng(4).standard_normal(g.n)
    rng = np.random.default_rng(6)
    zs_eval = [rng.choice([-1.0, 1.0], g.n) for _ in range(8)]

    def solve_loss(Lv, z, want_grad=False):
        Lx = (L[0], L[1], Lv)
        U = oracle.transpose(*Lx)
        az = oracle.spmv(*A, z)
        _, Z = oracle.apply(Lx, U, az)
        d = Z - z
        if not want_grad:
            return float(d @ d)
        return float(d @ d), oracle.apply_adjoint(Lx, U, az, 2.0 * d)["dL"]

    def grad(th, t):
        zs = [rng.choice([-1.0, 1.0], g.n) for _ in range(4)]
        return sum(solve_loss(th, z, True)[1] for z in zs) / len(zs)

    l0 = np.mean([solve_loss(g.Lic, z) for z in zs_eval])
    Lopt = _adam_on_values(g.Lic, grad, steps=150, lr=2e-3 * np.abs(g.Lic).mean(), keep_diag_positive=g.diag)
    l1 = np.mean([solve_loss(Lopt, z) for z in zs_eval])
    k0, k1 = _iters(A, g.Lic, L, b), _iters(A, Lopt, L, b)
    print(f"solve loss {l0:.4e} -> {l1:.4e} ({100 * (l1 - l0) / l0:+.1f}%); PCG iterations {k0} -> {k1}")
    assert l1 < 0.95 * l0
    assert k1 >= k0 - 2
