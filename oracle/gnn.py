"""Oracle (test infrastructure only) of the learned correction of the IC(0)
factor: L_pred = L_IC + GNN(A) (Eq. 2).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module; it shares no code with the GPU library. Plain numpy in FP64,
written for clarity (whole-array numpy steps, no blocking or fusion).

What it computes, in the paper's order:
  * the graph: nodes are the unknowns, edges the stored entries of tril(A)
    (the pattern of L, diagonal included), given in CSR order of L;
  * node features x in R^9 (supplementary Table 2): degree, max / min / mean /
    variance of the neighbours' degrees, diagonal dominance, diagonal decay,
    and a sine / cosine position embedding;
  * edge input e in R^1: the entry of A divided by the standard deviation of
    the stored entries of tril(A) (Model Architecture);
  * graph normalization of x on entry to the first block;
  * three message-passing blocks (supplementary Eqs. 7-9): an edge updater
    (two layers, hidden width 8, tanh) on [e, x_row, x_col], sum and mean
    aggregation over the edges incident to a node, a node updater (two
    layers, hidden 8, tanh) on [x, sum, mean]; blocks 2 and 3 take the skip
    concatenation [e_original, e_current] as their edge input;
  * the output g (one value per edge) corrects the factor: off the diagonal
    L = L_IC + sqrt(s) g (s the input scale, so the correction is made in the
    scaled matrix's units), on the diagonal L = L_IC exp(g / 2) (exponential
    then square root, which keeps the diagonal positive);
  * the loss of Eq. 5 with one Rademacher probe z, normalized by ||A z||^2:
    ||L L^T z - A z||^2 / ||A z||^2, with A z by Algorithm 1 and L L^T z by
    Algorithm 2 on COO triples;
  * the gradient of that loss with respect to every parameter, by hand.

Readings where the paper is silent (listed in the design notes): undirected
aggregation (an edge counts at both of its nodes, the diagonal once); the
position embedding angle pi i / n; dominance |a_ii| / sum_j |a_ij|; decay
max_{j != i} |a_ij| / |a_ii|; node width 9 in every block; the parameter count
is this layout's (904), not the paper's 1,958 (parity unpinned for that count).
"""

from __future__ import annotations

import numpy as np

NODE_DIM = 9
HIDDEN = 8
EDGE_IN = (1, 2, 2)
GN_EPS = 1e-5


def param_layout():
    """[(name, shape)] in storage order of the flat parameter vector."""
    lay = [("gn_alpha", (NODE_DIM,)), ("gn_gamma", (NODE_DIM,)), ("gn_beta", (NODE_DIM,))]
    for b in range(3):
        din = EDGE_IN[b] + 2 * NODE_DIM
        lay += [(f"e{b}_W1", (HIDDEN, din)), (f"e{b}_b1", (HIDDEN,)), (f"e{b}_w2", (HIDDEN,)), (f"e{b}_b2", (1,))]
        if b < 2:
            lay += [(f"n{b}_W1", (HIDDEN, NODE_DIM + 2)), (f"n{b}_b1", (HIDDEN,)),
                    (f"n{b}_W2", (NODE_DIM, HIDDEN)), (f"n{b}_b2", (NODE_DIM,))]
    return lay


def num_params():
    return sum(int(np.prod(s)) for _, s in param_layout())


def unpack(theta):
    """Flat vector -> dict of arrays (views)."""
    out, o = {}, 0
    for name, shape in param_layout():
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    assert o == theta.size
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in param_layout()])


def init_params(seed, zero_output=True):
    """Seeded initial parameters: graph normalization alpha = gamma = 1,
    beta = 0; weights uniform in +-1/sqrt(fan_in), biases 0; with zero_output
    the last edge layer is zero, so the network starts at L_pred = L_IC."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in param_layout():
        if name in ("gn_alpha", "gn_gamma"):
            d[name] = np.ones(shape)
        elif name == "gn_beta" or "_b" in name:
            d[name] = np.zeros(shape)
        else:
            fan_in = shape[-1] if len(shape) == 2 else HIDDEN
            d[name] = rng.uniform(-1.0, 1.0, shape) / np.sqrt(fan_in)
    if zero_output:
        d["e2_w2"] = np.zeros(HIDDEN)
        d["e2_b2"] = np.zeros(1)
    return pack(d)


# ------------------------------------------------------------------ graph

class Graph:
    """Edges of L's pattern (rows r >= cols c, CSR order of L) and the full
    symmetric A as COO triples for the loss."""

    def __init__(self, A, L):
        arp, aci, aval = (np.asarray(a) for a in A)
        lrp, lci, lval = (np.asarray(a) for a in L)
        self.n = n = len(arp) - 1
        self.A = (arp.astype(np.int64), aci.astype(np.int64), aval.astype(np.float64))
        self.r = np.repeat(np.arange(n), np.diff(lrp))
        self.c = lci.astype(np.int64)
        self.Lic = lval.astype(np.float64)
        self.diag = self.r == self.c
        # A's entries on L's pattern (the edge inputs)
        a_row = np.repeat(np.arange(n), np.diff(arp))
        amap = {(int(i), int(j)): v for i, j, v in zip(a_row, aci, aval)}
        self.a_edge = np.array([amap[(int(i), int(j))] for i, j in zip(self.r, self.c)], np.float64)
        self.a_rows = a_row
        # incident edges per node: an edge counts at its row and at its column,
        # the diagonal once
        self.deg_inc = (np.bincount(self.r, minlength=n) + np.bincount(self.c[~self.diag], minlength=n)).astype(
            np.float64)


def node_features(g: Graph):
    """x in R^{n x 9} (supplementary Table 2)."""
    arp, aci, aval = g.A
    n = g.n
    deg = np.diff(arp).astype(np.float64) - 1.0  # neighbours (the diagonal is stored)
    x = np.zeros((n, NODE_DIM))
    for i in range(n):
        cols = aci[arp[i]:arp[i + 1]]
        vals = aval[arp[i]:arp[i + 1]]
        off = cols != i
        nd = deg[cols[off]]
        x[i, 0] = deg[i]
        if nd.size:
            x[i, 1] = nd.max()
            x[i, 2] = nd.min()
            x[i, 3] = nd.mean()
            x[i, 4] = nd.var()
        aii = abs(vals[~off][0])
        x[i, 5] = aii / np.abs(vals).sum()
        x[i, 6] = np.abs(vals[off]).max() / aii if off.any() else 0.0
        x[i, 7] = np.sin(np.pi * i / n)
        x[i, 8] = np.cos(np.pi * i / n)
    return x


def edge_scale(g: Graph):
    """Standard deviation of the stored entries of tril(A) (population)."""
    return float(np.std(g.a_edge))


# ------------------------------------------------------- COO algorithms

def coo_matvec(rows, cols, vals, z):
    """Algorithm 1: gather z by column, scale by the values, scatter-sum by row."""
    zs = z[cols]
    return np.bincount(rows, weights=vals * zs, minlength=z.size)


def coo_llt_matvec(rows, cols, vals, z):
    """Algorithm 2: L L^T z with L as COO (rows, cols, vals): gather z by row,
    scatter-sum by column (L^T z), gather that by column, scatter-sum by row."""
    zs = z[rows]
    u = np.bincount(cols, weights=vals * zs, minlength=z.size)
    us = u[cols]
    return np.bincount(rows, weights=vals * us, minlength=z.size)


# ---------------------------------------------------------------- network

def _agg(g: Graph, e):
    """Sum over the edges incident to each node (undirected, diagonal once)."""
    s = np.bincount(g.r, weights=e, minlength=g.n)
    s += np.bincount(g.c[~g.diag], weights=e[~g.diag], minlength=g.n)
    return s


def forward(g: Graph, theta, x=None, keep=False):
    """Network output g_k per edge (and the intermediates when keep)."""
    P = unpack(theta)
    if x is None:
        x = node_features(g)
    s = edge_scale(g)
    e0 = g.a_edge / s
    mu = x.mean(0)
    d = x - P["gn_alpha"] * mu
    sd = np.sqrt((d * d).mean(0) + GN_EPS)
    h = P["gn_gamma"] * d / sd + P["gn_beta"]
    cache = dict(x=x, mu=mu, d=d, sd=sd, s=s, e0=e0, hs=[h], ins=[], qs=[], nins=[], Qs=[], es=[])
    e_prev = None
    for b in range(3):
        ein = e0[:, None] if b == 0 else np.stack([e0, e_prev], 1)
        inp = np.concatenate([ein, h[g.r], h[g.c]], 1)
        q = np.tanh(inp @ P[f"e{b}_W1"].T + P[f"e{b}_b1"])
        e = q @ P[f"e{b}_w2"] + P[f"e{b}_b2"][0]
        cache["ins"].append(inp)
        cache["qs"].append(q)
        cache["es"].append(e)
        if b < 2:
            sm = _agg(g, e)
            nin = np.concatenate([h, sm[:, None], (sm / g.deg_inc)[:, None]], 1)
            Q = np.tanh(nin @ P[f"n{b}_W1"].T + P[f"n{b}_b1"])
            h = Q @ P[f"n{b}_W2"].T + P[f"n{b}_b2"]
            cache["nins"].append(nin)
            cache["Qs"].append(Q)
            cache["hs"].append(h)
        e_prev = e
    return (e_prev, cache) if keep else e_prev


def corrected_factor(g: Graph, out, scale):
    """Eq. 2 with the diagonal kept positive (see the module notes)."""
    return np.where(g.diag, g.Lic * np.exp(out / 2.0), g.Lic + np.sqrt(scale) * out)


def predict(g: Graph, theta, x=None):
    """L_pred values on L's pattern."""
    out, cache = forward(g, theta, x, keep=True)
    return corrected_factor(g, out, cache["s"])


def loss(g: Graph, Lval, z):
    """||L L^T z - A z||^2 / ||A z||^2 (Eq. 5, one probe, normalized)."""
    arp, aci, aval = g.A
    az = coo_matvec(g.a_rows, aci, aval, z)
    llz = coo_llt_matvec(g.r, g.c, Lval, z)
    r = llz - az
    return float(r @ r / (az @ az))


def loss_and_grad_L(g: Graph, Lval, z):
    """Eq. 5's loss for probe z and its derivative with respect to L's stored
    values: with u = L^T z and r = L L^T z - A z, d||r||^2 / dL_ab =
    2 (r_a u_b + z_a (L^T r)_b), divided by ||A z||^2."""
    arp, aci, aval = g.A
    az = coo_matvec(g.a_rows, aci, aval, z)
    u = np.bincount(g.c, weights=Lval * z[g.r], minlength=g.n)      # L^T z
    llz = np.bincount(g.r, weights=Lval * u[g.c], minlength=g.n)    # L u
    r = llz - az
    den = az @ az
    lval = float(r @ r / den)
    ltr = np.bincount(g.c, weights=Lval * r[g.r], minlength=g.n)    # L^T r
    dL = 2.0 / den * (r[g.r] * u[g.c] + z[g.r] * ltr[g.c])
    return lval, dL


def loss_and_grad(g: Graph, theta, z, x=None):
    """(loss, d loss / d theta) with the backward pass written out."""
    P = unpack(theta)
    out, C = forward(g, theta, x, keep=True)
    Lval = corrected_factor(g, out, C["s"])
    lval, dL = loss_and_grad_L(g, Lval, z)
    dout = np.where(g.diag, dL * Lval / 2.0, dL * np.sqrt(C["s"]))

    G = {name: np.zeros(shape) for name, shape in param_layout()}
    de = dout
    dh_next = np.zeros((g.n, NODE_DIM))  # gradient reaching the node state entering the current block
    for b in (2, 1, 0):
        # edge updater of block b
        q, inp = C["qs"][b], C["ins"][b]
        G[f"e{b}_b2"][0] += de.sum()
        G[f"e{b}_w2"] += q.T @ de
        dp = np.outer(de, P[f"e{b}_w2"]) * (1.0 - q * q)
        G[f"e{b}_W1"] += dp.T @ inp
        G[f"e{b}_b1"] += dp.sum(0)
        dinp = dp @ P[f"e{b}_W1"]
        ein_w = EDGE_IN[b]
        dh = dh_next.copy()
        np.add.at(dh, g.r, dinp[:, ein_w:ein_w + NODE_DIM])
        np.add.at(dh, g.c, dinp[:, ein_w + NODE_DIM:])
        de_prev = dinp[:, 1] if b > 0 else None  # the skip input's current-e part
        if b == 0:
            dh0 = dh
            break
        # node updater of block b-1 produced the node state used here
        nb = b - 1
        Q, nin = C["Qs"][nb], C["nins"][nb]
        G[f"n{nb}_b2"] += dh.sum(0)
        G[f"n{nb}_W2"] += dh.T @ Q
        dP = (dh @ P[f"n{nb}_W2"]) * (1.0 - Q * Q)
        G[f"n{nb}_W1"] += dP.T @ nin
        G[f"n{nb}_b1"] += dP.sum(0)
        dnin = dP @ P[f"n{nb}_W1"]
        dh_next = dnin[:, :NODE_DIM]
        ds = dnin[:, NODE_DIM] + dnin[:, NODE_DIM + 1] / g.deg_inc
        # the aggregation gathered the edges of block b-1
        de = de_prev + ds[g.r] + np.where(g.diag, 0.0, ds[g.c])
    # graph normalization: h = gamma * d / sd + beta, d = x - alpha * mu
    x, mu, d, sd = C["x"], C["mu"], C["d"], C["sd"]
    n = g.n
    G["gn_beta"] += dh0.sum(0)
    G["gn_gamma"] += (dh0 * d / sd).sum(0)
    dd = dh0 * P["gn_gamma"] / sd
    dsd = (dh0 * P["gn_gamma"] * d).sum(0) * (-1.0 / sd ** 2)
    dd += dsd * d / (n * sd)
    G["gn_alpha"] += -(dd.sum(0)) * mu
    return lval, pack(G)


# ----------------------------------------------------------------- Adam

def adam_step(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), step t >= 1; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
