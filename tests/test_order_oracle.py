"""Pins of the multicolour-ordering oracle (oracle/order.py) on the CPU."""

import numpy as np
import pytest

import oracle
from oracle import order as O
from synth import dense_to_csr, laplacian7, q1_elasticity


def q1(E, sigma=1.0, seed=3):
    p = q1_elasticity(E, sigma, seed)
    return (p.row_ptr, p.col, p.val)


def test_splitmix64_reference_outputs():
    # published SplitMix64 outputs: state 0 and state 1234567, first draw
    assert O.splitmix64(0) == 0xE220A8397B1DCDAF
    assert O.splitmix64(1234567) == 6457827717110365317


def test_nodes_of_q1_are_dof_triples():
    A = q1(3)
    ptr = O.nodes(A)
    n = len(A[0]) - 1
    assert np.array_equal(ptr, np.arange(0, n + 1, 3))


@pytest.mark.parametrize("E", [2, 3, 4])
def test_colouring_valid_and_greedy(E):
    A = q1(E)
    ptr = O.nodes(A)
    adj = O.node_graph(A, ptr)
    col, pr = O.greedy_colors(adj, seed=7)
    key = [(pr[v], v) for v in range(len(adj))]
    for v, nb in enumerate(adj):
        assert all(col[u] != col[v] for u in nb)               # proper colouring
        higher = [u for u in nb if key[u] > key[v]]
        # first fit in priority order: every smaller colour is taken by a
        # higher-priority neighbour, and no lower-priority neighbour decided v
        assert set(range(col[v])) <= {int(col[u]) for u in higher}
    # the 2x2x2 node blocks of the grid are cliques of the node graph
    assert col.max() + 1 >= 8


def test_colouring_of_a_path_and_a_clique():
    # path graph (tridiagonal): first fit in any order uses at most 3 colours
    T = np.diag(np.full(20, 4.0)) + np.diag(np.full(19, -1.0), 1) + np.diag(np.full(19, -1.0), -1)
    perm, col, nc = O.color_order(dense_to_csr(T), seed=1)
    assert nc <= 3 and all(col[i] != col[i + 1] for i in range(19))
    # every row of a dense matrix has the same column list: rows group into two
    # nodes of 3, which are adjacent
    D = np.full((6, 6), 1.0) + 6 * np.eye(6)
    perm, col, nc = O.color_order(dense_to_csr(D), seed=1)
    assert nc == 2 and sorted(col.tolist()) == [0, 1]


def test_permute_equals_dense_product():
    A = q1(2, 1.5, 9)
    n = len(A[0]) - 1
    perm, col, nc = O.color_order(A, seed=3)
    assert sorted(perm.tolist()) == list(range(n))
    Ap = O.permute(A, perm)
    D = np.zeros((n, n))
    for i in range(n):
        D[i, A[1][A[0][i]:A[0][i + 1]]] = A[2][A[0][i]:A[0][i + 1]]
    Dp = np.zeros((n, n))
    for i in range(n):
        Dp[i, Ap[1][Ap[0][i]:Ap[0][i + 1]]] = Ap[2][Ap[0][i]:Ap[0][i + 1]]
    assert np.array_equal(Dp, D[np.ix_(perm, perm)])
    for i in range(n):
        assert np.all(np.diff(Ap[1][Ap[0][i]:Ap[0][i + 1]]) > 0)


def test_coloured_factor_has_few_levels_and_solves_the_same_system():
    A = q1(3, 1.0, 4)
    n = len(A[0]) - 1
    perm, col, nc = O.color_order(A, seed=0)
    Ap = O.permute(A, perm)
    st, L, *_ = oracle.ic0_shifted(*Ap)
    assert st == oracle.OK
    lev, nlev = oracle.levels_lower(L[0], L[1])
    assert nlev <= 3 * nc                                       # colours x DOFs per node
    st0, L0, *_ = oracle.ic0_shifted(*A)
    assert oracle.levels_lower(L0[0], L0[1])[1] > 3 * nc         # natural order: 21E - 9 levels
    b = np.random.default_rng(1).standard_normal(n)
    r = oracle.pcg(Ap, L, oracle.transpose(*L), b[perm], rtol=1e-11)
    x = np.empty(n)
    x[perm] = r["x"]
    assert np.linalg.norm(oracle.spmv(*A, x) - b) <= 1e-10 * np.linalg.norm(b)


def test_laplacian_single_row_nodes():
    A = laplacian7(5, 4, 3)
    ptr = O.nodes(A)
    # no two consecutive rows of the 7-point Laplacian share a column list
    assert np.array_equal(ptr, np.arange(len(A[0])))
    perm, col, nc = O.color_order(A, seed=2)
    adj = O.node_graph(A, ptr)
    assert all(col[u] != col[v] for v, nb in enumerate(adj) for u in nb)


# ------------------------------------------------- block multicolour order

def test_block_colouring_of_a_block_grid_is_the_parity_pattern():
    """Mesh blocks numbered like the nodes (x fastest): first fit in id order
    on the 27-neighbour block grid gives the 8-colour parity pattern, colour
    determined by (bx mod 2, by mod 2, bz mod 2)."""
    from synth import node_blocks
    E, bs = 7, 2
    A = q1(E)
    blk, nblk = node_blocks(E, bs)
    perm, col, nc = O.block_color_order(A, blk, nblk=nblk)
    nb = -(-(E + 1) // bs)
    b = np.arange(nblk)
    par = (b % nb) % 2 + 2 * (((b // nb) % nb) % 2) + 4 * ((b // (nb * nb)) % 2)
    assert nc == 8
    for p in range(8):  # one colour per parity class, and all different
        assert len(set(col[par == p].tolist())) == 1
    assert len({int(col[par == p][0]) for p in range(8)}) == 8


def test_block_colouring_of_a_path_alternates():
    """One block per row of a tridiagonal matrix: the block graph is a path, so
    first fit in id order alternates two colours."""
    A = dense_to_csr(np.diag(np.full(9, 4.0)) + np.diag(np.full(8, -1.0), 1) + np.diag(np.full(8, -1.0), -1))
    perm, col, nc = O.block_color_order(A, np.arange(9))
    assert nc == 2 and np.array_equal(col, np.arange(9) % 2)
    assert np.array_equal(perm, np.r_[np.arange(0, 9, 2), np.arange(1, 9, 2)])


@pytest.mark.parametrize("bs", [2, 3])
def test_block_order_layout_and_colouring(bs):
    from synth import node_blocks
    E = 4
    A = q1(E)
    blk, nblk = node_blocks(E, bs)
    perm, col, nc = O.block_color_order(A, blk, nblk=nblk)
    n = len(A[0]) - 1
    assert sorted(perm.tolist()) == list(range(n))
    adj = O.block_graph(A, blk, nblk)
    for b, nb in enumerate(adj):
        assert all(col[c] != col[b] for c in nb)                # proper colouring of the blocks
        assert all(b in adj[c] for c in nb)                     # symmetric pattern, symmetric graph
    key = [(int(col[blk[r]]), int(blk[r]), int(r)) for r in perm]
    assert key == sorted(key)                                   # rows by (colour, block, row)
    # a node's three rows stay together and in order
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    assert np.all(pos[1::3] == pos[0::3] + 1) and np.all(pos[2::3] == pos[0::3] + 2)


def test_block_order_of_a_single_block_is_the_identity():
    A = laplacian7(4, 3, 2)
    n = len(A[0]) - 1
    perm, col, nc = O.block_color_order(A, np.zeros(n, np.int64))
    assert np.array_equal(perm, np.arange(n)) and nc == 1


def test_block_ordered_factor_solves_the_same_system():
    """IC(0)-PCG on the block-ordered system returns the permuted solution of the
    original one (same iteration bound, same true residual)."""
    from synth import node_blocks
    E = 4
    A = q1(E)
    blk, nblk = node_blocks(E, 2)
    perm, _, _ = O.block_color_order(A, blk, nblk=nblk)
    Ap = O.permute(A, perm)
    n = len(A[0]) - 1
    b = np.random.default_rng(2).standard_normal(n)
    st, L, alpha, _, _ = oracle.ic0_shifted(*Ap)
    assert st == oracle.OK
    out = oracle.pcg(Ap, L, oracle.transpose(*L), b[perm], rtol=1e-10)
    x = np.empty(n)
    x[perm] = out["x"]
    r = b - oracle.spmv(*A, x)
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)
