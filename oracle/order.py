"""Oracle (test infrastructure only) of the multicolour ordering applied as a
symmetric permutation before the factorization.

The paper names the triangular solves as the dominant added cost and points
to a layout of the preconditioner with more parallelism as the next step
(supplementary Additional Results). This module fixes what that reordering
computes, in plain numpy and Python loops (small inputs only):

  * nodes: consecutive rows with identical column lists, cut into pieces of
    at most 3 rows (the unknowns of one mesh node);
  * node graph: u ~ v when a row of u stores a column of v (u != v);
  * priorities: SplitMix64 (Steele, Lea and Flood; Vigna's constants) of
    seed + node id, ties broken by the larger id;
  * colours: greedy first-fit in decreasing priority order, i.e. each node
    takes the smallest colour not used by its higher-priority neighbours
    (Jones-Plassmann computes exactly this colouring in parallel rounds);
  * order: nodes sorted by (colour, node id), each node's rows kept together
    and in order; perm[new row] = old row;
  * the permuted matrix P A P^T: entry (i, j) = A[perm[i], perm[j]], rows
    with ascending columns;
  * block multicolour: for a caller's partition of the rows into blocks, the
    block graph (b ~ c when a row of b stores a column of c) coloured first
    fit in block id order, rows sorted by (colour of their block, block, row).

Only the tests use it; it shares no code with the GPU library.
"""

from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (one step: x + golden gamma, then the
    two xor-shift-multiply rounds and a final xor-shift)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def nodes(A, gmax=3):
    """Node starts: rows grouped as consecutive runs with identical column
    lists, cut into pieces of at most gmax rows. Returns ptr (len nnodes + 1)."""
    rp, ci, _ = A
    n = len(rp) - 1
    ptr = [0]
    run_len = 1
    for i in range(1, n):
        same = (rp[i + 1] - rp[i] == rp[i] - rp[i - 1]) and \
            np.array_equal(ci[rp[i]:rp[i + 1]], ci[rp[i - 1]:rp[i]])
        if same and run_len < gmax:
            run_len += 1
        else:
            ptr.append(i)
            run_len = 1
    ptr.append(n)
    return np.asarray(ptr, np.int64)


def node_graph(A, ptr):
    """Adjacency lists of the node graph (sorted, without self)."""
    rp, ci, _ = A
    n = len(rp) - 1
    node_of = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    adj = []
    for v in range(len(ptr) - 1):
        cols = np.concatenate([ci[rp[i]:rp[i + 1]] for i in range(ptr[v], ptr[v + 1])])
        nb = np.unique(node_of[cols])
        adj.append(nb[nb != v])
    return adj


def greedy_colors(adj, seed):
    """First-fit colours in decreasing (priority, id) order."""
    m = len(adj)
    pr = [splitmix64((seed + v) & MASK64) for v in range(m)]
    order = sorted(range(m), key=lambda v: (pr[v], v), reverse=True)
    col = np.full(m, -1, np.int64)
    for v in order:
        used = {int(col[u]) for u in adj[v] if col[u] >= 0}
        c = 0
        while c in used:
            c += 1
        col[v] = c
    return col, pr


def color_order(A, seed=0):
    """(perm int32: new row -> old row, node colours, number of colours)."""
    ptr = nodes(A)
    adj = node_graph(A, ptr)
    col, _ = greedy_colors(adj, seed)
    order = sorted(range(len(adj)), key=lambda v: (col[v], v))
    perm = np.concatenate([np.arange(ptr[v], ptr[v + 1]) for v in order]).astype(np.int32)
    return perm, col, int(col.max()) + 1 if len(col) else 0


def permute(A, perm):
    """P A P^T as CSR with ascending columns."""
    rp, ci, v = A
    n = len(rp) - 1
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    out_rp = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for i in range(n):
        o = perm[i]
        c = inv[ci[rp[o]:rp[o + 1]]]
        s = np.argsort(c, kind="stable")
        cols.append(c[s])
        vals.append(v[rp[o]:rp[o + 1]][s])
        out_rp[i + 1] = out_rp[i] + len(c)
    return out_rp, np.concatenate(cols).astype(np.int32), np.concatenate(vals).astype(np.float64)


def block_graph(A, blk, nblk):
    """Adjacency lists of the block graph of a row partition blk: b ~ c when a
    row of block b stores a column of block c (b != c); sorted."""
    rp, ci, _ = A
    n = len(rp) - 1
    adj = [set() for _ in range(nblk)]
    for i in range(n):
        b = int(blk[i])
        for c in blk[ci[rp[i]:rp[i + 1]]]:
            if int(c) != b:
                adj[b].add(int(c))
    return [np.array(sorted(s), np.int64) for s in adj]


def first_fit_in_id_order(adj):
    """Sequential greedy colouring: vertex 0, 1, 2, ... each takes the smallest
    colour not used by its already coloured (lower id) neighbours."""
    col = np.full(len(adj), -1, np.int64)
    for v in range(len(adj)):
        used = {int(col[u]) for u in adj[v] if u < v}
        c = 0
        while c in used:
            c += 1
        col[v] = c
    return col


def block_color_order(A, blk, nblk=None):
    """Block multicolour order of a row partition (blk[i] = block of row i):
    the block graph coloured first-fit in block id order, rows sorted by
    (colour of their block, block, row). Returns (perm int32: new row -> old
    row, block colours, number of colours)."""
    blk = np.asarray(blk, np.int64)
    nblk = int(blk.max()) + 1 if nblk is None else int(nblk)
    adj = block_graph(A, blk, nblk)
    col = first_fit_in_id_order(adj)
    rows = np.arange(len(blk))
    perm = np.lexsort((rows, blk, col[blk])).astype(np.int32)  # last key is the primary one
    return perm, col, int(col.max()) + 1 if len(col) else 0
