"""Shared helpers of the GPU parity tests (inputs from synth, expectations from
the oracle only)."""

from __future__ import annotations

import functools

import numpy as np

import oracle
from synth import build_workload, dense_to_csr, laplacian7, q1_elasticity, tridiagonal_spd


@functools.lru_cache(maxsize=None)
def workload_problem(name):
    prob, b = build_workload(name)
    return prob, b


@functools.lru_cache(maxsize=None)
def oracle_factor(key):
    """Oracle IC(0) (with the shift rule) of a named test matrix."""
    A = named_matrix(key)
    st, L, alpha, restarts, mp = oracle.ic0_shifted(*A)
    assert st == oracle.OK
    U = oracle.transpose(*L)
    return A, L, U, alpha


def random_lower_pattern(n, density, seed):
    """Random lower-triangular pattern with a dominant diagonal (ragged rows)."""
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        k = rng.binomial(i, density) if i > 0 else 0
        c = np.sort(rng.choice(i, size=k, replace=False)) if k else np.zeros(0, int)
        rows.extend([i] * (k + 1))
        cols.extend(list(c) + [i])
    rows = np.asarray(rows); cols = np.asarray(cols)
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    vals = rng.uniform(-1, 1, cols.shape[0])
    diag = cols == rows
    vals[diag] = 1.0 + rng.uniform(0, 1, diag.sum()) * 4
    return rp, cols.astype(np.int32), vals


@functools.lru_cache(maxsize=None)
def named_matrix(key):
    """SPD test matrices by name (CSR numpy triple)."""
    if key.startswith("w:"):
        p, _ = workload_problem(key[2:])
        return p.row_ptr, p.col, p.val
    if key.startswith("q1e"):
        E, sigma = key[3:].split("s")
        p = q1_elasticity(int(E), float(sigma), 77)
        return p.row_ptr, p.col, p.val
    if key == "lap7":
        return laplacian7(12, 9, 7)
    if key == "tridiag":
        return dense_to_csr(tridiagonal_spd(300, seed=3))
    if key == "kershaw":
        from synth import kershaw4
        return dense_to_csr(kershaw4())
    raise KeyError(key)


def relerr(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
