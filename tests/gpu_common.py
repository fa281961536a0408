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


def ulp_perturbed(A, seed):
    """A with every stored value moved by one unit in the last place, up or
    down at random, keeping A exactly symmetric (the upper triangle is drawn,
    the lower mirrors it): a rounding-sized change that reaches every product
    A p of a Krylov iteration."""
    rp, ci, v = (np.asarray(a) for a in A)
    n = len(rp) - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    lo, hi = np.minimum(rows, ci).astype(np.int64), np.maximum(rows, ci).astype(np.int64)
    # one sign per unordered pair (i, j): a hash of the pair, the same from both sides
    with np.errstate(over="ignore"):
        h = lo * np.int64(0x27D4EB2F165667C5) + hi * np.int64(0x165667B19E3779F9) + np.int64(seed)
    up = ((h >> 29) & 1).astype(bool)
    vp = np.where(up, np.nextafter(v, np.inf), np.nextafter(v, -np.inf))
    return rp, ci, vp


def rounding_bars(A, b, k, kind, seed=7, factor=10.0):
    """Tolerances of a GPU solve against the oracle derived from the iteration's
    own sensitivity to rounding: the oracle run on ulp_perturbed(A) against the
    oracle on A, (i) x after the same k steps, relative difference d, (ii) the
    iterations to rtol 1e-8, difference dk. Returns (max(factor * d, 1e-12),
    max(1, 2 * dk)): the GPU may differ from the oracle by `factor` times what
    a one-ulp change of every entry of A causes (its summation orders differ
    from the oracle's by a few ulps per sum), and stop within twice the
    perturbed run's shift of the stopping step."""
    Ap = ulp_perturbed(A, seed)
    x0 = oracle.pcg_simple(A, b, kind, rtol=0.0, max_iter=k, max_replace=0)["x"]
    x1 = oracle.pcg_simple(Ap, b, kind, rtol=0.0, max_iter=k, max_replace=0)["x"]
    n = len(b)
    k0 = oracle.pcg_simple(A, b, kind, rtol=1e-8, max_iter=20 * n)["iters"]
    k1 = oracle.pcg_simple(Ap, b, kind, rtol=1e-8, max_iter=20 * n)["iters"]
    return max(factor * relerr(x1, x0), 1e-12), max(1, 2 * abs(k1 - k0))


def stop_agrees(k, k0, hist, rtol=1e-8, factor=2.0):
    """A stopping step k agrees with the oracle's k0 when they differ by at
    most one, or when the oracle's own recurrence residual (hist[j] =
    ||r_j|| / ||b||) stays within `factor` * rtol at every step between them:
    near rtol the recurrence residual moves by tens of percent from one step
    to the next, so two runs whose iterates differ only by rounding may cross
    rtol anywhere on such a plateau."""
    if abs(k - k0) <= 1:
        return True
    return all(hist[j] <= factor * rtol for j in range(min(k, k0), max(k, k0) + 1) if j < len(hist))
