"""Small seeded test matrices in CSR form (row_ptr int64, col int32, val float64)."""

from __future__ import annotations

import numpy as np


def dense_to_csr(M: np.ndarray, keep_zeros_pattern: np.ndarray | None = None):
    """CSR of a dense matrix. The pattern is the nonzeros of M, or the given
    boolean pattern (explicit zeros kept) when supplied. Diagonal always kept."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    pat = (M != 0) if keep_zeros_pattern is None else np.asarray(keep_zeros_pattern, bool)
    pat = pat | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(pat)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, cols.astype(np.int32), M[rows, cols].copy()


def tridiagonal_spd(n: int, seed: int = 0):
    """Random diagonally dominant SPD tridiagonal matrix (dense)."""
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, 1.0, n - 1)
    d = 2.5 + rng.uniform(0.0, 1.0, n)
    M = np.diag(d) + np.diag(off, -1) + np.diag(off, 1)
    return M


def dense_spd(n: int, seed: int = 0, cond: float = 100.0):
    """Random dense SPD matrix with condition number about cond."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    M = (Q * lam) @ Q.T
    return 0.5 * (M + M.T)


def spectrum_spd(n: int, eigenvalues, seed: int = 0):
    """Dense SPD A = Q diag(lam) Q^T whose eigenvalues take only the listed
    values (each value repeated over a random subset of the n slots)."""
    rng = np.random.default_rng(seed)
    eigenvalues = np.asarray(eigenvalues, dtype=np.float64)
    k = eigenvalues.shape[0]
    lam = np.concatenate([eigenvalues, eigenvalues[rng.integers(0, k, n - k)]])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    M = (Q * lam) @ Q.T
    return 0.5 * (M + M.T)


def banded_spd(n: int, bw: int, seed: int = 0):
    """Random SPD band matrix with full band (half bandwidth bw), diagonally dominant."""
    rng = np.random.default_rng(seed)
    M = np.zeros((n, n))
    for k in range(1, bw + 1):
        v = rng.uniform(-1.0, 1.0, n - k)
        M += np.diag(v, -k) + np.diag(v, k)
    M += np.diag(2.0 * bw + 1.0 + rng.uniform(0, 1, n))
    return M


def kershaw4():
    """A 4x4 SPD matrix on which incomplete Cholesky with zero fill breaks down:
    exact Cholesky pivots are 3, 5/3, 3/5, 1/3, but the zero-fill factor's last
    squared pivot is 3 - 4/3 - 20/3 = -5."""
    return np.array([[3.0, -2.0, 0.0, 2.0],
                     [-2.0, 3.0, -2.0, 0.0],
                     [0.0, -2.0, 3.0, -2.0],
                     [2.0, 0.0, -2.0, 3.0]])


def laplacian7(nx: int, ny: int, nz: int):
    """7-point finite-difference Laplacian (Dirichlet) on an nx*ny*nz grid, CSR."""
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    for (dz, dy, dx) in [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]:
        z0, z1 = max(0, -dz), nz - max(0, dz)
        y0, y1 = max(0, -dy), ny - max(0, dy)
        x0, x1 = max(0, -dx), nx - max(0, dx)
        src = idx[z0:z1, y0:y1, x0:x1].reshape(-1)
        dst = idx[z0 + dz:z1 + dz, y0 + dy:y1 + dy, x0 + dx:x1 + dx].reshape(-1)
        rows.append(src); cols.append(dst)
        vals.append(np.full(src.shape[0], 6.0 if (dx, dy, dz) == (0, 0, 0) else -1.0))
    rows = np.concatenate(rows); cols = np.concatenate(cols); vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    return np.cumsum(row_ptr), cols.astype(np.int32), vals
