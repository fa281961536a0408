"""Synthetic elasticity generator: closed forms and invariants (CPU)."""

import numpy as np
import pytest

from synth import (body_load, expected_sizes, q1_elasticity, q1_unit_stiffness,
                   rigid_body_modes, traction_loads, build_workload)


@pytest.mark.parametrize("E", [1, 2, 3, 5, 8])
def test_sizes_closed_form(E):
    p = q1_elasticity(E, 1.0, 7)
    n, nnz = expected_sizes(E)
    assert p.n == n
    assert p.nnz == nnz
    rl = np.diff(p.row_ptr)
    assert rl.max() <= 81
    # sorted columns and a diagonal in every row
    for i in range(p.n):
        c = p.col[p.row_ptr[i]:p.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
        assert i in c


def test_q1_8_matches_stated_sizes():
    p, b = build_workload("q1_8")
    assert p.n == 1944 and p.n // 3 == 648 and p.nnz == 123750
    assert b.shape == (1944,)


@pytest.mark.parametrize("E", [2, 4, 8])
def test_bitwise_symmetry(E):
    A = q1_elasticity(E, 1.5, 11).to_scipy()
    D = A - A.T
    assert D.nnz == 0 or np.all(D.data == 0)
    At = A.T.tocsr()
    At.sort_indices()
    assert np.array_equal(At.indices, A.indices)
    assert np.array_equal(At.data.view(np.uint64), A.data.view(np.uint64))


def test_unit_stiffness_rigid_modes():
    K = q1_unit_stiffness()
    assert np.array_equal(K, K.T)
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-12) == 6
    assert ev[6] > 1e-3
    # nodes of the unit cube, local a = ax + 2 ay + 4 az
    xyz = np.array([[a & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float)
    M = np.zeros((24, 6))
    for a in range(8):
        x, y, z = xyz[a]
        M[3 * a:3 * a + 3, :3] = np.eye(3)
        M[3 * a:3 * a + 3, 3] = [0, -z, y]
        M[3 * a:3 * a + 3, 4] = [z, 0, -x]
        M[3 * a:3 * a + 3, 5] = [-y, x, 0]
    assert np.abs(K @ M).max() < 1e-13


@pytest.mark.parametrize("E", [3, 6])
def test_rigid_modes_vanish_away_from_clamp(E):
    p = q1_elasticity(E, 1.0, 3)
    A = p.to_scipy()
    R = A @ rigid_body_modes(E)
    k = np.repeat(np.arange(1, E + 1), 3 * (E + 1) ** 2)
    scale = np.abs(p.val).max()
    assert np.abs(R[k >= 2]).max() < 1e-12 * scale * (E + 1)
    assert np.abs(R[k == 1]).max() > 1e-3  # the clamp breaks the invariance


@pytest.mark.parametrize("E", [1, 2, 3])
def test_spd_small(E):
    D = q1_elasticity(E, 2.0, 5).to_scipy().toarray()
    assert np.linalg.eigvalsh(D).min() > 0


def test_body_load_total():
    # total body force -E^3; the clamped layer takes half of the bottom layer's share
    for E in (2, 5, 9):
        b = body_load(E, 0.0, None)
        assert abs(b[2::3].sum() + (E ** 3 - 0.5 * E ** 2)) < 1e-9
        assert np.all(b[0::3] == 0) and np.all(b[1::3] == 0)


def test_traction_columns():
    E = 4
    B = traction_loads(E, 3, 99)
    base = body_load(E, 0.0, None)
    N1 = E + 1
    top = slice(3 * N1 * N1 * (E - 1), None)
    for c in range(3):
        t = np.random.default_rng(99 + c).standard_normal((E * E, 3))
        d = (B[:, c] - base)
        assert abs(d.sum() - t.sum()) < 1e-9  # all traction lands on the top nodes
        assert np.all(d[:3 * N1 * N1 * (E - 1)] == 0)
        assert np.abs(d[top]).max() > 0


def test_modulus_lognormal_seeded():
    p1 = q1_elasticity(3, 2.0, 1003)
    p2 = q1_elasticity(3, 2.0, 1003)
    assert np.array_equal(p1.val, p2.val)
    z = np.random.default_rng(1003).standard_normal(27)
    assert np.allclose(p1.modulus, np.exp(2.0 * z))
