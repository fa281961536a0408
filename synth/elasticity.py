"""Synthetic 3D linear-elasticity stiffness matrices (trilinear hexahedra).

Stand-in for the paper's 3D static structural FE matrices (Datasets section):
those matrices are not available here, so the solver is exercised on a
textbook Q1 finite-element discretisation of isotropic linear elasticity on a
box of unit cubes, clamped on the face z = 0.

Mesh and numbering
  * E^3 unit cubes, nodes (i, j, k) with 0 <= i, j, k <= E.
  * Nodes with k = 0 are clamped and eliminated from the system.
  * Free node id = i + (E+1) * (j + (E+1) * (k-1)); DOF = 3*node + d,
    d = 0, 1, 2 for the x, y, z displacement.
  * Element id = ex + E * (ey + E * ez). Element e has Young's modulus
    E_e = exp(sigma * N(0,1)), drawn in element-id order from
    numpy.random.default_rng(seed_A); Poisson ratio nu = 0.3 everywhere.

Element matrix
  K_e = E_e * K_unit with K_unit the 24x24 stiffness of a unit cube for E = 1,
  integrated with 2x2x2 Gauss points (exact for this integrand on cubes) and
  symmetrised as (K + K^T)/2 so that assembly gives a bitwise-symmetric A.

Pattern
  Structural: every DOF pair of two nodes that share an element is stored,
  explicit zeros included. Rows hold ascending column indices and always a
  diagonal entry. Per row at most 81 entries.

Assembly order
  Entry (n, m) sums E_e * K_unit blocks over the elements shared by nodes n
  and m in ascending element id, which is the same ordered list for (m, n);
  with K_unit exactly symmetric this makes A bitwise symmetric.
"""

from __future__ import annotations

import dataclasses
import numpy as np

NU = 0.3

# Synthetic workloads by name: element grid E, lognormal sigma of Young's
# modulus, right-hand sides, and the seeds (seed_A draws the element moduli,
# seed_b the right-hand side(s)).
WORKLOADS = {
    "q1_8": dict(E=8, sigma=1.0, nrhs=1, rhs="body+noise", seed_A=1000, seed_b=2000),
    "q1_40": dict(E=40, sigma=1.5, nrhs=1, rhs="body+noise", seed_A=1001, seed_b=2001),
    "q1_48_block8": dict(E=48, sigma=1.0, nrhs=8, rhs="normal", seed_A=1002, seed_b=3000),
    "q1_100": dict(E=100, sigma=2.0, nrhs=1, rhs="body+noise", seed_A=1003, seed_b=2003),
    "q1_150_loads16": dict(E=150, sigma=1.5, nrhs=16, rhs="traction", seed_A=1004, seed_b=2004),
}


def expected_sizes(E: int) -> tuple[int, int]:
    """Closed forms for the clamped box: n = 3 (E+1)^2 E and
    nnz(A) = 9 (3E+1)^2 (3E-2) (all in-bounds 27-point node neighbours)."""
    return 3 * (E + 1) ** 2 * E, 9 * (3 * E + 1) ** 2 * (3 * E - 2)


def q1_unit_stiffness(nu: float = NU) -> np.ndarray:
    """24x24 stiffness of a unit cube, E = 1, local node a = ax + 2 ay + 4 az,
    local DOF 3a + d. Voigt order (xx, yy, zz, yz, xz, xy), engineering shear."""
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    g = 1.0 / np.sqrt(3.0)
    sgn = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                    for a in range(8)], dtype=np.float64)
    K = np.zeros((24, 24))
    for xi in (-g, g):
        for eta in (-g, g):
            for zeta in (-g, g):
                # derivatives wrt reference coordinates, then x = (xi+1)/2
                fx = 1 + sgn[:, 0] * xi
                fy = 1 + sgn[:, 1] * eta
                fz = 1 + sgn[:, 2] * zeta
                dxi = sgn[:, 0] * fy * fz / 8.0
                deta = sgn[:, 1] * fx * fz / 8.0
                dzeta = sgn[:, 2] * fx * fy / 8.0
                dx, dy, dz = 2 * dxi, 2 * deta, 2 * dzeta
                B = np.zeros((6, 24))
                for a in range(8):
                    c = 3 * a
                    B[0, c] = dx[a]
                    B[1, c + 1] = dy[a]
                    B[2, c + 2] = dz[a]
                    B[3, c + 1] = dz[a]
                    B[3, c + 2] = dy[a]
                    B[4, c] = dz[a]
                    B[4, c + 2] = dx[a]
                    B[5, c] = dy[a]
                    B[5, c + 1] = dx[a]
                K += B.T @ D @ B * (1.0 / 8.0)  # det J = 1/8, unit weights
    return 0.5 * (K + K.T)


@dataclasses.dataclass
class ElasticityProblem:
    E: int
    sigma: float
    seed_A: int
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]
    modulus: np.ndarray  # float64 [E^3] element Young's moduli

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


# 27 node offsets (dk, dj, di) in ascending order of the neighbour's node id.
_OFFS = np.array([(di, dj, dk) for dk in (-1, 0, 1) for dj in (-1, 0, 1) for di in (-1, 0, 1)],
                 dtype=np.int64)
# 8 candidate elements around a node, ascending element id: (cz, cy, cx) lexicographic,
# element = (i-1+cx, j-1+cy, k-1+cz).
_CANDS = np.array([(cx, cy, cz) for cz in (0, 1) for cy in (0, 1) for cx in (0, 1)],
                  dtype=np.int64)


def _block_table(Ku: np.ndarray):
    """For every (offset, candidate) pair, the local node numbers of the centre node
    (a) and of the neighbour (b) in that candidate element, or -1 when the
    neighbour is not a vertex of the candidate element."""
    tab = np.full((27, 8, 2), -1, dtype=np.int64)
    for o, (di, dj, dk) in enumerate(_OFFS):
        for c, (cx, cy, cz) in enumerate(_CANDS):
            ax, ay, az = 1 - cx, 1 - cy, 1 - cz
            bx, by, bz = ax + di, ay + dj, az + dk
            if 0 <= bx <= 1 and 0 <= by <= 1 and 0 <= bz <= 1:
                tab[o, c, 0] = ax + 2 * ay + 4 * az
                tab[o, c, 1] = bx + 2 * by + 4 * bz
    return tab


def q1_elasticity(E: int, sigma: float, seed_A: int, nu: float = NU,
                  chunk_layers: int = 8) -> ElasticityProblem:
    """Assemble the clamped Q1 elasticity matrix as CSR (see module docstring)."""
    if E < 1:
        raise ValueError("E must be >= 1")
    rng = np.random.default_rng(seed_A)
    modulus = np.exp(sigma * rng.standard_normal(E ** 3))
    Ku = q1_unit_stiffness(nu)
    tab = _block_table(Ku)
    N1 = E + 1
    nn = N1 * N1 * E
    n = 3 * nn

    # per node: valid neighbour offsets and row lengths
    ii = np.arange(N1)
    # valid offsets per node factorise over the axes
    vx = np.stack([(ii + d >= 0) & (ii + d <= E) for d in (-1, 0, 1)], axis=1)          # [N1,3]
    kk = np.arange(1, E + 1)
    vz = np.stack([(kk + d >= 1) & (kk + d <= E) for d in (-1, 0, 1)], axis=1)          # [E,3]
    cnt_x = vx.sum(1)
    cnt_z = vz.sum(1)
    nb = (cnt_z[:, None, None] * cnt_x[None, :, None] * cnt_x[None, None, :]).reshape(-1)  # [nn] (k,j,i)
    row_len = np.repeat(3 * nb, 3)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)

    off_node = _OFFS[:, 0] + N1 * (_OFFS[:, 1] + N1 * _OFFS[:, 2])  # [27]

    for k0 in range(1, E + 1, chunk_layers):
        k1 = min(E + 1, k0 + chunk_layers)
        K_, J_, I_ = np.meshgrid(np.arange(k0, k1), np.arange(N1), np.arange(N1), indexing="ij")
        I_ = I_.reshape(-1); J_ = J_.reshape(-1); K_ = K_.reshape(-1)
        node = I_ + N1 * (J_ + N1 * (K_ - 1))
        m = node.shape[0]
        # neighbour validity [m,27]
        ni = I_[:, None] + _OFFS[None, :, 0]
        nj = J_[:, None] + _OFFS[None, :, 1]
        nk = K_[:, None] + _OFFS[None, :, 2]
        valid = (ni >= 0) & (ni <= E) & (nj >= 0) & (nj <= E) & (nk >= 1) & (nk <= E)
        blocks = np.zeros((m, 27, 3, 3))
        for c, (cx, cy, cz) in enumerate(_CANDS):
            ex = I_ - 1 + cx
            ey = J_ - 1 + cy
            ez = K_ - 1 + cz
            ein = (ex >= 0) & (ex < E) & (ey >= 0) & (ey < E) & (ez >= 0) & (ez < E)
            eid = np.where(ein, ex + E * (ey + E * ez), 0)
            w = np.where(ein, modulus[eid], 0.0)
            for o in range(27):
                a, b = tab[o, c]
                if a < 0:
                    continue
                kb = Ku[3 * a:3 * a + 3, 3 * b:3 * b + 3]
                # add only where the element exists, so the sequence of additions
                # is exactly the shared elements in ascending id
                upd = blocks[:, o] + w[:, None, None] * kb[None]
                blocks[:, o] = np.where(ein[:, None, None], upd, blocks[:, o])
        # CSR order inside row (node, d): valid offsets ascending, then d'
        vals = np.transpose(blocks, (0, 2, 1, 3))  # [m, d, o, d']
        mask = np.broadcast_to(valid[:, None, :, None], vals.shape)
        cols = 3 * (node[:, None, None, None] + off_node[None, None, :, None]) + \
            np.arange(3)[None, None, None, :]
        cols = np.broadcast_to(cols, vals.shape)
        s = int(row_ptr[3 * node[0]])
        e = int(row_ptr[3 * (node[-1] + 1)])
        val[s:e] = vals[mask]
        col[s:e] = cols[mask].astype(np.int32)
    return ElasticityProblem(E=E, sigma=sigma, seed_A=seed_A, row_ptr=row_ptr, col=col,
                             val=val, modulus=modulus)


def _incident_counts(E: int) -> np.ndarray:
    """Number of elements around each free node, node order."""
    cx = np.full(E + 1, 2.0)
    cx[0] = cx[E] = 1.0
    cz = np.full(E, 2.0)
    cz[E - 1] = 1.0  # k = E (top face); k = 1..E-1 interior in z
    return (cz[:, None, None] * cx[None, :, None] * cx[None, None, :]).reshape(-1)


def body_load(E: int, noise_std: float = 0.1, seed_b: int | None = None) -> np.ndarray:
    """Consistent nodal load of the unit body force (0, 0, -1): each element
    passes 1/8 of its volume to each vertex. Optional i.i.d. N(0, noise_std^2)
    noise on every free DOF from default_rng(seed_b)."""
    nn = (E + 1) ** 2 * E
    b = np.zeros(3 * nn)
    b[2::3] = -_incident_counts(E) / 8.0
    if seed_b is not None and noise_std > 0:
        rng = np.random.default_rng(seed_b)
        b = b + rng.normal(0.0, noise_std, 3 * nn)
    return b


def traction_loads(E: int, nrhs: int, seed_b: int) -> np.ndarray:
    """Load cases: column c is the body load plus a random surface traction on
    the top face z = E: per top quad a traction t ~ N(0, I_3) drawn from
    default_rng(seed_b + c), a quarter to each of its four vertices.
    Returns an (n, nrhs) C-contiguous array."""
    N1 = E + 1
    nn = N1 * N1 * E
    out = np.empty((3 * nn, nrhs))
    base = body_load(E, 0.0, None)
    qy, qx = np.meshgrid(np.arange(E), np.arange(E), indexing="ij")
    qx = qx.reshape(-1); qy = qy.reshape(-1)
    top = N1 * N1 * (E - 1)
    for c in range(nrhs):
        t = np.random.default_rng(seed_b + c).standard_normal((E * E, 3))
        f = np.zeros((nn, 3))
        for ax in (0, 1):
            for ay in (0, 1):
                nodes = top + (qx + ax) + N1 * (qy + ay)
                np.add.at(f, nodes, 0.25 * t)
        out[:, c] = base + f.reshape(-1)
    return np.ascontiguousarray(out)


def rigid_body_modes(E: int) -> np.ndarray:
    """Six rigid-body fields (3 translations, 3 infinitesimal rotations) sampled
    at the free nodes, shape (n, 6). A Q1 element annihilates them, so A m
    vanishes on rows of nodes whose element neighbourhood avoids the clamped
    layer (k >= 2)."""
    N1 = E + 1
    K_, J_, I_ = np.meshgrid(np.arange(1, E + 1), np.arange(N1), np.arange(N1), indexing="ij")
    x = I_.reshape(-1).astype(float)
    y = J_.reshape(-1).astype(float)
    z = K_.reshape(-1).astype(float)
    nn = x.shape[0]
    M = np.zeros((3 * nn, 6))
    for d in range(3):
        M[d::3, d] = 1.0
    # rotations about x, y, z: u = w x r
    M[1::3, 3] = -z; M[2::3, 3] = y
    M[0::3, 4] = z;  M[2::3, 4] = -x
    M[0::3, 5] = -y; M[1::3, 5] = x
    return M


def node_blocks(E: int, bs: int) -> tuple[np.ndarray, int]:
    """Partition of the rows of the E^3 clamped Q1 matrix into mesh blocks of
    bs x bs x bs nodes (a node's 3 rows in one block): block id per row
    (int32) and the block count. Input structure only (like coordinates)."""
    N1 = E + 1
    nb = -(-N1 // bs)
    nbz = -(-E // bs)
    node = np.arange(N1 * N1 * E)
    I = node % N1
    J = (node // N1) % N1
    K = node // (N1 * N1)  # free layers 1..E, numbered from 0
    b = (I // bs) + nb * ((J // bs) + nb * (K // bs))
    return np.repeat(b, 3).astype(np.int32), int(nb * nb * nbz)


def build_workload(name: str, with_rhs: bool = True):
    """Matrix and right-hand side(s) of a named synthetic workload.
    Returns (ElasticityProblem, B) with B of shape (n,) or (n, nrhs)."""
    w = WORKLOADS[name]
    prob = q1_elasticity(w["E"], w["sigma"], w["seed_A"])
    if not with_rhs:
        return prob, None
    E = w["E"]
    if w["rhs"] == "body+noise":
        B = body_load(E, 0.1, w["seed_b"])
    elif w["rhs"] == "traction":
        B = traction_loads(E, w["nrhs"], w["seed_b"])
    elif w["rhs"] == "normal":
        B = np.random.default_rng(w["seed_b"]).standard_normal((prob.n, w["nrhs"]))
    else:
        raise ValueError(w["rhs"])
    return prob, B
