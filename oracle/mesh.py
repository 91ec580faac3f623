"""Structured P1 triangulation of the unit square and element-by-element assembly.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The discretization follows the paper's finite-element setting (Sec. 2.3:
continuous Lagrange basis, mass-weighted inner products; Sec. 5.1: the Poisson
coefficient problem on the unit square).  Readings where the paper is silent:

* mesh: N x N cells, each split by the diagonal from (x_i, y_j) to
  (x_{i+1}, y_{j+1}) into a lower and an upper triangle; nodes numbered
  k(i, j) = j (N+1) + i.
* triangle t = 2 (j N + i) + s with s = 0 (lower) or 1 (upper); vertices are
  stored as (a, r, b) where r is the right-angle vertex:
      lower: (k(i,j), k(i+1,j), k(i+1,j+1)),  upper: (k(i,j), k(i,j+1), k(i+1,j+1)).
* the coefficient e^m is integrated with the one-point centroid rule, i.e.
  c_T = exp((m_a + m_r + m_b) / 3) on each triangle.
* white noise for prior draws lives at the three edge midpoints of every
  triangle (index 3 t + e, edges e0 = (a, r), e1 = (r, b), e2 = (a, b)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class Mesh:
    """Right-diagonal triangulation of [0,1]^2 with N cells per side."""

    def __init__(self, N: int):
        if N < 1:
            raise ValueError("N must be >= 1")
        self.N = N
        self.h = 1.0 / N
        self.n = (N + 1) * (N + 1)
        x = np.arange(N + 1) * self.h
        X, Y = np.meshgrid(x, x)  # X[j, i] = x_i, Y[j, i] = y_j
        self.xy = np.column_stack([X.reshape(-1), Y.reshape(-1)])
        tris = np.empty((2 * N * N, 3), dtype=np.int64)
        t = 0
        for j in range(N):
            for i in range(N):
                k00 = self.node(i, j)
                k10 = self.node(i + 1, j)
                k01 = self.node(i, j + 1)
                k11 = self.node(i + 1, j + 1)
                tris[t] = (k00, k10, k11)      # lower triangle, right angle at (i+1, j)
                tris[t + 1] = (k00, k01, k11)  # upper triangle, right angle at (i, j+1)
                t += 2
        self.tris = tris
        jj = np.arange(self.n) // (N + 1)
        # Dirichlet nodes of the state: bottom (y = 0) and top (y = 1) edges.
        self.dirichlet = (jj == 0) | (jj == N)
        self.free = ~self.dirichlet
        # boundary edges of the whole square (for the Robin mass)
        edges = []
        for i in range(N):
            edges.append((self.node(i, 0), self.node(i + 1, 0)))
            edges.append((self.node(i, N), self.node(i + 1, N)))
        for j in range(N):
            edges.append((self.node(0, j), self.node(0, j + 1)))
            edges.append((self.node(N, j), self.node(N, j + 1)))
        self.bedges = np.array(edges, dtype=np.int64)

    def node(self, i: int, j: int) -> int:
        return j * (self.N + 1) + i

    # -- per-triangle geometry ------------------------------------------------
    def tri_geometry(self, t: int):
        """Area and the 3x2 matrix of basis-function gradients of triangle t.

        With D = [P1 - P0; P2 - P0] the affine map is x = P0 + D^T xi, so
        grad(phi_1) and grad(phi_2) are the columns of D^{-1} and
        grad(phi_0) = -(grad(phi_1) + grad(phi_2)).
        """
        P = self.xy[self.tris[t]]
        D = np.array([P[1] - P[0], P[2] - P[0]])
        area = 0.5 * abs(np.linalg.det(D))
        Dinv = np.linalg.inv(D)
        g1, g2 = Dinv[:, 0], Dinv[:, 1]
        return area, np.array([-(g1 + g2), g1, g2])


def _assemble(mesh: Mesh, Ae: np.ndarray) -> sp.csr_matrix:
    """Sum element matrices Ae[t] (shape (ntri, 3, 3)) into an n x n sparse matrix."""
    v = mesh.tris
    rows = np.repeat(v, 3, axis=1).reshape(-1)      # v[t,a] repeated over b
    cols = np.tile(v, (1, 3)).reshape(-1)           # v[t,b] for each a
    return sp.csr_matrix((Ae.reshape(-1), (rows, cols)), shape=(mesh.n, mesh.n))


class Geometry:
    """Per-triangle areas and basis gradients, evaluated for all triangles at once.

    Same formulas as Mesh.tri_geometry (checked against it in the tests).
    """

    def __init__(self, mesh: Mesh):
        P = mesh.xy[mesh.tris]                     # (nt, 3, 2)
        D = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]], axis=1)  # (nt, 2, 2)
        self.area = 0.5 * np.abs(np.linalg.det(D))
        Dinv = np.linalg.inv(D)
        g1, g2 = Dinv[:, :, 0], Dinv[:, :, 1]
        self.grads = np.stack([-(g1 + g2), g1, g2], axis=1)  # (nt, 3, 2)


def coefficient(mesh: Mesh, m: np.ndarray) -> np.ndarray:
    """c_T = exp of the centroid value of the P1 field m (centroid quadrature)."""
    return np.exp(m[mesh.tris].mean(axis=1))


def stiffness(mesh: Mesh, geo: Geometry, cT: np.ndarray,
              Theta: np.ndarray | None = None) -> sp.csr_matrix:
    """A_ij = sum_T c_T |T| grad(phi_i) . Theta grad(phi_j)  (weak form, Eq. poisson_weak)."""
    Th = np.eye(2) if Theta is None else np.asarray(Theta, dtype=float)

    G = geo.grads
    Ae = np.einsum('tai,ij,tbj->tab', G, Th, G) * (cT * geo.area)[:, None, None]
    return _assemble(mesh, Ae)


def mass(mesh: Mesh, geo: Geometry) -> sp.csr_matrix:
    """M_ij = int phi_i phi_j: element matrix |T|/12 (1 + delta_ij) (Sec. 2.3)."""
    base = (np.ones((3, 3)) + np.eye(3)) / 12.0

    return _assemble(mesh, geo.area[:, None, None] * base[None])


def boundary_mass(mesh: Mesh) -> sp.csr_matrix:
    """int_{boundary} phi_i phi_j: (len/6) [[2,1],[1,2]] on every boundary edge."""
    rows, cols, vals = [], [], []
    for (a, b) in mesh.bedges:
        L = np.linalg.norm(mesh.xy[b] - mesh.xy[a])
        Me = L / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]])
        v = (a, b)
        for p in range(2):
            for q in range(2):
                rows.append(v[p])
                cols.append(v[q])
                vals.append(Me[p, q])
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.n, mesh.n))


def point_location(mesh: Mesh, x: float, y: float):
    """Triangle containing (x, y) and its barycentric weights.

    The cell is (min(floor(x/h), N-1), min(floor(y/h), N-1)); inside the cell the
    lower triangle is taken when the local x offset is >= the local y offset.  A
    point on a shared edge gets the same interpolated value from either side
    because P1 functions are continuous there.
    """
    N, h = mesh.N, mesh.h
    i = min(int(np.floor(x / h)), N - 1)
    j = min(int(np.floor(y / h)), N - 1)
    xi, zeta = x / h - i, y / h - j
    t = 2 * (j * N + i) + (0 if xi >= zeta else 1)
    P = mesh.xy[mesh.tris[t]]
    # barycentric coordinates by solving the 3x3 affine system
    Aff = np.vstack([P.T, np.ones(3)])
    lam = np.linalg.solve(Aff, np.array([x, y, 1.0]))
    return t, lam


def observation_operator(mesh: Mesh, pts: np.ndarray) -> sp.csr_matrix:
    """B (q x n): row o evaluates the P1 interpolant at point o (sum of deltas, Sec. 5.1)."""
    rows, cols, vals = [], [], []
    for o, (x, y) in enumerate(pts):
        t, lam = point_location(mesh, float(x), float(y))
        for a in range(3):
            rows.append(o)
            cols.append(mesh.tris[t, a])
            vals.append(lam[a])
    return sp.csr_matrix((vals, (rows, cols)), shape=(pts.shape[0], mesh.n))


def mass_factor(mesh: Mesh, geo: Geometry) -> sp.csr_matrix:
    """Rectangular factor C_M (n x 6N^2) with C_M C_M^T = M (Appendix C).

    The quadrature is the three-edge-midpoint rule on each triangle, exact for
    quadratics, so the P1 mass matrix is B^T D B summed over elements with
    D = diag(|T|/3) and B the basis values at the midpoints (1/2 at the two
    endpoints of the edge, 0 at the opposite vertex).  C_e = G_e^T B^T D^{1/2}.
    Column 3 t + e belongs to edge e of triangle t: e0=(a,r), e1=(r,b), e2=(a,b).
    """
    edge_vertices = ((0, 1), (1, 2), (0, 2))
    rows, cols, vals = [], [], []
    for t in range(mesh.tris.shape[0]):
        w = np.sqrt(geo.area[t] / 3.0)
        for e, (va, vb) in enumerate(edge_vertices):
            col = 3 * t + e
            for v in (va, vb):
                rows.append(mesh.tris[t, v])
                cols.append(col)
                vals.append(0.5 * w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(mesh.n, 3 * mesh.tris.shape[0]))


def anisotropic_theta(theta1: float, theta2: float, alpha: float) -> np.ndarray:
    """s.p.d. tensor with eigenvalues (theta1, theta2) along v = (sin a, cos a), w = (cos a, -sin a).

    The matrix printed in Sec. 5.1 is not s.p.d. for the stated parameters; this
    is the reading that keeps the stated eigenvalues and directions.
    """
    v = np.array([np.sin(alpha), np.cos(alpha)])
    w = np.array([np.cos(alpha), -np.sin(alpha)])
    return theta1 * np.outer(v, v) + theta2 * np.outer(w, w)
