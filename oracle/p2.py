"""Continuous quadratic (P2) state space on the structured triangulation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's Poisson experiment (Sec. 5.1) discretizes the state u and the
adjoints with quadratic Lagrange elements and the parameter m with linear
ones.  This module is the state side of that pairing; the parameter, the
prior and the coefficient c_T = exp(mean of m over the triangle's vertices)
stay exactly as in ``mesh`` and ``model``.

Degrees of freedom: the vertices and the edge midpoints of the triangulation.
On this mesh they are the nodes of the (2N+1) x (2N+1) grid of spacing h/2:
node (I, J) sits at (I h/2, J h/2) and is numbered J (2N+1) + I.  Even I and
even J: a vertex; odd I, even J: the midpoint of a horizontal edge; even I,
odd J: of a vertical edge; odd I and odd J: of a cell's diagonal.

For a triangle with vertices (a, r, b) (as stored in ``mesh.Mesh``) the six
local degrees of freedom are ordered (a, r, b, mid(a,r), mid(r,b), mid(a,b)),
with the basis psi_v = lam_v (2 lam_v - 1) at vertex v and
psi_e = 4 lam_v lam_w on edge e = (v, w), lam the barycentric coordinates.
Gradients of P2 functions are linear, so every element integral of a product
of two gradients is a quadratic, integrated exactly by the three-edge-midpoint
rule (weights |T|/3).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import mesh as msh

# local edges (v, w) of the three midpoint degrees of freedom
EDGES = ((0, 1), (1, 2), (0, 2))


class P2Space:
    """Quadratic Lagrange space on ``mesh`` (same triangles, 6 dofs each)."""

    def __init__(self, mesh: msh.Mesh, geo: msh.Geometry):
        N = mesh.N
        self.mesh, self.geo = mesh, geo
        self.N = N
        self.side = 2 * N + 1
        self.n = self.side * self.side
        g = np.arange(self.side) * (0.5 / N)
        X, Y = np.meshgrid(g, g)
        self.xy = np.column_stack([X.reshape(-1), Y.reshape(-1)])
        # fine-grid coordinates of each vertex of each triangle
        vij = np.column_stack([mesh.tris.reshape(-1) % (N + 1), mesh.tris.reshape(-1) // (N + 1)])
        V = 2 * vij.reshape(-1, 3, 2)                       # (nt, 3, 2) as fine (I, J)
        dofs = np.empty((mesh.tris.shape[0], 6), dtype=np.int64)
        for a in range(3):
            dofs[:, a] = V[:, a, 1] * self.side + V[:, a, 0]
        for e, (v, w) in enumerate(EDGES):
            M = (V[:, v] + V[:, w]) // 2
            dofs[:, 3 + e] = M[:, 1] * self.side + M[:, 0]
        self.tri_dofs = dofs
        J = np.arange(self.n) // self.side
        self.dirichlet = (J == 0) | (J == 2 * N)
        self.free = ~self.dirichlet
        # u = 1 on the top edge, 0 on the bottom edge (Sec. 5.1)
        self.uD = np.zeros(self.n)
        self.uD[J == 2 * N] = 1.0
        self.Ke = self._element_stiffness()

    # -- basis ------------------------------------------------------------------
    @staticmethod
    def basis_values(lam: np.ndarray) -> np.ndarray:
        """The six basis functions at barycentric coordinates lam (..., 3)."""
        out = [lam[..., v] * (2.0 * lam[..., v] - 1.0) for v in range(3)]
        out += [4.0 * lam[..., v] * lam[..., w] for (v, w) in EDGES]
        return np.stack(out, axis=-1)

    def basis_gradients(self, lam: np.ndarray) -> np.ndarray:
        """Gradients of the six basis functions at lam (3,) on every triangle: (nt, 6, 2).

        grad psi_v = (4 lam_v - 1) grad lam_v,  grad psi_(v,w) = 4 (lam_w grad lam_v + lam_v grad lam_w).
        """
        G = self.geo.grads                                   # (nt, 3, 2): grad lam
        out = [(4.0 * lam[v] - 1.0) * G[:, v] for v in range(3)]
        out += [4.0 * (lam[w] * G[:, v] + lam[v] * G[:, w]) for (v, w) in EDGES]
        return np.stack(out, axis=1)

    def _element_stiffness(self) -> np.ndarray:
        """K_e[t] = int_T grad psi_i . grad psi_j (unit coefficient), (nt, 6, 6)."""
        Ke = np.zeros((self.mesh.tris.shape[0], 6, 6))
        for (v, w) in EDGES:
            lam = np.zeros(3)
            lam[v] = lam[w] = 0.5
            Gq = self.basis_gradients(lam)
            Ke += np.einsum('tai,tbi->tab', Gq, Gq) * (self.geo.area / 3.0)[:, None, None]
        return Ke

    # -- assembled operators --------------------------------------------------------
    def stiffness(self, cT: np.ndarray) -> sp.csr_matrix:
        """A_ij = sum_T c_T int_T grad psi_i . grad psi_j (Eq. eq:poisson_weak with a P2 state)."""
        Ae = self.Ke * cT[:, None, None]
        d = self.tri_dofs
        rows = np.repeat(d, 6, axis=1).reshape(-1)
        cols = np.tile(d, (1, 6)).reshape(-1)
        return sp.csr_matrix((Ae.reshape(-1), (rows, cols)), shape=(self.n, self.n))

    def tri_forms(self, v: np.ndarray, w: np.ndarray) -> np.ndarray:
        """Per-triangle int_T grad v . grad w for P2 vectors v, w."""
        vt, wt = v[self.tri_dofs], w[self.tri_dofs]
        return np.einsum('ta,tab,tb->t', vt, self.Ke, wt)

    def observation_operator(self, pts: np.ndarray) -> sp.csr_matrix:
        """B (q x n): row o evaluates the P2 function at point o (point location as in mesh)."""
        rows, cols, vals = [], [], []
        for o, (x, y) in enumerate(pts):
            t, lam = msh.point_location(self.mesh, float(x), float(y))
            psi = self.basis_values(lam)
            for a in range(6):
                rows.append(o)
                cols.append(self.tri_dofs[t, a])
                vals.append(psi[a])
        return sp.csr_matrix((vals, (rows, cols)), shape=(pts.shape[0], self.n))

    def interpolate_p1(self, v1: np.ndarray) -> np.ndarray:
        """The P1 function v1 (vertex values) as a P2 vector: vertices keep their
        values, each edge midpoint takes the mean of its edge's two ends."""
        out = np.zeros(self.n)
        vt = v1[self.mesh.tris]
        out[self.tri_dofs[:, :3]] = vt
        for e, (v, w) in enumerate(EDGES):
            out[self.tri_dofs[:, 3 + e]] = 0.5 * (vt[:, v] + vt[:, w])
        return out
