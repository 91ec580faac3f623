"""Pins of the oracle's quadratic (P2) state space (the state discretization of
the paper's Poisson experiment, Sec. 5.1).

* element stiffness: for every pair of quadratic polynomials v, w the
  element form v_T^T K_T w_T equals int_T grad v . grad w computed by an
  independent rule (collapsed Gauss-Legendre, exact for these degrees); the
  vertex-vertex block equals the closed form
  K_ij = |T| grad(lam_i) . grad(lam_j) (1 if i = j else -1/3) and a vertex
  does not couple with the midpoint of the opposite edge (both from the
  moments int lam_i lam_j = |T| (1 + delta_ij) / 12); zero row sums;
* the observation operator reproduces quadratic polynomials exactly at any
  point, and the P1 -> P2 embedding is exact for linear functions;
* the assembled stiffness keeps the P1 Galerkin identity P^T A_2 P = A_1 with
  P the P1 -> P2 embedding (P1 functions are P2 functions; same coefficient);
* forward solve: u = y exactly for a coefficient constant on vertical strips
  of cells and for a constant m; a manufactured
  solution converges at third order in L2 (constant coefficient, so that the
  centroid rule of e^m adds no error).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import mesh as msh
from oracle import model
from oracle import p2 as p2sp


def _space(N):
    me = msh.Mesh(N)
    geo = msh.Geometry(me)
    return me, geo, p2sp.P2Space(me, geo)


def _collapsed_rule(P, order=6):
    """Points and weights on triangle P (3x2) from a Duffy-collapsed Gauss-Legendre rule."""
    g, w = np.polynomial.legendre.leggauss(order)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    pts, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            s, t = a, b * (1.0 - a)             # (s, t) in the unit triangle
            jac = (1.0 - a)
            pts.append(P[0] + s * (P[1] - P[0]) + t * (P[2] - P[0]))
            wts.append(wa * wb * jac)
    area2 = abs(np.linalg.det(np.array([P[1] - P[0], P[2] - P[0]])))
    return np.array(pts), np.array(wts) * area2


# quadratic polynomials and their gradients
POLYS = [
    (lambda x, y: np.ones_like(x), lambda x, y: (0 * x, 0 * x)),
    (lambda x, y: x, lambda x, y: (1 + 0 * x, 0 * x)),
    (lambda x, y: y, lambda x, y: (0 * x, 1 + 0 * x)),
    (lambda x, y: x * x, lambda x, y: (2 * x, 0 * x)),
    (lambda x, y: x * y, lambda x, y: (y, x)),
    (lambda x, y: y * y - 0.5 * x, lambda x, y: (-0.5 + 0 * x, 2 * y)),
]


def test_element_stiffness_integrates_quadratics_exactly():
    me, geo, S = _space(3)
    for t in (0, 1, 7, 12):
        P = me.xy[me.tris[t]]
        X, W = _collapsed_rule(P)
        dofs = S.xy[S.tri_dofs[t]]
        for fv, gv in POLYS:
            for fw, gw in POLYS:
                vt, wt = fv(dofs[:, 0], dofs[:, 1]), fw(dofs[:, 0], dofs[:, 1])
                a = vt @ S.Ke[t] @ wt
                gvx, gvy = gv(X[:, 0], X[:, 1])
                gwx, gwy = gw(X[:, 0], X[:, 1])
                ref = np.sum(W * (gvx * gwx + gvy * gwy))
                assert abs(a - ref) <= 1e-13 * max(1.0, abs(ref)), (t, a, ref)


def test_element_stiffness_closed_forms():
    me, geo, S = _space(2)
    for t in range(me.tris.shape[0]):
        K = S.Ke[t]
        G = geo.grads[t]
        A = geo.area[t]
        for i in range(3):
            for j in range(3):
                ref = A * (G[i] @ G[j]) * (1.0 if i == j else -1.0 / 3.0)
                assert abs(K[i, j] - ref) <= 1e-14
        # vertex i against the midpoint of the opposite edge
        for i, e in ((0, 4), (1, 5), (2, 3)):
            assert abs(K[i, e]) <= 1e-14
        # vertex v against the midpoint of an edge (v, w): (4/3) |T| grad lam_v . grad lam_w
        for e, (v, w) in enumerate(p2sp.EDGES):
            for a, b in ((v, w), (w, v)):
                assert abs(K[a, 3 + e] - 4.0 / 3.0 * A * (G[a] @ G[b])) <= 1e-14
        np.testing.assert_allclose(K.sum(axis=1), 0.0, atol=1e-14)
        np.testing.assert_allclose(K, K.T, atol=0)


def test_dof_numbering_and_embedding():
    me, geo, S = _space(4)
    assert S.n == 81
    # every triangle's dofs sit at its vertices and edge midpoints
    for t in range(me.tris.shape[0]):
        V = me.xy[me.tris[t]]
        D = S.xy[S.tri_dofs[t]]
        np.testing.assert_allclose(D[:3], V, atol=0)
        for e, (v, w) in enumerate(p2sp.EDGES):
            np.testing.assert_allclose(D[3 + e], 0.5 * (V[v] + V[w]), atol=1e-15)
    lin = 0.3 + 2.0 * me.xy[:, 0] - 1.5 * me.xy[:, 1]
    np.testing.assert_allclose(S.interpolate_p1(lin), 0.3 + 2.0 * S.xy[:, 0] - 1.5 * S.xy[:, 1], atol=1e-14)


def test_observation_reproduces_quadratics():
    me, geo, S = _space(5)
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 1, size=(40, 2))
    pts[:4] = [[0.0, 0.0], [1.0, 1.0], [0.4, 0.4], [0.2, 0.6]]  # corners, a diagonal, a vertex
    B = S.observation_operator(pts)
    for f, _ in POLYS:
        np.testing.assert_allclose(B @ f(S.xy[:, 0], S.xy[:, 1]), f(pts[:, 0], pts[:, 1]), atol=1e-14)


def test_galerkin_identity_with_p1():
    me, geo, S = _space(6)
    rng = np.random.default_rng(5)
    cT = np.exp(rng.normal(size=me.tris.shape[0]))
    A2 = S.stiffness(cT)
    A1 = msh.stiffness(me, geo, cT)
    P = sp.csr_matrix(np.column_stack([S.interpolate_p1(e) for e in np.eye(me.n)]))
    np.testing.assert_allclose((P.T @ A2 @ P).toarray(), A1.toarray(), atol=1e-13)


@pytest.mark.parametrize("N", [4, 16])
def test_p2_solution_exact_for_strip_coefficients(N):
    """A coefficient constant on each vertical strip of cells (both triangles of
    a cell alike) makes u = y the exact weak solution, and y is a P2 function:
    the discrete solution is y to rounding.  With the centroid rule of a P1
    field the two triangles of a cell differ, so this goes through the
    assembled stiffness; Problem.forward is checked with a constant m."""
    me, geo, S = _space(N)
    i_cell = (np.arange(me.tris.shape[0]) // 2) % N
    cT = np.exp(np.sin(3.0 * (i_cell + 0.5) / N) - 1.0)
    A = S.stiffness(cT).tocsr()
    f = S.free
    u = S.uD.copy()
    import scipy.sparse.linalg as spla
    u[f] = spla.spsolve(A[f][:, f].tocsc(), -(A @ S.uD)[f])
    np.testing.assert_allclose(u, S.xy[:, 1], atol=2e-13)
    prob = model.Problem(N, 0.1, 0.5, state_degree=2)
    np.testing.assert_allclose(prob.forward(np.full(prob.n, -1.3)), S.xy[:, 1], atol=2e-13)


def _mms_error_p2(N, eps=0.3, m0=-0.7):
    """L2 error for u = y + eps sin(pi y) cos(pi x), -e^m0 lap u = f, P2 state."""
    prob = model.Problem(N, 0.1, 0.5, state_degree=2)
    me, geo, S = prob.mesh, prob.geo, prob.S
    pi = np.pi
    c = np.exp(m0)

    def u_ex(x, y):
        return y + eps * np.sin(pi * y) * np.cos(pi * x)

    def f(x, y):
        return c * 2.0 * eps * pi * pi * np.sin(pi * y) * np.cos(pi * x)

    rules = []
    for t in range(me.tris.shape[0]):
        P = me.xy[me.tris[t]]
        X, W = _collapsed_rule(P, order=5)
        T = np.vstack([P.T, np.ones(3)])
        lam = np.linalg.solve(T, np.vstack([X.T, np.ones(len(X))])).T   # barycentric of each point
        rules.append((X, W, p2sp.P2Space.basis_values(lam)))            # psi: (npts, 6)
    load = np.zeros(S.n)
    for t, (X, W, psi) in enumerate(rules):
        np.add.at(load, S.tri_dofs[t], psi.T @ (W * f(X[:, 0], X[:, 1])))
    uh = prob.forward(np.full(me.n, m0), f_load=load)
    err2 = sum(np.sum(W * (psi @ uh[S.tri_dofs[t]] - u_ex(X[:, 0], X[:, 1])) ** 2)
               for t, (X, W, psi) in enumerate(rules))
    return np.sqrt(err2)


def test_p2_manufactured_solution_third_order():
    errs = [_mms_error_p2(N) for N in (4, 8, 16)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-4, errs
    for r in rates:
        assert 2.8 < r < 3.3, (errs, rates)
