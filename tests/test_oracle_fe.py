"""Pins of the oracle's finite-element assembly against closed forms.

Each test checks the oracle against something other than itself: hand-derived
matrices, the exact integrals of linear functions, the five-point form of the
stiffness on the right-diagonal mesh, and the exact discrete solution u = y
when m varies with x only.
"""
import os

import numpy as np
import pytest

from oracle import mesh as msh
from oracle import model

GOLD = os.path.join(os.path.dirname(__file__), "golden", "p1_matrices_N1.txt")


def _read_golden():
    blocks, cur = {}, None
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            blocks[cur] = []
        else:
            blocks[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


def test_golden_single_cell():
    g = _read_golden()
    me = msh.Mesh(1)
    geo = msh.Geometry(me)
    K = msh.stiffness(me, geo, np.ones(2)).toarray()
    np.testing.assert_allclose(K, g["stiffness"], atol=1e-15)
    np.testing.assert_allclose(msh.mass(me, geo).toarray() * 24, g["mass*24"], atol=1e-14)
    np.testing.assert_allclose(msh.boundary_mass(me).toarray() * 6, g["boundary_mass*6"], atol=1e-14)
    B = msh.observation_operator(me, np.array([[0.75, 0.25]])).toarray()
    np.testing.assert_allclose(B, g["observation"], atol=1e-15)


def test_geometry_vectorized_matches_per_triangle():
    me = msh.Mesh(5)
    geo = msh.Geometry(me)
    for t in (0, 1, 17, 48, 49):
        a, G = me.tri_geometry(t)
        assert abs(a - geo.area[t]) < 1e-15
        np.testing.assert_allclose(G, geo.grads[t], atol=1e-12)
    assert abs(geo.area.sum() - 1.0) < 1e-13
    np.testing.assert_allclose(geo.area, 0.5 / 25)


def _five_point_reference(N, cT):
    """Stiffness built edge by edge from the five-point form:
    horizontal edge (i,j)-(i+1,j) weight (c_L(i,j) + c_U(i,j-1)) / 2, vertical edge
    (i,j)-(i,j+1) weight (c_U(i,j) + c_L(i-1,j)) / 2 (missing triangles omitted),
    zero weight on the diagonal edge, A = sum_e w_e (e_a - e_b)(e_a - e_b)^T."""
    n = (N + 1) ** 2
    A = np.zeros((n, n))
    k = lambda i, j: j * (N + 1) + i
    cL = lambda i, j: cT[2 * (j * N + i)] if (0 <= i < N and 0 <= j < N) else 0.0
    cU = lambda i, j: cT[2 * (j * N + i) + 1] if (0 <= i < N and 0 <= j < N) else 0.0
    for j in range(N + 1):
        for i in range(N + 1):
            if i < N:
                w = 0.5 * (cL(i, j) + cU(i, j - 1))
                a, b = k(i, j), k(i + 1, j)
                A[a, a] += w; A[b, b] += w; A[a, b] -= w; A[b, a] -= w
            if j < N:
                w = 0.5 * (cU(i, j) + cL(i - 1, j))
                a, b = k(i, j), k(i, j + 1)
                A[a, a] += w; A[b, b] += w; A[a, b] -= w; A[b, a] -= w
    return A


@pytest.mark.parametrize("N", [2, 3, 6])
def test_stiffness_is_five_point(N):
    me = msh.Mesh(N)
    geo = msh.Geometry(me)
    rng = np.random.default_rng(3)
    m = rng.normal(size=me.n)
    cT = msh.coefficient(me, m)
    A = msh.stiffness(me, geo, cT).toarray()
    np.testing.assert_allclose(A, _five_point_reference(N, cT), atol=1e-13)
    np.testing.assert_allclose(A.sum(axis=1), 0.0, atol=1e-13)   # zero row sums
    off = A - np.diag(np.diag(A))
    assert (off <= 1e-15).all()                                  # M-matrix sign pattern


def test_constant_coefficient_scales_laplacian():
    me = msh.Mesh(4)
    geo = msh.Geometry(me)
    c = 0.7
    A1 = msh.stiffness(me, geo, msh.coefficient(me, np.zeros(me.n))).toarray()
    Ac = msh.stiffness(me, geo, msh.coefficient(me, np.full(me.n, c))).toarray()
    np.testing.assert_allclose(Ac, np.exp(c) * A1, rtol=1e-13, atol=1e-13)
    # interior row of the unit stiffness is the standard 5-point Laplacian
    i = me.node(2, 2)
    row = A1[i]
    assert abs(row[i] - 4.0) < 1e-13
    for nb in (me.node(1, 2), me.node(3, 2), me.node(2, 1), me.node(2, 3)):
        assert abs(row[nb] + 1.0) < 1e-13
    assert abs(row[me.node(3, 3)]) < 1e-14 and abs(row[me.node(1, 1)]) < 1e-14


def test_mass_and_boundary_mass_integrate_exactly():
    me = msh.Mesh(7)
    geo = msh.Geometry(me)
    M = msh.mass(me, geo)
    Mb = msh.boundary_mass(me)
    one = np.ones(me.n)
    x, y = me.xy[:, 0], me.xy[:, 1]
    assert abs(one @ (M @ one) - 1.0) < 1e-13          # area
    assert abs(x @ (M @ x) - 1.0 / 3.0) < 1e-13         # int x^2
    assert abs(x @ (M @ y) - 1.0 / 4.0) < 1e-13         # int x y
    assert abs(one @ (Mb @ one) - 4.0) < 1e-13          # perimeter
    # int_boundary x^2 ds = 1/3 (bottom) + 1/3 (top) + 0 (left) + 1 (right)
    assert abs(x @ (Mb @ x) - 5.0 / 3.0) < 1e-13


def test_anisotropic_stiffness_on_linear_functions():
    me = msh.Mesh(5)
    geo = msh.Geometry(me)
    Th = msh.anisotropic_theta(2.0, 0.5, np.pi / 4)
    np.testing.assert_allclose(np.linalg.eigvalsh(Th), [0.5, 2.0], atol=1e-14)
    K = msh.stiffness(me, geo, np.ones(me.tris.shape[0]), Th)
    a = np.array([0.3, -1.1])
    b = np.array([0.8, 0.4])
    f = me.xy @ a
    g = me.xy @ b
    # int grad f . Theta grad g over the unit square = a^T Theta b
    assert abs(f @ (K @ g) - a @ Th @ b) < 1e-12


def test_observation_reproduces_linear_functions():
    me = msh.Mesh(9)
    rng = np.random.default_rng(5)
    pts = rng.uniform(0.0, 1.0, size=(50, 2))
    pts[0] = (1.0, 1.0)          # corner clamps into the last cell
    pts[1] = (0.5, 0.5)          # on the diagonal of a cell
    B = msh.observation_operator(me, pts)
    f = 0.3 + 1.7 * me.xy[:, 0] - 0.6 * me.xy[:, 1]
    np.testing.assert_allclose(B @ f, 0.3 + 1.7 * pts[:, 0] - 0.6 * pts[:, 1], atol=1e-13)
    assert B.nnz <= 3 * pts.shape[0]
    np.testing.assert_allclose(np.asarray(B.sum(axis=1)).ravel(), 1.0, atol=1e-14)


def test_mass_factor_is_exact_rectangular_decomposition():
    me = msh.Mesh(5)
    geo = msh.Geometry(me)
    C = msh.mass_factor(me, geo)
    assert C.shape == (me.n, 6 * 25)
    np.testing.assert_allclose((C @ C.T).toarray(), msh.mass(me, geo).toarray(), atol=1e-15)


@pytest.mark.parametrize("N", [4, 16])
def test_forward_exact_when_coefficient_depends_on_x_only(N):
    prob = model.Problem(N, 0.1, 0.5)
    x = prob.mesh.xy[:, 0]
    m = np.sin(3.0 * x) - 1.0
    u = prob.forward(m)
    np.testing.assert_allclose(u, prob.mesh.xy[:, 1], atol=2e-13)


def _mms_error(N, eps=0.3, mu=0.6):
    """L2 error of the FE solution for u = y + eps sin(pi y) cos(pi x), m = mu cos(pi x) cos(pi y)."""
    prob = model.Problem(N, 0.1, 0.5)
    me, geo = prob.mesh, prob.geo
    pi = np.pi

    def fields(x, y):
        m = mu * np.cos(pi * x) * np.cos(pi * y)
        mx = -mu * pi * np.sin(pi * x) * np.cos(pi * y)
        my = -mu * pi * np.cos(pi * x) * np.sin(pi * y)
        ux = -eps * pi * np.sin(pi * y) * np.sin(pi * x)
        uy = 1.0 + eps * pi * np.cos(pi * y) * np.cos(pi * x)
        lap = -2.0 * eps * pi * pi * np.sin(pi * y) * np.cos(pi * x)
        f = -np.exp(m) * (mx * ux + my * uy + lap)
        u = y + eps * np.sin(pi * y) * np.cos(pi * x)
        return m, f, u

    mnod, _, _ = fields(me.xy[:, 0], me.xy[:, 1])
    # load vector int f phi_k with the 3 edge-midpoint rule per triangle
    load = np.zeros(me.n)
    err2 = 0.0
    P = me.xy[me.tris]
    mids = [(0, 1), (1, 2), (0, 2)]
    for (a, b) in mids:
        X = 0.5 * (P[:, a] + P[:, b])
        _, f, _ = fields(X[:, 0], X[:, 1])
        w = geo.area / 3.0
        for v in range(3):
            phi = 0.5 if v in (a, b) else 0.0
            np.add.at(load, me.tris[:, v], w * f * phi)
    uh = prob.forward(mnod, f_load=load)
    for (a, b) in mids:
        X = 0.5 * (P[:, a] + P[:, b])
        _, _, uex = fields(X[:, 0], X[:, 1])
        uhx = 0.5 * (uh[me.tris[:, a]] + uh[me.tris[:, b]])
        err2 += np.sum(geo.area / 3.0 * (uhx - uex) ** 2)
    return np.sqrt(err2)


def test_manufactured_solution_second_order():
    errs = [_mms_error(N) for N in (8, 16, 32)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-3
    for r in rates:
        assert 1.8 < r < 2.3, (errs, rates)


def test_discrete_maximum_principle_gives_unit_noise_scale():
    prob = model.Problem(16, 0.1, 0.5)
    rng = np.random.default_rng(11)
    m = -2.0 + rng.normal(size=prob.n)
    u = prob.forward(m)
    assert u.min() >= -1e-14 and u.max() <= 1.0 + 1e-14
    assert abs(np.abs(u).max() - 1.0) < 1e-15
