"""Pins for the oracle's first-order (3-node flat) elements, the paper's other
element type (Section 2.2; Tables 1, 3, 5 and 7).

Checked against what geometry and potential theory fix: the linear shape
functions' nodal values and derivatives, the closed-form integral of 1/R over
a flat triangle from a vertex, the area of a polyhedron, DOF counts and solid
angles (the free term) on a flat-faced cube, Gauss's law, the direct-solution
errors the paper prints for the sphere (Tables 1 and 5) with their O(h^2)
convergence, and the fast product on a kernel whose Taylor series ends
(equal to the direct sum).
"""

import math
import os

import numpy as np
import pytest

import bem_inputs
import oracle
from oracle import analytic

from test_oracle_quadrature import closed_form_inv_r_from_vertex


@pytest.fixture(scope="module")
def sphere_p1(oracle_lib):
    m = bem_inputs.linear(bem_inputs.icosphere(2))
    om = oracle.OracleMesh(m.xyz, m.elem)
    S, K, c = om.assemble()
    return om, S, K, c


def test_linear_shape_functions(oracle_lib):
    corners = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)]
    for b, (s, t) in enumerate(corners):
        L, Ls, Lt = oracle.shape(s, t, nn=3)
        assert np.array_equal(L[:3], np.eye(3)[b]) and np.all(L[3:] == 0.0)
    rng = np.random.default_rng(5)
    for s, t in rng.uniform(0, 0.5, (5, 2)):
        L, Ls, Lt = oracle.shape(s, t, nn=3)
        assert abs(L.sum() - 1.0) < 1e-15
        assert np.array_equal(Ls[:3], [-1.0, 1.0, 0.0]) and np.array_equal(Lt[:3], [-1.0, 0.0, 1.0])
        # linear interpolation reproduces the coordinates themselves
        assert abs(L[1] - s) < 1e-15 and abs(L[2] - t) < 1e-15


def test_flat_element_map_and_corner_integral(oracle_lib):
    X = np.array([[0.1, -0.2, 0.3], [1.3, 0.1, 0.2], [0.2, 0.9, 0.5]])
    cr = np.cross(X[1] - X[0], X[2] - X[0])
    for s, t in ((0.2, 0.3), (0.6, 0.1)):
        y, n, J = oracle.elem_point(X, s, t)
        assert np.allclose(y, (1 - s - t) * X[0] + s * X[1] + t * X[2], atol=1e-15)
        assert abs(J - np.linalg.norm(cr)) < 1e-14 and np.allclose(n, cr / np.linalg.norm(cr), atol=1e-15)
    mesh = oracle.OracleMesh(X, np.arange(3, dtype=np.int32)[None, :])
    cls, S, K = mesh.pair(0, 0, X[0])
    assert cls == 2
    ref = closed_form_inv_r_from_vertex(X[0], X[1], X[2])
    assert abs((S.sum() * 4 * math.pi).real - ref) / ref < 1e-9
    assert np.all(S[3:] == 0.0) and np.abs(K).max() < 1e-15


def test_polyhedron_area(oracle_lib):
    m = bem_inputs.linear(bem_inputs.icosphere(2))
    tri = m.xyz[m.elem]
    exact = 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1).sum()
    s, t, w = oracle.rule(0)
    area = sum(wi * oracle.elem_point(tri[e], si, ti)[2] for e in range(m.n_elem) for si, ti, wi in zip(s, t, w))
    assert abs(area - exact) < 1e-13 * exact


@pytest.mark.parametrize("n", [1, 3])
def test_cube_dof_counts_and_solid_angles(oracle_lib, n):
    """Flat faces: the free term is exactly the fraction of the exterior
    solid angle, 1/2 on a face, 3/4 on an edge, 7/8 at a corner."""
    m = bem_inputs.linear(bem_inputs.cube(n))
    om = oracle.OracleMesh(m.xyz, m.elem)
    assert om.n_dof == 6 * (n + 1) ** 2
    on = np.isclose(np.abs(om.dof_xyz), 1.0).sum(1)
    mult = np.bincount(om.dof_node, minlength=m.n_nodes)
    xon = np.isclose(np.abs(m.xyz), 1.0).sum(1)
    assert np.all(mult[xon == 3] == 3) and np.all(mult[xon == 2] == 2) and np.all(mult[xon == 1] == 1)
    c = om.free_term()
    for k, want in ((1, 0.5), (2, 0.75), (3, 0.875)):
        if np.any(on == k):
            assert np.abs(c[on == k] - want).max() < 2e-4, (k, np.abs(c[on == k] - want).max())


def test_gauss_law(sphere_p1):
    om, *_ = sphere_p1
    ones = np.ones(om.n_dof)
    inside = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1]])
    outside = np.array([[0.0, 0.0, 1.5], [2.0, 1.0, 0.0]])
    assert np.allclose(om.layer_potential(inside, sigma_d=ones), -1.0, atol=1e-6)
    assert np.allclose(om.layer_potential(outside, sigma_d=ones), 0.0, atol=1e-6)


def _paper_direct_errors():
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "sphere_p1_direct_error.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                g, n, e = line.split()
                rows[(g, int(n))] = float(e)
    return rows


@pytest.mark.parametrize("green,k,subs", [(oracle.LAPLACE, 0.0, (2, 3, 4)), (oracle.HELMHOLTZ, 2.0, (2, 3))])
def test_direct_solution_error_matches_tables_1_and_5(oracle_lib, green, k, subs):
    """Interior point source, Neumann data given, dense solve: the rms error
    of the recovered potential falls at second order in h and lies within
    20% of the direct-solution errors the paper prints for the same spheres
    (Tables 1 and 5; the source position is not given there)."""
    paper = _paper_direct_errors()
    errs = []
    for sub in subs:
        m = bem_inputs.linear(bem_inputs.icosphere(sub))
        om = oracle.OracleMesh(m.xyz, m.elem)
        S, K, c = om.assemble(green, k)
        phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal, k=k)
        x = np.linalg.solve(np.diag(c) - K, -S @ chi)
        err = np.sqrt(np.mean(np.abs(x - phi) ** 2))
        ref = paper[("laplace" if green == oracle.LAPLACE else "helmholtz", m.n_nodes)]
        assert om.n_dof == m.n_nodes
        assert 0.8 < err / ref < 1.2, (m.n_nodes, err, ref)
        errs.append(err)
    assert all(a / b > 3 for a, b in zip(errs, errs[1:]))


@pytest.mark.parametrize("op", [oracle.OP_S_REG, oracle.OP_K_REG])
def test_fmm_exact_for_terminating_taylor_series(oracle_lib, op):
    m = bem_inputs.linear(bem_inputs.icosphere(3))
    om = oracle.OracleMesh(m.xyz, m.elem)
    x = bem_inputs.random_vector(om.n_dof, 12)[0]
    T = oracle.OracleTree(om, B=16, theta=0.7)
    yf = T.fmm_matvec(x, op, green=oracle.R2, order=3)
    yd = om.matvec_rows(x, op, green=oracle.R2)
    assert np.linalg.norm(yf - yd) / np.linalg.norm(yd) < 1e-13


def test_fmm_converges_to_direct(oracle_lib):
    m = bem_inputs.linear(bem_inputs.icosphere(3))
    om = oracle.OracleMesh(m.xyz, m.elem)
    x = bem_inputs.random_vector(om.n_dof, 13)[0]
    T = oracle.OracleTree(om, B=16, theta=0.6)
    yd = om.matvec_rows(x, oracle.OP_A)
    errs = [np.linalg.norm(T.fmm_matvec(x, oracle.OP_A, order=p) - yd) / np.linalg.norm(yd) for p in (2, 4, 8)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6
