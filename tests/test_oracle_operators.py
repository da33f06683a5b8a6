"""Pins for the oracle's DOF indexing and collocation operators (Sections 2.1, 2.3; Eqs. 1-3).

Checked against what geometry and potential theory fix: DOF counts on a
cube, solid angles (the free term) at faces, edges and corners, Gauss's law
inside and outside, potentials of a uniform layer on the unit sphere,
Green's identity for an interior point source (with its convergence rate),
the centred-source worked example, the uniform stream and the rigid-sphere
modal series.
"""

import numpy as np
import pytest

import bem_inputs
import oracle
from oracle import analytic, gmres


@pytest.fixture(scope="module")
def sphere2(oracle_lib):
    m = bem_inputs.icosphere(2)
    om = oracle.OracleMesh(m.xyz, m.elem)
    S, K, c = om.assemble()
    return om, S, K, c


@pytest.fixture(scope="module")
def cube4(oracle_lib):
    m = bem_inputs.cube(4)
    om = oracle.OracleMesh(m.xyz, m.elem)
    return om


# ---------------------------------------------------------------- Section 2.3
@pytest.mark.parametrize("n", [1, 2, 4, 7])
def test_cube_dof_counts(oracle_lib, n):
    m = bem_inputs.cube(n)
    om = oracle.OracleMesh(m.xyz, m.elem)
    assert om.n_dof == 6 * (2 * n + 1) ** 2
    mult = np.bincount(om.dof_node, minlength=m.n_nodes)
    x = m.xyz
    on = np.isclose(np.abs(x), 1.0).sum(1)  # number of coordinates on the cube's faces
    assert np.all(mult[on == 3] == 3)  # corners
    assert np.all(mult[on == 2] == 2)  # edges
    assert np.all(mult[on == 1] == 1)  # faces
    # DOF normals are the face normals
    assert np.allclose(np.abs(om.dof_normal).max(1), 1.0)


def test_sphere_has_one_dof_per_node(oracle_lib):
    m = bem_inputs.icosphere(2)
    om = oracle.OracleMesh(m.xyz, m.elem)
    assert om.n_dof == m.n_nodes == 642
    assert np.all(np.sort(om.dof_node) == np.arange(m.n_nodes))
    assert np.allclose(np.einsum("ij,ij->i", om.dof_normal, om.dof_xyz / np.linalg.norm(om.dof_xyz, axis=1)[:, None]), 1, atol=1e-2)


# ---------------------------------------------------------------- Eq. 2
def test_free_term_solid_angles_on_cube(cube4):
    """C = 1 + PV int dG0/dn = fraction of the exterior solid angle: 1/2 on a
    face, 3/4 on an edge, 7/8 at a corner (flat faces: exact geometry)."""
    om = cube4
    c = om.free_term()
    on = np.isclose(np.abs(om.dof_xyz), 1.0).sum(1)
    for k, want in ((1, 0.5), (2, 0.75), (3, 0.875)):
        assert np.abs(c[on == k] - want).max() < 2e-4, (k, np.abs(c[on == k] - want).max())


def test_free_term_on_sphere(sphere2):
    om, S, K, c = sphere2
    assert np.abs(c - 0.5).max() < 1.5e-3  # the faceted sphere's kinks only


def test_gauss_law_inside_outside(sphere2):
    om, *_ = sphere2
    inside = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1], [0.0, 0.0, 0.8]])
    outside = np.array([[0.0, 0.0, 1.5], [2.0, 1.0, 0.0]])
    ones = np.ones(om.n_dof)
    # double layer of unit density: -1 inside, 0 outside (n out of the body)
    assert np.allclose(om.layer_potential(inside, sigma_d=ones), -1.0, atol=1e-5)
    assert np.allclose(om.layer_potential(outside, sigma_d=ones), 0.0, atol=1e-5)
    # single layer of unit density on the unit sphere: 1 inside, 1/|x| outside
    assert np.allclose(om.layer_potential(inside[:2], sigma_s=ones), 1.0, atol=2e-3)
    assert np.allclose(om.layer_potential(outside, sigma_s=ones), 1 / np.linalg.norm(outside, axis=1), atol=2e-3)


def test_single_layer_row_sums_unit_sphere(sphere2):
    om, S, K, c = sphere2
    # integral of G over the unit sphere from a point on it is 1
    assert np.abs(S.sum(1) - 1.0).max() < 1e-4


# ---------------------------------------------------------------- Eqs. 1, 3
def test_centred_source_worked_example(sphere2):
    """Source at the centre: phi = 1/4pi, chi = -1/4pi; c phi - K phi = -S chi."""
    om, S, K, c = sphere2
    phi = np.full(om.n_dof, 1 / (4 * np.pi))
    chi = -phi
    lhs = c * phi - K @ phi
    rhs = -S @ chi
    assert np.abs(lhs - 1 / (4 * np.pi)).max() < 5e-4 / (4 * np.pi) * 4
    assert np.abs(rhs - 1 / (4 * np.pi)).max() < 1e-4
    # the literal sign reading (A = C + K) fails this example
    assert np.abs((c * phi + K @ phi) - rhs).max() > 0.05


def test_greens_identity_converges_h4(oracle_lib):
    errs = []
    for sub in (1, 2, 3):
        m = bem_inputs.icosphere(sub)
        om = oracle.OracleMesh(m.xyz, m.elem)
        S, K, c = om.assemble()
        phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal)
        x = np.linalg.solve(np.diag(c) - K, -S @ chi)
        errs.append(np.sqrt(np.mean(np.abs(x - phi) ** 2)))
    assert errs[1] < 1e-5 and errs[2] < 1e-6
    assert errs[0] / errs[1] > 8 and errs[1] / errs[2] > 8


def test_uniform_stream_sphere(sphere2):
    om, S, K, c = sphere2
    d = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    _, chi = analytic.uniform_stream(om.dof_xyz, om.dof_normal, d)
    phi_s = np.linalg.solve(np.diag(c) - K, -S @ chi)
    assert np.abs(phi_s - 0.5 * om.dof_xyz @ d).max() < 2e-4


def test_cube_point_source(oracle_lib):
    m = bem_inputs.cube(3)
    om = oracle.OracleMesh(m.xyz, m.elem)
    S, K, c = om.assemble()
    phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal)
    x = np.linalg.solve(np.diag(c) - K, -S @ chi)
    err = np.sqrt(np.mean(np.abs(x - phi) ** 2)) / np.sqrt(np.mean(phi ** 2))
    assert err < 5e-3


# ---------------------------------------------------------------- Helmholtz
def test_rigid_sphere_series_two_forms():
    ct = np.linspace(-1, 1, 41)
    for ka in (0.5, 2.0, 10.0):
        a = analytic.rigid_sphere_total(ka, ct)
        b = analytic.rigid_sphere_total_textbook(ka, ct)
        assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_rigid_sphere_helmholtz_solve(oracle_lib):
    ka = 2.0
    m = bem_inputs.icosphere(3)
    om = oracle.OracleMesh(m.xyz, m.elem)
    S, K, c = om.assemble(oracle.HELMHOLTZ, ka)
    inc, chi = analytic.plane_wave(om.dof_xyz, om.dof_normal, ka)
    phi_s = np.linalg.solve(np.diag(c) - K, -S @ chi)
    ref = analytic.rigid_sphere_total(ka, om.dof_xyz[:, 2] / np.linalg.norm(om.dof_xyz, axis=1))
    err = np.abs(phi_s + inc - ref).max() / np.abs(ref).max()
    assert err < 2e-3


def test_helmholtz_point_source_identity(oracle_lib):
    k = 2.0
    m = bem_inputs.icosphere(2)
    om = oracle.OracleMesh(m.xyz, m.elem)
    S, K, c = om.assemble(oracle.HELMHOLTZ, k)
    phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal, k=k)
    x = np.linalg.solve(np.diag(c) - K, -S @ chi)
    err = np.sqrt(np.mean(np.abs(x - phi) ** 2))
    assert err < 5e-5  # the paper's Table 4 (N = 642, k = 2) reports 4.3e-5 for its source


def test_matvec_rows_equal_dense(sphere2):
    om, S, K, c = sphere2
    x = bem_inputs.random_vector(om.n_dof, 3)[0]
    rows = np.array([0, 17, 333, 641])
    for op, ref in ((oracle.OP_S, S @ x), (oracle.OP_K, K @ x), (oracle.OP_A, c * x - K @ x), (oracle.OP_RHS, -S @ x)):
        y = om.matvec_rows(x, op, rows=rows)
        assert np.abs(y - ref[rows]).max() < 1e-14 * np.abs(ref).max()


# ---------------------------------------------------------------- GMRES
@pytest.mark.parametrize("restart", [5, 50])
def test_gmres_matches_dense_solve(restart):
    rng = np.random.default_rng(7)
    n = 120
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) / np.sqrt(n) + 1j * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = gmres.gmres(lambda v: A @ v, b, tol=1e-12, restart=restart)
    assert info["converged"]
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) < 1e-10


def test_gmres_exact_in_n_steps():
    rng = np.random.default_rng(8)
    n = 20
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, info = gmres.gmres(lambda v: A @ v, b, tol=1e-13, restart=50)
    assert info["iterations"] <= n
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-12


@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_representation_formula_reproduces_point_source_field(sphere2, green, k):
    """Field evaluation (Section 3.5): with the exact surface values of the
    field of a point source inside the body, D[phi] - S[chi] is that field at
    points outside (Green's representation, C = 1 there) and vanishes inside
    (C = 0), for Laplace and Helmholtz; a sign or term error in either layer
    breaks one of the two."""
    from oracle import analytic

    om, *_ = sphere2
    xs = np.array([0.1, 0.2, 0.3])
    phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal, xs=xs, k=k)
    outside = np.array([[1.5, 0.0, 0.0], [0.0, -2.0, 0.5], [0.8, 0.9, 1.0], [0.0, 0.0, -3.0]])
    inside = np.array([[0.0, 0.0, -0.3], [-0.4, 0.1, 0.2], [0.2, -0.1, 0.0]])
    u_out = om.layer_potential(outside, green, k, sigma_d=phi) - om.layer_potential(outside, green, k, sigma_s=chi)
    u_in = om.layer_potential(inside, green, k, sigma_d=phi) - om.layer_potential(inside, green, k, sigma_s=chi)
    R = np.linalg.norm(outside - xs, axis=1)
    want = np.exp(1j * k * R) / (4 * np.pi * R)
    # measured 1.4e-4 / 1.8e-4 outside and 6e-5 inside on 320 elements (the
    # discretisation error); a wrong sign on either layer gives O(1)
    assert np.abs(u_out - want).max() / np.abs(want).max() < 5e-4
    assert np.abs(u_in).max() < 5e-4 * np.abs(want).max()
