"""Pins for the oracle's element and quadrature code (Sections 2.1-2.2).

Each check compares against something the oracle does not compute itself:
exact monomial integrals, published Gauss-Legendre values, and the closed-form
integral of 1/R over a flat triangle from one of its vertices.
"""

import math
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def exact_monomial(a, b):
    # integral of s^a t^b over {s,t >= 0, s+t <= 1} = a! b! / (a+b+2)!
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def test_seven_point_rule_degree_five(oracle_lib):
    s, t, w = oracle.rule(0)
    assert len(w) == 7
    for a in range(6):
        for b in range(6 - a):
            assert abs(np.sum(w * s ** a * t ** b) - exact_monomial(a, b)) < 1e-16 * 50
    # degree 6 is not integrated exactly by a degree-5 rule
    errs = [abs(np.sum(w * s ** a * t ** (6 - a)) - exact_monomial(a, 6 - a)) for a in range(7)]
    assert max(errs) > 1e-8


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_subdivision_rule_exact_and_partitioned(oracle_lib, d):
    s, t, w = oracle.rule(1, d)
    assert len(w) == 7 * 4 ** d
    assert abs(w.sum() - 0.5) < 1e-15
    assert np.all(s >= -1e-15) and np.all(t >= -1e-15) and np.all(s + t <= 1 + 1e-15)
    for a in range(6):
        for b in range(6 - a):
            assert abs(np.sum(w * s ** a * t ** b) - exact_monomial(a, b)) < 1e-15


def test_gauss_legendre_matches_published_table(oracle_lib):
    ref = np.loadtxt(os.path.join(GOLDEN, "gauss_legendre_8.txt"))
    # the singular rule for corner node 0 is a tensor Duffy rule: u on [0,1] maps to x = 2u - 1
    s, t, w = oracle.rule(2, 0, 8)
    u = np.unique(np.round(s + t, 14))  # s + t = u for corner 0 (P=(0,0), A=(1,0), B=(0,1))
    x = np.sort(2 * u - 1)
    assert np.allclose(np.sort(np.abs(x))[::2], ref[:, 0], atol=2e-15)
    # summing the v-direction weights leaves w_i u_i, with w_i half the [-1,1] weight
    uu = np.round(s + t, 14)
    for ui in np.unique(uu):
        wi = w[uu == ui].sum() / ui
        j = np.argmin(np.abs(ref[:, 0] - abs(2 * ui - 1)))
        assert abs(2 * wi - ref[j, 1]) < 2e-14


@pytest.mark.parametrize("node", range(6))
def test_singular_rules_integrate_polynomials(oracle_lib, node):
    s, t, w = oracle.rule(2, node, 8)
    assert abs(w.sum() - 0.5) < 1e-14
    for a in range(5):
        for b in range(5 - a):
            assert abs(np.sum(w * s ** a * t ** b) - exact_monomial(a, b)) < 1e-14


def test_shape_functions_partition_and_interpolate(oracle_lib):
    nodes = [(0, 0), (1, 0), (0, 1), (0.5, 0), (0.5, 0.5), (0, 0.5)]
    for b, (s, t) in enumerate(nodes):
        L, Ls, Lt = oracle.shape(s, t)
        assert np.allclose(L, np.eye(6)[b], atol=1e-15)
    rng = np.random.default_rng(1)
    for _ in range(20):
        s, t = rng.random(2) * 0.5
        L, Ls, Lt = oracle.shape(s, t)
        assert abs(L.sum() - 1) < 1e-15 and abs(Ls.sum()) < 1e-14 and abs(Lt.sum()) < 1e-14
        # derivative against a central difference
        h = 1e-6
        Lp, _, _ = oracle.shape(s + h, t)
        Lm, _, _ = oracle.shape(s - h, t)
        assert np.allclose((Lp - Lm) / (2 * h), Ls, atol=1e-8)


def flat_element(P0, P1, P2):
    P0, P1, P2 = (np.asarray(p, float) for p in (P0, P1, P2))
    return np.array([P0, P1, P2, (P0 + P1) / 2, (P1 + P2) / 2, (P2 + P0) / 2])


def closed_form_inv_r_from_vertex(P, A, B):
    """Integral of 1/|x - P| over the flat triangle (P, A, B): in polar
    coordinates about P the radial integral is the distance to the edge AB,
    h / cos(psi), whose integral is h ln tan(pi/4 + psi/2)."""
    P, A, B = (np.asarray(v, float) for v in (P, A, B))
    e = (B - A) / np.linalg.norm(B - A)
    foot = A + np.dot(P - A, e) * e
    h = np.linalg.norm(foot - P)
    ang = lambda X: math.atan2(np.dot(X - foot, e), h)  # signed angle from the perpendicular
    F = lambda psi: h * math.log(math.tan(math.pi / 4 + psi / 2))
    return F(ang(B)) - F(ang(A))


def test_duffy_corner_against_closed_form(oracle_lib):
    X = flat_element([0.1, -0.2, 0.3], [1.3, 0.1, 0.2], [0.2, 0.9, 0.5])
    ref = closed_form_inv_r_from_vertex(X[0], X[1], X[2])
    mesh = oracle.OracleMesh(X, np.arange(6, dtype=np.int32)[None, :])
    cls, S, K = mesh.pair(0, 0, X[0])
    assert cls == 2
    got = (S.sum() * 4 * math.pi).real
    assert abs(got - ref) / ref < 1e-9  # the 12 x 12 rule the pair integrals use
    # the same Duffy map with 16 x 16 points converges to the closed form
    s, t, w = oracle.rule(2, 0, 16)
    tot = 0.0
    for si, ti, wi in zip(s, t, w):
        y, n, J = oracle.elem_point(X, si, ti)
        tot += wi * J / np.linalg.norm(y - X[0])
    assert abs(tot - ref) / ref < 1e-13
    # the flat element has (x - y).n = 0: the double-layer integral vanishes
    assert np.abs(K).max() < 1e-15


def test_duffy_midside_against_closed_form(oracle_lib):
    X = flat_element([0.0, 0.0, 0.0], [1.0, 0.2, 0.0], [0.3, 1.1, 0.0])
    ref = closed_form_inv_r_from_vertex(X[3], X[1], X[2]) + closed_form_inv_r_from_vertex(X[3], X[2], X[0])
    mesh = oracle.OracleMesh(X, np.arange(6, dtype=np.int32)[None, :])
    cls, S, _ = mesh.pair(0, 3, X[3])
    assert cls == 2
    assert abs((S.sum() * 4 * math.pi).real - ref) / ref < 1e-9


def _collapsed_gauss(n):
    """Independent fine rule on the reference triangle: s = u(1-v), t = uv, Jacobian u."""
    x, w = np.polynomial.legendre.leggauss(n)
    u, wu = (x + 1) / 2, w / 2
    U, V = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu) * U
    return (U * (1 - V)).ravel(), (U * V).ravel(), W.ravel()


def test_near_singular_rule_converges(oracle_lib):
    """A target 0.6 h above a curved element: the subdivision rule the oracle
    picks agrees with an independent 96 x 96 collapsed Gauss rule."""
    import bem_inputs

    m = bem_inputs.icosphere(1)
    mesh = oracle.OracleMesh(m.xyz, m.elem)
    e = 3
    X = m.xyz[m.elem[e]]
    cm = X[:3].mean(0)
    h = np.max(np.linalg.norm(X - cm, axis=1))
    x = cm * (1 + 0.6 * h / np.linalg.norm(cm))
    cls, S, K = mesh.pair(e, -1, x)
    assert cls == 1
    s, t, w = _collapsed_gauss(96)
    refS = np.zeros(6)
    refK = np.zeros(6)
    for si, ti, wi in zip(s, t, w):
        y, n, J = oracle.elem_point(X, si, ti)
        L, _, _ = oracle.shape(si, ti)
        r = x - y
        R = np.linalg.norm(r)
        refS += wi * J * L / (4 * np.pi * R)
        refK += wi * J * L * np.dot(r, n) / (4 * np.pi * R ** 3)
    assert np.abs(S.real - refS).max() < 2e-5 * np.abs(refS).max()
    assert np.abs(K.real - refK).max() < 3e-4 * np.abs(refK).max()  # double layer at 0.6 h: the rule's real accuracy


def test_sphere_area_converges(oracle_lib):
    import bem_inputs

    s, t, w = oracle.rule(0)
    errs = []
    for sub in (1, 2, 3):
        m = bem_inputs.icosphere(sub)
        area = 0.0
        for en in m.elem:
            X = m.xyz[en]
            for si, ti, wi in zip(s, t, w):
                area += wi * oracle.elem_point(X, si, ti)[2]
        errs.append(abs(area - 4 * np.pi))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3 * 4 * np.pi
    assert errs[1] / errs[2] > 10  # quadratic elements: error falls like h^4
