"""Pins for the oracle's tree, lists, derivatives, shifts and fast product
(Sections 3.1-3.6; Eqs. 9-14).

Pinned against: harmonicity of the Green's functions (Laplacian identity on
every computed derivative), closed forms and finite differences at low order,
exactness of the binomial shifts, brute-force tree invariants and pair
coverage, a smooth kernel whose Taylor series terminates (the fast product
must then equal the direct sum to rounding), and the direct product itself.
"""

import itertools

import numpy as np
import pytest

import bem_inputs
import oracle


def test_multi_index_order(oracle_lib):
    e = oracle.multi_index(3)
    assert e.shape == (20, 3)
    assert list(map(tuple, e[:4])) == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    assert np.all(np.diff(e.sum(1)) >= 0)


def _idx(p):
    e = oracle.multi_index(p)
    return {tuple(v): i for i, v in enumerate(e)}, e


@pytest.mark.parametrize("green,k", [(oracle.LAPLACE, 0.0), (oracle.HELMHOLTZ, 1.7), (oracle.HELMHOLTZ, 6.0)])
def test_derivatives_satisfy_helmholtz_equation(oracle_lib, green, k):
    H = 16
    idx, e = _idx(H)
    for r in ([0.7, -0.4, 0.5], [1.5, 0.2, -2.0], [0.1, 0.35, 0.2]):
        D = oracle.derivs(np.array(r), H, green, k)
        for (a, b, c), i in idx.items():
            if a + b + c > H - 2:
                continue
            lap = D[idx[(a + 2, b, c)]] + D[idx[(a, b + 2, c)]] + D[idx[(a, b, c + 2)]]
            scale = max(abs(D[idx[(a + 2, b, c)]]), abs(D[idx[(a, b + 2, c)]]), abs(D[idx[(a, b, c + 2)]]), 1e-300)
            assert abs(lap + k * k * D[i]) <= 1e-10 * scale, ((a, b, c), r)


def test_derivatives_closed_forms(oracle_lib):
    idx, _ = _idx(4)
    r = np.array([0.3, -0.7, 0.45])
    x, y, z = r
    R = np.linalg.norm(r)
    D = oracle.derivs(r, 4)
    assert abs(D[0] - 1 / (4 * np.pi * R)) < 1e-15
    assert abs(D[idx[(1, 0, 0)]] + x / (4 * np.pi * R ** 3)) < 1e-14
    assert abs(D[idx[(1, 1, 0)]] - 3 * x * y / (4 * np.pi * R ** 5)) < 1e-14
    assert abs(D[idx[(0, 0, 2)]] - (3 * z * z - R * R) / (4 * np.pi * R ** 5)) < 1e-14
    # Helmholtz first derivative: d/dx e^{jkR}/(4 pi R) = (jkR - 1) e^{jkR} x / (4 pi R^3)
    k = 2.3
    Dh = oracle.derivs(r, 4, oracle.HELMHOLTZ, k)
    assert abs(Dh[idx[(1, 0, 0)]] - (1j * k * R - 1) * np.exp(1j * k * R) * x / (4 * np.pi * R ** 3)) < 1e-14


def test_helmholtz_derivatives_finite_difference(oracle_lib):
    """Each derivative of order <= 4 against a fourth-order central difference
    of the order below it."""
    idx, e = _idx(6)
    r = np.array([0.6, 0.2, -0.5])
    k = 3.1
    D = oracle.derivs(r, 6, oracle.HELMHOLTZ, k)
    h = 1e-3
    f = lambda rr: oracle.derivs(rr, 6, oracle.HELMHOLTZ, k)
    for (a, b, c), i in idx.items():
        if a + b + c > 3:
            continue
        for d in range(3):
            g = [a, b, c]
            g[d] += 1
            dr = np.zeros(3)
            dr[d] = h
            fd = (8 * (f(r + dr)[i] - f(r - dr)[i]) - (f(r + 2 * dr)[i] - f(r - 2 * dr)[i])) / (12 * h)
            order_scale = np.abs(D[e.sum(1) == sum(g)]).max()
            assert abs(fd - D[idx[tuple(g)]]) < 1e-7 * order_scale


def test_shift_operators_are_exact(oracle_lib):
    p = 8
    rng = np.random.default_rng(3)
    pts = rng.random((50, 3)) - 0.5
    w = rng.standard_normal(50)
    c_child = np.array([0.1, -0.05, 0.2])
    c_par = np.array([-0.2, 0.15, 0.05])
    Mc = oracle.mono_moments(p, c_child, pts, w)
    Mp = oracle.m2m(p, c_child - c_par, Mc)
    assert np.abs(Mp - oracle.mono_moments(p, c_par, pts, w)).max() < 1e-13 * np.abs(Mp).max()
    # L2L: a polynomial re-expanded about another centre evaluates identically
    idx, e = _idx(p)
    F = rng.standard_normal(len(e))
    Fc = oracle.l2l(p, c_child - c_par, F)
    for x in rng.random((5, 3)) - 0.5:
        v1 = sum(F[i] * np.prod((x - c_par) ** e[i]) for i in range(len(e)))
        v2 = sum(Fc[i] * np.prod((x - c_child) ** e[i]) for i in range(len(e)))
        assert abs(v1 - v2) < 1e-12 * max(1, abs(v1))


def test_local_expansion_single_source_converges(oracle_lib):
    """One source, one target, two centres: the error of the truncated M2L
    product falls roughly like rho^(p+1) with rho the separation ratio."""
    src = np.array([[0.05, -0.03, 0.04]])
    cs, ct = np.zeros(3), np.array([1.0, 0.2, -0.1])
    x = ct + np.array([-0.06, 0.05, 0.02])
    exact = 1 / (4 * np.pi * np.linalg.norm(x - src[0]))
    errs = []
    for p in (2, 4, 6, 8):
        idx, e = _idx(p)
        M = oracle.mono_moments(p, cs, src, np.ones(1))
        D = oracle.derivs(ct - cs, 2 * p)
        idx2, _ = _idx(2 * p)
        import math
        fact = lambda g: math.factorial(int(g[0])) * math.factorial(int(g[1])) * math.factorial(int(g[2]))
        F = np.zeros(len(e), complex)
        for bi, bb in enumerate(e):
            for ai, aa in enumerate(e):
                F[bi] += (-1) ** aa.sum() * D[idx2[tuple(aa + bb)]] * M[ai] / (fact(aa) * fact(bb))
        val = sum(F[i] * np.prod((x - ct) ** e[i]) for i in range(len(e)))
        errs.append(abs(val - exact) / exact)
    assert errs[-1] < 1e-9
    assert all(errs[i + 1] < errs[i] * 0.1 for i in range(3))


# ---------------------------------------------------------------- tree
@pytest.fixture(scope="module")
def small_tree(oracle_lib):
    m = bem_inputs.icosphere(3)
    om = oracle.OracleMesh(m.xyz, m.elem)
    return om, oracle.OracleTree(om, B=16, theta=0.7)


def _keys_inside(T, b, keys):
    s = 3 * (21 - T.level[b])
    return (keys >> s) == T.prefix[b]


def test_tree_partition_and_leaf_sizes(small_tree):
    om, T = small_tree
    leaves = np.flatnonzero(T.leaf)
    # every element and target belongs to exactly one leaf
    ecount = np.zeros(om.n_el, int)
    tcount = np.zeros(om.n_dof, int)
    for b in leaves:
        ecount[T.eperm[T.eb[b]:T.ee[b]]] += 1
        tcount[T.tperm[T.tb[b]:T.te[b]]] += 1
    assert np.all(ecount == 1) and np.all(tcount == 1)
    assert np.all(T.ee[leaves] - T.eb[leaves] <= T.B)
    # non-leaves hold more than B elements; children nest in parents
    nl = np.flatnonzero(T.leaf == 0)
    assert np.all(T.ee[nl] - T.eb[nl] > T.B)
    for b in range(1, T.n_box):
        p = T.parent[b]
        assert T.level[p] == T.level[b] - 1 and T.prefix[b] >> 3 == T.prefix[p]
        assert T.eb[p] <= T.eb[b] and T.ee[b] <= T.ee[p]
    # boxes ordered by (level, prefix)
    order = np.lexsort((T.prefix, T.level))
    assert np.all(order == np.arange(T.n_box))


def test_tree_radii_cover(small_tree):
    om, T = small_tree
    for b in range(T.n_box):
        els = T.eperm[T.eb[b]:T.ee[b]]
        pts = om.xyz[om.elem[els].ravel()] if len(els) else np.zeros((0, 3))
        tg = om.dof_xyz[T.tperm[T.tb[b]:T.te[b]]]
        allp = np.concatenate([pts, tg])
        dmax = np.linalg.norm(allp - T.centre[b], axis=1).max()
        assert dmax <= T.radius[b] * (1 + 1e-15)
        # centres are the geometric centres of the Morton cells
        h = T.side / 2 ** T.level[b]
        lo = T.corner + h * np.floor((T.centre[b] - T.corner) / h)
        assert np.allclose(T.centre[b], lo + h / 2)
    # Eq. 13 on every parent
    for b in np.flatnonzero(T.leaf == 0):
        ch = range(T.child_begin[b], T.child_begin[b] + T.nchild[b])
        hc = T.side / 2 ** (T.level[b] + 1)
        assert T.radius[b] == max(T.radius[c] for c in ch) + (np.sqrt(3.0) * hc) * 0.5


def _sep(T, a, b):
    return np.linalg.norm(T.centre[a] - T.centre[b]) > (T.radius[a] + T.radius[b]) / T.theta


def test_lists_respect_criterion_and_cover_each_pair_once(small_tree):
    om, T = small_tree
    near = [set(T.near_idx[T.near_ptr[b]:T.near_ptr[b + 1]]) for b in range(T.n_box)]
    inter = [set(T.inter_idx[T.inter_ptr[b]:T.inter_ptr[b + 1]]) for b in range(T.n_box)]
    for b in range(T.n_box):
        for s in inter[b]:
            assert _sep(T, b, s)
        for s in near[b]:
            assert (not _sep(T, b, s)) or False
        assert list(T.near_idx[T.near_ptr[b]:T.near_ptr[b + 1]]) == sorted(near[b])
    # brute force: every (target leaf, element) pair is covered exactly once by
    # an interaction-list entry of the target leaf or an ancestor, or a near entry of the leaf
    def anc(b):
        out = []
        while b >= 0:
            out.append(b)
            b = T.parent[b]
        return out

    elem_box_chain = {}
    for b in np.flatnonzero(T.leaf):
        for e in T.eperm[T.eb[b]:T.ee[b]]:
            elem_box_chain[e] = set(anc(b))
    for t in np.flatnonzero(T.leaf):
        if T.te[t] == T.tb[t]:
            continue
        chain = anc(t)
        for e in range(om.n_el):
            src = elem_box_chain[e]
            n = sum(len(inter[a] & src) for a in chain) + len(near[t] & src)
            assert n == 1, (t, e, n)


def test_tree_brute_force_small_mesh(oracle_lib):
    """On an 80-element mesh, rebuild boxes by enumerating every Morton prefix."""
    m = bem_inputs.icosphere(2)
    sel = m.elem[:80]
    om = oracle.OracleMesh(m.xyz, sel)
    T = oracle.OracleTree(om, B=6, theta=1.0)
    # keys recomputed here from the definition
    scale = 2 ** 21 / T.side

    def key(p):
        q = np.clip(np.floor((p - T.corner) * scale), 0, 2 ** 21 - 1).astype(np.int64)
        k = 0
        for bit in range(21):
            for d in range(3):
                k |= int((q[d] >> bit) & 1) << (3 * bit + 2 - d)
        return k

    ek = np.array([key(((m.xyz[en[0]] + m.xyz[en[1]]) + m.xyz[en[2]]) / 3.0) for en in sel])
    tk = np.array([key(p) for p in om.dof_xyz])
    assert np.all(np.sort(ek) == ek[T.eperm])
    boxes = set()
    frontier = [(0, 0)]
    while frontier:
        lev, pre = frontier.pop()
        s = 3 * (21 - lev)
        ne = np.sum((ek >> s) == pre) if lev else len(ek)
        nt = np.sum((tk >> s) == pre) if lev else len(tk)
        if ne + nt == 0:
            continue
        boxes.add((lev, pre))
        if ne > 6 and lev < 21:
            frontier += [(lev + 1, (pre << 3) | c) for c in range(8)]
    assert boxes == set(zip(T.level.tolist(), T.prefix.tolist()))


# ---------------------------------------------------------------- fast product
@pytest.fixture(scope="module")
def fmm_case(oracle_lib):
    m = bem_inputs.icosphere(3)
    om = oracle.OracleMesh(m.xyz, m.elem)
    x = bem_inputs.random_vector(om.n_dof, 11)[0]
    return om, x


@pytest.mark.parametrize("op", [oracle.OP_S_REG, oracle.OP_K_REG])
def test_fmm_exact_for_terminating_taylor_series(fmm_case, op):
    """G = |r|^2 has a Taylor series ending at degree 2: the fast product must
    equal the direct 7-point sum to rounding, which proves that every
    (target, source) pair is counted once through the lists and shifts."""
    om, x = fmm_case
    for theta in (1.0, 0.5):
        T = oracle.OracleTree(om, B=16, theta=theta)
        for p in (2, 5):
            yf = T.fmm_matvec(x, op, green=oracle.R2, order=p)
            yd = om.matvec_rows(x, op, green=oracle.R2)
            assert np.linalg.norm(yf - yd) / np.linalg.norm(yd) < 1e-13


def test_fmm_converges_to_direct(fmm_case):
    om, x = fmm_case
    T = oracle.OracleTree(om, B=32, theta=0.7)
    yd = om.matvec_rows(x, oracle.OP_A)
    errs = []
    for p in (2, 4, 8):
        yf = T.fmm_matvec(x, oracle.OP_A, order=p)
        errs.append(np.linalg.norm(yf - yd) / np.linalg.norm(yd))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


def test_fmm_helmholtz_to_direct(fmm_case):
    om, x = fmm_case
    k = 2.0
    T = oracle.OracleTree(om, B=32, theta=0.7, kappa=3.0, k=k)
    for op in (oracle.OP_A, oracle.OP_RHS):
        yd = om.matvec_rows(x, op, oracle.HELMHOLTZ, k)
        yf = T.fmm_matvec(x, op, oracle.HELMHOLTZ, k, order=8)
        assert np.linalg.norm(yf - yd) / np.linalg.norm(yd) < 1e-5


# ---------------------------------------------------------------- level-dependent order (Section 3.6)
def _quadrature_sources(om, x):
    """Points, normals and strengths wJ sum_a L_a x_a of the 7-point rule on
    every element (element id order)."""
    s, t, w = oracle.rule(0)
    ys, ns, qs = [], [], []
    for e in range(om.n_el):
        X6 = om.xyz[om.elem[e]]
        for q in range(len(w)):
            y, n, J = oracle.elem_point(X6, s[q], t[q])
            L, _, _ = oracle.shape(s[q], t[q])
            ys.append(y)
            ns.append(n)
            qs.append(w[q] * J * np.dot(L, x[om.elem_dofs[e]]))
    return np.array(ys), np.array(ns), np.array(qs)


@pytest.mark.parametrize("op", [oracle.OP_S_REG, oracle.OP_K_REG])
def test_level_order_drops_exactly_the_truncated_terms(fmm_case, op):
    """G = |r|^2 with L_min = 1: only the deepest level has order 1, every
    coarser level order >= 2, which the kernel needs.  Then the fast product
    differs from the direct sum by exactly the terms the order-1 expansions
    drop.  A source in a deepest-level leaf S keeps its charge and dipole
    about c_S but loses its second moment, whose field is the constant
    sigma |y - c_S|^2 (single layer) or 2 sigma n . (y - c_S) (double layer);
    a target in a deepest-level leaf T loses the quadratic part of its far
    field about c_T, Q_far |x - c_T|^2, where Q_far is the total far strength
    (single layer; the double layer's far field is linear in x).  With
    L_min = 2 every order is >= 2 and the product equals the direct sum."""
    om, x = fmm_case
    T = oracle.OracleTree(om, B=16, theta=0.7)
    lmax = int(T.level.max())
    dbl = op == oracle.OP_K_REG
    y, n, qs = _quadrature_sources(om, x)
    leaf_of_q = np.zeros(len(qs), np.int64)
    for b in np.nonzero(T.leaf)[0]:
        for se in range(T.eb[b], T.ee[b]):
            leaf_of_q[7 * T.eperm[se]:7 * T.eperm[se] + 7] = b
    c_q = T.centre[leaf_of_q]
    drop_src = 2.0 * qs * np.einsum("ij,ij->i", n, y - c_q) if dbl else qs * np.sum((y - c_q) ** 2, 1)
    deep_src = T.level[leaf_of_q] == lmax
    expect = om.matvec_rows(x, op, green=oracle.R2)
    n_deep_targets = 0
    for b in np.nonzero(T.leaf)[0]:
        if T.te[b] == T.tb[b]:
            continue
        # near boxes (leaves, or larger boxes beside a coarse leaf) are summed directly
        far = np.ones(len(qs), bool)
        for s in T.near_idx[T.near_ptr[b]:T.near_ptr[b + 1]]:
            for se in range(T.eb[s], T.ee[s]):
                far[7 * T.eperm[se]:7 * T.eperm[se] + 7] = False
        for tpos in range(T.tb[b], T.te[b]):
            i = T.tperm[tpos]
            xi = om.xyz[om.dof_node[i]]
            expect[i] -= np.sum(drop_src[far & deep_src])
            if T.level[b] == lmax and not dbl:
                expect[i] -= np.sum(qs[far]) * np.sum((xi - T.centre[b]) ** 2)
                n_deep_targets += 1
    assert T.inter_idx.size and (dbl or n_deep_targets)
    yf = T.fmm_matvec(x, op, green=oracle.R2, order=5, order_min=1)
    yd = om.matvec_rows(x, op, green=oracle.R2)
    assert np.linalg.norm(yf - yd) / np.linalg.norm(yd) > 1e-6  # the truncation is visible
    assert np.linalg.norm(yf - expect) / np.linalg.norm(yd) < 1e-13
    y2 = T.fmm_matvec(x, op, green=oracle.R2, order=5, order_min=2)
    assert np.linalg.norm(y2 - yd) / np.linalg.norm(yd) < 1e-13


def test_level_order_error_ordering(fmm_case):
    """Laplace: order_min >= order is the uniform product bit for bit, and
    the error against the direct product falls as L_min rises (Section 4's
    reference runs use L_min = 3 and 4 with L_max = 8)."""
    om, x = fmm_case
    T = oracle.OracleTree(om, B=16, theta=0.7)
    yd = om.matvec_rows(x, oracle.OP_A)
    y8 = T.fmm_matvec(x, oracle.OP_A, order=8)
    assert np.array_equal(T.fmm_matvec(x, oracle.OP_A, order=8, order_min=8), y8)
    errs = [np.linalg.norm(T.fmm_matvec(x, oracle.OP_A, order=8, order_min=m) - yd) / np.linalg.norm(yd)
            for m in (2, 3, 4)]
    e8 = np.linalg.norm(y8 - yd) / np.linalg.norm(yd)
    assert errs[0] > errs[1] > errs[2] > e8


@pytest.mark.parametrize("name,B", [("sphere1280", 16), ("cube4", 8)])
def test_attached_radii_cover_attached_elements(oracle_lib, name, B):
    """Attach mode: every node of every element holding a leaf target's node
    lies within the leaf's radius (brute force over the mesh); single-owner
    radii miss some of them, and attach radii are never smaller."""
    m = bem_inputs.workload(name)
    om = oracle.OracleMesh(m.xyz, m.elem)
    Ta = oracle.OracleTree(om, B=B, theta=1.0, attach=True)
    To = oracle.OracleTree(om, B=B, theta=1.0)
    assert np.array_equal(Ta.level, To.level) and np.all(Ta.radius >= To.radius)
    holders = [[] for _ in range(m.n_nodes)]
    for e, en in enumerate(m.elem):
        for g in en:
            holders[g].append(e)
    missed = 0
    for b in np.nonzero(Ta.leaf)[0]:
        c = Ta.centre[b]
        for t in range(Ta.tb[b], Ta.te[b]):
            g = om.dof_node[Ta.tperm[t]]
            pts = m.xyz[m.elem[holders[g]].ravel()]
            d = np.sqrt(((pts - c) ** 2).sum(1)).max()
            assert d <= Ta.radius[b] * (1 + 1e-15)
            missed += d > To.radius[b]
    assert missed > 0


@pytest.mark.parametrize("op", [oracle.OP_S_REG, oracle.OP_K_REG])
def test_literal_tree_exact_for_terminating_taylor_series(fmm_case, op):
    """The paper's tree read literally (boxes over the DOF points, every
    DOF's basis function a source over its element patch): with G = |r|^2 the
    fast product equals the direct sum, so every (DOF, element slot) piece is
    counted exactly once; leaves hold at most B DOFs."""
    om, x = fmm_case
    for B in (8, 16):
        T = oracle.OracleTree(om, B=B, theta=0.7, literal=True)
        assert np.array_equal(T.eb, T.tb) and np.array_equal(T.ee, T.te)
        assert np.all((T.te - T.tb)[T.leaf.astype(bool)] <= B) and T.inter_idx.size
        yf = T.fmm_matvec(x, op, green=oracle.R2, order=3)
        yd = om.matvec_rows(x, op, green=oracle.R2)
        assert np.linalg.norm(yf - yd) / np.linalg.norm(yd) < 1e-13


def test_literal_tree_converges_to_direct(fmm_case):
    om, x = fmm_case
    T = oracle.OracleTree(om, B=16, theta=0.7, literal=True)
    yd = om.matvec_rows(x, oracle.OP_A)
    errs = [np.linalg.norm(T.fmm_matvec(x, oracle.OP_A, order=p) - yd) / np.linalg.norm(yd) for p in (2, 4, 8)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6
