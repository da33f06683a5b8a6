"""GPU parity: the HIP library through its C interface against the oracle.

Bars: DOF layout, tree and lists bit-exact; direct FP64 product within 1e-10
relative of the oracle's dense definition; FP64 fast product within 1e-11 of
the oracle's fast product (same tree, same order); both fast products, FP64
and mixed precision, within the stated truncation tolerance 1e-6 of the
oracle's direct product, and the mixed one within 1e-6 of the oracle's fast
product on the same tree; solves to a 1e-8 residual.  Every product bar holds
in two measures: the 2-norm of the error over the 2-norm of the reference,
and the largest row error over the largest reference row (so that one bad
row cannot hide in the norm).

The bare double layer K enters the solve only through A x = c.x - K x, and
its absolute error is A's; its error is therefore stated relative to the
norm of A x on the same x (K x itself is small: relative to its own norm the
same error reads about 100 times larger).
"""

import numpy as np
import pytest

import bem_inputs
import oracle
from oracle import analytic

from gpu_common import context, mesh_by_name, rel, relmax, say, to_dev

pytestmark = pytest.mark.gpu

THETA = 0.5  # the library's default separation factor
PRODUCT_TOL = 1e-6  # stated truncation tolerance of the fast product (order 8), both precisions


def check_product(y, ref, tol, label, norm_ref=None):
    """Both error measures of a product against its reference: 2-norm and
    largest row, each relative to norm_ref (default: the reference)."""
    y, ref = np.asarray(y), np.asarray(ref)
    nr = ref if norm_ref is None else np.asarray(norm_ref)
    e2 = float(np.linalg.norm(y - ref) / np.linalg.norm(nr))
    em = float(np.abs(y - ref).max() / np.abs(nr).max())
    say(f"    {label}: 2-norm {e2:.2e} max-row {em:.2e} (bar {tol:.0e})")
    assert e2 < tol and em < tol, (label, e2, em)
    return e2, em


def _bem():
    import paper_0908_0673_amd as bem

    return bem


_cache = {}


def setup(name, B=32, theta=THETA, kappa=0.0, k_hint=0.0, order_min=0, attach=False):
    key = (name, B, theta, kappa, k_hint, order_min, attach)
    if key not in _cache:
        bem = _bem()
        say(f"[setup] mesh={name} B={B} theta={theta} kappa={kappa} order_min={order_min}")
        m = mesh_by_name(name)
        ctx = context()
        mesh = bem.bem_mesh_load(ctx, m.xyz, m.elem)
        # attach: False, True (attached radii) or "literal" (the paper's tree read literally)
        tree = bem.bem_tree_build(ctx, mesh, B=B, order=8, theta=theta, kappa=kappa, k_hint=k_hint,
                                  order_min=order_min, attach_radii=2 if attach == "literal" else int(attach))
        om = oracle.OracleMesh(m.xyz, m.elem)
        ot = oracle.OracleTree(om, B=B, theta=theta, kappa=kappa if kappa > 0 else float("inf"), k=k_hint,
                               attach=bool(attach), literal=attach == "literal")
        _cache[key] = (m, ctx, mesh, tree, om, ot)
    return _cache[key]


# ---------------------------------------------------------------- DOFs, tree
@pytest.mark.parametrize("name", ["sphere320", "cube4", "perturbed", "cube1", "sphere1280_p1", "cube4_p1",
                                  "perturbed_p1", "icosphere1_p1"])
def test_dof_layout_matches_oracle(name):
    m, ctx, mesh, tree, om, ot = setup(name)
    d = mesh.dofs()
    assert mesh.n_dof == om.n_dof
    assert np.array_equal(d["elem_dofs"], om.elem_dofs)
    assert np.array_equal(d["dof_node"], om.dof_node)
    assert np.allclose(d["dof_normal"], om.dof_normal, atol=1e-14)


TREE_CASES = [("sphere320", 32, 1.0), ("sphere320", 8, 0.6), ("sphere1280", 16, 0.6), ("cube4", 8, 1.0),
              ("cube4", 32, 0.5), ("perturbed", 10, 0.6), ("ellipsoid", 12, 0.7), ("sphere20480", 32, 0.6),
              ("cube24300", 32, 0.6), ("sphere1280_p1", 16, 0.6), ("cube4_p1", 8, 0.6), ("sphere20480_p1", 32, 0.6)]


ATTACH_CASES = [("sphere1280", 16, 1.0, True), ("cube4", 8, 1.0, True), ("sphere1280_p1", 16, 1.0, True),
                ("perturbed", 10, 0.6, True), ("sphere1280", 32, 1.0, "literal"), ("cube4", 16, 1.0, "literal"),
                ("sphere1280_p1", 16, 1.0, "literal"), ("sphere20480", 64, 0.6, "literal")]


@pytest.mark.parametrize("name,B,theta,attach", [c + (False,) for c in TREE_CASES] + ATTACH_CASES)
def test_tree_and_lists_bit_exact(name, B, theta, attach):
    """Attached radii (the paper's r_C over the elements attached to a leaf's
    vertices) included."""
    m, ctx, mesh, tree, om, ot = setup(name, B=B, theta=theta, attach=attach)
    ex = tree.export()
    say(f"  boxes {ex['level'].size} leaves {ex['n_leaf']} near {ex['near_idx'].size} inter {ex['inter_idx'].size}")
    assert ex["level"].size == ot.n_box
    assert np.array_equal(ex["root"][:3], ot.corner) and ex["root"][3] == ot.side
    lit = attach == "literal"  # the element fields then describe element pieces, not the oracle's DOF ranges
    for k, o in (("level", ot.level), ("leaf", ot.leaf), ("parent", ot.parent), ("nchild", ot.nchild),
                 ("elem_begin", ot.eb), ("elem_end", ot.ee), ("tgt_begin", ot.tb), ("tgt_end", ot.te)):
        if lit and k.startswith("elem"):
            continue
        assert np.array_equal(ex[k].astype(np.int64), np.asarray(o, np.int64)), k
    assert np.array_equal(ex["prefix"].astype(np.uint64), ot.prefix.astype(np.uint64))
    has_child = ot.nchild > 0
    assert np.array_equal(ex["child_begin"][has_child], ot.child_begin[has_child])
    # FP64 bit patterns of centres and radii
    assert np.array_equal(ex["centre"].view(np.uint64), ot.centre.view(np.uint64))
    assert np.array_equal(ex["radius"].view(np.uint64), ot.radius.view(np.uint64))
    assert lit or np.array_equal(ex["elem_perm"], ot.eperm)
    assert np.array_equal(ex["tgt_perm"], ot.tperm)
    if lit:  # every box's pieces are the elements holding its DOFs, each slot in one piece
        assert np.all(ex["elem_end"] >= ex["elem_begin"]) and ex["elem_begin"][0] == 0
        assert np.all((ex["tgt_end"] - ex["tgt_begin"])[ex["leaf"] == 1] <= B)
    assert np.array_equal(ex["near_ptr"], ot.near_ptr) and np.array_equal(ex["near_idx"], ot.near_idx)
    assert np.array_equal(ex["inter_ptr"], ot.inter_ptr) and np.array_equal(ex["inter_idx"], ot.inter_idx)


def test_tree_root_is_leaf_for_tiny_mesh():
    m, ctx, mesh, tree, om, ot = setup("icosphere0")  # 20 elements <= B
    ex = tree.export()
    assert ex["level"].size == 1 and ex["leaf"][0] == 1
    assert list(ex["near_idx"]) == [0] and ex["inter_idx"].size == 0


# ---------------------------------------------------------------- direct product
OPS = [0, 1, 2, 3]  # S, K, A, RHS


@pytest.mark.parametrize("name", ["sphere320", "sphere320_p1"])
@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_direct_matches_oracle_dense(name, green, k):
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup(name)
    cplx = green == 1
    x = bem_inputs.random_vector(om.n_dof, 21, complex_=cplx)[0]
    xd = to_dev(x, cplx)
    yd = xd.clone()
    S, K, c = om.assemble(green, k)
    refs = {0: S @ x, 1: K @ x, 2: c * x - K @ x, 3: -(S @ x)}
    for op in OPS:
        say(f"  direct green={green} op={op}")
        bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_DIRECT, bem.BEM_PREC_FP64, xd, yd)
        y = yd.cpu().numpy()[0]
        ref = refs[op] if cplx else refs[op].real
        assert rel(y, ref) < 1e-10 and relmax(y, ref) < 1e-10, (op, rel(y, ref))


def test_direct_on_cube_with_sharp_edges():
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("cube4")
    x = bem_inputs.random_vector(om.n_dof, 22)[0]
    xd = to_dev(x, False)
    yd = xd.clone()
    S, K, c = om.assemble()
    bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_DIRECT, bem.BEM_PREC_FP64, xd, yd)
    assert rel(yd.cpu().numpy()[0], (c * x - K @ x).real) < 1e-10


def test_free_term_shared_by_trees_of_one_mesh():
    """The free term is computed once per mesh and tree hierarchy (leaf size,
    depth, kind) and copied by later trees of that hierarchy: a later tree
    with another separation factor and wavenumber bound gives the first
    tree's product A bitwise, a tree of another leaf size computes its own,
    and all are within 1e-10 of the oracle's dense definition."""
    bem = _bem()
    m = mesh_by_name("cube4")
    ctx = context()
    mesh = bem.bem_mesh_load(ctx, m.xyz, m.elem)
    om = oracle.OracleMesh(m.xyz, m.elem)
    S, K, c = om.assemble()
    x = bem_inputs.random_vector(om.n_dof, 23)[0]
    xd = to_dev(x, False)
    yd = xd.clone()
    ys = []
    for B, theta, kappa, k_hint in ((32, 0.5, 0.0, 0.0), (16, 0.5, 0.0, 0.0), (32, 0.6, 2.2, 3.0)):
        tree = bem.bem_tree_build(ctx, mesh, B=B, order=8, theta=theta, kappa=kappa, k_hint=k_hint)
        bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_DIRECT, bem.BEM_PREC_FP64, xd, yd)
        ys.append(yd.cpu().numpy()[0].copy())
        tree.close()
    mesh.close()
    ref = (c * x - K @ x).real
    for y in ys:
        assert rel(y, ref) < 1e-10 and relmax(y, ref) < 1e-10
    assert np.array_equal(ys[0], ys[2])


# ---------------------------------------------------------------- fast product
@pytest.mark.parametrize("name", ["sphere320", "sphere1280", "cube4", "perturbed", "sphere1280_p1", "cube4_p1",
                                  "perturbed_p1"])
@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_fmm_matches_oracle(name, green, k):
    """Every operator, both precisions: the FP64 fast product equals the
    oracle's fast product on the same tree (1e-11), the mixed one deviates
    from it by at most 1e-6, and both are within the truncation tolerance
    1e-6 of the oracle's direct product (C1 is the 320-element sphere)."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup(name)
    cplx = green == 1
    x = bem_inputs.random_vector(om.n_dof, 23, complex_=cplx)[0]
    xd = to_dev(x, cplx)
    yd = xd.clone()
    fix = (lambda v: v) if cplx else (lambda v: v.real)
    dref = {op: fix(om.matvec_rows(x, op, green, k)) for op in OPS}
    for op in OPS:
        ref = fix(ot.fmm_matvec(x, op, green, k))
        nref = dref[2] if op == 1 else None  # K: relative to A x (see the module docstring)
        for prec in (bem.BEM_PREC_FP64, bem.BEM_PREC_MIXED):
            say(f"  fmm {name} green={green} op={op} prec={prec}")
            bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_FMM, prec, xd, yd)
            y = yd.cpu().numpy()[0]
            if prec == bem.BEM_PREC_FP64:
                check_product(y, ref, 1e-11, "fp64 vs oracle fast product", nref)
            else:
                check_product(y, ref, PRODUCT_TOL, "mixed vs oracle fast product", nref)
            check_product(y, dref[op], PRODUCT_TOL, "vs oracle direct product", nref)


@pytest.mark.parametrize("name,B", [("sphere1280", 32), ("cube4", 16), ("sphere1280_p1", 16)])
@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_literal_tree_products_match_oracle(name, B, green, k):
    """The paper's tree read literally (DOF sources over their element
    patches, B counting DOFs, attached radii): the direct product equals the
    oracle's dense one (the element pieces partition every element's shape
    functions), the FP64 fast product the oracle's literal fast product, and
    the mixed one within 1e-6 of it (2-norm and largest row)."""
    bem = _bem()
    cplx = green == 1
    m, ctx, mesh, tree, om, ot = setup(name, B=B, theta=1.0, order_min=3, attach="literal")
    x = bem_inputs.random_vector(om.n_dof, 28, complex_=cplx)[0]
    xd = to_dev(x, cplx)
    yd = xd.clone()
    for op in (bem.BEM_OP_A, bem.BEM_OP_RHS):
        dref = om.matvec_rows(x, op, green, k)
        bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_DIRECT, bem.BEM_PREC_FP64, xd, yd)
        e_dir = rel(yd.cpu().numpy()[0], dref if cplx else dref.real)
        ref = ot.fmm_matvec(x, op, green, k, order=8, order_min=3)
        ref = ref if cplx else ref.real
        bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_FMM, bem.BEM_PREC_FP64, xd, yd)
        e64 = rel(yd.cpu().numpy()[0], ref)
        bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_FMM, bem.BEM_PREC_MIXED, xd, yd)
        e32 = rel(yd.cpu().numpy()[0], ref)
        say(f"  literal {name} green={green} op={op}: direct {e_dir:.2e} fp64 {e64:.2e} mixed {e32:.2e} "
            f"(truncation {rel(ref, dref if cplx else dref.real):.2e})")
        assert e_dir < 1e-10 and e64 < 1e-11
        check_product(yd.cpu().numpy()[0], ref, PRODUCT_TOL, "mixed vs oracle fast product")


@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_fmm_attached_radii_matches_oracle(green, k):
    """The paper's tree settings (attached radii, theta = 1, L_min = 3): the
    FP64 product against the oracle's on the same tree, and its error against
    the direct product far below that of the single-owner radii."""
    bem = _bem()
    cplx = green == 1
    errs = {}
    for attach in (False, True):
        m, ctx, mesh, tree, om, ot = setup("sphere1280", B=16, theta=1.0, order_min=3, attach=attach)
        x = bem_inputs.random_vector(om.n_dof, 27, complex_=cplx)[0]
        xd = to_dev(x, cplx)
        yd = xd.clone()
        ref = ot.fmm_matvec(x, bem.BEM_OP_A, green, k, order=8, order_min=3)
        ref = ref if cplx else ref.real
        bem.bem_matvec(ctx, tree, green, k, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_FP64, xd, yd)
        y = yd.cpu().numpy()[0]
        dref = om.matvec_rows(x, bem.BEM_OP_A, green, k)
        errs[attach] = rel(y, dref if cplx else dref.real)
        say(f"  attach={attach} green={green}: vs oracle fmm {rel(y, ref):.2e}, vs direct {errs[attach]:.2e}")
        assert rel(y, ref) < 1e-11
    assert errs[True] < 0.5 * errs[False]


@pytest.mark.parametrize("name,B", [("sphere1280", 16), ("sphere1280", 4), ("cube4", 8)])
@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_fmm_level_dependent_order_matches_oracle(name, B, green, k):
    """Section 3.6's level-dependent order, L_l = min(8, L_min + l_max - l),
    at the paper's L_min = 3 and 4: the FP64 product against the oracle's
    fast product with the same orders (1e-11), the mixed one within 1e-6 of
    it (2-norm and largest row)."""
    bem = _bem()
    cplx = green == 1
    for m_ in (3, 4):
        m, ctx, mesh, tree, om, ot = setup(name, B=B, order_min=m_)
        x = bem_inputs.random_vector(om.n_dof, 26, complex_=cplx)[0]
        xd = to_dev(x, cplx)
        yd = xd.clone()
        levels = ot.level.max()
        for op in (bem.BEM_OP_A, bem.BEM_OP_RHS):
            ref = ot.fmm_matvec(x, op, green, k, order=8, order_min=m_)
            ref = ref if cplx else ref.real
            bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_FMM, bem.BEM_PREC_FP64, xd, yd)
            e64 = rel(yd.cpu().numpy()[0], ref)
            bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_FMM, bem.BEM_PREC_MIXED, xd, yd)
            e32 = rel(yd.cpu().numpy()[0], ref)
            say(f"  {name} L_min={m_} l_max={levels} green={green} op={op}: fp64 {e64:.2e} mixed {e32:.2e}")
            assert e64 < 1e-11, (op, e64)
            check_product(yd.cpu().numpy()[0], ref, PRODUCT_TOL, "mixed vs oracle fast product")


@pytest.mark.parametrize("name", ["sphere1280", "sphere5120"])
@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_fmm_mixed_error_against_oracle(name, green, k):
    """The mixed-precision product against the oracle's direct product on
    every row, all four operators, within 1e-6 in both measures."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup(name)
    cplx = green == 1
    x = bem_inputs.random_vector(om.n_dof, 24, complex_=cplx)[0]
    xd = to_dev(x, cplx)
    yd = xd.clone()
    fix = (lambda v: v) if cplx else (lambda v: v.real)
    dref = {op: fix(om.matvec_rows(x, op, green, k)) for op in OPS}
    for op in OPS:
        bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_FMM, bem.BEM_PREC_MIXED, xd, yd)
        check_product(yd.cpu().numpy()[0], dref[op], PRODUCT_TOL, f"mixed {name} green={green} op={op}",
                      dref[2] if op == 1 else None)


@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_mixed_product_scales_exactly(green, k):
    """The mixed product of 2^s x is 2^s times that of x, bit for bit, for
    s = -40 and 40: every step is linear and a power-of-two factor commutes
    with rounding, so this holds while nothing overflows or underflows.  The
    matrix-instruction products carry their operands as fp16 terms (largest
    finite value 65504), so it holds only because each moment vector and
    each operator row is brought into range by its own power-of-two scale."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere1280")
    cplx = green == 1
    x = bem_inputs.random_vector(om.n_dof, 31, complex_=cplx)[0]
    y1 = to_dev(x, cplx)
    bem.bem_matvec(ctx, tree, green, k, 2, bem.BEM_FMM, bem.BEM_PREC_MIXED, to_dev(x, cplx), y1)
    base = y1.cpu().numpy()[0]
    for s in (-40, 40):
        xs = to_dev(x * 2.0 ** s, cplx)
        ys = xs.clone()
        bem.bem_matvec(ctx, tree, green, k, 2, bem.BEM_FMM, bem.BEM_PREC_MIXED, xs, ys)
        got = ys.cpu().numpy()[0] * 2.0 ** -s
        say(f"    green={green} s={s}: largest difference {np.abs(got - base).max():.3e}")
        assert np.array_equal(got, base), (green, s)


def test_multiple_rhs_equal_single_calls():
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    X = bem_inputs.random_vector(om.n_dof, 25, nrhs=3)
    xd = to_dev(X, False)
    yd = xd.clone()
    for prec in (bem.BEM_PREC_FP64, bem.BEM_PREC_MIXED):
        bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, xd, yd)
        Y = yd.cpu().numpy()
        for r in range(3):
            x1 = xd[r:r + 1].clone()
            y1 = x1.clone()
            bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, x1, y1)
            assert np.array_equal(y1.cpu().numpy()[0], Y[r])


def test_repeat_is_bitwise_identical():
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere1280")
    x = bem_inputs.random_vector(om.n_dof, 26)[0]
    xd = to_dev(x, False)
    y1, y2 = xd.clone(), xd.clone()
    for prec in (bem.BEM_PREC_FP64, bem.BEM_PREC_MIXED):
        bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, xd, y1)
        bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, prec, xd, y2)
        assert np.array_equal(y1.cpu().numpy(), y2.cpu().numpy())


# ---------------------------------------------------------------- full-size workloads, sampled rows
@pytest.mark.parametrize("name, B, theta", [("sphere20480", 32, THETA), ("cube24300", 32, THETA),
                                           ("sphere20480", 48, 0.5), ("cube24300", 48, 0.55)])
def test_full_size_fmm_sampled_rows(name, B, theta):
    """C2 at full size (the 20480-element sphere and the 24300-element cube),
    96 sampled rows of the oracle's direct product, both precisions, the
    system operator A and the right-hand-side operator -S, in both error
    measures; the last two cases are the trees the benchmark times (over
    all rows their largest row errors are 2.5e-7 and 2.4e-7)."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup(name, B=B, theta=theta)
    x = bem_inputs.random_vector(om.n_dof, 27)[0]
    xd = to_dev(x, False)
    yd = xd.clone()
    rng = np.random.default_rng(28)
    rows = np.sort(rng.choice(om.n_dof, 96, replace=False))
    for op in (bem.BEM_OP_A, bem.BEM_OP_RHS):
        ref = om.matvec_rows(x, op, rows=rows).real
        for prec in (bem.BEM_PREC_FP64, bem.BEM_PREC_MIXED):
            say(f"  full size {name} B={B} op={op} prec={prec}")
            bem.bem_matvec(ctx, tree, 0, 0.0, op, bem.BEM_FMM, prec, xd, yd)
            check_product(yd.cpu().numpy()[0][rows], ref, PRODUCT_TOL, "sampled rows")


# C3 tree: the wavenumber bound k (r1 + r2) <= kappa on the lists at ka = 10,
# leaf size and separation factor: the cheapest setting of a sweep (B 24-64,
# theta 0.45-0.7, kappa 1.5-3, errors over all 60842 rows) whose largest row
# error stays below 1e-6 with a margin (3.2e-7); kappa = 2.3 already reaches
# 1e-6 - 3e-6 at its worst rows
C3_KAPPA, C3_B, C3_THETA = 2.2, 64, 0.5


@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_helmholtz_geodesic_ka10_sampled_rows(prec):
    """C3: Helmholtz at ka = 10 on the geodesic sphere of 30420 elements.
    Order-8 Taylor expansions of e^{jkR}/R need the bound k (r1 + r2) <= kappa
    on the interaction lists (without it the product is off by ~1e-3, with
    kappa = 3 by ~5e-6); with kappa = 2.2 both precisions meet the 1e-6
    tolerance against the oracle's direct rows for A and -S, in both
    measures."""
    bem = _bem()
    ka = 10.0
    m, ctx, mesh, tree, om, ot = setup("geodesic30420", B=C3_B, theta=C3_THETA, kappa=C3_KAPPA, k_hint=ka)
    x = bem_inputs.random_vector(om.n_dof, 31, complex_=True)[0]
    xd = to_dev(x, True)
    yd = xd.clone()
    rows = np.sort(np.random.default_rng(32).choice(om.n_dof, 64, replace=False))
    for op in (bem.BEM_OP_A, bem.BEM_OP_RHS):
        ref = om.matvec_rows(x, op, green=oracle.HELMHOLTZ, k=ka, rows=rows)
        bem.bem_matvec(ctx, tree, 1, ka, op, bem.BEM_FMM, prec, xd, yd)
        check_product(yd.cpu().numpy()[0][rows], ref, PRODUCT_TOL, f"geodesic ka=10 op={op} prec={prec}")


def test_solve_helmholtz_rigid_sphere_ka10():
    """C3: rigid unit sphere at ka = 10 (geodesic, 30420 elements, ~20 per
    wavelength), plane wave along +z, mixed-precision GMRES to an FP64 residual of 1e-8;
    the total surface field against the series solution (measured 5.8e-6 rms,
    2.3e-5 max relative)."""
    bem = _bem()
    ka = 10.0
    m, ctx, mesh, tree, om, ot = setup("geodesic30420", B=C3_B, theta=C3_THETA, kappa=C3_KAPPA, k_hint=ka)
    inc, chi = analytic.plane_wave(om.dof_xyz, om.dof_normal, ka)
    chid = to_dev(chi, True)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 1, ka, chid, phid, tol=1e-8, precision=bem.BEM_PREC_MIXED)
    say(f"  ka=10 solve info={info}")
    assert info[0]["status"] == 0 and info[0]["residual"] <= 1e-8
    tot = phid.cpu().numpy()[0] + inc
    ref = analytic.rigid_sphere_total(ka, om.dof_xyz[:, 2] / np.linalg.norm(om.dof_xyz, axis=1))
    say(f"    error vs series: rms {rel(tot, ref):.2e} max {relmax(tot, ref):.2e}")
    assert rel(tot, ref) < 2e-5 and relmax(tot, ref) < 1e-4


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_point_source_cube24300(prec):
    """C2 cube: sharp edges and corners, 24300 elements (49686 DOFs), point
    source inside; FP64 and mixed-precision solves to 1e-8 against the
    analytic surface potential (measured 4.6e-7 relative)."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("cube24300")
    phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal)
    chid = to_dev(chi, False)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-8, precision=prec)
    say(f"  cube solve prec={prec} info={info}")
    assert info[0]["status"] == 0 and info[0]["residual"] <= 1e-8
    x = phid.cpu().numpy()[0]
    say(f"    error vs analytic {rel(x, phi.real):.2e}")
    assert rel(x, phi.real) < 2e-6


# ---------------------------------------------------------------- solver
@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_first_order_solve_matches_oracle_and_table(green, k):
    """First-order elements (the paper's Tables 1 and 5): the point-source
    problem on the 642-node sphere, FMM solve to 1e-8 against the oracle's
    dense solve (same discretisation), whose error the paper prints as
    3.46e-4 (Laplace) and 3.15e-4 (Helmholtz k = 2)."""
    bem = _bem()
    cplx = green == 1
    m, ctx, mesh, tree, om, ot = setup("sphere1280_p1", kappa=3.0 if cplx else 0.0, k_hint=k)
    phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal, k=k)
    S, K, c = om.assemble(green, k)
    x_or = np.linalg.solve(np.diag(c) - K, -S @ chi)
    chid = to_dev(chi, cplx)
    for prec in (0, 1):
        phid = chid.clone()
        info = bem.bem_solve(ctx, tree, green, k, chid, phid, tol=1e-8, precision=prec)
        x = phid.cpu().numpy()[0]
        err = np.sqrt(np.mean(np.abs(x - phi) ** 2))
        say(f"  p1 green={green} prec={prec} info={info} vs dense {rel(x, x_or if cplx else x_or.real):.2e} "
            f"vs analytic {err:.3e}")
        assert info[0]["status"] == 0 and info[0]["residual"] <= 1e-8
        assert rel(x, x_or if cplx else x_or.real) < 2e-6
        assert 0.8 < err / (3.46e-4 if green == 0 else 3.15e-4) < 1.2


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_point_source_sphere(prec):
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal)
    S, K, c = om.assemble()
    x_or = np.linalg.solve(np.diag(c) - K, -S @ chi).real
    chid = to_dev(chi, False)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-8, precision=prec)
    say(f"  solve prec={prec} info={info}")
    x = phid.cpu().numpy()[0]
    assert info[0]["status"] == 0 and info[0]["residual"] <= 1e-8
    # the FMM operator differs from the dense one by the truncation error
    assert rel(x, x_or) < 2e-6
    assert np.sqrt(np.mean((x - phi.real) ** 2)) < 1e-5


@pytest.mark.parametrize("green, prec", [(0, 0), (0, 1), (1, 1)])
def test_multi_rhs_solve_equals_single_solves(green, prec):
    """Right-hand sides solved together run in lock step (shared products,
    one host synchronisation per step) and must reproduce the single solves
    bit for bit, iteration counts included."""
    bem = _bem()
    k = 2.0 if green else 0.0
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    rng = np.random.default_rng(41)
    chi = rng.standard_normal((3, om.n_dof))
    if green:
        chi = chi + 1j * rng.standard_normal((3, om.n_dof))
    chi[1] *= 1e-3  # different scales converge at different steps
    chid = to_dev(chi, bool(green))
    phid = chid.clone()
    infos = bem.bem_solve(ctx, tree, green, k, chid, phid, tol=1e-8, precision=prec)
    together = phid.cpu().numpy()
    for r in range(3):
        c1 = chid[r:r + 1].clone()
        p1 = c1.clone()
        i1 = bem.bem_solve(ctx, tree, green, k, c1, p1, tol=1e-8, precision=prec)[0]
        assert i1 == infos[r], (r, i1, infos[r])
        assert np.array_equal(p1.cpu().numpy()[0], together[r]), r


def test_solve_helmholtz_rigid_sphere():
    bem = _bem()
    ka = 2.0
    m, ctx, mesh, tree, om, ot = setup("sphere1280", kappa=3.0, k_hint=ka)
    inc, chi = analytic.plane_wave(om.dof_xyz, om.dof_normal, ka)
    chid = to_dev(chi, True)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 1, ka, chid, phid, tol=1e-8, precision=bem.BEM_PREC_MIXED)
    say(f"  helmholtz solve info={info}")
    assert info[0]["status"] == 0
    tot = phid.cpu().numpy()[0] + inc
    ref = analytic.rigid_sphere_total(ka, om.dof_xyz[:, 2] / np.linalg.norm(om.dof_xyz, axis=1))
    assert relmax(tot, ref) < 2e-3


def test_solve_reports_noconv():
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    _, chi = analytic.point_source(om.dof_xyz, om.dof_normal)
    chid = to_dev(chi, False)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-14, restart=2, max_restarts=1)
    assert info[0]["status"] == bem.BEM_ENOCONV and info[0]["residual"] > 1e-14


@pytest.mark.parametrize("krylov", [0, 1])
def test_solve_step_budget_stops_with_noconv(krylov):
    """max_iters caps the Krylov steps of every right-hand side: a solve that
    needs more stops after exactly that many, reports BEM_ENOCONV with the
    FP64 residual of its last iterate, and that iterate is the one an
    uncapped solve has after the same steps (GMRES: the first cycle's)."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere1280")
    rng = np.random.default_rng(44)
    chi = rng.standard_normal((2, om.n_dof))
    chid = to_dev(chi, False)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-12, max_iters=3, krylov=krylov)
    say(f"  capped krylov={krylov}: {info}")
    for i in info:
        assert i["status"] == bem.BEM_ENOCONV and i["iterations"] == 3 and i["residual"] > 1e-12
    full = chid.clone()
    info_full = bem.bem_solve(ctx, tree, 0, 0.0, chid, full, tol=1e-12, krylov=krylov)
    assert all(i["status"] == 0 and i["iterations"] > 3 for i in info_full)
    # a capped run is a shorter run: its residual lies above the converged one
    assert all(c["residual"] > f["residual"] for c, f in zip(info, info_full))


def test_solve_time_budget_stops_every_rhs():
    """max_seconds: once the call's wall time runs out (here at the first
    check, after one step), every right-hand side stops where it is."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere1280")
    chi = np.random.default_rng(45).standard_normal((3, om.n_dof))
    chid = to_dev(chi, False)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-12, max_seconds=1e-9)
    say(f"  timed out: {info}")
    assert all(i["status"] == bem.BEM_ENOCONV and i["iterations"] == 1 for i in info)
    with pytest.raises(bem.BemError) as e:
        bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, max_iters=-1, raise_on_noconv=True)
    assert e.value.code == bem.BEM_EINVAL


def test_wavenumber_bound_rejects_k_above_k_hint():
    """A tree whose lists carry the wavenumber bound (kappa > 0) holds the
    truncation tolerance only for k <= k_hint: Helmholtz calls above it, or
    on such a tree built without k_hint, are rejected; Laplace is unaffected."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320", kappa=2.3, k_hint=3.0)
    x = to_dev(bem_inputs.random_vector(om.n_dof, 3, complex_=True)[0], True)
    y = x.clone()
    bem.bem_matvec(ctx, tree, 1, 3.0, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_FP64, x, y)  # k = k_hint
    bem.bem_matvec(ctx, tree, 1, 1.5, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_FP64, x, y)  # below it
    for call in (lambda: bem.bem_matvec(ctx, tree, 1, 3.5, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_FP64, x, y),
                 lambda: bem.bem_solve(ctx, tree, 1, 3.5, x, y, raise_on_noconv=True),
                 lambda: bem.bem_field(ctx, tree, 1, 3.5, x, x.clone(),
                                       to_dev(np.full((2, 3), 3.0), False).reshape(2, 3))):
        with pytest.raises(bem.BemError) as e:
            call()
        assert e.value.code == bem.BEM_EINVAL
    m2, ctx2, mesh2, tree2, *_ = setup("sphere320", kappa=2.3, k_hint=0.0)
    with pytest.raises(bem.BemError) as e:
        bem.bem_matvec(ctx2, tree2, 1, 1.0, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_FP64, x, y)
    assert e.value.code == bem.BEM_EINVAL
    xr = to_dev(np.ones(om.n_dof), False)
    bem.bem_matvec(ctx2, tree2, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_FP64, xr, xr.clone())


# ---------------------------------------------------------------- BiCGSTAB (the paper's solver)
@pytest.mark.parametrize("prec", [0, 1])
def test_bicgstab_point_source_sphere(prec):
    """BiCGSTAB to an FP64 residual of 1e-8 reaches the dense oracle's
    solution and the analytic one as GMRES does, and agrees with the GMRES
    solution to the tolerance (the system is of the second kind, so a
    residual of 1e-8 bounds the error to about that)."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    phi, chi = analytic.point_source(om.dof_xyz, om.dof_normal)
    S, K, c = om.assemble()
    x_or = np.linalg.solve(np.diag(c) - K, -S @ chi).real
    chid = to_dev(chi, False)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-8, precision=prec, krylov=bem.BEM_KRYLOV_BICGSTAB)
    say(f"  bicgstab prec={prec} info={info}")
    assert info[0]["status"] == 0 and info[0]["residual"] <= 1e-8
    x = phid.cpu().numpy()[0]
    assert rel(x, x_or) < 2e-6
    assert np.sqrt(np.mean((x - phi.real) ** 2)) < 1e-5
    pg = chid.clone()
    bem.bem_solve(ctx, tree, 0, 0.0, chid, pg, tol=1e-8, precision=prec)
    say(f"    vs GMRES {rel(x, pg.cpu().numpy()[0]):.2e}")
    assert rel(x, pg.cpu().numpy()[0]) < 1e-7


def test_bicgstab_helmholtz_rigid_sphere():
    """Complex BiCGSTAB (inner products conjugate the first argument) on the
    rigid sphere at ka = 2, mixed precision: the series solution as for
    GMRES, and the GMRES solution to the tolerance."""
    bem = _bem()
    ka = 2.0
    m, ctx, mesh, tree, om, ot = setup("sphere1280", kappa=3.0, k_hint=ka)
    inc, chi = analytic.plane_wave(om.dof_xyz, om.dof_normal, ka)
    chid = to_dev(chi, True)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 1, ka, chid, phid, tol=1e-8, precision=bem.BEM_PREC_MIXED,
                         krylov=bem.BEM_KRYLOV_BICGSTAB)
    say(f"  helmholtz bicgstab info={info}")
    assert info[0]["status"] == 0 and info[0]["residual"] <= 1e-8
    x = phid.cpu().numpy()[0]
    ref = analytic.rigid_sphere_total(ka, om.dof_xyz[:, 2] / np.linalg.norm(om.dof_xyz, axis=1))
    assert relmax(x + inc, ref) < 2e-3
    pg = chid.clone()
    bem.bem_solve(ctx, tree, 1, ka, chid, pg, tol=1e-8, precision=bem.BEM_PREC_MIXED)
    say(f"    vs GMRES {rel(x, pg.cpu().numpy()[0]):.2e}")
    assert rel(x, pg.cpu().numpy()[0]) < 1e-7


@pytest.mark.parametrize("green", [0, 1])
def test_bicgstab_multi_rhs_equals_single_solves(green):
    """Right-hand sides given together are solved one after the other with
    the same kernels, so each equals its solve alone bit for bit."""
    bem = _bem()
    k = 2.0 if green else 0.0
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    rng = np.random.default_rng(43)
    chi = rng.standard_normal((2, om.n_dof))
    if green:
        chi = chi + 1j * rng.standard_normal((2, om.n_dof))
    chi[1] *= 1e-3
    chid = to_dev(chi, bool(green))
    phid = chid.clone()
    kw = dict(tol=1e-8, precision=bem.BEM_PREC_MIXED, krylov=bem.BEM_KRYLOV_BICGSTAB)
    infos = bem.bem_solve(ctx, tree, green, k, chid, phid, **kw)
    together = phid.cpu().numpy()
    for r in range(2):
        c1 = chid[r:r + 1].clone()
        p1 = c1.clone()
        i1 = bem.bem_solve(ctx, tree, green, k, c1, p1, **kw)[0]
        assert i1 == infos[r], (r, i1, infos[r])
        assert np.array_equal(p1.cpu().numpy()[0], together[r]), r


def test_bicgstab_reports_noconv_and_rejects_bad_method():
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    _, chi = analytic.point_source(om.dof_xyz, om.dof_normal)
    chid = to_dev(chi, False)
    phid = chid.clone()
    info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-14, restart=2, max_restarts=1,
                         krylov=bem.BEM_KRYLOV_BICGSTAB)
    say(f"  bicgstab noconv info={info}")
    assert info[0]["status"] == bem.BEM_ENOCONV and info[0]["residual"] > 1e-14
    # one cycle of two steps; the right-hand side and the closing FP64 residual
    assert info[0]["iterations"] == 2 and info[0]["matvecs"] == 1 + 2 * 2 + 1
    with pytest.raises(bem.BemError) as e:
        bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, krylov=7, raise_on_noconv=True)
    assert e.value.code == bem.BEM_EINVAL


# ---------------------------------------------------------------- errors
def test_invalid_arguments():
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    x = to_dev(np.zeros(om.n_dof), False)
    xc = to_dev(np.zeros(om.n_dof, complex), True)
    with pytest.raises(bem.BemError) as e:
        bem.bem_matvec(ctx, tree, 1, 0.0, 0, 1, 0, xc, xc.clone())  # Helmholtz with k = 0
    assert e.value.code == bem.BEM_EINVAL
    with pytest.raises(bem.BemError) as e:
        bem.bem_matvec(ctx, tree, 0, 0.0, 0, 1, 0, x, x)  # aliasing x and y
    assert e.value.code == bem.BEM_EINVAL
    with pytest.raises(bem.BemError) as e:
        bem.bem_mesh_load(ctx, m.xyz, m.elem + 100000)  # node index out of range
    assert e.value.code == bem.BEM_EINVAL
    with pytest.raises(bem.BemError) as e:
        bem.bem_tree_build(ctx, mesh, order=12)
    assert e.value.code == bem.BEM_EUNSUPPORTED
    with pytest.raises(bem.BemError) as e:
        bem.bem_tree_build(ctx, mesh, attach_radii=3)
    assert e.value.code == bem.BEM_EINVAL
    with pytest.raises(bem.BemError) as e:
        bem.bem_tree_build(ctx, mesh, order_min=-1)
    assert e.value.code == bem.BEM_EINVAL
    with pytest.raises(ValueError):
        bem.bem_mesh_load(ctx, m.xyz, m.elem[:, :4])  # 4-node elements do not exist
    with pytest.raises(bem.BemError) as e:
        bem.bem_mesh_load(ctx, m.xyz, m.elem[:, :3] + 100000)  # first-order node out of range
    assert e.value.code == bem.BEM_EINVAL


def test_kernel_event_timing_modes():
    """bem_ctx_timing modes 2-4 bracket the heavy kernels with events without
    changing the product: 2 times both, 3 the near field only, 4 the M2L
    products only, one pair per product; other modes are rejected."""
    import torch

    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    x = to_dev(bem_inputs.random_vector(om.n_dof, 1)[0], False)
    ref = torch.empty_like(x)
    bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_MIXED, x, ref)
    try:
        for mode, timed in ((2, {"m2l", "p2p"}), (3, {"p2p"}), (4, {"m2l"})):
            ctx.timing(mode)
            y = torch.empty_like(x)
            for _ in range(3):
                bem.bem_matvec(ctx, tree, 0, 0.0, bem.BEM_OP_A, bem.BEM_FMM, bem.BEM_PREC_MIXED, x, y)
            got = ctx.timing(0)
            assert torch.equal(y, ref)
            assert {k for k, (ms, n) in got.items() if n} == timed, (mode, got)
            assert all(got[k][1] == 3 and got[k][0] > 0.0 for k in timed)
        with pytest.raises(bem.BemError) as e:
            ctx.timing(5)
        assert e.value.code == bem.BEM_EINVAL
    finally:
        ctx.timing(0)


# ---------------------------------------------------------------- field evaluation
def _field_points(rng, n_out, n_in):
    d = rng.standard_normal((n_out + n_in, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = np.concatenate([rng.uniform(1.4, 4.0, n_out), rng.uniform(0.0, 0.6, n_in)])
    far = np.array([[40.0, -30.0, 20.0]])  # beyond the root: its expansion alone
    return np.concatenate([d * r[:, None], far])


@pytest.mark.parametrize("name", ["perturbed", "perturbed_p1", "perturbed:literal"])
@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_field_matches_oracle_layer_potentials(name, green, k):
    """bem_field (Section 3.5, tree-accelerated) against the oracle's direct
    layer potentials D[phi] - S[chi] at points outside and inside the body and
    one far beyond the root, for seeded phi and chi: within the expansion
    tolerance (1e-6 of the largest value), two right-hand sides at once equal
    to one at a time, bit for bit."""
    import torch

    bem = _bem()
    mesh_name, _, tree_kind = name.partition(":")  # ":literal": the paper's tree (element pieces as sources)
    m, ctx, mesh, tree, om, ot = setup(mesh_name, attach="literal" if tree_kind else False)
    rng = np.random.default_rng(35 + green)
    pts = _field_points(rng, 48, 16)
    phi = rng.standard_normal((2, om.n_dof))
    chi = rng.standard_normal((2, om.n_dof))
    if green:
        phi = phi + 1j * rng.standard_normal((2, om.n_dof))
        chi = chi + 1j * rng.standard_normal((2, om.n_dof))
    pd = torch.tensor(pts, dtype=torch.float64, device="cuda:0")
    u2 = bem.bem_field(ctx, tree, green, k, to_dev(phi, green == 1), to_dev(chi, green == 1), pd).cpu().numpy()
    for r in range(2):
        u1 = bem.bem_field(ctx, tree, green, k, to_dev(phi[r:r + 1], green == 1), to_dev(chi[r:r + 1], green == 1),
                           pd).cpu().numpy()[0]
        assert np.array_equal(u1, u2[r])
        ref = om.layer_potential(pts, green, k, sigma_d=phi[r]) - om.layer_potential(pts, green, k, sigma_s=chi[r])
        if not green:
            ref = ref.real
        err = np.abs(u1 - ref).max() / np.abs(ref).max()
        say(f"  field green={green} rhs {r}: max error {err:.2e} (largest |u| {np.abs(ref).max():.3e})")
        assert err < 1e-6
    # the truncation error falls with theta as the order-8 expansion predicts
    errs = []
    for th in (0.6, 0.4, 0.25, 0.15):
        u = bem.bem_field(ctx, tree, green, k, to_dev(phi[:1], green == 1), to_dev(chi[:1], green == 1), pd,
                          theta=th).cpu().numpy()[0]
        ref = om.layer_potential(pts, green, k, sigma_d=phi[0]) - om.layer_potential(pts, green, k, sigma_s=chi[0])
        errs.append(np.abs(u - (ref if green else ref.real)).max() / np.abs(ref).max())
    say(f"  field green={green}: error at theta 0.6 / 0.4 / 0.25 / 0.15: {errs}")
    assert errs[0] > errs[1] > errs[2] > errs[3]


def test_field_of_solved_point_source_problem():
    """End to end: solve the exterior Neumann problem for a point source
    inside the sphere, then evaluate the field outside: it is the source's
    own field 1/(4 pi |x - xs|) (analytic), up to the discretisation."""
    import torch

    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere5120")
    xs = np.array([0.1, 0.2, 0.3])
    phi_a, chi = analytic.point_source(om.dof_xyz, om.dof_normal, xs=xs)
    chid = to_dev(chi.real, False)
    phid = torch.zeros_like(chid)
    info = bem.bem_solve(ctx, tree, 0, 0.0, chid, phid, tol=1e-10)
    assert info[0]["status"] == 0
    pts = _field_points(np.random.default_rng(5), 32, 0)
    u = bem.bem_field(ctx, tree, 0, 0.0, phid, chid, torch.tensor(pts, dtype=torch.float64, device="cuda:0"))
    u = u.cpu().numpy()[0]
    want = 1.0 / (4 * np.pi * np.linalg.norm(pts - xs, axis=1))
    err = np.abs(u - want).max() / np.abs(want).max()
    say(f"  solved field vs analytic: {err:.2e}")
    assert err < 2e-5


def test_field_rejects_bad_arguments():
    import torch

    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere320")
    x = to_dev(np.zeros(om.n_dof), False)
    pts = torch.zeros((4, 3), dtype=torch.float64, device="cuda:0") + 2.0
    with pytest.raises(bem.BemError) as e:
        bem.bem_field(ctx, tree, 1, 0.0, to_dev(np.zeros(om.n_dof, complex), True), to_dev(np.zeros(om.n_dof, complex), True), pts)
    assert e.value.code == bem.BEM_EINVAL
    with pytest.raises(ValueError):
        bem.bem_field(ctx, tree, 0, 0.0, x, x, pts.float())
    u = bem.bem_field(ctx, tree, 0, 0.0, x, x, pts)  # zero densities: zero field
    assert torch.count_nonzero(u) == 0


# ---------------------------------------------------------------- autotuned launch choices
@pytest.mark.parametrize("green,k,prec", [(0, 0.0, 1), (0, 0.0, 0), (1, 2.0, 1)])
def test_autotuned_products_equal_untuned_ones(green, k, prec):
    """The autotuner picks launch choices that change the speed of the fast
    product but not its arithmetic: on a shape class no product has tuned
    yet, the default choice (autotuning off) and the tuned one (the first
    product with autotuning on times every candidate) give the same bits."""
    import paper_0908_0673_amd as bem

    m = bem_inputs.icosphere(3)
    rng = np.random.default_rng(71 + 3 * green + prec)
    x = rng.standard_normal((2, 2562)) + (1j * rng.standard_normal((2, 2562)) if green else 0)
    ref = None
    for tune in (False, True):
        ctx = bem.Context(0)
        if not tune:
            ctx.autotune(forget=True)  # every shape class untuned again
        before = ctx.autotune(tune)
        mesh = bem.bem_mesh_load(ctx, m.xyz, m.elem)
        tree = bem.bem_tree_build(ctx, mesh, B=32, order=8, theta=0.5)
        xd = to_dev(x, green == 1)
        yd = xd.clone()
        bem.bem_matvec(ctx, tree, green, k, bem.BEM_OP_A, bem.BEM_FMM, prec, xd, yd)
        after = ctx.autotune(tune)
        y = yd.cpu().numpy()
        say(f"  autotune={tune}: classes tuned {before} -> {after}")
        if tune:
            assert before == 0 and after == 1
            assert np.array_equal(y, ref)
        else:
            assert before == 0 and after == 0
            ref = y
        tree.close()
        mesh.close()
        ctx.close()


@pytest.mark.parametrize("green,k", [(0, 0.0), (1, 2.0)])
def test_m2l_in_slabs_equals_one_slab(green, k):
    """The multipole-to-local step runs slab by slab over runs of target boxes
    whose interaction slots fit the tree's bound (the product's work space):
    with many small slabs the FP64 products equal the one-slab products bit
    for bit (each pair's translation and each box's sum are the same) and the
    oracle's fast product; the mixed ones, whose per-box sums the product
    kernel starts over runs of pairs that the slabs cut differently, agree to
    FP32 rounding."""
    bem = _bem()
    m, ctx, mesh, tree, om, ot = setup("sphere1280")
    small = bem.bem_tree_build(ctx, mesh, B=32, order=8, theta=THETA, m2l_slab_slots=700)
    cplx = green == 1
    x = bem_inputs.random_vector(om.n_dof, 81, nrhs=2, complex_=cplx)
    xd = to_dev(x, cplx)
    y1, y2 = xd.clone(), xd.clone()
    for op in (bem.BEM_OP_A, bem.BEM_OP_RHS):
        for prec in (bem.BEM_PREC_FP64, bem.BEM_PREC_MIXED):
            bem.bem_matvec(ctx, tree, green, k, op, bem.BEM_FMM, prec, xd, y1)
            bem.bem_matvec(ctx, small, green, k, op, bem.BEM_FMM, prec, xd, y2)
            if prec == bem.BEM_PREC_FP64:
                assert np.array_equal(y1.cpu().numpy(), y2.cpu().numpy()), (op, prec)
            else:
                check_product(y2.cpu().numpy(), y1.cpu().numpy(), 1e-6, f"slabs op={op} mixed vs one slab")
        ref = ot.fmm_matvec(x[0], op, green, k)
        bem.bem_matvec(ctx, small, green, k, op, bem.BEM_FMM, bem.BEM_PREC_FP64, xd, y2)
        check_product(y2.cpu().numpy()[0], ref if cplx else ref.real, 1e-11, f"slabs op={op} fp64 vs oracle fast")
    with pytest.raises(bem.BemError) as e:
        bem.bem_tree_build(ctx, mesh, m2l_slab_slots=-5)
    assert e.value.code == bem.BEM_EINVAL
    small.close()
