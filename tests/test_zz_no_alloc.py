"""The no-allocation product (bem_matvec_noalloc) through the C interface:
its results equal bem_matvec's bit for bit on the same tree and inputs, on
two calls in a row (the second with a smaller mesh and fewer right-hand
sides, so the shared scratch holds the first call's contents), for both
Green's functions, precisions and methods; unprepared trees and oversized
products are refused before any device work."""

from __future__ import annotations

import numpy as np
import pytest

import bem_inputs
from gpu_common import context, say, to_dev

pytestmark = pytest.mark.gpu


def _bem():
    import paper_0908_0673_amd as bem

    return bem


def _tree(ctx, mesh):
    bem = _bem()
    m = bem.bem_mesh_load(ctx, mesh.xyz, mesh.elem)
    return m, bem.bem_tree_build(ctx, m, B=32, order=8, theta=0.5, kappa=2.3, k_hint=2.0)


CASES = [(g, k, op, meth, prec) for g, k in ((0, 0.0), (1, 2.0)) for op in (2, 3)
         for meth, prec in ((1, 0), (1, 1), (0, 0))]


def test_noalloc_equals_matvec_on_two_calls_in_a_row():
    bem = _bem()
    ctx = context()
    big, small = _tree(ctx, bem_inputs.icosphere(3)), _tree(ctx, bem_inputs.icosphere(2))
    for (mesh, tree), nrhs, seed in ((big, 3, 61), (small, 1, 62)):
        for g, k, op, meth, prec in CASES:
            x = to_dev(bem_inputs.random_vector(mesh.n_dof, seed, nrhs=nrhs, complex_=g == 1), g == 1)
            ref = x.clone()
            bem.bem_matvec(ctx, tree, g, k, op, meth, prec, x, ref)  # builds the tables, then the reference
            bem.bem_matvec(ctx, tree, g, k, op, meth, prec, x, ref)
            y = x.clone()
            bem.bem_matvec_noalloc(ctx, tree, g, k, op, meth, prec, x, y)
            a, b = y.cpu().numpy(), ref.cpu().numpy()
            say(f"  n_dof={mesh.n_dof} nrhs={nrhs} green={g} op={op} method={meth} prec={prec}: "
                f"max |diff| {np.abs(a - b).max():.1e}")
            assert np.array_equal(a, b)


def test_noalloc_refuses_unprepared_trees_and_oversized_products():
    bem = _bem()
    ctx = context()
    mesh, tree = _tree(ctx, bem_inputs.icosphere(2))
    x = to_dev(bem_inputs.random_vector(mesh.n_dof, 63)[0], False)
    y = x.clone()
    with pytest.raises(bem.BemError) as e:  # nothing built on this tree yet
        bem.bem_matvec_noalloc(ctx, tree, 0, 0.0, 2, 1, 1, x, y)
    assert e.value.code == bem.BEM_ESTATE
    bem.bem_matvec(ctx, tree, 0, 0.0, 2, 1, 1, x, y)
    bem.bem_matvec_noalloc(ctx, tree, 0, 0.0, 2, 1, 1, x, y)
    # many right-hand sides at once: more work space than the scratch holds
    X = to_dev(np.ones((8000, mesh.n_dof)), False)
    Y = X.clone()
    with pytest.raises(bem.BemError) as e:
        bem.bem_matvec_noalloc(ctx, tree, 0, 0.0, 2, 1, 1, X, Y)
    assert e.value.code == bem.BEM_EINVAL and "scratch" in str(e.value)
    # the refusal left the scratch usable
    y2 = x.clone()
    bem.bem_matvec_noalloc(ctx, tree, 0, 0.0, 2, 1, 1, x, y2)
    assert np.array_equal(y2.cpu().numpy(), y.cpu().numpy())
