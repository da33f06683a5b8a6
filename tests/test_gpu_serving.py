"""Serving layer (bem_server_*): every right-hand side served concurrently,
merged or after eviction must equal bem_solve's result for it alone, bit for
bit (the server runs the same solve; batching, lanes and arrival order must
not leak into the numbers).  Inputs: the seeded meshes and vectors of
bem_inputs; the references are the library's own single solves, whose
accuracy the parity tests pin against the oracle."""

from __future__ import annotations

import numpy as np
import pytest

import bem_inputs
from gpu_common import context, perturbed_sphere, say, to_dev

pytestmark = pytest.mark.gpu

SOLVE = dict(tol=1e-8, restart=50, precision=1)  # mixed-precision steps, FP64 residuals
TREE = dict(B=32, order=8, theta=0.6)


def _bem():
    import paper_0908_0673_amd as bem

    return bem


def _meshes():
    return [bem_inputs.icosphere(2), perturbed_sphere(3, 11), bem_inputs.cube(4)]


def _reference(mesh, green, k, chi):
    """bem_solve on a fresh mesh and tree of the test's own context, one
    right-hand side at a time."""
    bem = _bem()
    ctx = context()
    m = bem.bem_mesh_load(ctx, mesh.xyz, mesh.elem)
    t = bem.bem_tree_build(ctx, m, **TREE)
    out = []
    for row in np.atleast_2d(chi):
        d = to_dev(row[None], green == 1)
        p = d.clone()
        bem.bem_solve(ctx, t, green, k, d, p, **SOLVE)
        out.append(p.cpu().numpy()[0])
    return np.array(out)


def _requests(rng, ids, ndofs):
    reqs = []
    for i in range(8):
        j = int(rng.integers(len(ids)))
        green = int(rng.integers(2))
        k = 2.0 if green else 0.0
        nrhs = int(rng.integers(1, 4))
        chi = rng.standard_normal((nrhs, ndofs[j]))
        if green:
            chi = chi + 1j * rng.standard_normal((nrhs, ndofs[j]))
        reqs.append((j, green, k, chi))
    return reqs


def test_server_results_equal_single_solves():
    bem = _bem()
    meshes = _meshes()
    rng = np.random.default_rng(20090908)
    srv = bem.Server(lanes=2, max_batch_rhs=8, precision=1, **TREE)
    try:
        ids, ndofs = zip(*[srv.add_mesh(m.xyz, m.elem) for m in meshes])
        reqs = _requests(rng, ids, ndofs)
        tickets = [srv.submit(ids[j], g, k, chi) for j, g, k, chi in reqs]
        results = [srv.poll(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    say(f"  server stats {st}")
    assert st["completed"] == len(reqs) and st["rhs_solved"] == sum(c.shape[0] for *_, c in reqs)
    for (j, g, k, chi), (rc, phi, info, lat) in zip(reqs, results):
        assert rc == 0 and all(i["status"] == 0 for i in info)
        assert lat > 0.0
        ref = _reference(meshes[j], g, k, chi)
        assert np.array_equal(phi, ref if g else ref.real), f"mesh {j} green {g}: served result differs"


def test_server_evicts_under_a_small_budget_and_still_agrees():
    bem = _bem()
    meshes = _meshes()
    rng = np.random.default_rng(7)
    # a budget below one mesh: every switch of mesh evicts the previous one
    srv = bem.Server(lanes=1, hbm_budget=1 << 20, max_batch_rhs=4, precision=1, **TREE)
    try:
        ids, ndofs = zip(*[srv.add_mesh(m.xyz, m.elem) for m in meshes])
        order = [0, 1, 2, 0, 1]
        reqs = [(j, 0, 0.0, rng.standard_normal((1, ndofs[j]))) for j in order]
        res = []
        for j, g, k, chi in reqs:  # one at a time, so the mesh changes every request
            res.append(srv.poll(srv.submit(ids[j], g, k, chi)))
        st = srv.stats()
    finally:
        srv.close()
    say(f"  server stats {st}")
    assert st["evictions"] >= 3 and st["trees_built"] == len(order)
    for (j, g, k, chi), (rc, phi, info, lat) in zip(reqs, res):
        assert rc == 0
        assert np.array_equal(phi, _reference(meshes[j], g, k, chi).real)


def test_server_merges_waiting_requests_of_one_problem():
    bem = _bem()
    big, small = bem_inputs.icosphere(4), bem_inputs.icosphere(2)
    rng = np.random.default_rng(3)
    srv = bem.Server(lanes=1, max_batch_rhs=16, precision=1, **TREE)
    try:
        ib, nb = srv.add_mesh(big.xyz, big.elem)
        i_s, ns = srv.add_mesh(small.xyz, small.elem)
        first = srv.submit(ib, 0, 0.0, rng.standard_normal((1, nb)))  # keeps the lane busy
        chis = [rng.standard_normal((1, ns)) for _ in range(5)]
        tickets = [srv.submit(i_s, 0, 0.0, c) for c in chis]
        res = [srv.poll(t) for t in tickets]
        srv.poll(first)
        st = srv.stats()
    finally:
        srv.close()
    say(f"  server stats {st}")
    assert st["completed"] == 6 and st["batches"] < 6
    ref = _reference(small, 0, 0.0, np.concatenate(chis))
    for i, (rc, phi, info, lat) in enumerate(res):
        assert rc == 0 and np.array_equal(phi[0], ref[i].real)


def test_server_rejects_bad_requests():
    bem = _bem()
    m = bem_inputs.icosphere(2)
    srv = bem.Server(lanes=1)
    try:
        mid, nd = srv.add_mesh(m.xyz, m.elem)
        x = np.zeros((1, nd))
        with pytest.raises(bem.BemError):
            srv.submit(mid, 1, 0.0, x)  # Helmholtz needs k > 0
        with pytest.raises(ValueError):
            srv.submit(mid + 5, 0, 0.0, x)  # unknown mesh
        with pytest.raises(bem.BemError):
            srv.poll(12345)
    finally:
        srv.close()


def test_server_first_order_bicgstab_level_order():
    """The server with first-order meshes, BiCGSTAB and the level-dependent
    order: every served result equals bem_solve's with the same options."""
    bem = _bem()
    meshes = [bem_inputs.linear(bem_inputs.icosphere(3)), bem_inputs.linear(bem_inputs.cube(4))]
    rng = np.random.default_rng(11)
    srv = bem.Server(lanes=2, max_batch_rhs=4, precision=1, krylov=bem.BEM_KRYLOV_BICGSTAB, order_min=3, **TREE)
    try:
        ids, ndofs = zip(*[srv.add_mesh(m.xyz, m.elem) for m in meshes])
        reqs = _requests(rng, ids, ndofs)
        results = [srv.poll(t) for t in [srv.submit(ids[j], g, k, chi) for j, g, k, chi in reqs]]
    finally:
        srv.close()
    ctx = context()
    for (j, g, k, chi), (rc, phi, info, lat) in zip(reqs, results):
        assert rc == 0 and all(i["status"] == 0 for i in info)
        m = bem.bem_mesh_load(ctx, meshes[j].xyz, meshes[j].elem)
        t = bem.bem_tree_build(ctx, m, order_min=3, **TREE)
        for r, row in enumerate(np.atleast_2d(chi)):
            d = to_dev(row[None], g == 1)
            p = d.clone()
            bem.bem_solve(ctx, t, g, k, d, p, krylov=bem.BEM_KRYLOV_BICGSTAB, **SOLVE)
            ref = p.cpu().numpy()[0]
            assert np.array_equal(phi[r], ref if g else ref.real), f"mesh {j} green {g} rhs {r}"


def test_server_helmholtz_trees_of_their_own_k():
    """With the wavenumber bound on the lists (kappa > 0, no fixed k_hint),
    every Helmholtz batch is solved on a tree built for its k: results equal
    bem_solve's on such a tree, bit for bit."""
    bem = _bem()
    mesh = bem_inputs.icosphere(3)
    rng = np.random.default_rng(17)
    srv = bem.Server(lanes=2, max_batch_rhs=4, precision=1, kappa=3.0, **TREE)
    ks = (4.0, 7.5)
    try:
        mid, nd = srv.add_mesh(mesh.xyz, mesh.elem)
        chis = [rng.standard_normal((2, nd)) + 1j * rng.standard_normal((2, nd)) for _ in ks]
        res = [srv.poll(srv.submit(mid, 1, k, c)) for k, c in zip(ks, chis)]
    finally:
        srv.close()
    ctx = context()
    m = bem.bem_mesh_load(ctx, mesh.xyz, mesh.elem)
    for k, chi, (rc, phi, info, lat) in zip(ks, chis, res):
        assert rc == 0 and all(i["status"] == 0 for i in info)
        t = bem.bem_tree_build(ctx, m, kappa=3.0, k_hint=k, **TREE)
        for r in range(2):
            d = to_dev(chi[r][None], True)
            p = d.clone()
            bem.bem_solve(ctx, t, 1, k, d, p, **SOLVE)
            assert np.array_equal(phi[r], p.cpu().numpy()[0]), (k, r)
