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
TREE = dict(B=32, order=8, theta=0.5)


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


def _peak_alone(mesh, green=0, k=0.0, nrhs=1):
    """resident_peak of a one-lane server that has served one request of
    this mesh (its tree, caches and the solve's buffers)."""
    bem = _bem()
    srv = bem.Server(lanes=1, hbm_budget=8 << 30, precision=1, **TREE)
    try:
        mid, nd = srv.add_mesh(mesh.xyz, mesh.elem)
        chi = np.ones((nrhs, nd)) * (1 + 1j if green else 1.0)
        rc = srv.poll(srv.submit(mid, green, k, chi))[0]
        assert rc == 0
        return srv.stats()["resident_peak"]
    finally:
        srv.close()


def test_server_budget_is_a_hard_bound_and_eviction_keeps_results():
    """Admission by device-memory budget: with room for about one mesh per
    lane, requests cycling over eight meshes force evictions; the device bytes
    the server holds never pass the budget (sampled while requests are in
    flight, and the lanes' peaks summed), and every result still equals
    bem_solve's alone."""
    bem = _bem()
    meshes = [perturbed_sphere(3, seed) for seed in range(11, 19)]  # eight meshes of 1280 elements
    share = int(1.5 * max(_peak_alone(m) for m in meshes[:2]))
    budget = 2 * share  # each lane: one mesh's peak and a half, four meshes to serve
    rng = np.random.default_rng(7)
    srv = bem.Server(lanes=2, hbm_budget=budget, max_batch_rhs=4, precision=1, **TREE)
    samples = []
    try:
        ids, ndofs = zip(*[srv.add_mesh(m.xyz, m.elem) for m in meshes])
        order = [0, 1, 2, 3, 4, 5, 6, 7, 0, 2, 4, 6, 1, 3, 5, 7]
        reqs = [(j, 0, 0.0, rng.standard_normal((1, ndofs[j]))) for j in order]
        tickets = [srv.submit(ids[j], g, k, chi) for j, g, k, chi in reqs]
        res = {}
        while len(res) < len(tickets):
            samples.append(srv.stats()["resident_bytes"])
            for i, t in enumerate(tickets):
                if i not in res:
                    r = srv.poll(t, wait=False)
                    if r is not None:
                        res[i] = r
        st = srv.stats()
    finally:
        srv.close()
    say(f"  budget {budget} share {share} stats {st} largest sample {max(samples)}")
    assert st["evictions"] >= 1 and st["trees_built"] > len(meshes)
    assert max(samples) <= budget and st["resident_peak"] <= budget and st["rejected"] == 0
    for i, (j, g, k, chi) in enumerate(reqs):
        rc, phi, info, lat = res[i]
        assert rc == 0
        assert np.array_equal(phi, _reference(meshes[j], g, k, chi).real)


def test_server_rejects_a_mesh_larger_than_a_lane_share():
    """A request that cannot fit even in an empty lane fails with BEM_ENOMEM
    (nothing of it stays resident) and the lane goes on serving."""
    bem = _bem()
    small, big = bem_inputs.icosphere(2), bem_inputs.icosphere(4)
    budget = int(1.5 * _peak_alone(small))
    srv = bem.Server(lanes=1, hbm_budget=budget, precision=1, **TREE)
    try:
        i_b, nb = srv.add_mesh(big.xyz, big.elem)
        i_s, ns = srv.add_mesh(small.xyz, small.elem)
        rc_big = srv.poll(srv.submit(i_b, 0, 0.0, np.ones((1, nb))))[0]
        chi = np.random.default_rng(9).standard_normal((1, ns))
        rc_small, phi, info, lat = srv.poll(srv.submit(i_s, 0, 0.0, chi))
        st = srv.stats()
    finally:
        srv.close()
    say(f"  budget {budget} stats {st}")
    assert rc_big == bem.BEM_ENOMEM and st["rejected"] == 1
    assert rc_small == 0 and np.array_equal(phi, _reference(small, 0, 0.0, chi).real)
    assert st["resident_peak"] <= budget


def test_server_step_budget_reports_noconv():
    """The solve options' step budget bounds every served batch: a request
    that needs more steps comes back as BEM_ENOCONV with its partial info."""
    bem = _bem()
    m = bem_inputs.icosphere(3)
    srv = bem.Server(lanes=1, precision=1, tol=1e-12, max_iters=2, **TREE)
    try:
        mid, nd = srv.add_mesh(m.xyz, m.elem)
        rc, phi, info, lat = srv.poll(srv.submit(mid, 0, 0.0, np.random.default_rng(5).standard_normal((2, nd))))
    finally:
        srv.close()
    assert rc == bem.BEM_ENOCONV
    assert all(i["status"] == bem.BEM_ENOCONV and i["iterations"] == 2 for i in info)


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


def _bucket_top(k):
    """Top of the server's wavenumber bucket of k: 2^(ceil(4 log2 k) / 4)."""
    return 2.0 ** (np.ceil(4.0 * np.log2(k) - 1e-12) / 4.0)


@pytest.mark.parametrize("helmholtz_B", [0, 48])
def test_server_helmholtz_trees_per_wavenumber_bucket(helmholtz_B):
    """With the wavenumber bound on the lists (kappa > 0, no fixed k_hint),
    Helmholtz batches are solved on the mesh's resident tree for their
    wavenumber bucket (lists built for the bucket's top, leaf size
    helmholtz_B when set): results equal bem_solve's on such a tree, bit for
    bit, and wavenumbers of one bucket share one tree."""
    bem = _bem()
    mesh = bem_inputs.icosphere(3)
    rng = np.random.default_rng(17)
    srv = bem.Server(lanes=1, max_batch_rhs=4, precision=1, kappa=2.2, helmholtz_B=helmholtz_B, **TREE)
    ks = (4.0, 7.5, 7.1)  # 7.5 and 7.1 share the bucket whose top is 8
    try:
        mid, nd = srv.add_mesh(mesh.xyz, mesh.elem)
        chis = [rng.standard_normal((2, nd)) + 1j * rng.standard_normal((2, nd)) for _ in ks]
        res = [srv.poll(srv.submit(mid, 1, k, c)) for k, c in zip(ks, chis)]
        st = srv.stats()
    finally:
        srv.close()
    assert st["trees_built"] == 2
    ctx = context()
    m = bem.bem_mesh_load(ctx, mesh.xyz, mesh.elem)
    for k, chi, (rc, phi, info, lat) in zip(ks, chis, res):
        assert rc == 0 and all(i["status"] == 0 for i in info)
        topts = dict(TREE, B=helmholtz_B) if helmholtz_B else TREE
        t = bem.bem_tree_build(ctx, m, kappa=2.2, k_hint=_bucket_top(k), **topts)
        for r in range(2):
            d = to_dev(chi[r][None], True)
            p = d.clone()
            bem.bem_solve(ctx, t, 1, k, d, p, **SOLVE)
            assert np.array_equal(phi[r], p.cpu().numpy()[0]), (k, r)
