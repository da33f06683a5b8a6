"""Synthetic surface meshes of 6-node quadratic or 3-node flat triangles.

Element node order (both the oracle and the GPU library assume it): the
three corners counter-clockwise seen from outside the body, then (6-node
elements) the mid-side nodes of edges 0-1, 1-2 and 2-0.  The paper's test surfaces are a
unit sphere refined from an initial surface and a cube of edge 2 centred on
the origin (Section 4); its cube meshes came from an external mesher that is
not available here, so structured cube meshes stand in for them.
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass
class Mesh:
    """Nodes ``xyz`` [n_nodes, 3] float64 and elements ``elem`` [n_el, 6] (or [n_el, 3]) int32."""

    name: str
    xyz: np.ndarray
    elem: np.ndarray

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_elem(self) -> int:
        return int(self.elem.shape[0])


def _icosahedron():
    """Unit icosahedron: vertices are the cyclic permutations of (0, +-1, +-phi)."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-phi, phi):
            v.append((0.0, s1, s2))
            v.append((s1, s2, 0.0))
            v.append((s2, 0.0, s1))
    v = np.array(v)
    # faces: triples whose pairwise distances are all the edge length 2
    faces = []
    for i, j, k in itertools.combinations(range(12), 3):
        if all(abs(np.linalg.norm(v[a] - v[b]) - 2.0) < 1e-9 for a, b in ((i, j), (j, k), (k, i))):
            faces.append([i, j, k])
    assert len(faces) == 20
    faces = np.array(faces)
    v = v / np.linalg.norm(v, axis=1)[:, None]
    return v, _orient_outward(v, faces)


def _orient_outward(v, faces):
    """Make every flat triangle counter-clockwise seen from outside (star-shaped about 0)."""
    out = faces.copy()
    a, b, c = v[faces[:, 0]], v[faces[:, 1]], v[faces[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    out[flip, 1], out[flip, 2] = faces[flip, 2], faces[flip, 1]
    return out


def _quadratic_from_linear(v, faces, project):
    """Add one mid-side node per edge; ``project`` maps chord midpoints onto the surface."""
    edge_id = {}
    mids = []
    elem = np.empty((faces.shape[0], 6), dtype=np.int32)
    nv = v.shape[0]
    for e, (a, b, c) in enumerate(faces):
        ids = []
        for p, q in ((a, b), (b, c), (c, a)):
            key = (min(p, q), max(p, q))
            if key not in edge_id:
                edge_id[key] = nv + len(mids)
                mids.append(0.5 * (v[p] + v[q]))
            ids.append(edge_id[key])
        elem[e] = (a, b, c, ids[0], ids[1], ids[2])
    m = np.array(mids).reshape(-1, 3)
    xyz = np.concatenate([v, project(m)], axis=0)
    return xyz, elem


def _to_sphere(p):
    return p / np.linalg.norm(p, axis=1)[:, None]


def icosphere(subdivisions: int) -> Mesh:
    """Unit sphere: icosahedron, ``subdivisions`` mid-point splits with projection.

    Two subdivisions give 320 elements and 642 nodes; five give 20480 and 40962.
    """
    v, f = _icosahedron()
    for _ in range(subdivisions):
        edge_id = {}
        verts = list(v)
        nf = []
        for a, b, c in f:
            m = []
            for p, q in ((a, b), (b, c), (c, a)):
                key = (min(p, q), max(p, q))
                if key not in edge_id:
                    edge_id[key] = len(verts)
                    w = v[p] + v[q]
                    verts.append(w / np.linalg.norm(w))
                m.append(edge_id[key])
            ab, bc, ca = m
            nf += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]
        v = np.array(verts)
        f = np.array(nf)
    xyz, elem = _quadratic_from_linear(v, f, _to_sphere)
    return Mesh(f"icosphere{subdivisions}", xyz, elem)


def geodesic_sphere(freq: int) -> Mesh:
    """Unit sphere: each icosahedron face split into ``freq``**2 triangles, projected.

    Frequency 39 gives 30420 elements and 60842 nodes.
    """
    v, f = _icosahedron()
    key_id = {}
    pts = []

    def node(face, i, j):
        a, b, c = face
        w = {a: freq - i - j, b: i, c: j}
        key = tuple(sorted((vid, wt) for vid, wt in w.items() if wt))
        if key not in key_id:
            key_id[key] = len(pts)
            p = sum(v[vid] * wt for vid, wt in w.items()) / freq
            pts.append(p)
        return key_id[key]

    tris = []
    for face in f:
        for i in range(freq):
            for j in range(freq - i):
                p00, p10, p01 = node(face, i, j), node(face, i + 1, j), node(face, i, j + 1)
                tris.append([p00, p10, p01])
                if i + j < freq - 1:
                    tris.append([p10, node(face, i + 1, j + 1), p01])
    pv = _to_sphere(np.array(pts))
    tris = _orient_outward(pv, np.array(tris))
    xyz, elem = _quadratic_from_linear(pv, tris, _to_sphere)
    return Mesh(f"geodesic{freq}", xyz, elem)


def cube(n: int, half: float = 1.0) -> Mesh:
    """Cube [-half, half]^3; each face an n x n grid of squares cut along one diagonal.

    Nodes sit on the surface of a (2n+1)^3 lattice; faces share their edge
    nodes, so the mesh is conforming and sharp edges carry shared geometric nodes.
    """
    m = 2 * n
    ids = {}
    pts = []

    def nid(p):
        p = tuple(int(x) for x in p)
        if p not in ids:
            ids[p] = len(pts)
            pts.append(p)
        return ids[p]

    ex, ey, ez = np.eye(3, dtype=int)
    # (fixed axis value, u axis, v axis) with u x v = outward normal
    faces = [
        (m * ex, ey, ez), (0 * ex, ez, ey),
        (m * ey, ez, ex), (0 * ey, ex, ez),
        (m * ez, ex, ey), (0 * ez, ey, ex),
    ]
    elem = []
    for base, u, w in faces:
        for a in range(n):
            for b in range(n):
                def P(i, j):
                    return nid(base + (2 * a + i) * u + (2 * b + j) * w)
                p00, p20, p22, p02 = P(0, 0), P(2, 0), P(2, 2), P(0, 2)
                elem.append([p00, p20, p22, P(1, 0), P(2, 1), P(1, 1)])
                elem.append([p00, p22, p02, P(1, 1), P(1, 2), P(0, 1)])
    xyz = (np.array(pts, dtype=np.float64) / n - 1.0) * half
    return Mesh(f"cube{n}", xyz, np.array(elem, dtype=np.int32))


def ellipsoid(freq: int, axes) -> Mesh:
    """Geodesic sphere of frequency ``freq`` with nodes scaled by semi-axes ``axes``."""
    s = geodesic_sphere(freq)
    return Mesh(f"ellipsoid{freq}", s.xyz * np.asarray(axes, dtype=np.float64)[None, :], s.elem)


def linear(m: Mesh) -> Mesh:
    """The flat 3-node triangulation on the corners of a 6-node mesh (the
    surface's first-order mesh of the same refinement); nodes renumbered in
    order of first use by the corners."""
    corners = m.elem[:, :3]
    used = np.unique(corners)
    remap = np.full(m.n_nodes, -1, np.int64)
    remap[used] = np.arange(used.size)
    return Mesh(m.name + "_p1", m.xyz[used].copy(), remap[corners].astype(np.int32))


# Named workloads with the sizes of the paper's test surfaces.
WORKLOADS = {
    "sphere320": lambda: icosphere(2),       # 320 elements, 642 nodes
    "sphere1280": lambda: icosphere(3),
    "sphere5120": lambda: icosphere(4),
    "sphere20480": lambda: icosphere(5),     # 20480 elements, 40962 nodes
    "cube24300": lambda: cube(45),           # 24300 elements, 49686 DOFs
    "geodesic30420": lambda: geodesic_sphere(39),  # 30420 elements, 60842 nodes
}


def workload(name: str) -> Mesh:
    """A named mesh; the suffix ``_p1`` gives the first-order mesh on the
    corners of the named one (e.g. ``sphere20480_p1``: 20480 flat triangles,
    10242 nodes)."""
    if name.endswith("_p1"):
        return linear(workload(name[:-3]))
    if name in WORKLOADS:
        return WORKLOADS[name]()
    if name.startswith("cube"):
        return cube(int(name[4:]))
    if name.startswith("geodesic"):
        return geodesic_sphere(int(name[8:]))
    if name.startswith("icosphere"):
        return icosphere(int(name[9:]))
    raise KeyError(name)
