"""Seeded streams of independent solve requests (shapes, sizes, equations,
wavenumbers, right-hand-side counts, plane-wave directions, arrival times)
for the serving measurements.  Geometry and random draws only.

Per request (numpy default_rng(seed), spawned per request):
  n_tri     log-uniform in [lo, hi]
  shape     uniform over {sphere, cube, ellipsoid}
            sphere / ellipsoid: geodesic frequency m = max(4, round(sqrt(n_tri / 20)))
            cube: n = max(2, round(sqrt(n_tri / 12))) squares per face edge
            ellipsoid semi-axes uniform in [0.5, 2]^3, applied to the sphere nodes
  equation  Laplace or Helmholtz with probability 1/2; ka uniform in [ka_lo, ka_hi],
            k = ka / a with a the body's circumradius about the origin (1 for
            the unit sphere, sqrt(3) for the cube [-1, 1]^3, the largest
            semi-axis for an ellipsoid)
  nrhs      uniform in 1..nrhs_max, each with direction g / |g|, g ~ N(0, I3)
Arrivals are a Poisson process of unit rate (scaled by the caller).
"""

from __future__ import annotations

import numpy as np

from .meshes import Mesh, cube, ellipsoid, geodesic_sphere


def _mesh(shape: str, n_tri: int, axes) -> Mesh:
    if shape == "cube":
        return cube(max(2, int(round(np.sqrt(n_tri / 12.0)))))
    m = max(4, int(round(np.sqrt(n_tri / 20.0))))
    if shape == "sphere":
        return geodesic_sphere(m)
    return ellipsoid(m, axes)


def request_stream(count: int, seed: int, n_tri=(2000, 80000), ka=(1.0, 25.0), nrhs_max: int = 32,
                   uniform_size: bool = False, nrhs_fixed: int = 0):
    """List of dicts: key (a mesh identity), shape, n_tri, green (0 Laplace,
    1 Helmholtz), k, ka, a, nrhs, dirs [nrhs, 3], t (arrival time at unit rate);
    meshes are generated lazily by ``mesh_of(request)``.  uniform_size draws
    n_tri uniformly instead of log-uniformly; nrhs_fixed > 0 gives every
    request that many right-hand sides."""
    root = np.random.default_rng(seed)
    children = root.spawn(count)
    t = 0.0
    out = []
    for rng in children:
        if uniform_size:
            nt = int(round(rng.uniform(n_tri[0], n_tri[1])))
        else:
            nt = int(round(np.exp(rng.uniform(np.log(n_tri[0]), np.log(n_tri[1])))))
        shape = ("sphere", "cube", "ellipsoid")[int(rng.integers(3))]
        axes = tuple(float(a) for a in rng.uniform(0.5, 2.0, 3)) if shape == "ellipsoid" else None
        green = int(rng.integers(2))
        ka_draw = float(rng.uniform(*ka)) if green else 0.0
        a = 1.0 if shape == "sphere" else (3.0 ** 0.5 if shape == "cube" else max(axes))
        k = ka_draw / a
        nrhs = nrhs_fixed if nrhs_fixed > 0 else int(rng.integers(1, nrhs_max + 1))
        g = rng.standard_normal((nrhs, 3))
        dirs = g / np.linalg.norm(g, axis=1, keepdims=True)
        t += float(rng.exponential(1.0))
        if shape == "cube":
            key = ("cube", max(2, int(round(np.sqrt(nt / 12.0)))))
        else:
            key = (shape, max(4, int(round(np.sqrt(nt / 20.0)))), axes)
        out.append({"key": key, "shape": shape, "n_tri": nt, "axes": axes, "green": green, "k": k, "ka": ka_draw,
                    "a": a, "nrhs": nrhs, "dirs": dirs, "t": t})
    return out


def mesh_of(req) -> Mesh:
    return _mesh(req["shape"], req["n_tri"], req["axes"])
