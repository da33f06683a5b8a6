"""Shared helpers of the GPU tests: one context per process, meshes from
bem_inputs on both sides, and relative-error measures."""

from __future__ import annotations

import functools

import numpy as np

import bem_inputs


def say(*a):
    print(*a, flush=True)


@functools.lru_cache(maxsize=None)
def context():
    import paper_0908_0673_amd as bem

    return bem.Context(0)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def relmax(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())


def to_dev(x, complex_: bool):
    import torch

    dt = torch.complex128 if complex_ else torch.float64
    x = np.asarray(x)
    if not complex_:
        x = x.real
    return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda:0").reshape(-1, x.shape[-1])


def perturbed_sphere(sub: int, seed: int, amp: float = 0.02):
    """Icosphere with every node moved radially by a seeded random factor."""
    m = bem_inputs.icosphere(sub)
    rng = np.random.default_rng(seed)
    f = 1.0 + amp * rng.standard_normal(m.n_nodes)
    return bem_inputs.Mesh(f"perturbed{sub}_{seed}", m.xyz * f[:, None], m.elem)


def mesh_by_name(name: str):
    if name.endswith("_p1"):  # first-order mesh on the corners of the named one
        return bem_inputs.linear(mesh_by_name(name[:-3]))
    if name.startswith("perturbed"):
        return perturbed_sphere(3, 5)
    if name.startswith("ellipsoid"):
        return bem_inputs.ellipsoid(8, (1.7, 0.8, 0.6))
    return bem_inputs.workload(name)
