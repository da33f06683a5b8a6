"""Closed-form fields used to pin the oracle (TEST INFRASTRUCTURE ONLY).

* Point source inside the surface (Section 4): phi = G(|x - x_s|), chi = dphi/dn.
* Rigid sphere in a plane wave e^{jk d.x} (time factor e^{-j w t}, outgoing G):
  surface total field from the modal series, with the Wronskian
  j_n y_n' - j_n' y_n = 1/z^2 folded in.
* Uniform stream past the unit sphere (Laplace): phi_s = (d.x)/2 on the surface.
"""

from __future__ import annotations

import numpy as np
from scipy import special


def point_source(x, normals, xs=(0.1, 0.2, 0.3), k=0.0):
    """phi and chi = grad(phi).n for G = e^{jkR}/(4 pi R) (k = 0: Laplace)."""
    r = np.asarray(x) - np.asarray(xs)[None, :]
    R = np.linalg.norm(r, axis=1)
    e = np.exp(1j * k * R)
    phi = e / (4 * np.pi * R)
    dphi_dR = (1j * k * R - 1.0) * e / (4 * np.pi * R ** 2)
    chi = dphi_dR * np.einsum("ij,ij->i", r, normals) / R
    return phi, chi


def plane_wave(x, normals, k, d=(0.0, 0.0, 1.0)):
    """Incident e^{jk d.x} and the sound-hard scattered-field data chi_s = -d(phi_inc)/dn."""
    d = np.asarray(d, dtype=float)
    phase = np.exp(1j * k * (np.asarray(x) @ d))
    chi_s = -1j * k * (np.asarray(normals) @ d) * phase
    return phase, chi_s


def rigid_sphere_total(ka, cos_theta, a=1.0):
    """Total surface field on a rigid sphere of radius a, unit incident plane wave."""
    cos_theta = np.asarray(cos_theta, dtype=float)
    nmax = int(ka + 4.0 * ka ** (1.0 / 3.0) + 12)
    out = np.zeros(cos_theta.shape, np.complex128)
    for n in range(nmax + 1):
        hp = special.spherical_jn(n, ka, derivative=True) + 1j * special.spherical_yn(n, ka, derivative=True)
        out += (1j ** (n + 1)) * (2 * n + 1) * special.eval_legendre(n, cos_theta) / (ka ** 2 * hp)
    return out


def rigid_sphere_total_textbook(ka, cos_theta):
    """Same field written as incident + scattered modal sums (independent form)."""
    cos_theta = np.asarray(cos_theta, dtype=float)
    nmax = int(ka + 4.0 * ka ** (1.0 / 3.0) + 12)
    out = np.zeros(cos_theta.shape, np.complex128)
    for n in range(nmax + 1):
        jn = special.spherical_jn(n, ka)
        jnp = special.spherical_jn(n, ka, derivative=True)
        hn = jn + 1j * special.spherical_yn(n, ka)
        hnp = jnp + 1j * special.spherical_yn(n, ka, derivative=True)
        out += (1j ** n) * (2 * n + 1) * (jn - jnp / hnp * hn) * special.eval_legendre(n, cos_theta)
    return out


def uniform_stream(x, normals, d=(0.0, 0.0, 1.0)):
    """phi_inc = d.x and chi_s = -d.n; on the unit sphere phi_s = (d.x)/2."""
    d = np.asarray(d, dtype=float)
    return np.asarray(x) @ d, -(np.asarray(normals) @ d)
