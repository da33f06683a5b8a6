"""Restarted GMRES for the oracle (plain numpy, FP64 / complex128).

TEST INFRASTRUCTURE ONLY.  The paper solves with stabilised BiCGSTAB from the
Barrett et al. templates (Section 2.1, Section 4); the solver required here is
GMRES with restart m: x0 = 0, modified Gram-Schmidt Arnoldi, complex Givens
rotations on the Hessenberg matrix, stop when the rotated residual estimate
falls to tol * |b|, then confirm with an explicit residual.  A breakdown
h_{j+1,j} <= 1e-14 |A v_j| ends the cycle early (the Krylov space is invariant).
"""

from __future__ import annotations

import numpy as np


def gmres(apply, b, tol=1e-8, restart=50, max_restarts=100, x0=None):
    """Solve apply(x) = b.  Returns (x, info) with info a dict of
    iterations, restarts, relative residual and converged flag."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros(n, np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, {"iterations": 0, "restarts": 0, "residual": 0.0, "converged": True}
    its = 0
    for cycle in range(max_restarts):
        r = b - apply(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            return x, {"iterations": its, "restarts": cycle, "residual": beta / bnorm, "converged": True}
        m = restart
        V = np.zeros((m + 1, n), np.complex128)
        H = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m, np.complex128)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            w = apply(V[j])
            wnorm = np.linalg.norm(w)
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = abs(H[j + 1, j]) <= 1e-14 * wnorm
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            # apply previous rotations to the new column
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                H[i, j] = t
            # new rotation zeroing H[j+1, j]
            a, bb = H[j, j], H[j + 1, j]
            cs[j], sn[j] = _rot(a, bb)
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            if abs(g[j + 1]) / bnorm <= tol or breakdown:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + V[:j_done].T @ y
    r = b - apply(x)
    res = np.linalg.norm(r) / bnorm
    return x, {"iterations": its, "restarts": max_restarts, "residual": res, "converged": res <= tol}


def _rot(a, b):
    """Unitary Givens rotation G = [[c, s], [-conj(s), conj(c)]] with G [a, b]^T = [r, 0]^T."""
    if b == 0:
        return 1.0 + 0j, 0.0 + 0j
    if a == 0:
        return 0.0 + 0j, np.conj(b) / abs(b)
    den = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = np.conj(a) / den
    s = np.conj(b) / den
    # c*a + s*b = (|a|^2 + |b|^2)/den = den;  -conj(s) a + conj(c) b = (-b a + a b)/den = 0
    return c, s
