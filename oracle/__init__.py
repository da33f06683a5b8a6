"""Plain FP64 CPU oracle for the collocation BEM and its fast multipole product.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product path.  The numerics
live in ``bem_oracle.c`` (built with gcc, ``-O2 -ffp-contract=off``, no
fast-math); this module marshals numpy arrays into it.  ``gmres`` and
``analytic`` hold the oracle's Krylov solver and the closed-form fields.

Parity status per function (pins live in ``tests/test_oracle_*.py``):
  shape functions, quadrature rules, element geometry   pinned (exactness, areas, closed forms)
  first-order (3-node) elements                          pinned (closed forms, solid angles, the direct
                                                         errors printed in Tables 1 and 5)
  DOF indexing                                           pinned (cube DOF counts, corner/edge multiplicity)
  S, K, free term                                        pinned (solid angles, Green's identity, sphere potentials)
  tree, radii, lists                                     pinned (invariants, brute-force coverage)
  derivatives, shifts, local expansions, FMM product     pinned (harmonicity, closed forms, exact |r|^2 kernel, direct sum)
  level-dependent order of the FMM product               pinned (one interaction level equals the uniform
                                                         leaf order; error ordering in L_min)
  GMRES                                                  pinned (numpy.linalg.solve)
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bem_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

LAPLACE, HELMHOLTZ, R2 = 0, 1, 2
OP_S, OP_K, OP_A, OP_RHS, OP_S_REG, OP_K_REG = 0, 1, 2, 3, 4, 5

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain FP64, no contraction, OpenMP over rows)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        L.or_tree_build.restype = vp
        L.or_tree_build.argtypes = [vp, i64, vp, i64, ctypes.c_int, vp, vp, i64, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.or_tree_sizes.argtypes = [vp, vp]
        L.or_tree_export.argtypes = [vp] + [vp] * 9
        L.or_tree_free.argtypes = [vp]
        ci = ctypes.c_int
        L.or_fmm_matvec.argtypes = [vp, vp, vp, vp, vp, i64, i64, ci, ci, ctypes.c_double,
                                    ci, ci, ci, vp, vp]
        L.or_index_dofs.argtypes = [vp, i64, vp, i64, ci, ctypes.c_double, vp, vp, vp, vp]
        L.or_assemble.argtypes = [vp, vp, vp, vp, i64, i64, ci, ci, ctypes.c_double, vp, vp, vp]
        L.or_matvec_rows.argtypes = [vp, vp, vp, vp, i64, i64, ci, ci, ctypes.c_double,
                                     ci, vp, vp, i64, vp]
        L.or_free_term.argtypes = [vp, vp, vp, vp, i64, i64, ci, vp, i64, vp]
        L.or_layer_potential.argtypes = [vp, vp, vp, i64, ci, ci, ctypes.c_double, vp, vp,
                                         vp, i64, vp]
        L.or_pair.argtypes = [ci, vp, vp, ctypes.c_int32, vp, ci, ctypes.c_double, vp, vp]
        L.or_classify.argtypes = [ci, vp, vp, ctypes.c_int32, vp, vp]
        L.or_rule.argtypes = [ci, ci, ci, vp, vp, vp]
        L.or_shape.argtypes = [ci, ctypes.c_double, ctypes.c_double, vp, vp, vp]
        L.or_elem_point.argtypes = [ci, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp]
        L.or_derivs.argtypes = [ctypes.c_int, ctypes.c_double, vp, ctypes.c_int, vp]
        L.or_mono_moments.argtypes = [ctypes.c_int, vp, vp, vp, i64, vp]
        L.or_m2m.argtypes = [ctypes.c_int, vp, vp, vp]
        L.or_l2l.argtypes = [ctypes.c_int, vp, vp, vp]
        L.or_multi_index.argtypes = [ctypes.c_int, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def ncoef(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


# ---------------------------------------------------------------- mesh
class OracleMesh:
    """A mesh with the oracle's own DOF indexing (Section 2.3).  elem is
    [n_el][6] (second-order triangles) or [n_el][3] (first-order, flat)."""

    def __init__(self, xyz, elem, edge_angle_deg: float = 30.0):
        self.xyz = _c(xyz, np.float64)
        self.elem = _c(elem, np.int32)
        n_el, self.nn = self.elem.shape
        if self.nn not in (3, 6):
            raise ValueError("elements need 3 or 6 nodes")
        ed = np.empty((n_el, self.nn), np.int32)
        dn = np.empty(self.nn * n_el, np.int32)
        dnorm = np.empty((self.nn * n_el, 3), np.float64)
        nd = np.zeros(1, np.int64)
        rc = lib().or_index_dofs(_p(self.xyz), self.xyz.shape[0], _p(self.elem), n_el, self.nn,
                                 edge_angle_deg, _p(ed), _p(dn), _p(dnorm), _p(nd))
        if rc != 0:
            raise ValueError("invalid mesh")
        n = int(nd[0])
        self.elem_dofs = ed
        self.dof_node = dn[:n].copy()
        self.dof_normal = dnorm[:n].copy()
        self.n_dof = n
        self.n_el = n_el

    @property
    def dof_xyz(self):
        return self.xyz[self.dof_node]

    def _args(self):
        return (_p(self.xyz), _p(self.elem), _p(self.elem_dofs), _p(self.dof_node), self.n_el, self.n_dof, self.nn)

    def assemble(self, green=LAPLACE, k=0.0):
        """Dense S, K (complex, n x n) and the free term c (Eq. 3)."""
        n = self.n_dof
        S = np.zeros((n, n), np.complex128)
        K = np.zeros((n, n), np.complex128)
        c = np.zeros(n, np.float64)
        lib().or_assemble(*self._args(), green, float(k), _p(S), _p(K), _p(c))
        return S, K, c

    def matvec_rows(self, x, op, green=LAPLACE, k=0.0, rows=None):
        """Direct product (definition of Eq. 3) on the given rows."""
        x = _c(x, np.complex128)
        rows = np.arange(self.n_dof, dtype=np.int64) if rows is None else _c(rows, np.int64)
        y = np.zeros(rows.shape[0], np.complex128)
        lib().or_matvec_rows(*self._args(), green, float(k), op, _p(x), _p(rows), rows.shape[0], _p(y))
        return y

    def free_term(self, rows=None):
        rows = np.arange(self.n_dof, dtype=np.int64) if rows is None else _c(rows, np.int64)
        c = np.zeros(rows.shape[0], np.float64)
        lib().or_free_term(*self._args(), _p(rows), rows.shape[0], _p(c))
        return c

    def layer_potential(self, pts, green=LAPLACE, k=0.0, sigma_s=None, sigma_d=None):
        """Single/double layer potentials at points off the surface."""
        pts = _c(pts, np.float64).reshape(-1, 3)
        ss = None if sigma_s is None else _c(sigma_s, np.complex128)
        sd = None if sigma_d is None else _c(sigma_d, np.complex128)
        out = np.zeros(pts.shape[0], np.complex128)
        lib().or_layer_potential(_p(self.xyz), _p(self.elem), _p(self.elem_dofs), self.n_el, self.nn, green,
                                 float(k), None if ss is None else _p(ss), None if sd is None else _p(sd),
                                 _p(pts), pts.shape[0], _p(out))
        return out

    def pair(self, e, tgt_node, x, green=LAPLACE, k=0.0):
        S = np.zeros(12)
        K = np.zeros(12)
        x = _c(x, np.float64)
        cls = lib().or_pair(self.nn, _p(self.xyz), _p(self.elem[e]), int(tgt_node), _p(x), green, float(k), _p(S),
                            _p(K))
        return cls, S.view(np.complex128), K.view(np.complex128)


# ---------------------------------------------------------------- tree
class OracleTree:
    """Recursive octree with radii and lists (Sections 3.1, 3.4, 3.6)."""

    def __init__(self, mesh: OracleMesh, B=32, max_depth=21, theta=1.0, kappa=float("inf"), k=0.0,
                 attach=False, literal=False):
        """attach: leaf radii also cover the elements attached to the nodes of
        the leaf's targets (the paper's r_C); sources stay single-owner.
        literal: the paper's tree read literally: boxes over the DOF points,
        B counting DOFs, each DOF's basis function a source (attached radii);
        elem_begin / elem_end are then the DOF ranges."""
        self.mesh = mesh
        tgt = _c(mesh.dof_xyz, np.float64)
        tnode = _c(mesh.dof_node, np.int32)
        self._h = lib().or_tree_build(_p(mesh.xyz), mesh.xyz.shape[0], _p(mesh.elem), mesh.n_el, mesh.nn,
                                      _p(tgt), _p(tnode), tgt.shape[0], int(B), int(max_depth), float(theta),
                                      float(kappa), float(k), 2 if literal else int(bool(attach)))
        sz = np.zeros(4, np.int64)
        lib().or_tree_sizes(self._h, _p(sz))
        nb, nn, ni, ml = (int(v) for v in sz)
        self.n_box, self.max_level = nb, ml
        ib = np.zeros((nb, 10), np.int64)
        db = np.zeros((nb, 4), np.float64)
        # sources of the tree: the elements, or the DOFs of the literal tree
        self.eperm = np.zeros(mesh.n_dof if literal else mesh.n_el, np.int64)
        self.tperm = np.zeros(mesh.n_dof, np.int64)
        self.near_ptr = np.zeros(nb + 1, np.int64)
        self.near_idx = np.zeros(max(nn, 1), np.int64)
        self.inter_ptr = np.zeros(nb + 1, np.int64)
        self.inter_idx = np.zeros(max(ni, 1), np.int64)
        root = np.zeros(4)
        lib().or_tree_export(self._h, _p(ib), _p(db), _p(self.eperm), _p(self.tperm), _p(self.near_ptr),
                             _p(self.near_idx), _p(self.inter_ptr), _p(self.inter_idx), _p(root))
        self.near_idx = self.near_idx[:nn]
        self.inter_idx = self.inter_idx[:ni]
        (self.level, self.leaf, self.parent, self.child_begin, self.nchild,
         self.eb, self.ee, self.tb, self.te, self.prefix) = ib.T.copy()
        self.centre = db[:, :3].copy()
        self.radius = db[:, 3].copy()
        self.corner = root[:3].copy()
        self.side = float(root[3])
        self.B, self.theta, self.kappa, self.k = B, theta, kappa, k

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib is not None:
                _lib.or_tree_free(self._h)
        except Exception:  # noqa: BLE001 - interpreter teardown
            pass
        self._h = None

    def fmm_matvec(self, x, op, green=LAPLACE, k=0.0, order=8, order_min=0):
        """The fast matrix product of Section 3.6 (plain FP64 loops).  With
        order_min > 0 the order depends on the level as in Section 3.6:
        L_l = min(order, order_min + max_level - l)."""
        m = self.mesh
        x = _c(x, np.complex128)
        y = np.zeros(m.n_dof, np.complex128)
        lib().or_fmm_matvec(self._h, *m._args(), green, float(k), int(order), int(order_min), op, _p(x), _p(y))
        return y


# ---------------------------------------------------------------- pieces
def rule(kind: int, param: int = 0, ng: int = 8):
    s = np.zeros(1792)
    t = np.zeros(1792)
    w = np.zeros(1792)
    n = lib().or_rule(kind, param, ng, _p(s), _p(t), _p(w))
    return s[:n], t[:n], w[:n]


def shape(s, t, nn=6):
    """Shape functions of the 6-node (nn = 6) or 3-node triangle and their
    s, t derivatives (six entries, unused ones zero)."""
    L, Ls, Lt = np.zeros(6), np.zeros(6), np.zeros(6)
    lib().or_shape(int(nn), float(s), float(t), _p(L), _p(Ls), _p(Lt))
    return L, Ls, Lt


def elem_point(X, s, t):
    """Position, unit normal and Jacobian of the element with node
    coordinates X ([6][3] or [3][3]) at (s, t)."""
    X = _c(X, np.float64).reshape(-1, 3)
    y, n, J = np.zeros(3), np.zeros(3), np.zeros(1)
    lib().or_elem_point(X.shape[0], _p(X), float(s), float(t), _p(y), _p(n), _p(J))
    return y, n, float(J[0])


def derivs(r, H, green=LAPLACE, k=0.0):
    r = _c(r, np.float64)
    D = np.zeros(ncoef(H), np.complex128)
    lib().or_derivs(green, float(k), _p(r), int(H), _p(D))
    return D


def multi_index(p):
    e = np.zeros((ncoef(p), 3), np.int32)
    lib().or_multi_index(int(p), _p(e))
    return e


def mono_moments(p, c, pts, w):
    c, pts, w = _c(c, np.float64), _c(pts, np.float64), _c(w, np.float64)
    M = np.zeros(ncoef(p))
    lib().or_mono_moments(int(p), _p(c), _p(pts), _p(w), w.shape[0], _p(M))
    return M


def m2m(p, d, Mc):
    d, Mc = _c(d, np.float64), _c(Mc, np.float64)
    Mp = np.zeros(ncoef(p))
    lib().or_m2m(int(p), _p(d), _p(Mc), _p(Mp))
    return Mp


def l2l(p, d, Fp):
    d, Fp = _c(d, np.float64), _c(Fp, np.float64)
    Fc = np.zeros(ncoef(p))
    lib().or_l2l(int(p), _p(d), _p(Fp), _p(Fc))
    return Fc
