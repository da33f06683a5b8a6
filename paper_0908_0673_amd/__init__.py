"""MI355X fast-multipole boundary element library (arXiv 0908.0673, Carley, BEM3D).

Thin Python binding of ``libbem.so`` (C interface in ``include/bem.h``):
argument marshalling only.  Every step of the computation runs in the
library's HIP kernels; PyTorch provides device memory (through its caching
allocator) and the stream.  Importing works without a GPU; creating a
:class:`Context` needs the built library and a device, and fails loudly
otherwise.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbem.so")

BEM_OK, BEM_EINVAL, BEM_ENOMEM, BEM_EDEVICE, BEM_ENOCONV, BEM_ESTATE, BEM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
BEM_EAGAIN = -7
BEM_LAPLACE, BEM_HELMHOLTZ = 0, 1
BEM_OP_S, BEM_OP_K, BEM_OP_A, BEM_OP_RHS = 0, 1, 2, 3
BEM_DIRECT, BEM_FMM = 0, 1
BEM_PREC_FP64, BEM_PREC_MIXED = 0, 1
BEM_KRYLOV_GMRES, BEM_KRYLOV_BICGSTAB = 0, 1

EXPORTED = [
    "bem_ctx_create", "bem_ctx_destroy", "bem_ctx_timing", "bem_ctx_autotune", "bem_ctx_device_bytes", "bem_last_error",
    "bem_mesh_load", "bem_mesh_dofs", "bem_mesh_free",
    "bem_tree_build", "bem_tree_export", "bem_tree_free", "bem_tree_stats_get", "bem_matvec", "bem_matvec_noalloc",
    "bem_solve", "bem_field",
    "bem_server_create", "bem_server_add_mesh", "bem_server_mesh_dofs", "bem_server_submit", "bem_server_poll",
    "bem_server_stats_get",
    "bem_server_destroy",
]


class BemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC), ("free", _FREE), ("user", ctypes.c_void_p)]


class _MeshOpts(ctypes.Structure):
    _fields_ = [("edge_angle_deg", ctypes.c_double), ("nodes_per_elem", ctypes.c_int)]


class _TreeOpts(ctypes.Structure):
    _fields_ = [("max_elems_per_leaf", ctypes.c_int), ("order", ctypes.c_int), ("theta", ctypes.c_double),
                ("kappa", ctypes.c_double), ("max_depth", ctypes.c_int), ("k_hint", ctypes.c_double),
                ("order_min", ctypes.c_int), ("attach_radii", ctypes.c_int), ("m2l_slab_slots", ctypes.c_int)]


class _TreeView(ctypes.Structure):
    _fields_ = [("n_box", ctypes.c_int64), ("n_elem", ctypes.c_int64), ("n_target", ctypes.c_int64),
                ("n_near", ctypes.c_int64), ("n_inter", ctypes.c_int64), ("n_leaf", ctypes.c_int64),
                ("max_level", ctypes.c_int32), ("root", ctypes.c_double * 4)] + [
        (n, ctypes.c_void_p) for n in ("level", "leaf", "parent", "child_begin", "nchild", "elem_begin", "elem_end",
                                       "tgt_begin", "tgt_end", "prefix", "centre", "radius", "elem_perm", "tgt_perm",
                                       "near_ptr", "inter_ptr", "near_idx", "inter_idx")]


class _TreeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_m2l", "n_m2l_same_level", "n_p2p", "n_corr_pairs", "n_leaf",
                                              "n_box", "n_quad")]


class _SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double), ("max_iters", ctypes.c_int),
                ("method", ctypes.c_int), ("krylov", ctypes.c_int), ("max_seconds", ctypes.c_double)]


class _ServerOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("lanes", ctypes.c_int), ("hbm_budget", ctypes.c_int64),
                ("max_batch_rhs", ctypes.c_int), ("tree", _TreeOpts), ("solve", _SolveOpts),
                ("helmholtz_B", ctypes.c_int)]


class _ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "batches", "rhs_solved", "evictions",
                                              "trees_built", "resident_bytes", "resident_peak", "rejected")]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("residual", ctypes.c_double), ("status", ctypes.c_int)]


_lib = None
_live = []  # handles still open, closed in reverse order before torch shuts down


def _close_all():
    while _live:
        ref = _live.pop()
        obj = ref()
        if obj is not None:
            try:
                obj.close()
            except Exception:  # noqa: BLE001
                pass


atexit.register(_close_all)


def _track(obj):
    _live.append(weakref.ref(obj))


def load_library(path: str = LIB_PATH):
    """Loads libbem.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_0908_0673_amd/build.py (hipcc, gfx950)")
    # torch first: the library then binds to the HIP runtime torch has loaded
    # (one runtime per process), whichever of the two a caller touches first
    import torch  # noqa: F401

    L = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.bem_ctx_create.argtypes = [i32, vp, ctypes.POINTER(_Allocator), ctypes.POINTER(vp)]
    L.bem_ctx_destroy.argtypes = [vp]
    L.bem_ctx_destroy.restype = None
    L.bem_ctx_timing.argtypes = [vp, i32, vp, vp]
    L.bem_ctx_device_bytes.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.bem_ctx_autotune.argtypes = [vp, i32, ctypes.POINTER(i64)]
    L.bem_last_error.argtypes = [vp]
    L.bem_last_error.restype = ctypes.c_char_p
    L.bem_mesh_load.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(_MeshOpts), ctypes.POINTER(vp)]
    L.bem_mesh_dofs.argtypes = [vp, ctypes.POINTER(i64), vp, vp, vp, vp]
    L.bem_mesh_free.argtypes = [vp]
    L.bem_mesh_free.restype = None
    L.bem_tree_build.argtypes = [vp, vp, ctypes.POINTER(_TreeOpts), ctypes.POINTER(vp)]
    L.bem_tree_export.argtypes = [vp, ctypes.POINTER(_TreeView)]
    L.bem_tree_free.argtypes = [vp]
    L.bem_tree_free.restype = None
    L.bem_tree_stats_get.argtypes = [vp, vp, i32, dbl, ctypes.POINTER(_TreeStats)]
    L.bem_matvec.argtypes = [vp, vp, i32, dbl, i32, i32, i32, i32, vp, vp]
    L.bem_matvec_noalloc.argtypes = [vp, vp, i32, dbl, i32, i32, i32, i32, vp, vp]
    L.bem_solve.argtypes = [vp, vp, i32, dbl, i32, vp, vp, ctypes.POINTER(_SolveOpts), ctypes.POINTER(_SolveInfo)]
    L.bem_field.argtypes = [vp, vp, i32, dbl, dbl, i32, vp, vp, i64, vp, vp]
    L.bem_server_create.argtypes = [ctypes.POINTER(_ServerOpts), ctypes.POINTER(vp)]
    L.bem_server_add_mesh.argtypes = [vp, vp, i64, vp, i64, ctypes.POINTER(_MeshOpts), ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(i64)]
    L.bem_server_mesh_dofs.argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    L.bem_server_submit.argtypes = [vp, ctypes.c_int32, i32, dbl, i32, vp, ctypes.POINTER(i64)]
    L.bem_server_poll.argtypes = [vp, i64, i32, vp, ctypes.POINTER(_SolveInfo), ctypes.POINTER(dbl)]
    L.bem_server_stats_get.argtypes = [vp, ctypes.POINTER(_ServerStats)]
    L.bem_server_destroy.argtypes = [vp]
    L.bem_server_destroy.restype = None
    _lib = L
    return L


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """A device, a stream (torch's current stream unless given) and torch's caching allocator."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self.torch = torch
        L = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the library runs on gfx950 only")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        dev = device

        def _a(user, nbytes, stream_):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream_ or 0)
            except Exception:  # noqa: BLE001 - reported to the library as NULL (BEM_ENOMEM)
                return None

        def _f(user, ptr, stream_):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:  # noqa: BLE001 - only at interpreter teardown
                pass

        self._cb = (_ALLOC(_a), _FREE(_f))
        self._alloc = _Allocator(self._cb[0], self._cb[1], None)
        h = ctypes.c_void_p()
        rc = L.bem_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._alloc), ctypes.byref(h))
        if rc != 0:
            raise BemError(rc, "bem_ctx_create failed: " + L.bem_last_error(None).decode())
        self.h = h
        self.L = L
        _track(self)

    def check(self, rc, what):
        if rc != 0:
            raise BemError(rc, f"{what}: {self.L.bem_last_error(self.h).decode()}")
        return rc

    PHASES = ("strength", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "combine", "direct", "other", "m2l_aux")

    def timing(self, mode):
        """Sets the event timing mode (0 / False off, 1 / True per phase with
        every phase on one stream, 2 the two heavy kernels only with the usual
        scheduling), zeroing the counters when it changes; returns the
        accumulated {phase: (ms, products)} before the switch."""
        ms = np.zeros(len(self.PHASES))
        n = np.zeros(len(self.PHASES), np.int64)
        self.check(self.L.bem_ctx_timing(self.h, int(mode), _np_ptr(ms), _np_ptr(n)), "bem_ctx_timing")
        return {p: (float(ms[i]), int(n[i])) for i, p in enumerate(self.PHASES)}

    def autotune(self, enable=True, forget=False):
        """Turns the launch-choice autotuner on or off for this context
        (forget: first empty the process's table of tuned shape classes, and
        turn it on); returns the number of shape classes tuned so far."""
        n = ctypes.c_int64()
        mode = 2 if forget else int(bool(enable))
        self.check(self.L.bem_ctx_autotune(self.h, mode, ctypes.byref(n)), "bem_ctx_autotune")
        return n.value

    def device_bytes(self, reset_peak=False):
        """(live, peak) device bytes held by the library through this context."""
        live, peak = ctypes.c_int64(), ctypes.c_int64()
        self.check(self.L.bem_ctx_device_bytes(self.h, int(reset_peak), ctypes.byref(live), ctypes.byref(peak)),
                   "bem_ctx_device_bytes")
        return live.value, peak.value

    def close(self):
        if getattr(self, "h", None):
            self.L.bem_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class Mesh:
    def __init__(self, ctx: Context, xyz, elem, edge_angle_deg: float = 30.0):
        self.ctx = ctx
        xyz = np.ascontiguousarray(xyz, np.float64)
        elem = np.ascontiguousarray(elem, np.int32)
        if elem.ndim != 2 or elem.shape[1] not in (3, 6):
            raise ValueError("elements need 3 or 6 nodes")
        h = ctypes.c_void_p()
        self.nodes_per_elem = int(elem.shape[1])
        opts = _MeshOpts(edge_angle_deg, self.nodes_per_elem)
        ctx.check(ctx.L.bem_mesh_load(ctx.h, _np_ptr(xyz), xyz.shape[0], _np_ptr(elem), elem.shape[0],
                                      ctypes.byref(opts), ctypes.byref(h)), "bem_mesh_load")
        self.h = h
        _track(self)
        n = ctypes.c_int64()
        ctx.check(ctx.L.bem_mesh_dofs(h, ctypes.byref(n), None, None, None, None), "bem_mesh_dofs")
        self.n_dof = int(n.value)
        self.n_elem = int(elem.shape[0])

    def dofs(self):
        n = self.n_dof
        ed = np.zeros((self.n_elem, self.nodes_per_elem), np.int32)
        dn = np.zeros(n, np.int32)
        dx = np.zeros((n, 3))
        nr = np.zeros((n, 3))
        self.ctx.check(self.ctx.L.bem_mesh_dofs(self.h, None, _np_ptr(ed), _np_ptr(dn), _np_ptr(dx), _np_ptr(nr)),
                       "bem_mesh_dofs")
        return {"elem_dofs": ed, "dof_node": dn, "dof_xyz": dx, "dof_normal": nr}

    def close(self):
        if getattr(self, "h", None):
            self.ctx.L.bem_mesh_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


class Tree:
    def __init__(self, ctx: Context, mesh: Mesh, B=32, order=8, theta=0.5, kappa=0.0, max_depth=21, k_hint=0.0,
                 order_min=0, attach_radii=False, m2l_slab_slots=0):
        self.ctx, self.mesh = ctx, mesh
        opts = _TreeOpts(B, order, theta, kappa, max_depth, k_hint, order_min, int(attach_radii), int(m2l_slab_slots))
        h = ctypes.c_void_p()
        ctx.check(ctx.L.bem_tree_build(ctx.h, mesh.h, ctypes.byref(opts), ctypes.byref(h)), "bem_tree_build")
        self.h = h
        self.n_dof = mesh.n_dof
        _track(self)

    def export(self):
        v = _TreeView()
        self.ctx.check(self.ctx.L.bem_tree_export(self.h, ctypes.byref(v)), "bem_tree_export")
        nb, ne, nt, nn, ni = v.n_box, v.n_elem, v.n_target, v.n_near, v.n_inter
        out = {
            "level": np.zeros(nb, np.int32), "leaf": np.zeros(nb, np.int32), "parent": np.zeros(nb, np.int32),
            "child_begin": np.zeros(nb, np.int32), "nchild": np.zeros(nb, np.int32),
            "elem_begin": np.zeros(nb, np.int64), "elem_end": np.zeros(nb, np.int64),
            "tgt_begin": np.zeros(nb, np.int64), "tgt_end": np.zeros(nb, np.int64),
            "prefix": np.zeros(nb, np.uint64), "centre": np.zeros((nb, 3)), "radius": np.zeros(nb),
            "elem_perm": np.zeros(ne, np.int32), "tgt_perm": np.zeros(nt, np.int32),
            "near_ptr": np.zeros(nb + 1, np.int64), "inter_ptr": np.zeros(nb + 1, np.int64),
            "near_idx": np.zeros(max(nn, 1), np.int32), "inter_idx": np.zeros(max(ni, 1), np.int32),
        }
        for k, a in out.items():
            setattr(v, k, _np_ptr(a))
        self.ctx.check(self.ctx.L.bem_tree_export(self.h, ctypes.byref(v)), "bem_tree_export")
        out["near_idx"] = out["near_idx"][:nn]
        out["inter_idx"] = out["inter_idx"][:ni]
        out["root"] = np.array(list(v.root))
        out["max_level"] = int(v.max_level)
        out["n_leaf"] = int(v.n_leaf)
        return out

    def stats(self, green=BEM_LAPLACE, k=0.0):
        st = _TreeStats()
        self.ctx.check(self.ctx.L.bem_tree_stats_get(self.ctx.h, self.h, green, k, ctypes.byref(st)),
                       "bem_tree_stats_get")
        return {n: int(getattr(st, n)) for n, _ in _TreeStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.ctx.L.bem_tree_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def _check_vec(t, n, green):
    import torch

    want = torch.complex128 if green == BEM_HELMHOLTZ else torch.float64
    if not t.is_cuda or t.dtype != want or not t.is_contiguous() or t.numel() % n != 0:
        raise ValueError(f"expected a contiguous {want} device tensor of nrhs x {n} values")
    return t.numel() // n


def bem_mesh_load(ctx: Context, xyz, elem, edge_angle_deg: float = 30.0) -> Mesh:
    return Mesh(ctx, xyz, elem, edge_angle_deg)


def bem_tree_build(ctx: Context, mesh: Mesh, **opts) -> Tree:
    return Tree(ctx, mesh, **opts)


def bem_matvec(ctx: Context, tree: Tree, green: int, k: float, op: int, method: int, precision: int, x, y) -> None:
    """y = op(x) on the device; x, y are torch tensors [nrhs, n_dof]."""
    nrhs = _check_vec(x, tree.n_dof, green)
    if _check_vec(y, tree.n_dof, green) != nrhs:
        raise ValueError("x and y differ in shape")
    ctx.check(ctx.L.bem_matvec(ctx.h, tree.h, green, float(k), op, method, precision, nrhs,
                               ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())), "bem_matvec")


def bem_matvec_noalloc(ctx: Context, tree: Tree, green: int, k: float, op: int, method: int, precision: int, x,
                       y) -> None:
    """bem_matvec with its work space in the library's fixed per-device
    scratch (no device allocation); the tree's tables must exist (one
    bem_matvec call with the same arguments builds them)."""
    nrhs = _check_vec(x, tree.n_dof, green)
    if _check_vec(y, tree.n_dof, green) != nrhs:
        raise ValueError("x and y differ in shape")
    ctx.check(ctx.L.bem_matvec_noalloc(ctx.h, tree.h, green, float(k), op, method, precision, nrhs,
                                       ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())),
              "bem_matvec_noalloc")


def bem_solve(ctx: Context, tree: Tree, green: int, k: float, chi, phi, tol=1e-8, restart=50, max_restarts=100,
              precision=BEM_PREC_FP64, inner_tol=0.0, max_iters=0, method=BEM_FMM, raise_on_noconv=False,
              krylov=BEM_KRYLOV_GMRES, max_seconds=0.0):
    """Solves c.phi - K phi = -S chi; returns a list of per-rhs info dicts.
    max_iters / max_seconds: step budget per right-hand side and wall-time
    budget of the call (0: none); a right-hand side that runs out reports
    BEM_ENOCONV with its last iterate."""
    nrhs = _check_vec(chi, tree.n_dof, green)
    if _check_vec(phi, tree.n_dof, green) != nrhs:
        raise ValueError("chi and phi differ in shape")
    opts = _SolveOpts(tol, restart, max_restarts, precision, inner_tol, max_iters, method, krylov, max_seconds)
    info = (_SolveInfo * nrhs)()
    rc = ctx.L.bem_solve(ctx.h, tree.h, green, float(k), nrhs, ctypes.c_void_p(chi.data_ptr()),
                         ctypes.c_void_p(phi.data_ptr()), ctypes.byref(opts), info)
    if rc != 0 and (rc != BEM_ENOCONV or raise_on_noconv):
        ctx.check(rc, "bem_solve")
    return [{n: getattr(i, n) for n, _ in _SolveInfo._fields_} for i in info]


def bem_field(ctx: Context, tree: Tree, green: int, k: float, phi, chi, pts, theta: float = 0.0):
    """Potential at points off the surface from the surface solution:
    u(x) = D[phi](x) - S[chi](x) (tree-accelerated, FP64; theta <= 0: 0.25).
    phi, chi are device tensors [nrhs, n_dof]; pts a float64 device tensor
    [n_pts, 3].  Returns u, a device tensor [nrhs, n_pts] of phi's dtype."""
    import torch

    nrhs = _check_vec(phi, tree.n_dof, green)
    if _check_vec(chi, tree.n_dof, green) != nrhs:
        raise ValueError("phi and chi differ in shape")
    if not pts.is_cuda or pts.dtype != torch.float64 or not pts.is_contiguous() or pts.dim() != 2 or pts.shape[1] != 3:
        raise ValueError("pts must be a contiguous float64 device tensor [n_pts, 3]")
    n_pts = pts.shape[0]
    u = torch.empty((nrhs, max(1, n_pts)), dtype=phi.dtype, device=phi.device)
    ctx.check(ctx.L.bem_field(ctx.h, tree.h, green, float(k), float(theta), nrhs, ctypes.c_void_p(phi.data_ptr()),
                              ctypes.c_void_p(chi.data_ptr()), n_pts, ctypes.c_void_p(pts.data_ptr()),
                              ctypes.c_void_p(u.data_ptr())), "bem_field")
    return u[:, :n_pts]


class Server:
    """Batched / concurrent solves of many problems on one GPU (bem_server_*).

    Host arrays in, host arrays out: meshes are registered once
    (add_mesh -> (id, n_dof)); submit() queues a solve of nrhs right-hand
    sides ([nrhs, n_dof] float64, or complex128 for Helmholtz) and returns a
    ticket; poll() returns (status, phi, infos, latency_s), or None while the
    request is pending and wait is False."""

    def __init__(self, device=0, lanes=4, hbm_budget=32 << 30, max_batch_rhs=32, tol=1e-8, restart=50,
                 max_restarts=100, precision=BEM_PREC_FP64, inner_tol=0.0, max_iters=0, method=BEM_FMM,
                 krylov=BEM_KRYLOV_GMRES, B=32, order=8, theta=0.5, kappa=0.0, max_depth=21, order_min=0,
                 k_hint=0.0, attach_radii=0, max_seconds=0.0, helmholtz_B=0):
        self.L = load_library()
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the library runs on gfx950 only")
        o = _ServerOpts()
        o.device, o.lanes, o.hbm_budget, o.max_batch_rhs = device, lanes, int(hbm_budget), max_batch_rhs
        # kappa > 0 with k_hint = 0: Helmholtz requests use a tree per wavenumber
        # bucket (leaf size helmholtz_B, or B when 0); with k_hint > 0 the mesh's
        # one tree serves every k up to k_hint
        o.tree = _TreeOpts(B, order, theta, kappa, max_depth, k_hint, order_min, int(attach_radii))
        o.helmholtz_B = int(helmholtz_B)
        o.solve = _SolveOpts(tol, restart, max_restarts, precision, inner_tol, max_iters, method, krylov, max_seconds)
        h = ctypes.c_void_p()
        rc = self.L.bem_server_create(ctypes.byref(o), ctypes.byref(h))
        if rc != 0:
            raise BemError(rc, "bem_server_create failed")
        self.h = h.value
        self._meta = {}  # ticket -> (nrhs, n_dof, complex)
        self._ndof = {}
        _track(self)

    def add_mesh(self, xyz, elem, edge_angle_deg: float = 30.0):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        elem = np.ascontiguousarray(elem, dtype=np.int32)
        mid, nd = ctypes.c_int32(), ctypes.c_int64()
        if elem.ndim != 2 or elem.shape[1] not in (3, 6):
            raise ValueError("elements need 3 or 6 nodes")
        rc = self.L.bem_server_add_mesh(self.h, _np_ptr(xyz), xyz.shape[0], _np_ptr(elem), elem.shape[0],
                                        ctypes.byref(_MeshOpts(edge_angle_deg, int(elem.shape[1]))),
                                        ctypes.byref(mid), ctypes.byref(nd))
        if rc != 0:
            raise BemError(rc, "bem_server_add_mesh failed")
        self._ndof[mid.value] = nd.value
        return mid.value, nd.value

    def mesh_dofs(self, mesh_id: int) -> dict:
        """DOF layout of a registered mesh: dof_xyz, dof_normal [n_dof, 3]."""
        nd = self._ndof[mesh_id]
        xyz, nrm = np.empty((nd, 3)), np.empty((nd, 3))
        rc = self.L.bem_server_mesh_dofs(self.h, mesh_id, None, _np_ptr(xyz), _np_ptr(nrm))
        if rc != 0:
            raise BemError(rc, "bem_server_mesh_dofs failed")
        return {"dof_xyz": xyz, "dof_normal": nrm}

    def submit(self, mesh_id: int, green: int, k: float, chi) -> int:
        cplx = green == BEM_HELMHOLTZ
        chi = np.ascontiguousarray(np.atleast_2d(chi), dtype=np.complex128 if cplx else np.float64)
        nrhs, nd = chi.shape
        if nd != self._ndof.get(mesh_id, -1):
            raise ValueError("chi does not match the mesh's DOF count")
        t = ctypes.c_int64()
        rc = self.L.bem_server_submit(self.h, mesh_id, green, float(k), nrhs, _np_ptr(chi), ctypes.byref(t))
        if rc != 0:
            raise BemError(rc, "bem_server_submit failed")
        self._meta[t.value] = (nrhs, nd, cplx)
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        if ticket not in self._meta:
            raise BemError(BEM_EINVAL, "unknown ticket")
        nrhs, nd, cplx = self._meta[ticket]
        phi = np.empty((nrhs, nd), dtype=np.complex128 if cplx else np.float64)
        info = (_SolveInfo * nrhs)()
        lat = ctypes.c_double()
        rc = self.L.bem_server_poll(self.h, ticket, int(wait), _np_ptr(phi), info, ctypes.byref(lat))
        if rc == BEM_EAGAIN:
            return None
        if rc == BEM_EINVAL:
            raise BemError(rc, "unknown ticket")
        del self._meta[ticket]
        return rc, phi, [{n: getattr(i, n) for n, _ in _SolveInfo._fields_} for i in info], lat.value

    def stats(self) -> dict:
        st = _ServerStats()
        rc = self.L.bem_server_stats_get(self.h, ctypes.byref(st))
        if rc != 0:
            raise BemError(rc, "bem_server_stats_get failed")
        return {n: getattr(st, n) for n, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.L.bem_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass
