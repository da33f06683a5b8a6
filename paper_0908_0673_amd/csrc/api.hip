// The C interface declared in include/bem.h: argument checks, defaults,
// error capture, and the calls into the tree, quadrature, product and solver
// units.  No exception crosses this file's functions.
#include <cmath>
#include <map>
#include <mutex>
#include <new>

#include "kernels.h"

using bem::Ctx;
using bem::Error;

namespace {

template <class F>
int guard(Ctx *c, F &&f) {
    try {
        if (c) {
            hipError_t e = hipSetDevice(c->device);
            if (e != hipSuccess) bem::fail(BEM_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
        }
        f();
        return BEM_OK;
    } catch (const Error &e) {
        if (c) c->err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        return BEM_ENOMEM;
    } catch (const std::exception &e) {
        if (c) c->err = e.what();
        return BEM_EINVAL;
    }
}

thread_local std::string g_err;

// Work space of bem_matvec_noalloc: one array per device, holding the
// per-product buffers (strengths, expansions, near-field partial sums, the
// multipole-to-local moments and results) of every such call on that device.
// It is held from the moment the library's code is loaded on a device until
// the process ends.  Host code never passes the array's name to a kernel: it
// stands for the host-side shadow, not a device address; each device's copy
// is reached through the address hipGetSymbolAddress returns for it.
constexpr size_t SCRATCH_BYTES = BEM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch;  // device -> its copy of scratch

// Resolves the device address of `scratch` on the current device (once per
// device; called by bem_ctx_create with its device current).
char *scratch_on_current_device(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it != g_scratch.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        bem::fail(BEM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = (char *)ptr;
    return (char *)ptr;
}

// A tree built with the wavenumber bound k (r1 + r2) <= kappa on its lists
// (Section 3.6's separation test with the Helmholtz bound) keeps the
// truncation error of the Taylor expansions in check only for the k it was
// built for (k_hint) and smaller ones.
void check_wavenumber(const bem_tree &t, int g, double k) {
    if (g != BEM_HELMHOLTZ || !(t.kappa > 0.0) || !std::isfinite(t.kappa)) return;
    BEM_REQUIRE(t.k_hint > 0.0, BEM_EINVAL,
                "this tree has the wavenumber bound (kappa > 0) but no k_hint: its lists hold no bound for "
                "any Helmholtz k; build it with k_hint >= k");
    BEM_REQUIRE(k <= t.k_hint, BEM_EINVAL,
                "Helmholtz k above the k_hint this tree's lists were built for (kappa bound)");
}

}  // namespace

extern "C" {

int bem_ctx_create(int device, void *hip_stream, const bem_allocator *alloc, bem_ctx **out) {
    if (!out) return BEM_EINVAL;
    *out = nullptr;
    bem_ctx *ctx = new (std::nothrow) bem_ctx;
    if (!ctx) return BEM_ENOMEM;
    ctx->c.device = device;
    ctx->c.stream = (hipStream_t)hip_stream;
    if (alloc && alloc->alloc && alloc->free) {
        ctx->c.alloc = *alloc;
        ctx->c.has_alloc = true;
    }
    int rc = guard(&ctx->c, [&] {
        int n = 0;
        BEM_HIP(hipGetDeviceCount(&n));
        BEM_REQUIRE(device >= 0 && device < n, BEM_EINVAL, "no such device");
        (void)scratch_on_current_device(device);  // the device is current here (guard)
    });
    if (rc != BEM_OK) {
        g_err = ctx->c.err;
        delete ctx;
        return rc;
    }
    *out = ctx;
    return BEM_OK;
}

void bem_ctx_destroy(bem_ctx *ctx) { delete ctx; }

int bem_ctx_timing(bem_ctx *ctx, int enable, double *ms, int64_t *launches) {
    if (!ctx) return BEM_EINVAL;
    Ctx &c = ctx->c;
    // the events recorded since the last call are read back now
    const int rc = guard(&c, [&] {
        if (c.ev_used || c.kev_used) {
            c.sync();
            c.collect();
        }
    });
    if (rc != BEM_OK) return rc;
    if (ms)
        for (int i = 0; i < BEM_NPHASE; i++) ms[i] = c.phase_ms[i];
    if (launches)
        for (int i = 0; i < BEM_NPHASE; i++) launches[i] = c.phase_n[i];
    if (enable < 0 || enable > 4) return BEM_EINVAL;
    if (enable && c.timing != enable) {
        for (int i = 0; i < BEM_NPHASE; i++) { c.phase_ms[i] = 0.0; c.phase_n[i] = 0; }
    }
    c.timing = enable;
    return BEM_OK;
}

int bem_ctx_autotune(bem_ctx *ctx, int enable, int64_t *classes) {
    if (!ctx || enable < 0 || enable > 2) return BEM_EINVAL;
    if (enable == 2) bem::forget_tuned_classes();
    ctx->c.autotune = enable != 0;
    if (classes) *classes = bem::tuned_classes();
    return BEM_OK;
}

int bem_ctx_device_bytes(bem_ctx *ctx, int reset_peak, int64_t *live, int64_t *peak) {
    if (!ctx) return BEM_EINVAL;
    Ctx &c = ctx->c;
    if (live) *live = (int64_t)c.bytes_live.load();
    if (peak) *peak = (int64_t)c.bytes_peak.load();
    if (reset_peak) c.bytes_peak = c.bytes_live.load();
    return BEM_OK;
}

const char *bem_last_error(const bem_ctx *ctx) { return ctx ? ctx->c.err.c_str() : g_err.c_str(); }

int bem_mesh_load(bem_ctx *ctx, const double *node_xyz, int64_t n_nodes, const int32_t *elem_nodes, int64_t n_elem,
                  const bem_mesh_opts *opts, bem_mesh **out) {
    if (!ctx || !out) return BEM_EINVAL;
    *out = nullptr;
    bem_mesh *m = nullptr;
    int rc = guard(&ctx->c, [&] {
        BEM_REQUIRE(node_xyz && elem_nodes, BEM_EINVAL, "NULL mesh arrays");
        BEM_REQUIRE(n_elem >= 1 && n_nodes >= 3, BEM_EINVAL, "empty mesh");
        BEM_REQUIRE(n_elem < (int64_t)1 << 28, BEM_EINVAL, "too many elements");
        double tol = (opts && opts->edge_angle_deg > 0.0) ? opts->edge_angle_deg : 30.0;
        const int nn = (opts && opts->nodes_per_elem) ? opts->nodes_per_elem : 6;
        m = new bem_mesh;
        m->ctx = &ctx->c;
        bem::load_mesh_host(*m, node_xyz, n_nodes, elem_nodes, n_elem, nn, tol);
        n_nodes = m->n_nodes;
        std::vector<double> dxyz(3 * m->n_dof);
        for (int64_t i = 0; i < m->n_dof; i++)
            for (int d = 0; d < 3; d++) dxyz[3 * i + d] = m->h_xyz[3 * (int64_t)m->h_dof_node[i] + d];
        Ctx &c = ctx->c;
        m->xyz.alloc(&c, 3 * n_nodes);
        m->xyz.upload(m->h_xyz.data(), 3 * n_nodes);
        m->elem.alloc(&c, 6 * n_elem);
        m->elem.upload(m->h_elem.data(), 6 * n_elem);
        m->elem_dofs.alloc(&c, 6 * n_elem);
        m->elem_dofs.upload(m->h_elem_dofs.data(), 6 * n_elem);
        m->dof_node.alloc(&c, m->n_dof);
        m->dof_node.upload(m->h_dof_node.data(), m->n_dof);
        m->dof_xyz.alloc(&c, 3 * m->n_dof);
        m->dof_xyz.upload(dxyz.data(), 3 * m->n_dof);
        c.sync();
    });
    if (rc != BEM_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return BEM_OK;
}

int bem_mesh_dofs(const bem_mesh *m, int64_t *n_dof, int32_t *elem_dofs, int32_t *dof_node, double *dof_xyz,
                  double *dof_normal) {
    if (!m) return BEM_EINVAL;
    if (n_dof) *n_dof = m->n_dof;
    if (elem_dofs) {
        const int nn = m->linear ? 3 : 6;  // the columns the mesh was given with
        for (int64_t e = 0; e < m->n_el; e++)
            for (int a = 0; a < nn; a++) elem_dofs[nn * e + a] = m->h_elem_dofs[6 * e + a];
    }
    if (dof_node) std::copy(m->h_dof_node.begin(), m->h_dof_node.end(), dof_node);
    if (dof_normal) std::copy(m->h_dof_normal.begin(), m->h_dof_normal.end(), dof_normal);
    if (dof_xyz)
        for (int64_t i = 0; i < m->n_dof; i++)
            for (int d = 0; d < 3; d++) dof_xyz[3 * i + d] = m->h_xyz[3 * (int64_t)m->h_dof_node[i] + d];
    return BEM_OK;
}

void bem_mesh_free(bem_mesh *m) { delete m; }

int bem_tree_build(bem_ctx *ctx, const bem_mesh *mesh, const bem_tree_opts *opts, bem_tree **out) {
    if (!ctx || !mesh || !out) return BEM_EINVAL;
    *out = nullptr;
    bem_tree *t = nullptr;
    int rc = guard(&ctx->c, [&] {
        BEM_REQUIRE(mesh->ctx == &ctx->c, BEM_ESTATE, "mesh belongs to another context");
        t = new bem_tree;
        t->ctx = &ctx->c;
        t->mesh = mesh;
        if (opts) {
            if (opts->max_elems_per_leaf > 0) t->B = opts->max_elems_per_leaf;
            if (opts->order > 0) t->order = opts->order;
            if (opts->theta > 0.0) t->theta = opts->theta;
            t->kappa = opts->kappa;
            if (opts->max_depth > 0) t->max_depth = opts->max_depth;
            t->k_hint = opts->k_hint;
            t->order_min = opts->order_min;
            BEM_REQUIRE(opts->attach_radii >= 0 && opts->attach_radii <= 2, BEM_EINVAL, "attach_radii must be 0, 1 or 2");
            t->attach = opts->attach_radii != 0;
            t->literal = opts->attach_radii == 2;
            BEM_REQUIRE(opts->m2l_slab_slots >= 0, BEM_EINVAL, "m2l_slab_slots must be >= 0");
            if (opts->m2l_slab_slots > 0) t->m2l_slab = opts->m2l_slab_slots;
        }
        BEM_REQUIRE(t->order_min >= 0, BEM_EINVAL, "order_min must be >= 0");
        if (t->order_min >= t->order) t->order_min = 0;
        BEM_REQUIRE(t->order >= 1 && t->order <= 8, BEM_EUNSUPPORTED, "expansion order must be 1..8");
        BEM_REQUIRE(t->max_depth <= bem::MAXLEV, BEM_EINVAL, "max_depth must be <= 21");
        BEM_REQUIRE(t->theta > 0.0 && t->theta <= 1.0, BEM_EINVAL, "theta must be in (0, 1]");
        {
            bem::SetupTimer st_(ctx->c, "tree and lists");
            bem::build_tree(*t);
        }
        {
            bem::SetupTimer st_(ctx->c, "geometry in tree order");
            bem::build_geometry(*t);
        }
        ctx->c.sync();
    });
    if (rc != BEM_OK) {
        delete t;
        return rc;
    }
    *out = t;
    return BEM_OK;
}

int bem_tree_export(const bem_tree *t, bem_tree_view *v) {
    if (!t || !v) return BEM_EINVAL;
    Ctx *c = t->ctx;
    return guard(c, [&] {
        v->n_box = t->n_box;
        v->n_elem = t->n_el;
        v->n_target = t->n_tgt;
        v->n_near = t->n_near;
        v->n_inter = t->n_inter;
        v->n_leaf = t->n_leaf;
        v->max_level = t->max_level;
        for (int d = 0; d < 3; d++) v->root[d] = t->corner[d];
        v->root[3] = t->side;
        auto cp = [](auto &buf, auto *dst, size_t n) {
            if (!dst) return;
            auto h = buf.download(n);
            std::copy(h.begin(), h.end(), dst);
        };
        cp(t->level, v->level, t->n_box);
        cp(t->leaf, v->leaf, t->n_box);
        cp(t->parent, v->parent, t->n_box);
        cp(t->child_begin, v->child_begin, t->n_box);
        cp(t->nchild, v->nchild, t->n_box);
        cp(t->eb, v->elem_begin, t->n_box);
        cp(t->ee, v->elem_end, t->n_box);
        cp(t->tb, v->tgt_begin, t->n_box);
        cp(t->te, v->tgt_end, t->n_box);
        cp(t->prefix, v->prefix, t->n_box);
        cp(t->centre, v->centre, 3 * t->n_box);
        cp(t->radius, v->radius, t->n_box);
        cp(t->eperm, v->elem_perm, t->n_el);
        cp(t->tperm, v->tgt_perm, t->n_tgt);
        cp(t->near_ptr, v->near_ptr, t->n_box + 1);
        cp(t->inter_ptr, v->inter_ptr, t->n_box + 1);
        cp(t->near_idx, v->near_idx, t->n_near);
        cp(t->inter_idx, v->inter_idx, t->n_inter);
    });
}

void bem_tree_free(bem_tree *t) { delete t; }

int bem_tree_stats_get(bem_ctx *ctx, const bem_tree *tc, bem_green g, double k, bem_tree_stats *st) {
    if (!ctx || !tc || !st) return BEM_EINVAL;
    bem_tree *t = const_cast<bem_tree *>(tc);
    return guard(&ctx->c, [&] {
        (void)g;
        (void)k;
        bem::plan_fmm(*t);
        bem::build_pairs(*t);
        st->n_box = t->n_box;
        st->n_leaf = t->n_leaf;
        st->n_quad = t->n_q;
        st->n_p2p = t->n_p2p_pairs;
        st->n_corr_pairs = t->n_pairs;
        int64_t m2l = 0, same = 0;
        for (int64_t b = 0; b < t->n_box; b++) {
            if (t->h_te[b] == t->h_tb[b]) continue;
            for (int64_t j = t->h_inter_ptr[b]; j < t->h_inter_ptr[b + 1]; j++) {
                m2l++;
                if (t->h_level[t->h_inter_idx[j]] == t->h_level[b]) same++;
            }
        }
        st->n_m2l = m2l;
        st->n_m2l_same_level = same;
    });
}

int bem_matvec(bem_ctx *ctx, const bem_tree *tc, bem_green g, double k, bem_op op, bem_method m, bem_precision p,
               int nrhs, const void *x_dev, void *y_dev) {
    if (!ctx || !tc) return BEM_EINVAL;
    bem_tree *t = const_cast<bem_tree *>(tc);
    return guard(&ctx->c, [&] {
        BEM_REQUIRE(t->ctx == &ctx->c, BEM_ESTATE, "tree belongs to another context");
        BEM_REQUIRE(nrhs >= 1 && nrhs <= 65535, BEM_EINVAL, "nrhs must be in 1..65535");
        BEM_REQUIRE(x_dev && y_dev && x_dev != y_dev, BEM_EINVAL, "x and y must be distinct device buffers");
        BEM_REQUIRE(g == BEM_LAPLACE || g == BEM_HELMHOLTZ, BEM_EINVAL, "unknown Green's function");
        BEM_REQUIRE(g != BEM_HELMHOLTZ || (k > 0.0 && std::isfinite(k)), BEM_EINVAL, "Helmholtz needs k > 0");
        BEM_REQUIRE(op >= BEM_OP_S && op <= BEM_OP_RHS, BEM_EINVAL, "unknown operator");
        BEM_REQUIRE(m == BEM_DIRECT || m == BEM_FMM, BEM_EINVAL, "unknown method");
        BEM_REQUIRE(p == BEM_PREC_FP64 || p == BEM_PREC_MIXED, BEM_EINVAL, "unknown precision");
        check_wavenumber(*t, g, k);
        bem::matvec(*t, g, g == BEM_HELMHOLTZ ? k : 0.0, op, m, p, nrhs, x_dev, y_dev);
    });
}

int bem_matvec_noalloc(bem_ctx *ctx, const bem_tree *tc, bem_green g, double k, bem_op op, bem_method m,
                       bem_precision p, int nrhs, const void *x_dev, void *y_dev) {
    if (!ctx || !tc) return BEM_EINVAL;
    bem_tree *t = const_cast<bem_tree *>(tc);
    Ctx &c = ctx->c;
    return guard(&c, [&] {
        BEM_REQUIRE(t->ctx == &c, BEM_ESTATE, "tree belongs to another context");
        BEM_REQUIRE(nrhs >= 1 && nrhs <= 65535, BEM_EINVAL, "nrhs must be in 1..65535");
        BEM_REQUIRE(x_dev && y_dev && x_dev != y_dev, BEM_EINVAL, "x and y must be distinct device buffers");
        BEM_REQUIRE(g == BEM_LAPLACE || g == BEM_HELMHOLTZ, BEM_EINVAL, "unknown Green's function");
        BEM_REQUIRE(g != BEM_HELMHOLTZ || (k > 0.0 && std::isfinite(k)), BEM_EINVAL, "Helmholtz needs k > 0");
        BEM_REQUIRE(op >= BEM_OP_S && op <= BEM_OP_RHS, BEM_EINVAL, "unknown operator");
        BEM_REQUIRE(m == BEM_DIRECT || m == BEM_FMM, BEM_EINVAL, "unknown method");
        BEM_REQUIRE(p == BEM_PREC_FP64 || p == BEM_PREC_MIXED, BEM_EINVAL, "unknown precision");
        check_wavenumber(*t, g, k);
        const double kk = g == BEM_HELMHOLTZ ? k : 0.0;
        BEM_REQUIRE(c.timing == 0, BEM_ESTATE, "bem_matvec_noalloc runs with phase timing off");
        BEM_REQUIRE(bem::product_ready(*t, g, kk, op, m, p), BEM_ESTATE,
                    "the tree's tables for this product are not built: call bem_matvec once with the same "
                    "green, k, op, method and precision first");
        char *base = nullptr;
        {
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            auto it = g_scratch.find(c.device);
            BEM_REQUIRE(it != g_scratch.end(), BEM_ESTATE, "no scratch resolved for this device");
            base = it->second;
        }
        struct ArenaScope {  // the arena holds for this product only, whatever happens in it
            Ctx &c;
            ArenaScope(Ctx &c_, char *b) : c(c_) {
                c.arena = b;
                c.arena_size = SCRATCH_BYTES;
                c.arena_used = 0;
            }
            ~ArenaScope() {
                c.arena = nullptr;
                c.arena_size = c.arena_used = 0;
            }
        } scope(c, base);
        bem::matvec(*t, g, kk, op, m, p, nrhs, x_dev, y_dev);
    });
}

int bem_solve(bem_ctx *ctx, const bem_tree *tc, bem_green g, double k, int nrhs, const void *chi_dev, void *phi_dev,
              const bem_solve_opts *opts, bem_solve_info *info) {
    if (!ctx || !tc) return BEM_EINVAL;
    bem_tree *t = const_cast<bem_tree *>(tc);
    int status = BEM_OK;
    int rc = guard(&ctx->c, [&] {
        BEM_REQUIRE(t->ctx == &ctx->c, BEM_ESTATE, "tree belongs to another context");
        BEM_REQUIRE(nrhs >= 1, BEM_EINVAL, "nrhs must be >= 1");
        BEM_REQUIRE(chi_dev && phi_dev && chi_dev != phi_dev, BEM_EINVAL, "chi and phi must be distinct buffers");
        BEM_REQUIRE(g == BEM_LAPLACE || g == BEM_HELMHOLTZ, BEM_EINVAL, "unknown Green's function");
        BEM_REQUIRE(g != BEM_HELMHOLTZ || (k > 0.0 && std::isfinite(k)), BEM_EINVAL, "Helmholtz needs k > 0");
        bem_solve_opts o{};
        if (opts) o = *opts;
        if (!(o.tol > 0.0)) o.tol = 1e-8;
        if (o.restart <= 0) o.restart = 50;
        if (o.max_restarts <= 0) o.max_restarts = 100;
        if (!(o.inner_tol > 0.0)) o.inner_tol = 1e-6;
        if (!opts) o.method = BEM_FMM;
        BEM_REQUIRE(o.krylov == BEM_KRYLOV_GMRES || o.krylov == BEM_KRYLOV_BICGSTAB, BEM_EINVAL,
                    "unknown Krylov method");
        BEM_REQUIRE(o.krylov != BEM_KRYLOV_GMRES || o.restart <= 90, BEM_EINVAL, "GMRES restart must be <= 90");
        BEM_REQUIRE(o.method == BEM_FMM || o.method == BEM_DIRECT, BEM_EINVAL, "unknown method");
        BEM_REQUIRE(o.max_iters >= 0 && o.max_seconds >= 0.0, BEM_EINVAL, "max_iters and max_seconds must be >= 0");
        check_wavenumber(*t, g, k);
        status = bem::solve(*t, g, g == BEM_HELMHOLTZ ? k : 0.0, nrhs, chi_dev, phi_dev, o, info);
    });
    if (rc != BEM_OK) return rc;
    if (status != BEM_OK) ctx->c.err = "solver did not reach the tolerance";
    return status;
}

int bem_field(bem_ctx *ctx, const bem_tree *tc, bem_green g, double k, double theta, int nrhs, const void *phi_dev,
              const void *chi_dev, int64_t n_pts, const double *pts_dev, void *u_dev) {
    if (!ctx || !tc) return BEM_EINVAL;
    bem_tree *t = const_cast<bem_tree *>(tc);
    return guard(&ctx->c, [&] {
        BEM_REQUIRE(t->ctx == &ctx->c, BEM_ESTATE, "tree belongs to another context");
        BEM_REQUIRE(nrhs >= 1 && nrhs <= 65535, BEM_EINVAL, "nrhs must be in 1..65535");
        BEM_REQUIRE(n_pts >= 0 && n_pts <= 0x7fffffff, BEM_EINVAL, "n_pts must be in 0..2^31-1");
        BEM_REQUIRE(phi_dev && chi_dev && (n_pts == 0 || (pts_dev && u_dev)), BEM_EINVAL, "missing buffer");
        BEM_REQUIRE(u_dev != phi_dev && u_dev != chi_dev, BEM_EINVAL, "u must not alias phi or chi");
        BEM_REQUIRE(g == BEM_LAPLACE || g == BEM_HELMHOLTZ, BEM_EINVAL, "unknown Green's function");
        BEM_REQUIRE(g != BEM_HELMHOLTZ || (k > 0.0 && std::isfinite(k)), BEM_EINVAL, "Helmholtz needs k > 0");
        BEM_REQUIRE(!(theta > 1.0) && !std::isnan(theta), BEM_EINVAL, "theta must be at most 1");
        check_wavenumber(*t, g, k);
        bem::field(*t, g, g == BEM_HELMHOLTZ ? k : 0.0, theta, nrhs, phi_dev, chi_dev, n_pts, pts_dev, u_dev);
    });
}

}  // extern "C"
