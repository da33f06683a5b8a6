// Serving layer: concurrent and batched solves of many independent problems
// on one GPU (declared in include/bem.h).  Host code only: worker threads,
// per-lane contexts (each with its own stream and a hard bound on the device
// bytes it holds), a mesh registry with lane affinity, trees per
// (mesh, wavenumber bucket) kept resident under least-recently-used
// eviction, and per-lane request queues from which a worker merges the
// waiting requests of one (mesh, Green, k) into a single
// multi-right-hand-side solve.  Every right-hand side goes through bem_solve
// with the server's options on the tree its request maps to, so its result
// is the one bem_solve gives for it alone on such a tree.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "kernels.h"

namespace {

using clk = std::chrono::steady_clock;

struct Request {
    int64_t ticket = 0;
    int32_t mesh = 0;
    int green = 0;
    double k = 0.0;
    int nrhs = 0;
    std::vector<char> chi, phi;  // host copies, [nrhs][n_dof] values
    std::vector<bem_solve_info> info;
    int status = BEM_OK;
    bool done = false;
    clk::time_point t_submit, t_done;
};

// A resident tree of a mesh, for the wavenumbers up to k_hint (0: the tree
// without the wavenumber bound on its lists).
struct TreeEntry {
    double k_hint = 0.0;
    bem_tree *tree = nullptr;
    uint64_t last_use = 0;
};

struct MeshEntry {
    std::vector<double> xyz;
    std::vector<int32_t> elem;
    std::vector<int32_t> elem_dofs, dof_node;
    std::vector<double> dof_normal;
    bem_mesh_opts mopts{};
    int64_t n_nodes = 0, n_elem = 0, n_dof = 0;
    int lane = 0;
    bem_mesh *mesh = nullptr;  // resident objects, owned by the lane's context
    std::vector<TreeEntry> trees;
};

struct Lane {
    bem_ctx *ctx = nullptr;
    std::thread th;
    std::deque<Request *> q;
};

}  // namespace

struct bem_server {
    bem_server_opts o{};
    std::vector<std::unique_ptr<Lane>> lanes;
    std::vector<std::unique_ptr<MeshEntry>> meshes;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    int64_t next_ticket = 1;
    uint64_t use_clock = 0;
    double bytes_per_elem = 4.0e4;  // running estimate of a resident tree's device bytes per element
    bem_server_stats st{};
};

namespace {

size_t value_bytes(int green) { return green == BEM_HELMHOLTZ ? 16 : 8; }

// Top of the wavenumber bucket of k: 2^(ceil(4 log2 k) / 4), so that the
// wavenumbers of one bucket differ by at most 19% and share a tree whose
// lists carry the bound k (r1 + r2) <= kappa for the bucket's top.
double bucket_top(double k) { return std::exp2(std::ceil(4.0 * std::log2(k) - 1e-12) / 4.0); }

// k_hint of the tree a request of (green, k) is solved on.
double tree_key(const bem_server *s, int green, double k) {
    const bem_tree_opts &to = s->o.tree;
    if (!(to.kappa > 0.0) || !std::isfinite(to.kappa)) return 0.0;  // no wavenumber bound: one tree
    if (to.k_hint > 0.0) return to.k_hint;                          // fixed: one tree for k <= k_hint
    return green == BEM_HELMHOLTZ ? bucket_top(k) : 0.0;
}

// Bytes a solve of nrhs right-hand sides needs beyond its resident tree
// (whose per-product work buffers stay with it): Krylov bases and vectors,
// right-hand-side and staging buffers, the strengths and expansions of nrhs
// at once (a coarse upper estimate; the lane's bound is the hard limit).
size_t solve_bytes(const bem_server *s, int green, int64_t n_dof, int64_t n_elem, int nrhs) {
    const int m = s->o.solve.restart > 0 ? s->o.solve.restart : 50;
    const size_t vb = value_bytes(green);
    return (size_t)nrhs * (size_t)n_dof * vb * (size_t)(m + 12) + (size_t)nrhs * (size_t)n_elem * 7 * vb * 3 +
           ((size_t)4 << 20);
}

// Detaches the lane's least recently used tree other than (keep_mesh,
// keep_key) under the server lock; the caller frees it outside the lock (the
// lane's own thread: the only user of its context).  A mesh whose last tree
// goes is detached with it.  Returns false when nothing is left to evict.
bool detach_lru(bem_server *s, int lane, int32_t keep_mesh, double keep_key, bem_tree **tree, bem_mesh **mesh) {
    *tree = nullptr;
    *mesh = nullptr;
    MeshEntry *vm = nullptr;
    size_t vt = 0;
    for (size_t i = 0; i < s->meshes.size(); i++) {
        MeshEntry *m = s->meshes[i].get();
        if (m->lane != lane) continue;
        for (size_t j = 0; j < m->trees.size(); j++) {
            if ((int32_t)i == keep_mesh && m->trees[j].k_hint == keep_key) continue;
            if (!vm || m->trees[j].last_use < vm->trees[vt].last_use) {
                vm = m;
                vt = j;
            }
        }
    }
    if (!vm) {  // meshes left without trees (other than the one in use)
        for (size_t i = 0; i < s->meshes.size(); i++) {
            MeshEntry *m = s->meshes[i].get();
            if (m->lane == lane && m->mesh && m->trees.empty() && (int32_t)i != keep_mesh) {
                *mesh = m->mesh;
                m->mesh = nullptr;
                s->st.evictions++;
                return true;
            }
        }
        return false;
    }
    *tree = vm->trees[vt].tree;
    vm->trees.erase(vm->trees.begin() + (std::ptrdiff_t)vt);
    if (vm->trees.empty() && vm != s->meshes[keep_mesh].get()) {
        *mesh = vm->mesh;
        vm->mesh = nullptr;
    }
    s->st.evictions++;
    return true;
}

// One batch on the lane's context: the mesh and tree built if missing, the
// right-hand sides staged through buffers of the context, the solve, the
// results copied back.  Throws nothing; returns a bem_status.
int run_batch(bem_server *s, Lane &L, MeshEntry &me, TreeEntry &te, double key, int green, double k, int nrhs,
              const std::vector<char> &chi, std::vector<char> &phi, std::vector<bem_solve_info> &info) {
    bem_ctx *ctx = L.ctx;
    bem::Ctx &c = ctx->c;
    int rc = BEM_OK;
    if (!me.mesh) rc = bem_mesh_load(ctx, me.xyz.data(), me.n_nodes, me.elem.data(), me.n_elem, &me.mopts, &me.mesh);
    if (rc != BEM_OK) return rc;
    const bool fresh = !te.tree;
    const size_t before = c.bytes_live;
    if (fresh) {
        bem_tree_opts to = s->o.tree;
        to.k_hint = key;
        if (key > 0.0 && s->o.helmholtz_B > 0) to.max_elems_per_leaf = s->o.helmholtz_B;  // a per-wavenumber tree
        rc = bem_tree_build(ctx, me.mesh, &to, &te.tree);
        if (rc != BEM_OK) return rc;
        std::lock_guard<std::mutex> lk(s->mu);
        s->st.trees_built++;
    }
    const size_t vb = value_bytes(green), bytes = (size_t)nrhs * (size_t)me.n_dof * vb;
    try {
        bem::DBuf<char> dchi, dphi;
        dchi.alloc(&c, bytes);
        dphi.alloc(&c, bytes);
        BEM_HIP(hipMemcpyAsync(dchi.p, chi.data(), bytes, hipMemcpyHostToDevice, c.stream));
        rc = bem_solve(ctx, te.tree, (bem_green)green, k, nrhs, dchi.p, dphi.p, &s->o.solve, info.data());
        if (rc == BEM_OK || rc == BEM_ENOCONV) {
            BEM_HIP(hipMemcpyAsync(phi.data(), dphi.p, bytes, hipMemcpyDeviceToHost, c.stream));
            BEM_HIP(hipStreamSynchronize(c.stream));
        }
    } catch (const bem::Error &e) {
        return e.code;
    } catch (...) {
        return BEM_ENOMEM;
    }
    if (fresh && (rc == BEM_OK || rc == BEM_ENOCONV)) {
        // a resident tree's bytes per element (tree, corrections, plans,
        // operators; the solve's own buffers are freed by now)
        std::lock_guard<std::mutex> lk(s->mu);
        const double per = (double)(c.bytes_live > before ? c.bytes_live - before : 0) / (double)me.n_elem;
        s->bytes_per_elem = std::max(s->bytes_per_elem * 0.9, per);
    }
    return rc;
}

void worker(bem_server *s, int lane) {
    Lane &L = *s->lanes[lane];
    (void)hipSetDevice(s->o.device);
    const size_t limit = L.ctx->c.limit;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_work.wait(lk, [&] { return s->stop || !L.q.empty(); });
        if (L.q.empty()) {
            if (s->stop) return;
            continue;
        }
        // the oldest request and the waiting requests of the same problem
        std::vector<Request *> batch{L.q.front()};
        L.q.pop_front();
        int nrhs = batch[0]->nrhs;
        for (auto it = L.q.begin(); it != L.q.end();) {
            Request *r = *it;
            if (r->mesh == batch[0]->mesh && r->green == batch[0]->green && r->k == batch[0]->k &&
                nrhs + r->nrhs <= s->o.max_batch_rhs) {
                batch.push_back(r);
                nrhs += r->nrhs;
                it = L.q.erase(it);
            } else {
                ++it;
            }
        }
        const int32_t mid = batch[0]->mesh;
        MeshEntry &me = *s->meshes[mid];
        const int green = batch[0]->green;
        const double k = batch[0]->k;
        const double key = tree_key(s, green, k);
        // the batch's tree entry (looked up again after every eviction: erasing
        // another entry of this mesh moves it)
        auto entry = [&]() -> TreeEntry * {
            for (auto &t : me.trees)
                if (t.k_hint == key) return &t;
            me.trees.push_back(TreeEntry{key, nullptr, 0});
            return &me.trees.back();
        };
        entry()->last_use = ++s->use_clock;
        const size_t vb = value_bytes(green), n = (size_t)me.n_dof;
        std::vector<char> chi(nrhs * n * vb), phi(nrhs * n * vb);
        size_t off = 0;
        for (Request *r : batch) {
            std::memcpy(chi.data() + off, r->chi.data(), r->chi.size());
            off += r->chi.size();
        }
        std::vector<bem_solve_info> info(nrhs);
        // admission: make room for the batch's estimate by evicting the
        // lane's least recently used trees (the bound itself is enforced by
        // the context's allocator)
        const size_t need = (entry()->tree ? 0 : (size_t)(s->bytes_per_elem * me.n_elem)) +
                            solve_bytes(s, green, me.n_dof, me.n_elem, nrhs);
        int rc = BEM_OK;
        for (;;) {
            std::vector<std::pair<bem_tree *, bem_mesh *>> gone;
            while (L.ctx->c.bytes_live + L.ctx->c.cached + need > limit) {
                bem_tree *t = nullptr;
                bem_mesh *m = nullptr;
                if (!detach_lru(s, lane, mid, key, &t, &m)) break;
                gone.emplace_back(t, m);
            }
            lk.unlock();
            for (auto &g : gone) {  // device frees outside the lock
                if (g.first) bem_tree_free(g.first);
                if (g.second) bem_mesh_free(g.second);
            }
            if (L.ctx->c.bytes_live + L.ctx->c.cached + need > limit) L.ctx->c.trim_cache();
            lk.lock();
            TreeEntry *te = entry();
            lk.unlock();
            rc = run_batch(s, L, me, *te, key, green, k, nrhs, chi, phi, info);
            lk.lock();
            if (rc != BEM_ENOMEM) break;
            // past the lane's bound: one more tree goes and the batch runs again
            bem_tree *t = nullptr;
            bem_mesh *m = nullptr;
            if (!detach_lru(s, lane, mid, key, &t, &m)) break;  // nothing left: the batch does not fit
            lk.unlock();
            if (t) bem_tree_free(t);
            if (m) bem_mesh_free(m);
            L.ctx->c.trim_cache();
            lk.lock();
        }
        if (rc == BEM_ENOMEM) {  // keep nothing of a batch that does not fit
            for (size_t j = 0; j < me.trees.size(); j++)
                if (me.trees[j].k_hint == key) {
                    bem_tree *t = me.trees[j].tree;
                    me.trees.erase(me.trees.begin() + (std::ptrdiff_t)j);
                    lk.unlock();
                    if (t) bem_tree_free(t);
                    L.ctx->c.trim_cache();
                    lk.lock();
                    break;
                }
            s->st.rejected += (int64_t)batch.size();
        }
        const auto now = clk::now();
        off = 0;
        int ri = 0;
        for (Request *r : batch) {
            const size_t sz = r->chi.size();
            r->phi.assign(phi.data() + off, phi.data() + off + sz);
            r->info.assign(info.begin() + ri, info.begin() + ri + r->nrhs);
            off += sz;
            ri += r->nrhs;
            r->status = rc;
            if (rc == BEM_OK)
                for (const auto &x : r->info)
                    if (x.status != BEM_OK) r->status = x.status;
            r->done = true;
            r->t_done = now;
            r->chi.clear();
            r->chi.shrink_to_fit();
        }
        s->st.batches++;
        s->st.rhs_solved += nrhs;
        s->st.completed += (int64_t)batch.size();
        s->cv_done.notify_all();
    }
}

int lane_of_new_mesh(bem_server *s) {
    // the lane with the fewest registered elements
    std::vector<int64_t> load(s->lanes.size(), 0);
    for (auto &m : s->meshes) load[m->lane] += m->n_elem;
    return (int)(std::min_element(load.begin(), load.end()) - load.begin());
}

}  // namespace

extern "C" {

int bem_server_create(const bem_server_opts *opts, bem_server **out) {
    if (!out) return BEM_EINVAL;
    *out = nullptr;
    bem_server_opts o{};
    if (opts) o = *opts;
    if (o.lanes == 0) o.lanes = 4;
    if (o.hbm_budget == 0) o.hbm_budget = (int64_t)32 << 30;
    if (o.max_batch_rhs == 0) o.max_batch_rhs = 32;
    if (o.lanes < 1 || o.lanes > 64 || o.hbm_budget < 0 || o.max_batch_rhs < 1) return BEM_EINVAL;
    if (o.solve.max_iters < 0 || o.solve.max_seconds < 0.0 || o.helmholtz_B < 0) return BEM_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || o.device < 0 || o.device >= ndev) return BEM_EDEVICE;
    if (hipSetDevice(o.device) != hipSuccess) return BEM_EDEVICE;
    auto s = std::make_unique<bem_server>();
    s->o = o;
    auto unwind = [&](int rc) {
        for (auto &l : s->lanes) {
            hipStream_t ls = l->ctx->c.stream;
            bem_ctx_destroy(l->ctx);
            (void)hipStreamDestroy(ls);
        }
        return rc;
    };
    for (int i = 0; i < o.lanes; i++) {
        auto L = std::make_unique<Lane>();
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return unwind(BEM_EDEVICE);
        int rc = bem_ctx_create(o.device, st, nullptr, &L->ctx);
        if (rc != BEM_OK) {
            (void)hipStreamDestroy(st);
            return unwind(rc);
        }
        L->ctx->c.limit = (size_t)(o.hbm_budget / o.lanes);  // the lane's share: a hard bound
        L->ctx->c.cache_limit = std::min(L->ctx->c.cache_limit, L->ctx->c.limit / 4);
        s->lanes.push_back(std::move(L));
    }
    bem_server *raw = s.release();
    for (int i = 0; i < o.lanes; i++) raw->lanes[i]->th = std::thread(worker, raw, i);
    *out = raw;
    return BEM_OK;
}

int bem_server_add_mesh(bem_server *s, const double *node_xyz, int64_t n_nodes, const int32_t *elem_nodes,
                        int64_t n_elem, const bem_mesh_opts *opts, int32_t *mesh_id, int64_t *n_dof) {
    if (!s || !node_xyz || !elem_nodes || !mesh_id || n_elem < 1 || n_nodes < 3) return BEM_EINVAL;
    auto me = std::make_unique<MeshEntry>();
    if (opts) me->mopts = *opts;
    const int nn = me->mopts.nodes_per_elem ? me->mopts.nodes_per_elem : 6;
    if (nn != 3 && nn != 6) return BEM_EINVAL;
    me->xyz.assign(node_xyz, node_xyz + 3 * n_nodes);
    me->elem.assign(elem_nodes, elem_nodes + (int64_t)nn * n_elem);
    me->n_nodes = n_nodes;
    me->n_elem = n_elem;
    // DOF indexing on the host, as bem_mesh_load does it
    try {
        bem_mesh tmp;
        bem::load_mesh_host(tmp, node_xyz, n_nodes, elem_nodes, n_elem, nn,
                            me->mopts.edge_angle_deg > 0.0 ? me->mopts.edge_angle_deg : 30.0);
        me->n_dof = tmp.n_dof;
        me->elem_dofs.resize((size_t)nn * n_elem);  // the columns the mesh was given with
        for (int64_t e = 0; e < n_elem; e++)
            for (int a = 0; a < nn; a++) me->elem_dofs[nn * e + a] = tmp.h_elem_dofs[6 * e + a];
        me->dof_node = tmp.h_dof_node;
        me->dof_normal = tmp.h_dof_normal;
    } catch (const bem::Error &e) {
        return e.code;
    } catch (...) {
        return BEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    me->lane = lane_of_new_mesh(s);
    *mesh_id = (int32_t)s->meshes.size();
    if (n_dof) *n_dof = me->n_dof;
    s->meshes.push_back(std::move(me));
    return BEM_OK;
}

int bem_server_mesh_dofs(bem_server *s, int32_t mesh_id, int32_t *elem_dofs, double *dof_xyz, double *dof_normal) {
    if (!s) return BEM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (mesh_id < 0 || mesh_id >= (int32_t)s->meshes.size()) return BEM_EINVAL;
    const MeshEntry &m = *s->meshes[mesh_id];
    if (elem_dofs) std::memcpy(elem_dofs, m.elem_dofs.data(), sizeof(int32_t) * m.elem_dofs.size());
    if (dof_xyz)
        for (int64_t i = 0; i < m.n_dof; i++)
            for (int d = 0; d < 3; d++) dof_xyz[3 * i + d] = m.xyz[3 * (int64_t)m.dof_node[i] + d];
    if (dof_normal) std::memcpy(dof_normal, m.dof_normal.data(), sizeof(double) * m.dof_normal.size());
    return BEM_OK;
}

int bem_server_submit(bem_server *s, int32_t mesh_id, bem_green g, double k, int nrhs, const void *chi_host,
                      int64_t *ticket) {
    if (!s || !chi_host || !ticket || nrhs < 1) return BEM_EINVAL;
    if (g != BEM_LAPLACE && g != BEM_HELMHOLTZ) return BEM_EINVAL;
    if (g == BEM_HELMHOLTZ && !(k > 0.0 && std::isfinite(k))) return BEM_EINVAL;
    const bem_tree_opts &to = s->o.tree;
    if (g == BEM_HELMHOLTZ && to.kappa > 0.0 && std::isfinite(to.kappa) && to.k_hint > 0.0 && k > to.k_hint)
        return BEM_EINVAL;  // the fixed tree's lists hold the bound only up to k_hint
    std::lock_guard<std::mutex> lk(s->mu);
    if (mesh_id < 0 || mesh_id >= (int32_t)s->meshes.size()) return BEM_EINVAL;
    MeshEntry &me = *s->meshes[mesh_id];
    if (nrhs > s->o.max_batch_rhs) return BEM_EINVAL;
    auto r = std::make_unique<Request>();
    r->ticket = s->next_ticket++;
    r->mesh = mesh_id;
    r->green = g;
    r->k = g == BEM_HELMHOLTZ ? k : 0.0;
    r->nrhs = nrhs;
    const size_t bytes = (size_t)nrhs * me.n_dof * value_bytes(g);
    r->chi.assign((const char *)chi_host, (const char *)chi_host + bytes);
    r->t_submit = clk::now();
    Lane &L = *s->lanes[me.lane];
    L.q.push_back(r.get());
    *ticket = r->ticket;
    s->reqs[r->ticket] = std::move(r);
    s->st.submitted++;
    s->cv_work.notify_all();
    return BEM_OK;
}

int bem_server_poll(bem_server *s, int64_t ticket, int wait, void *phi_host, bem_solve_info *info,
                    double *latency_s) {
    if (!s) return BEM_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return BEM_EINVAL;
    Request *r = it->second.get();
    if (!r->done) {
        if (!wait) return BEM_EAGAIN;
        s->cv_done.wait(lk, [&] { return r->done; });
    }
    if (phi_host && !r->phi.empty()) std::memcpy(phi_host, r->phi.data(), r->phi.size());
    if (info)
        for (int i = 0; i < r->nrhs && i < (int)r->info.size(); i++) info[i] = r->info[i];
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    const int rc = r->status;
    s->reqs.erase(it);
    return rc;
}

int bem_server_stats_get(bem_server *s, bem_server_stats *st) {
    if (!s || !st) return BEM_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *st = s->st;
    int64_t b = 0, peak = 0;
    for (auto &l : s->lanes) {
        b += (int64_t)(l->ctx->c.bytes_live + l->ctx->c.cached);
        peak += (int64_t)l->ctx->c.held_peak;
    }
    st->resident_bytes = b;
    st->resident_peak = peak;
    return BEM_OK;
}

void bem_server_destroy(bem_server *s) {
    if (!s) return;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        // finish what is queued
        s->cv_done.wait(lk, [&] {
            for (auto &l : s->lanes)
                if (!l->q.empty()) return false;
            for (auto &r : s->reqs)
                if (!r.second->done) return false;
            return true;
        });
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &l : s->lanes)
        if (l->th.joinable()) l->th.join();
    (void)hipSetDevice(s->o.device);
    for (auto &m : s->meshes) {
        for (auto &t : m->trees)
            if (t.tree) bem_tree_free(t.tree);
        if (m->mesh) bem_mesh_free(m->mesh);
    }
    for (auto &l : s->lanes) {
        hipStream_t st = l->ctx->c.stream;
        bem_ctx_destroy(l->ctx);
        (void)hipStreamDestroy(st);
    }
    delete s;
}

}  // extern "C"
