// Serving layer: concurrent and batched solves of many independent problems
// on one GPU (declared in include/bem.h).  Host code only: worker threads,
// per-lane contexts (each with its own stream), a mesh registry with lane
// affinity and least-recently-used eviction under a device-memory budget,
// and per-lane request queues from which a worker merges the waiting
// requests of one (mesh, Green, k) into a single multi-right-hand-side solve.
// Every right-hand side goes through bem_solve with the server's options, so
// its result is the one bem_solve gives for it alone.
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

struct MeshEntry {
    std::vector<double> xyz;
    std::vector<int32_t> elem;
    std::vector<int32_t> elem_dofs, dof_node;
    std::vector<double> dof_normal;
    bem_mesh_opts mopts{};
    int64_t n_nodes = 0, n_elem = 0, n_dof = 0;
    int lane = 0;
    bem_mesh *mesh = nullptr;  // resident objects, owned by the lane's context
    bem_tree *tree = nullptr;
    size_t bytes = 0;          // device bytes of mesh + tree + caches when last measured
    uint64_t last_use = 0;
};

struct Lane {
    bem_ctx *ctx = nullptr;
    std::thread th;
    std::deque<Request *> q;
    size_t pending_rhs = 0;
    void *dchi = nullptr, *dphi = nullptr;  // device staging of the right-hand sides
    size_t dbytes = 0;
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
    double bytes_per_elem = 4.0e4;  // running estimate of a resident mesh's device bytes per element
    bem_server_stats st{};
};

namespace {

size_t value_bytes(int green) { return green == BEM_HELMHOLTZ ? 16 : 8; }

// Evicts the lane's least recently used idle meshes until `need` more bytes
// fit its share of the budget.  Called by the lane's worker (the only user of
// its context) with the server lock held.
void make_room(bem_server *s, int lane, size_t need, int32_t keep) {
    Lane &L = *s->lanes[lane];
    const size_t share = (size_t)(s->o.hbm_budget / s->o.lanes);
    if (L.ctx->c.bytes_live + L.ctx->c.cached + need > share) L.ctx->c.trim_cache();
    while (L.ctx->c.bytes_live + need > share) {
        MeshEntry *victim = nullptr;
        int32_t vid = -1;
        for (size_t i = 0; i < s->meshes.size(); i++) {
            MeshEntry *m = s->meshes[i].get();
            if (m->lane != lane || !m->mesh || (int32_t)i == keep) continue;
            if (!victim || m->last_use < victim->last_use) {
                victim = m;
                vid = (int32_t)i;
            }
        }
        if (!victim) break;  // nothing left to evict: a mesh larger than the share is served alone
        (void)vid;
        bem_tree_free(victim->tree);
        bem_mesh_free(victim->mesh);
        victim->tree = nullptr;
        victim->mesh = nullptr;
        s->st.evictions++;
    }
}

void worker(bem_server *s, int lane) {
    Lane &L = *s->lanes[lane];
    (void)hipSetDevice(s->o.device);
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
        L.pending_rhs -= nrhs;
        MeshEntry &me = *s->meshes[batch[0]->mesh];
        me.last_use = ++s->use_clock;
        const int green = batch[0]->green;
        const double k = batch[0]->k;
        const size_t vb = value_bytes(green), n = (size_t)me.n_dof;
        int rc = BEM_OK;
        if (!me.mesh) {
            make_room(s, lane, (size_t)(s->bytes_per_elem * me.n_elem), batch[0]->mesh);
            s->st.trees_built++;
        }
        std::vector<char> chi(nrhs * n * vb), phi(nrhs * n * vb);
        size_t off = 0;
        for (Request *r : batch) {
            std::memcpy(chi.data() + off, r->chi.data(), r->chi.size());
            off += r->chi.size();
        }
        std::vector<bem_solve_info> info(nrhs);
        lk.unlock();
        // device work of this lane, outside the lock
        bem_ctx *ctx = L.ctx;
        if (!me.mesh) {
            const size_t before = ctx->c.bytes_live;
            rc = bem_mesh_load(ctx, me.xyz.data(), me.n_nodes, me.elem.data(), me.n_elem, &me.mopts, &me.mesh);
            if (rc == BEM_OK) rc = bem_tree_build(ctx, me.mesh, &s->o.tree, &me.tree);
            if (rc == BEM_OK) {
                me.bytes = ctx->c.bytes_live - before;
            } else {
                // leave the mesh unbuilt; a later request retries
                if (me.tree) bem_tree_free(me.tree);
                if (me.mesh) bem_mesh_free(me.mesh);
                me.tree = nullptr;
                me.mesh = nullptr;
            }
        }
        const size_t need = 2 * nrhs * n * vb;
        if (rc == BEM_OK && L.dbytes < need) {
            if (L.dchi) (void)hipFree(L.dchi);
            if (L.dphi) (void)hipFree(L.dphi);
            L.dchi = L.dphi = nullptr;
            L.dbytes = 0;
            if (hipMalloc(&L.dchi, need / 2) != hipSuccess || hipMalloc(&L.dphi, need / 2) != hipSuccess)
                rc = BEM_ENOMEM;
            else
                L.dbytes = need;
        }
        hipStream_t st = ctx->c.stream;
        if (rc == BEM_OK && (hipMemcpyAsync(L.dchi, chi.data(), nrhs * n * vb, hipMemcpyHostToDevice, st) != hipSuccess ||
                             hipStreamSynchronize(st) != hipSuccess))
            rc = BEM_EDEVICE;
        // Helmholtz with the wavenumber bound on the lists (tree.kappa > 0) and
        // no fixed k_hint: the batch gets a tree of its own k, freed after it
        bem_tree *own = nullptr;
        if (rc == BEM_OK && green == BEM_HELMHOLTZ && s->o.tree.kappa > 0.0 && s->o.tree.k_hint == 0.0) {
            bem_tree_opts to = s->o.tree;
            to.k_hint = k;
            rc = bem_tree_build(ctx, me.mesh, &to, &own);
        }
        if (rc == BEM_OK) {
            const size_t before = ctx->c.bytes_live;
            rc = bem_solve(ctx, own ? own : me.tree, (bem_green)green, k, nrhs, L.dchi, L.dphi, &s->o.solve,
                           info.data());
            // the first solve of a (Green, k) caches its corrections on the tree
            if (!own) me.bytes += ctx->c.bytes_live > before ? ctx->c.bytes_live - before : 0;
            if (rc == BEM_OK || rc == BEM_ENOCONV) {
                if (hipMemcpyAsync(phi.data(), L.dphi, nrhs * n * vb, hipMemcpyDeviceToHost, st) != hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess)
                    rc = BEM_EDEVICE;
            }
        }
        if (own) bem_tree_free(own);
        lk.lock();
        if (me.bytes && me.n_elem)
            s->bytes_per_elem = std::max(s->bytes_per_elem * 0.5, (double)me.bytes / (double)me.n_elem);
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
    L.pending_rhs += nrhs;
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
    int64_t b = 0;
    for (auto &l : s->lanes) b += (int64_t)(l->ctx->c.bytes_live + l->ctx->c.cached) + (int64_t)l->dbytes;
    st->resident_bytes = b;
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
        if (m->tree) bem_tree_free(m->tree);
        if (m->mesh) bem_mesh_free(m->mesh);
    }
    for (auto &l : s->lanes) {
        if (l->dchi) (void)hipFree(l->dchi);
        if (l->dphi) (void)hipFree(l->dphi);
        hipStream_t st = l->ctx->c.stream;
        bem_ctx_destroy(l->ctx);
        (void)hipStreamDestroy(st);
    }
    delete s;
}

}  // extern "C"
