// Octree build on the device (Sections 3.1, 3.4, 3.6).
//
// This translation unit is compiled with -ffp-contract=off: every
// floating-point step that decides the tree (root cube, key quantisation,
// centres, radii, the separation test) is a plain IEEE operation, so the tree
// and its lists are reproducible bit for bit by any implementation of the
// same formulas.
//
//  1. Root: a cube around all nodes, side = largest extent * (1 + 2^-20),
//     centred on the bounding box.
//  2. Keys: element key point = mean of the three corner nodes; targets are
//     the DOF positions.  Each coordinate is quantised to 21 bits and the bits
//     are interleaved (x highest in each triplet) into a 63-bit Morton key.
//  3. One stable radix sort of all items (elements first, then targets, so
//     equal keys keep elements before targets and ids ascending).
//  4. Level by level: the active items (those inside boxes split at the level
//     above) are cut into runs of equal key prefix; each run is a box.  A box
//     is split when it holds more than B elements and lies above max_depth.
//     Boxes come out ordered by (level, prefix).
//  5. Radii (Section 3.4): a leaf's radius is the largest distance from its
//     centre to a node of an element it owns or to a target it owns; a
//     parent's is the largest child radius plus half a child diagonal (Eq. 13).
//  6. Lists (Section 3.6): each box scans its parent's near list; a leaf
//     entry is kept whole, a non-leaf entry contributes its children; each
//     candidate goes to the interaction list when well separated (Eq. 14 with
//     the safety factor theta and, for Helmholtz, the k (r1 + r2) <= kappa
//     bound), else to the near list.  Boxes holding no element are skipped.
#include <cmath>

#include "kernels.h"

namespace bem {

namespace {

constexpr int BS = 256;

__device__ __host__ inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __host__ inline uint64_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return v;
}

__device__ inline uint64_t quantise(double x, double corner, double scale) {
    double v = floor((x - corner) * scale);
    if (v < 0.0) v = 0.0;
    if (v > 2097151.0) v = 2097151.0;
    return (uint64_t)v;
}

// per-block min/max of node coordinates
__global__ void k_bbox_partial(const double *xyz, int64_t n, double *part /* [nb][6] */) {
    __shared__ double s[6][BS];
    double lo[3], hi[3];
    for (int d = 0; d < 3; d++) { lo[d] = xyz[d]; hi[d] = xyz[d]; }
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS)
        for (int d = 0; d < 3; d++) {
            double v = xyz[3 * i + d];
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
        }
    for (int d = 0; d < 3; d++) { s[d][threadIdx.x] = lo[d]; s[3 + d][threadIdx.x] = hi[d]; }
    __syncthreads();
    for (int o = BS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int d = 0; d < 3; d++) {
                s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + o]);
                s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + o]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; d++) part[6 * blockIdx.x + d] = s[d][0];
}

// root cube: out = corner[3], side, scale
__global__ void k_root(const double *part, int nb, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double lo[3], hi[3];
    for (int d = 0; d < 3; d++) { lo[d] = part[d]; hi[d] = part[3 + d]; }
    for (int b = 1; b < nb; b++)
        for (int d = 0; d < 3; d++) {
            lo[d] = fmin(lo[d], part[6 * b + d]);
            hi[d] = fmax(hi[d], part[6 * b + 3 + d]);
        }
    double ext = 0.0;
    for (int d = 0; d < 3; d++)
        if (hi[d] - lo[d] > ext) ext = hi[d] - lo[d];
    double side = ext * (1.0 + 0x1p-20);
    for (int d = 0; d < 3; d++) out[d] = (lo[d] + hi[d]) * 0.5 - side * 0.5;
    out[3] = side;
    out[4] = 2097152.0 / side;
}

// lit: the literal tree, whose sources are the DOFs (n_el = n_tgt, keyed at the DOF points)
__global__ void k_keys(const double *xyz, const int32_t *elem, int64_t n_el, const double *dof_xyz, int64_t n_tgt,
                       int lit, const double *root, uint64_t *key, int32_t *val) {
    int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n_el + n_tgt) return;
    double p[3];
    if (i < n_el && lit) {
        for (int d = 0; d < 3; d++) p[d] = dof_xyz[3 * i + d];
    } else if (i < n_el) {
        const int32_t *en = elem + 6 * i;
        for (int d = 0; d < 3; d++)
            p[d] = ((xyz[3 * (int64_t)en[0] + d] + xyz[3 * (int64_t)en[1] + d]) + xyz[3 * (int64_t)en[2] + d]) / 3.0;
    } else {
        for (int d = 0; d < 3; d++) p[d] = dof_xyz[3 * (i - n_el) + d];
    }
    uint64_t q0 = quantise(p[0], root[0], root[4]);
    uint64_t q1 = quantise(p[1], root[1], root[4]);
    uint64_t q2 = quantise(p[2], root[2], root[4]);
    key[i] = (spread3(q0) << 2) | (spread3(q1) << 1) | spread3(q2);
    val[i] = (int32_t)i;
}

__global__ void k_is_elem(const int32_t *val, int64_t n, int64_t n_el, int64_t *flag) {
    int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i < n) flag[i] = val[i] < n_el ? 1 : 0;
}

__global__ void k_perms(const int32_t *val, const int64_t *E, int64_t n, int64_t n_el, int32_t *eperm, int32_t *tperm) {
    int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    int32_t v = val[i];
    if (v < n_el) eperm[E[i]] = v;
    else tperm[i - E[i]] = (int32_t)(v - n_el);
}

__device__ inline uint64_t pfx(uint64_t key, int level) { return level == 0 ? 0ull : key >> (3 * (MAXLEV - level)); }

__global__ void k_heads(const uint64_t *key, const int32_t *active, int64_t n, int level, int32_t *head) {
    int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n) return;
    int h = 0;
    if (active[i]) h = (i == 0 || !active[i - 1] || pfx(key[i], level) != pfx(key[i - 1], level)) ? 1 : 0;
    head[i] = h;
}

__global__ void k_box_ranges(const int32_t *active, const int32_t *head, const int32_t *hs, int64_t n, int64_t *first,
                             int64_t *last) {
    int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n || !active[i]) return;
    int32_t b = hs[i] + head[i] - 1;
    if (head[i]) first[b] = i;
    if (i == n - 1 || !active[i + 1] || head[i + 1]) last[b] = i;
}

__global__ void k_box_fill(const uint64_t *key, const int64_t *E, const int64_t *first, const int64_t *last,
                           const int32_t *item_box, int64_t nb, int64_t off, int level, int B, int max_depth,
                           int32_t *blevel, int32_t *bleaf, int32_t *bparent, int64_t *beb, int64_t *bee, int64_t *btb,
                           int64_t *bte, uint64_t *bprefix) {
    int64_t b = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (b >= nb) return;
    int64_t f = first[b], l = last[b] + 1;
    int64_t eb = E[f], ee = E[l];
    int64_t g = off + b;
    blevel[g] = level;
    beb[g] = eb;
    bee[g] = ee;
    btb[g] = f - eb;
    bte[g] = l - ee;
    bprefix[g] = pfx(key[f], level);
    bparent[g] = level == 0 ? -1 : item_box[f];
    bleaf[g] = ((ee - eb) > B && level < max_depth) ? 0 : 1;
}

__global__ void k_update_items(const int32_t *head, const int32_t *hs, int64_t n, int64_t off, const int32_t *bleaf,
                               int32_t *active, int32_t *item_box) {
    int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n || !active[i]) return;
    int32_t b = (int32_t)(off + hs[i] + head[i] - 1);
    item_box[i] = b;
    active[i] = bleaf[b] ? 0 : 1;
}

__global__ void k_children(const int32_t *parent, int64_t n_box, int32_t *child_begin, int32_t *nchild) {
    int64_t b = 1 + (int64_t)blockIdx.x * BS + threadIdx.x;
    if (b >= n_box) return;
    int32_t p = parent[b];
    if (parent[b - 1] != p || b == 1) child_begin[p] = (int32_t)b;
    if (b == n_box - 1 || parent[b + 1] != p) {
        // first child: walk back is avoided by counting from the level order:
        // children of p are contiguous and end at b
        int64_t f = b;
        while (f > 1 && parent[f - 1] == p) f--;
        nchild[p] = (int32_t)(b - f + 1);
    }
}

__global__ void k_centres(const int32_t *level, const uint64_t *prefix, int64_t n_box, const double *root,
                          double *centre) {
    int64_t b = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (b >= n_box) return;
    double h = ldexp(root[3], -level[b]);
    uint64_t p = prefix[b];
    uint64_t ip[3] = {compact3(p >> 2), compact3(p >> 1), compact3(p)};
    for (int d = 0; d < 3; d++) centre[3 * b + d] = root[d] + h * ((double)ip[d] + 0.5);
}

__device__ inline double dist3(const double *a, const double *b) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt((dx * dx + dy * dy) + dz * dz);
}

// one wave per leaf box; with node_ptr (attached radii) the nodes of every
// element holding a target's geometric node count too
__global__ void k_leaf_radius(const int32_t *leaf, const int64_t *eb, const int64_t *ee, const int64_t *tb,
                              const int64_t *te, const double *centre, const int32_t *eperm, const int32_t *tperm,
                              const int32_t *elem, const double *xyz, const double *dof_xyz, const int32_t *dof_node,
                              const int64_t *node_ptr, const int32_t *node_elems, int owned, int64_t n_box,
                              double *radius) {
    int64_t b = (int64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (b >= n_box || !leaf[b]) return;
    const double *c = centre + 3 * b;
    double r = 0.0;
    int64_t ne = owned ? 6 * (ee[b] - eb[b]) : 0;  // owned elements (none in the literal tree)
    for (int64_t j = lane; j < ne; j += 64) {
        int32_t e = eperm[eb[b] + j / 6];
        double v = dist3(xyz + 3 * (int64_t)elem[6 * (int64_t)e + j % 6], c);
        r = fmax(r, v);
    }
    for (int64_t j = tb[b] + lane; j < te[b]; j += 64) {
        r = fmax(r, dist3(dof_xyz + 3 * (int64_t)tperm[j], c));
        if (!node_ptr) continue;
        const int32_t g = dof_node[tperm[j]];
        for (int64_t p = node_ptr[g]; p < node_ptr[g + 1]; p++)
            for (int a = 0; a < 6; a++) r = fmax(r, dist3(xyz + 3 * (int64_t)elem[6 * (int64_t)node_elems[p] + a], c));
    }
    r = wave_max(r);
    if (lane == 0) radius[b] = r;
}

__global__ void k_parent_radius(const int32_t *leaf, const int32_t *child_begin, const int32_t *nchild,
                                const int32_t *level, int64_t lo, int64_t hi, const double *root, double *radius) {
    int64_t b = lo + (int64_t)blockIdx.x * BS + threadIdx.x;
    if (b >= hi || leaf[b]) return;
    double rc = 0.0;
    for (int c = 0; c < nchild[b]; c++) {
        double v = radius[child_begin[b] + c];
        if (v > rc) rc = v;
    }
    double hc = ldexp(root[3], -(level[b] + 1));
    radius[b] = rc + (sqrt(3.0) * hc) * 0.5;
}

struct SepArgs {
    double theta, kappa, k;
    int use_kappa;
};

__device__ inline bool well_separated(const double *centre, const double *radius, int64_t X, int64_t Y, SepArgs a) {
    double s = radius[X] + radius[Y];
    if (a.use_kappa && a.k * s > a.kappa) return false;
    return dist3(centre + 3 * X, centre + 3 * Y) > s / a.theta;
}

// count (pass 0) or emit (pass 1) the lists of the boxes [lo, hi)
template <int PASS>
__global__ void k_lists(int64_t lo, int64_t hi, const int32_t *parent, const int32_t *leaf, const int32_t *child_begin,
                        const int32_t *nchild, const int64_t *eb, const int64_t *ee, const double *centre,
                        const double *radius, SepArgs sa, const int64_t *near_ptr, const int32_t *near_idx,
                        int64_t *cnt_near, int64_t *cnt_inter, const int64_t *off_near, const int64_t *off_inter,
                        int64_t base_near, int64_t base_inter, int32_t *out_near, int32_t *out_inter) {
    int64_t b = lo + (int64_t)blockIdx.x * BS + threadIdx.x;
    if (b >= hi) return;
    int64_t P = parent[b];
    int64_t wn = 0, wi = 0;
    if (PASS == 1) {
        wn = base_near + off_near[b - lo];
        wi = base_inter + off_inter[b - lo];
    }
    int64_t cn = 0, ci = 0;
    // leaves of the parent's near list first (their ids precede every box of this level) ...
    for (int64_t j = near_ptr[P]; j < near_ptr[P + 1]; j++) {
        int64_t N = near_idx[j];
        if (!leaf[N] || ee[N] == eb[N]) continue;
        if (well_separated(centre, radius, b, N, sa)) {
            if (PASS == 1) out_inter[wi + ci] = (int32_t)N;
            ci++;
        } else {
            if (PASS == 1) out_near[wn + cn] = (int32_t)N;
            cn++;
        }
    }
    // ... then the children of its non-leaf entries, in ascending order
    for (int64_t j = near_ptr[P]; j < near_ptr[P + 1]; j++) {
        int64_t N = near_idx[j];
        if (leaf[N]) continue;
        for (int c = 0; c < nchild[N]; c++) {
            int64_t C = child_begin[N] + c;
            if (ee[C] == eb[C]) continue;
            if (well_separated(centre, radius, b, C, sa)) {
                if (PASS == 1) out_inter[wi + ci] = (int32_t)C;
                ci++;
            } else {
                if (PASS == 1) out_near[wn + cn] = (int32_t)C;
                cn++;
            }
        }
    }
    if (PASS == 0) {
        cnt_near[b - lo] = cn;
        cnt_inter[b - lo] = ci;
    }
}

__global__ void k_write_ptr(int64_t lo, int64_t hi, const int64_t *off, int64_t base, int64_t *ptr) {
    int64_t b = lo + (int64_t)blockIdx.x * BS + threadIdx.x;
    if (b <= hi) ptr[b] = base + off[b - lo];
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

// The literal tree's sources are the DOFs' basis functions, each over its
// element patch.  The product runs on element pieces: for every element and
// every leaf holding one of its DOFs, one piece with the element's points
// and the shape functions of those DOFs only (a slot mask).  Pieces are
// ordered by their first DOF's sorted position, so every box's pieces are
// the range between its DOF range's bounds; the tree's element fields then
// describe the pieces (eperm: the element of each piece).
void expand_literal_sources(bem_tree &t) {
    Ctx &c = *t.ctx;
    const bem_mesh &m = *t.mesh;
    const int na = m.linear ? 3 : 6;
    std::vector<int32_t> tperm = t.tperm.download(t.n_tgt);
    std::vector<int64_t> pos(t.n_tgt), leaf_of(t.n_tgt, -1);
    for (int64_t s = 0; s < t.n_tgt; s++) pos[tperm[s]] = s;
    for (int64_t b = 0; b < t.n_box; b++)
        if (t.h_leaf[b])
            for (int64_t s = t.h_tb[b]; s < t.h_te[b]; s++) leaf_of[s] = b;
    struct Piece {
        int64_t key;
        int32_t elem;
        uint8_t mask;
    };
    std::vector<Piece> pc;
    pc.reserve(2 * m.n_el);
    for (int64_t e = 0; e < m.n_el; e++) {
        uint8_t done = 0;
        for (int a = 0; a < na; a++) {
            if (done >> a & 1) continue;
            const int64_t lf = leaf_of[pos[m.h_elem_dofs[6 * e + a]]];
            Piece p{INT64_MAX, (int32_t)e, 0};
            for (int b = a; b < na; b++) {
                const int64_t sp = pos[m.h_elem_dofs[6 * e + b]];
                if (leaf_of[sp] != lf) continue;
                p.mask |= (uint8_t)(1u << b);
                p.key = std::min(p.key, sp);
            }
            done |= p.mask;
            pc.push_back(p);
        }
    }
    std::stable_sort(pc.begin(), pc.end(), [](const Piece &x, const Piece &y) { return x.key < y.key; });
    const int64_t np = (int64_t)pc.size();
    std::vector<int32_t> eperm(np);
    std::vector<uint8_t> mask(np);
    std::vector<int64_t> keys(np);
    for (int64_t i = 0; i < np; i++) {
        eperm[i] = pc[i].elem;
        mask[i] = pc[i].mask;
        keys[i] = pc[i].key;
    }
    for (int64_t b = 0; b < t.n_box; b++) {
        t.h_eb[b] = std::lower_bound(keys.begin(), keys.end(), t.h_tb[b]) - keys.begin();
        t.h_ee[b] = std::lower_bound(keys.begin(), keys.end(), t.h_te[b]) - keys.begin();
    }
    t.n_el = np;
    t.eperm.alloc(&c, std::max<int64_t>(1, np));
    t.eperm.upload(eperm.data(), np);
    t.se_mask.alloc(&c, std::max<int64_t>(1, np));
    t.se_mask.upload(mask.data(), np);
    t.eb.upload(t.h_eb.data(), t.n_box);
    t.ee.upload(t.h_ee.data(), t.n_box);
    c.sync();
}

void build_tree(bem_tree &t) {
    Ctx &c = *t.ctx;
    const bem_mesh &m = *t.mesh;
    // the literal tree keys its sources at the DOF points (eb/ee are then DOF
    // ranges until the sources are expanded into element pieces at the end)
    const int64_t n_el = t.literal ? m.n_dof : m.n_el, n_tgt = m.n_dof, n = n_el + n_tgt;
    t.n_el = n_el;
    t.n_tgt = n_tgt;

    // 1. root cube
    unsigned nbb = std::min<unsigned>(nblocks(m.n_nodes, BS), 256);
    DBuf<double> part, root;
    part.alloc(&c, 6 * nbb);
    root.alloc(&c, 8);
    k_bbox_partial<<<nbb, BS, 0, c.stream>>>(m.xyz.p, m.n_nodes, part.p);
    BEM_LAUNCH_CHECK();
    k_root<<<1, 64, 0, c.stream>>>(part.p, nbb, root.p);
    BEM_LAUNCH_CHECK();

    // 2-3. keys and the stable sort
    DBuf<uint64_t> key;
    DBuf<int32_t> val;
    key.alloc(&c, n);
    val.alloc(&c, n);
    k_keys<<<nblocks(n, BS), BS, 0, c.stream>>>(m.xyz.p, m.elem.p, n_el, m.dof_xyz.p, n_tgt, (int)t.literal, root.p,
                                                key.p, val.p);
    BEM_LAUNCH_CHECK();
    radix_sort_pairs(c, key.p, val.p, n, 63);

    DBuf<int64_t> flag, E;
    flag.alloc(&c, n);
    E.alloc(&c, n + 1);
    k_is_elem<<<nblocks(n, BS), BS, 0, c.stream>>>(val.p, n, n_el, flag.p);
    BEM_LAUNCH_CHECK();
    scan_exclusive<int64_t>(c, flag.p, E.p, n);
    t.eperm.alloc(&c, n_el);
    t.tperm.alloc(&c, n_tgt);
    k_perms<<<nblocks(n, BS), BS, 0, c.stream>>>(val.p, E.p, n, n_el, t.eperm.p, t.tperm.p);
    BEM_LAUNCH_CHECK();

    // 4. boxes, level by level
    DBuf<int32_t> active, item_box, head, hs;
    active.alloc(&c, n);
    item_box.alloc(&c, n);
    head.alloc(&c, n);
    hs.alloc(&c, n + 1);
    k_fill_i32<<<nblocks(n, BS), BS, 0, c.stream>>>(active.p, n, 1);
    BEM_LAUNCH_CHECK();
    DBuf<int64_t> first, last;
    first.alloc(&c, n);
    last.alloc(&c, n);
    size_t cap = (size_t)std::max<int64_t>(2 * n, 64);
    t.level.alloc(&c, cap);
    t.leaf.alloc(&c, cap);
    t.parent.alloc(&c, cap);
    t.eb.alloc(&c, cap);
    t.ee.alloc(&c, cap);
    t.tb.alloc(&c, cap);
    t.te.alloc(&c, cap);
    t.prefix.alloc(&c, cap);
    int64_t off = 0;
    t.level_off.assign(1, 0);
    for (int l = 0; l <= MAXLEV; l++) {
        k_heads<<<nblocks(n, BS), BS, 0, c.stream>>>(key.p, active.p, n, l, head.p);
        BEM_LAUNCH_CHECK();
        scan_exclusive<int32_t>(c, head.p, hs.p, n);
        int64_t nb = read_scalar(c, hs.p + n);
        if (nb == 0) break;
        if ((size_t)(off + nb) > cap) {
            size_t nc = std::max<size_t>(2 * cap, off + nb);
            t.level.grow(nc, off); t.leaf.grow(nc, off); t.parent.grow(nc, off);
            t.eb.grow(nc, off); t.ee.grow(nc, off); t.tb.grow(nc, off); t.te.grow(nc, off);
            t.prefix.grow(nc, off);
            cap = nc;
        }
        k_box_ranges<<<nblocks(n, BS), BS, 0, c.stream>>>(active.p, head.p, hs.p, n, first.p, last.p);
        BEM_LAUNCH_CHECK();
        k_box_fill<<<nblocks(nb, BS), BS, 0, c.stream>>>(key.p, E.p, first.p, last.p, item_box.p, nb, off, l, t.B,
                                                         t.max_depth, t.level.p, t.leaf.p, t.parent.p, t.eb.p, t.ee.p,
                                                         t.tb.p, t.te.p, t.prefix.p);
        BEM_LAUNCH_CHECK();
        k_update_items<<<nblocks(n, BS), BS, 0, c.stream>>>(head.p, hs.p, n, off, t.leaf.p, active.p, item_box.p);
        BEM_LAUNCH_CHECK();
        off += nb;
        t.level_off.push_back(off);
    }
    t.n_box = off;
    t.max_level = (int)t.level_off.size() - 2;

    // topology and centres
    t.child_begin.alloc(&c, t.n_box);
    t.nchild.alloc(&c, t.n_box);
    k_fill_i32<<<nblocks(t.n_box, BS), BS, 0, c.stream>>>(t.child_begin.p, t.n_box, -1);
    BEM_LAUNCH_CHECK();
    t.nchild.zero();
    if (t.n_box > 1) {
        k_children<<<nblocks(t.n_box - 1, BS), BS, 0, c.stream>>>(t.parent.p, t.n_box, t.child_begin.p, t.nchild.p);
        BEM_LAUNCH_CHECK();
    }
    t.centre.alloc(&c, 3 * t.n_box);
    t.radius.alloc(&c, t.n_box);
    k_centres<<<nblocks(t.n_box, BS), BS, 0, c.stream>>>(t.level.p, t.prefix.p, t.n_box, root.p, t.centre.p);
    BEM_LAUNCH_CHECK();

    // 5. radii: leaves, then parents bottom-up.  Attached radii (Section 3.6's
    // r_C over the elements attached to a leaf's vertices) need the elements
    // holding each node: CSR built on the host from the element slots that
    // can be targets (corners only for first-order meshes).
    DBuf<int64_t> node_ptr;
    DBuf<int32_t> node_elems;
    if (t.attach) {
        const int na = m.linear ? 3 : 6;
        std::vector<int64_t> np(m.n_nodes + 1, 0);
        for (int64_t i = 0; i < 6 * m.n_el; i++)
            if (i % 6 < na) np[m.h_elem[i] + 1]++;
        for (int64_t g = 0; g < m.n_nodes; g++) np[g + 1] += np[g];
        std::vector<int32_t> ne(np[m.n_nodes]);
        std::vector<int64_t> fill(np.begin(), np.end() - 1);
        for (int64_t i = 0; i < 6 * m.n_el; i++)
            if (i % 6 < na) ne[fill[m.h_elem[i]]++] = (int32_t)(i / 6);
        node_ptr.alloc(&c, np.size());
        node_ptr.upload(np.data(), np.size());
        node_elems.alloc(&c, std::max<size_t>(1, ne.size()));
        if (!ne.empty()) node_elems.upload(ne.data(), ne.size());
    }
    k_leaf_radius<<<nblocks(t.n_box, BS / 64), BS, 0, c.stream>>>(t.leaf.p, t.eb.p, t.ee.p, t.tb.p, t.te.p, t.centre.p,
                                                                  t.eperm.p, t.tperm.p, m.elem.p, m.xyz.p,
                                                                  m.dof_xyz.p, m.dof_node.p, node_ptr.p,
                                                                  node_elems.p, (int)!t.literal, t.n_box,
                                                                  t.radius.p);
    BEM_LAUNCH_CHECK();
    for (int l = t.max_level; l >= 0; l--) {
        int64_t lo = t.level_off[l], hi = t.level_off[l + 1];
        k_parent_radius<<<nblocks(hi - lo, BS), BS, 0, c.stream>>>(t.leaf.p, t.child_begin.p, t.nchild.p, t.level.p,
                                                                    lo, hi, root.p, t.radius.p);
        BEM_LAUNCH_CHECK();
    }

    // 6. lists, top-down
    SepArgs sa{t.theta, t.kappa, t.k_hint, (t.kappa > 0.0 && std::isfinite(t.kappa)) ? 1 : 0};
    t.near_ptr.alloc(&c, t.n_box + 1);
    t.inter_ptr.alloc(&c, t.n_box + 1);
    size_t ncap = (size_t)std::max<int64_t>(64, 32 * t.n_box), icap = ncap;
    t.near_idx.alloc(&c, ncap);
    t.inter_idx.alloc(&c, icap);
    {
        int64_t h_np[2] = {0, 1}, h_ip[2] = {0, 0};
        int32_t zero = 0;
        BEM_HIP(hipMemcpyAsync(t.near_ptr.p, h_np, sizeof h_np, hipMemcpyHostToDevice, c.stream));
        BEM_HIP(hipMemcpyAsync(t.inter_ptr.p, h_ip, sizeof h_ip, hipMemcpyHostToDevice, c.stream));
        BEM_HIP(hipMemcpyAsync(t.near_idx.p, &zero, sizeof zero, hipMemcpyHostToDevice, c.stream));
        c.sync();
    }
    int64_t tot_near = 1, tot_inter = 0;
    DBuf<int64_t> cn, ci, on, oi;
    for (int l = 1; l <= t.max_level; l++) {
        int64_t lo = t.level_off[l], hi = t.level_off[l + 1], nl = hi - lo;
        cn.alloc(&c, nl);
        ci.alloc(&c, nl);
        on.alloc(&c, nl + 1);
        oi.alloc(&c, nl + 1);
        k_lists<0><<<nblocks(nl, BS), BS, 0, c.stream>>>(lo, hi, t.parent.p, t.leaf.p, t.child_begin.p, t.nchild.p,
                                                         t.eb.p, t.ee.p, t.centre.p, t.radius.p, sa, t.near_ptr.p,
                                                         t.near_idx.p, cn.p, ci.p, nullptr, nullptr, 0, 0, nullptr,
                                                         nullptr);
        BEM_LAUNCH_CHECK();
        scan_exclusive<int64_t>(c, cn.p, on.p, nl);
        scan_exclusive<int64_t>(c, ci.p, oi.p, nl);
        int64_t add_n = read_scalar(c, on.p + nl), add_i = read_scalar(c, oi.p + nl);
        if ((size_t)(tot_near + add_n) > ncap) {
            size_t nc = std::max<size_t>(2 * ncap, tot_near + add_n);
            t.near_idx.grow(nc, tot_near);
            ncap = nc;
        }
        if ((size_t)(tot_inter + add_i) > icap) {
            size_t nc = std::max<size_t>(2 * icap, tot_inter + add_i);
            t.inter_idx.grow(nc, tot_inter);
            icap = nc;
        }
        k_lists<1><<<nblocks(nl, BS), BS, 0, c.stream>>>(lo, hi, t.parent.p, t.leaf.p, t.child_begin.p, t.nchild.p,
                                                         t.eb.p, t.ee.p, t.centre.p, t.radius.p, sa, t.near_ptr.p,
                                                         t.near_idx.p, nullptr, nullptr, on.p, oi.p, tot_near,
                                                         tot_inter, t.near_idx.p, t.inter_idx.p);
        BEM_LAUNCH_CHECK();
        k_write_ptr<<<nblocks(nl + 1, BS), BS, 0, c.stream>>>(lo, hi, on.p, tot_near, t.near_ptr.p);
        BEM_LAUNCH_CHECK();
        k_write_ptr<<<nblocks(nl + 1, BS), BS, 0, c.stream>>>(lo, hi, oi.p, tot_inter, t.inter_ptr.p);
        BEM_LAUNCH_CHECK();
        tot_near += add_n;
        tot_inter += add_i;
    }
    t.n_near = tot_near;
    t.n_inter = tot_inter;
    std::vector<double> hroot(8);
    {
        auto r = root.download(5);
        for (int d = 0; d < 3; d++) t.corner[d] = r[d];
        t.side = r[3];
    }

    // host copies used to plan the passes
    t.h_level = t.level.download(t.n_box);
    t.h_leaf = t.leaf.download(t.n_box);
    t.h_parent = t.parent.download(t.n_box);
    t.h_nchild = t.nchild.download(t.n_box);
    t.h_eb = t.eb.download(t.n_box);
    t.h_ee = t.ee.download(t.n_box);
    t.h_tb = t.tb.download(t.n_box);
    t.h_te = t.te.download(t.n_box);
    t.h_near_ptr = t.near_ptr.download(t.n_box + 1);
    t.h_inter_ptr = t.inter_ptr.download(t.n_box + 1);
    t.h_near_idx = t.near_idx.download(t.n_near);
    t.h_inter_idx = t.inter_idx.download(t.n_inter);
    t.n_leaf = 0;
    for (int64_t b = 0; b < t.n_box; b++) t.n_leaf += t.h_leaf[b];
    if (t.literal) expand_literal_sources(t);
}

}  // namespace bem
