// Library-internal objects (mesh, tree, per-Green caches) and the host-side
// launchers each translation unit provides.
#pragma once

#include <memory>

#include "common.h"

// Opaque handles of the C interface.
struct bem_ctx {
    bem::Ctx c;
};

struct bem_mesh {
    bem::Ctx *ctx = nullptr;
    int64_t n_nodes = 0, n_el = 0, n_dof = 0;
    // first-order (3-node flat) elements, carried as 6-node elements whose
    // mid-side nodes are appended edge midpoints (see load_mesh_host)
    bool linear = false;
    std::vector<double> h_xyz, h_dof_normal;
    std::vector<int32_t> h_elem, h_elem_dofs, h_dof_node;
    bem::DBuf<double> xyz;        // [n_nodes][3]
    bem::DBuf<int32_t> elem;      // [n_el][6]
    bem::DBuf<int32_t> elem_dofs; // [n_el][6]
    bem::DBuf<int32_t> dof_node;  // [n_dof]
    bem::DBuf<double> dof_xyz;    // [n_dof][3]
    // Free terms computed by trees of this mesh, one per tree hierarchy (leaf
    // size, depth, tree kind).  Trees of one hierarchy find the same
    // correction pairs in the same order and sum them the same way, so a
    // later tree copies the stored one instead of repeating the all-points
    // sum: the copy is bitwise what it would compute.  A cache (the mesh's
    // geometry does not change), filled and read by the trees.
    struct FreeTerm {
        int B = 0, max_depth = 0;
        bool attach = false, literal = false;
        bem::DBuf<double> c;  // [n_dof], DOF order
    };
    mutable std::vector<std::unique_ptr<FreeTerm>> free_terms;
};

namespace bem {

// Singular / near-singular corrections for one (Green, k), on the tree's pair list.
struct Corr {
    int green = -1;
    double k = 0.0;
    uint64_t last_use = 0;  // tree's use counter at the last lookup (least recently used goes first)
    DBuf<double> S, K;  // [n_pairs][6] (x2 interleaved when complex): accurate - 7-point
};

// Interaction slots whose multipole-to-local results are held at once (a slab
// of target boxes), unless the tree's options set another bound: 2^20 slots
// of 176 complex FP64 values are 2.9 GB.
constexpr int64_t M2L_SLAB_SLOTS = (int64_t)1 << 20;

// Helmholtz wavenumbers whose corrections and M2L plans a tree keeps at once;
// looking up another one drops the least recently used (Laplace ones stay).
constexpr int MAX_K_CACHED = 3;

// Drops the least recently used Helmholtz entry of `v` (entries with fields
// green and last_use) while it holds MAX_K_CACHED or more of them.
template <class T>
void evict_wavenumbers(std::vector<std::unique_ptr<T>> &v) {
    for (;;) {
        int n = 0;
        size_t lru = v.size();
        for (size_t i = 0; i < v.size(); i++) {
            if (v[i]->green != BEM_HELMHOLTZ) continue;
            n++;
            if (lru == v.size() || v[i]->last_use < v[lru]->last_use) lru = i;
        }
        if (n < MAX_K_CACHED) return;
        v.erase(v.begin() + (std::ptrdiff_t)lru);
    }
}

// Expansion operator tables for one order p.
struct FmmTables {
    int p = -1, P = 0, P2 = 0;
    DBuf<int8_t> exps;        // [P2][3]
    DBuf<int32_t> m2m_ptr;    // [P+1] terms of each target coefficient
    DBuf<int16_t> m2m_src;    // [nnz] source coefficient
    DBuf<double> m2m_c64;     // [8][nnz] per child octant
    DBuf<float> m2m_c32;
    DBuf<int32_t> l2l_ptr;
    DBuf<int16_t> l2l_src;
    DBuf<double> l2l_c64;
    DBuf<float> l2l_c32;
    std::vector<int8_t> h_exps;
    DBuf<double> inv_fact64;  // [P2] 1 / alpha!
    DBuf<float> inv_fact32;
    int nnz_m2m = 0, nnz_l2l = 0;
};

// Tasks of one wave each over the pairs of an M2L plan, for one column width;
// the tasks of slab s are [slab_task0[s], slab_task0[s + 1]).
struct M2lTasks {
    int cols = 0;
    int64_t n_task = 0;
    std::vector<int64_t> slab_task0;
    DBuf<int32_t> task_class, task_first, task_count;
    // level-dependent order only: contraction steps of 4 and row tiles of 16
    // that cover the largest source and target orders of each task's pairs
    DBuf<int32_t> task_kt, task_mt;
};

// Canonical displacement classes of the interaction pairs for one (Green, k),
// their derivative tables and expanded operators (multipole-to-local
// translation on the matrix cores).
struct M2lPlan {
    int green = -1;
    double k = 0.0;
    uint64_t last_use = 0;
    int64_t n_class = 0, n_pairs = 0;
    DBuf<double> D64;                 // [n_class][P2] (x2 interleaved when complex), canonical separations
    DBuf<int32_t> cls_delta;          // level difference of the class
    DBuf<int32_t> pair_slot;          // interaction-list slot of each pair, grouped by class
    DBuf<int32_t> pair_src;           // source box of each pair
    DBuf<int32_t> pair_mom;           // canonical moment vector (source box, symmetry) of each pair
    int64_t n_u = 0;                  // used (source box, symmetry) combinations
    DBuf<int32_t> u_src, u_sym;
    // Pairs grouped by slab (a run of target boxes whose interaction slots
    // fit M2L_SLAB_SLOTS, so that the per-pair results of one slab at a time
    // bound the work space), then by class, largest first: group i is class
    // h_class_order[i] of slab h_group_slab[i], pairs [first, first + count)
    std::vector<int32_t> h_class_order, h_class_first, h_class_count, h_group_slab;
    // slab s: interaction slots [slab_slot0[s], slab_slot0[s + 1]) and target
    // boxes m2l_boxes[slab_box0[s] .. slab_box0[s + 1])
    std::vector<int64_t> slab_slot0, slab_box0;
    int64_t slab_max_slots = 0;
    bool var = false;                 // level-dependent order: per-pair steps and row tiles below
    std::vector<int32_t> h_pair_kt, h_pair_mt;
    std::vector<std::unique_ptr<M2lTasks>> tasks;
    DBuf<int32_t> pk;                 // packed multi-indices of the contraction rows
    DBuf<int32_t> sym_in;             // symmetry tables: moments into the canonical frame,
    DBuf<int16_t> sym_red;            // results back to the pair's frame
    DBuf<int32_t> slot_sym;           // symmetry of each interaction-list slot
    DBuf<float> T32;                  // expanded operators, built on first use per precision
    DBuf<double> T64;
    DBuf<uint16_t> T2;                // two-term fp16 splits of the scaled operators (mixed path with one order)
    DBuf<float> cls_scale;            // [class] power-of-two scale of each split operator
    DBuf<uint8_t> sym_perm;           // [7][OUT_LD] compact symmetry table of the split kernel
    std::vector<int32_t> h_pair_slot, h_pair_sym;
    // Mixed path with one order: partial slots of the per-target sums the
    // product kernel forms itself (built on first use for `parts_g` pairs
    // per pass): pair -> partial slot, the pairs' symmetries, and the slots
    // of each M2L target box (m2l_boxes order), contiguous, box by box.
    int parts_g = 0;
    int64_t parts_max = 0;            // largest number of partial slots of one slab
    DBuf<int32_t> pair_part, pair_sym;
    DBuf<int64_t> part_ptr;           // [n_m2l_boxes + 1]
    std::vector<int64_t> h_part_ptr;
    template <class R>
    DBuf<R> &expanded_buf();
};
template <>
inline DBuf<float> &M2lPlan::expanded_buf<float>() { return T32; }
template <>
inline DBuf<double> &M2lPlan::expanded_buf<double>() { return T64; }

// Stored P2M weights (per source leaf and DOF, single and double layer);
// geometry only, built once per tree.
struct PassTables {
    bool built = false;
    int64_t n_w = 0;
    DBuf<int64_t> woff;   // [n_leaf_src + 1]
    DBuf<int32_t> wdof;   // [n_w] DOF of each weight row
    DBuf<double> W64[2];  // [n_w][P], index 0 single layer, 1 double layer
    DBuf<float> W32[2];
};

// Number of expansion coefficients of the boxes of each level (Section 3.6:
// the order may fall towards the leaves); passed to kernels by value.
struct LevelP {
    int32_t P[MAXLEV + 1];
};

// Launch choices of the fast product that change its speed but not its
// arithmetic (every sum runs over the same terms in the same order whatever
// they are): the near field's blocks per CU while it runs beside the far
// field (0: as many as fit) and the waves per M2L block.  The autotuner times
// candidates on the first product of each shape class and keeps the fastest
// (one table per process, shared by all contexts and trees).
struct LaunchChoice {
    int p2p_per_cu = 4;
    int m2l_waves = 4;
    bool m2l_room = false;  // the near field's blocks leave LDS for one M2L block per CU
};

// Per-matvec work buffers, grown on demand and kept on the tree.
struct Work {
    DBuf<char> strength, mom, loc, yacc, m2l_out, m2l_mom, p2p_part;
};

// Device work space of `bytes` for one product: the next 256-byte aligned
// piece of the context's arena when one is set (nothing is allocated; a
// product that does not fit fails with BEM_EINVAL), else the tree's buffer
// `buf`, grown on demand.
inline void *work_buf(Ctx &c, DBuf<char> &buf, size_t bytes) {
    if (c.arena) {
        const size_t at = (c.arena_used + 255) & ~(size_t)255;
        BEM_REQUIRE(at + bytes <= c.arena_size, BEM_EINVAL,
                    "the product needs more work space than the no-allocation scratch holds (" +
                        std::to_string(at + bytes) + " > " + std::to_string(c.arena_size) + " bytes)");
        c.arena_used = at + bytes;
        return c.arena + at;
    }
    buf.ensure(&c, bytes);
    return buf.p;
}

}  // namespace bem

struct bem_tree {
    bem::Ctx *ctx = nullptr;
    const bem_mesh *mesh = nullptr;
    int B = 32, order = 8, max_depth = 21;
    int order_min = 0;  // level-dependent order when > 0 (see level_p)
    bool attach = false;  // leaf radii over the elements attached to the leaf's target nodes
    bool literal = false; // the paper's tree read literally: DOF sources, B counting DOFs (attach too)
    double theta = 0.5, kappa = 0.0, k_hint = 0.0;
    int64_t m2l_slab = bem::M2L_SLAB_SLOTS;  // interaction slots whose M2L results are held at once
    int64_t n_box = 0, n_leaf = 0, n_near = 0, n_inter = 0, n_el = 0, n_tgt = 0, n_q = 0;
    int max_level = 0;
    double corner[3] = {0, 0, 0}, side = 0;
    std::vector<int64_t> level_off;  // [max_level + 2]

    // boxes, canonical (level, prefix) order
    bem::DBuf<int32_t> level, leaf, parent, child_begin, nchild;
    bem::DBuf<int64_t> eb, ee, tb, te;
    bem::DBuf<uint64_t> prefix;
    bem::DBuf<double> centre, radius;  // [n_box][3], [n_box]
    bem::DBuf<int32_t> eperm, tperm;   // sorted position -> element / DOF
    bem::DBuf<uint8_t> se_mask;        // literal tree: shape-function slots of each element piece (else empty)
    bem::DBuf<int64_t> near_ptr, inter_ptr;
    bem::DBuf<int32_t> near_idx, inter_idx;

    // geometry in sorted element order (Section 2.2 with the 7-point rule)
    bem::DBuf<int32_t> se_dofs;  // [n_el][6]
    bem::DBuf<int32_t> se_nodes; // [n_el][6]
    bem::DBuf<double> q64;       // SoA [7][n_q]: x y z wJ nx ny nz
    bem::DBuf<float> q32;
    bem::DBuf<double> t64;       // SoA [3][n_tgt] sorted targets
    bem::DBuf<float> t32;
    bem::DBuf<double> L7;        // [7][6] shape functions at the rule points

    // host copies for planning
    std::vector<int32_t> h_level, h_leaf, h_parent, h_nchild;
    std::vector<int64_t> h_tb, h_te, h_eb, h_ee, h_near_ptr, h_inter_ptr;
    std::vector<int32_t> h_near_idx, h_inter_idx;

    // P2P work items: (target leaf, first sorted target, count <= 64)
    bem::DBuf<int32_t> p2p_box, p2p_t0, p2p_nt;
    int64_t n_p2p_items = 0, n_p2p_pairs = 0;
    // P2P work units: shares of an item's near points (item, [f0, f1)), and
    // the units of each item ([item_unit[i], item_unit[i + 1]))
    int64_t n_p2p_units = 0;
    bem::DBuf<int32_t> p2p_unit_order, p2p_unit_item, p2p_item_unit;
    bem::DBuf<int32_t> p2p_tgt_item;  // item of each sorted target
    bem::DBuf<int64_t> p2p_unit_f;
    bem::DBuf<int32_t> leaf_ids;       // leaf boxes with elements (P2M)
    int64_t n_leaf_src = 0;
    bem::DBuf<int32_t> tleaf_ids;      // leaf boxes with targets (L2P)
    int64_t n_leaf_tgt = 0;
    bem::DBuf<int32_t> tgt_leaf;       // [n_tgt][4]: leaf box, its first target, its target count, 0
    bem::DBuf<int32_t> m2l_boxes;      // boxes with a non-empty interaction list and targets below
    int64_t n_m2l_boxes = 0;
    std::vector<std::vector<int32_t>> m2m_level_boxes;  // non-leaf boxes per level
    std::vector<bem::DBuf<int32_t>> d_m2m_level_boxes;
    std::vector<bem::DBuf<int32_t>> d_level_boxes;      // boxes with targets per level
    std::vector<std::vector<int32_t>> l2l_level_boxes;  // non-leaf boxes with targets per level
    std::vector<bem::DBuf<int32_t>> d_l2l_level_boxes;
    bem::PassTables pass;
    // coarsest level whose moments are read (as an interaction source, directly
    // or through a coarser source) and coarsest level holding a non-zero local
    // expansion: M2M stops at the first, L2L starts at the second
    int m2m_top = 0, l2l_top = 0;

    // (target, element) pairs needing the singular / near-singular rules: CSR by sorted target
    bool has_pairs = false;
    int64_t n_pairs = 0;
    bem::DBuf<int64_t> pair_ptr;   // [n_tgt + 1]
    bem::DBuf<int32_t> pair_elem;  // sorted element index
    bem::DBuf<int32_t> pair_info;  // class (1 near, 2 singular) | param << 4
    bem::DBuf<int32_t> pair_row;   // sorted target index
    bool planned = false;
    std::vector<int64_t> h_level_down;

    std::vector<std::unique_ptr<bem::Corr>> corr;
    std::vector<std::unique_ptr<bem::M2lPlan>> m2l;
    uint64_t k_uses = 0;  // lookups of corr / m2l (orders their least recent use)
    std::vector<uint64_t> h_prefix;
    bem::DBuf<double> free_term;  // [n_dof], DOF order
    bool has_free_term = false;
    std::unique_ptr<bem::FmmTables> tables;
    bem::Work work;
};

namespace bem {

// scan_sort.hip
template <class T>
void scan_exclusive(Ctx &c, const T *in, T *out, int64_t n);  // out has n + 1 entries
void radix_sort_pairs(Ctx &c, uint64_t *keys, int32_t *vals, int64_t n, int key_bits);

// mesh.cpp (host)
void index_dofs(bem_mesh &m, double tol_deg);
// host arrays of a mesh from nn-node elements (nn = 6 or 3) and its DOF indexing
void load_mesh_host(bem_mesh &m, const double *xyz, int64_t n_nodes, const int32_t *elem, int64_t n_el, int nn,
                    double tol_deg);

// tree.hip
void build_tree(bem_tree &t);

// geom.hip
void build_geometry(bem_tree &t);
void rule7(double s[7], double t[7], double w[7]);

// quad.hip
void build_pairs(bem_tree &t);
Corr &get_corr(bem_tree &t, int green, double k);
void build_free_term(bem_tree &t);

// fmm.hip
void direct_regular_unit_double_layer(bem_tree &t, double *out);
void rule_shapes(bem_tree &t);  // t.L7: the six shape functions at the 7 rule points
void fmm_tables(bem_tree &t);
void plan_fmm(bem_tree &t);
LevelP level_p(const bem_tree &t);  // coefficients per level: min(order, order_min + max_level - l)
void matvec(bem_tree &t, int green, double k, int op, int method, int prec, int nrhs, const void *x, void *y);
// whether every table such a product reads exists already (an earlier
// product with the same arguments built them), so that it allocates nothing
// beyond its work space
bool product_ready(const bem_tree &t, int green, double k, int op, int method, int prec);
// the launch choice of a fast product of this tree (tuned or default), and
// the number of shape classes tuned so far in this process
LaunchChoice launch_choice(const bem_tree &t, int green, int prec, int op, bool *tuned);
int64_t tuned_classes();
void forget_tuned_classes();

// passes.hip
void build_pass_tables(bem_tree &t);
template <class V, class R, class XV>
void p2m_apply(bem_tree &t, bool dbl, int nrhs, const XV *x, V *mom);
template <class V, class R>
void m2m_apply(bem_tree &t, int nrhs, V *mom, int top = -1);  // levels down to top (default: m2m_top)
template <class V, class R>
void l2l_apply(bem_tree &t, int nrhs, V *loc);

// m2l.hip
M2lPlan &get_m2l_plan(bem_tree &t, int green, double k);
template <class V, class R>
void m2l_prepare(bem_tree &t, M2lPlan &pl, int waves);
bool m2l_ready(const M2lPlan &pl, int prec, int waves);
// LDS of one block of the M2L product kernel a product of precision prec
// with `waves` waves per block launches on this plan
size_t m2l_block_lds(const M2lPlan &pl, int prec, int waves);  // operators and tasks of precision prec exist
template <class V, class R>
void m2l_apply(bem_tree &t, M2lPlan &pl, int nrhs, const V *mom, V *loc, int waves);

// field.hip
void field(bem_tree &t, int green, double k, double theta, int nrhs, const void *phi, const void *chi, int64_t n_pts,
           const double *pts, void *u);

// solve.hip
int solve(bem_tree &t, int green, double k, int nrhs, const void *chi, void *phi, const bem_solve_opts &o,
          bem_solve_info *info);

}  // namespace bem
