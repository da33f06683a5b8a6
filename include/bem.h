/*
 * bem.h - C interface of the MI355X (gfx950) fast-multipole boundary element
 * library for the collocation Laplace and Helmholtz integral equations over
 * curved 6-node triangles (M. J. Carley, "BEM3D: a free adaptive fast
 * multipole boundary element library", arXiv 0908.0673).
 *
 * Problem statement (Section 2.1, Eqs. 1-3).  A closed surface S with unit
 * normal n pointing out of the body into the unbounded domain, Green's
 * function G = 1/(4 pi R) (Laplace) or G = e^{jkR}/(4 pi R) (Helmholtz).  For
 * every collocation point (DOF) i the library discretises
 *
 *     c_i phi_i - sum_j K_ij phi_j = - sum_j S_ij chi_j               (1)
 *
 *     S_ij = sum_{m owns j} int_{S_m} L_j G dS,
 *     K_ij = sum_{m owns j} PV int_{S_m} L_j dG/dn_1 dS,
 *     c_i  = 1 + sum_j K0_ij   (K0: K with the Laplace kernel, Eq. 2),
 *
 * with chi = dphi/dn the prescribed Neumann data.  The fast product is the
 * adaptive Taylor-series multipole method of Sections 3.1-3.6.
 *
 * Conventions shared by every entry point:
 *  - All functions return a bem_status; 0 is success.  A failing call leaves
 *    its output handles NULL and records a message for bem_last_error().  No
 *    function aborts the process or throws across this interface.
 *  - "host" pointers are read (or written) during the call only.  "device"
 *    pointers are caller-owned device memory on the context's device; the
 *    library never frees them.
 *  - Device vectors hold nrhs right-hand sides as [nrhs][n_dof]: float64 for
 *    Laplace, interleaved complex128 (re, im) for Helmholtz.
 *  - All device work is ordered on the context's stream (bem_matvec may
 *    also use a second internal stream of the context, joined back into the
 *    context's stream before it returns).  bem_matvec returns once its work
 *    is enqueued (stream-ordered, like a kernel launch; the first call for a
 *    (g, k) also waits for its set-up); every other call returns when its
 *    work has completed.  A context is not thread-safe.
 */
#ifndef BEM_H
#define BEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BEM_OK = 0,
    BEM_EINVAL = -1,        /* bad argument or mesh */
    BEM_ENOMEM = -2,        /* device or host allocation failed */
    BEM_EDEVICE = -3,       /* a HIP runtime call failed */
    BEM_ENOCONV = -4,       /* the solver hit its iteration cap (outputs still written) */
    BEM_ESTATE = -5,        /* handle misuse (wrong context, freed object) */
    BEM_EUNSUPPORTED = -6,  /* valid request the library does not implement (e.g. order > 8) */
    BEM_EAGAIN = -7         /* (serving) the request has not completed yet */
} bem_status;

typedef enum { BEM_LAPLACE = 0, BEM_HELMHOLTZ = 1 } bem_green;

/* Operators of Eq. (1): S x, K x, the system operator A x = c.x - K x, and
 * the right-hand side b = -S chi. */
typedef enum { BEM_OP_S = 0, BEM_OP_K = 1, BEM_OP_A = 2, BEM_OP_RHS = 3 } bem_op;

/* BEM_DIRECT: every (target, element) pair summed directly with the same
 * quadrature (the paper's baseline, Section 2.1).  BEM_FMM: Section 3.6. */
typedef enum { BEM_DIRECT = 0, BEM_FMM = 1 } bem_method;

/* BEM_PREC_FP64: every step in double precision.  BEM_PREC_MIXED: regular
 * near-field sums and all expansion passes in single precision with single
 * accumulation; the singular / near-singular corrections, the free term and
 * the combination stay double. */
typedef enum { BEM_PREC_FP64 = 0, BEM_PREC_MIXED = 1 } bem_precision;

/* Krylov method of bem_solve.  BEM_KRYLOV_GMRES: restarted GMRES with
 * classical Gram-Schmidt applied twice.  BEM_KRYLOV_BICGSTAB: BiCGSTAB, the
 * paper's solver (Section 2.1), two products per step. */
typedef enum { BEM_KRYLOV_GMRES = 0, BEM_KRYLOV_BICGSTAB = 1 } bem_krylov;

/* Device memory provider.  alloc returns device memory of at least `bytes`
 * usable on `stream` (NULL on failure); free releases it.  Passing NULL for
 * the allocator makes the library use hipMalloc / hipFree. */
typedef struct {
    void *(*alloc)(void *user, size_t bytes, void *stream);
    void (*free)(void *user, void *ptr, void *stream);
    void *user;
} bem_allocator;

typedef struct bem_ctx bem_ctx;
typedef struct bem_mesh bem_mesh;
typedef struct bem_tree bem_tree;

/* Creates a context on HIP device `device` whose work goes to `hip_stream`
 * (a hipStream_t; NULL = the default stream).  The stream and the allocator's
 * user data must outlive the context. */
int bem_ctx_create(int device, void *hip_stream, const bem_allocator *alloc, bem_ctx **out);
void bem_ctx_destroy(bem_ctx *ctx);
/* Message of the last failing call on this context (never NULL). */
const char *bem_last_error(const bem_ctx *ctx);

/* Phase timing (profiling aid).  While enabled, every product records HIP
 * events on the context's stream between its phases and accumulates the
 * elapsed device time per phase:
 *   0 strengths, 1 P2M, 2 M2M, 3 M2L products, 4 L2L, 5 L2P (no longer a
 *   kernel of its own: the local expansions are evaluated inside phase 7),
 *   6 P2P (near field), 7 corrections, L2P + combination, 8 direct sum,
 *   9 other, 10 the M2L
 *   gathers around the products (moments into the canonical frames, results
 *   summed into the local expansions).
 * While timing is enabled every phase runs on the context's stream; without
 * it the near field runs concurrently with the far field on a second
 * stream, so the per-phase times are those of the serialized product.
 * enable = 1 turns phase timing on and zeroes the counters; 2 instead times
 * only the two heavy kernels (the M2L products as phase 3 and the near field
 * as phase 6, each with events on the stream it runs on) and leaves the
 * scheduling of the product unchanged; 3 and 4 do the same for the near
 * field only and for the M2L products only (one event pair per product);
 * 0 turns timing off.  Other values give BEM_EINVAL.
 * Products do not wait for their events: each call of bem_ctx_timing first
 * synchronises the context's stream and reads back the events recorded
 * since the previous call.  ms and launches (host arrays of BEM_NPHASE, may
 * be NULL) then receive the accumulated milliseconds and the number of
 * products timed per phase. */
#define BEM_NPHASE 11
int bem_ctx_timing(bem_ctx *ctx, int enable, double *ms, int64_t *launches);

/* Autotuning of the fast product's launch choices (tile shapes that change
 * its speed but not its results, bit for bit: the near field's blocks per CU
 * while the far field runs beside it, the waves per multipole-to-local
 * block).  With enable = 1 (the default) the first product of a shape class
 * (Green's function, precision, layer, and the near-field pair and
 * interaction counts on a grid of factors sqrt(2)) times the candidates on
 * its own input and keeps the fastest in a table of the process shared by
 * all contexts; enable = 0 uses the tuned choice where one exists and the
 * defaults otherwise, without tuning; enable = 2 empties the process's table
 * (every shape class is tuned again) and turns tuning on.  *classes (may be
 * NULL) receives the number of shape classes tuned so far.  BEM_EINVAL for
 * other values. */
int bem_ctx_autotune(bem_ctx *ctx, int enable, int64_t *classes);

/* Device bytes the library holds through this context for meshes, trees and
 * work buffers (live), and the largest such figure since the context was
 * created or since the last call with reset_peak = 1 (peak: the memory a
 * setup and solve needed, the counterpart of the paper's memory columns).
 * Freed blocks kept for reuse are not counted.  Either pointer may be NULL. */
int bem_ctx_device_bytes(bem_ctx *ctx, int reset_peak, int64_t *live, int64_t *peak);

/* ------------------------------------------------------------------ mesh */
typedef struct {
    double edge_angle_deg; /* normals closer than this share a DOF (Section 2.3); 0 -> 30 */
    int nodes_per_elem;    /* 6 (second-order curved triangles) or 3 (first-order flat
                              triangles, unknowns linear over each); 0 -> 6 */
} bem_mesh_opts;

/* Loads a mesh of 6-node or 3-node triangles (Section 2.2).
 *   node_xyz   host [n_nodes][3] float64 node coordinates
 *   elem_nodes host [n_elem][6] int32: corners 0,1,2 counter-clockwise seen
 *              from outside the body, then the mid-side nodes of edges 0-1,
 *              1-2 and 2-0 (isoparametric: geometry and data share nodes);
 *              with opts->nodes_per_elem = 3, [n_elem][3]: the corners of
 *              flat triangles, the data linear over each
 * Collocation points are the nodes.  Nodes where the element normals differ
 * by more than opts->edge_angle_deg get one DOF per group of normals (sharp
 * edges and corners, Section 2.3); elements are visited in order and each
 * group's reference normal is that of its first element.
 * Errors: BEM_EINVAL for n_elem < 1, node indices out of range, or an element
 * with a vanishing Jacobian at a node. */
int bem_mesh_load(bem_ctx *ctx, const double *node_xyz, int64_t n_nodes, const int32_t *elem_nodes,
                  int64_t n_elem, const bem_mesh_opts *opts, bem_mesh **out);

/* Copies the DOF layout to host buffers (each may be NULL):
 *   elem_dofs [n_elem][nodes_per_elem] int32, dof_node [n_dof] int32 (geometric node of a
 *   DOF), dof_xyz [n_dof][3], dof_normal [n_dof][3] (normalised mean of the
 *   element normals of the DOF's group). */
int bem_mesh_dofs(const bem_mesh *mesh, int64_t *n_dof, int32_t *elem_dofs, int32_t *dof_node,
                  double *dof_xyz, double *dof_normal);
void bem_mesh_free(bem_mesh *mesh);

/* ------------------------------------------------------------------ tree */
typedef struct {
    int max_elems_per_leaf; /* B: a box holding more elements is split (Section 3.1); 0 -> 32 */
    int order;              /* Taylor order p of moments and local expansions; 0 -> 8, max 8 */
    double theta;           /* boxes are well separated iff |c1 - c2| > (r1 + r2)/theta (Eq. 14 has
                               theta = 1); 0 -> 0.5 */
    double kappa;           /* Helmholtz only: also require k (r1 + r2) <= kappa; 0 or inf -> none */
    int max_depth;          /* deepest level, <= 21; 0 -> 21 */
    double k_hint;          /* wavenumber the kappa rule uses when building the lists */
    int order_min;          /* L_min of the level-dependent order (Section 3.6): boxes at level l
                               use order min(order, order_min + l_max - l), l_max the deepest
                               level; 0 (or >= order) -> `order` at every level */
    int attach_radii;       /* 1: a leaf's convergence radius also covers every node of every
                               element attached to the geometric nodes of its targets (the
                               paper's r_C, Section 3.6, over the elements attached to a leaf's
                               vertices, Section 3.1); sources stay owned by one leaf each.
                               2: the paper's tree read literally: boxes over the DOF points
                               alone, max_elems_per_leaf then counting DOFs, every DOF's basis
                               function a source over its element patch, radii as for 1; the
                               element fields of bem_tree_export then describe element pieces
                               (the part of an element in one leaf's basis functions).
                               0: owned elements and targets only */
    int m2l_slab_slots;     /* interaction-list slots whose multipole-to-local results a product
                               holds at once: the translations run slab by slab over runs of
                               target boxes, which bounds the product's work space (176 values
                               per slot); 0 -> 2^20 */
} bem_tree_opts;

/* Builds the octree over the mesh on the device (Section 3.1): element keys
 * are the means of the corner nodes, targets are the DOF positions, both
 * Morton-coded on 21 bits per axis inside a padded root cube and radix
 * sorted; then convergence radii (Section 3.4, Eq. 13) and the near-field
 * and interaction lists (Section 3.6, Eq. 14), level by level.  The tree
 * borrows the mesh: free the tree first. */
int bem_tree_build(bem_ctx *ctx, const bem_mesh *mesh, const bem_tree_opts *opts, bem_tree **out);

/* Host view of a built tree.  Call once with the pointer fields NULL to get
 * the sizes, then again with buffers of those sizes (any may stay NULL). */
typedef struct {
    int64_t n_box, n_elem, n_target, n_near, n_inter, n_leaf;
    int32_t max_level;
    double root[4]; /* corner x, y, z and side of the root cube */
    int32_t *level, *leaf, *parent, *child_begin, *nchild;         /* [n_box] */
    int64_t *elem_begin, *elem_end, *tgt_begin, *tgt_end;            /* [n_box], sorted orders */
    uint64_t *prefix;                                                 /* [n_box] Morton prefix */
    double *centre;                                                   /* [n_box][3] */
    double *radius;                                                   /* [n_box] */
    int32_t *elem_perm, *tgt_perm;                                    /* sorted position -> id */
    int64_t *near_ptr, *inter_ptr;                                    /* [n_box + 1] */
    int32_t *near_idx, *inter_idx;                                    /* [n_near], [n_inter] */
} bem_tree_view;

int bem_tree_export(const bem_tree *tree, bem_tree_view *view);
void bem_tree_free(bem_tree *tree);

/* Work statistics of a tree for a (Green, k): M2L pairs, near-field pair
 * count of target DOFs x source quadrature points, correction entries.  */
typedef struct {
    int64_t n_m2l, n_m2l_same_level, n_p2p, n_corr_pairs, n_leaf, n_box;
    int64_t n_quad;
} bem_tree_stats;
int bem_tree_stats_get(bem_ctx *ctx, const bem_tree *tree, bem_green g, double k, bem_tree_stats *st);

/* ------------------------------------------------------------------ products */
/* y = op(x) for nrhs vectors (layout above).  x_dev and y_dev are device
 * buffers of nrhs * n_dof values and must not overlap.  The first call for a
 * given (g, k) builds and caches the singular / near-singular corrections
 * and the free term on the tree (Section 2.1; Section 3.6, "precomputed and
 * stored as a sparse matrix").
 * Errors: BEM_EINVAL for nrhs < 1, k <= 0 with Helmholtz, NULL buffers, and
 * for a Helmholtz k that the tree's lists do not cover: a tree built with the
 * wavenumber bound (kappa > 0) holds its error bound only for k <= k_hint, so
 * such a tree rejects Helmholtz products with k > k_hint (and every
 * Helmholtz product when k_hint = 0). */
int bem_matvec(bem_ctx *ctx, const bem_tree *tree, bem_green g, double k, bem_op op, bem_method m,
               bem_precision p, int nrhs, const void *x_dev, void *y_dev);

/* bem_matvec without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, stream ordering and results (bit
 * for bit) as bem_matvec.  The product's work space (strengths, expansions,
 * near-field partial sums, multipole-to-local buffers) comes from one fixed
 * array of BEM_NOALLOC_SCRATCH_BYTES per device, which the library holds from
 * the moment its code is loaded on the device until the process ends; the
 * call makes no hipMalloc / hipFree and no allocator callback.  All calls on
 * one device share that array and it keeps the last call's contents: calls
 * that overlap on one GPU (other contexts, streams or threads) race, so
 * callers serialise them.
 * Errors: those of bem_matvec; BEM_ESTATE while the tree's tables for this
 * (g, k, op, m, p) are not built (one bem_matvec call with the same
 * arguments builds them) or while phase timing is on; BEM_EINVAL when the
 * product needs more work space than the array holds (the message gives
 * both sizes). */
#define BEM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int bem_matvec_noalloc(bem_ctx *ctx, const bem_tree *tree, bem_green g, double k, bem_op op, bem_method m,
                       bem_precision p, int nrhs, const void *x_dev, void *y_dev);

/* ------------------------------------------------------------------ solve */
typedef struct {
    double tol;          /* relative residual |b - A x| / |b| to reach; 0 -> 1e-8 */
    int restart;         /* GMRES: restart length, 0 -> 50, at most 90.  BiCGSTAB: steps
                            per cycle, 0 -> 50; a cycle ends early once the updated
                            residual meets tol, and every cycle starts from the FP64
                            residual b - A x */
    int max_restarts;    /* cycles per solve; 0 -> 100 */
    bem_precision precision; /* FP64: the Krylov method on the FP64 FMM operator.  MIXED: the
                                same method, whose steps use the mixed product once the relative
                                residual r satisfies inner_tol * r <= tol / 10 (relaxed
                                inexact Krylov); every residual that decides convergence
                                (each cycle start and the end) uses the FP64 product */
    double inner_tol;    /* MIXED only: bound on the mixed product's relative deviation
                            from the FP64 product; 0 -> 1e-6 */
    int max_iters;       /* budget of Krylov steps per right-hand side (GMRES: Arnoldi steps,
                            BiCGSTAB: steps of two products); a right-hand side that spends it
                            stops where it is; 0 -> none beyond restart x max_restarts */
    bem_method method;   /* operator used (BEM_FMM unless set) */
    bem_krylov krylov;   /* BEM_KRYLOV_GMRES (0) or BEM_KRYLOV_BICGSTAB */
    double max_seconds;  /* wall-clock budget of the whole call, checked after every step;
                            when it runs out every right-hand side stops where it is;
                            0 -> none */
} bem_solve_opts;

typedef struct {
    int iterations;      /* total inner Krylov iterations */
    int restarts;        /* cycles restarted from an FP64 residual b - A x above tol */
    int matvecs;         /* operator applications, FP64 and mixed */
    double residual;     /* final |b - A x| / |b| with the FP64 operator */
    int status;          /* BEM_OK, or BEM_ENOCONV: tol not reached within max_restarts cycles,
                            max_iters steps or max_seconds (phi then holds the last iterate,
                            residual its FP64 residual) */
} bem_solve_info;

/* Solves Eq. (1) for phi given chi, for each of nrhs right-hand sides
 * (Section 2.1): b = -S chi with the FP64 operator, then GMRES(restart)
 * (default) or BiCGSTAB, the paper's solver, from x0 = 0.  GMRES advances the
 * right-hand sides in lock step with one batched product per step; BiCGSTAB
 * solves them one after the other.  chi_dev and phi_dev are
 * device buffers of nrhs * n_dof values; info is a host array of nrhs.
 * Returns BEM_ENOCONV (with phi and info written) if a right-hand side did
 * not converge within its cycle, step or time budget.
 * Errors: BEM_EINVAL as for bem_matvec, for restart > 90 with GMRES, negative
 * max_iters or max_seconds, and for a Helmholtz k above the wavenumber the
 * tree's lists were built for (see bem_matvec). */
int bem_solve(bem_ctx *ctx, const bem_tree *tree, bem_green g, double k, int nrhs,
              const void *chi_dev, void *phi_dev, const bem_solve_opts *opts, bem_solve_info *info);

/* ------------------------------------------------------------------ field
 * Potential at points off the surface from the surface solution
 * (Section 3.5, accelerated field evaluation; Eq. 1 with C = 1 outside the
 * body and 0 inside):
 *     u(x) = sum over the 7 rule points y of every element of
 *            wJ(y) [phi(y) dG/dn1(x, y) - chi(y) G(x, y)],
 * phi and chi interpolated from their DOF values.  The tree's moments (double
 * layer of phi minus single layer of chi) are shifted to the root and each
 * point descends the tree: a box far from it (|x - c| > r_C / theta, the
 * paper's test at theta = 1, and for Helmholtz k r_C <= 0.75) contributes
 * its order-p multipole expansion, a leaf that is not far its direct
 * 7-point sum.  theta <= 0 selects 0.25 (about 1e-6 of the direct sum
 * at order 8); theta > 1 gives BEM_EINVAL.  FP64 throughout; the 7-point
 * rule is accurate for points a few element sizes away from the surface
 * (points on it are not allowed).
 *   phi_dev, chi_dev: [nrhs][n_dof] device, f64 (Laplace) or c128 interleaved
 *                     (Helmholtz), DOF order of bem_mesh_dofs
 *   pts_dev:          [n_pts][3] f64 device
 *   u_dev:            [nrhs][n_pts] device, same value type as phi
 * Buffers are caller-owned and read / written on the context's stream;
 * returns after the work is complete.  BEM_EINVAL for nrhs < 1, missing or
 * aliased buffers, k <= 0 for Helmholtz. */
int bem_field(bem_ctx *ctx, const bem_tree *tree, bem_green g, double k, double theta, int nrhs,
              const void *phi_dev, const void *chi_dev, int64_t n_pts, const double *pts_dev, void *u_dev);

/* ------------------------------------------------------------------ serving
 * Batched / concurrent solves for many independent problems on one GPU (no
 * counterpart in the paper: a production layer around the solve above).
 * A server runs `lanes` workers, each with its own context (HIP stream of
 * its own, default priority) and host thread.  Meshes are registered once and
 * stay with one lane, which builds their device mesh and trees on first use
 * and keeps them resident.  A mesh holds one tree per wavenumber bucket: with
 * the wavenumber bound on (tree.kappa > 0, tree.k_hint = 0) a Helmholtz
 * request of wavenumber k uses the tree whose lists hold for every k up to
 * the bucket's top 2^(ceil(4 log2 k) / 4) (buckets 19% wide), Laplace
 * requests a tree without the bound; otherwise one tree per mesh.
 * Admission by device-memory budget: every lane's context is bounded by
 * hbm_budget / lanes bytes (everything it holds: meshes, trees, their
 * per-wavenumber caches, Krylov bases, staging and freed blocks kept for
 * reuse), so the server never holds more than hbm_budget.  Before a batch a
 * lane evicts its least recently used trees until the batch's estimate fits;
 * an allocation that would still pass the bound makes the lane evict one more
 * tree and run the batch again; a batch that does not fit even in an empty
 * lane fails with BEM_ENOMEM.  Requests queue per lane in arrival order; a
 * worker takes the oldest request and merges the waiting requests with the
 * same (mesh, Green, k) into one solve, up to max_batch_rhs right-hand sides
 * (continuous batching).  Every right-hand side is solved exactly as
 * bem_solve solves it on the same tree with the same options, so results do
 * not depend on batching, lanes, eviction or arrival order; the solve
 * options' step and time budgets (max_iters, max_seconds) bound each batch.
 * Host buffers passed to the server are copied at the call; results are
 * copied out by bem_server_poll.  The server calls are thread-safe. */
typedef struct bem_server bem_server;

typedef struct {
    int device;              /* HIP device */
    int lanes;               /* concurrent workers; 0 -> 4 */
    int64_t hbm_budget;      /* device bytes the server may hold in total; 0 -> 32 GiB */
    int max_batch_rhs;       /* most right-hand sides merged into one solve; 0 -> 32 */
    bem_tree_opts tree;      /* tree options of every mesh (zero fields -> defaults).  With
                                kappa > 0 and k_hint = 0, Helmholtz requests use trees per
                                wavenumber bucket (above); with k_hint > 0 every mesh has one
                                tree, whose lists hold for every k <= k_hint, and requests
                                with a larger k are refused */
    bem_solve_opts solve;    /* solve options of every request (zero fields -> defaults) */
    int helmholtz_B;         /* leaf size of the per-wavenumber-bucket Helmholtz trees (kappa > 0,
                                k_hint = 0); 0 -> tree.B.  High wavenumbers favour larger leaves:
                                the bound leaves few boxes small enough to interact */
} bem_server_opts;

typedef struct {
    int64_t submitted, completed, batches, rhs_solved, evictions, trees_built;
    int64_t resident_bytes;  /* device bytes held by the lanes now (live and kept for reuse) */
    int64_t resident_peak;   /* sum over the lanes of the most each has held at once (>= the
                                largest resident_bytes; at most hbm_budget) */
    int64_t rejected;        /* requests that failed with BEM_ENOMEM (larger than a lane's share) */
} bem_server_stats;

/* Starts the workers.  Errors: BEM_EINVAL for bad options, BEM_EDEVICE. */
int bem_server_create(const bem_server_opts *opts, bem_server **out);
/* Registers a mesh (arguments as bem_mesh_load, host arrays copied) and
 * returns its id and DOF count (the layout of chi / phi below).  The DOF
 * indexing runs here on the host; device work waits for the first request. */
int bem_server_add_mesh(bem_server *s, const double *node_xyz, int64_t n_nodes, const int32_t *elem_nodes,
                        int64_t n_elem, const bem_mesh_opts *opts, int32_t *mesh_id, int64_t *n_dof);
/* DOF layout of a registered mesh (as bem_mesh_dofs; each buffer may be NULL). */
int bem_server_mesh_dofs(bem_server *s, int32_t mesh_id, int32_t *elem_dofs, double *dof_xyz, double *dof_normal);
/* Queues a solve of c.phi - K phi = -S chi for nrhs right-hand sides; chi_host
 * is [nrhs][n_dof] float64 (Laplace) or interleaved complex128 (Helmholtz),
 * copied here.  Returns a ticket.  Errors: BEM_EINVAL (unknown mesh, nrhs < 1
 * or above max_batch_rhs, k <= 0 for Helmholtz, a Helmholtz k above the
 * server's fixed tree.k_hint when tree.kappa > 0). */
int bem_server_submit(bem_server *s, int32_t mesh_id, bem_green g, double k, int nrhs, const void *chi_host,
                      int64_t *ticket);
/* Result of a ticket: with wait != 0 blocks until it completes.  When done,
 * copies phi ([nrhs][n_dof], may be NULL) and info ([nrhs], may be NULL),
 * sets *latency_s (may be NULL) to the time from submission to completion,
 * releases the ticket and returns the solve's status (BEM_OK or
 * BEM_ENOCONV, or the error that stopped it, e.g. BEM_ENOMEM for a request
 * larger than a lane's share of the budget).  Returns BEM_EAGAIN if not
 * done and wait == 0, BEM_EINVAL for an unknown ticket. */
int bem_server_poll(bem_server *s, int64_t ticket, int wait, void *phi_host, bem_solve_info *info,
                    double *latency_s);
int bem_server_stats_get(bem_server *s, bem_server_stats *st);
/* Finishes the queued work, stops the workers and frees everything. */
void bem_server_destroy(bem_server *s);

#ifdef __cplusplus
}
#endif
#endif /* BEM_H */
