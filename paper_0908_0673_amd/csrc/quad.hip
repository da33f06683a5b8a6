// Singular and near-singular element quadrature (Section 2.1) as sparse
// corrections, and the free term of Eq. (2).
//
// The regular 7-point rule is applied to every (target, element) pair by the
// near-field sums and, in the far field, through the expansions.  For the
// pairs where it is not accurate the exact contribution is restored by a
// sparse correction "accurate rule minus 7-point rule", stored per pair and
// element node (Section 3.6: the near-field part is kept as a sparse matrix
// for re-use).  Classification of a pair (target DOF x at geometric node g,
// element m with corner mean c_m and h_m = largest |node - c_m|):
//   singular       g is a node of m: Duffy rule about that node, one collapsed
//                  triangle for a corner, two for a mid-side node, 12 x 12
//                  Gauss-Legendre points each;
//   near-singular  |x - c_m| < 2 h_m: 4^d equal sub-triangles with the 7-point
//                  rule, d the least integer >= 1 with h_m / 2^d <= |x - c_m| / 2,
//                  at most 4;
//   regular        otherwise.
// The tests on squared distances use plain IEEE operations (this unit is
// compiled without contraction), so the classification is reproducible.
//
// Pairs are found per target by walking the tree: an element in box X can be
// near a target only if the target lies within 5 r_X of the box centre
// (h_m <= 2 r_X and |c_m - c_X| <= r_X).
#include <cmath>

#include "greens.h"
#include "kernels.h"

namespace bem {

namespace {

constexpr int NG = 12;  // Gauss-Legendre points per direction of the Duffy rule

struct Gauss {
    double x[NG], w[NG];  // on [0, 1]
};

// Gauss-Legendre nodes on [0, 1] by Newton iteration on the Legendre recurrence.
Gauss gauss_legendre01() {
    Gauss g;
    const int n = NG;
    for (int i = 0; i < n; i++) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 60; it++) {
            double p1 = 1.0, p2 = 0.0;
            for (int k = 1; k <= n; k++) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * k - 1.0) * x * p2 - (k - 1.0) * p3) / k;
            }
            dp = n * (x * p1 - p2) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p1 = 1.0, p2 = 0.0;
        for (int k = 1; k <= n; k++) {
            double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * k - 1.0) * x * p2 - (k - 1.0) * p3) / k;
        }
        dp = n * (x * p1 - p2) / (x * x - 1.0);
        g.x[i] = 0.5 * (1.0 - x);
        g.w[i] = 1.0 / ((1.0 - x * x) * dp * dp);
    }
    return g;
}

struct R7 {
    double s[7], t[7], w[7];
};

__device__ inline double dsq(double a0, double a1, double a2) { return (a0 * a0 + a1 * a1) + a2 * a2; }

// classification of (target at x with geometric node g, sorted element se)
// Per sorted element: the centroid of its corner nodes and h^2, the largest
// squared distance from it to the element's six nodes (the element's extent
// as the classification below uses it), [n_el][4].
__global__ void k_elem_extent(int64_t n_el, const int32_t *se_nodes, const double *xyz, double *ext) {
    const int64_t se = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (se >= n_el) return;
    const int32_t *en = se_nodes + 6 * se;
    double cm[3];
    for (int d = 0; d < 3; d++)
        cm[d] = ((xyz[3 * (int64_t)en[0] + d] + xyz[3 * (int64_t)en[1] + d]) + xyz[3 * (int64_t)en[2] + d]) / 3.0;
    double h2 = 0.0;
    for (int a = 0; a < 6; a++) {
        const double *p = xyz + 3 * (int64_t)en[a];
        double v = dsq(p[0] - cm[0], p[1] - cm[1], p[2] - cm[2]);
        if (v > h2) h2 = v;
    }
    ext[4 * se] = cm[0];
    ext[4 * se + 1] = cm[1];
    ext[4 * se + 2] = cm[2];
    ext[4 * se + 3] = h2;
}

// Per box: the largest element extent h (square root of h^2 above) over the
// box's elements, one wave per box.
__global__ void k_box_extent(int64_t n_box, const int64_t *eb, const int64_t *ee, const double *ext, double *hbox) {
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    double m = 0.0;
    for (int64_t e = eb[b] + lane; e < ee[b]; e += 64) m = fmax(m, ext[4 * e + 3]);
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) hbox[b] = sqrt(m);
}

__device__ inline int classify(const int32_t *se_nodes, const double *ext, int64_t se, int32_t g, const double x[3],
                               int *param) {
    const int32_t *en = se_nodes + 6 * se;
    for (int a = 0; a < 6; a++)
        if (en[a] == g) { *param = a; return 2; }
    const double4 e4 = *(const double4 *)(ext + 4 * se);
    const double cm[3] = {e4.x, e4.y, e4.z}, h2 = e4.w;
    double d2 = dsq(x[0] - cm[0], x[1] - cm[1], x[2] - cm[2]);
    if (!(d2 < 4.0 * h2)) return 0;
    int d = 1;
    double f = 4.0;
    while (d < 4 && 4.0 * h2 > d2 * f) { d++; f *= 4.0; }
    *param = d;
    return 1;
}

// PASS 0: count pairs per sorted target; PASS 1: write them.  A depth-first
// walk from the root visits the boxes in tree order; a box is skipped when the
// target is farther from its centre than its radius plus twice its largest
// element extent (with a relative margin), since every element the
// classification accepts lies within twice its extent of the target and
// within the box's radius of its centre.
template <int PASS>
__global__ void k_pairs(int64_t n_tgt, const double *t64, const int32_t *tperm, const int32_t *dof_node,
                        const double *ext, const int32_t *se_nodes, const int32_t *leaf, const int32_t *child_begin,
                        const int32_t *nchild, const int64_t *eb, const int64_t *ee, const double *centre,
                        const double *radius, const double *hbox, int64_t *count, const int64_t *row_ptr,
                        int32_t *pair_elem,
                        int32_t *pair_info, int32_t *pair_row) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tgt) return;
    double x[3] = {t64[t], t64[n_tgt + t], t64[2 * n_tgt + t]};
    int32_t g = dof_node[tperm[t]];
    int32_t stack[192];
    int sp = 0;
    stack[sp++] = 0;
    int64_t cnt = 0, w = PASS ? row_ptr[t] : 0;
    while (sp > 0) {
        int32_t X = stack[--sp];
        const double *c = centre + 3 * (int64_t)X;
        double dd = sqrt(dsq(x[0] - c[0], x[1] - c[1], x[2] - c[2]));
        if (dd > (radius[X] + 2.0 * hbox[X]) * (1.0 + 1e-9) + 1e-300) continue;
        if (ee[X] == eb[X]) continue;
        if (leaf[X]) {
            for (int64_t se = eb[X]; se < ee[X]; se++) {
                int param = 0;
                int cls = classify(se_nodes, ext, se, g, x, &param);
                if (cls == 0) continue;
                if (PASS == 1) {
                    pair_elem[w + cnt] = (int32_t)se;
                    pair_info[w + cnt] = cls | (param << 4);
                    pair_row[w + cnt] = (int32_t)t;
                }
                cnt++;
            }
        } else {
            for (int ch = nchild[X] - 1; ch >= 0; ch--) stack[sp++] = child_begin[X] + ch;
        }
    }
    if (PASS == 0) count[t] = cnt;
}

// One wave per pair: (accurate rule - 7-point rule) integrals of L_a G and L_a dG/dn1.
// lin: first-order elements, L = (1 - s - t, s, t, 0, 0, 0) (the element map
// stays the quadratic one through the edge midpoints, which is flat).
template <bool HELM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HELM ? 1 : 4, HELM ? 2 : 4)))
k_corr_values(int64_t n_pairs, const int32_t *pair_elem, const int32_t *pair_info, const int32_t *pair_row,
              const double *t64, int64_t n_tgt, const int32_t *se_nodes, const uint8_t *se_mask, const double *xyz,
              double k, int lin, Gauss gq_arg, R7 r7_arg, double *Sout, double *Kout) {
    // the rules are indexed per point: kept in LDS (a by-value kernel
    // argument indexed at run time would be copied to scratch per thread)
    __shared__ Gauss gq;
    __shared__ R7 r7;
    __shared__ double V3[3][2], MID[3][2];
    if (threadIdx.x < NG) {
        gq.x[threadIdx.x] = gq_arg.x[threadIdx.x];
        gq.w[threadIdx.x] = gq_arg.w[threadIdx.x];
    }
    if (threadIdx.x < 7) {
        r7.s[threadIdx.x] = r7_arg.s[threadIdx.x];
        r7.t[threadIdx.x] = r7_arg.t[threadIdx.x];
        r7.w[threadIdx.x] = r7_arg.w[threadIdx.x];
    }
    if (threadIdx.x < 3) {
        const double v3[3][2] = {{0, 0}, {1, 0}, {0, 1}};
        const double mid[3][2] = {{0.5, 0.0}, {0.5, 0.5}, {0.0, 0.5}};
        for (int d = 0; d < 2; d++) {
            V3[threadIdx.x][d] = v3[threadIdx.x][d];
            MID[threadIdx.x][d] = mid[threadIdx.x][d];
        }
    }
    __syncthreads();
    int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    int lane = threadIdx.x & 63;
    if (p >= n_pairs) return;
    int64_t se = pair_elem[p];
    int info = pair_info[p], cls = info & 15, param = info >> 4;
    int64_t row = pair_row[p];
    double x[3] = {t64[row], t64[n_tgt + row], t64[2 * n_tgt + row]};
    double X[6][3];
    for (int a = 0; a < 6; a++)
        for (int d = 0; d < 3; d++) X[a][d] = xyz[3 * (int64_t)se_nodes[6 * se + a] + d];
    using V = typename std::conditional<HELM, cx<double>, double>::type;
    V S[6], K[6];
    for (int a = 0; a < 6; a++) { S[a] = V(0.0); K[a] = V(0.0); }

    int npts;
    if (cls == 2) npts = (param < 3 ? 1 : 2) * NG * NG;
    else npts = 7 << (2 * param);
    for (int j = lane; j < npts + 7; j += 64) {
        double s, t, w;
        if (j >= npts) {  // minus the regular rule
            int q = j - npts;
            s = r7.s[q]; t = r7.t[q]; w = -r7.w[q];
        } else if (cls == 2) {
            int sub = j / (NG * NG), rem = j % (NG * NG);
            double u = gq.x[rem / NG], v = gq.x[rem % NG];
            double P[2], A[2], B[2];
            if (param < 3) {
                P[0] = V3[param][0]; P[1] = V3[param][1];
                A[0] = V3[(param + 1) % 3][0]; A[1] = V3[(param + 1) % 3][1];
                B[0] = V3[(param + 2) % 3][0]; B[1] = V3[(param + 2) % 3][1];
            } else {
                int c0 = param - 3, c1 = (param - 2) % 3, c2 = (param - 1) % 3;
                P[0] = MID[c0][0]; P[1] = MID[c0][1];
                int ia = sub == 0 ? c1 : c2, ib = sub == 0 ? c2 : c0;
                A[0] = V3[ia][0]; A[1] = V3[ia][1];
                B[0] = V3[ib][0]; B[1] = V3[ib][1];
            }
            double det = fabs((A[0] - P[0]) * (B[1] - A[1]) - (A[1] - P[1]) * (B[0] - A[0]));
            s = P[0] + u * (A[0] - P[0]) + u * v * (B[0] - A[0]);
            t = P[1] + u * (A[1] - P[1]) + u * v * (B[1] - A[1]);
            w = gq.w[rem / NG] * gq.w[rem % NG] * u * det;
        } else {
            int sub = j / 7, q = j % 7;
            double A[2] = {0, 0}, B[2] = {1, 0}, C[2] = {0, 1};
            for (int l = param - 1; l >= 0; l--) {
                int dg = (sub >> (2 * l)) & 3;
                double ab[2] = {0.5 * (A[0] + B[0]), 0.5 * (A[1] + B[1])};
                double bc[2] = {0.5 * (B[0] + C[0]), 0.5 * (B[1] + C[1])};
                double ca[2] = {0.5 * (C[0] + A[0]), 0.5 * (C[1] + A[1])};
                if (dg == 0) { B[0] = ab[0]; B[1] = ab[1]; C[0] = ca[0]; C[1] = ca[1]; }
                else if (dg == 1) { A[0] = ab[0]; A[1] = ab[1]; C[0] = bc[0]; C[1] = bc[1]; }
                else if (dg == 2) { A[0] = ca[0]; A[1] = ca[1]; B[0] = bc[0]; B[1] = bc[1]; }
                else { A[0] = ab[0]; A[1] = ab[1]; B[0] = bc[0]; B[1] = bc[1]; C[0] = ca[0]; C[1] = ca[1]; }
            }
            s = A[0] + r7.s[q] * (B[0] - A[0]) + r7.t[q] * (C[0] - A[0]);
            t = A[1] + r7.s[q] * (B[1] - A[1]) + r7.t[q] * (C[1] - A[1]);
            w = r7.w[q] / (double)(1 << (2 * param));
        }
        double y[3], n[3], J, L[6];
        elem_map(X, s, t, y, n, &J, L);
        if (lin) {
            L[0] = 1.0 - s - t; L[1] = s; L[2] = t;
            L[3] = L[4] = L[5] = 0.0;
        }
        double r[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
        double r2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
        double rn = r[0] * n[0] + r[1] * n[1] + r[2] * n[2];
        V G, dG;
        if constexpr (HELM) green_helmholtz<double>(r2, rn, k, &G, &dG);
        else green_laplace<double>(r2, rn, &G, &dG);
        double wj = w * J;
        for (int a = 0; a < 6; a++) {
            double f = wj * L[a];
            S[a] += G * f;
            K[a] += dG * f;
        }
    }
    const int mk = se_mask ? se_mask[se] : 0x3f;  // literal tree: the piece's own slots
    for (int a = 0; a < 6; a++) {
        S[a] = (mk >> a & 1) ? wave_sum(S[a]) : V(0.0);
        K[a] = (mk >> a & 1) ? wave_sum(K[a]) : V(0.0);
    }
    if (lane == 0) {
        for (int a = 0; a < 6; a++) {
            if constexpr (HELM) {
                Sout[2 * (6 * p + a)] = S[a].re; Sout[2 * (6 * p + a) + 1] = S[a].im;
                Kout[2 * (6 * p + a)] = K[a].re; Kout[2 * (6 * p + a) + 1] = K[a].im;
            } else {
                Sout[6 * p + a] = S[a];
                Kout[6 * p + a] = K[a];
            }
        }
    }
}

// free term, in DOF order: c = 1 + (regular sum over all points) + sum of the Laplace K corrections
__global__ void k_free_term(int64_t n_tgt, const int32_t *tperm, const double *reg, const int64_t *row_ptr,
                            const double *K0, double *c) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tgt) return;
    double acc = reg[t];
    for (int64_t p = row_ptr[t]; p < row_ptr[t + 1]; p++)
        for (int a = 0; a < 6; a++) acc += K0[6 * p + a];
    c[tperm[t]] = 1.0 + acc;
}

}  // namespace

void build_pairs(bem_tree &t) {
    if (t.has_pairs) return;
    Ctx &c = *t.ctx;
    SetupTimer st_(c, "correction pair search");
    const bem_mesh &m = *t.mesh;
    DBuf<int64_t> cnt;
    cnt.alloc(&c, t.n_tgt);
    t.pair_ptr.alloc(&c, t.n_tgt + 1);
    DBuf<double> ext;  // element extents, as the classification uses them
    ext.alloc(&c, 4 * (size_t)std::max<int64_t>(1, t.n_el));
    k_elem_extent<<<nblocks(t.n_el, 256), 256, 0, c.stream>>>(t.n_el, t.se_nodes.p, m.xyz.p, ext.p);
    BEM_LAUNCH_CHECK();
    DBuf<double> hbox;
    hbox.alloc(&c, (size_t)std::max<int64_t>(1, t.n_box));
    k_box_extent<<<(unsigned)t.n_box, 64, 0, c.stream>>>(t.n_box, t.eb.p, t.ee.p, ext.p, hbox.p);
    BEM_LAUNCH_CHECK();
    unsigned nb = nblocks(t.n_tgt, 64);
    k_pairs<0><<<nb, 64, 0, c.stream>>>(t.n_tgt, t.t64.p, t.tperm.p, m.dof_node.p, ext.p, t.se_nodes.p, t.leaf.p,
                                        t.child_begin.p, t.nchild.p, t.eb.p, t.ee.p, t.centre.p, t.radius.p, hbox.p,
                                        cnt.p, nullptr, nullptr, nullptr, nullptr);
    BEM_LAUNCH_CHECK();
    scan_exclusive<int64_t>(c, cnt.p, t.pair_ptr.p, t.n_tgt);
    t.n_pairs = read_scalar(c, t.pair_ptr.p + t.n_tgt);
    t.pair_elem.alloc(&c, t.n_pairs);
    t.pair_info.alloc(&c, t.n_pairs);
    t.pair_row.alloc(&c, t.n_pairs);
    k_pairs<1><<<nb, 64, 0, c.stream>>>(t.n_tgt, t.t64.p, t.tperm.p, m.dof_node.p, ext.p, t.se_nodes.p, t.leaf.p,
                                        t.child_begin.p, t.nchild.p, t.eb.p, t.ee.p, t.centre.p, t.radius.p, hbox.p,
                                        nullptr, t.pair_ptr.p, t.pair_elem.p, t.pair_info.p, t.pair_row.p);
    BEM_LAUNCH_CHECK();
    c.sync();
    t.has_pairs = true;
}

Corr &get_corr(bem_tree &t, int green, double k) {
    if (green == BEM_LAPLACE) k = 0.0;
    for (auto &p : t.corr)
        if (p->green == green && p->k == k) {
            p->last_use = ++t.k_uses;
            return *p;
        }
    build_pairs(t);
    Ctx &c = *t.ctx;
    SetupTimer st_(c, "corrections");
    if (green == BEM_HELMHOLTZ) evict_wavenumbers(t.corr);
    auto cr = std::make_unique<Corr>();
    cr->green = green;
    cr->k = k;
    cr->last_use = ++t.k_uses;
    const int cw = green == BEM_HELMHOLTZ ? 2 : 1;
    cr->S.alloc(&c, (size_t)6 * cw * t.n_pairs);
    cr->K.alloc(&c, (size_t)6 * cw * t.n_pairs);
    if (t.n_pairs > 0) {
        Gauss gq = gauss_legendre01();
        R7 r7;
        rule7(r7.s, r7.t, r7.w);
        unsigned nb = nblocks(t.n_pairs, 4);
        if (green == BEM_HELMHOLTZ)
            k_corr_values<true><<<nb, 256, 0, c.stream>>>(t.n_pairs, t.pair_elem.p, t.pair_info.p, t.pair_row.p,
                                                          t.t64.p, t.n_tgt, t.se_nodes.p, t.se_mask.p, t.mesh->xyz.p,
                                                          k, (int)t.mesh->linear, gq, r7, cr->S.p, cr->K.p);
        else
            k_corr_values<false><<<nb, 256, 0, c.stream>>>(t.n_pairs, t.pair_elem.p, t.pair_info.p, t.pair_row.p,
                                                           t.t64.p, t.n_tgt, t.se_nodes.p, t.se_mask.p, t.mesh->xyz.p,
                                                           0.0, (int)t.mesh->linear, gq, r7, cr->S.p, cr->K.p);
        BEM_LAUNCH_CHECK();
    }
    c.sync();
    t.corr.push_back(std::move(cr));
    return *t.corr.back();
}

void build_free_term(bem_tree &t) {
    if (t.has_free_term) return;
    Ctx &c = *t.ctx;
    SetupTimer st_(c, "free term");
    const bem_mesh &m = *t.mesh;
    for (const auto &f : m.free_terms)
        if (f->B == t.B && f->max_depth == t.max_depth && f->attach == t.attach && f->literal == t.literal) {
            t.free_term.alloc(&c, t.n_tgt);
            BEM_HIP(hipMemcpyAsync(t.free_term.p, f->c.p, sizeof(double) * t.n_tgt, hipMemcpyDeviceToDevice,
                                   c.stream));
            c.sync();
            t.has_free_term = true;
            return;
        }
    Corr &lap = get_corr(t, BEM_LAPLACE, 0.0);
    DBuf<double> reg;
    reg.alloc(&c, t.n_tgt);
    // regular 7-point sum of dG0/dn1 over every point: the double layer of a unit density
    direct_regular_unit_double_layer(t, reg.p);
    t.free_term.alloc(&c, t.n_tgt);
    k_free_term<<<nblocks(t.n_tgt, 256), 256, 0, c.stream>>>(t.n_tgt, t.tperm.p, reg.p, t.pair_ptr.p, lap.K.p,
                                                            t.free_term.p);
    BEM_LAUNCH_CHECK();
    auto f = std::make_unique<bem_mesh::FreeTerm>();
    f->B = t.B;
    f->max_depth = t.max_depth;
    f->attach = t.attach;
    f->literal = t.literal;
    f->c.alloc(m.ctx ? m.ctx : &c, t.n_tgt);
    BEM_HIP(hipMemcpyAsync(f->c.p, t.free_term.p, sizeof(double) * t.n_tgt, hipMemcpyDeviceToDevice, c.stream));
    c.sync();
    m.free_terms.push_back(std::move(f));
    t.has_free_term = true;
}

}  // namespace bem
