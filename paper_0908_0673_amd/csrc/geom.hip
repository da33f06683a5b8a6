// Geometry precompute (Section 2.2): for every element in tree order, its
// six node ids and DOF ids, and for every point of the 7-point degree-5 rule
// the position, unit normal and weight x area Jacobian, stored
// structure-of-arrays in FP64 and FP32 so that the near-field sums read them
// coalesced.  Targets (DOF positions) are stored in tree order the same way.
#include <cmath>

#include "kernels.h"

namespace bem {

// Radon's 7-point rule of degree 5 on the reference triangle {s, t >= 0,
// s + t <= 1}; the weights sum to the triangle's area 1/2.
void rule7(double s[7], double t[7], double w[7]) {
    const double q = std::sqrt(15.0);
    const double a1 = (6.0 - q) / 21.0, a2 = (6.0 + q) / 21.0;
    const double w0 = 9.0 / 80.0, w1 = (155.0 - q) / 2400.0, w2 = (155.0 + q) / 2400.0;
    const double ss[7] = {1.0 / 3.0, a1, a1, 1.0 - 2.0 * a1, a2, a2, 1.0 - 2.0 * a2};
    const double tt[7] = {1.0 / 3.0, a1, 1.0 - 2.0 * a1, a1, a2, 1.0 - 2.0 * a2, a2};
    const double ww[7] = {w0, w1, w1, w1, w2, w2, w2};
    for (int i = 0; i < 7; i++) { s[i] = ss[i]; t[i] = tt[i]; w[i] = ww[i]; }
}

namespace {

struct Rule7 {
    double s[7], t[7], w[7];
};

__global__ void k_geom(const int32_t *eperm, const int32_t *elem, const int32_t *elem_dofs, const double *xyz,
                       int64_t n_el, Rule7 r, int32_t *se_nodes, int32_t *se_dofs, double *q64, float *q32) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 7 * n_el) return;
    int64_t se = i / 7;
    int q = (int)(i % 7);
    int64_t e = eperm[se];
    const int32_t *en = elem + 6 * e;
    if (q < 6) {
        se_nodes[6 * se + q] = en[q];
        se_dofs[6 * se + q] = elem_dofs[6 * e + q];
    }
    double s = r.s[q], t = r.t[q], z = 1.0 - s - t;
    double L[6] = {z * (2.0 * z - 1.0), s * (2.0 * s - 1.0), t * (2.0 * t - 1.0), 4.0 * z * s, 4.0 * s * t, 4.0 * t * z};
    double Ls[6] = {1.0 - 4.0 * z, 4.0 * s - 1.0, 0.0, 4.0 * (z - s), 4.0 * t, -4.0 * t};
    double Lt[6] = {1.0 - 4.0 * z, 0.0, 4.0 * t - 1.0, -4.0 * s, 4.0 * s, 4.0 * (z - t)};
    double y[3] = {0, 0, 0}, a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int k = 0; k < 6; k++) {
        const double *p = xyz + 3 * (int64_t)en[k];
        for (int d = 0; d < 3; d++) {
            y[d] += L[k] * p[d];
            a[d] += Ls[k] * p[d];
            b[d] += Lt[k] * p[d];
        }
    }
    double n[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double J = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double v[7] = {y[0], y[1], y[2], r.w[q] * J, n[0] / J, n[1] / J, n[2] / J};
    const int64_t nq = 7 * n_el;
    for (int k = 0; k < 7; k++) {
        q64[k * nq + i] = v[k];
        q32[k * nq + i] = (float)v[k];
    }
}

__global__ void k_targets(const int32_t *tperm, const double *dof_xyz, int64_t n, double *t64, float *t32) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *p = dof_xyz + 3 * (int64_t)tperm[i];
    for (int d = 0; d < 3; d++) {
        t64[d * n + i] = p[d];
        t32[d * n + i] = (float)p[d];
    }
}

}  // namespace

void build_geometry(bem_tree &t) {
    Ctx &c = *t.ctx;
    const bem_mesh &m = *t.mesh;
    Rule7 r;
    rule7(r.s, r.t, r.w);
    t.n_q = 7 * t.n_el;
    t.se_nodes.alloc(&c, 6 * t.n_el);
    t.se_dofs.alloc(&c, 6 * t.n_el);
    t.q64.alloc(&c, 7 * t.n_q);
    t.q32.alloc(&c, 7 * t.n_q);
    k_geom<<<nblocks(t.n_q, 256), 256, 0, c.stream>>>(t.eperm.p, m.elem.p, m.elem_dofs.p, m.xyz.p, t.n_el, r,
                                                       t.se_nodes.p, t.se_dofs.p, t.q64.p, t.q32.p);
    BEM_LAUNCH_CHECK();
    t.t64.alloc(&c, 3 * t.n_tgt);
    t.t32.alloc(&c, 3 * t.n_tgt);
    k_targets<<<nblocks(t.n_tgt, 256), 256, 0, c.stream>>>(t.tperm.p, m.dof_xyz.p, t.n_tgt, t.t64.p, t.t32.p);
    BEM_LAUNCH_CHECK();
}

}  // namespace bem
