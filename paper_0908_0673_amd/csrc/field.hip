// Accelerated evaluation of the potential at points off the surface, after
// the solve (Section 3.5): with C(x) = 1 outside the body and 0 inside, the
// boundary integral equation (Eq. 1) gives the field from the surface values,
//
//     u(x) = integral over S of  phi(y) dG/dn1(x, y) - chi(y) G(x, y)  dS(y),
//
// here with the 7-point rule on every element (points are expected to stay a
// few element sizes away from the surface, where that rule is accurate).
// The tree and its expansions are reused: the moments of the double layer of
// phi minus those of the single layer of chi (both through the stored P2M
// weights) are shifted up to the root, and every point descends the tree from
// the root: a box far from the point contributes its multipole expansion
// evaluated at the point, a leaf that is not far contributes the direct
// 7-point sum over its elements, and any other box is opened.  The paper
// calls a box far when |x - c| > r_C; here a safety factor theta applies as
// in the interaction lists (|x - c| > r_C / theta), which is the paper's
// test at theta = 1.  A single expansion evaluated at a point is the whole of
// the far contribution there (no near field or free term beside it), so the
// field takes a smaller theta than the product: 0.25 unless given, which
// keeps order 8 within about 1e-6 of the direct sum.  For Helmholtz a far box
// must also satisfy k r_C <= 0.75: the expansion of e^{jkR} about the box
// centre converges like (k r_C)^(p+1) / (p+1)!, which at order 8 leaves
// about 2e-7 there, whatever the distance.  FP64 throughout.
//
// The multipole evaluation is the b = 0 row of the scaled translation of
// m2l.hip: with r = (x - c)/rho and wavenumber k rho,
//     u += (1 / rho) sum_a (-1)^|a| D_a(r) Mh_a,
// the derivatives D_a of G by the recursion of Section 3.3 (greens.h).
#include <cmath>
#include <type_traits>

#include "greens.h"
#include "kernels.h"

namespace bem {

namespace {

constexpr int FIELD_STACK = 256;  // depth-first stack per point (depth 21 x 7 children + 1 fits)
constexpr double FIELD_KAPPA = 0.75;  // Helmholtz: largest k r_C of a box whose expansion is used

// sigma_q = wJ_q sum_a L_a(q) x(DOF of the element's node a), [rhs][n_q]
template <class V>
__global__ void k_field_strength(const V *x, int64_t n_dof, const int32_t *se_dofs, const uint8_t *se_mask,
                                 const double *wj, int64_t n_q, const double *L7, V *s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (i >= n_q) return;
    const int64_t e = i / 7;
    const int q = (int)(i % 7);
    const V *xr = x + (int64_t)rhs * n_dof;
    V acc = V(0.0);
    const int mk = se_mask ? se_mask[e] : 0x3f;  // literal tree: the piece's own slots
    for (int a = 0; a < 6; a++)
        if (mk >> a & 1) acc += xr[se_dofs[6 * e + a]] * L7[6 * q + a];
    s[(int64_t)rhs * n_q + i] = acc * wj[i];
}

template <class V>
__global__ void k_sub_into(V *a, const V *b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] -= b[i];
}

struct FieldTree {
    const int32_t *leaf, *child_begin, *nchild, *level;
    const int64_t *eb, *ee;
    const double *centre, *radius;
    double side, theta;
};

// One wave per (point, right-hand side); the descent is uniform over the
// wave, whose lanes share the expansion coefficients or the leaf's points.
template <bool HELM>
__global__ void __launch_bounds__(64) k_field(const double *pts, int64_t n_pts, FieldTree T, double k, int p,
                                              const int8_t *exps,
                                              const typename std::conditional<HELM, cx<double>, double>::type *mom,
                                              int64_t n_box, const double *q64, int64_t n_q,
                                              const typename std::conditional<HELM, cx<double>, double>::type *sphi,
                                              const typename std::conditional<HELM, cx<double>, double>::type *schi,
                                              typename std::conditional<HELM, cx<double>, double>::type *u) {
    using V = typename std::conditional<HELM, cx<double>, double>::type;
    extern __shared__ unsigned char smem[];
    const int P = deriv_count(p);
    V *A = (V *)smem, *B = A + P, *g = B + P;
    __shared__ int32_t stack[FIELD_STACK];
    __shared__ int sp;
    const int64_t pt = blockIdx.x;
    const int rhs = blockIdx.y, lane = threadIdx.x;
    const double x[3] = {pts[3 * pt], pts[3 * pt + 1], pts[3 * pt + 2]};
    const V *M = mom + (int64_t)rhs * n_box * P;
    const V *sp_phi = sphi + (int64_t)rhs * n_q, *sp_chi = schi + (int64_t)rhs * n_q;
    V acc = V(0.0);
    if (lane == 0) {
        stack[0] = 0;
        sp = 1;
    }
    __syncthreads();
    while (sp > 0) {
        const int X = stack[sp - 1];
        __syncthreads();  // every lane has read the top before it is popped
        if (lane == 0) sp--;
        if (T.ee[X] == T.eb[X]) {
            __syncthreads();
            continue;
        }
        const double *c = T.centre + 3 * (int64_t)X;
        const double d0 = x[0] - c[0], d1 = x[1] - c[1], d2 = x[2] - c[2];
        const double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2), r = T.radius[X];
        const bool far = (!HELM || k * r <= FIELD_KAPPA) && dist > r / T.theta;
        if (far) {
            const double rho = ldexp(T.side, -T.level[X]);
            const double rb[3] = {d0 / rho, d1 / rho, d2 / rho};
            const V *D = derivs_block<HELM>(rb, k * rho, p, exps, A, B, g);
            const V *Mx = M + (int64_t)X * P;
            V s = V(0.0);
            for (int a = lane; a < P; a += 64) {
                const int na = exps[3 * a] + exps[3 * a + 1] + exps[3 * a + 2];
                const V t = D[a] * Mx[a];
                s += (na & 1) ? V(0.0) - t : t;
            }
            acc += s * (1.0 / rho);
        } else if (T.leaf[X]) {
            for (int64_t j = 7 * T.eb[X] + lane; j < 7 * T.ee[X]; j += 64) {
                const double r0 = x[0] - q64[j], r1 = x[1] - q64[n_q + j], r2 = x[2] - q64[2 * n_q + j];
                const double rr = r0 * r0 + r1 * r1 + r2 * r2;
                const double rn = r0 * q64[4 * n_q + j] + r1 * q64[5 * n_q + j] + r2 * q64[6 * n_q + j];
                V G, dG;
                if constexpr (HELM) green_helmholtz<double>(rr, rn, k, &G, &dG);
                else green_laplace<double>(rr, rn, &G, &dG);
                acc += dG * sp_phi[j] - G * sp_chi[j];
            }
        } else if (lane == 0) {
            const int nc = T.nchild[X], cb = T.child_begin[X];
            for (int ch = nc - 1; ch >= 0; ch--) stack[sp++] = cb + ch;  // children visited in order
        }
        __syncthreads();  // the stack and the derivative scratch are free again
    }
    if constexpr (HELM) {
        acc.re = wave_sum(acc.re);
        acc.im = wave_sum(acc.im);
    } else {
        acc = wave_sum(acc);
    }
    if (lane == 0) u[(int64_t)rhs * n_pts + pt] = acc;
}

template <bool HELM>
void field_t(bem_tree &t, double k, double theta, int nrhs, const void *phi, const void *chi, int64_t n_pts,
             const double *pts, void *u) {
    using V = typename std::conditional<HELM, cx<double>, double>::type;
    Ctx &c = *t.ctx;
    fmm_tables(t);
    plan_fmm(t);
    rule_shapes(t);
    build_pass_tables(t);
    const int P = t.tables->P;
    const int64_t nq = t.n_q, nd = t.mesh->n_dof, nexp = t.n_box * (int64_t)P * nrhs;
    DBuf<V> sphi, schi, mom, tmp;
    sphi.alloc(&c, (size_t)nq * nrhs);
    schi.alloc(&c, (size_t)nq * nrhs);
    mom.alloc(&c, (size_t)nexp);
    tmp.alloc(&c, (size_t)nexp);
    mom.zero();
    tmp.zero();
    const dim3 gs(nblocks(nq, 256), nrhs);
    k_field_strength<V><<<gs, 256, 0, c.stream>>>((const V *)phi, nd, t.se_dofs.p, t.se_mask.p, t.q64.p + 3 * nq, nq,
                                                  t.L7.p, sphi.p);
    BEM_LAUNCH_CHECK();
    k_field_strength<V><<<gs, 256, 0, c.stream>>>((const V *)chi, nd, t.se_dofs.p, t.se_mask.p, t.q64.p + 3 * nq, nq,
                                                  t.L7.p, schi.p);
    BEM_LAUNCH_CHECK();
    // moments of the double layer of phi minus those of the single layer of chi
    p2m_apply<V, double, V>(t, true, nrhs, (const V *)phi, mom.p);
    p2m_apply<V, double, V>(t, false, nrhs, (const V *)chi, tmp.p);
    k_sub_into<V><<<nblocks(nexp, 256), 256, 0, c.stream>>>(mom.p, tmp.p, nexp);
    BEM_LAUNCH_CHECK();
    m2m_apply<V, double>(t, nrhs, mom.p, 0);  // a point far away may use the coarsest boxes
    if (n_pts > 0) {
        const FieldTree T{t.leaf.p, t.child_begin.p, t.nchild.p, t.level.p, t.eb.p, t.ee.p, t.centre.p, t.radius.p,
                          t.side, theta > 0.0 ? theta : 0.25};
        const size_t sh = sizeof(V) * (2 * (size_t)P + t.order + 1);
        k_field<HELM><<<dim3((unsigned)n_pts, nrhs), 64, sh, c.stream>>>(
            pts, n_pts, T, k, t.order, t.tables->exps.p, mom.p, t.n_box, t.q64.p, nq, sphi.p, schi.p, (V *)u);
        BEM_LAUNCH_CHECK();
    }
    c.sync();  // the work buffers are released on return
}

}  // namespace

void field(bem_tree &t, int green, double k, double theta, int nrhs, const void *phi, const void *chi, int64_t n_pts,
           const double *pts, void *u) {
    if (green == BEM_HELMHOLTZ) field_t<true>(t, k, theta, nrhs, phi, chi, n_pts, pts, u);
    else field_t<false>(t, 0.0, theta, nrhs, phi, chi, n_pts, pts, u);
}

}  // namespace bem
