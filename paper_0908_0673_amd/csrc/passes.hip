// Upward and downward passes of the fast product (Sections 3.2, 3.6) other
// than the multipole-to-local translation.  Scaled expansions as in fmm.hip:
// Mh_a = M_a / (a! rho^|a|), Fh_b = F_b rho^|b|, rho = side of the box's level.
//
// P2M uses stored weights (Eq. 8): for every leaf and every DOF u touched by
// its elements,
//     W[u][a] = sum over the leaf's elements e, their nodes j with DOF u and
//               the 7 rule points q of  wJ_q L_j(q) Phi_a(y_q),
// with Phi_a(y) = u^a / a! (single layer) or sum_d n_d u^(a - e_d)/(a - e_d)!
// / rho (double layer), u = (y - c)/rho.  The weights depend on the geometry
// only (not on G or k), so they are built once per tree and layer type and the
// moments are one small product per leaf: Mh = W^T x.
//
// (L2P, the evaluation of the local expansions at the targets, runs inside
// the combination kernel of fmm.hip.)
//
// M2M and L2L: a child centre is offset from its parent's by s rho_parent / 4
// with s in {-1, +1}^3 (s_d = +1 when bit d of the child octant is set), so
// every shift coefficient is a magnitude times the sign s^g of some
// multi-index g.  Summing the eight children (M2M) or the eight child
// outputs (L2L) by the parity of g first (a Walsh-Hadamard combination) leaves
// one table read per shift term:
//   M2M  Mh'_a = sum_{g <= a} (4^-|g| / g!) 2^-(|a| - |g|) S_{g mod 2}[a - g],
//        S_pi[d] = sum_children (-1)^{|pi & ~oct|} Mh_child[d]        (Eq. 10)
//   L2L  Fh_child[b] += sum_pi (-1)^{|pi & ~oct|} T_pi[b],
//        T_pi[b] = sum_{a >= b, (a - b) mod 2 = pi} C(a, b) 4^-|a - b| 2^-|b| Fh[a]   (Eq. 11)
#include <cmath>

#include "kernels.h"

namespace bem {

namespace {

__host__ __device__ constexpr int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ inline int midx(int a, int b, int c) {
    int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

// ---------------------------------------------------------------- P2M weights (setup, FP64)
template <bool DBL>
__global__ void k_p2m_weights(const int32_t *leaves, const int64_t *eb, const int64_t *ee, const int32_t *level,
                              const double *centre, double side, const double *q64, int64_t n_q, const double *L7,
                              const int32_t *slot, const uint8_t *se_mask, const int64_t *woff, int p,
                              const int8_t *exps, LevelP lp, double *W) {
    // per element of the leaf: the powers u_d^k / k! of its 7 rule points
    // (formed once, in LDS) and their normals and weights
    __shared__ double pw[7][3][MAX_ORDER + 1];
    __shared__ double qn[7][4];  // n1, n2, n3, wJ
    const int P = ncoef(p);
    const int b = leaves[blockIdx.x];
    const int Pb = lp.P[level[b]];  // rows past the leaf's order stay zero
    const double rho = ldexp(side, -level[b]), irho = 1.0 / rho;
    const double cc[3] = {centre[3 * b], centre[3 * b + 1], centre[3 * b + 2]};
    const int64_t off = woff[blockIdx.x];
    const int a = threadIdx.x;  // one coefficient per thread (blockDim >= P)
    const int e0 = a < P ? exps[3 * a] : 0, e1 = a < P ? exps[3 * a + 1] : 0, e2 = a < P ? exps[3 * a + 2] : 0;
    for (int64_t e = eb[b]; e < ee[b]; e++) {
        __syncthreads();  // the previous element's tables have been read
        if (threadIdx.x < 21) {
            const int q = threadIdx.x / 3, d = threadIdx.x % 3;
            const double u = (q64[d * n_q + 7 * e + q] - cc[d]) * irho;
            pw[q][d][0] = 1.0;
            for (int k = 1; k <= p; k++) pw[q][d][k] = pw[q][d][k - 1] * u / k;
        } else if (threadIdx.x < 28) {
            const int q = threadIdx.x - 21;
            const int64_t qi = 7 * e + q;
            qn[q][0] = q64[4 * n_q + qi];
            qn[q][1] = q64[5 * n_q + qi];
            qn[q][2] = q64[6 * n_q + qi];
            qn[q][3] = q64[3 * n_q + qi];
        }
        __syncthreads();
        if (a >= Pb) continue;
        double phi[7];
        for (int q = 0; q < 7; q++) {
            const double *p0 = pw[q][0], *p1 = pw[q][1], *p2 = pw[q][2];
            double v;
            if (!DBL) {
                v = p0[e0] * p1[e1] * p2[e2];
            } else {
                v = 0.0;
                if (e0) v += qn[q][0] * p0[e0 - 1] * p1[e1] * p2[e2];
                if (e1) v += qn[q][1] * p0[e0] * p1[e1 - 1] * p2[e2];
                if (e2) v += qn[q][2] * p0[e0] * p1[e1] * p2[e2 - 1];
                v *= irho;
            }
            phi[q] = v * qn[q][3];
        }
        const int mk = se_mask ? se_mask[e] : 0x3f;  // literal tree: the piece's own slots
        for (int j = 0; j < 6; j++) {
            if (!(mk >> j & 1)) continue;
            double w = 0.0;
            for (int q = 0; q < 7; q++) w += L7[6 * q + j] * phi[q];
            W[(off + slot[6 * e + j]) * P + a] += w;
        }
    }
}

template <class R>
__global__ void k_to_r(const double *in, int64_t n, R *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (R)in[i];
}

// ---------------------------------------------------------------- P2M apply
template <class V, class R, class XV>
__global__ void k_p2m_apply(const int32_t *leaves, const int64_t *woff, const int32_t *wdof, const R *W, int P,
                            const XV *x, int64_t n_dof, V *mom, int64_t n_box) {
    far_field_priority();
    __shared__ V xs[256];
    const int b = leaves[blockIdx.x], rhs = blockIdx.y;
    const int64_t o0 = woff[blockIdx.x], o1 = woff[blockIdx.x + 1];
    const XV *xr = x + (int64_t)rhs * n_dof;
    V acc[2] = {V(0.0), V(0.0)};
    for (int64_t ub = o0; ub < o1; ub += 256) {
        const int nu = (int)min<int64_t>(256, o1 - ub);
        __syncthreads();
        for (int i = threadIdx.x; i < nu; i += blockDim.x) xs[i] = vcast<V>(xr[wdof[ub + i]]);
        __syncthreads();
        for (int r = 0; r < 2; r++) {
            const int a = threadIdx.x + r * blockDim.x;
            if (a >= P) break;
            V sacc = acc[r];
            // batches of 16 weight rows, all loads of a batch in flight together
            for (int i0 = 0; i0 < nu; i0 += 16) {
                R wv[16];
#pragma unroll
                for (int i = 0; i < 16; i++) wv[i] = i0 + i < nu ? W[(ub + i0 + i) * P + a] : R(0);
#pragma unroll
                for (int i = 0; i < 16; i++)
                    if (i0 + i < nu) sacc += xs[i0 + i] * wv[i];
            }
            acc[r] = sacc;
        }
    }
    for (int r = 0; r < 2; r++) {
        const int a = threadIdx.x + r * blockDim.x;
        if (a < P) mom[((int64_t)rhs * n_box + b) * P + a] = acc[r];
    }
}

// ---------------------------------------------------------------- M2M / L2L
// Children sit at c_parent + (rho/4) s with s in {-1, 1}^3.  With parity
// class pi (the parities of the shift multi-index g), the sign of a child's
// term is (-1)^popc(pi & m), m = the child's complemented octant bits, so the
// eight parity sums of the children are the Walsh-Hadamard transform over m
// of the children's values, and a parent's eight per-parity terms go back to
// the children by the same transform.  An 8-lane group computes it with three
// butterfly shuffles: lane j ends holding the transform at index j.
template <class V>
__device__ inline V wht8(V v, int j) {
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
        V u;
        if constexpr (std::is_same<V, float>::value || std::is_same<V, double>::value) {
            u = __shfl_xor(v, o, 64);
        } else {
            u.re = __shfl_xor(v.re, o, 64);
            u.im = __shfl_xor(v.im, o, 64);
        }
        v = (j & o) ? u - v : v + u;
    }
    return v;
}

template <class V>
__device__ inline V sum8(V v) {
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
        if constexpr (std::is_same<V, float>::value || std::is_same<V, double>::value) {
            v += __shfl_xor(v, o, 64);
        } else {
            v.re += __shfl_xor(v.re, o, 64);
            v.im += __shfl_xor(v.im, o, 64);
        }
    }
    return v;
}

// grid (parents, coefficient groups of 32, rhs); block 256 = 32 coefficient
// slots x 8 lanes.  The children's moments are all loaded at once and
// transformed into the eight parity sums S[pi] (LDS); then each lane sums the
// shift terms of one parity class for a coefficient of the block's group and
// the eight lanes are added by shuffles.
template <class V, class R>
__global__ void __launch_bounds__(256) k_m2m(const int32_t *boxes, const int32_t *child_begin, const int32_t *nchild,
                                             const uint64_t *prefix, int p, int Pout, const int8_t *exps, V *mom,
                                             int64_t n_box) {
    far_field_priority();
    constexpr int NIT = (ncoef(MAX_ORDER) + 31) / 32;
    extern __shared__ unsigned char smem[];
    const int P = ncoef(p);
    V *S = (V *)smem;                // [8][P] parity sums of the children
    R *c4 = (R *)(S + 8 * P);        // 4^-k / k!
    R *p2 = c4 + (MAX_ORDER + 1);    // 2^-k
    __shared__ int cof[8];           // child by complemented octant bits, -1 if absent
    const int b = boxes[blockIdx.x], rhs = blockIdx.z;
    const int tid = threadIdx.x, j = tid & 7, grp = tid >> 3;
    V *base = mom + (int64_t)rhs * n_box * P;
    if (tid < 8) {
        const int nc = nchild[b], cb = child_begin[b];
        // each octant holds at most one child: gather the child whose bits complement to tid
        int who = -1;
        for (int ch = 0; ch < nc; ch++)
            if (((~(int)(prefix[cb + ch] & 7u)) & 7) == tid) who = cb + ch;
        cof[tid] = who;
    }
    if (tid <= p) {
        double fct = 1.0;
        for (int k = 2; k <= tid; k++) fct *= k;
        c4[tid] = (R)(ldexp(1.0, -2 * tid) / fct);
        p2[tid] = (R)ldexp(1.0, -tid);
    }
    __syncthreads();
    const int cj = cof[j];
    V x[NIT];
#pragma unroll
    for (int it = 0; it < NIT; it++) {
        const int d = grp + 32 * it;
        x[it] = (cj >= 0 && d < P) ? base[(int64_t)cj * P + d] : V(0.0);
    }
#pragma unroll
    for (int it = 0; it < NIT; it++) {
        const int d = grp + 32 * it;
        if (32 * it < P) {  // uniform: the whole group takes part in the shuffles
            const V s = wht8(x[it], j);
            if (d < P) S[j * P + d] = s;
        }
    }
    __syncthreads();
    const int pi = j, p0 = (pi >> 2) & 1, p1 = (pi >> 1) & 1, p2b = pi & 1;
    {
        const int a = blockIdx.y * 32 + grp;
        V acc = V(0.0);
        if (a < P) {
            const int a0 = exps[3 * a], a1 = exps[3 * a + 1], a2 = exps[3 * a + 2], na = a0 + a1 + a2;
            for (int g0 = p0; g0 <= a0; g0 += 2)
                for (int g1 = p1; g1 <= a1; g1 += 2)
                    for (int g2 = p2b; g2 <= a2; g2 += 2) {
                        const R mag = c4[g0] * c4[g1] * c4[g2] * p2[na - g0 - g1 - g2];
                        acc += S[pi * P + midx(a0 - g0, a1 - g1, a2 - g2)] * mag;
                    }
        }
        acc = sum8(acc);
        // terms past the parent's order (Pout coefficients) are not kept
        if (a < P && pi == 0) base[(int64_t)b * P + a] = a < Pout ? acc : V(0.0);
    }
}

// grid (parents, coefficient groups of 32, rhs); block 256 = 32 coefficients x
// 8 parity classes; each lane sums the parent's terms of one parity class,
// the group's transform gives lane j the value of the child with
// complemented octant bits j, and every lane updates its child at once.
template <class V, class R>
__global__ void __launch_bounds__(256) k_l2l(const int32_t *boxes, const int32_t *child_begin, const int32_t *nchild,
                                             const uint64_t *prefix, const int64_t *tb, const int64_t *te, int p,
                                             int Pc, const int8_t *exps, V *loc, int64_t n_box) {
    far_field_priority();
    extern __shared__ unsigned char smem[];
    const int P = ncoef(p);
    V *F = (V *)smem;
    R *q4 = (R *)(F + P);            // 4^-k
    R *bn = q4 + (MAX_ORDER + 1);    // binomials [p+1][p+1]
    __shared__ int cof[8];           // wanted child by complemented octant bits, -1 if none
    const int b = boxes[blockIdx.x], rhs = blockIdx.z;
    const int tid = threadIdx.x;
    V *base = loc + (int64_t)rhs * n_box * P;
    for (int i = tid; i < P; i += blockDim.x) F[i] = base[(int64_t)b * P + i];
    if (tid <= p) q4[tid] = (R)ldexp(1.0, -2 * tid);
    for (int i = tid; i < (p + 1) * (p + 1); i += blockDim.x) {
        const int n = i / (p + 1), k = i % (p + 1);
        double v = 0.0;
        if (k <= n) {
            v = 1.0;
            for (int j = 1; j <= k; j++) v = v * (n - k + j) / j;
        }
        bn[i] = (R)v;
    }
    if (tid < 8) {
        const int nc = nchild[b], cb = child_begin[b];
        int who = -1;
        for (int ch = 0; ch < nc; ch++) {
            const int c = cb + ch;
            if (((~(int)(prefix[c] & 7u)) & 7) == tid && te[c] > tb[c]) who = c;
        }
        cof[tid] = who;
    }
    __syncthreads();
    const int bi = blockIdx.y * 32 + (tid >> 3), pi = tid & 7;
    const int cj = cof[pi];
    V old = V(0.0);
    if (bi < P && cj >= 0) old = base[(int64_t)cj * P + bi];  // in flight while the terms are summed
    V T = V(0.0);
    if (bi < P) {
        const int b0 = exps[3 * bi], b1 = exps[3 * bi + 1], b2 = exps[3 * bi + 2];
        const int p0 = (pi >> 2) & 1, p1 = (pi >> 1) & 1, p2 = pi & 1;
        for (int a0 = b0 + p0; a0 <= p; a0 += 2)
            for (int a1 = b1 + p1; a0 + a1 <= p; a1 += 2)
                for (int a2 = b2 + p2; a0 + a1 + a2 <= p; a2 += 2) {
                    const R mag = bn[a0 * (p + 1) + b0] * bn[a1 * (p + 1) + b1] * bn[a2 * (p + 1) + b2] *
                                  q4[a0 - b0] * q4[a1 - b1] * q4[a2 - b2];
                    T += F[midx(a0, a1, a2)] * mag;
                }
        T = T * (R)ldexp(1.0, -(b0 + b1 + b2));
    }
    const V v = wht8(T, pi);
    // the children keep the terms of their own order (Pc coefficients)
    if (bi < Pc && cj >= 0) base[(int64_t)cj * P + bi] = old + v;
}

}  // namespace

// ---------------------------------------------------------------- setup
LevelP level_p(const bem_tree &t) {
    LevelP lp{};
    for (int l = 0; l <= MAXLEV; l++) {
        int L = t.order;
        if (t.order_min > 0) L = std::min(t.order, t.order_min + std::max(0, t.max_level - l));
        lp.P[l] = ncoef(L);
    }
    return lp;
}

void build_pass_tables(bem_tree &t) {
    if (t.pass.built) return;
    Ctx &c = *t.ctx;
    fmm_tables(t);
    plan_fmm(t);
    SetupTimer st_(c, "P2M weights and L2P monomials");
    FmmTables &T = *t.tables;
    const int p = t.order, P = T.P;
    // DOF slots of each source leaf
    std::vector<int32_t> sed = t.se_dofs.download(6 * t.n_el);
    std::vector<int32_t> leaves = t.leaf_ids.download(t.n_leaf_src);
    std::vector<int64_t> woff(leaves.size() + 1, 0);
    std::vector<int32_t> wdof, slot(6 * t.n_el, 0);
    // literal tree: a piece contributes through its own slots only
    const std::vector<uint8_t> mk = t.se_mask.p ? t.se_mask.download(t.n_el) : std::vector<uint8_t>(t.n_el, 0x3f);
    for (size_t i = 0; i < leaves.size(); i++) {
        const int b = leaves[i];
        std::vector<int32_t> u;
        for (int64_t e = t.h_eb[b]; e < t.h_ee[b]; e++)
            for (int j = 0; j < 6; j++)
                if (mk[e] >> j & 1) u.push_back(sed[6 * e + j]);
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        for (int64_t e = t.h_eb[b]; e < t.h_ee[b]; e++)
            for (int j = 0; j < 6; j++)
                if (mk[e] >> j & 1)
                    slot[6 * e + j] = (int32_t)(std::lower_bound(u.begin(), u.end(), sed[6 * e + j]) - u.begin());
        wdof.insert(wdof.end(), u.begin(), u.end());
        woff[i + 1] = (int64_t)wdof.size();
    }
    PassTables &pt = t.pass;
    pt.n_w = (int64_t)wdof.size();
    pt.woff.alloc(&c, woff.size());
    pt.woff.upload(woff.data(), woff.size());
    pt.wdof.alloc(&c, wdof.size());
    pt.wdof.upload(wdof.data(), wdof.size());
    DBuf<int32_t> dslot;
    dslot.alloc(&c, slot.size());
    dslot.upload(slot.data(), slot.size());
    const size_t nw = (size_t)pt.n_w * P;
    const unsigned wbs = (unsigned)std::max(192, (P + 63) / 64 * 64);  // one thread per coefficient
    const LevelP lp = level_p(t);
    for (int dbl = 0; dbl < 2; dbl++) {
        pt.W64[dbl].alloc(&c, nw);
        pt.W64[dbl].zero();
        pt.W32[dbl].alloc(&c, nw);
        if (t.n_leaf_src) {
            if (dbl)
                k_p2m_weights<true><<<(unsigned)t.n_leaf_src, wbs, 0, c.stream>>>(
                    t.leaf_ids.p, t.eb.p, t.ee.p, t.level.p, t.centre.p, t.side, t.q64.p, t.n_q, t.L7.p, dslot.p,
                    t.se_mask.p, pt.woff.p, p, T.exps.p, lp, pt.W64[dbl].p);
            else
                k_p2m_weights<false><<<(unsigned)t.n_leaf_src, wbs, 0, c.stream>>>(
                    t.leaf_ids.p, t.eb.p, t.ee.p, t.level.p, t.centre.p, t.side, t.q64.p, t.n_q, t.L7.p, dslot.p,
                    t.se_mask.p, pt.woff.p, p, T.exps.p, lp, pt.W64[dbl].p);
            BEM_LAUNCH_CHECK();
        }
        k_to_r<float><<<nblocks(nw, 256), 256, 0, c.stream>>>(pt.W64[dbl].p, nw, pt.W32[dbl].p);
        BEM_LAUNCH_CHECK();
    }
    c.sync();
    pt.built = true;
}

// ---------------------------------------------------------------- launchers
template <class V, class R, class XV>
void p2m_apply(bem_tree &t, bool dbl, int nrhs, const XV *x, V *mom) {
    if (!t.n_leaf_src) return;
    Ctx &c = *t.ctx;
    const int P = t.tables->P;
    const R *W = std::is_same<R, float>::value ? (const R *)t.pass.W32[dbl].p : (const R *)t.pass.W64[dbl].p;
    dim3 g((unsigned)t.n_leaf_src, nrhs);
    k_p2m_apply<V, R, XV><<<g, 192, 0, c.stream>>>(t.leaf_ids.p, t.pass.woff.p, t.pass.wdof.p, W, P, x, t.n_tgt,
                                                   mom, t.n_box);
    BEM_LAUNCH_CHECK();
}

template <class V, class R>
void m2m_apply(bem_tree &t, int nrhs, V *mom, int top) {
    Ctx &c = *t.ctx;
    const int p = t.order, P = t.tables->P;
    const size_t sh = sizeof(V) * 8 * P + sizeof(R) * 2 * (MAX_ORDER + 1);
    const LevelP lp = level_p(t);
    for (int l = t.max_level - 1; l >= (top < 0 ? t.m2m_top : top); l--) {
        int64_t nb = (int64_t)t.m2m_level_boxes[l].size();
        if (!nb) continue;
        dim3 g((unsigned)nb, (P + 31) / 32, nrhs);
        k_m2m<V, R><<<g, 256, sh, c.stream>>>(t.d_m2m_level_boxes[l].p, t.child_begin.p, t.nchild.p, t.prefix.p, p,
                                              lp.P[l], t.tables->exps.p, mom, t.n_box);
        BEM_LAUNCH_CHECK();
    }
}

template <class V, class R>
void l2l_apply(bem_tree &t, int nrhs, V *loc) {
    Ctx &c = *t.ctx;
    const int p = t.order, P = t.tables->P;
    const size_t sh = sizeof(V) * P + sizeof(R) * ((MAX_ORDER + 1) + (p + 1) * (p + 1));
    const LevelP lp = level_p(t);
    for (int l = t.l2l_top; l < t.max_level; l++) {
        int64_t nb = (int64_t)t.l2l_level_boxes[l].size();
        if (!nb) continue;
        dim3 g((unsigned)nb, (P + 31) / 32, nrhs);
        k_l2l<V, R><<<g, 256, sh, c.stream>>>(t.d_l2l_level_boxes[l].p, t.child_begin.p, t.nchild.p, t.prefix.p,
                                              t.tb.p, t.te.p, p, lp.P[l + 1], t.tables->exps.p, loc, t.n_box);
        BEM_LAUNCH_CHECK();
    }
}

#define BEM_PASSES(V, R, XV)                                                   \
    template void p2m_apply<V, R, XV>(bem_tree &, bool, int, const XV *, V *); \
    template void m2m_apply<V, R>(bem_tree &, int, V *, int);                  \
    template void l2l_apply<V, R>(bem_tree &, int, V *);
BEM_PASSES(double, double, double)
BEM_PASSES(float, float, double)
BEM_PASSES(cx<double>, double, cx<double>)
BEM_PASSES(cx<float>, float, cx<double>)

}  // namespace bem
