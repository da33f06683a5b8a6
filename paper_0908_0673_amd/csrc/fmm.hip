// The fast matrix product of Section 3.6 and the direct product it is
// checked against (Section 2.1), templated on the real type R (double for
// the FP64 path, float for the mixed path) and the value type V (R for
// Laplace, cx<R> for Helmholtz).
//
// Expansions are stored scaled by the box side rho of their level:
//   moments  Mh_a = M_a / (a! rho^|a|),  M_a = sum_q s_q (y_q - c)^a   (Eqs. 6-8)
//   locals   Fh_b = F_b rho^|b|,         f(x) = sum_b F_b (x - c)^b     (Eq. 9)
// so that every stored number is O(1) whatever the level, the child-parent
// shifts (Eqs. 10, 11) become eight fixed matrices (one per octant; the
// child-centre offset is a quarter of the parent side on each axis), and the
// multipole-to-local product needs the derivatives of G only at the
// normalised separation r / rho with wavenumber k rho.
//
//   strengths  s_q = wJ_q sum_a L_a(q) x_dof(a)             (7-point rule)
//   P2M        leaves: moments of their own points; the double layer uses
//              the moment of n . grad_y of each monomial
//   M2M        levels bottom-up, Eq. (10)
//   M2L        every box, its interaction list, Eq. (9) read as
//              F_b = sum_a (-1)^|a| d^(a+b)G M_a / (a! b!), derivatives by the
//              radial recursion and Eq. (12) (Section 3.3)
//   L2L        levels top-down, Eq. (11) with its binomial factors
//   L2P        local expansion at each target of each leaf
//   P2P        7-point sums over the near-list boxes' points, tiles in LDS
//   correction sparse (accurate - 7-point) terms, free term, combination (FP64)
#include <cmath>
#include <type_traits>

#include "greens.h"
#include "kernels.h"

namespace bem {

namespace {

__host__ __device__ inline int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ inline int midx(int a, int b, int c) {
    int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

template <bool C, class R> using val_t = typename std::conditional<C, cx<R>, R>::type;

// ---------------------------------------------------------------- strengths
template <class V, class R, class XV>
__global__ void k_strength(const XV *x, int64_t n_dof, const int32_t *se_dofs, const R *wj, int64_t n_q,
                           const double *L7 /* [7][6] */, V *s) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    if (i >= n_q) return;
    int64_t se = i / 7;
    int q = (int)(i % 7);
    const XV *xr = x + (int64_t)rhs * n_dof;
    XV acc = XV(0.0);
    for (int a = 0; a < 6; a++) acc += xr[se_dofs[6 * se + a]] * L7[6 * q + a];
    s[(int64_t)rhs * n_q + i] = vcast<V>(acc) * wj[i];
}

// ---------------------------------------------------------------- P2M
// one 64-thread block per source leaf; lanes own coefficients, points in batches of 64
template <class V, class R, bool DBL>
__global__ void k_p2m(const int32_t *boxes, const int64_t *eb, const int64_t *ee, const int32_t *level,
                      const double *centre, double side, const double *q64, const R *q, int64_t n_q, const V *s,
                      int p, const int8_t *exps, V *mom, int64_t n_box) {
    extern __shared__ unsigned char smem[];
    const int np1 = p + 1, P = ncoef(p);
    R *pw = (R *)smem;                       // [64][3][np1]  u^k / k!
    V *sv = (V *)(pw + 64 * 3 * np1);        // [64] strength (/rho for the double layer)
    R *nv = (R *)(sv + 64);                  // [64][3] normals
    const int b = boxes[blockIdx.x], rhs = blockIdx.y, lane = threadIdx.x;
    const double rho = ldexp(side, -level[b]);
    const R irho = (R)(1.0 / rho);
    const double irho64 = 1.0 / rho;
    const double cx0 = centre[3 * b], cx1 = centre[3 * b + 1], cx2 = centre[3 * b + 2];
    constexpr int MAXC = 5;  // up to ncoef(10) = 286 coefficients per 64 lanes
    V acc[MAXC];
    int ea[MAXC][3];
    for (int j = 0; j < MAXC; j++) {
        acc[j] = V(0.0);
        int a = lane + 64 * j;
        if (a < P) { ea[j][0] = exps[3 * a]; ea[j][1] = exps[3 * a + 1]; ea[j][2] = exps[3 * a + 2]; }
    }
    const int64_t q0 = 7 * eb[b], q1 = 7 * ee[b];
    const V *sr = s + (int64_t)rhs * n_q;
    for (int64_t base = q0; base < q1; base += 64) {
        int64_t qi = base + lane;
        if (qi < q1) {
            R u[3] = {(R)((q64[qi] - cx0) * irho64), (R)((q64[n_q + qi] - cx1) * irho64),
                      (R)((q64[2 * n_q + qi] - cx2) * irho64)};
            for (int d = 0; d < 3; d++) {
                R v = 1;
                pw[(lane * 3 + d) * np1] = v;
                for (int k = 1; k <= p; k++) {
                    v = v * u[d] / (R)k;
                    pw[(lane * 3 + d) * np1 + k] = v;
                }
            }
            V sq = sr[qi];
            if (DBL) {
                sq = sq * irho;
                for (int d = 0; d < 3; d++) nv[3 * lane + d] = q[(4 + d) * n_q + qi];
            }
            sv[lane] = sq;
        } else {
            sv[lane] = V(0.0);
            for (int d = 0; d < 3; d++) {
                for (int k = 0; k <= p; k++) pw[(lane * 3 + d) * np1 + k] = 0;
                nv[3 * lane + d] = 0;
            }
        }
        __syncthreads();
        int nb = (int)min<int64_t>(64, q1 - base);
        for (int j = 0; j < MAXC; j++) {
            int a = lane + 64 * j;
            if (a >= P) break;
            const int e0 = ea[j][0], e1 = ea[j][1], e2 = ea[j][2];
            V m = acc[j];
            for (int i = 0; i < nb; i++) {
                const R *px = pw + (i * 3) * np1, *py = px + np1, *pz = py + np1;
                R mono;
                if (!DBL) {
                    mono = px[e0] * py[e1] * pz[e2];
                } else {
                    mono = 0;
                    if (e0) mono += nv[3 * i] * px[e0 - 1] * py[e1] * pz[e2];
                    if (e1) mono += nv[3 * i + 1] * px[e0] * py[e1 - 1] * pz[e2];
                    if (e2) mono += nv[3 * i + 2] * px[e0] * py[e1] * pz[e2 - 1];
                }
                m += sv[i] * mono;
            }
            acc[j] = m;
        }
        __syncthreads();
    }
    V *out = mom + ((int64_t)rhs * n_box + b) * P;
    for (int j = 0; j < MAXC; j++) {
        int a = lane + 64 * j;
        if (a < P) out[a] = acc[j];
    }
}

// ---------------------------------------------------------------- M2M / L2L
// out[box] (+)= sum over inputs of table(octant) . in ; threads own target coefficients.
// M2M: boxes are parents, inputs their children (octant = child prefix & 7).
// L2L: boxes are children, the input is the parent (octant = own prefix & 7).
template <class V, class R, bool UP>
__global__ void k_shift(const int32_t *boxes, const int32_t *parent, const int32_t *child_begin, const int32_t *nchild,
                        const uint64_t *prefix, int P, const int32_t *ptr, const int16_t *src, const R *coef, int nnz,
                        V *buf, int64_t n_box) {
    extern __shared__ unsigned char smem[];
    V *in = (V *)smem;
    const int b = boxes[blockIdx.x], rhs = blockIdx.y;
    V *base = buf + (int64_t)rhs * n_box * P;
    V acc = V(0.0);
    const int a = threadIdx.x;
    int ninp = UP ? nchild[b] : 1;
    for (int c = 0; c < ninp; c++) {
        int from = UP ? child_begin[b] + c : parent[b];
        int oct = (int)((UP ? prefix[from] : prefix[b]) & 7u);
        for (int j = threadIdx.x; j < P; j += blockDim.x) in[j] = base[(int64_t)from * P + j];
        __syncthreads();
        if (a < P) {
            const R *cf = coef + (int64_t)oct * nnz;
            for (int t = ptr[a]; t < ptr[a + 1]; t++) acc += in[src[t]] * cf[t];
        }
        __syncthreads();
    }
    if (a < P) {
        if (UP) base[(int64_t)b * P + a] = acc;
        else base[(int64_t)b * P + a] += acc;
    }
}

// ---------------------------------------------------------------- L2P
template <class V, class R>
__global__ void k_l2p(const int32_t *boxes, const int64_t *tb, const int64_t *te, const int32_t *level,
                      const double *centre, double side, const double *t, int64_t n_tgt, int p, const V *loc,
                      int64_t n_box, V *y) {
    extern __shared__ unsigned char smem[];
    V *F = (V *)smem;
    const int b = boxes[blockIdx.x], rhs = blockIdx.y, P = ncoef(p);
    for (int j = threadIdx.x; j < P; j += blockDim.x) F[j] = loc[((int64_t)rhs * n_box + b) * P + j];
    __syncthreads();
    const double irho = 1.0 / ldexp(side, -level[b]);
    for (int64_t i = tb[b] + threadIdx.x; i < te[b]; i += blockDim.x) {
        R u0 = (R)((t[i] - centre[3 * b]) * irho), u1 = (R)((t[n_tgt + i] - centre[3 * b + 1]) * irho),
          u2 = (R)((t[2 * n_tgt + i] - centre[3 * b + 2]) * irho);
        V acc = V(0.0);
        R xa = 1;
        for (int a = 0; a <= p; a++) {
            R xab = xa;
            for (int bb = 0; bb <= p - a; bb++) {
                R xabc = xab;
                for (int c = 0; c <= p - a - bb; c++) {
                    acc += F[midx(a, bb, c)] * xabc;
                    xabc *= u2;
                }
                xab *= u1;
            }
            xa *= u0;
        }
        y[(int64_t)rhs * n_tgt + i] = acc;
    }
}

// ---------------------------------------------------------------- P2P
constexpr int P2P_BS = 256;
constexpr int P2P_TILE = 256;
constexpr int P2P_CH = 256;  // near-list entries per chunk

__device__ inline float inv_sqrt(float v) { return rsqrtf(v); }
__device__ inline double inv_sqrt(double v) { return 1.0 / sqrt(v); }

// One block per work item (a target leaf and up to 64 of its targets).  The
// near-list boxes' points are streamed through LDS tiles; each wave takes a
// quarter of a tile, its lanes split into (target, sub-stream) pairs.  The
// target-source difference is formed in FP64 (the coordinates are FP64) and
// only then rounded to R, so that close pairs keep their relative accuracy in
// the mixed path; per-tile partial sums in R are added into an FP64 total.
template <class V, class R, bool DBL, bool HELM>
__global__ void __launch_bounds__(P2P_BS) k_p2p(const int32_t *wi_box, const int32_t *wi_t0, const int32_t *wi_nt,
                                                const int64_t *nptr, const int32_t *nidx, const int64_t *eb,
                                                const int64_t *ee, const double *q64, const R *q, int64_t n_q,
                                                const V *s, const double *t64, int64_t n_tgt, R k, V *y) {
    using VD = typename std::conditional<HELM, cx<double>, double>::type;
    __shared__ int64_t pref[P2P_CH + 1];
    __shared__ int64_t qbeg[P2P_CH];
    __shared__ double sx[P2P_TILE], sy[P2P_TILE], sz[P2P_TILE];
    __shared__ R snx[DBL ? P2P_TILE : 1], sny[DBL ? P2P_TILE : 1], snz[DBL ? P2P_TILE : 1];
    __shared__ V ss[P2P_TILE];
    __shared__ VD red[P2P_BS / 64][64];
    const int w = blockIdx.x, rhs = blockIdx.y;
    const int b = wi_box[w], t0 = wi_t0[w], nt = wi_nt[w];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int tpw = 1;
    while (tpw < nt) tpw <<= 1;
    const int nsub = 64 / tpw, tl = lane % tpw, sub = lane / tpw;
    const int64_t ti = t0 + (tl < nt ? tl : 0);
    const double x0 = t64[ti], x1 = t64[n_tgt + ti], x2 = t64[2 * n_tgt + ti];
    const V *sr = s + (int64_t)rhs * n_q;
    VD total = VD(0.0);
    const int64_t j0 = nptr[b], j1 = nptr[b + 1];
    for (int64_t cb = j0; cb < j1; cb += P2P_CH) {
        const int nc = (int)min<int64_t>(P2P_CH, j1 - cb);
        if (tid < nc) {
            int32_t nb_ = nidx[cb + tid];
            qbeg[tid] = 7 * eb[nb_];
            pref[tid + 1] = 7 * (ee[nb_] - eb[nb_]);
        }
        if (tid == 0) pref[0] = 0;
        __syncthreads();
        if (tid == 0)
            for (int i = 1; i <= nc; i++) pref[i] += pref[i - 1];
        __syncthreads();
        const int64_t total_pts = pref[nc];
        for (int64_t tb0 = 0; tb0 < total_pts; tb0 += P2P_TILE) {
            const int64_t f = tb0 + tid;
            if (f < total_pts) {
                int lo = 0, hi = nc - 1;
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (pref[mid] <= f) lo = mid; else hi = mid - 1;
                }
                const int64_t qi = qbeg[lo] + (f - pref[lo]);
                sx[tid] = q64[qi];
                sy[tid] = q64[n_q + qi];
                sz[tid] = q64[2 * n_q + qi];
                if (DBL) {
                    snx[tid] = q[4 * n_q + qi];
                    sny[tid] = q[5 * n_q + qi];
                    snz[tid] = q[6 * n_q + qi];
                }
                ss[tid] = sr[qi];
            }
            __syncthreads();
            const int nin = (int)min<int64_t>(P2P_TILE, total_pts - tb0);
            const int kb = wave * 64, ke = min(nin, kb + 64);
            V acc = V(0.0);
            for (int kk = kb + sub; kk < ke; kk += nsub) {
                const R d0 = (R)(x0 - sx[kk]), d1 = (R)(x1 - sy[kk]), d2 = (R)(x2 - sz[kk]);
                const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const R ir = inv_sqrt(r2);
                const R g = (R)kInv4Pi * ir;
                if constexpr (HELM) {
                    const R kr = k * r2 * ir;
                    R sn, cs;
                    vsincos(kr, &sn, &cs);
                    cx<R> kv;
                    if (DBL) {
                        const R f = g * (d0 * snx[kk] + d1 * sny[kk] + d2 * snz[kk]) * ir * ir;
                        kv = cx<R>(f * (cs + kr * sn), f * (sn - kr * cs));
                    } else {
                        kv = cx<R>(g * cs, g * sn);
                    }
                    acc += kv * ss[kk];
                } else {
                    if (DBL) acc += ss[kk] * (g * (d0 * snx[kk] + d1 * sny[kk] + d2 * snz[kk]) * ir * ir);
                    else acc += ss[kk] * g;
                }
            }
            total += vcast<VD>(acc);
            __syncthreads();
        }
    }
    // reduce over sub-streams of the wave (lanes tl, tl + tpw, ...)
    for (int o = 32; o >= tpw; o >>= 1) {
        if constexpr (HELM) {
            total.re += __shfl_xor(total.re, o, 64);
            total.im += __shfl_xor(total.im, o, 64);
        } else {
            total += __shfl_xor(total, o, 64);
        }
    }
    if (sub == 0) red[wave][tl] = total;
    __syncthreads();
    if (tid < nt) {
        VD v = red[0][tid];
        for (int wv = 1; wv < P2P_BS / 64; wv++) v += red[wv][tid];
        V *dst = y + (int64_t)rhs * n_tgt + t0 + tid;
        *dst = vcast<V>(vcast<VD>(*dst) + v);
    }
}

// ---------------------------------------------------------------- direct (FP64)
template <class V, bool DBL, bool HELM>
__global__ void __launch_bounds__(256) k_direct(const double *q, int64_t n_q, const V *s, const double *t,
                                                int64_t n_tgt, double k, V *y) {
    __shared__ double sx[256], sy[256], sz[256], snx[256], sny[256], snz[256];
    __shared__ V ss[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int rhs = blockIdx.y;
    const int64_t ii = i < n_tgt ? i : n_tgt - 1;
    const double x0 = t[ii], x1 = t[n_tgt + ii], x2 = t[2 * n_tgt + ii];
    const V *sr = s + (int64_t)rhs * n_q;
    V acc = V(0.0);
    for (int64_t base = 0; base < n_q; base += 256) {
        int64_t j = base + threadIdx.x;
        if (j < n_q) {
            sx[threadIdx.x] = q[j]; sy[threadIdx.x] = q[n_q + j]; sz[threadIdx.x] = q[2 * n_q + j];
            snx[threadIdx.x] = q[4 * n_q + j]; sny[threadIdx.x] = q[5 * n_q + j]; snz[threadIdx.x] = q[6 * n_q + j];
            ss[threadIdx.x] = sr[j];
        }
        __syncthreads();
        int m = (int)min<int64_t>(256, n_q - base);
        for (int kk = 0; kk < m; kk++) {
            double d0 = x0 - sx[kk], d1 = x1 - sy[kk], d2 = x2 - sz[kk];
            double r2 = d0 * d0 + d1 * d1 + d2 * d2;
            double rn = d0 * snx[kk] + d1 * sny[kk] + d2 * snz[kk];
            if constexpr (HELM) {
                cx<double> G, dG;
                green_helmholtz<double>(r2, rn, k, &G, &dG);
                acc += (DBL ? dG : G) * ss[kk];
            } else {
                double G, dG;
                green_laplace<double>(r2, rn, &G, &dG);
                acc += ss[kk] * (DBL ? dG : G);
            }
        }
        __syncthreads();
    }
    if (i < n_tgt) y[(int64_t)rhs * n_tgt + i] = acc;
}

// ---------------------------------------------------------------- correction + combine (FP64)
template <class XV, class AV>
__global__ void k_combine(int64_t n_tgt, const int32_t *tperm, const AV *yacc, const int64_t *row_ptr,
                          const int32_t *pair_elem, const int32_t *se_dofs, const XV *corr, const double *cfree,
                          const XV *x, int op, XV *y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int rhs = blockIdx.y;
    if (t >= n_tgt) return;
    const XV *xr = x + (int64_t)rhs * n_tgt;
    XV acc = vcast<XV>(yacc[(int64_t)rhs * n_tgt + t]);
    for (int64_t p = row_ptr[t]; p < row_ptr[t + 1]; p++) {
        const int32_t *dof = se_dofs + 6 * (int64_t)pair_elem[p];
        const XV *cp = corr + 6 * p;
        for (int a = 0; a < 6; a++) acc += cp[a] * xr[dof[a]];
    }
    const int64_t i = tperm[t];
    XV out;
    if (op == BEM_OP_A) out = xr[i] * cfree[i] - acc;
    else if (op == BEM_OP_RHS) out = -acc;
    else out = acc;
    y[(int64_t)rhs * n_tgt + i] = out;
}

__global__ void k_unit_strength(const double *wj, int64_t n, double *s) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) s[i] = wj[i];
}

}  // namespace

// ---------------------------------------------------------------- tables
void fmm_tables(bem_tree &t) {
    if (t.tables && t.tables->p == t.order) return;
    Ctx &c = *t.ctx;
    auto T = std::make_unique<FmmTables>();
    const int p = t.order, P = ncoef(p), P2 = ncoef(2 * p);
    T->p = p; T->P = P; T->P2 = P2;
    std::vector<int8_t> ex(3 * P2);
    for (int n = 0; n <= 2 * p; n++)
        for (int a = n; a >= 0; a--)
            for (int b = n - a; b >= 0; b--) {
                int i = midx(a, b, n - a - b);
                ex[3 * i] = (int8_t)a; ex[3 * i + 1] = (int8_t)b; ex[3 * i + 2] = (int8_t)(n - a - b);
            }
    std::vector<double> fct(2 * p + 2, 1.0);
    for (int i = 1; i < (int)fct.size(); i++) fct[i] = fct[i - 1] * i;
    std::vector<double> invf(P2);
    for (int i = 0; i < P2; i++) invf[i] = 1.0 / (fct[ex[3 * i]] * fct[ex[3 * i + 1]] * fct[ex[3 * i + 2]]);
    auto binom = [&](int n, int k) { return fct[n] / (fct[k] * fct[n - k]); };
    auto dbar = [](int oct, int d) { return ((oct >> (2 - d)) & 1) ? 0.25 : -0.25; };
    // M2M: Mh'_a = sum_{g <= a} (dbar^g / g!) 2^-|a-g| Mh_{a-g}
    std::vector<int32_t> mptr(P + 1, 0);
    std::vector<int16_t> msrc;
    std::vector<std::vector<double>> mcoef(8);
    for (int i = 0; i < P; i++) {
        int a0 = ex[3 * i], a1 = ex[3 * i + 1], a2 = ex[3 * i + 2];
        for (int g0 = 0; g0 <= a0; g0++)
            for (int g1 = 0; g1 <= a1; g1++)
                for (int g2 = 0; g2 <= a2; g2++) {
                    msrc.push_back((int16_t)midx(a0 - g0, a1 - g1, a2 - g2));
                    int rest = (a0 - g0) + (a1 - g1) + (a2 - g2);
                    for (int o = 0; o < 8; o++)
                        mcoef[o].push_back(std::pow(dbar(o, 0), g0) * std::pow(dbar(o, 1), g1) *
                                           std::pow(dbar(o, 2), g2) / (fct[g0] * fct[g1] * fct[g2]) *
                                           std::ldexp(1.0, -rest));
                }
        mptr[i + 1] = (int32_t)msrc.size();
    }
    // L2L: Fh''_b = sum_{a >= b} C(a, b) dbar^(a-b) 2^-|b| Fh_a
    std::vector<int32_t> lptr(P + 1, 0);
    std::vector<int16_t> lsrc;
    std::vector<std::vector<double>> lcoef(8);
    for (int i = 0; i < P; i++) {
        int b0 = ex[3 * i], b1 = ex[3 * i + 1], b2 = ex[3 * i + 2];
        for (int j = 0; j < P; j++) {
            int a0 = ex[3 * j], a1 = ex[3 * j + 1], a2 = ex[3 * j + 2];
            if (a0 < b0 || a1 < b1 || a2 < b2) continue;
            lsrc.push_back((int16_t)j);
            for (int o = 0; o < 8; o++)
                lcoef[o].push_back(binom(a0, b0) * binom(a1, b1) * binom(a2, b2) * std::pow(dbar(o, 0), a0 - b0) *
                                   std::pow(dbar(o, 1), a1 - b1) * std::pow(dbar(o, 2), a2 - b2) *
                                   std::ldexp(1.0, -(b0 + b1 + b2)));
        }
        lptr[i + 1] = (int32_t)lsrc.size();
    }
    T->nnz_m2m = (int)msrc.size();
    T->nnz_l2l = (int)lsrc.size();
    auto flat = [](const std::vector<std::vector<double>> &v) {
        std::vector<double> o;
        for (auto &x : v) o.insert(o.end(), x.begin(), x.end());
        return o;
    };
    auto to32 = [](const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); };
    auto m64 = flat(mcoef), l64 = flat(lcoef);
    auto m32 = to32(m64), l32 = to32(l64);
    auto if32 = to32(invf);
    T->exps.alloc(&c, ex.size()); T->exps.upload(ex.data(), ex.size());
    T->h_exps = ex;
    T->inv_fact64.alloc(&c, P2); T->inv_fact64.upload(invf.data(), P2);
    T->inv_fact32.alloc(&c, P2); T->inv_fact32.upload(if32.data(), P2);
    T->m2m_ptr.alloc(&c, P + 1); T->m2m_ptr.upload(mptr.data(), P + 1);
    T->m2m_src.alloc(&c, msrc.size()); T->m2m_src.upload(msrc.data(), msrc.size());
    T->m2m_c64.alloc(&c, m64.size()); T->m2m_c64.upload(m64.data(), m64.size());
    T->m2m_c32.alloc(&c, m32.size()); T->m2m_c32.upload(m32.data(), m32.size());
    T->l2l_ptr.alloc(&c, P + 1); T->l2l_ptr.upload(lptr.data(), P + 1);
    T->l2l_src.alloc(&c, lsrc.size()); T->l2l_src.upload(lsrc.data(), lsrc.size());
    T->l2l_c64.alloc(&c, l64.size()); T->l2l_c64.upload(l64.data(), l64.size());
    T->l2l_c32.alloc(&c, l32.size()); T->l2l_c32.upload(l32.data(), l32.size());
    c.sync();
    t.tables = std::move(T);
}

// ---------------------------------------------------------------- plan
static DBuf<int32_t> upload_i32(Ctx &c, const std::vector<int32_t> &v) {
    DBuf<int32_t> d;
    d.alloc(&c, v.size());
    d.upload(v.data(), v.size());
    return d;
}

void plan_fmm(bem_tree &t) {
    if (t.planned) return;
    Ctx &c = *t.ctx;
    std::vector<int32_t> src_leaves, tgt_leaves, m2l, wb, wt0, wnt;
    for (int64_t b = 0; b < t.n_box; b++) {
        bool has_t = t.h_te[b] > t.h_tb[b];
        if (t.h_leaf[b] && t.h_ee[b] > t.h_eb[b]) src_leaves.push_back((int32_t)b);
        if (t.h_leaf[b] && has_t) {
            tgt_leaves.push_back((int32_t)b);
            for (int64_t t0 = t.h_tb[b]; t0 < t.h_te[b]; t0 += 64) {
                wb.push_back((int32_t)b);
                wt0.push_back((int32_t)t0);
                wnt.push_back((int32_t)std::min<int64_t>(64, t.h_te[b] - t0));
            }
        }
        if (has_t && t.h_inter_ptr[b + 1] > t.h_inter_ptr[b]) m2l.push_back((int32_t)b);
    }
    t.leaf_ids = upload_i32(c, src_leaves);
    t.n_leaf_src = (int64_t)src_leaves.size();
    t.tleaf_ids = upload_i32(c, tgt_leaves);
    t.n_leaf_tgt = (int64_t)tgt_leaves.size();
    t.m2l_boxes = upload_i32(c, m2l);
    t.n_m2l_boxes = (int64_t)m2l.size();
    t.p2p_box = upload_i32(c, wb);
    t.p2p_t0 = upload_i32(c, wt0);
    t.p2p_nt = upload_i32(c, wnt);
    t.n_p2p_items = (int64_t)wb.size();
    // near-field pair count: targets x source points
    t.n_p2p_pairs = 0;
    for (int64_t b = 0; b < t.n_box; b++) {
        if (!t.h_leaf[b]) continue;
        int64_t ns = 0;
        for (int64_t j = t.h_near_ptr[b]; j < t.h_near_ptr[b + 1]; j++) {
            int32_t s = t.h_near_idx[j];
            ns += 7 * (t.h_ee[s] - t.h_eb[s]);
        }
        t.n_p2p_pairs += ns * (t.h_te[b] - t.h_tb[b]);
    }
    t.m2m_level_boxes.assign(t.max_level + 1, {});
    t.d_m2m_level_boxes.clear();
    t.d_level_boxes.clear();
    for (int l = 0; l <= t.max_level; l++) {
        std::vector<int32_t> up, down;
        for (int64_t b = t.level_off[l]; b < t.level_off[l + 1]; b++) {
            if (!t.h_leaf[b]) up.push_back((int32_t)b);
            if (l > 0 && t.h_te[b] > t.h_tb[b]) down.push_back((int32_t)b);
        }
        t.m2m_level_boxes[l] = up;
        t.d_m2m_level_boxes.push_back(upload_i32(c, up));
        t.d_level_boxes.push_back(upload_i32(c, down));
        t.h_level_down.push_back((int64_t)down.size());
    }
    c.sync();
    t.planned = true;
}

// ---------------------------------------------------------------- drivers
void direct_regular_unit_double_layer(bem_tree &t, double *out) {
    Ctx &c = *t.ctx;
    dim3 g(nblocks(t.n_tgt, 256), 1);
    k_direct<double, true, false><<<g, 256, 0, c.stream>>>(t.q64.p, t.n_q, t.q64.p + 3 * t.n_q, t.t64.p, t.n_tgt,
                                                           0.0, out);
    BEM_LAUNCH_CHECK();
}

namespace {

template <class V, class R, class XV, bool HELM>
void run_matvec(bem_tree &t, double k, int op, int method, int nrhs, const XV *x, XV *y) {
    Ctx &c = *t.ctx;
    const bool dbl = (op == BEM_OP_K || op == BEM_OP_A);
    const int64_t nq = t.n_q, nt = t.n_tgt;
    Corr &cr = get_corr(t, HELM ? BEM_HELMHOLTZ : BEM_LAPLACE, k);
    if (op == BEM_OP_A) build_free_term(t);
    M2lPlan *pl = method == BEM_FMM ? &get_m2l_plan(t, HELM ? BEM_HELMHOLTZ : BEM_LAPLACE, k) : nullptr;
    const R *q = std::is_same<R, float>::value ? (const R *)t.q32.p : (const R *)t.q64.p;
    const R *tg = std::is_same<R, float>::value ? (const R *)t.t32.p : (const R *)t.t64.p;
    // work buffers
    t.work.strength.ensure(&c, sizeof(V) * nq * nrhs);
    t.work.yacc.ensure(&c, sizeof(V) * nt * nrhs);
    V *s = (V *)t.work.strength.p;
    V *yacc = (V *)t.work.yacc.p;
    if (!t.L7.p) {
        // shape functions at the 7 rule points
        std::vector<double> L7(42);
        double rs[7], rt[7], rw[7];
        rule7(rs, rt, rw);
        for (int qq = 0; qq < 7; qq++) {
            double S_ = rs[qq], T_ = rt[qq], Z = 1.0 - S_ - T_;
            double L[6] = {Z * (2 * Z - 1), S_ * (2 * S_ - 1), T_ * (2 * T_ - 1), 4 * Z * S_, 4 * S_ * T_, 4 * T_ * Z};
            for (int a = 0; a < 6; a++) L7[6 * qq + a] = L[a];
        }
        t.L7.alloc(&c, 42);
        t.L7.upload(L7.data(), 42);
    }
    c.mark(9);
    dim3 gs(nblocks(nq, 256), nrhs);
    k_strength<V, R, XV><<<gs, 256, 0, c.stream>>>(x, nt, t.se_dofs.p, q + 3 * nq, nq, t.L7.p, s);
    BEM_LAUNCH_CHECK();
    c.mark(0);

    if (method == BEM_DIRECT) {
        if constexpr (std::is_same<R, double>::value) {
            dim3 g(nblocks(nt, 256), nrhs);
            if (dbl) k_direct<V, true, HELM><<<g, 256, 0, c.stream>>>(t.q64.p, nq, s, t.t64.p, nt, k, yacc);
            else k_direct<V, false, HELM><<<g, 256, 0, c.stream>>>(t.q64.p, nq, s, t.t64.p, nt, k, yacc);
            BEM_LAUNCH_CHECK();
            c.mark(8);
        } else {
            fail(BEM_EUNSUPPORTED, "the direct product runs in FP64 only");
        }
    } else {
        fmm_tables(t);
        plan_fmm(t);
        FmmTables &T = *t.tables;
        const int p = t.order, P = T.P, P2 = T.P2;
        const size_t nexp = (size_t)t.n_box * P * nrhs;
        t.work.mom.ensure(&c, sizeof(V) * nexp);
        t.work.loc.ensure(&c, sizeof(V) * nexp);
        V *mom = (V *)t.work.mom.p, *loc = (V *)t.work.loc.p;
        const R *mc = std::is_same<R, float>::value ? (const R *)T.m2m_c32.p : (const R *)T.m2m_c64.p;
        const R *lc = std::is_same<R, float>::value ? (const R *)T.l2l_c32.p : (const R *)T.l2l_c64.p;
        // upward pass (boxes without elements keep zero moments)
        BEM_HIP(hipMemsetAsync(mom, 0, sizeof(V) * nexp, c.stream));
        if (t.n_leaf_src) {
            dim3 g((unsigned)t.n_leaf_src, nrhs);
            size_t sh = sizeof(R) * 64 * 3 * (p + 1) + sizeof(V) * 64 + sizeof(R) * 64 * 3;
            if (dbl) k_p2m<V, R, true><<<g, 64, sh, c.stream>>>(t.leaf_ids.p, t.eb.p, t.ee.p, t.level.p, t.centre.p,
                                                                 t.side, t.q64.p, q, nq, s, p, T.exps.p, mom,
                                                                 t.n_box);
            else k_p2m<V, R, false><<<g, 64, sh, c.stream>>>(t.leaf_ids.p, t.eb.p, t.ee.p, t.level.p, t.centre.p,
                                                              t.side, t.q64.p, q, nq, s, p, T.exps.p, mom, t.n_box);
            BEM_LAUNCH_CHECK();
        }
        c.mark(1);
        const int sbs = P <= 64 ? 64 : (P <= 128 ? 128 : (P <= 192 ? 192 : 320));
        for (int l = t.max_level - 1; l >= 0; l--) {
            int64_t nb = (int64_t)t.m2m_level_boxes[l].size();
            if (!nb) continue;
            dim3 g((unsigned)nb, nrhs);
            k_shift<V, R, true><<<g, sbs, sizeof(V) * P, c.stream>>>(t.d_m2m_level_boxes[l].p, t.parent.p,
                                                                       t.child_begin.p, t.nchild.p, t.prefix.p, P,
                                                                       T.m2m_ptr.p, T.m2m_src.p, mc, T.nnz_m2m, mom,
                                                                       t.n_box);
            BEM_LAUNCH_CHECK();
        }
        c.mark(2);
        // interactions
        BEM_HIP(hipMemsetAsync(loc, 0, sizeof(V) * nexp, c.stream));
        c.mark(9);
        m2l_apply<V, R>(t, *pl, nrhs, mom, loc);
        c.mark(3);
        // downward pass
        for (int l = 1; l <= t.max_level; l++) {
            int64_t nb = t.h_level_down[l];
            if (!nb) continue;
            dim3 g((unsigned)nb, nrhs);
            k_shift<V, R, false><<<g, sbs, sizeof(V) * P, c.stream>>>(t.d_level_boxes[l].p, t.parent.p,
                                                                        t.child_begin.p, t.nchild.p, t.prefix.p, P,
                                                                        T.l2l_ptr.p, T.l2l_src.p, lc, T.nnz_l2l, loc,
                                                                        t.n_box);
            BEM_LAUNCH_CHECK();
        }
        c.mark(4);
        if (t.n_leaf_tgt) {
            dim3 g((unsigned)t.n_leaf_tgt, nrhs);
            k_l2p<V, R><<<g, 64, sizeof(V) * P, c.stream>>>(t.tleaf_ids.p, t.tb.p, t.te.p, t.level.p, t.centre.p,
                                                             t.side, t.t64.p, nt, p, loc, t.n_box, yacc);
            BEM_LAUNCH_CHECK();
        }
        c.mark(5);
        if (t.n_p2p_items) {
            dim3 g((unsigned)t.n_p2p_items, nrhs);
            if (dbl)
                k_p2p<V, R, true, HELM><<<g, P2P_BS, 0, c.stream>>>(t.p2p_box.p, t.p2p_t0.p, t.p2p_nt.p,
                                                                    t.near_ptr.p, t.near_idx.p, t.eb.p, t.ee.p,
                                                                    t.q64.p, q, nq, s, t.t64.p, nt, (R)k, yacc);
            else
                k_p2p<V, R, false, HELM><<<g, P2P_BS, 0, c.stream>>>(t.p2p_box.p, t.p2p_t0.p, t.p2p_nt.p,
                                                                     t.near_ptr.p, t.near_idx.p, t.eb.p, t.ee.p,
                                                                     t.q64.p, q, nq, s, t.t64.p, nt, (R)k, yacc);
            BEM_LAUNCH_CHECK();
        }
        c.mark(6);
    }
    // corrections and combination in FP64
    const XV *corr = (const XV *)(dbl ? cr.K.p : cr.S.p);
    dim3 g(nblocks(nt, 256), nrhs);
    k_combine<XV, V><<<g, 256, 0, c.stream>>>(nt, t.tperm.p, yacc, t.pair_ptr.p, t.pair_elem.p, t.se_dofs.p, corr,
                                             op == BEM_OP_A ? t.free_term.p : nullptr, x, op, y);
    BEM_LAUNCH_CHECK();
    c.mark(7);
}

}  // namespace

void matvec(bem_tree &t, int green, double k, int op, int method, int prec, int nrhs, const void *x, void *y) {
    if (green == BEM_HELMHOLTZ) {
        using XV = cx<double>;
        if (prec == BEM_PREC_FP64 || method == BEM_DIRECT)
            run_matvec<cx<double>, double, XV, true>(t, k, op, method, nrhs, (const XV *)x, (XV *)y);
        else
            run_matvec<cx<float>, float, XV, true>(t, k, op, method, nrhs, (const XV *)x, (XV *)y);
    } else {
        if (prec == BEM_PREC_FP64 || method == BEM_DIRECT)
            run_matvec<double, double, double, false>(t, 0.0, op, method, nrhs, (const double *)x, (double *)y);
        else
            run_matvec<float, float, double, false>(t, 0.0, op, method, nrhs, (const double *)x, (double *)y);
    }
}

}  // namespace bem
