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
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <unordered_map>

#include "greens.h"
#include "kernels.h"

namespace bem {

namespace {

__host__ __device__ constexpr int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ inline int midx(int a, int b, int c) {
    int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

template <bool C, class R> using val_t = typename std::conditional<C, cx<R>, R>::type;

// ---------------------------------------------------------------- strengths
template <class V, class R, class XV>
__global__ void k_strength(const XV *x, int64_t n_dof, const int32_t *se_dofs, const uint8_t *se_mask, const R *wj,
                           int64_t n_q, const double *L7 /* [7][6] */, V *s, uint32_t *zero, int64_t n_zero) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int rhs = blockIdx.y;
    // the same launch clears n_zero words (the expansions of the fast product)
    if (zero && rhs == 0)
        for (int64_t z = i; z < n_zero; z += (int64_t)gridDim.x * blockDim.x) zero[z] = 0u;
    if (i >= n_q) return;
    int64_t se = i / 7;
    int q = (int)(i % 7);
    const XV *xr = x + (int64_t)rhs * n_dof;
    XV acc = XV(0.0);
    if (!se_mask) {
        for (int a = 0; a < 6; a++) acc += xr[se_dofs[6 * se + a]] * L7[6 * q + a];
    } else {  // literal tree: the piece's own shape-function slots
        const int mk = se_mask[se];
        for (int a = 0; a < 6; a++)
            if (mk >> a & 1) acc += xr[se_dofs[6 * se + a]] * L7[6 * q + a];
    }
    s[(int64_t)rhs * n_q + i] = vcast<V>(acc) * wj[i];
}

// ---------------------------------------------------------------- P2P
constexpr int P2P_BS = 256;
constexpr int P2P_TILE = 256;
constexpr int P2P_CH = 256;  // near-list entries per chunk
#ifndef P2P_TPL
#define P2P_TPL 4  // targets per lane
#endif

// 1/sqrt(v) for v > 0 far from the denormal range (squared distances of
// distinct points): the hardware estimate, which is within 1 ulp in single
// precision; in double precision it is refined by two Newton steps
// y <- y + y (1/2 - (v/2) y^2), each of which squares the relative error.
__device__ inline float inv_sqrt(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ inline double inv_sqrt(double v) {
    double y = __builtin_amdgcn_rsq(v);
    const double h = 0.5 * v;
    for (int i = 0; i < 2; i++) y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

// sin and cos of x for the FP64 near field's phases k r: Cody-Waite reduction by
// the nearest multiple q of pi/2 (pi/2 split in three parts, each product
// q * part formed exactly inside an fma), Taylor polynomials of sin and cos
// on the reduced argument |r| <= pi/4 (the first omitted term is below half
// an ulp there) and the quadrant q mod 4.  No range branch; the reduction
// stays accurate while |x| < 2^40, far beyond k times any near-field
// distance.
__device__ inline void sincos_near(double x, double *s, double *c) {
    const double q = rint(x * 0.6366197723675814);
    double r = fma(-q, 1.5707963267948966, x);
    r = fma(-q, 6.123233995736766e-17, r);
    r = fma(-q, -1.4973849048591698e-33, r);
    const double r2 = r * r;
    double ps = fma(r2, 2.8114572543455206e-15, -7.647163731819816e-13);  // 1/17!, -1/15!
    ps = fma(r2, ps, 1.6059043836821613e-10);                          // 1/13!
    ps = fma(r2, ps, -2.505210838544172e-08);                          // -1/11!
    ps = fma(r2, ps, 2.7557319223985893e-06);                          // 1/9!
    ps = fma(r2, ps, -1.984126984126984e-04);                          // -1/7!
    ps = fma(r2, ps, 8.333333333333333e-03);                           // 1/5!
    ps = fma(r2, ps, -1.6666666666666666e-01);                         // -1/3!
    const double sr = fma(r * r2, ps, r);
    double pc = fma(r2, 4.779477332387385e-14, -1.1470745597729725e-11);  // 1/16!, -1/14!
    pc = fma(r2, pc, 2.08767569878681e-09);                            // 1/12!
    pc = fma(r2, pc, -2.755731922398589e-07);                          // -1/10!
    pc = fma(r2, pc, 2.48015873015873e-05);                            // 1/8!
    pc = fma(r2, pc, -1.388888888888889e-03);                          // -1/6!
    pc = fma(r2, pc, 4.1666666666666664e-02);                          // 1/4!
    pc = fma(r2, pc, -0.5);
    const double cr = fma(r2, pc, 1.0);
    const int n = (int)q;
    const double u = (n & 1) ? cr : sr, v = (n & 1) ? sr : cr;
    *s = (n & 2) ? -u : u;
    *c = ((n + 1) & 2) ? -v : v;
}

// sin and cos of x in single precision from the matrix-core generation's
// transcendental unit: x in revolutions (x / 2 pi), its fractional part, then
// the hardware sine and cosine of a fraction of a turn.  The near field's
// phases k r stay within a few turns, where the reduction to [0, 1) is exact
// and the hardware functions keep the products within the stated tolerance
// (checked against the oracle with the rest of the mixed-precision path).
__device__ inline void sincos_turns(float x, float *s, float *c) {
    const float f = __builtin_amdgcn_fractf(x * 0.159154943f);  // 1 / (2 pi)
    *s = __builtin_amdgcn_sinf(f);
    *c = __builtin_amdgcn_cosf(f);
}
__device__ inline void sincos_turns(double x, double *s, double *c) { sincos_near(x, s, c); }

template <class R> struct r4;
template <> struct r4<float> { using type = float4; };
template <> struct r4<double> { using type = double4; };

__device__ inline float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One (target, source point) pair; d is the target minus the point, ns the
// point's record for one right-hand side.  Laplace: the record holds
// (s n, s), so the double layer is (d . s n) / r^3 and the single layer s / r.
// Helmholtz: the record holds (n, Re s) and Im s; the value is a (u + j v)
// times s with a = 1/r, u + j v = e^{jkr} (single layer) or a = (d . n) / r^3,
// u = cos kr + kr sin kr, v = sin kr - kr cos kr (double layer: the normal
// derivative at the point of e^{jkr}/r), and the complex product is
// accumulated by four fused multiply-adds.  The 1/(4 pi) of G is applied
// once per target by the caller.  p2p_pair forms what every right-hand side
// shares (Laplace: 1/r and 1/r^3; Helmholtz: a u and a v), p2p_acc adds one
// right-hand side's term, by the same operations whatever the number of
// right-hand sides the kernel serves at once.
template <class R>
struct PairTerm {
    R x, y;
};
template <bool DBL, bool HELM, class R>
__device__ inline PairTerm<R> p2p_pair(R d0, R d1, R d2, typename r4<R>::type ns, R k) {
    const R r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const R ir = inv_sqrt(r2);
    if constexpr (HELM) {
        const R kr = k * (r2 * ir);
        R sn, cs;
        sincos_turns(kr, &sn, &cs);
        R a, u, v;
        if (DBL) {
            R t = d1 * ns.y;
            t = fmar(d0, ns.x, t);
            t = fmar(d2, ns.z, t);
            a = t * (ir * ir) * ir;
            u = fmar(kr, sn, cs);
            v = fmar(-kr, cs, sn);
        } else {
            a = ir;
            u = cs;
            v = sn;
        }
        return {a * u, a * v};
    } else {
        return {ir, (ir * ir) * ir};
    }
}
template <bool DBL, bool HELM, class R, class A>
__device__ inline void p2p_acc(A &acc, const PairTerm<R> &pt, R d0, R d1, R d2, typename r4<R>::type ns, R si) {
    if constexpr (HELM) {
        acc.re = fmar(pt.x, ns.w, acc.re);
        acc.re = fmar(-pt.y, si, acc.re);
        acc.im = fmar(pt.x, si, acc.im);
        acc.im = fmar(pt.y, ns.w, acc.im);
    } else if constexpr (DBL) {
        R t = d1 * ns.y;
        t = fmar(d0, ns.x, t);
        t = fmar(d2, ns.z, t);
        acc = fmar(t, pt.y, acc);
    } else {
        acc = fmar(ns.w, pt.x, acc);
    }
}

// One block per work item (a target leaf and up to 64 of its targets).  The
// near-list boxes' points (contiguous runs in tree order) are split into four
// equal shares, one per wave; each wave streams its share in batches of 64
// points, one per lane, through its own LDS slot as packed records (position,
// normal and strength), loading the next batch into registers while it
// computes the current one, so no block barrier sits inside the loop.  Each
// lane holds TPL targets, so every LDS read serves TPL interactions; lanes not
// needed for targets split a batch into sub-streams.  The target-point
// difference is formed in FP64 and only then rounded to R, so that close pairs
// keep their relative accuracy in the mixed path: the double layer's
// numerator n . d of two nearby points of a smooth surface is of the order of
// |d|^2 / (radius of curvature), and a difference of FP32 coordinates taken
// relative to a common origin a leaf side away (one subtraction instead of
// two instructions per axis) puts errors of about 1e-5 into products of the
// 20480-element sphere.  Per-batch partial sums in R are added into an FP64
// total.  A block serves NR right-hand sides (grid y: groups of NR): each
// pair's geometry is formed once and its terms added per right-hand side,
// every right-hand side's sums running exactly as with NR = 1 (bitwise the
// same results).
template <class V, class R, bool DBL, bool HELM, int TPL, int NR>
__global__ void __launch_bounds__(P2P_BS) k_p2p(const int32_t *unit_order, const int32_t *unit_item,
                                                const int64_t *unit_f, int64_t n_unit, const int32_t *wi_box,
                                                const int32_t *wi_t0, const int32_t *wi_nt, const int64_t *nptr,
                                                const int32_t *nidx, const int64_t *eb, const int64_t *ee,
                                                const double *q64, const R *q, int64_t n_q, const V *s,
                                                const double *t64, int64_t n_tgt, R k, int nrhs,
                                                typename std::conditional<HELM, cx<double>, double>::type *part) {
    using VD = typename std::conditional<HELM, cx<double>, double>::type;
    using R4 = typename r4<R>::type;
    constexpr int NW = P2P_BS / 64;
    // positions within the item's near-point sequence and point indices fit
    // 32 bits (the planner checks the point count)
    __shared__ int32_t pref[P2P_CH + 1];
    __shared__ int32_t qbeg[P2P_CH];
    __shared__ double2 sxy[NW][2][64];
    __shared__ double szz[NW][2][64];
    __shared__ R4 sns[NW][2][64][NR];
    __shared__ R ssi[NW][2][HELM ? 64 : 1][NR];
    __shared__ VD red[NW][64];
    __shared__ VD subs[NW][64];
    const int u = unit_order[blockIdx.x], rhs0 = blockIdx.y * NR;  // the block's first right-hand side
    const int w = unit_item[u];
    const int32_t u0 = (int32_t)unit_f[2 * u], u1 = (int32_t)unit_f[2 * u + 1];  // the unit's share of the item's near points
    const int b = wi_box[w], t0 = wi_t0[w], nt = wi_nt[w];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // tpw lanes hold the item's targets, TPL each (the last one repeated to
    // fill a lane); the wave's lanes form nsub such groups, each streaming
    // every nsub-th point (leftover lanes idle)
    const int tpw = (nt + TPL - 1) / TPL, nsub = 64 / tpw, tl = lane % tpw, sub = lane / tpw;
    double xt[TPL][3];
#pragma unroll
    for (int q = 0; q < TPL; q++) {
        const int ti = t0 + min(TPL * tl + q, nt - 1);
        xt[q][0] = t64[ti];
        xt[q][1] = t64[n_tgt + ti];
        xt[q][2] = t64[2 * n_tgt + ti];
    }
    const V *sr[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) sr[r] = s + (int64_t)min(rhs0 + r, nrhs - 1) * n_q;
    const double *qx = q64, *qy = q64 + n_q, *qz = q64 + 2 * n_q;
    const R *qnx = q + 4 * n_q, *qny = q + 5 * n_q, *qnz = q + 6 * n_q;
    VD tot[TPL][NR];
#pragma unroll
    for (int q = 0; q < TPL; q++)
#pragma unroll
        for (int r = 0; r < NR; r++) tot[q][r] = VD(0.0);
    const int64_t j0 = nptr[b], j1 = nptr[b + 1];
    int32_t base = 0;  // position of the chunk's first point in the item's near-point sequence
    for (int64_t cb = j0; cb < j1 && base < u1; cb += P2P_CH) {
        const int nc = (int)min<int64_t>(P2P_CH, j1 - cb);
        // run lengths of the chunk's near-list boxes, scanned by the first wave
        if (tid < 64) {
            int32_t carry = 0;
            for (int base = 0; base < nc; base += 64) {
                const int i = base + lane;
                int32_t len = 0;
                if (i < nc) {
                    const int32_t nb_ = nidx[cb + i];
                    qbeg[i] = (int32_t)(7 * eb[nb_]);
                    len = (int32_t)(7 * (ee[nb_] - eb[nb_]));
                }
                int32_t incl = len;
                for (int o = 1; o < 64; o <<= 1) {
                    const int32_t u = __shfl_up(incl, o, 64);
                    if (lane >= o) incl += u;
                }
                if (i < nc) pref[i + 1] = carry + incl;
                carry += __shfl(incl, 63, 64);
            }
            if (lane == 0) pref[0] = 0;
        }
        __syncthreads();
        const int32_t total = pref[nc];
        // this wave's share of the unit's points in the chunk
        const int32_t g0 = max(0, u0 - base), g1 = min(total, u1 - base);
        const int32_t gn = max(0, g1 - g0), per = (gn + NW - 1) / NW;
        const int32_t f0 = g0 + min(gn, per * wave), f1 = g0 + min(gn, per * wave + per);
        base += total;
        int e = 0;  // run holding this lane's current point
        // raw point records are loaded a batch ahead and only combined (strength
        // into the normal) when stored, so the loads stay in flight meanwhile
        double rx = 0.0, ry = 0.0, rz = 0.0;
        R rnx = 0, rny = 0, rnz = 0;
        V rs[NR];
#pragma unroll
        for (int r = 0; r < NR; r++) rs[r] = V(0.0);
        auto fetch = [&](int32_t f) {
            if (f < f1) {
                while (pref[e + 1] <= f) e++;
                const uint32_t qi = (uint32_t)(qbeg[e] + (f - pref[e]));
                rx = qx[qi];
                ry = qy[qi];
                rz = qz[qi];
#pragma unroll
                for (int r = 0; r < NR; r++) rs[r] = sr[r][qi];
                if (DBL) {
                    rnx = qnx[qi];
                    rny = qny[qi];
                    rnz = qnz[qi];
                }
            }
        };
        fetch(f0 + lane);
        int buf = 0;
        for (int32_t fb = f0; fb < f1; fb += 64) {
            {
                sxy[wave][buf][lane] = make_double2(rx, ry);
                szz[wave][buf][lane] = rz;
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    R4 ns;
                    ns.w = re_part(rs[r]);
                    const R sc = HELM ? (R)1 : ns.w;  // Laplace: strength folded into the normal
                    ns.x = rnx * sc;
                    ns.y = rny * sc;
                    ns.z = rnz * sc;
                    sns[wave][buf][lane][r] = ns;
                    if constexpr (HELM) ssi[wave][buf][lane][r] = rs[r].im;
                }
            }
            __builtin_amdgcn_wave_barrier();
            fetch(fb + 64 + lane);  // next batch in flight while this one is computed
            const int nin = min(64, f1 - fb);
            V acc[TPL][NR];
#pragma unroll
            for (int q = 0; q < TPL; q++)
#pragma unroll
                for (int r = 0; r < NR; r++) acc[q][r] = V(0.0);
#pragma unroll 1
            for (int kk = sub < nsub ? sub : nin; kk < nin; kk += nsub) {
                const double2 cxy = sxy[wave][buf][kk];
                const double cz = szz[wave][buf][kk];
                R4 cns[NR];
                R csi[NR];
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    cns[r] = sns[wave][buf][kk][r];
                    csi[r] = HELM ? ssi[wave][buf][HELM ? kk : 0][r] : (R)0;
                }
#pragma unroll
                for (int q = 0; q < TPL; q++) {
                    const R d0 = (R)(xt[q][0] - cxy.x), d1 = (R)(xt[q][1] - cxy.y), d2 = (R)(xt[q][2] - cz);
                    const PairTerm<R> pt = p2p_pair<DBL, HELM>(d0, d1, d2, cns[0], k);
#pragma unroll
                    for (int r = 0; r < NR; r++) p2p_acc<DBL, HELM>(acc[q][r], pt, d0, d1, d2, cns[r], csi[r]);
                }
            }
#pragma unroll
            for (int q = 0; q < TPL; q++)
#pragma unroll
                for (int r = 0; r < NR; r++) tot[q][r] += vcast<VD>(acc[q][r]);
            buf ^= 1;
        }
        __syncthreads();  // pref / qbeg are rewritten by the next chunk
    }
    // per right-hand side: reduce over the wave's groups (lanes tl, tl + tpw,
    // ...), in group order, then over the waves in wave order
#pragma unroll
    for (int r = 0; r < NR; r++) {
#pragma unroll
        for (int q = 0; q < TPL; q++) {
            subs[wave][lane] = tot[q][r];
            __builtin_amdgcn_wave_barrier();
            if (sub == 0) {
                VD v = tot[q][r];
                for (int k = 1; k < nsub; k++) v += subs[wave][tl + k * tpw];
                if (TPL * tl + q < 64) red[wave][TPL * tl + q] = v;
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        if (tid < nt && rhs0 + r < nrhs) {
            VD v = red[0][tid];
            for (int wv = 1; wv < NW; wv++) v += red[wv][tid];
            part[((int64_t)(rhs0 + r) * n_unit + u) * 64 + tid] = v;
        }
        if (NR > 1) __syncthreads();  // red is rewritten for the next right-hand side
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
// y(DOF of sorted target t) = the operator's combination of the far field,
// the near-field partial sums of t's item (times 1/4pi), the
// singular / near-singular corrections and, for A, the free term.  Eight
// lanes per target share its correction pairs and meet by shuffles.  The far
// field is either a finished value per target (yacc, direct product) or, for
// the fast product, the local expansion evaluated at the target (Section 3.2),
// folded in here: the monomials u^b of the target's position u in its leaf's
// frame (scaled by the leaf's side) are products of powers of u's three
// components, which three lanes of the target form in FP64 and leave in LDS
// in the expansion's precision; the target's eight lanes then take every
// eighth coefficient, and the sum over lanes runs in FP64.
template <class XV, class AV, class R, class VD>
__global__ void __launch_bounds__(256) k_combine(int64_t n_tgt, const int32_t *tperm, const AV *yacc,
                                                 const int32_t *tgt_leaf, const double *t64, const double *centre,
                                                 const int32_t *level, double side, const int8_t *exps, int order,
                                                 const AV *loc, int P, int64_t n_box, const int32_t *tgt_item,
                                                 const int32_t *item_unit, const int32_t *wi_t0, const VD *part,
                                                 int64_t n_unit, const int64_t *row_ptr, const int32_t *pair_elem,
                                                 const int32_t *se_dofs, const XV *corr, const double *cfree,
                                                 const XV *x, int op, XV *y) {
    __shared__ R pw[32][3][MAX_ORDER + 1];      // powers of the block's targets' coordinates
    __shared__ int32_t ex[ncoef(MAX_ORDER)];    // exponents a | b << 8 | c << 16 of each coefficient
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int l8 = threadIdx.x & 7, slot = threadIdx.x >> 3, rhs = blockIdx.y;
    const bool ok = t < n_tgt;
    const XV *xr = x + (int64_t)rhs * n_tgt;
    XV acc = XV(0.0);
    if (loc) {  // the same for the whole block
        for (int i = threadIdx.x; i < P; i += blockDim.x)
            ex[i] = exps[3 * i] | (exps[3 * i + 1] << 8) | (exps[3 * i + 2] << 16);
        const int b = ok ? tgt_leaf[4 * t] : 0;
        if (ok && l8 < 3) {
            const double u = (t64[l8 * n_tgt + t] - centre[3 * b + l8]) * ldexp(1.0 / side, level[b]);
            double v = 1.0;
            for (int k = 0; k <= order; k++) {
                pw[slot][l8][k] = (R)v;
                v *= u;
            }
        }
        __syncthreads();
        if (ok) {
            const AV *F = loc + ((int64_t)rhs * n_box + b) * P;
            const R *p0 = pw[slot][0], *p1 = pw[slot][1], *p2 = pw[slot][2];
            AV a = AV(0.0);
#pragma unroll 4
            for (int i = l8; i < P; i += 8) {
                const int e = ex[i];
                a += F[i] * (p0[e & 255] * p1[(e >> 8) & 255] * p2[e >> 16]);
            }
            acc = vcast<XV>(a);
        }
    }
    if (ok) {
        for (int64_t p = row_ptr[t] + l8; p < row_ptr[t + 1]; p += 8) {
            const int32_t *dof = se_dofs + 6 * (int64_t)pair_elem[p];
            const XV *cp = corr + 6 * p;
            for (int a = 0; a < 6; a++) acc += cp[a] * xr[dof[a]];
        }
        if (part && l8 == 1) {
            const int32_t w = tgt_item[t];
            const int64_t o = t - wi_t0[w];
            VD v = VD(0.0);
            for (int32_t u = item_unit[w]; u < item_unit[w + 1]; u++) v += part[((int64_t)rhs * n_unit + u) * 64 + o];
            v = v * kInv4Pi;
            acc += vcast<XV>(v);
        }
        if (yacc && l8 == 0) acc += vcast<XV>(yacc[(int64_t)rhs * n_tgt + t]);
    }
#pragma unroll
    for (int o = 1; o < 8; o <<= 1) {
        if constexpr (std::is_same<XV, double>::value) {
            acc += __shfl_xor(acc, o, 64);
        } else {
            acc.re += __shfl_xor(acc.re, o, 64);
            acc.im += __shfl_xor(acc.im, o, 64);
        }
    }
    if (!ok || l8) return;
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
    SetupTimer st_(*t.ctx, "near and far plans");
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
    {
        std::vector<int32_t> tl(4 * std::max<int64_t>(1, t.n_tgt), 0);
        for (int32_t b : tgt_leaves)
            for (int64_t i = t.h_tb[b]; i < t.h_te[b]; i++) {
                tl[4 * i] = b;
                tl[4 * i + 1] = (int32_t)t.h_tb[b];
                tl[4 * i + 2] = (int32_t)(t.h_te[b] - t.h_tb[b]);
            }
        t.tgt_leaf = upload_i32(c, tl);
    }
    t.m2l_boxes = upload_i32(c, m2l);
    t.n_m2l_boxes = (int64_t)m2l.size();
    t.p2p_box = upload_i32(c, wb);
    t.p2p_t0 = upload_i32(c, wt0);
    t.p2p_nt = upload_i32(c, wnt);
    t.n_p2p_items = (int64_t)wb.size();
    // work units: each item's near points split into shares of about equal
    // cost (points x lanes per point), so that blocks balance over the CUs;
    // dispatched most expensive first
    {
        const size_t ni = wb.size();
        std::vector<int64_t> npts(ni);
        std::vector<double> cpp(ni);  // cost per point: a wave covers 64 / ceil(nt / 2) points per step
        double total = 0.0;
        for (size_t i = 0; i < ni; i++) {
            const int32_t b = wb[i];
            int64_t n = 0;
            for (int64_t j = t.h_near_ptr[b]; j < t.h_near_ptr[b + 1]; j++) {
                const int32_t s = t.h_near_idx[j];
                n += 7 * (t.h_ee[s] - t.h_eb[s]);
            }
            const int nsub = 64 / ((wnt[i] + 1) / 2);
            npts[i] = n;
            cpp[i] = 1.0 / nsub;
            total += n * cpp[i];
        }
        int n_cu = 256;
        (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, c.device);
        const double target = std::max(total / (16.0 * std::max(1, n_cu)), 1.0);
        std::vector<int32_t> uitem, iunit(ni + 1, 0);
        std::vector<int64_t> uf;
        std::vector<double> ucost;
        for (size_t i = 0; i < ni; i++) {
            iunit[i] = (int32_t)uitem.size();
            int64_t parts = (int64_t)std::ceil(npts[i] * cpp[i] / target);
            // at least one batch of 64 points per wave in a unit
            parts = std::max<int64_t>(1, std::min<int64_t>(parts, npts[i] / (64 * (P2P_BS / 64))));
            for (int64_t k = 0; k < parts; k++) {
                uitem.push_back((int32_t)i);
                uf.push_back(npts[i] * k / parts);
                uf.push_back(npts[i] * (k + 1) / parts);
                ucost.push_back((double)(npts[i] * (k + 1) / parts - npts[i] * k / parts) * cpp[i]);
            }
        }
        iunit[ni] = (int32_t)uitem.size();
        std::vector<int32_t> order(uitem.size());
        for (size_t i = 0; i < order.size(); i++) order[i] = (int32_t)i;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ucost[a] > ucost[b]; });
        t.n_p2p_units = (int64_t)uitem.size();
        t.p2p_unit_order = upload_i32(c, order);
        t.p2p_unit_item = upload_i32(c, uitem);
        t.p2p_item_unit = upload_i32(c, iunit);
        t.p2p_unit_f.alloc(&c, uf.size());
        t.p2p_unit_f.upload(uf.data(), uf.size());
        std::vector<int32_t> titem(std::max<int64_t>(1, t.n_tgt), 0);
        for (size_t i = 0; i < ni; i++)
            for (int32_t k = 0; k < wnt[i]; k++) titem[wt0[i] + k] = (int32_t)i;
        t.p2p_tgt_item = upload_i32(c, titem);
    }
    BEM_REQUIRE(t.n_q < ((int64_t)1 << 31), BEM_EUNSUPPORTED, "more quadrature points than the near-field kernel indexes");
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
    t.l2l_level_boxes.assign(t.max_level + 1, {});
    t.d_m2m_level_boxes.clear();
    t.d_l2l_level_boxes.clear();
    t.d_level_boxes.clear();
    for (int l = 0; l <= t.max_level; l++) {
        std::vector<int32_t> up, down, par;
        for (int64_t b = t.level_off[l]; b < t.level_off[l + 1]; b++) {
            if (!t.h_leaf[b]) up.push_back((int32_t)b);
            if (l > 0 && t.h_te[b] > t.h_tb[b]) down.push_back((int32_t)b);
            if (!t.h_leaf[b] && t.h_te[b] > t.h_tb[b]) par.push_back((int32_t)b);
        }
        t.m2m_level_boxes[l] = up;
        t.l2l_level_boxes[l] = par;
        t.d_m2m_level_boxes.push_back(upload_i32(c, up));
        t.d_l2l_level_boxes.push_back(upload_i32(c, par));
        t.d_level_boxes.push_back(upload_i32(c, down));
        t.h_level_down.push_back((int64_t)down.size());
    }
    // levels the upward and downward passes can skip
    {
        int src_min = t.max_level + 1, tgt_min = t.max_level + 1;
        for (int64_t b = 0; b < t.n_box; b++) {
            if (t.h_te[b] == t.h_tb[b]) continue;
            if (t.h_inter_ptr[b + 1] > t.h_inter_ptr[b]) tgt_min = std::min(tgt_min, (int)t.h_level[b]);
            for (int64_t j = t.h_inter_ptr[b]; j < t.h_inter_ptr[b + 1]; j++)
                src_min = std::min(src_min, (int)t.h_level[t.h_inter_idx[j]]);
        }
        t.m2m_top = std::min(src_min, t.max_level);
        t.l2l_top = std::min(tgt_min, t.max_level);
    }
    c.sync();
    t.planned = true;
}

// ---------------------------------------------------------------- drivers
void rule_shapes(bem_tree &t) {
    if (t.L7.p) return;
    // shape functions at the 7 rule points
    std::vector<double> L7(42);
    double rs[7], rt[7], rw[7];
    rule7(rs, rt, rw);
    for (int qq = 0; qq < 7; qq++) {
        double S_ = rs[qq], T_ = rt[qq], Z = 1.0 - S_ - T_;
        double L[6] = {Z * (2 * Z - 1), S_ * (2 * S_ - 1), T_ * (2 * T_ - 1), 4 * Z * S_, 4 * S_ * T_, 4 * T_ * Z};
        if (t.mesh->linear) {  // first-order elements: linear on the corners, nothing on the mid-side slots
            L[0] = Z; L[1] = S_; L[2] = T_;
            L[3] = L[4] = L[5] = 0.0;
        }
        for (int a = 0; a < 6; a++) L7[6 * qq + a] = L[a];
    }
    t.L7.alloc(t.ctx, 42);
    t.L7.upload(L7.data(), 42);
}

// The regular 7-point double layer of a unit density at every target (the
// regular part of the free term, Eq. 2): sum over all rule points y of
// wJ n1.(x - y) / (4 pi |x - y|^3), FP64.  Grid (target tiles of 256, point
// splits): each block sums its share of the points for its targets into a
// partial sum per split, and the splits are added in order afterwards (so
// that even small meshes fill the GPU); 1/|x - y| is the hardware estimate
// refined twice by Newton (a few ulp, like the division and square root it
// replaces).
// qmul (literal tree, else NULL): each point's share of the unit density,
// the sum of its piece's shape functions there.
__global__ void __launch_bounds__(256) k_unit_double_layer(const double *q, int64_t n_q, int64_t per_split,
                                                           const double *qmul, const double *t, int64_t n_tgt,
                                                           double *part) {
    __shared__ double sx[256], sy[256], sz[256], sn0[256], sn1[256], sn2[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x, ii = min(i, n_tgt - 1);
    const double x0 = t[ii], x1 = t[n_tgt + ii], x2 = t[2 * n_tgt + ii];
    const int64_t j0 = (int64_t)blockIdx.y * per_split, j1 = min(n_q, j0 + per_split);
    double acc = 0.0;
    for (int64_t base = j0; base < j1; base += 256) {
        const int64_t j = base + threadIdx.x;
        if (j < j1) {
            const double wj = qmul ? q[3 * n_q + j] * qmul[j] : q[3 * n_q + j];
            sx[threadIdx.x] = q[j];
            sy[threadIdx.x] = q[n_q + j];
            sz[threadIdx.x] = q[2 * n_q + j];
            sn0[threadIdx.x] = wj * q[4 * n_q + j];
            sn1[threadIdx.x] = wj * q[5 * n_q + j];
            sn2[threadIdx.x] = wj * q[6 * n_q + j];
        }
        __syncthreads();
        const int m = (int)min<int64_t>(256, j1 - base);
        for (int kk = 0; kk < m; kk++) {
            const double d0 = x0 - sx[kk], d1 = x1 - sy[kk], d2 = x2 - sz[kk];
            const double ir = inv_sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            acc += (d0 * sn0[kk] + d1 * sn1[kk] + d2 * sn2[kk]) * (ir * ir * ir);
        }
        __syncthreads();
    }
    if (i < n_tgt) part[(int64_t)blockIdx.y * n_tgt + i] = acc;
}

__global__ void k_sum_splits(const double *part, int splits, int64_t n, double *y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int s = 0; s < splits; s++) acc += part[(int64_t)s * n + i];
    y[i] = acc * kInv4Pi;
}

void direct_regular_unit_double_layer(bem_tree &t, double *out) {
    Ctx &c = *t.ctx;
    const int64_t tiles = nblocks(t.n_tgt, 256);
    const int splits = (int)std::max<int64_t>(1, std::min<int64_t>(nblocks(t.n_q, 256), 2048 / std::max<int64_t>(1, tiles)));
    const int64_t per = (t.n_q + splits - 1) / splits;
    DBuf<double> part, qmul;
    part.alloc(&c, (size_t)splits * t.n_tgt);
    if (t.se_mask.p) {
        rule_shapes(t);
        const std::vector<double> L7 = t.L7.download(42);
        const std::vector<uint8_t> mk = t.se_mask.download(t.n_el);
        std::vector<double> qm(t.n_q, 0.0);
        for (int64_t v = 0; v < t.n_el; v++)
            for (int q = 0; q < 7; q++)
                for (int a = 0; a < 6; a++)
                    if (mk[v] >> a & 1) qm[7 * v + q] += L7[6 * q + a];
        qmul.alloc(&c, t.n_q);
        qmul.upload(qm.data(), t.n_q);
    }
    k_unit_double_layer<<<dim3((unsigned)tiles, (unsigned)splits), 256, 0, c.stream>>>(t.q64.p, t.n_q, per, qmul.p,
                                                                                      t.t64.p, t.n_tgt, part.p);
    BEM_LAUNCH_CHECK();
    k_sum_splits<<<nblocks(t.n_tgt, 256), 256, 0, c.stream>>>(part.p, splits, t.n_tgt, out);
    BEM_LAUNCH_CHECK();
}

namespace {

template <class V, class R, class XV, bool HELM>
void run_matvec(bem_tree &t, double k, int op, int method, int nrhs, const XV *x, XV *y, const LaunchChoice &lc) {
    Ctx &c = *t.ctx;
    const bool dbl = (op == BEM_OP_K || op == BEM_OP_A);
    const int64_t nq = t.n_q, nt = t.n_tgt;
    Corr &cr = get_corr(t, HELM ? BEM_HELMHOLTZ : BEM_LAPLACE, k);
    if (op == BEM_OP_A) build_free_term(t);
    M2lPlan *pl = method == BEM_FMM ? &get_m2l_plan(t, HELM ? BEM_HELMHOLTZ : BEM_LAPLACE, k) : nullptr;
    const R *q = std::is_same<R, float>::value ? (const R *)t.q32.p : (const R *)t.q64.p;
    const R *tg = std::is_same<R, float>::value ? (const R *)t.t32.p : (const R *)t.t64.p;
    // work buffers
    V *s = (V *)work_buf(c, t.work.strength, sizeof(V) * nq * nrhs);
    V *yacc = method == BEM_DIRECT ? (V *)work_buf(c, t.work.yacc, sizeof(V) * nt * nrhs) : nullptr;
    rule_shapes(t);
    if (method == BEM_FMM) {
        fmm_tables(t);
        plan_fmm(t);
        build_pass_tables(t);
        m2l_prepare<V, R>(t, *pl, lc.m2l_waves);
    }
    // moments and locals of the fast product in one buffer, cleared by the strength launch
    V *mom = nullptr, *loc = nullptr;
    void *p2p_part = nullptr;  // near-field partial sums of the fast product
    size_t nexp = 0;
    if (method == BEM_FMM) {
        nexp = (size_t)t.n_box * t.tables->P * nrhs;
        mom = (V *)work_buf(c, t.work.mom, 2 * sizeof(V) * nexp);
        loc = mom + nexp;
    }
    c.mark(9);
    dim3 gs(nblocks(nq, 256), nrhs);
    k_strength<V, R, XV><<<gs, 256, 0, c.stream>>>(x, nt, t.se_dofs.p, t.se_mask.p, q + 3 * nq, nq, t.L7.p, s,
                                                   (uint32_t *)mom, (int64_t)(2 * sizeof(V) * nexp / 4));
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
        using PD = typename std::conditional<HELM, cx<double>, double>::type;
        PD *part = nullptr;
        if (t.n_p2p_items) {
            part = (PD *)work_buf(c, t.work.p2p_part, sizeof(PD) * 64 * (size_t)t.n_p2p_units * nrhs);
            p2p_part = part;
        }
        // While it runs beside the far field, the near-field kernel asks for
        // enough LDS that at most lc.p2p_per_cu of its blocks share a CU,
        // which leaves registers and wave slots for the far-field kernels
        // (their matrix-core and latency-bound work then overlaps its VALU
        // work); with lc.m2l_room the blocks share what one M2L product block
        // leaves of the CU's LDS, so that one such block fits beside them.
        // 0 asks for no more than the kernel's own LDS.
        const size_t m2l_lds = lc.m2l_room && pl ? m2l_block_lds(*pl, std::is_same<R, float>::value ? BEM_PREC_MIXED : BEM_PREC_FP64, lc.m2l_waves) : 0;
        auto near_lds = [&](const void *fn) -> unsigned {
            if (lc.p2p_per_cu <= 0) return 0u;
            // per kernel, blocks per CU and room (one device model)
            static thread_local std::map<std::tuple<const void *, int, size_t>, unsigned> memo;
            const auto key = std::make_tuple(fn, lc.p2p_per_cu, m2l_lds);
            auto it = memo.find(key);
            if (it != memo.end()) return it->second;
            hipFuncAttributes fa;
            BEM_HIP(hipFuncGetAttributes(&fa, fn));
            int lds = 0;
            BEM_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, c.device));
            const long avail = (long)lds - (m2l_lds ? (long)m2l_lds + 1024 : 0);
            const long pad = avail / lc.p2p_per_cu - (long)fa.sharedSizeBytes - 256;
            return memo[key] = pad > 0 ? (unsigned)pad : 0u;
        };
        // Several right-hand sides: two per block, sharing each pair's geometry.
        auto near_field = [&](hipStream_t st) {
            const bool beside = st != c.stream;
            c.kbegin(st, 6);
            constexpr int TPL = P2P_TPL;
            auto launch = [&](auto nr, auto dl) {
                constexpr int NR = decltype(nr)::value;
                constexpr bool DL = decltype(dl)::value;
                const void *fn = (const void *)k_p2p<V, R, DL, HELM, TPL, NR>;
                dim3 g((unsigned)t.n_p2p_units, (unsigned)((nrhs + NR - 1) / NR));
                k_p2p<V, R, DL, HELM, TPL, NR><<<g, P2P_BS, beside ? near_lds(fn) : 0, st>>>(
                    t.p2p_unit_order.p, t.p2p_unit_item.p, t.p2p_unit_f.p, t.n_p2p_units, t.p2p_box.p, t.p2p_t0.p,
                    t.p2p_nt.p, t.near_ptr.p, t.near_idx.p, t.eb.p, t.ee.p, t.q64.p, q, nq, s, t.t64.p, nt, (R)k, nrhs,
                    part);
            };
            using one = std::integral_constant<int, 1>;
            using two = std::integral_constant<int, 2>;
            using yes = std::true_type;
            using no = std::false_type;
            if (nrhs > 1) {
                if (dbl) launch(two(), yes());
                else launch(two(), no());
            } else {
                if (dbl) launch(one(), yes());
                else launch(one(), no());
            }
            BEM_LAUNCH_CHECK();
            c.kend(st);
        };
        // The near field depends only on the strengths and writes only its
        // own partial sums: it runs on the second stream, concurrently with
        // the far-field passes, and is joined before its sums are added.
        // While phases are being timed everything stays on one stream.
        const bool overlap = t.n_p2p_items && c.timing != 1;
        // The near field starts as soon as the strengths are in (beside the
        // upward pass), except for the complex FP64 kernel, which starts after
        // M2M: it slows the latency-bound upward pass more than it gains
        // (measured both ways for all four variants on the 40962-DOF sphere).
        constexpr bool early = !(HELM && std::is_same<R, double>::value);
        if (overlap && early) {
            hipStream_t side = c.side_stream();
            c.fork();
            near_field(side);
        }
        // upward pass (boxes without elements keep zero moments)
        p2m_apply<V, R, XV>(t, dbl, nrhs, x, mom);
        c.mark(1);
        m2m_apply<V, R>(t, nrhs, mom);
        c.mark(2);
        // interactions
        c.mark(9);
        if (overlap && !early) {
            hipStream_t side = c.side_stream();
            c.fork();
            near_field(side);
        }
        m2l_apply<V, R>(t, *pl, nrhs, mom, loc, lc.m2l_waves);
        // downward pass
        l2l_apply<V, R>(t, nrhs, loc);
        c.mark(4);
        // (the local expansions are evaluated at the targets in the combination)
        if (t.n_p2p_items) {
            if (overlap) c.join();
            else near_field(c.stream);
        }
        c.mark(6);
    }
    // near-field sums, corrections and combination in FP64
    using VD = typename std::conditional<HELM, cx<double>, double>::type;
    const XV *corr = (const XV *)(dbl ? cr.K.p : cr.S.p);
    const VD *part = (const VD *)p2p_part;
    dim3 g(nblocks(8 * nt, 256), nrhs);
    const bool fmm = method == BEM_FMM;
    k_combine<XV, V, R, VD><<<g, 256, 0, c.stream>>>(
        nt, t.tperm.p, fmm ? nullptr : yacc, t.tgt_leaf.p, t.t64.p, t.centre.p, t.level.p, t.side,
        fmm ? t.tables->exps.p : nullptr, t.order, fmm ? loc : nullptr, fmm ? t.tables->P : 0, t.n_box,
        t.p2p_tgt_item.p, t.p2p_item_unit.p, t.p2p_t0.p, part, t.n_p2p_units, t.pair_ptr.p,
        t.pair_elem.p, t.se_dofs.p, corr, op == BEM_OP_A ? t.free_term.p : nullptr, x, op, y);
    BEM_LAUNCH_CHECK();
    c.mark(7);
}

}  // namespace

// ---------------------------------------------------------------- launch choices
namespace {

std::mutex g_tune_mu;
std::map<std::array<int64_t, 5>, LaunchChoice> g_tuned;  // shape class -> fastest launch choice

// Shape class of a fast product: Green's function, precision, layer, and the
// near-field pair and interaction-slot counts on a grid of factors sqrt(2).
std::array<int64_t, 5> shape_class(const bem_tree &t, int green, int prec, int op) {
    auto b = [](int64_t v) { return (int64_t)std::lround(2.0 * std::log2((double)std::max<int64_t>(1, v))); };
    const bool dbl = op == BEM_OP_K || op == BEM_OP_A;
    return {green, prec == BEM_PREC_MIXED ? 1 : 0, dbl ? 1 : 0, b(t.n_p2p_pairs), b(t.n_inter)};
}

LaunchChoice default_choice(int green, int prec) {
    LaunchChoice lc;
    // complex near-field blocks are heavier: three per CU (measured)
    if (green == BEM_HELMHOLTZ) lc.p2p_per_cu = 3;
    (void)prec;
    return lc;
}

template <class V, class R, class XV, bool HELM>
void run_with(bem_tree &t, double k, int op, int method, int nrhs, const void *x, void *y, const LaunchChoice &lc) {
    run_matvec<V, R, XV, HELM>(t, k, op, method, nrhs, (const XV *)x, (XV *)y, lc);
}

}  // namespace

int64_t tuned_classes() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return (int64_t)g_tuned.size();
}

void forget_tuned_classes() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
}

LaunchChoice launch_choice(const bem_tree &t, int green, int prec, int op, bool *tuned) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(shape_class(t, green, prec, op));
    if (tuned) *tuned = it != g_tuned.end();
    return it != g_tuned.end() ? it->second : default_choice(green, prec);
}

bool product_ready(const bem_tree &t, int green, double k, int op, int method, int prec) {
    if (green == BEM_LAPLACE) k = 0.0;
    bool corr = false;
    for (auto &p : t.corr) corr = corr || (p->green == green && p->k == k);
    if (!corr || !t.L7.p || (op == BEM_OP_A && !t.has_free_term)) return false;
    if (method == BEM_DIRECT) return true;
    if (!t.tables || t.tables->p != t.order || !t.planned || !t.pass.built) return false;
    // the near field runs on the context's second stream, created by the first product
    if (t.n_p2p_items && !t.ctx->side) return false;
    const LaunchChoice lc = launch_choice(t, green, prec, op, nullptr);
    for (auto &pl : t.m2l)
        if (pl->green == green && pl->k == k) return m2l_ready(*pl, prec, lc.m2l_waves);
    return false;
}

void matvec(bem_tree &t, int green, double k, int op, int method, int prec, int nrhs, const void *x, void *y) {
    Ctx &c = *t.ctx;
    c.prod_seq++;
    if (c.timing && (c.ev_used > 4096 || c.kev_used > 4096)) {  // bound the pool of pending events
        c.sync();
        c.collect();
    }
    using CD = cx<double>;
    using CF = cx<float>;
    const bool f64 = prec == BEM_PREC_FP64 || method == BEM_DIRECT;
    auto run_n = [&](const LaunchChoice &lc, int n) {
        if (green == BEM_HELMHOLTZ) {
            if (f64) run_with<CD, double, CD, true>(t, k, op, method, n, x, y, lc);
            else run_with<CF, float, CD, true>(t, k, op, method, n, x, y, lc);
        } else {
            if (f64) run_with<double, double, double, false>(t, 0.0, op, method, n, x, y, lc);
            else run_with<float, float, double, false>(t, 0.0, op, method, n, x, y, lc);
        }
    };
    auto run = [&](const LaunchChoice &lc) { run_n(lc, nrhs); };
    auto run1 = [&](const LaunchChoice &lc) { run_n(lc, 1); };  // the first right-hand side alone
    bool tuned = false;
    if (method == BEM_FMM) plan_fmm(t);  // the shape class reads the plan's pair counts
    LaunchChoice lc = method == BEM_FMM ? launch_choice(t, green, prec, op, &tuned) : LaunchChoice{};
    if (method == BEM_FMM && !tuned && c.autotune && !c.arena && !c.timing && t.n_p2p_items) {
        // Autotuner: the first product of an untuned shape class sets up
        // everything with the default choice, then times candidates on the
        // first right-hand side alone (event pairs on the context's stream
        // around whole products, which end on that stream after the near
        // field's stream has joined it; best of two each): the M2L waves per
        // block (4 or 8) first, then the near field's blocks per CU (with or
        // without LDS left for one M2L block) with the best of those, then
        // the waves again.  (One block per CU and two-wave M2L blocks, never
        // competitive where measured, are not tried.)  The products write y;
        // the product proper follows with the fastest choice.
        run1(lc);
        hipEvent_t e0, e1;
        BEM_HIP(hipEventCreate(&e0));
        BEM_HIP(hipEventCreate(&e1));
        static const bool log = std::getenv("BEM_TUNE_LOG") != nullptr;  // candidates' times on stderr
        auto time_of = [&](const LaunchChoice &cand) {
            float best = 1e30f;
            for (int rep = 0; rep < 2; rep++) {
                BEM_HIP(hipEventRecord(e0, c.stream));
                run1(cand);
                BEM_HIP(hipEventRecord(e1, c.stream));
                BEM_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                BEM_HIP(hipEventElapsedTime(&ms, e0, e1));
                best = std::min(best, ms);
            }
            if (log)
                std::fprintf(stderr, "bem tune: n_tgt %lld green %d prec %d op %d: near blocks/CU %d%s, M2L waves %d: %.4f ms\n",
                             (long long)t.n_tgt, green, prec, op, cand.p2p_per_cu, cand.m2l_room ? " + M2L room" : "",
                             cand.m2l_waves, best);
            return best;
        };
        LaunchChoice best = lc;
        float tbest = time_of(lc);
        // complex mixed products run at most four M2L waves per block
        const bool w8 = !(green == BEM_HELMHOLTZ && !f64);
        if (w8) {
            LaunchChoice cand = best;
            cand.m2l_waves = 8;
            const float tm = time_of(cand);
            if (tm < tbest) { tbest = tm; best = cand; }
        }
        const LaunchChoice base = best;
        for (int room = 0; room < 2; room++)
            for (int pc : {2, 3, 4, 6, 0}) {
                if ((pc == base.p2p_per_cu && room == (int)base.m2l_room) || (room && (pc == 0 || pc > 3))) continue;
                LaunchChoice cand = base;
                cand.p2p_per_cu = pc;
                cand.m2l_room = room;
                const float tm = time_of(cand);
                if (tm < tbest) { tbest = tm; best = cand; }
            }
        // the waves per M2L block once more, beside the chosen near field
        const LaunchChoice fin = best;
        for (int w : {4, 8}) {
            if (w == fin.m2l_waves || (w == 8 && !w8)) continue;
            LaunchChoice cand = fin;
            cand.m2l_waves = w;
            const float tm = time_of(cand);
            if (tm < tbest) { tbest = tm; best = cand; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned.emplace(shape_class(t, green, prec, op), best);  // a concurrent tuner's entry stays
            lc = g_tuned[shape_class(t, green, prec, op)];
        }
    }
    run(lc);
}

}  // namespace bem
