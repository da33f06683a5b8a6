// Green's functions of Eqs. (1a/b) and the element map, as device functions.
#pragma once

#include <type_traits>

#include "common.h"

namespace bem {

constexpr double kInv4Pi = 0.079577471545947667884;  // 1 / (4 pi)

// G(R) and its normal derivative at the source point, dG/dn1 = n1 . grad_y G
// with r = x - y:  Laplace   G = 1/(4 pi R),        dG/dn1 = (r.n1)/(4 pi R^3)
//                  Helmholtz G = e^{jkR}/(4 pi R),   dG/dn1 = (1 - jkR) e^{jkR} (r.n1)/(4 pi R^3)
template <class R>
__device__ inline void green_laplace(R r2, R rn, R *G, R *dG) {
    R inv = (R)1 / sqrt(r2);
    R g = (R)kInv4Pi * inv;
    *G = g;
    *dG = g * rn * inv * inv;
}

template <class R>
__device__ inline void green_helmholtz(R r2, R rn, R k, cx<R> *G, cx<R> *dG) {
    R Rr = sqrt(r2);
    R inv = (R)1 / Rr;
    R sn, cs;
    vsincos(k * Rr, &sn, &cs);
    R g = (R)kInv4Pi * inv;
    *G = cx<R>(g * cs, g * sn);
    // (1 - jkR)(cs + j sn) = (cs + kR sn) + j (sn - kR cs)
    R kr = k * Rr;
    R f = g * rn * inv * inv;
    *dG = cx<R>(f * (cs + kr * sn), f * (sn - kr * cs));
}

// Derivatives d^g G(r) for |g| <= H (graded multi-index order, exps[3 * i]
// the exponents of index i), Laplace or Helmholtz with wavenumber kk: the
// radial functions G^(h)(R), h = 0..H, then d^g G^(h) for |g| <= H - h with h
// descending, each level from the previous one (Section 3.3, Eq. 12).  All
// threads of the block take part; A and B (ncoef(H) values each) and g (H +
// 1 values) are LDS scratch; returns the buffer holding the result.
__host__ __device__ constexpr int deriv_count(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__device__ inline int deriv_index(int a, int b, int c) {
    const int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}
template <bool HELM>
__device__ typename std::conditional<HELM, cx<double>, double>::type *derivs_block(
    const double r[3], double kk, int H, const int8_t *exps, typename std::conditional<HELM, cx<double>, double>::type *A,
    typename std::conditional<HELM, cx<double>, double>::type *B,
    typename std::conditional<HELM, cx<double>, double>::type *g) {
    using V = typename std::conditional<HELM, cx<double>, double>::type;
    const int tid = threadIdx.x;
    const double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2], Rr = sqrt(R2);
    if (tid == 0) {
        if constexpr (!HELM) {
            g[0] = kInv4Pi / Rr;
            for (int h = 0; h < H; h++) g[h + 1] = g[h] * (-(double)(2 * h + 1) / R2);
        } else {
            double sn, cs;
            sincos(kk * Rr, &sn, &cs);
            const double f = kInv4Pi / Rr, kr = kk * Rr, f3 = f / R2;
            g[0] = V(f * cs, f * sn);
            if (H >= 1) g[1] = V(f3 * (-cs - kr * sn), f3 * (kr * cs - sn));
            for (int h = 1; h < H; h++) g[h + 1] = (g[h] * (double)(2 * h + 1) + g[h - 1] * (kk * kk)) * (-1.0 / R2);
        }
        A[0] = g[H];
    }
    __syncthreads();
    V *prev = A, *cur = B;
    for (int h = H - 1; h >= 0; h--) {
        const int m = deriv_count(H - h);
        for (int i = tid; i < m; i += blockDim.x) {
            V v;
            if (i == 0) {
                v = g[h];
            } else {
                int al[3] = {exps[3 * i], exps[3 * i + 1], exps[3 * i + 2]};
                int d = al[0] > 0 ? 0 : (al[1] > 0 ? 1 : 2);
                al[d]--;
                v = prev[deriv_index(al[0], al[1], al[2])] * r[d];
                if (al[d] > 0) {
                    int ad = al[d];
                    al[d]--;
                    v += prev[deriv_index(al[0], al[1], al[2])] * (double)ad;
                }
            }
            cur[i] = v;
        }
        __syncthreads();
        V *t = prev; prev = cur; cur = t;
    }
    return prev;
}

// Quadratic 6-node triangle: shape functions and their s, t derivatives.
__device__ inline void shape6(double s, double t, double L[6], double Ls[6], double Lt[6]) {
    double z = 1.0 - s - t;
    L[0] = z * (2.0 * z - 1.0); L[1] = s * (2.0 * s - 1.0); L[2] = t * (2.0 * t - 1.0);
    L[3] = 4.0 * z * s; L[4] = 4.0 * s * t; L[5] = 4.0 * t * z;
    Ls[0] = 1.0 - 4.0 * z; Ls[1] = 4.0 * s - 1.0; Ls[2] = 0.0; Ls[3] = 4.0 * (z - s); Ls[4] = 4.0 * t; Ls[5] = -4.0 * t;
    Lt[0] = 1.0 - 4.0 * z; Lt[1] = 0.0; Lt[2] = 4.0 * t - 1.0; Lt[3] = -4.0 * s; Lt[4] = 4.0 * s; Lt[5] = 4.0 * (z - t);
}

// Position y, unit normal n and area Jacobian J of the element with nodes X at (s, t).
__device__ inline void elem_map(const double X[6][3], double s, double t, double y[3], double n[3], double *J,
                                double L[6]) {
    double Ls[6], Lt[6];
    shape6(s, t, L, Ls, Lt);
    double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    for (int d = 0; d < 3; d++) y[d] = 0.0;
    for (int k = 0; k < 6; k++)
        for (int d = 0; d < 3; d++) {
            y[d] += L[k] * X[k][d];
            a[d] += Ls[k] * X[k][d];
            b[d] += Lt[k] * X[k][d];
        }
    double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    double j = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    *J = j;
    for (int d = 0; d < 3; d++) n[d] = c[d] / j;
}

}  // namespace bem
