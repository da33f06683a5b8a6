// Iterative solution of Eq. (3) (Section 2.1: the paper uses a matrix-free
// Krylov solver around the fast product; GMRES with restart replaces its
// BiCGSTAB here).
//
// GMRES(m) from x0 = 0: Arnoldi with classical Gram-Schmidt applied twice
// (CGS2), the Hessenberg column rotated by complex Givens rotations on the
// device, one residual-estimate word read by the host per iteration, and a
// device back-substitution at the end of each cycle.  All Krylov arithmetic
// is FP64 (complex128 for Helmholtz); the inner products reduce in a fixed
// order, so repeated solves are bitwise identical.
//
// Precision modes:
//   FP64   GMRES on the FP64 operator to tol.
//   MIXED  outer refinement in FP64: d = GMRES(A_mixed, r, inner_tol);
//          x += d; r = b - A_64 x; until |r| / |b| <= tol.
#include <cmath>

#include "kernels.h"

namespace bem {

namespace {

constexpr int RBS = 256;

__device__ inline double cj(double v) { return v; }
__device__ inline cx<double> cj(cx<double> v) { return conj(v); }
__device__ inline double abs2(double v) { return v * v; }
__device__ inline double abs2(cx<double> v) { return v.re * v.re + v.im * v.im; }

// partial[i][blk] = sum over the block's chunk of conj(Vi) w
template <class V>
__global__ void k_dots(const V *basis, int64_t ld, const V *w, int64_t n, V *partial, int nblk) {
    __shared__ V red[RBS];
    const int i = blockIdx.y;
    const V *vi = basis + (int64_t)i * ld;
    V acc = V(0.0);
    for (int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x; e < n; e += (int64_t)nblk * RBS)
        acc += cj(vi[e]) * w[e];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = RBS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)i * nblk + blockIdx.x] = red[0];
}

// out[i] (+)= sum of partial[i][:] in order
template <class V>
__global__ void k_dots_finish(const V *partial, int nblk, int m, V *out, int accumulate) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    V acc = V(0.0);
    for (int b = 0; b < nblk; b++) acc += partial[(int64_t)i * nblk + b];
    if (accumulate) out[i] += acc;
    else out[i] = acc;
}

// w -= sum_{i < m} h[i] Vi
template <class V>
__global__ void k_subtract(const V *basis, int64_t ld, const V *h, int m, V *w, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    if (e >= n) return;
    V acc = w[e];
    for (int i = 0; i < m; i++) acc -= h[i] * basis[(int64_t)i * ld + e];
    w[e] = acc;
}

template <class V>
__global__ void k_scale_into(const V *w, const V *hcol, int j, V *out, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    if (e >= n) return;
    double inv = 1.0 / re_part(hcol[j + 1]);
    out[e] = w[e] * inv;
}

template <class V>
__global__ void k_axpy(V a_dummy, const V *x, V *y, int64_t n, double alpha) {
    int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    if (e < n) y[e] += x[e] * alpha;
}

template <class V>
__global__ void k_lincomb(const V *basis, int64_t ld, const V *yv, int m, V *x, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    if (e >= n) return;
    V acc = x[e];
    for (int i = 0; i < m; i++) acc += yv[i] * basis[(int64_t)i * ld + e];
    x[e] = acc;
}

// hcol holds column j of the Hessenberg matrix (j + 2 entries) with
// hcol[j+1] = |w| real.  Applies the previous rotations, forms the new one,
// stores the rotated column into H and updates g.  est[0] = |g[j+1]|.
template <class V>
__global__ void k_givens(V *H, int ldh, const V *hcol, V *cs, V *sn, V *g, int j, double *est) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    V col[96];
    for (int i = 0; i <= j + 1; i++) col[i] = hcol[i];
    for (int i = 0; i < j; i++) {
        V t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -(cj(sn[i]) * col[i]) + cj(cs[i]) * col[i + 1];
        col[i] = t;
    }
    V a = col[j], b = col[j + 1];
    double na = sqrt(abs2(a)), nbv = sqrt(abs2(b));
    V c, s;
    if (nbv == 0.0) { c = V(1.0); s = V(0.0); }
    else if (na == 0.0) { c = V(0.0); s = cj(b) * (1.0 / nbv); }
    else {
        double den = sqrt(abs2(a) + abs2(b));
        c = cj(a) * (1.0 / den);
        s = cj(b) * (1.0 / den);
    }
    cs[j] = c;
    sn[j] = s;
    col[j] = c * a + s * b;
    col[j + 1] = V(0.0);
    for (int i = 0; i <= j + 1; i++) H[(int64_t)i * ldh + j] = col[i];
    V gj = g[j];
    g[j + 1] = -(cj(s) * gj);
    g[j] = c * gj;
    est[0] = sqrt(abs2(g[j + 1]));
}

// y = R^{-1} g for the leading m x m upper triangle of H
template <class V>
__global__ void k_backsolve(const V *H, int ldh, const V *g, int m, V *y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = m - 1; i >= 0; i--) {
        V acc = g[i];
        for (int k = i + 1; k < m; k++) acc -= H[(int64_t)i * ldh + k] * y[k];
        V d = H[(int64_t)i * ldh + i];
        double dd = abs2(d);
        y[i] = acc * cj(d) * (1.0 / dd);
    }
}

template <class V>
__global__ void k_add(V *a, const V *b, int m) {
    for (int i = threadIdx.x; i < m; i += blockDim.x) a[i] += b[i];
}

template <class V>
__global__ void k_sub(const V *a, const V *b, V *out, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    if (e < n) out[e] = a[e] - b[e];
}

template <class V>
__global__ void k_set_real(V *h, int i, const double *v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) h[i] = V(sqrt(*v));
}

template <class V>
__global__ void k_norm2_to(const V *hv, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = re_part(hv[0]);
}

template <class V>
struct Krylov {
    Ctx &c;
    int64_t n;
    int m;
    int nblk;
    DBuf<V> basis, w, hcol, hc2, H, cs, sn, g, y, partial, tmp;
    DBuf<double> est;  // [0] residual estimate, [1] scratch
    double *h_est = nullptr;

    Krylov(Ctx &c_, int64_t n_, int m_) : c(c_), n(n_), m(m_) {
        nblk = (int)std::min<int64_t>(256, nblocks(n, RBS));
        basis.alloc(&c, (size_t)(m + 1) * n);
        w.alloc(&c, n);
        tmp.alloc(&c, n);
        hcol.alloc(&c, m + 2);
        hc2.alloc(&c, m + 2);
        H.alloc(&c, (size_t)(m + 1) * m);
        cs.alloc(&c, m);
        sn.alloc(&c, m);
        g.alloc(&c, m + 1);
        y.alloc(&c, m);
        partial.alloc(&c, (size_t)(m + 2) * nblk);
        est.alloc(&c, 2);
        BEM_HIP(hipHostMalloc((void **)&h_est, sizeof(double), hipHostMallocDefault));
    }
    ~Krylov() {
        if (h_est) (void)hipHostFree(h_est);
    }
    V *vec(int i) { return basis.p + (int64_t)i * n; }

    // out[0..cnt) (= or +=) conj(V_i) . v
    void dots(const V *base, int cnt, const V *v, V *out, bool acc) {
        dim3 g2(nblk, cnt);
        k_dots<V><<<g2, RBS, 0, c.stream>>>(base, n, v, n, partial.p, nblk);
        BEM_LAUNCH_CHECK();
        k_dots_finish<V><<<nblocks(cnt, 64), 64, 0, c.stream>>>(partial.p, nblk, cnt, out, acc ? 1 : 0);
        BEM_LAUNCH_CHECK();
    }
    double norm(const V *v) {
        dots(v, 1, v, hc2.p, false);
        k_norm2_to<V><<<1, 1, 0, c.stream>>>(hc2.p, est.p + 1);
        BEM_LAUNCH_CHECK();
        double v2 = read_scalar(c, est.p + 1);
        return std::sqrt(v2);
    }
};

// GMRES(m) on apply(); x holds the initial guess and receives the result.
template <class V, class F>
int gmres(Krylov<V> &K, F &&apply, const V *b, V *x, double tol, int max_cycles, int *iters, int *matvecs,
          double *relres, bool zero_x0) {
    Ctx &c = K.c;
    const int64_t n = K.n;
    const int m = K.m;
    const unsigned nb = nblocks(n, RBS);
    double bnorm = K.norm(b);
    if (bnorm == 0.0) {
        zero_fill(c, x, sizeof(V) * n);
        *relres = 0.0;
        return BEM_OK;
    }
    for (int cycle = 0; cycle < max_cycles; cycle++) {
        // r = b - A x, into V0
        if (zero_x0 && cycle == 0) {
            BEM_HIP(hipMemcpyAsync(K.vec(0), b, sizeof(V) * n, hipMemcpyDeviceToDevice, c.stream));
        } else {
            apply(x, K.tmp.p);
            (*matvecs)++;
            k_sub<V><<<nb, RBS, 0, c.stream>>>(b, K.tmp.p, K.vec(0), n);
            BEM_LAUNCH_CHECK();
        }
        double beta = K.norm(K.vec(0));
        *relres = beta / bnorm;
        if (beta / bnorm <= tol) return BEM_OK;
        {
            double inv = 1.0 / beta;
            zero_fill(c, K.tmp.p, sizeof(V) * n);
            k_axpy<V><<<nb, RBS, 0, c.stream>>>(V(0.0), K.vec(0), K.tmp.p, n, inv);
            BEM_LAUNCH_CHECK();
            BEM_HIP(hipMemcpyAsync(K.vec(0), K.tmp.p, sizeof(V) * n, hipMemcpyDeviceToDevice, c.stream));
        }
        std::vector<V> g0(m + 1, V(0.0));
        g0[0] = V(beta);
        K.g.upload(g0.data(), m + 1);
        int jdone = 0;
        bool converged = false;
        for (int j = 0; j < m; j++) {
            apply(K.vec(j), K.w.p);
            (*matvecs)++;
            double wnorm = K.norm(K.w.p);
            // CGS2
            K.dots(K.basis.p, j + 1, K.w.p, K.hcol.p, false);
            k_subtract<V><<<nb, RBS, 0, c.stream>>>(K.basis.p, n, K.hcol.p, j + 1, K.w.p, n);
            BEM_LAUNCH_CHECK();
            K.dots(K.basis.p, j + 1, K.w.p, K.hc2.p, false);
            k_subtract<V><<<nb, RBS, 0, c.stream>>>(K.basis.p, n, K.hc2.p, j + 1, K.w.p, n);
            BEM_LAUNCH_CHECK();
            k_add<V><<<1, 64, 0, c.stream>>>(K.hcol.p, K.hc2.p, j + 1);  // h = h1 + h2
            BEM_LAUNCH_CHECK();
            double hn = K.norm(K.w.p);  // leaves |w|^2 in est[1]
            k_set_real<V><<<1, 1, 0, c.stream>>>(K.hcol.p, j + 1, K.est.p + 1);
            BEM_LAUNCH_CHECK();
            bool breakdown = hn <= 1e-14 * wnorm;
            if (!breakdown) {
                k_scale_into<V><<<nb, RBS, 0, c.stream>>>(K.w.p, K.hcol.p, j, K.vec(j + 1), n);
                BEM_LAUNCH_CHECK();
            }
            k_givens<V><<<1, 1, 0, c.stream>>>(K.H.p, m, K.hcol.p, K.cs.p, K.sn.p, K.g.p, j, K.est.p);
            BEM_LAUNCH_CHECK();
            BEM_HIP(hipMemcpyAsync(K.h_est, K.est.p, sizeof(double), hipMemcpyDeviceToHost, c.stream));
            c.sync();
            (*iters)++;
            jdone = j + 1;
            *relres = *K.h_est / bnorm;
            if (*relres <= tol || breakdown) {
                converged = true;
                break;
            }
        }
        k_backsolve<V><<<1, 1, 0, c.stream>>>(K.H.p, m, K.g.p, jdone, K.y.p);
        BEM_LAUNCH_CHECK();
        k_lincomb<V><<<nb, RBS, 0, c.stream>>>(K.basis.p, n, K.y.p, jdone, x, n);
        BEM_LAUNCH_CHECK();
        (void)converged;
    }
    // final explicit residual
    apply(x, K.tmp.p);
    (*matvecs)++;
    k_sub<V><<<nb, RBS, 0, c.stream>>>(b, K.tmp.p, K.w.p, n);
    BEM_LAUNCH_CHECK();
    *relres = K.norm(K.w.p) / bnorm;
    return *relres <= tol ? BEM_OK : BEM_ENOCONV;
}

template <class V>
int solve_t(bem_tree &t, int green, double k, int nrhs, const V *chi, V *phi, const bem_solve_opts &o,
            bem_solve_info *info) {
    Ctx &c = *t.ctx;
    const int64_t n = t.mesh->n_dof;
    const int m = o.restart;
    const int method = o.method;
    Krylov<V> K(c, n, m);
    DBuf<V> b, r, d;
    b.alloc(&c, n);
    r.alloc(&c, n);
    d.alloc(&c, n);
    int status = BEM_OK;
    for (int rhs = 0; rhs < nrhs; rhs++) {
        bem_solve_info inf{};
        const V *ch = chi + (int64_t)rhs * n;
        V *x = phi + (int64_t)rhs * n;
        matvec(t, green, k, BEM_OP_RHS, method, BEM_PREC_FP64, 1, ch, b.p);
        inf.matvecs++;
        auto A64 = [&](const V *in, V *out) { matvec(t, green, k, BEM_OP_A, method, BEM_PREC_FP64, 1, in, out); };
        auto A32 = [&](const V *in, V *out) { matvec(t, green, k, BEM_OP_A, method, BEM_PREC_MIXED, 1, in, out); };
        int st;
        double res = 0.0;
        if (o.precision == BEM_PREC_FP64 || method == BEM_DIRECT) {
            zero_fill(c, x, sizeof(V) * n);
            st = gmres(K, A64, b.p, x, o.tol, o.max_restarts, &inf.iterations, &inf.matvecs, &res, true);
        } else {
            zero_fill(c, x, sizeof(V) * n);
            BEM_HIP(hipMemcpyAsync(r.p, b.p, sizeof(V) * n, hipMemcpyDeviceToDevice, c.stream));
            double bnorm = K.norm(b.p);
            st = BEM_ENOCONV;
            for (int it = 0; it < o.max_refine; it++) {
                zero_fill(c, d.p, sizeof(V) * n);
                double inner = 0.0;
                gmres(K, A32, r.p, d.p, o.inner_tol, o.max_restarts, &inf.iterations, &inf.matvecs, &inner, true);
                k_axpy<V><<<nblocks(n, RBS), RBS, 0, c.stream>>>(V(0.0), d.p, x, n, 1.0);
                BEM_LAUNCH_CHECK();
                A64(x, K.tmp.p);
                inf.matvecs++;
                k_sub<V><<<nblocks(n, RBS), RBS, 0, c.stream>>>(b.p, K.tmp.p, r.p, n);
                BEM_LAUNCH_CHECK();
                inf.refinements++;
                res = bnorm > 0 ? K.norm(r.p) / bnorm : 0.0;
                if (res <= o.tol) { st = BEM_OK; break; }
            }
        }
        inf.residual = res;
        inf.status = st;
        if (st != BEM_OK) status = st;
        if (info) info[rhs] = inf;
    }
    c.sync();
    return status;
}

}  // namespace

int solve(bem_tree &t, int green, double k, int nrhs, const void *chi, void *phi, const bem_solve_opts &o,
          bem_solve_info *info) {
    if (green == BEM_HELMHOLTZ)
        return solve_t<cx<double>>(t, green, k, nrhs, (const cx<double> *)chi, (cx<double> *)phi, o, info);
    return solve_t<double>(t, green, k, nrhs, (const double *)chi, (double *)phi, o, info);
}

}  // namespace bem
