// Iterative solution of Eq. (3) (Section 2.1: the paper uses a matrix-free
// Krylov solver, BiCGSTAB, around the fast product).  GMRES with restart is
// the default here; BiCGSTAB is the other option (bicgstab() below).
//
// GMRES(m) from x0 = 0: Arnoldi with classical Gram-Schmidt applied twice
// (CGS2), the Hessenberg column rotated by complex Givens rotations on the
// device, one residual-estimate word read by the host per iteration, and a
// device back-substitution at the end of each cycle.  All Krylov arithmetic
// is FP64 (complex128 for Helmholtz); the inner products reduce in a fixed
// order, so repeated solves are bitwise identical.
//
// Precision modes (both methods):
//   FP64   the method on the FP64 operator to tol.
//   MIXED  the same method, whose steps switch to the mixed-precision
//          product once the residual is small enough for its error not to
//          matter (relaxed inexact Krylov); the residual that decides
//          convergence is always formed with the FP64 product.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>

#include "kernels.h"

namespace bem {

namespace {

constexpr int RBS = 256;

// Budget of a solve: Krylov steps per right-hand side (0: none) and the wall
// time of the whole call (0: none), checked on the host after every step.
struct Budget {
    int max_iters;
    double max_seconds;
    std::chrono::steady_clock::time_point t0;
    Budget(int it, double sec) : max_iters(it), max_seconds(sec), t0(std::chrono::steady_clock::now()) {}
    bool out_of_steps(int iters) const { return max_iters > 0 && iters >= max_iters; }
    bool out_of_time() const {
        return max_seconds > 0.0 &&
               std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() >= max_seconds;
    }
};

__device__ inline double cj(double v) { return v; }
__device__ inline cx<double> cj(cx<double> v) { return conj(v); }
__device__ inline double abs2(double v) { return v * v; }
__device__ inline double abs2(cx<double> v) { return v.re * v.re + v.im * v.im; }

constexpr int DOT_BLK = 64;  // blocks of a reduction over a vector

// Partial sums cross blocks (and the XCDs' separate L2 caches) through
// device-scope atomic stores and loads.
__device__ inline void st_dev(double *p, double v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline double ld_dev(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_dev(cx<double> *p, cx<double> v) {
    st_dev(&p->re, v.re);
    st_dev(&p->im, v.im);
}
__device__ inline cx<double> ld_dev(const cx<double> *p) { return cx<double>(ld_dev(&p->re), ld_dev(&p->im)); }

// Sum over the block's threads by a fixed tree; the result is returned to
// every thread.
template <class V>
__device__ V block_sum(V v, V *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = RBS / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const V s = red[0];
    __syncthreads();
    return s;
}

// Row `row` of a reduction has gridDim.x blocks, each of which has stored its
// partial sum at part[row * gridDim.x + blockIdx.x].  Returns, in every
// thread, the row's total (partial sums added in block order, so the result
// does not depend on which block finishes last) to the block that finishes
// the row last, and false to the others.  The row's counter is left at zero.
template <class V>
__device__ bool row_total(V *part, unsigned *count, int row, V *red, V *total) {
    __shared__ int last;
    const int nblk = gridDim.x;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(count + row, 1u) == (unsigned)nblk - 1;
        if (last) {
            atomicExch(count + row, 0u);
            __threadfence();
        }
    }
    __syncthreads();
    if (!last) return false;
    if ((int)threadIdx.x < nblk) red[threadIdx.x] = ld_dev(part + (int64_t)row * nblk + threadIdx.x);
    __syncthreads();
    V t = V(0.0);
    for (int b = 0; b < nblk; b++) t += red[b];
    *total = t;
    return true;
}

// Grid (nblk, rows + 1): row r < rows reduces conj(V_r) . w (V_r at basis +
// r ld), row `rows` reduces conj(w) . w.  Totals go to out[r] (the last row
// to out[rows]); with acc, acc[r] += total as well for r < rows; with
// host_self, the real part of the last row's total also goes to that
// host-mapped word.
template <class V>
__global__ void __launch_bounds__(RBS) k_rows(const V *basis, int64_t ld, const V *w, int64_t n, int rows, V *part,
                                              unsigned *count, V *out, V *acc, double *host_self) {
    __shared__ V red[RBS];
    const int r = blockIdx.y, nblk = gridDim.x;
    const V *v = r < rows ? basis + (int64_t)r * ld : w;
    V s = V(0.0);
    for (int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x; e < n; e += (int64_t)nblk * RBS) s += cj(v[e]) * w[e];
    s = block_sum(s, red);
    if (threadIdx.x == 0) st_dev(part + (int64_t)r * nblk + blockIdx.x, s);
    V t;
    if (!row_total(part, count, r, red, &t)) return;
    if (threadIdx.x == 0) {
        out[r] = t;
        if (r < rows && acc) acc[r] += t;
        if (r == rows && host_self) *host_self = re_part(t);
    }
}

// Givens update of the Hessenberg least-squares problem at step j: hcol
// holds column j (j + 2 entries, hcol[j+1] = |w| real).  Applies the
// previous rotations, forms the new one, stores the rotated column into H,
// updates g and returns |g[j+1]|, the residual estimate.
template <class V>
__device__ double givens_step(V *H, int ldh, const V *hcol, V *cs, V *sn, V *g, int j) {
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
    return sqrt(abs2(g[j + 1]));
}

// Second half of Arnoldi step j (after the first Gram-Schmidt pass and the
// second pass's coefficients h2 = hc2[0..j]): w -= sum_{i <= j} h2[i] V_i,
// then |w|^2 reduced over the grid.  The block that completes the sum ends
// the step: hcol[j+1] = |w|, the breakdown test (|w| <= 1e-14 |w before the
// orthogonalisation|, from wn2), the Givens update, and for the host (the
// host-mapped words hout[0] = residual estimate, hout[1] = breakdown) and the
// device (*flag = breakdown).
template <class V>
__global__ void __launch_bounds__(RBS) k_arnoldi_end(const V *basis, int64_t ld, const V *h2, V *w, int64_t n,
                                                     V *part, unsigned *count, V *hcol, const V *wn2, V *H, int ldh,
                                                     V *cs, V *sn, V *g, int j, int *flag, double *hout) {
    __shared__ V red[RBS];
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x; e < n; e += (int64_t)gridDim.x * RBS) {
        V acc = w[e];
        for (int i = 0; i <= j; i++) acc -= h2[i] * basis[(int64_t)i * ld + e];
        w[e] = acc;
        s += abs2(acc);
    }
    V t;
    {
        const V bs = block_sum(V(s), red);
        if (threadIdx.x == 0) st_dev(part + blockIdx.x, bs);
    }
    if (!row_total(part, count, 0, red, &t)) return;
    if (threadIdx.x != 0) return;
    const double hn = sqrt(re_part(t)), wn = sqrt(re_part(wn2[0]));
    const int breakdown = hn <= 1e-14 * wn;
    hcol[j + 1] = V(hn);
    const double est = givens_step(H, ldh, hcol, cs, sn, g, j);
    *flag = breakdown;
    hout[0] = est;
    hout[1] = breakdown;
}

// w -= sum_{i < m} h[i] Vi
template <class V>
__global__ void k_subtract(const V *basis, int64_t ld, const V *h, int m, V *w, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x; e < n; e += (int64_t)gridDim.x * RBS) {
        V acc = w[e];
        for (int i = 0; i < m; i++) acc -= h[i] * basis[(int64_t)i * ld + e];
        w[e] = acc;
    }
}

// V_{j+1} = w / hcol[j+1] unless step j broke down
template <class V>
__global__ void k_scale_into(const V *w, const V *hcol, int j, const int *flag, V *out, int64_t n) {
    if (*flag) return;
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
__global__ void k_sub(const V *a, const V *b, V *out, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    if (e < n) out[e] = a[e] - b[e];
}

// ---------------------------------------------------------------- BiCGSTAB
// Scalars on the device, in the slots written by the reductions:
//   [0] rho = (rh, r)  [1] |r|^2   [2] (rh, v)   [3] |v|^2 (unused)
//   [4] (t, s)         [5] |s|^2   [6] |t|^2     [8] rho of the previous step
//   [9] alpha          [10] omega
// (inner products conjugate their first argument).  Each vector kernel forms
// the scalars it needs itself, so no host round trip sits inside a step.
enum { BI_RHO = 0, BI_V = 2, BI_TS = 4, BI_TT = 6, BI_RHO0 = 8, BI_ALPHA = 9, BI_OMEGA = 10, BI_NS = 12 };

__device__ inline double vdiv(double a, double b) { return a / b; }
__device__ inline cx<double> vdiv(cx<double> a, cx<double> b) { return a * conj(b) * (1.0 / abs2(b)); }

// p = r + beta (p - omega v), beta = (rho / rho0) (alpha / omega)
template <class V>
__global__ void k_bicg_p(const V *sc, const V *r, const V *v, V *p, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    if (e >= n) return;
    const V beta = vdiv(sc[BI_RHO], sc[BI_RHO0]) * vdiv(sc[BI_ALPHA], sc[BI_OMEGA]);
    p[e] = r[e] + beta * (p[e] - sc[BI_OMEGA] * v[e]);
}

// alpha = rho / (rh, v); s = r - alpha v; the step's rho becomes rho0
template <class V>
__global__ void k_bicg_s(V *sc, const V *r, const V *v, V *s, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    const V alpha = vdiv(sc[BI_RHO], sc[BI_V]);
    if (e < n) s[e] = r[e] - alpha * v[e];
    if (e == 0) {
        sc[BI_ALPHA] = alpha;
        sc[BI_RHO0] = sc[BI_RHO];
    }
}

// omega = (t, s) / |t|^2; x += alpha p + omega s; r = s - omega t.  On a
// breakdown (alpha or omega not finite: (rh, v) = 0 or t = 0) x is kept and
// r is set to NaN, so that the host ends the cycle and restarts from x.
__device__ inline bool vfinite(double v) { return isfinite(v); }
__device__ inline bool vfinite(cx<double> v) { return isfinite(v.re) && isfinite(v.im); }

template <class V>
__global__ void k_bicg_x(V *sc, const V *p, const V *s, const V *t, V *x, V *r, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * RBS + threadIdx.x;
    const V omega = sc[BI_TS] * (1.0 / re_part(sc[BI_TT]));
    const V alpha = sc[BI_ALPHA];
    const bool ok = vfinite(alpha) && vfinite(omega);  // the same for every thread
    if (e < n) {
        if (ok) {
            x[e] = x[e] + alpha * p[e] + omega * s[e];
            r[e] = s[e] - omega * t[e];
        } else {
            r[e] = V(NAN);
        }
    }
    if (e == 0) sc[BI_OMEGA] = omega;
}

template <class V>
__global__ void k_bicg_reset(V *sc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        for (int i = 0; i < BI_NS; i++) sc[i] = V(0.0);
        sc[BI_RHO0] = V(1.0);
        sc[BI_ALPHA] = V(1.0);
        sc[BI_OMEGA] = V(1.0);
    }
}

template <class V>
struct Krylov {
    Ctx &c;
    int64_t n;
    int m;
    int nblk;
    DBuf<V> basis, w, hcol, hc2, H, cs, sn, g, y, part, tmp;
    DBuf<unsigned> count;  // completed blocks per reduction row, zero between launches
    DBuf<int> flag;        // breakdown of the last Arnoldi step
    // pinned, host-mapped words written by the kernels and read after a
    // stream sync: [0] residual estimate, [1] breakdown, [2] |v|^2 of norm_async
    double *h_out = nullptr, *d_out = nullptr;

    Krylov(Ctx &c_, int64_t n_, int m_) : c(c_), n(n_), m(m_) {
        nblk = (int)std::min<int64_t>(DOT_BLK, nblocks(n, RBS));
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
        part.alloc(&c, (size_t)(m + 2) * nblk);
        count.alloc(&c, m + 2);
        count.zero();
        flag.alloc(&c, 1);
        BEM_HIP(hipHostMalloc((void **)&h_out, 4 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
        BEM_HIP(hipHostGetDevicePointer((void **)&d_out, h_out, 0));
    }
    ~Krylov() {
        if (h_out) (void)hipHostFree(h_out);
    }
    V *vec(int i) { return basis.p + (int64_t)i * n; }

    // out[i] = conj(V_i) . v for i < cnt (V_i at base + i n) and out[cnt] =
    // |v|^2; with acc, acc[i] += out[i] for i < cnt; with host_self, |v|^2
    // also goes to that host-mapped word.  One launch.
    void rows(const V *base, int cnt, const V *v, V *out, V *acc, double *host_self) {
        dim3 g2(nblk, cnt + 1);
        k_rows<V><<<g2, RBS, 0, c.stream>>>(base, n, v, n, cnt, part.p, count.p, out, acc, host_self);
        BEM_LAUNCH_CHECK();
    }
    // |v|^2 into h_out[2] (read after a stream sync)
    void norm_async(const V *v) { rows(nullptr, 0, v, hc2.p, nullptr, d_out + 2); }
};

// |v_i| of each (K_i, v_i), with one stream sync for all of them.
template <class V>
std::vector<double> norms(std::vector<Krylov<V> *> &K, const std::vector<const V *> &v) {
    for (size_t i = 0; i < K.size(); i++) K[i]->norm_async(v[i]);
    if (!K.empty()) K[0]->c.sync();
    std::vector<double> out(K.size());
    for (size_t i = 0; i < K.size(); i++) out[i] = std::sqrt(K[i]->h_out[2]);
    return out;
}

// Lock-step GMRES(m) for several right-hand sides.  Each right-hand side r
// runs exactly the iteration a solve of r alone runs (its own Krylov space,
// rotations, decisions and kernels, in the same order); only the operator
// products of the right-hand sides that need one at a step are applied
// together, as one multi-vector product (whose columns equal single
// products bit for bit), and the host reads every residual estimate of a
// step after one synchronisation.  x_r holds the initial guess (zero when
// zero_x0) and receives the result.
//
// apply(in, out, cnt, prec) is the operator in precision prec.  Residuals at
// the start of a cycle are always FP64 products.  Inside a cycle a step uses
// the mixed product once the right-hand side's current relative residual is
// at most mixed_below (never when negative): the relaxation of inexact
// Krylov methods (Simoncini and Szyld 2003; Bouras and Fraysse 2005), where
// a product error of relative size d at a step whose residual is r perturbs
// the attained residual by about d r, so d r <= tol / 10 keeps the FP64
// residual at the end within tol.  A cycle whose FP64 residual misses tol
// restarts from there (counted in restarts[r]).
template <class V, class F>
void gmres(std::vector<Krylov<V> *> &K, F &&apply, V *stage_in, V *stage_out, const std::vector<const V *> &b,
           const std::vector<V *> &x, double tol, int max_cycles, double mixed_below, const Budget &bud, int *iters,
           int *matvecs, int *restarts, double *relres, int *status, bool zero_x0) {
    const size_t nr = K.size();
    if (!nr) return;
    Ctx &c = K[0]->c;
    const int64_t n = K[0]->n;
    const int m = K[0]->m;
    const unsigned nb = nblocks(n, RBS);
    // A x_r for the right-hand sides in `set`, through the staging buffers
    auto apply_set = [&](const std::vector<size_t> &set, const std::vector<const V *> &in,
                         const std::vector<V *> &out, int prec) {
        if (set.empty()) return;
        if (set.size() == 1) {  // a single product needs no staging
            apply(in[0], out[0], 1, prec);
            matvecs[set[0]]++;
            return;
        }
        for (size_t i = 0; i < set.size(); i++)
            BEM_HIP(hipMemcpyAsync(stage_in + (int64_t)i * n, in[i], sizeof(V) * n, hipMemcpyDeviceToDevice, c.stream));
        apply(stage_in, stage_out, (int)set.size(), prec);
        for (size_t i = 0; i < set.size(); i++) {
            BEM_HIP(hipMemcpyAsync(out[i], stage_out + (int64_t)i * n, sizeof(V) * n, hipMemcpyDeviceToDevice,
                                   c.stream));
            matvecs[set[i]]++;
        }
    };
    std::vector<double> bnorm;
    {
        std::vector<Krylov<V> *> Ks(K.begin(), K.end());
        bnorm = norms(Ks, std::vector<const V *>(b.begin(), b.end()));
    }
    std::vector<size_t> act;  // right-hand sides still iterating
    for (size_t r = 0; r < nr; r++) {
        status[r] = BEM_ENOCONV;
        if (bnorm[r] == 0.0) {
            zero_fill(c, x[r], sizeof(V) * n);
            relres[r] = 0.0;
            status[r] = BEM_OK;
        } else {
            act.push_back(r);
        }
    }
    std::vector<size_t> spent;  // right-hand sides out of steps or time: stopped where they are
    for (int cycle = 0; cycle < max_cycles && !act.empty(); cycle++) {
        // r0 = b - A x into V0
        if (zero_x0 && cycle == 0) {
            for (size_t r : act)
                BEM_HIP(hipMemcpyAsync(K[r]->vec(0), b[r], sizeof(V) * n, hipMemcpyDeviceToDevice, c.stream));
        } else {
            std::vector<const V *> in;
            std::vector<V *> out;
            for (size_t r : act) {
                in.push_back(x[r]);
                out.push_back(K[r]->tmp.p);
            }
            apply_set(act, in, out, BEM_PREC_FP64);
            for (size_t r : act) {
                k_sub<V><<<nb, RBS, 0, c.stream>>>(b[r], K[r]->tmp.p, K[r]->vec(0), n);
                BEM_LAUNCH_CHECK();
            }
        }
        std::vector<Krylov<V> *> Ka;
        std::vector<const V *> v0;
        for (size_t r : act) {
            Ka.push_back(K[r]);
            v0.push_back(K[r]->vec(0));
        }
        const std::vector<double> beta = norms(Ka, v0);
        std::vector<size_t> run;  // right-hand sides running this cycle's Arnoldi process
        std::vector<double> beta_run;
        for (size_t i = 0; i < act.size(); i++) {
            const size_t r = act[i];
            relres[r] = beta[i] / bnorm[r];
            if (relres[r] <= tol) status[r] = BEM_OK;
            else {
                if (cycle > 0) restarts[r]++;
                run.push_back(r);
                beta_run.push_back(beta[i]);
            }
        }
        act = run;
        for (size_t i = 0; i < run.size(); i++) {
            Krylov<V> &Kr = *K[run[i]];
            const double inv = 1.0 / beta_run[i];
            zero_fill(c, Kr.tmp.p, sizeof(V) * n);
            k_axpy<V><<<nb, RBS, 0, c.stream>>>(V(0.0), Kr.vec(0), Kr.tmp.p, n, inv);
            BEM_LAUNCH_CHECK();
            BEM_HIP(hipMemcpyAsync(Kr.vec(0), Kr.tmp.p, sizeof(V) * n, hipMemcpyDeviceToDevice, c.stream));
            std::vector<V> g0(m + 1, V(0.0));
            g0[0] = V(beta_run[i]);
            Kr.g.upload(g0.data(), m + 1);
        }
        std::vector<int> jdone(nr, 0);
        std::vector<size_t> live = run;  // still in this cycle's Arnoldi process
        for (int j = 0; j < m && !live.empty(); j++) {
            for (int prec : {BEM_PREC_FP64, BEM_PREC_MIXED}) {
                std::vector<size_t> set;
                std::vector<const V *> in;
                std::vector<V *> out;
                for (size_t r : live) {
                    const bool mixed = relres[r] <= mixed_below;
                    if (mixed != (prec == BEM_PREC_MIXED)) continue;
                    set.push_back(r);
                    in.push_back(K[r]->vec(j));
                    out.push_back(K[r]->w.p);
                }
                apply_set(set, in, out, prec);
            }
            // CGS2: h1 and |w|^2 in one launch, w -= V h1, h2 (added into h),
            // then w -= V h2 with |w|, the breakdown test, the Givens update and
            // the residual estimate in one launch, and V_{j+1} = w / |w|
            for (size_t r : live) {
                Krylov<V> &Kr = *K[r];
                Kr.rows(Kr.basis.p, j + 1, Kr.w.p, Kr.hcol.p, nullptr, nullptr);
                k_subtract<V><<<nb, RBS, 0, c.stream>>>(Kr.basis.p, n, Kr.hcol.p, j + 1, Kr.w.p, n);
                BEM_LAUNCH_CHECK();
                Kr.rows(Kr.basis.p, j + 1, Kr.w.p, Kr.hc2.p, Kr.hcol.p, nullptr);
                k_arnoldi_end<V><<<Kr.nblk, RBS, 0, c.stream>>>(Kr.basis.p, n, Kr.hc2.p, Kr.w.p, n, Kr.part.p,
                                                                 Kr.count.p, Kr.hcol.p, Kr.hcol.p + j + 1, Kr.H.p, m,
                                                                 Kr.cs.p, Kr.sn.p, Kr.g.p, j, Kr.flag.p, Kr.d_out);
                BEM_LAUNCH_CHECK();
                k_scale_into<V><<<nb, RBS, 0, c.stream>>>(Kr.w.p, Kr.hcol.p, j, Kr.flag.p, Kr.vec(j + 1), n);
                BEM_LAUNCH_CHECK();
            }
            c.sync();
            std::vector<size_t> next;
            const bool late = bud.out_of_time();
            for (size_t i = 0; i < live.size(); i++) {
                const size_t r = live[i];
                iters[r]++;
                jdone[r] = j + 1;
                relres[r] = K[r]->h_out[0] / bnorm[r];
                const bool breakdown = K[r]->h_out[1] != 0.0;
                if (relres[r] <= tol || breakdown) continue;
                if (late || bud.out_of_steps(iters[r])) {
                    spent.push_back(r);  // leaves the cycle; its iterate is formed below
                    continue;
                }
                next.push_back(r);
            }
            live = next;
        }
        for (size_t r : run) {
            Krylov<V> &Kr = *K[r];
            k_backsolve<V><<<1, 1, 0, c.stream>>>(Kr.H.p, m, Kr.g.p, jdone[r], Kr.y.p);
            BEM_LAUNCH_CHECK();
            k_lincomb<V><<<nb, RBS, 0, c.stream>>>(Kr.basis.p, n, Kr.y.p, jdone[r], x[r], n);
            BEM_LAUNCH_CHECK();
        }
        // a right-hand side that has spent its budget starts no further cycle
        if (!spent.empty()) {
            std::vector<size_t> keep;
            for (size_t r : act)
                if (std::find(spent.begin(), spent.end(), r) == spent.end()) keep.push_back(r);
            act = keep;
        }
        if (bud.out_of_time()) {  // every right-hand side stops where it is
            spent.insert(spent.end(), act.begin(), act.end());
            act.clear();
        }
    }
    act.insert(act.end(), spent.begin(), spent.end());
    std::sort(act.begin(), act.end());
    // final explicit residual of those that did not stop at a cycle start
    if (!act.empty()) {
        std::vector<const V *> in;
        std::vector<V *> out;
        for (size_t r : act) {
            in.push_back(x[r]);
            out.push_back(K[r]->tmp.p);
        }
        apply_set(act, in, out, BEM_PREC_FP64);
        std::vector<Krylov<V> *> Ka;
        std::vector<const V *> wa;
        for (size_t r : act) {
            k_sub<V><<<nb, RBS, 0, c.stream>>>(b[r], K[r]->tmp.p, K[r]->w.p, n);
            BEM_LAUNCH_CHECK();
            Ka.push_back(K[r]);
            wa.push_back(K[r]->w.p);
        }
        const std::vector<double> rn = norms(Ka, wa);
        for (size_t i = 0; i < act.size(); i++) {
            const size_t r = act[i];
            relres[r] = rn[i] / bnorm[r];
            status[r] = relres[r] <= tol ? BEM_OK : BEM_ENOCONV;
        }
    }
}

// BiCGSTAB (van der Vorst 1992; the paper's Krylov solver, Section 2.1) for
// one right-hand side from x = 0.  Each cycle starts from the FP64 residual
// r = b - A x (r itself at the first), runs up to `steps` steps of two
// products each and ends early once the recursively updated residual meets
// tol; a cycle whose FP64 residual then misses tol restarts from x (counted
// in restarts).  Products switch to the mixed precision below mixed_below
// as in gmres().  Inner products reduce in a fixed order; the host reads |r|
// once per step.
template <class V, class F>
void bicgstab(Krylov<V> &K, F &&apply, const V *b, V *x, double tol, int max_cycles, int steps, double mixed_below,
              const Budget &bud, int *iters, int *matvecs, int *restarts, double *relres, int *status) {
    Ctx &c = K.c;
    const int64_t n = K.n;
    const unsigned nb = nblocks(n, RBS);
    V *r = K.vec(0), *rh = K.vec(1), *p = K.vec(2), *v = K.vec(3), *s = K.vec(4), *tv = K.vec(5), *tmp = K.tmp.p;
    DBuf<V> sc;
    sc.alloc(&c, BI_NS);
    std::vector<Krylov<V> *> Kv{&K};
    const double bnorm = norms(Kv, std::vector<const V *>{b})[0];
    *status = BEM_ENOCONV;
    if (bnorm == 0.0) {
        zero_fill(c, x, sizeof(V) * n);
        *relres = 0.0;
        *status = BEM_OK;
        return;
    }
    bool spent = bud.out_of_time();  // out of steps or time: the FP64 residual of x, then stop
    for (int cycle = 0;; cycle++) {
        // r = b - A x in FP64 (b itself while x = 0)
        if (cycle == 0) {
            BEM_HIP(hipMemcpyAsync(r, b, sizeof(V) * n, hipMemcpyDeviceToDevice, c.stream));
        } else {
            apply(x, tmp, 1, BEM_PREC_FP64);
            (*matvecs)++;
            k_sub<V><<<nb, RBS, 0, c.stream>>>(b, tmp, r, n);
            BEM_LAUNCH_CHECK();
        }
        BEM_HIP(hipMemcpyAsync(rh, r, sizeof(V) * n, hipMemcpyDeviceToDevice, c.stream));
        k_bicg_reset<V><<<1, 1, 0, c.stream>>>(sc.p);
        BEM_LAUNCH_CHECK();
        zero_fill(c, p, sizeof(V) * n);
        zero_fill(c, v, sizeof(V) * n);
        K.rows(rh, 1, r, sc.p + BI_RHO, nullptr, K.d_out + 2);  // rho and |r|^2
        c.sync();
        double rel = std::sqrt(K.h_out[2]) / bnorm;
        *relres = rel;
        if (rel <= tol) {
            *status = BEM_OK;
            return;
        }
        if (cycle >= max_cycles || spent || !(rel == rel)) return;  // out of budget, or the iterate is not finite
        if (cycle > 0) (*restarts)++;
        for (int it = 0; it < steps; it++) {
            const int prec = rel <= mixed_below ? BEM_PREC_MIXED : BEM_PREC_FP64;
            k_bicg_p<V><<<nb, RBS, 0, c.stream>>>(sc.p, r, v, p, n);
            BEM_LAUNCH_CHECK();
            apply(p, v, 1, prec);
            K.rows(rh, 1, v, sc.p + BI_V, nullptr, nullptr);
            k_bicg_s<V><<<nb, RBS, 0, c.stream>>>(sc.p, r, v, s, n);
            BEM_LAUNCH_CHECK();
            apply(s, tv, 1, prec);
            *matvecs += 2;
            K.rows(tv, 1, s, sc.p + BI_TS, nullptr, nullptr);
            K.rows(nullptr, 0, tv, sc.p + BI_TT, nullptr, nullptr);
            k_bicg_x<V><<<nb, RBS, 0, c.stream>>>(sc.p, p, s, tv, x, r, n);
            BEM_LAUNCH_CHECK();
            K.rows(rh, 1, r, sc.p + BI_RHO, nullptr, K.d_out + 2);
            c.sync();
            (*iters)++;
            rel = std::sqrt(K.h_out[2]) / bnorm;
            if (!(rel == rel) || rel <= tol) break;  // converged, or broke down (x kept): FP64 residual, restart
            if (bud.out_of_steps(*iters) || bud.out_of_time()) {
                spent = true;
                break;
            }
        }
    }
}

template <class V>
int solve_t(bem_tree &t, int green, double k, int nrhs, const V *chi, V *phi, const bem_solve_opts &o,
            bem_solve_info *info) {
    const Budget bud(o.max_iters, o.max_seconds);
    Ctx &c = *t.ctx;
    const int64_t n = t.mesh->n_dof;
    const int m = o.restart;
    const int method = o.method;
    std::vector<std::unique_ptr<Krylov<V>>> Kown;
    std::vector<Krylov<V> *> K;
    for (int r = 0; r < nrhs; r++) {
        Kown.push_back(std::make_unique<Krylov<V>>(c, n, m));
        K.push_back(Kown.back().get());
    }
    DBuf<V> b, sin, sout;
    b.alloc(&c, (size_t)nrhs * n);
    sin.alloc(&c, (size_t)nrhs * n);
    sout.alloc(&c, (size_t)nrhs * n);
    std::vector<bem_solve_info> inf(nrhs);
    for (auto &i : inf) i = bem_solve_info{};
    std::vector<int> iters(nrhs, 0), mv(nrhs, 0), rs(nrhs, 0), st(nrhs, BEM_ENOCONV);
    std::vector<double> res(nrhs, 0.0);
    // right-hand sides b = -S chi, all at once (columns equal single products)
    matvec(t, green, k, BEM_OP_RHS, method, BEM_PREC_FP64, nrhs, chi, b.p);
    for (auto &i : inf) i.matvecs++;
    auto A = [&](const V *in, V *out, int cnt, int prec) {
        matvec(t, green, k, BEM_OP_A, method, prec, cnt, in, out);
    };
    auto col = [&](V *base, int r) { return base + (int64_t)r * n; };
    std::vector<const V *> bv;
    std::vector<V *> xv;
    for (int r = 0; r < nrhs; r++) {
        bv.push_back(col(b.p, r));
        xv.push_back(col(phi, r));
        zero_fill(c, xv[r], sizeof(V) * n);
    }
    // MIXED: steps whose residual r satisfies inner_tol * r <= tol / 10 use the
    // mixed product (inner_tol bounds its relative deviation from the FP64 one)
    const bool mixed = o.precision == BEM_PREC_MIXED && method == BEM_FMM;
    const double mixed_below = mixed ? 0.1 * o.tol / o.inner_tol : -1.0;
    if (o.krylov == BEM_KRYLOV_BICGSTAB) {
        // one right-hand side after the other, each with its own vectors
        for (int r = 0; r < nrhs; r++) {
            Krylov<V> Kb(c, n, 6);
            bicgstab(Kb, A, bv[r], xv[r], o.tol, o.max_restarts, o.restart, mixed_below, bud, &iters[r], &mv[r],
                     &rs[r], &res[r], &st[r]);
        }
    } else {
        gmres(K, A, sin.p, sout.p, bv, xv, o.tol, o.max_restarts, mixed_below, bud, iters.data(), mv.data(),
              rs.data(), res.data(), st.data(), true);
    }
    for (int r = 0; r < nrhs; r++) {
        inf[r].iterations += iters[r];
        inf[r].matvecs += mv[r];
        inf[r].restarts = rs[r];
        inf[r].residual = res[r];
        inf[r].status = st[r];
    }
    c.sync();
    int status = BEM_OK;
    for (int r = 0; r < nrhs; r++) {
        if (inf[r].status != BEM_OK) status = inf[r].status;
        if (info) info[r] = inf[r];
    }
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
