// Multipole-to-local translation (Eq. 9) as batched MFMA products.
//
// With moments and locals scaled by their box sides (see fmm.hip), the
// translation from a source box s to a target box t is
//
//   Fh_b(t) += (rho_t/rho_s)^|b| / (b! rho_s) * sum_a D_{a+b}(r) (-1)^|a| Mh_a(s)
//
// where D are the derivatives of G at r = (c_t - c_s)/rho_s with wavenumber
// k rho_s (the source side is never smaller than the target side: interaction
// lists hold same-level boxes and coarser leaves).  Because box centres sit
// on the lattice of their level, 2^(dl+1) r is an integer vector (dl = level
// difference), so pairs fall into a small number of exact displacement
// classes: (dl, 2^(dl+1) r) for Laplace, whose scaled operator does not
// depend on the level, plus the source level for Helmholtz.  Each class's
// derivative table is computed once per tree (FP64, Section 3.3 recursion)
// and the pairs of a class form one dense product
//
//     OUT[b, j] = sum_a T_c[b, a] M'[a, j],    T_c[b, a] = D_c[a + b]
//
// run on the matrix cores (v_mfma 16x16x4, FP32 or FP64): one wave takes a
// class and up to 16 pair columns (8 complex pairs as 16 real columns), the
// class table lives in LDS indexed by packed multi-index keys so that the
// A operand T_c[b, a] is a single LDS read, and the M' columns (signed,
// divided by rho_s) are staged in LDS.  Each pair's result goes to its slot
// in the interaction list; a second kernel sums every target box's slots in
// list order, so the result does not depend on scheduling (no float atomics).
#include <cmath>
#include <unordered_map>

#include "greens.h"
#include "kernels.h"

namespace bem {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int MT = 11;              // 176 / 16 output row tiles (P = 165 at order 8)
constexpr int KT = 42;              // 168 / 4 contraction steps

__host__ __device__ inline int ncoef(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
__host__ __device__ inline int midx(int a, int b, int c) {
    int n = a + b + c;
    return n * (n + 1) * (n + 2) / 6 + (n - a) * (n - a + 1) / 2 + (n - a - b);
}

__device__ inline floatx4 mfma(float a, float b, floatx4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ inline doublex4 mfma(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row of the 16x16 result held in element r of a lane (column = lane % 16):
// the f32 instruction gives row 4 (lane / 16) + r, the f64 one row lane / 16 + 4 r.
__device__ inline int crow(float, int kq, int r) { return 4 * kq + r; }
__device__ inline int crow(double, int kq, int r) { return kq + 4 * r; }

template <class R> struct vec4;
template <> struct vec4<float> { using type = floatx4; };
template <> struct vec4<double> { using type = doublex4; };

// ---------------------------------------------------------------- class tables (FP64)
// One block per class: G^(h)(R), h = 0..H, then d^g G^(h) for |g| <= H - h,
// h descending (Section 3.3, Eq. 12), at the normalised separation.
template <bool HELM>
__global__ void k_class_derivs(const double *rbar, const double *kbar, int H, const int8_t *exps, double *D64,
                               float *D32) {
    using V = typename std::conditional<HELM, cx<double>, double>::type;
    extern __shared__ unsigned char smem[];
    const int P2 = ncoef(H);
    V *A = (V *)smem, *B = A + P2, *g = B + P2;
    const int c = blockIdx.x, tid = threadIdx.x;
    const double r[3] = {rbar[3 * c], rbar[3 * c + 1], rbar[3 * c + 2]};
    const double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2], Rr = sqrt(R2);
    if (tid == 0) {
        if constexpr (!HELM) {
            g[0] = kInv4Pi / Rr;
            for (int h = 0; h < H; h++) g[h + 1] = g[h] * (-(double)(2 * h + 1) / R2);
        } else {
            const double kk = kbar[c];
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
        const int m = ncoef(H - h);
        for (int i = tid; i < m; i += blockDim.x) {
            V v;
            if (i == 0) {
                v = g[h];
            } else {
                int al[3] = {exps[3 * i], exps[3 * i + 1], exps[3 * i + 2]};
                int d = al[0] > 0 ? 0 : (al[1] > 0 ? 1 : 2);
                al[d]--;
                v = prev[midx(al[0], al[1], al[2])] * r[d];
                if (al[d] > 0) {
                    int ad = al[d];
                    al[d]--;
                    v += prev[midx(al[0], al[1], al[2])] * (double)ad;
                }
            }
            cur[i] = v;
        }
        __syncthreads();
        V *t = prev; prev = cur; cur = t;
    }
    for (int i = tid; i < P2; i += blockDim.x) {
        if constexpr (HELM) {
            D64[2 * ((int64_t)c * P2 + i)] = prev[i].re;
            D64[2 * ((int64_t)c * P2 + i) + 1] = prev[i].im;
            D32[2 * ((int64_t)c * P2 + i)] = (float)prev[i].re;
            D32[2 * ((int64_t)c * P2 + i) + 1] = (float)prev[i].im;
        } else {
            D64[(int64_t)c * P2 + i] = prev[i];
            D32[(int64_t)c * P2 + i] = (float)prev[i];
        }
    }
}

struct M2lArgs {
    const int32_t *task_class, *task_first, *task_count, *pair_list, *inter_idx, *level, *cls_delta;
    const int32_t *pk;           // [KT*4] packed multi-index a | b << 5 | c << 10 (0 for padding)
    double side;
    int P, P2;
    int64_t n_box, n_inter;
};

constexpr int M2L_WAVES = 4;
constexpr int OUT_LD = MT * 16;  // row stride of the per-pair outputs (176)

// index of the multi-index sum of two packed multi-indices (graded order)
__device__ inline int sum_index(int packed) {
    const int a = packed & 31, b = (packed >> 5) & 31, c = packed >> 10;
    const int n = a + b + c, m = n - a;
    return (n * (n + 1) * (n + 2)) / 6 + ((m * (m + 1)) >> 1) + (m - b);
}

// Real values: a block of four waves takes one class and up to 64 of its
// pairs, 16 per wave; the class table is shared by the waves.
template <class R>
__global__ void __launch_bounds__(64 * M2L_WAVES) k_m2l_mfma(M2lArgs a, const R *D, const R *inv_fact, const R *mom,
                                                             R *out) {
    using V4 = typename vec4<R>::type;
    extern __shared__ unsigned char smem[];
    const int P = a.P, P2 = a.P2;
    R *Dc = (R *)smem;                         // [P2]
    R *rs = Dc + P2;                           // [OUT_LD] row scales of the class
    int *pk = (int *)(rs + OUT_LD);            // [KT*4]
    R *MsAll = (R *)(pk + KT * 4);             // [waves][KT*4][16]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, task = blockIdx.x;
    const int c = a.task_class[task], first = a.task_first[task], cnt = a.task_count[task];
    const int delta = a.cls_delta[c];
    for (int i = tid; i < P2; i += blockDim.x) Dc[i] = D[(int64_t)c * P2 + i];
    for (int i = tid; i < KT * 4; i += blockDim.x) pk[i] = a.pk[i];
    for (int i = tid; i < OUT_LD; i += blockDim.x) {
        R v = 0;
        if (i < P) {
            const int q = a.pk[i], nb = (q & 31) + ((q >> 5) & 31) + (q >> 10);
            v = inv_fact[i] * (R)ldexp(1.0, -delta * nb);
        }
        rs[i] = v;
    }
    __syncthreads();
    const int wfirst = first + 16 * wave, wcnt = min(16, cnt - 16 * wave);
    if (wcnt <= 0) return;
    R *Ms = MsAll + wave * (KT * 4 * 16);
    // sources and scales of the wave's columns, fetched in parallel
    int my_s = -1;
    R my_scale = 0;
    if (lane < wcnt) {
        my_s = a.inter_idx[a.pair_list[wfirst + lane]];
        my_scale = (R)ldexp(1.0 / a.side, a.level[my_s]);
    }
#pragma unroll 4
    for (int col = 0; col < 16; col++) {
        const int s = __shfl(my_s, col, 64);
        const R scale = __shfl(my_scale, col, 64);
        for (int al = lane; al < KT * 4; al += 64) {
            R v = 0;
            if (s >= 0 && al < P) {
                const int q = pk[al], na = (q & 31) + ((q >> 5) & 31) + (q >> 10);
                v = mom[(int64_t)s * P + al] * ((na & 1) ? -scale : scale);
            }
            Ms[al * 16 + col] = v;
        }
    }
    // each wave reads only the staging area it wrote: no block barrier is needed
    __builtin_amdgcn_wave_barrier();
    const int row = lane & 15, kq = lane >> 4;
    int pb[MT];
    for (int mt = 0; mt < MT; mt++) pb[mt] = pk[min(16 * mt + row, KT * 4 - 1)] * (16 * mt + row < P ? 1 : 0);
    V4 acc[MT];
    for (int mt = 0; mt < MT; mt++) acc[mt] = V4{0, 0, 0, 0};
    for (int kt = 0; kt < KT; kt++) {
        const int al = 4 * kt + kq;
        const int pa = pk[al];
        const R bv = Ms[al * 16 + row];
#pragma unroll
        for (int mt = 0; mt < MT; mt++) acc[mt] = mfma(Dc[sum_index(pb[mt] + pa)], bv, acc[mt]);
    }
    const int col = row;
    if (col < wcnt) {
        const int j = a.pair_list[wfirst + col];
        R *o = out + (int64_t)j * OUT_LD;
        for (int mt = 0; mt < MT; mt++)
            for (int r = 0; r < 4; r++) {
                const int b = 16 * mt + crow(R(0), kq, r);
                o[b] = acc[mt][r] * rs[b];
            }
    }
}

// Complex values: 8 pairs per wave, real and imaginary parts as 16 real columns.
template <class R>
__global__ void __launch_bounds__(64 * M2L_WAVES) k_m2l_mfma_cx(M2lArgs a, const R *D /* interleaved */,
                                                                const R *inv_fact, const cx<R> *mom, cx<R> *out) {
    using V4 = typename vec4<R>::type;
    extern __shared__ unsigned char smem[];
    const int P = a.P, P2 = a.P2;
    R *Dr = (R *)smem;
    R *Di = Dr + P2;
    R *rs = Di + P2;
    int *pk = (int *)(rs + OUT_LD);
    R *MsAll = (R *)(pk + KT * 4);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, task = blockIdx.x;
    const int c = a.task_class[task], first = a.task_first[task], cnt = a.task_count[task];
    const int delta = a.cls_delta[c];
    for (int i = tid; i < P2; i += blockDim.x) {
        Dr[i] = D[2 * ((int64_t)c * P2 + i)];
        Di[i] = D[2 * ((int64_t)c * P2 + i) + 1];
    }
    for (int i = tid; i < KT * 4; i += blockDim.x) pk[i] = a.pk[i];
    for (int i = tid; i < OUT_LD; i += blockDim.x) {
        R v = 0;
        if (i < P) {
            const int q = a.pk[i], nb = (q & 31) + ((q >> 5) & 31) + (q >> 10);
            v = inv_fact[i] * (R)ldexp(1.0, -delta * nb);
        }
        rs[i] = v;
    }
    __syncthreads();
    const int wfirst = first + 8 * wave, wcnt = min(8, cnt - 8 * wave);
    if (wcnt <= 0) return;
    R *Ms = MsAll + wave * (KT * 4 * 16);
    int my_s = -1;
    R my_scale = 0;
    if (lane < wcnt) {
        my_s = a.inter_idx[a.pair_list[wfirst + lane]];
        my_scale = (R)ldexp(1.0 / a.side, a.level[my_s]);
    }
#pragma unroll 2
    for (int p = 0; p < 8; p++) {
        const int s = __shfl(my_s, p, 64);
        const R scale = __shfl(my_scale, p, 64);
        for (int al = lane; al < KT * 4; al += 64) {
            R vr = 0, vi = 0;
            if (s >= 0 && al < P) {
                const int q = pk[al], na = (q & 31) + ((q >> 5) & 31) + (q >> 10);
                const R f = (na & 1) ? -scale : scale;
                const cx<R> m = mom[(int64_t)s * P + al];
                vr = m.re * f;
                vi = m.im * f;
            }
            Ms[al * 16 + p] = vr;
            Ms[al * 16 + 8 + p] = vi;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int row = lane & 15, kq = lane >> 4;
    int pb[MT];
    for (int mt = 0; mt < MT; mt++) pb[mt] = pk[min(16 * mt + row, KT * 4 - 1)] * (16 * mt + row < P ? 1 : 0);
    V4 accR[MT], accI[MT];
    for (int mt = 0; mt < MT; mt++) {
        accR[mt] = V4{0, 0, 0, 0};
        accI[mt] = V4{0, 0, 0, 0};
    }
    for (int kt = 0; kt < KT; kt++) {
        const int al = 4 * kt + kq;
        const int pa = pk[al];
        const R bv = Ms[al * 16 + row];
#pragma unroll
        for (int mt = 0; mt < MT; mt++) {
            const int ix = sum_index(pb[mt] + pa);
            accR[mt] = mfma(Dr[ix], bv, accR[mt]);
            accI[mt] = mfma(Di[ix], bv, accI[mt]);
        }
    }
    // lane with column p < 8 holds Tr.Mr and Ti.Mr of pair p; lane ^ 8 holds Tr.Mi and Ti.Mi
    const int p = row & 7;
    const bool lo = row < 8;
    const int j = (lo && p < wcnt) ? a.pair_list[wfirst + p] : -1;
    for (int mt = 0; mt < MT; mt++)
        for (int r = 0; r < 4; r++) {
            R trmi = __shfl_xor(accR[mt][r], 8, 64);
            R timi = __shfl_xor(accI[mt][r], 8, 64);
            const int b = 16 * mt + crow(R(0), kq, r);
            if (j >= 0) {
                const R f = rs[b];
                out[(int64_t)j * OUT_LD + b] = cx<R>((accR[mt][r] - timi) * f, (trmi + accI[mt][r]) * f);
            }
        }
}

// Fh(b) += sum of the b's interaction-list slots, in list order.
template <class V>
__global__ void k_m2l_reduce(const int32_t *boxes, const int64_t *iptr, int P, const V *out, V *loc) {
    const int b = boxes[blockIdx.x];
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        V acc = V(0.0);
        const int64_t j0 = iptr[b], j1 = iptr[b + 1];
        int64_t j = j0;
        for (; j + 4 <= j1; j += 4) {
            const V v0 = out[j * OUT_LD + i], v1 = out[(j + 1) * OUT_LD + i], v2 = out[(j + 2) * OUT_LD + i],
                    v3 = out[(j + 3) * OUT_LD + i];
            acc += v0;
            acc += v1;
            acc += v2;
            acc += v3;
        }
        for (; j < j1; j++) acc += out[j * OUT_LD + i];
        loc[(int64_t)b * P + i] += acc;
    }
}

struct ClassKey {
    int32_t d, q0, q1, q2, ls;
    bool operator==(const ClassKey &o) const {
        return d == o.d && q0 == o.q0 && q1 == o.q1 && q2 == o.q2 && ls == o.ls;
    }
};
struct ClassKeyHash {
    size_t operator()(const ClassKey &k) const {
        uint64_t h = (uint64_t)(uint32_t)k.d * 0x9E3779B97F4A7C15ull;
        for (int32_t v : {k.q0, k.q1, k.q2, k.ls}) h = (h ^ (uint32_t)v) * 0x100000001B3ull + (h >> 29);
        return (size_t)h;
    }
};

uint64_t compact3h(uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < 21; b++) r |= ((v >> (3 * b)) & 1u) << b;
    return r;
}

}  // namespace

M2lPlan &get_m2l_plan(bem_tree &t, int green, double k) {
    if (green == BEM_LAPLACE) k = 0.0;
    for (auto &p : t.m2l)
        if (p->green == green && p->k == k) return *p;
    Ctx &c = *t.ctx;
    fmm_tables(t);
    plan_fmm(t);
    FmmTables &T = *t.tables;
    const int p = t.order, P = T.P, P2 = T.P2, H = 2 * p;
    BEM_REQUIRE(P <= MT * 16 && P <= KT * 4, BEM_EUNSUPPORTED, "expansion order too high for the M2L tiles");
    const bool helm = green == BEM_HELMHOLTZ;
    auto pl = std::make_unique<M2lPlan>();
    pl->green = green;
    pl->k = k;
    if (t.h_prefix.empty()) t.h_prefix = t.prefix.download(t.n_box);
    // classes of the interaction pairs of boxes with targets
    std::unordered_map<ClassKey, int32_t, ClassKeyHash> id;
    std::vector<std::vector<int32_t>> members;
    std::vector<int32_t> cdelta;
    std::vector<double> rbar, kbar;
    for (int64_t b = 0; b < t.n_box; b++) {
        if (t.h_te[b] == t.h_tb[b]) continue;
        const uint64_t pb = t.h_prefix[b];
        const int64_t ib[3] = {(int64_t)compact3h(pb >> 2), (int64_t)compact3h(pb >> 1), (int64_t)compact3h(pb)};
        for (int64_t j = t.h_inter_ptr[b]; j < t.h_inter_ptr[b + 1]; j++) {
            const int32_t s = t.h_inter_idx[j];
            const int d = t.h_level[b] - t.h_level[s];
            const uint64_t ps = t.h_prefix[s];
            const int64_t is[3] = {(int64_t)compact3h(ps >> 2), (int64_t)compact3h(ps >> 1), (int64_t)compact3h(ps)};
            int64_t q[3];
            for (int e = 0; e < 3; e++) q[e] = (2 * ib[e] + 1) - ((2 * is[e] + 1) << d);
            ClassKey key{d, (int32_t)q[0], (int32_t)q[1], (int32_t)q[2], helm ? t.h_level[s] : -1};
            auto it = id.find(key);
            int32_t cid;
            if (it == id.end()) {
                cid = (int32_t)members.size();
                id.emplace(key, cid);
                members.emplace_back();
                cdelta.push_back(d);
                for (int e = 0; e < 3; e++) rbar.push_back(std::ldexp((double)q[e], -(d + 1)));
                kbar.push_back(k * std::ldexp(t.side, -t.h_level[s]));
            } else {
                cid = it->second;
            }
            members[cid].push_back((int32_t)j);
        }
    }
    pl->n_class = (int64_t)members.size();
    const int cols = (helm ? 8 : 16) * M2L_WAVES;
    std::vector<int32_t> plist, tc, tf, tn;
    for (int32_t cl = 0; cl < (int32_t)members.size(); cl++) {
        const int32_t base = (int32_t)plist.size();
        plist.insert(plist.end(), members[cl].begin(), members[cl].end());
        for (size_t o = 0; o < members[cl].size(); o += cols) {
            tc.push_back(cl);
            tf.push_back(base + (int32_t)o);
            tn.push_back((int32_t)std::min<size_t>(cols, members[cl].size() - o));
        }
    }
    pl->n_pairs = (int64_t)plist.size();
    pl->n_task = (int64_t)tc.size();
    auto up = [&](DBuf<int32_t> &d, const std::vector<int32_t> &v) {
        d.alloc(&c, v.size());
        d.upload(v.data(), v.size());
    };
    up(pl->pair_list, plist);
    up(pl->task_class, tc);
    up(pl->task_first, tf);
    up(pl->task_count, tn);
    up(pl->cls_delta, cdelta);
    // packed multi-indices of the contraction rows
    std::vector<int8_t> ex = T.h_exps;
    std::vector<int32_t> pk(KT * 4, 0);
    for (int i = 0; i < P; i++) pk[i] = ex[3 * i] | (ex[3 * i + 1] << 5) | (ex[3 * i + 2] << 10);
    up(pl->pk, pk);
    // class derivative tables
    const int cw = helm ? 2 : 1;
    pl->D64.alloc(&c, (size_t)cw * P2 * std::max<int64_t>(1, pl->n_class));
    pl->D32.alloc(&c, (size_t)cw * P2 * std::max<int64_t>(1, pl->n_class));
    if (pl->n_class) {
        DBuf<double> drb, dkb;
        drb.alloc(&c, rbar.size());
        drb.upload(rbar.data(), rbar.size());
        dkb.alloc(&c, kbar.size());
        dkb.upload(kbar.data(), kbar.size());
        size_t sh = (size_t)cw * sizeof(double) * (2 * P2 + H + 2);
        if (helm)
            k_class_derivs<true><<<(unsigned)pl->n_class, 256, sh, c.stream>>>(drb.p, dkb.p, H, T.exps.p, pl->D64.p,
                                                                               pl->D32.p);
        else
            k_class_derivs<false><<<(unsigned)pl->n_class, 256, sh, c.stream>>>(drb.p, dkb.p, H, T.exps.p, pl->D64.p,
                                                                                pl->D32.p);
        BEM_LAUNCH_CHECK();
        c.sync();
    }
    t.m2l.push_back(std::move(pl));
    return *t.m2l.back();
}

template <class V, class R>
void m2l_apply(bem_tree &t, M2lPlan &pl, int nrhs, const V *mom, V *loc) {
    Ctx &c = *t.ctx;
    FmmTables &T = *t.tables;
    const int P = T.P;
    if (!pl.n_task) return;
    t.work.m2l_out.ensure(&c, sizeof(V) * (size_t)std::max<int64_t>(1, t.n_inter) * OUT_LD);
    V *out = (V *)t.work.m2l_out.p;
    M2lArgs a{pl.task_class.p, pl.task_first.p, pl.task_count.p, pl.pair_list.p, t.inter_idx.p, t.level.p,
              pl.cls_delta.p, pl.pk.p, t.side, P, T.P2, t.n_box, t.n_inter};
    const int cw = std::is_same<V, R>::value ? 1 : 2;
    const size_t sh = sizeof(R) * (cw * T.P2 + OUT_LD) + sizeof(int) * KT * 4 + sizeof(R) * M2L_WAVES * KT * 4 * 16;
    const bool f32 = std::is_same<R, float>::value;
    const R *invf = f32 ? (const R *)T.inv_fact32.p : (const R *)T.inv_fact64.p;
    const R *D = f32 ? (const R *)pl.D32.p : (const R *)pl.D64.p;
    if (sh > 64 * 1024) {
        if constexpr (std::is_same<V, R>::value)
            BEM_HIP(hipFuncSetAttribute((const void *)k_m2l_mfma<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
        else
            BEM_HIP(hipFuncSetAttribute((const void *)k_m2l_mfma_cx<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)sh));
    }
    for (int rhs = 0; rhs < nrhs; rhs++) {
        const V *m = mom + (int64_t)rhs * t.n_box * P;
        V *l = loc + (int64_t)rhs * t.n_box * P;
        if constexpr (std::is_same<V, R>::value)
            k_m2l_mfma<R><<<(unsigned)pl.n_task, 64 * M2L_WAVES, sh, c.stream>>>(a, D, invf, m, out);
        else
            k_m2l_mfma_cx<R><<<(unsigned)pl.n_task, 64 * M2L_WAVES, sh, c.stream>>>(a, D, invf, m, out);
        BEM_LAUNCH_CHECK();
        k_m2l_reduce<V><<<(unsigned)t.n_m2l_boxes, 192, 0, c.stream>>>(t.m2l_boxes.p, t.inter_ptr.p, P, out, l);
        BEM_LAUNCH_CHECK();
    }
}

template void m2l_apply<double, double>(bem_tree &, M2lPlan &, int, const double *, double *);
template void m2l_apply<float, float>(bem_tree &, M2lPlan &, int, const float *, float *);
template void m2l_apply<cx<double>, double>(bem_tree &, M2lPlan &, int, const cx<double> *, cx<double> *);
template void m2l_apply<cx<float>, float>(bem_tree &, M2lPlan &, int, const cx<float> *, cx<float> *);

}  // namespace bem
