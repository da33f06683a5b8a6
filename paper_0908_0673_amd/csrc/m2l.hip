// Multipole-to-local translation (Eq. 9) as batched MFMA products.
//
// With moments and locals scaled by their box sides (see fmm.hip), the
// translation from a source box s to a target box t is
//
//   Fh_b(t) += (rho_t/rho_s)^|b| / (b! rho_s) * sum_a D_{a+b}(r) (-1)^|a| Mh_a(s)
//
// where D are the derivatives of G at r = (c_t - c_s)/rho_s with wavenumber
// k rho_s (the source side is never smaller than the target side: interaction
// lists hold same-level boxes and coarser leaves).  Box centres sit on the
// lattice of their level, so q = 2^(dl+1) r is an integer vector (dl = level
// difference).  G depends on |r| only, so for any signed permutation of the
// axes, r_e = s_e r'_{pi(e)}, the derivatives obey
//
//   D_g(r) = s^g D'_{g'}(r'),   g'_{pi(e)} = g_e,   s^g = prod_e s_e^(g_e),
//
// and every pair reduces to a canonical displacement r' = sorted |r|: the
// translation is the canonical operator applied to the moments permuted and
// signed into the canonical frame, its result permuted and signed back.
// Pairs therefore fall into few exact canonical classes, (dl, sorted |q|)
// for Laplace, whose scaled operator does not depend on the level, plus the
// source level for Helmholtz.  Each class's derivative table is computed once
// per tree (FP64, Section 3.3 recursion) and its pairs form one dense product
//
//     OUT[b', j] = sum_a' T_c[b', a'] M'[a', j],
//     T_c[b', a'] = rs_c[b'] (-1)^|a'| D'_c[a' + b'],  rs_c[b'] = 2^(-dl |b'|) / b'!
//
// run on the matrix cores (v_mfma 16x16x4 in FP64, or FP32 for mixed products
// with level-dependent orders; 16x16x32 fp16 on split operands for the other
// mixed products, below).  T_c is expanded
// once per tree into the A-operand order of the instruction, so a wave
// streams it with one coalesced 256-byte load per product; the canonical
// operators of a tree take a few MB and stay resident in the L2 caches.  One
// wave takes a class and up to 16 NCG pair columns (8 complex pairs as 16
// real columns); its B operands are the pairs' moments in the canonical
// frame, which a small kernel first writes once per used (source box,
// symmetry) combination so that the product reads them contiguously, and it
// stores each pair's canonical result whole (the stores are contiguous).
// Tasks are ordered so that every wave of a class is dispatched to the same
// XCD (blocks go round-robin over the 8 XCDs), whose L2 then holds that
// class's operator.  FP64 path: each pair's result goes to its slot in the
// interaction list, and a second kernel sums every target box's slots in
// list order.  Mixed path (one order for all levels): the products run on
// the fp16 instruction with split operands, and each wave sums its pairs of
// one target box in the box's frame before writing (see k_m2l_x2); a second
// kernel adds a box's partial sums in plan order.  Either way the result does
// not depend on scheduling (no float atomics).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <type_traits>

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
// One block per class: the derivatives of G up to order H at the class's
// normalised separation (greens.h, Section 3.3, Eq. 12).
template <bool HELM>
__global__ void k_class_derivs(const double *rbar, const double *kbar, int H, const int8_t *exps, double *D64) {
    using V = typename std::conditional<HELM, cx<double>, double>::type;
    extern __shared__ unsigned char smem[];
    const int P2 = ncoef(H);
    V *A = (V *)smem, *B = A + P2, *g = B + P2;
    const int c = blockIdx.x, tid = threadIdx.x;
    const double r[3] = {rbar[3 * c], rbar[3 * c + 1], rbar[3 * c + 2]};
    const V *D = derivs_block<HELM>(r, HELM ? kbar[c] : 0.0, H, exps, A, B, g);
    for (int i = tid; i < P2; i += blockDim.x) {
        if constexpr (HELM) {
            D64[2 * ((int64_t)c * P2 + i)] = D[i].re;
            D64[2 * ((int64_t)c * P2 + i) + 1] = D[i].im;
        } else {
            D64[(int64_t)c * P2 + i] = D[i];
        }
    }
}

constexpr int OUT_LD = MT * 16;                // row stride of the per-pair outputs (176)
constexpr int KIN = KT * 4;                    // contraction length (168)
constexpr int TSZ = MT * KT * 64;              // expanded operator, A-operand order
constexpr int NSYM = 48;                       // signed permutations of the axes
constexpr int32_t SYM_NEG = 1 << 30;           // symmetry-table flag: negate the value

// index of the multi-index sum of two packed multi-indices (graded order)
__device__ inline int sum_index(int packed) {
    const int a = packed & 31, b = (packed >> 5) & 31, c = packed >> 10;
    const int n = a + b + c, m = n - a;
    return (n * (n + 1) * (n + 2)) / 6 + ((m * (m + 1)) >> 1) + (m - b);
}

// T_c[b][a] = rs_c[b] (-1)^|a| D_c[a + b], laid out as [kt][mt][lane] with
// b = 16 mt + lane % 16, a = 4 kt + lane / 16; complex tables hold the real
// plane then the imaginary plane.
template <class R, bool HELM>
__global__ void k_expand_T(const double *D64, const int32_t *pk, const int32_t *cls_delta, const double *inv_fact,
                           int P, int P2, R *T) {
    const int c = blockIdx.x, mk = blockIdx.y, lane = threadIdx.x;
    const int kt = mk / MT, mt = mk % MT;
    const int b = 16 * mt + (lane & 15), al = 4 * kt + (lane >> 4);
    double vr = 0.0, vi = 0.0;
    if (b < P && al < P) {
        const int qa = pk[al], qb = pk[b];
        const int na = (qa & 31) + ((qa >> 5) & 31) + (qa >> 10);
        const int nb = (qb & 31) + ((qb >> 5) & 31) + (qb >> 10);
        const double f = inv_fact[b] * ldexp(1.0, -cls_delta[c] * nb) * ((na & 1) ? -1.0 : 1.0);
        const int ix = sum_index(qa + qb);
        if (HELM) {
            vr = f * D64[2 * ((int64_t)c * P2 + ix)];
            vi = f * D64[2 * ((int64_t)c * P2 + ix) + 1];
        } else {
            vr = f * D64[(int64_t)c * P2 + ix];
        }
    }
    const int64_t o = (int64_t)(HELM ? 2 * c : c) * TSZ + (int64_t)mk * 64 + lane;
    T[o] = (R)vr;
    if (HELM) T[o + TSZ] = (R)vi;
}

struct M2lArgs {
    const int32_t *task_class, *task_first, *task_count;
    const int32_t *pair_slot, *pair_src, *pair_mom, *level;
    const int32_t *task_kt, *task_mt;  // level-dependent order: steps and row tiles each task needs

    double side;
    int P;
    int64_t slot0;  // first interaction slot of the slab: results go to out[slot - slot0]
    // split path: partial slot and symmetry of each pair, the symmetry
    // table back to the pairs' frames; slot0 is then the slab's first partial
    const int32_t *pair_part, *pair_sym;
    const int16_t *sym_red;
    // split path: power-of-two exponent of each canonical moment vector and
    // 2^-exponent of each class's operator, undone on the results
    const int32_t *u_exp;
    const float *cls_scale;
    // split path: the symmetry table in compact form, sym_perm[o][i] = the
    // canonical row of row i under axis ordering o (o = sym / 8), then
    // sym_perm[6][i] = the axes along which row i's multi-index is odd (the
    // result is negated when an odd number of them are flipped, sym % 8)
    const uint8_t *sym_perm;
};

__device__ inline float abs_max(float x) { return fabsf(x); }
__device__ inline float abs_max(cx<float> x) { return fmaxf(fabsf(x.re), fabsf(x.im)); }
__device__ inline float scaled(float x, int e) { return ldexpf(x, e); }
__device__ inline cx<float> scaled(cx<float> x, int e) { return cx<float>(ldexpf(x.re, e), ldexpf(x.im, e)); }

// Moments in the canonical frame of each used (source box, symmetry)
// combination u: Mc[u][a'] = sign * M_src[index], (index, sign) = sym_in[sym][a'],
// zero past P.  One wave per combination.  With u_exp (FP32 values, the split
// path) each vector is scaled by 2^e, e = u_exp[u], so that its largest
// component lies in [2^14, 2^15) (e = 0 for a zero vector).
template <class V>
__global__ void k_m2l_canonical_moments(int64_t n_u, const int32_t *u_src, const int32_t *u_sym,
                                        const int32_t *sym_in, int P, const V *mom, V *Mc, int32_t *u_exp) {
    far_field_priority();
    const int64_t u = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    if (u >= n_u) return;
    const int lane = threadIdx.x & 63;
    const V *ms = mom + (int64_t)u_src[u] * P;
    const int32_t *si = sym_in + u_sym[u] * KIN;
    constexpr int NIT = (KIN + 63) / 64;
    int32_t e[NIT];
    V v[NIT];
#pragma unroll
    for (int it = 0; it < NIT; it++) {
        const int a = lane + 64 * it;
        e[it] = a < P ? si[a] : -1;
    }
#pragma unroll
    for (int it = 0; it < NIT; it++) v[it] = e[it] >= 0 ? ms[e[it] & 0xffff] : V(0.0);
    if constexpr (std::is_same<V, float>::value || std::is_same<V, cx<float>>::value) {
        if (u_exp) {  // the same for the whole wave
            float m = 0.0f;
#pragma unroll
            for (int it = 0; it < NIT; it++) m = fmaxf(m, abs_max(v[it]));
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
            const int ex = m > 0.0f ? 14 - ilogbf(m) : 0;
#pragma unroll
            for (int it = 0; it < NIT; it++) v[it] = scaled(v[it], ex);
            if (lane == 0) u_exp[u] = ex;
        }
    }
#pragma unroll
    for (int it = 0; it < NIT; it++) {
        const int a = lane + 64 * it;
        if (a < KIN) Mc[u * KIN + a] = (e[it] >= 0 && (e[it] & SYM_NEG)) ? V(0.0) - v[it] : v[it];
    }
}

// Blocks of W waves share one class: the class's expanded operator
// streams through a double-buffered LDS ring in chunks of KC contraction
// steps (coalesced 16-byte loads, one chunk ahead, one barrier per chunk), and
// every wave reads its A operands from there for its own 16 pair columns, so
// each operator byte is fetched once per block rather than once per wave.
// The B operands (the columns' canonical moments) stream per wave through a
// register ring NB steps ahead.  W (2, 4 or 8 waves per block) is a launch
// choice the product's autotuner makes per shape class; it does not change the
// arithmetic (each column's sums run over the same steps in the same order).
constexpr int M2L_NB = 8;

// Row split: with MS = 2 the block's waves pair up, each computing half of
// the output row tiles of the same 16 columns, which halves the accumulators
// per wave (used where they would otherwise limit the waves per SIMD).
template <class R, int NA>
constexpr int m2l_ms() {
    return sizeof(R) * NA >= 8 ? 2 : 1;
}

template <class R, int NA, int W>
struct M2lChunk {
    static constexpr int KC = sizeof(R) * NA == 4 ? 6 : (sizeof(R) * NA == 8 ? 3 : 2);
    static constexpr int NCH = KT / KC;
    static constexpr int CE = KC * MT * 64;                     // values per chunk and plane
    static constexpr int U4 = CE * NA * (int)sizeof(R) / 16;    // 16-byte pieces per chunk
    static constexpr int PER = (U4 + 64 * W - 1) / (64 * W);
    static_assert(KT % KC == 0, "chunks must tile the contraction");
};

// NA = 1: real values, 16 pair columns per wave.  NA = 2: complex values, 8
// pairs per wave as 16 real columns (real parts, then imaginary parts) against
// the operator's real and imaginary planes.  Columns without a pair compute
// on the first canonical moments and are not stored.
// VAR (level-dependent order): a task stops after the chunks that cover its
// sources' coefficients (the moments past them are zero, so the skipped
// products add nothing) and computes and stores only the row tiles that
// cover its targets' coefficients (the reduction reads no other row).
template <class R, int NA, bool VAR, int W>
__global__ void __launch_bounds__(64 * W) k_m2l(M2lArgs a, const R *T, const R *Mc, R *out) {
    far_field_priority();
    using V4 = typename vec4<R>::type;
    using CK = M2lChunk<R, NA, W>;
    constexpr int KC = CK::KC, NCH = CK::NCH, CE = CK::CE, U4 = CK::U4, PER = CK::PER, NB = M2L_NB;
    constexpr int MS = m2l_ms<R, NA>(), MTH = (MT + MS - 1) / MS;
    __shared__ __align__(16) R As[2][NA * CE];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, task = blockIdx.x;
    const int cnt = a.task_count[task];
    if (cnt == 0) return;  // the same for the whole block
    const int c = a.task_class[task], first = a.task_first[task];
    const int nch = VAR ? (a.task_kt[task] + KC - 1) / KC : NCH;  // the same for the whole block
    const int mtn = VAR ? a.task_mt[task] : MT;
    const int col = lane & 15, kq = lane >> 4;
    const int cg = w / MS, mt0 = (w % MS) * MTH;  // column group and first row tile of this wave
    const int p = NA == 1 ? 16 * cg + col : 8 * cg + (col & 7);
    const int64_t u = p < cnt ? a.pair_mom[first + p] : 0;
    // lane's entries of its column: real values, or the real / imaginary part
    const R *ms = Mc + (u * KIN + kq) * NA + (NA == 2 && col >= 8 ? 1 : 0);
    const uint4 *Tg = (const uint4 *)(T + (int64_t)c * NA * TSZ);
    // pieces past the chunk are clamped to its last one: those threads load
    // and store the same value as its owner, so no branch is needed
    auto fetch = [&](int ch, uint4 (&r)[PER]) {
#pragma unroll
        for (int i = 0; i < PER; i++) {
            const int x = min(tid + 64 * W * i, U4 - 1);
            const int q = x / (U4 / NA), off = x % (U4 / NA);
            r[i] = Tg[(int64_t)q * (TSZ * (int)sizeof(R) / 16) + (int64_t)ch * (U4 / NA) + off];
        }
    };
    auto stash = [&](int buf, const uint4 (&r)[PER]) {
#pragma unroll
        for (int i = 0; i < PER; i++) ((uint4 *)As[buf])[min(tid + 64 * W * i, U4 - 1)] = r[i];
    };
    uint4 r[PER];
    fetch(0, r);
    R B[NB];
#pragma unroll
    for (int i = 0; i < NB; i++) B[i] = ms[NA * 4 * i];
    V4 acc[NA][MTH];
#pragma unroll
    for (int q = 0; q < NA; q++)
#pragma unroll
        for (int j = 0; j < MTH; j++) acc[q][j] = V4{0, 0, 0, 0};
    stash(0, r);
    __syncthreads();
    if (NCH > 1) fetch(1, r);
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) {
        if (VAR && ch >= nch) break;  // uniform over the block: no barrier is skipped by part of it
        const R *Ab = As[ch & 1] + lane;
#pragma unroll
        for (int kk = 0; kk < KC; kk++) {
            const int kt = ch * KC + kk, sb = kt % NB;
#pragma unroll
            for (int j = 0; j < MTH; j++)
                if ((MS == 1 || mt0 + j < MT) && (!VAR || mt0 + j < mtn))  // the same for the whole wave
#pragma unroll
                    for (int q = 0; q < NA; q++)
                        acc[q][j] = mfma(Ab[q * CE + (kk * MT + mt0 + j) * 64], B[sb], acc[q][j]);
            if (kt + NB < KT) B[sb] = ms[NA * 4 * (kt + NB)];
        }
        if (ch + 1 < NCH) {
            stash((ch + 1) & 1, r);  // that buffer's last readers passed the previous barrier
            __syncthreads();
            if (ch + 2 < NCH) fetch(ch + 2, r);
        }
    }
    const R scale = (R)ldexp(1.0 / a.side, a.level[p < cnt ? a.pair_src[first + p] : 0]);  // 1 / rho_s
    if constexpr (NA == 1) {
        if (p < cnt) {
            R *o = out + ((int64_t)a.pair_slot[first + p] - a.slot0) * OUT_LD;
#pragma unroll
            for (int j = 0; j < MTH; j++)
                if ((MS == 1 || mt0 + j < MT) && (!VAR || mt0 + j < mtn))
#pragma unroll
                    for (int r4 = 0; r4 < 4; r4++) o[16 * (mt0 + j) + crow(R(0), kq, r4)] = acc[0][j][r4] * scale;
        }
    } else {
        // lane with column < 8 holds Tr.Mr and Ti.Mr of its pair; lane ^ 8 holds Tr.Mi and Ti.Mi
        const bool store = col < 8 && p < cnt;
        cx<R> *o = (cx<R> *)out + (store ? (int64_t)a.pair_slot[first + p] - a.slot0 : 0) * OUT_LD;
#pragma unroll
        for (int j = 0; j < MTH; j++)
            if ((MS == 1 || mt0 + j < MT) && (!VAR || mt0 + j < mtn))
#pragma unroll
                for (int r4 = 0; r4 < 4; r4++) {
                    const R trmi = __shfl_xor(acc[0][j][r4], 8, 64);
                    const R timi = __shfl_xor(acc[1][j][r4], 8, 64);
                    if (store)
                        o[16 * (mt0 + j) + crow(R(0), kq, r4)] =
                            cx<R>((acc[0][j][r4] - timi) * scale, (trmi + acc[1][j][r4]) * scale);
                }
    }
}

// ---------------------------------------------------------------- split-fp16 products
// The mixed path runs the products on the fp16 matrix instruction
// v_mfma_f32_16x16x32_f16 (FP32 accumulation), whose dense rate on this chip
// (that of the bf16 one, measured at about fifteen times the FP32
// instruction's) far exceeds the FP32 one.  Every operand x is carried as two
// fp16 terms, x1 = fp16(x) and x2 = fp16(x - x1) (eleven significant bits
// each, together x to about 2^-22 relative), and each product keeps the three
// cross terms of combined order up to three,
//     x y ~ x1 y1 + (x1 y2 + x2 y1),
// the dropped x2 y2 being below 2^-22 relative; the smaller terms are
// accumulated first.  fp16's exponent range is narrow, so both operands are
// first scaled by powers of two (exact): every class's operator and every
// canonical moment vector so that its largest entry lies in [2^14, 2^15).
// Entries far below that largest lose relative precision to fp16's subnormal
// range, but never more than 2^-38 of it in absolute terms (in the scaled
// units every entry contributes in proportion to its size).  The scales are
// undone on the results (SPLIT_TOP below; the canonical-moments kernel above
// uses the same 14).  The contraction runs over K3 = 192 >= P in blocks of 32;
// a chunk of the operator is one block of one plane (the real or imaginary part):
// 11 row tiles x 2 terms x 1 KB, the A operands of the instruction in lane
// order (lane l holds row l % 16, columns 8 (l / 16) .. + 7 of its 16 x 32
// tile).
constexpr int KB = 6;                  // contraction blocks of 32
constexpr int K3 = KB * 32;            // 192
constexpr int TILE2 = 512;             // fp16 values of one A tile of one term
constexpr int CH2 = MT * 2 * TILE2;    // fp16 values of one chunk (one block of one plane)
constexpr int SPLIT_TOP = 14;          // scaled operands' largest entries lie in [2^14, 2^15)

typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

__device__ inline floatx4 mfma_h(uint4 a, uint4 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(halfx8, a), __builtin_bit_cast(halfx8, b), c, 0,
                                                  0, 0);
}

// two-term fp16 split (bit patterns) of an FP64 or FP32 value
__device__ inline void split2(double x, uint16_t *t) {
    const _Float16 h = (_Float16)(float)x;
    const _Float16 l = (_Float16)(float)(x - (double)h);
    t[0] = __builtin_bit_cast(uint16_t, h);
    t[1] = __builtin_bit_cast(uint16_t, l);
}
__device__ inline void split2(float x, uint16_t *t) {
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)(x - (float)h);  // x - h is exact in FP32
    t[0] = __builtin_bit_cast(uint16_t, h);
    t[1] = __builtin_bit_cast(uint16_t, l);
}

// Scales of the split operators: cls_scale[c] = 2^(ilogb(m) - 14),
// m = max |T_c[b][a]| over both planes (1 for a zero operator), so that
// T_c / cls_scale[c] has its largest entry in [2^14, 2^15).  One block of 256
// threads per class, a thread per row.
template <bool HELM>
__global__ void __launch_bounds__(256) k_cls_scale(const double *D64, const int32_t *pk, const int32_t *cls_delta,
                                                   const double *inv_fact, int P, int P2, float *cls_scale) {
    __shared__ double red[256];
    const int c = blockIdx.x, b = threadIdx.x;
    double m = 0.0;
    if (b < P) {
        const int qb = pk[b];
        const int nb = (qb & 31) + ((qb >> 5) & 31) + (qb >> 10);
        for (int al = 0; al < P; al++) {
            const int64_t ix = (int64_t)c * P2 + sum_index(pk[al] + qb);
            m = HELM ? fmax(m, fmax(fabs(D64[2 * ix]), fabs(D64[2 * ix + 1]))) : fmax(m, fabs(D64[ix]));
        }
        m *= inv_fact[b] * ldexp(1.0, -cls_delta[c] * nb);
    }
    red[b] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (b < h) red[b] = fmax(red[b], red[b + h]);
        __syncthreads();
    }
    // (the exponent is kept within FP32's normal range: operators of any
    // physical class are many orders of magnitude inside it)
    if (b == 0) cls_scale[c] = red[0] > 0.0 ? ldexpf(1.0f, max(-120, min(120, ilogb(red[0]) - SPLIT_TOP))) : 1.0f;
}

// T_c of k_expand_T as two-term splits of its scaled values:
// T2[((c KB + kb) NA + q) CH2 + (mt 2 + s) TILE2 + 8 lane + i] is term s of
// plane q of T_c[b][a] / cls_scale[c] with b = 16 mt + lane % 16,
// a = 32 kb + 8 (lane / 16) + i.
template <bool HELM>
__global__ void k_expand_T2(const double *D64, const int32_t *pk, const int32_t *cls_delta, const double *inv_fact,
                            int P, int P2, const float *cls_scale, uint16_t *T2) {
    constexpr int NA = HELM ? 2 : 1;
    const int c = blockIdx.x, kb = blockIdx.y / MT, mt = blockIdx.y % MT, lane = threadIdx.x;
    const int b = 16 * mt + (lane & 15);
    for (int i = 0; i < 8; i++) {
        const int al = 32 * kb + 8 * (lane >> 4) + i;
        double v[2] = {0.0, 0.0};
        if (b < P && al < P) {
            const int qa = pk[al], qb = pk[b];
            const int na = (qa & 31) + ((qa >> 5) & 31) + (qa >> 10);
            const int nb = (qb & 31) + ((qb >> 5) & 31) + (qb >> 10);
            const double f = inv_fact[b] * ldexp(1.0, -cls_delta[c] * nb) * ((na & 1) ? -1.0 : 1.0) /
                             (double)cls_scale[c];
            const int ix = sum_index(qa + qb);
            if (HELM) {
                v[0] = f * D64[2 * ((int64_t)c * P2 + ix)];
                v[1] = f * D64[2 * ((int64_t)c * P2 + ix) + 1];
            } else {
                v[0] = f * D64[(int64_t)c * P2 + ix];
            }
        }
        for (int q = 0; q < NA; q++) {
            uint16_t tt[2];
            split2(v[q], tt);
            const int64_t o = ((int64_t)(c * KB + kb) * NA + q) * CH2 + (int64_t)(mt * 2) * TILE2 + 8 * lane + i;
            for (int s2 = 0; s2 < 2; s2++) T2[o + s2 * TILE2] = tt[s2];
        }
    }
}

// The lane's eight B values of contraction block kb: moments a = 32 kb +
// 8 (lane / 16) + i of its column (real, or for complex tasks the real or
// imaginary part), zero past the stored KIN; FP32 as the canonical moments
// kernel writes them (scaled), split into fp16 terms only in registers.
template <int NA>
__device__ inline void load_b(const float *mr, int kb, int kq, bool imag, float (&v)[8]) {
    const int a0 = 32 * kb + 8 * kq;
    if (a0 >= KIN) {  // KIN is a multiple of 8
#pragma unroll
        for (int i = 0; i < 8; i++) v[i] = 0.0f;
        return;
    }
    if constexpr (NA == 1) {
        const float4 x0 = *(const float4 *)(mr + a0), x1 = *(const float4 *)(mr + a0 + 4);
        v[0] = x0.x; v[1] = x0.y; v[2] = x0.z; v[3] = x0.w;
        v[4] = x1.x; v[5] = x1.y; v[6] = x1.z; v[7] = x1.w;
    } else {  // interleaved (re, im)
        const float4 *pp = (const float4 *)(mr + 2 * a0);
#pragma unroll
        for (int h = 0; h < 4; h++) {
            const float4 y = pp[h];
            v[2 * h] = imag ? y.y : y.x;
            v[2 * h + 1] = imag ? y.w : y.z;
        }
    }
}
__device__ inline void split_b(const float (&v)[8], uint4 (&B)[2]) {
    uint16_t t[8][2];
#pragma unroll
    for (int i = 0; i < 8; i++) split2(v[i], t[i]);
#pragma unroll
    for (int s2 = 0; s2 < 2; s2++)
        B[s2] = make_uint4(t[0][s2] | (uint32_t)t[1][s2] << 16, t[2][s2] | (uint32_t)t[3][s2] << 16,
                           t[4][s2] | (uint32_t)t[5][s2] << 16, t[6][s2] | (uint32_t)t[7][s2] << 16);
}

// The products of one task on the split operands (as k_m2l with FP32 values,
// NA = 1 real or 2 complex, every contraction block and row tile): blocks of
// W waves share the class's operator, streamed through a double-buffered LDS
// ring one chunk ahead (one barrier per chunk), each wave owning 16 columns
// whose B operands it loads from the split moments one contraction block
// ahead.  The per-column arithmetic does not depend on W.
template <int NA, int W>
__global__ void __launch_bounds__(64 * W) k_m2l_x2(M2lArgs a, const uint4 *T2, const float *Mc, float *out) {
    far_field_priority();
    constexpr int U4 = CH2 * 2 / 16;  // 16-byte pieces per chunk
    constexpr int PER = (U4 + 64 * W - 1) / (64 * W);
    constexpr int NCH = KB * NA;
    constexpr int TB = 7 * OUT_LD;  // bytes of the compact symmetry table
    static_assert(TB % 16 == 0, "whole 16-byte pieces");
    __shared__ uint4 As[2][U4];
    __shared__ uint4 Ts[TB / 16];  // copy of the compact symmetry table back to the pairs' frames
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, task = blockIdx.x;
    const int cnt = a.task_count[task];
    if (cnt == 0) return;  // the same for the whole block
    const int c = a.task_class[task], first = a.task_first[task];
    const int col = lane & 15, kq = lane >> 4;
    const int p = NA == 1 ? 16 * w + col : 8 * w + (col & 7);
    const int64_t u = p < cnt ? a.pair_mom[first + p] : 0;
    // this lane's B values: its column's moments (complex tasks: columns 8..15
    // take the imaginary parts of the pairs of columns 0..7)
    const float *mr = Mc + u * KIN * NA;
    const bool imag = NA == 2 && col >= 8;
    const uint4 *Tg = T2 + (int64_t)c * NCH * U4;
    // pieces past the chunk are clamped to its last one: those threads load
    // and store the same value as its owner, so no branch is needed
    auto fetch = [&](int ch, uint4 (&r)[PER]) {
#pragma unroll
        for (int i = 0; i < PER; i++) r[i] = Tg[(int64_t)ch * U4 + min(tid + 64 * W * i, U4 - 1)];
    };
    auto stash = [&](int buf, const uint4 (&r)[PER]) {
#pragma unroll
        for (int i = 0; i < PER; i++) As[buf][min(tid + 64 * W * i, U4 - 1)] = r[i];
    };
    uint4 r[PER];
    fetch(0, r);
    // the table is read only after the products, so its copy is taken while
    // the first chunk is on its way (visible after the first barrier)
    for (int x = tid; x < TB / 16; x += 64 * W) Ts[x] = ((const uint4 *)a.sym_perm)[x];
    uint4 B[2];
    float bn[8];  // the next block's values, in flight
    load_b<NA>(mr, 0, kq, imag, bn);
    split_b(bn, B);
    load_b<NA>(mr, 1, kq, imag, bn);
    floatx4 acc[NA][MT];
#pragma unroll
    for (int q = 0; q < NA; q++)
#pragma unroll
        for (int j = 0; j < MT; j++) acc[q][j] = floatx4{0, 0, 0, 0};
    stash(0, r);
    __syncthreads();
    fetch(1, r);
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) {
        const int kb = ch / NA, q = ch % NA;
        if (q == 0 && kb > 0) {
            split_b(bn, B);
            if (kb + 1 < KB) load_b<NA>(mr, kb + 1, kq, imag, bn);
        }
        const uint4 *Ab = As[ch & 1] + lane;
#pragma unroll
        for (int j = 0; j < MT; j++) {
            const uint4 a0 = Ab[(2 * j) * 64], a1 = Ab[(2 * j + 1) * 64];
            floatx4 x = acc[q][j];
            x = mfma_h(a1, B[0], x);
            x = mfma_h(a0, B[1], x);
            x = mfma_h(a0, B[0], x);
            acc[q][j] = x;
        }
        if (ch + 1 < NCH) {
            stash((ch + 1) & 1, r);  // that buffer's last readers passed the previous barrier
            __syncthreads();
            if (ch + 2 < NCH) fetch(ch + 2, r);
        }
    }
    // Each pair's canonical result, unscaled (1 / rho_s, the moment vector's
    // and the operator's power-of-two scales), is taken back to its own frame
    // (row i is the canonical row sym_perm[sym / 8][i], negated when an odd
    // number of the flipped axes sym % 8 are odd in row i) and summed with the
    // pairs that follow it in the wave and share its target box (runs of
    // consecutive pairs, which share a partial slot), in passes of G pairs
    // staged in the LDS ring; each run's sum is written once, to its slot.
    const float scale =
        (float)(ldexp(1.0 / a.side, a.level[p < cnt ? a.pair_src[first + p] : 0] - a.u_exp[u]) * a.cls_scale[c]);
    using VO = typename std::conditional<NA == 1, float, cx<float>>::type;
    constexpr int G = 8;                          // pairs per pass: 5.5 (real) or 11 KB of staging per wave
    constexpr int PW = NA == 1 ? 16 : 8;          // pairs per wave
    constexpr int SB = W * G * OUT_LD * (int)sizeof(VO);  // staging bytes of the block
    static_assert(SB % 16 == 0 && SB <= 2 * U4 * 16, "staging exceeds the LDS ring");
    VO *S = (VO *)&As[0][0] + w * G * OUT_LD;
    const uint8_t *perm = (const uint8_t *)Ts, *odd = perm + 6 * OUT_LD;
    VO *o = (VO *)out;
    __syncthreads();  // every wave is past its last operator reads
#pragma unroll
    for (int h = 0; h < PW / G; h++) {
        const int c0 = h * G;        // first column (pair) of the pass
        const int pb = PW * w + c0;  // the pass's first pair in the task
        int part[G], sym[G];
#pragma unroll
        for (int cc = 0; cc < G; cc++) {
            const bool ok = pb + cc < cnt;
            part[cc] = ok ? a.pair_part[first + pb + cc] : -1;
            sym[cc] = ok ? a.pair_sym[first + pb + cc] : 0;
        }
#pragma unroll
        for (int j = 0; j < MT; j++) {
            VO *d = S + (col - c0) * OUT_LD + 16 * j + 4 * kq;  // 16-byte aligned
            if constexpr (NA == 1) {
                if (col >= c0 && col < c0 + G)
                    *(float4 *)d = make_float4(acc[0][j][0] * scale, acc[0][j][1] * scale, acc[0][j][2] * scale,
                                               acc[0][j][3] * scale);
            } else {
                // lane with column < 8 holds Tr.Mr and Ti.Mr of its pair; lane ^ 8 holds Tr.Mi and Ti.Mi
                float re[4], im[4];
#pragma unroll
                for (int r4 = 0; r4 < 4; r4++) {
                    const float trmi = __shfl_xor(acc[0][j][r4], 8, 64);
                    const float timi = __shfl_xor(acc[1][j][r4], 8, 64);
                    re[r4] = (acc[0][j][r4] - timi) * scale;
                    im[r4] = (trmi + acc[1][j][r4]) * scale;
                }
                if (col >= c0 && col < c0 + G) {
                    ((float4 *)d)[0] = make_float4(re[0], im[0], re[1], im[1]);
                    ((float4 *)d)[1] = make_float4(re[2], im[2], re[3], im[3]);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const int i = lane + 64 * r;
            const bool row = i < a.P;
            const int od = row ? odd[i] : 0;
            VO x[G];
#pragma unroll
            for (int cc = 0; cc < G; cc++) {
                const int e = row ? perm[(sym[cc] >> 3) * OUT_LD + i] : 0;
                const VO v = S[cc * OUT_LD + e];
                x[cc] = (__popc(sym[cc] & od) & 1) ? VO(0.0f) - v : v;
            }
            VO v = x[0];
#pragma unroll
            for (int cc = 1; cc <= G; cc++) {
                const bool end = cc == G || part[cc] != part[cc - 1];  // the same for the whole wave
                if (end) {
                    if (row && part[cc - 1] >= 0) o[(int64_t)(part[cc - 1] - a.slot0) * OUT_LD + i] = v;
                    if (cc < G) v = x[cc];
                } else {
                    v += x[cc];
                }
            }
        }
        __builtin_amdgcn_wave_barrier();  // the next pass overwrites the staging
    }
}

// The split path's M2L sums: each target box's locals are the sum of its
// partial slots (contiguous, in plan order).  One block per box of the slab.
template <class V>
__global__ void __launch_bounds__(256) k_m2l_sum_parts(const int32_t *boxes, const int64_t *part_ptr, int64_t part0,
                                                       int P, const V *parts, V *loc) {
    far_field_priority();
    const int b = boxes[blockIdx.x];
    const int64_t k0 = part_ptr[blockIdx.x] - part0, k1 = part_ptr[blockIdx.x + 1] - part0;
    for (int i = threadIdx.x; i < P; i += blockDim.x) {
        V v = V(0.0f);
        int64_t k = k0;
        for (; k + 4 <= k1; k += 4) {  // four loads in flight, added in order
            const V x0 = parts[k * OUT_LD + i], x1 = parts[(k + 1) * OUT_LD + i];
            const V x2 = parts[(k + 2) * OUT_LD + i], x3 = parts[(k + 3) * OUT_LD + i];
            v += x0;
            v += x1;
            v += x2;
            v += x3;
        }
        for (; k < k1; k++) v += parts[k * OUT_LD + i];
        loc[(int64_t)b * P + i] = v;
    }
}

// Fh(b) = sum of the b's interaction-list slots, each slot's canonical result
// taken back to the pair's frame: row i of slot j is the canonical row
// red[sym_j][i], signed.  One block per target box: the symmetry table and
// the slots' symmetries are staged in LDS, wave w sums the slots j = w mod 4
// (in order) with the loads of RU slots in flight together, and the four
// partial sums are added in wave order (the result does not depend on
// scheduling).  The box's locals have no other contribution yet: they are
// written, not accumulated.
constexpr int RED_CH = 512;  // slots staged per pass
constexpr int RED_RU = 6;    // slots per wave in flight

template <class V>
__global__ void __launch_bounds__(256) k_m2l_reduce(const int32_t *boxes, const int64_t *iptr, const int32_t *slot_sym,
                                                    const int16_t *sym_red, int P, const int32_t *level, LevelP lp,
                                                    int64_t slot0, const V *out, V *loc) {
    far_field_priority();
    __shared__ __align__(16) int16_t tab[NSYM * OUT_LD];
    __shared__ int32_t ssym[RED_CH];
    __shared__ V part[4][3 * 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int b = boxes[blockIdx.x];
    const int Pt = lp.P[level[b]];  // the box's own order: rows past it are not formed
    const int64_t j0 = iptr[b], j1 = iptr[b + 1];
    for (int x = tid; x < NSYM * OUT_LD / 8; x += 256) ((int4 *)tab)[x] = ((const int4 *)sym_red)[x];
    V acc[3] = {V(0.0), V(0.0), V(0.0)};
    for (int64_t cb = j0; cb < j1; cb += RED_CH) {
        const int ns = (int)min<int64_t>(RED_CH, j1 - cb);
        __syncthreads();
        for (int x = tid; x < ns; x += 256) ssym[x] = slot_sym[cb + x];
        __syncthreads();
        for (int jb = w; jb < ns; jb += 4 * RED_RU) {
            V v[RED_RU][3];
            int sg[RED_RU][3];
#pragma unroll
            for (int k = 0; k < RED_RU; k++) {
                const int j = jb + 4 * k;
                const int g = j < ns ? ssym[j] : 0;
#pragma unroll
                for (int r = 0; r < 3; r++) {
                    const int i = lane + 64 * r;
                    const int e = (j < ns && i < Pt) ? tab[g * OUT_LD + i] : 0;
                    sg[k][r] = (j < ns && i < Pt) ? ((e & 0x100) ? -1 : 1) : 0;
                    v[k][r] = out[(cb + min(j, ns - 1) - slot0) * OUT_LD + (e & 0xff)];
                }
            }
#pragma unroll
            for (int k = 0; k < RED_RU; k++)
#pragma unroll
                for (int r = 0; r < 3; r++) {
                    if (sg[k][r] > 0) acc[r] += v[k][r];
                    else if (sg[k][r] < 0) acc[r] -= v[k][r];
                }
        }
    }
#pragma unroll
    for (int r = 0; r < 3; r++) part[w][lane + 64 * r] = acc[r];
    __syncthreads();
    for (int i = tid; i < P; i += 256)
        loc[(int64_t)b * P + i] = i < Pt ? ((part[0][i] + part[1][i]) + part[2][i]) + part[3][i] : V(0.0);
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

// Class ids by key in order of first appearance (open addressing, linear
// probing; the table is kept at most half full).
struct ClassIds {
    std::vector<ClassKey> keys;
    std::vector<int32_t> tab = std::vector<int32_t>(1024, -1);
    int32_t get(const ClassKey &k, bool &added) {
        size_t m = tab.size() - 1, h = ClassKeyHash()(k) & m;
        for (; tab[h] >= 0; h = (h + 1) & m)
            if (keys[tab[h]] == k) return tab[h];
        added = true;
        const int32_t id = (int32_t)keys.size();
        keys.push_back(k);
        tab[h] = id;
        if (2 * keys.size() > tab.size()) {
            tab.assign(2 * tab.size(), -1);
            m = tab.size() - 1;
            for (int32_t i = 0; i < (int32_t)keys.size(); i++) {
                size_t x = ClassKeyHash()(keys[i]) & m;
                while (tab[x] >= 0) x = (x + 1) & m;
                tab[x] = i;
            }
        }
        return id;
    }
};

uint64_t compact3h(uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < 21; b++) r |= ((v >> (3 * b)) & 1u) << b;
    return r;
}

// the six orderings of the axes; symmetry g = 8 * ordering + sign flips
constexpr int PERMS[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Symmetry tables.  For symmetry g (canonical component i = actual axis
// sigma(i), flipped axes f), canonical multi-index a' stands for the actual
// multi-index a with a_{sigma(i)} = a'_i, with sign prod over flipped axes of
// (-1)^(a_e).  in[g][a'] = index of a | SYM_NEG if negative (moments into the
// canonical frame); red[g][index of a] = a' | 0x100 if negative (results
// back to the pair's frame).
void symmetry_tables(const std::vector<int8_t> &ex, int P, std::vector<int32_t> &in, std::vector<int16_t> &red) {
    std::map<int, int> index;
    for (int i = 0; i < P; i++) index[ex[3 * i] | (ex[3 * i + 1] << 5) | (ex[3 * i + 2] << 10)] = i;
    in.assign((size_t)NSYM * KIN, 0);
    red.assign((size_t)NSYM * OUT_LD, 0);
    for (int g = 0; g < NSYM; g++) {
        const int *sg = PERMS[g / 8], flips = g % 8;
        for (int i = 0; i < P; i++) {
            int act[3];
            for (int k = 0; k < 3; k++) act[sg[k]] = ex[3 * i + k];
            int par = 0;
            for (int e = 0; e < 3; e++)
                if (flips & (1 << e)) par += act[e];
            const int ai = index.at(act[0] | (act[1] << 5) | (act[2] << 10));
            in[(size_t)g * KIN + i] = ai | ((par & 1) ? SYM_NEG : 0);
            red[(size_t)g * OUT_LD + ai] = (int16_t)(i | ((par & 1) ? 0x100 : 0));
        }
    }
}

}  // namespace

M2lPlan &get_m2l_plan(bem_tree &t, int green, double k) {
    if (green == BEM_LAPLACE) k = 0.0;
    for (auto &p : t.m2l)
        if (p->green == green && p->k == k) {
            p->last_use = ++t.k_uses;
            return *p;
        }
    Ctx &c = *t.ctx;
    if (green == BEM_HELMHOLTZ) evict_wavenumbers(t.m2l);
    fmm_tables(t);
    plan_fmm(t);
    SetupTimer st_(c, "M2L plan (classes, pairs, slabs, derivative tables)");
    FmmTables &T = *t.tables;
    const int p = t.order, P = T.P, P2 = T.P2, H = 2 * p;
    BEM_REQUIRE(P <= MT * 16 && P <= KIN && P <= 3 * 64, BEM_EUNSUPPORTED, "expansion order too high for the M2L tiles");
    const bool helm = green == BEM_HELMHOLTZ;
    auto pl = std::make_unique<M2lPlan>();
    pl->green = green;
    pl->k = k;
    pl->last_use = ++t.k_uses;
    if (t.h_prefix.empty()) t.h_prefix = t.prefix.download(t.n_box);
    // integer centre coordinates of every box, in half-widths of its own level
    std::vector<int64_t> bxyz((size_t)3 * t.n_box);
    for (int64_t b = 0; b < t.n_box; b++)
        for (int e = 0; e < 3; e++) bxyz[3 * b + e] = (int64_t)compact3h(t.h_prefix[b] >> (2 - e));
    // canonical classes of the interaction pairs of boxes with targets, ids in
    // order of first appearance; class and symmetry of every slot
    ClassIds id;
    std::vector<int32_t> cdelta, csize;
    std::vector<double> rbar, kbar;
    std::vector<int32_t> pcls(std::max<int64_t>(1, t.n_inter), -1), psym(std::max<int64_t>(1, t.n_inter), 0);
    for (int64_t b = 0; b < t.n_box; b++) {
        if (t.h_te[b] == t.h_tb[b]) continue;
        const int64_t *ib = &bxyz[3 * b];
        for (int64_t j = t.h_inter_ptr[b]; j < t.h_inter_ptr[b + 1]; j++) {
            const int32_t s = t.h_inter_idx[j];
            const int d = t.h_level[b] - t.h_level[s];
            const int64_t *is = &bxyz[3 * (int64_t)s];
            int64_t q[3], u[3];
            int flips = 0;
            for (int e = 0; e < 3; e++) {
                q[e] = (2 * ib[e] + 1) - ((2 * is[e] + 1) << d);
                u[e] = q[e] < 0 ? -q[e] : q[e];
                if (q[e] < 0) flips |= 1 << e;
            }
            // canonical order: |q| ascending (ties by axis)
            int perm = 0;
            for (; perm < 6; perm++) {
                const int *sg = PERMS[perm];
                if (u[sg[0]] <= u[sg[1]] && u[sg[1]] <= u[sg[2]]) break;
            }
            const int *sg = PERMS[perm];
            const ClassKey key{d, (int32_t)u[sg[0]], (int32_t)u[sg[1]], (int32_t)u[sg[2]], helm ? t.h_level[s] : -1};
            bool added = false;
            const int32_t cid = id.get(key, added);
            if (added) {
                cdelta.push_back(d);
                csize.push_back(0);
                for (int e = 0; e < 3; e++) rbar.push_back(std::ldexp((double)u[sg[e]], -(d + 1)));
                kbar.push_back(k * std::ldexp(t.side, -t.h_level[s]));
            }
            csize[cid]++;
            pcls[j] = cid;
            psym[j] = 8 * perm + flips;
        }
    }
    pl->n_class = (int64_t)csize.size();
    st_.lap("classes");
    if (st_.on) std::fprintf(stderr, "bem setup:   %lld classes, %lld interaction pairs\n", (long long)pl->n_class, (long long)t.n_inter);
    const LevelP lp = level_p(t);
    pl->var = t.order_min > 0 && t.order_min < t.order;
    // slabs: runs of consecutive target boxes (the reduction's boxes) whose
    // interaction slots fit t.m2l_slab (a box with more forms a slab alone)
    std::vector<int32_t> box_slab(t.n_box, -1);
    {
        int64_t s0 = -1, nb = 0;
        for (int64_t b = 0; b < t.n_box; b++) {
            if (t.h_te[b] == t.h_tb[b] || t.h_inter_ptr[b + 1] == t.h_inter_ptr[b]) continue;
            if (s0 < 0 || t.h_inter_ptr[b + 1] - s0 > t.m2l_slab) {
                s0 = t.h_inter_ptr[b];
                pl->slab_slot0.push_back(s0);
                pl->slab_box0.push_back(nb);
            }
            box_slab[b] = (int32_t)pl->slab_slot0.size() - 1;
            nb++;
        }
        pl->slab_slot0.push_back(t.n_inter);
        pl->slab_box0.push_back(nb);
        if (pl->slab_slot0.size() == 1) pl->slab_slot0.insert(pl->slab_slot0.begin(), 0);  // no pairs: one empty slab
        if (pl->slab_box0.size() == 1) pl->slab_box0.insert(pl->slab_box0.begin(), 0);
        for (size_t sl = 0; sl + 1 < pl->slab_slot0.size(); sl++) {
            // the slab's slots end where its last box's list ends
            int64_t end = pl->slab_slot0[sl];
            for (int64_t b = 0; b < t.n_box; b++)
                if (box_slab[b] == (int32_t)sl) end = t.h_inter_ptr[b + 1];
            pl->slab_max_slots = std::max(pl->slab_max_slots, end - pl->slab_slot0[sl]);
        }
    }
    const int n_slab = (int)pl->slab_slot0.size() - 1;
    st_.lap("slabs");
    // slot -> target box (for the slab of each pair)
    std::vector<int32_t> slot_box(std::max<int64_t>(1, t.n_inter), -1);
    for (int64_t b = 0; b < t.n_box; b++)
        for (int64_t j = t.h_inter_ptr[b]; j < t.h_inter_ptr[b + 1]; j++) slot_box[j] = (int32_t)b;
    // pairs grouped by slab, then by class, largest class first; within a
    // class in target-level order when the order depends on the level (so that
    // the pairs of a task mostly share their orders), else in slot order.
    // Two stable counting sorts: by target level, then by (slab, class rank).
    const int32_t ncl = (int32_t)pl->n_class;
    std::vector<int32_t> order(ncl), rank(ncl);
    for (int32_t i = 0; i < ncl; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return csize[x] > csize[y]; });
    for (int32_t i = 0; i < ncl; i++) rank[order[i]] = i;
    std::vector<int32_t> seq;
    seq.reserve(t.n_inter);
    if (pl->var) {
        std::vector<int64_t> lc(66, 0);
        for (int64_t j = 0; j < t.n_inter; j++)
            if (pcls[j] >= 0) lc[t.h_level[slot_box[j]] + 1]++;
        for (size_t l = 1; l < lc.size(); l++) lc[l] += lc[l - 1];
        seq.resize(lc.back());
        for (int64_t j = 0; j < t.n_inter; j++)
            if (pcls[j] >= 0) seq[lc[t.h_level[slot_box[j]]]++] = (int32_t)j;
    } else {
        for (int64_t j = 0; j < t.n_inter; j++)
            if (pcls[j] >= 0) seq.push_back((int32_t)j);
    }
    auto bucket = [&](int32_t j) { return (int64_t)box_slab[slot_box[j]] * ncl + rank[pcls[j]]; };
    std::vector<int64_t> bp((size_t)n_slab * ncl + 1, 0);
    for (int32_t j : seq) bp[bucket(j) + 1]++;
    for (size_t i = 1; i < bp.size(); i++) bp[i] += bp[i - 1];
    std::vector<int32_t> slot(seq.size()), src(seq.size()), sym(seq.size());
    {
        std::vector<int64_t> at(bp.begin(), bp.end() - 1);
        for (int32_t j : seq) slot[at[bucket(j)]++] = j;
    }
    for (size_t i = 0; i < slot.size(); i++) {
        src[i] = t.h_inter_idx[slot[i]];
        sym[i] = psym[slot[i]];
    }
    if (pl->var) {
        pl->h_pair_kt.resize(slot.size());
        pl->h_pair_mt.resize(slot.size());
        for (size_t i = 0; i < slot.size(); i++) {
            pl->h_pair_kt[i] = (lp.P[t.h_level[src[i]]] + 3) / 4;
            pl->h_pair_mt[i] = (lp.P[t.h_level[slot_box[slot[i]]]] + 15) / 16;
        }
    }
    for (size_t g = 0; g + 1 < bp.size(); g++) {
        if (bp[g + 1] == bp[g]) continue;
        pl->h_class_order.push_back(order[g % ncl]);
        pl->h_class_first.push_back((int32_t)bp[g]);
        pl->h_class_count.push_back((int32_t)(bp[g + 1] - bp[g]));
        pl->h_group_slab.push_back((int32_t)(g / ncl));
    }
    pl->n_pairs = (int64_t)slot.size();
    st_.lap("pairs by slab and class");
    pl->h_pair_slot = slot;
    pl->h_pair_sym = sym;
    auto up = [&](DBuf<int32_t> &d, const std::vector<int32_t> &v) {
        d.alloc(&c, std::max<size_t>(1, v.size()));
        if (!v.empty()) d.upload(v.data(), v.size());
    };
    up(pl->pair_slot, slot);
    up(pl->pair_src, src);
    // used (source box, symmetry) combinations: one canonical moment vector each
    {
        std::vector<int32_t> uid((size_t)t.n_box * NSYM, -1);
        std::vector<int32_t> pmom(slot.size()), usrc, usym;
        for (size_t i = 0; i < slot.size(); i++) {
            int32_t &u = uid[(size_t)src[i] * NSYM + sym[i]];
            if (u < 0) {
                u = (int32_t)usrc.size();
                usrc.push_back(src[i]);
                usym.push_back(sym[i]);
            }
            pmom[i] = u;
        }
        pl->n_u = (int64_t)usrc.size();
        up(pl->pair_mom, pmom);
        up(pl->u_src, usrc);
        up(pl->u_sym, usym);
    }
    st_.lap("moment vectors");
    up(pl->cls_delta, cdelta);
    // packed multi-indices of the rows and contraction indices
    std::vector<int32_t> pk(KIN, 0);
    for (int i = 0; i < P; i++) pk[i] = T.h_exps[3 * i] | (T.h_exps[3 * i + 1] << 5) | (T.h_exps[3 * i + 2] << 10);
    up(pl->pk, pk);
    std::vector<int32_t> sin;
    std::vector<int16_t> sred;
    symmetry_tables(T.h_exps, P, sin, sred);
    up(pl->sym_in, sin);
    pl->sym_red.alloc(&c, sred.size());
    pl->sym_red.upload(sred.data(), sred.size());
    {  // the compact form of sym_red that the split kernel reads
        std::vector<uint8_t> po((size_t)7 * OUT_LD, 0);
        for (int i = 0; i < P; i++) {
            for (int o = 0; o < 6; o++) po[(size_t)o * OUT_LD + i] = (uint8_t)(sred[(size_t)8 * o * OUT_LD + i] & 0xff);
            po[(size_t)6 * OUT_LD + i] =
                (uint8_t)((T.h_exps[3 * i] & 1) | (T.h_exps[3 * i + 1] & 1) << 1 | (T.h_exps[3 * i + 2] & 1) << 2);
        }
        for (int g = 0; g < NSYM; g++)
            for (int i = 0; i < P; i++) {
                const int neg = __builtin_popcount((g & 7) & po[(size_t)6 * OUT_LD + i]) & 1;
                BEM_REQUIRE(sred[(size_t)g * OUT_LD + i] == (po[(size_t)(g / 8) * OUT_LD + i] | (neg ? 0x100 : 0)),
                            BEM_EUNSUPPORTED, "compact symmetry table disagrees with the full one");
            }
        pl->sym_perm.alloc(&c, po.size());
        pl->sym_perm.upload(po.data(), po.size());
    }
    // symmetry of every interaction-list slot (slots outside the plan stay 0)
    std::vector<int32_t> ssym(std::max<int64_t>(1, t.n_inter), 0);
    for (size_t i = 0; i < slot.size(); i++) ssym[slot[i]] = sym[i];
    up(pl->slot_sym, ssym);
    st_.lap("tables");
    // class derivative tables at the canonical separations
    const int cw = helm ? 2 : 1;
    pl->D64.alloc(&c, (size_t)cw * P2 * std::max<int64_t>(1, pl->n_class));
    if (pl->n_class) {
        DBuf<double> drb, dkb;
        drb.alloc(&c, rbar.size());
        drb.upload(rbar.data(), rbar.size());
        dkb.alloc(&c, kbar.size());
        dkb.upload(kbar.data(), kbar.size());
        size_t sh = (size_t)cw * sizeof(double) * (2 * P2 + H + 2);
        if (helm)
            k_class_derivs<true><<<(unsigned)pl->n_class, 256, sh, c.stream>>>(drb.p, dkb.p, H, T.exps.p, pl->D64.p);
        else
            k_class_derivs<false><<<(unsigned)pl->n_class, 256, sh, c.stream>>>(drb.p, dkb.p, H, T.exps.p, pl->D64.p);
        BEM_LAUNCH_CHECK();
        c.sync();
    }
    t.m2l.push_back(std::move(pl));
    return *t.m2l.back();
}

namespace {

// Tasks of `cols` pairs, slab by slab: within a slab each class, largest
// first, goes to the least-loaded of the 8 XCD queues, and the queues are
// interleaved so that block i of the slab's launch runs on XCD i mod 8.
// Padding tasks have no pairs.
M2lTasks &get_tasks(Ctx &c, M2lPlan &pl, int cols) {
    for (auto &tk : pl.tasks)
        if (tk->cols == cols) return *tk;
    constexpr int NXCD = 8;
    std::vector<int32_t> tc, tf, tn, tkt, tmt;
    auto tk = std::make_unique<M2lTasks>();
    tk->cols = cols;
    // the tasks of groups [g0, g1) (one slab), appended in XCD-interleaved order
    auto slab_tasks = [&](size_t g0, size_t g1) {
        std::vector<std::vector<int32_t>> qc(NXCD), qf(NXCD), qn(NXCD), qk(NXCD), qm(NXCD);
        std::vector<int64_t> load(NXCD, 0);
        for (size_t i = g0; i < g1; i++) {
            const int32_t cl = pl.h_class_order[i], f0 = pl.h_class_first[i], n = pl.h_class_count[i];
            const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            for (int32_t o = 0; o < n; o += cols) {
                qc[x].push_back(cl);
                qf[x].push_back(f0 + o);
                qn[x].push_back(std::min(cols, n - o));
                if (pl.var) {
                    int32_t kt = 0, mt = 0;
                    for (int32_t j = f0 + o; j < f0 + o + qn[x].back(); j++) {
                        kt = std::max(kt, pl.h_pair_kt[j]);
                        mt = std::max(mt, pl.h_pair_mt[j]);
                    }
                    qk[x].push_back(kt);
                    qm[x].push_back(mt);
                }
                load[x]++;
            }
        }
        size_t qmax = 0;
        for (int x = 0; x < NXCD; x++) qmax = std::max(qmax, qc[x].size());
        const size_t base = tc.size();
        tc.resize(base + qmax * NXCD, 0);
        tf.resize(base + qmax * NXCD, 0);
        tn.resize(base + qmax * NXCD, 0);
        if (pl.var) {
            tkt.resize(base + qmax * NXCD, 0);
            tmt.resize(base + qmax * NXCD, 0);
        }
        for (int x = 0; x < NXCD; x++)
            for (size_t i = 0; i < qc[x].size(); i++) {
                tc[base + i * NXCD + x] = qc[x][i];
                tf[base + i * NXCD + x] = qf[x][i];
                tn[base + i * NXCD + x] = qn[x][i];
                if (pl.var) {
                    tkt[base + i * NXCD + x] = qk[x][i];
                    tmt[base + i * NXCD + x] = qm[x][i];
                }
            }
    };
    const int n_slab = (int)pl.slab_slot0.size() - 1;
    size_t g = 0;  // groups are in slab order
    for (int sl = 0; sl < n_slab; sl++) {
        tk->slab_task0.push_back((int64_t)tc.size());
        const size_t g0 = g;
        while (g < pl.h_class_order.size() && pl.h_group_slab[g] == sl) g++;
        slab_tasks(g0, g);
    }
    tk->slab_task0.push_back((int64_t)tc.size());
    tk->n_task = (int64_t)tc.size();
    auto up = [&](DBuf<int32_t> &d, const std::vector<int32_t> &v) {
        d.alloc(&c, std::max<size_t>(1, v.size()));
        if (!v.empty()) d.upload(v.data(), v.size());
    };
    up(tk->task_class, tc);
    up(tk->task_first, tf);
    up(tk->task_count, tn);
    if (pl.var) {
        up(tk->task_kt, tkt);
        up(tk->task_mt, tmt);
    }
    pl.tasks.push_back(std::move(tk));
    return *pl.tasks.back();
}

// expanded operators of the plan in precision R (built on first use)
template <class R>
const R *expanded(bem_tree &t, M2lPlan &pl) {
    Ctx &c = *t.ctx;
    FmmTables &T = *t.tables;
    DBuf<R> &buf = pl.expanded_buf<R>();
    if (!buf.p && pl.n_class) {
        const bool helm = pl.green == BEM_HELMHOLTZ;
        buf.alloc(&c, (size_t)(helm ? 2 : 1) * TSZ * pl.n_class);
        dim3 g((unsigned)pl.n_class, MT * KT);
        if (helm)
            k_expand_T<R, true><<<g, 64, 0, c.stream>>>(pl.D64.p, pl.pk.p, pl.cls_delta.p, T.inv_fact64.p, T.P, T.P2,
                                                        buf.p);
        else
            k_expand_T<R, false><<<g, 64, 0, c.stream>>>(pl.D64.p, pl.pk.p, pl.cls_delta.p, T.inv_fact64.p, T.P,
                                                         T.P2, buf.p);
        BEM_LAUNCH_CHECK();
        c.sync();
    }
    return buf.p;
}

// split operators of the plan and their scales (built on first use)
const uint16_t *expanded2(bem_tree &t, M2lPlan &pl) {
    Ctx &c = *t.ctx;
    FmmTables &T = *t.tables;
    if (!pl.T2.p && pl.n_class) {
        SetupTimer st_(c, "M2L split operators");
        const bool helm = pl.green == BEM_HELMHOLTZ;
        pl.cls_scale.alloc(&c, (size_t)pl.n_class);
        pl.T2.alloc(&c, (size_t)(helm ? 2 : 1) * KB * CH2 * pl.n_class);
        static_assert(OUT_LD <= 256, "one thread per operator row");
        dim3 g((unsigned)pl.n_class, KB * MT);
        if (helm) {
            k_cls_scale<true><<<(unsigned)pl.n_class, 256, 0, c.stream>>>(pl.D64.p, pl.pk.p, pl.cls_delta.p,
                                                                          T.inv_fact64.p, T.P, T.P2, pl.cls_scale.p);
            BEM_LAUNCH_CHECK();
            k_expand_T2<true><<<g, 64, 0, c.stream>>>(pl.D64.p, pl.pk.p, pl.cls_delta.p, T.inv_fact64.p, T.P, T.P2,
                                                      pl.cls_scale.p, pl.T2.p);
        } else {
            k_cls_scale<false><<<(unsigned)pl.n_class, 256, 0, c.stream>>>(pl.D64.p, pl.pk.p, pl.cls_delta.p,
                                                                           T.inv_fact64.p, T.P, T.P2, pl.cls_scale.p);
            BEM_LAUNCH_CHECK();
            k_expand_T2<false><<<g, 64, 0, c.stream>>>(pl.D64.p, pl.pk.p, pl.cls_delta.p, T.inv_fact64.p, T.P, T.P2,
                                                       pl.cls_scale.p, pl.T2.p);
        }
        BEM_LAUNCH_CHECK();
        c.sync();
    }
    return pl.T2.p;
}

// Partial slots of the split path's per-target sums: within each (slab,
// class) group of pairs, passes of G = 8 pairs from its first pair (the
// product kernel's waves take 16 real or 8 complex pairs from there); a run of consecutive pairs of one pass with the same target box
// shares a slot.  Slots are numbered box by box in m2l_boxes order (a slab's
// slots are then contiguous), within a box in pair order, so that a box's sum
// runs over one contiguous range in a fixed order.
void build_parts(bem_tree &t, M2lPlan &pl) {
    constexpr int G = 8;  // as the product kernel
    if (pl.parts_g == G) return;
    Ctx &c = *t.ctx;
    SetupTimer st_(c, "M2L partial slots");
    std::vector<int32_t> slot_box(std::max<int64_t>(1, t.n_inter), -1), box_x(t.n_box, -1);
    int32_t nx = 0;
    for (int64_t b = 0; b < t.n_box; b++) {
        for (int64_t j = t.h_inter_ptr[b]; j < t.h_inter_ptr[b + 1]; j++) slot_box[j] = (int32_t)b;
        if (t.h_te[b] > t.h_tb[b] && t.h_inter_ptr[b + 1] > t.h_inter_ptr[b]) box_x[b] = nx++;  // as plan_fmm
    }
    const size_t np = pl.h_pair_slot.size();
    std::vector<int32_t> run(np, 0), run_x;  // run of each pair; m2l-box index of each run
    for (size_t g = 0; g < pl.h_class_first.size(); g++) {
        const int64_t f0 = pl.h_class_first[g], f1 = f0 + pl.h_class_count[g];
        for (int64_t i = f0; i < f1; i++) {
            const int32_t x = box_x[slot_box[pl.h_pair_slot[i]]];
            const bool fresh = i == f0 || (i - f0) % G == 0 || run_x.back() != x;
            if (fresh) run_x.push_back(x);
            run[i] = (int32_t)run_x.size() - 1;
        }
    }
    // number the runs box by box (stable: pair order within a box)
    std::vector<int64_t> ptr((size_t)nx + 1, 0);
    for (int32_t x : run_x) ptr[(size_t)x + 1]++;
    for (int32_t x = 0; x < nx; x++) ptr[(size_t)x + 1] += ptr[(size_t)x];
    std::vector<int64_t> next(ptr.begin(), ptr.end() - 1);
    std::vector<int32_t> slot_of(run_x.size());
    for (size_t r = 0; r < run_x.size(); r++) slot_of[r] = (int32_t)next[(size_t)run_x[r]]++;
    std::vector<int32_t> part(np);
    for (size_t i = 0; i < np; i++) part[i] = slot_of[(size_t)run[i]];
    pl.pair_part.alloc(&c, std::max<size_t>(1, np));
    if (np) pl.pair_part.upload(part.data(), np);
    pl.pair_sym.alloc(&c, std::max<size_t>(1, np));
    if (np) pl.pair_sym.upload(pl.h_pair_sym.data(), np);
    pl.part_ptr.alloc(&c, ptr.size());
    pl.part_ptr.upload(ptr.data(), ptr.size());
    pl.h_part_ptr = ptr;
    pl.parts_max = 0;
    for (size_t sl = 0; sl + 1 < pl.slab_box0.size(); sl++)
        pl.parts_max = std::max(pl.parts_max, ptr[(size_t)pl.slab_box0[sl + 1]] - ptr[(size_t)pl.slab_box0[sl]]);
    pl.parts_g = G;
}

// waves per block of the split kernel: the complex one stages 11 KB per wave
// in its 44 KB LDS ring, which holds four
int split_waves(int na, int w) { return na == 2 && w > 4 ? 4 : w; }

// whether a product of precision R on this plan runs on the split operands
// (mixed precision with one order for all levels)
template <class R>
bool split_path(const M2lPlan &pl) {
    return std::is_same<R, float>::value && !pl.var;
}

// pairs per block of w waves: 16 real or 8 complex per column group (the
// FP32 and FP64 kernels with rows split over two waves have w / 2 groups)
template <class V, class R>
int m2l_cols(const M2lPlan &pl, int w) {
    constexpr int NA = std::is_same<V, R>::value ? 1 : 2;
    return (NA == 1 ? 16 : 8) * (split_path<R>(pl) ? split_waves(NA, w) : w / m2l_ms<R, NA>());
}

}  // namespace

bool m2l_ready(const M2lPlan &pl, int prec, int waves) {
    const bool helm = pl.green == BEM_HELMHOLTZ, f32 = prec == BEM_PREC_MIXED;
    const void *ops = f32 ? (split_path<float>(pl) ? (const void *)pl.T2.p : (const void *)pl.T32.p)
                          : (const void *)pl.T64.p;
    if (pl.n_class && !ops) return false;
    if (f32 && split_path<float>(pl) && pl.parts_g != 8) return false;
    const int cols = helm ? (f32 ? m2l_cols<cx<float>, float>(pl, waves) : m2l_cols<cx<double>, double>(pl, waves))
                          : (f32 ? m2l_cols<float, float>(pl, waves) : m2l_cols<double, double>(pl, waves));
    for (auto &tk : pl.tasks)
        if (tk->cols == cols) return true;
    return false;
}

namespace {

template <int W>
const void *m2l_kernel(const M2lPlan &pl, bool f32, bool helm) {
    if (f32 && !pl.var) return helm ? (const void *)k_m2l_x2<2, (W > 4 ? 4 : W)> : (const void *)k_m2l_x2<1, W>;
    if (f32) return helm ? (const void *)k_m2l<float, 2, true, W> : (const void *)k_m2l<float, 1, true, W>;
    if (pl.var) return helm ? (const void *)k_m2l<double, 2, true, W> : (const void *)k_m2l<double, 1, true, W>;
    return helm ? (const void *)k_m2l<double, 2, false, W> : (const void *)k_m2l<double, 1, false, W>;
}

}  // namespace

size_t m2l_block_lds(const M2lPlan &pl, int prec, int waves) {
    const bool f32 = prec == BEM_PREC_MIXED, helm = pl.green == BEM_HELMHOLTZ;
    const void *fn = waves == 2   ? m2l_kernel<2>(pl, f32, helm)
                     : waves == 8 ? m2l_kernel<8>(pl, f32, helm)
                                  : m2l_kernel<4>(pl, f32, helm);
    static std::mutex mu;
    static std::map<const void *, size_t> memo;  // one device model
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(fn);
    if (it != memo.end()) return it->second;
    hipFuncAttributes fa;
    BEM_HIP(hipFuncGetAttributes(&fa, fn));
    return memo[fn] = fa.sharedSizeBytes;
}

template <class V, class R>
void m2l_prepare(bem_tree &t, M2lPlan &pl, int waves) {
    if (split_path<R>(pl)) {
        expanded2(t, pl);
        build_parts(t, pl);
    } else
        expanded<R>(t, pl);
    get_tasks(*t.ctx, pl, m2l_cols<V, R>(pl, waves));
}

template <class V, class R>
void m2l_apply(bem_tree &t, M2lPlan &pl, int nrhs, const V *mom, V *loc, int waves) {
    Ctx &c = *t.ctx;
    FmmTables &T = *t.tables;
    const int P = T.P;
    M2lTasks &tk = get_tasks(c, pl, m2l_cols<V, R>(pl, waves));
    if (!tk.n_task || !pl.n_pairs) {
        c.mark(3);
        return;
    }
    constexpr int NA = std::is_same<V, R>::value ? 1 : 2;
    const bool split = split_path<R>(pl);
    if (split) build_parts(t, pl);
    // per-pair results of a slab, or its partial slots on the split path
    const int64_t out_rows = split ? pl.parts_max : pl.slab_max_slots;
    V *out = (V *)work_buf(c, t.work.m2l_out, sizeof(V) * (size_t)std::max<int64_t>(1, out_rows) * OUT_LD);
    const LevelP lp = level_p(t);
    // canonical moments, then (split path) their exponents
    const size_t mc_bytes = sizeof(V) * KIN * (size_t)std::max<int64_t>(1, pl.n_u);
    void *Mc = work_buf(c, t.work.m2l_mom, mc_bytes + (split ? sizeof(int32_t) * (size_t)std::max<int64_t>(1, pl.n_u) : 0));
    int32_t *u_exp = split ? (int32_t *)((char *)Mc + mc_bytes) : nullptr;
    const R *Tx = split ? nullptr : expanded<R>(t, pl);
    const uint4 *T2 = split ? (const uint4 *)expanded2(t, pl) : nullptr;
    for (int rhs = 0; rhs < nrhs; rhs++) {
        const V *m = mom + (int64_t)rhs * t.n_box * P;
        V *l = loc + (int64_t)rhs * t.n_box * P;
        k_m2l_canonical_moments<V><<<(unsigned)((pl.n_u + 3) / 4), 256, 0, c.stream>>>(
            pl.n_u, pl.u_src.p, pl.u_sym.p, pl.sym_in.p, P, m, (V *)Mc, u_exp);
        BEM_LAUNCH_CHECK();
        c.mark(10);
        // one slab of target boxes at a time: its pairs' results, then their sums
        for (size_t sl = 0; sl + 1 < pl.slab_slot0.size(); sl++) {
            const int64_t t0 = tk.slab_task0[sl], nt = tk.slab_task0[sl + 1] - t0;
            const int64_t b0 = pl.slab_box0[sl], nb = pl.slab_box0[sl + 1] - b0;
            // split path: results go to the slab's partial slots, from its first box's
            const int64_t part0 = split ? pl.h_part_ptr[(size_t)b0] : 0;
            M2lArgs a{tk.task_class.p + t0, tk.task_first.p + t0, tk.task_count.p + t0, pl.pair_slot.p,
                      pl.pair_src.p, pl.pair_mom.p, t.level.p, pl.var ? tk.task_kt.p + t0 : nullptr,
                      pl.var ? tk.task_mt.p + t0 : nullptr, t.side, P, split ? part0 : pl.slab_slot0[sl],
                      split ? pl.pair_part.p : nullptr, split ? pl.pair_sym.p : nullptr, pl.sym_red.p,
                      u_exp, split ? pl.cls_scale.p : nullptr, pl.sym_perm.p};
            c.kbegin(c.stream, 3);
            auto launch = [&](auto wv) {
                constexpr int W = decltype(wv)::value;
                if constexpr (std::is_same<R, float>::value) {
                    if (split) {
                        constexpr int WS = NA == 2 && W > 4 ? 4 : W;  // as split_waves
                        k_m2l_x2<NA, WS><<<(unsigned)nt, 64 * WS, 0, c.stream>>>(a, T2, (const float *)Mc, (float *)out);
                        return;
                    }
                }
                if (pl.var)
                    k_m2l<R, NA, true, W><<<(unsigned)nt, 64 * W, 0, c.stream>>>(a, Tx, (const R *)Mc, (R *)out);
                else
                    k_m2l<R, NA, false, W><<<(unsigned)nt, 64 * W, 0, c.stream>>>(a, Tx, (const R *)Mc, (R *)out);
            };
            if (nt > 0) {
                if (waves == 2) launch(std::integral_constant<int, 2>());
                else if (waves == 8) launch(std::integral_constant<int, 8>());
                else launch(std::integral_constant<int, 4>());
                BEM_LAUNCH_CHECK();
            }
            c.kend(c.stream);
            c.mark(3);
            if (nb > 0 && split) {
                k_m2l_sum_parts<V><<<(unsigned)nb, 256, 0, c.stream>>>(t.m2l_boxes.p + b0, pl.part_ptr.p + b0, part0,
                                                                       P, out, l);
                BEM_LAUNCH_CHECK();
            } else if (nb > 0) {
                k_m2l_reduce<V><<<(unsigned)nb, 256, 0, c.stream>>>(t.m2l_boxes.p + b0, t.inter_ptr.p, pl.slot_sym.p,
                                                                    pl.sym_red.p, P, t.level.p, lp, pl.slab_slot0[sl],
                                                                    out, l);
                BEM_LAUNCH_CHECK();
            }
            c.mark(10);
        }
    }
}

template void m2l_prepare<double, double>(bem_tree &, M2lPlan &, int);
template void m2l_prepare<float, float>(bem_tree &, M2lPlan &, int);
template void m2l_prepare<cx<double>, double>(bem_tree &, M2lPlan &, int);
template void m2l_prepare<cx<float>, float>(bem_tree &, M2lPlan &, int);
template void m2l_apply<double, double>(bem_tree &, M2lPlan &, int, const double *, double *, int);
template void m2l_apply<float, float>(bem_tree &, M2lPlan &, int, const float *, float *, int);
template void m2l_apply<cx<double>, double>(bem_tree &, M2lPlan &, int, const cx<double> *, cx<double> *, int);
template void m2l_apply<cx<float>, float>(bem_tree &, M2lPlan &, int, const cx<float> *, cx<float> *, int);

}  // namespace bem
