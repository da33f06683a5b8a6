// Device-wide exclusive scan and stable LSD radix sort (wave64, gfx950).
//
// The scan runs in three passes (tile sums, scan of the tile sums, tile scans
// with offsets); the radix sort does 8-bit digits per pass: a per-tile digit
// histogram, one exclusive scan of the digit-major histogram table, then a
// stable scatter in which each key's rank inside its tile comes from 64-bit
// ballots matching equal digits across a wave and per-wave digit counts in LDS.
#include "kernels.h"

namespace bem {

namespace {

constexpr int SCAN_BS = 256;
constexpr int SCAN_IPT = 4;
constexpr int SCAN_TILE = SCAN_BS * SCAN_IPT;

template <class T>
__device__ T block_exclusive_scan(T v, T *lds_waves, T *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) lds_waves[wave] = incl;
    __syncthreads();
    T base = 0, tot = 0;
    for (int w = 0; w < nw; w++) {
        T s = lds_waves[w];
        if (w < wave) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

template <class T>
__global__ void k_tile_sums(const T *in, int64_t n, T *sums) {
    __shared__ T lw[SCAN_BS / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_IPT;
    T s = 0;
    for (int i = 0; i < SCAN_IPT; i++)
        if (base + i < n) s += in[base + i];
    T tot;
    block_exclusive_scan(s, lw, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ void k_tile_scan(const T *in, T *out, int64_t n, const T *offsets) {
    __shared__ T lw[SCAN_BS / 64];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_IPT;
    T v[SCAN_IPT];
    T s = 0;
    for (int i = 0; i < SCAN_IPT; i++) {
        v[i] = (base + i < n) ? in[base + i] : T(0);
        s += v[i];
    }
    T tot;
    T ex = block_exclusive_scan(s, lw, &tot) + (offsets ? offsets[blockIdx.x] : T(0));
    for (int i = 0; i < SCAN_IPT; i++) {
        if (base + i < n) out[base + i] = ex;
        ex += v[i];
    }
    // out[n] receives the grand total (callers size `out` as n + 1)
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == SCAN_BS - 1) out[n] = ex;
}

// Zeroes [p, p + bytes): 16-byte stores over the aligned middle, byte stores
// for the unaligned head and tail (taken by the first threads).
__global__ void k_zero(unsigned char *p, size_t head, size_t n16, size_t tail) {
    const size_t i0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
    uint4 *m = (uint4 *)(p + head);
    for (size_t i = i0; i < n16; i += stride) m[i] = make_uint4(0u, 0u, 0u, 0u);
    if (i0 < head) p[i0] = 0;
    if (i0 < tail) p[head + 16 * n16 + i0] = 0;
}

}  // namespace

void zero_fill(Ctx &c, void *p, size_t bytes) {
    if (!bytes) return;
    unsigned char *b = (unsigned char *)p;
    size_t head = (16 - (size_t)((uintptr_t)b % 16)) % 16;
    if (head > bytes) head = bytes;
    const size_t n16 = (bytes - head) / 16, tail = bytes - head - 16 * n16;
    const unsigned nb = (unsigned)std::max<size_t>(1, std::min<size_t>((n16 + 255) / 256, 4096));
    k_zero<<<nb, 256, 0, c.stream>>>(b, head, n16, tail);
    BEM_LAUNCH_CHECK();
}

template <class T>
void scan_exclusive(Ctx &c, const T *in, T *out, int64_t n) {
    if (n == 0) {
        zero_fill(c, out, sizeof(T));
        return;
    }
    unsigned nb = nblocks(n, SCAN_TILE);
    if (nb == 1) {
        k_tile_scan<T><<<1, SCAN_BS, 0, c.stream>>>(in, out, n, nullptr);
        BEM_LAUNCH_CHECK();
        return;
    }
    DBuf<T> sums, offs;
    sums.alloc(&c, nb);
    offs.alloc(&c, nb + 1);
    k_tile_sums<T><<<nb, SCAN_BS, 0, c.stream>>>(in, n, sums.p);
    BEM_LAUNCH_CHECK();
    scan_exclusive<T>(c, sums.p, offs.p, nb);
    k_tile_scan<T><<<nb, SCAN_BS, 0, c.stream>>>(in, out, n, offs.p);
    BEM_LAUNCH_CHECK();
}

template void scan_exclusive<int32_t>(Ctx &, const int32_t *, int32_t *, int64_t);
template void scan_exclusive<int64_t>(Ctx &, const int64_t *, int64_t *, int64_t);

// ---------------------------------------------------------------- radix sort
namespace {

constexpr int RS_BS = 256;  // one key per thread; tile = 256 keys

__global__ void k_digit_hist(const uint64_t *keys, int64_t n, int shift, int32_t *hist /* [256][nb] */) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * RS_BS + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    __syncthreads();
    hist[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_digit_scatter(const uint64_t *keys, const int32_t *vals, int64_t n, int shift,
                                const int32_t *offs /* scanned [256][nb] */, uint64_t *okeys, int32_t *ovals) {
    __shared__ int32_t wc[RS_BS / 64][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = threadIdx.x; j < (RS_BS / 64) * 256; j += RS_BS) (&wc[0][0])[j] = 0;
    __syncthreads();
    int64_t i = (int64_t)blockIdx.x * RS_BS + threadIdx.x;
    bool valid = i < n;
    uint64_t key = valid ? keys[i] : 0;
    uint32_t d = (uint32_t)((key >> shift) & 255u);
    // lanes of this wave holding the same digit
    uint64_t same = __ballot(valid);
    for (int b = 0; b < 8; b++) {
        uint64_t bal = __ballot(valid && ((d >> b) & 1u));
        same &= ((d >> b) & 1u) ? bal : ~bal;
    }
    uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int rank_w = __popcll(same & lt);
    if (valid && rank_w == 0) wc[wave][d] = __popcll(same);
    __syncthreads();
    if (valid) {
        int before = 0;
        for (int w = 0; w < wave; w++) before += wc[w][d];
        int64_t pos = offs[(int64_t)d * gridDim.x + blockIdx.x] + before + rank_w;
        okeys[pos] = key;
        ovals[pos] = vals[i];
    }
}

}  // namespace

void radix_sort_pairs(Ctx &c, uint64_t *keys, int32_t *vals, int64_t n, int key_bits) {
    if (n <= 1) return;
    unsigned nb = nblocks(n, RS_BS);
    DBuf<uint64_t> k2;
    DBuf<int32_t> v2, hist, offs;
    k2.alloc(&c, n);
    v2.alloc(&c, n);
    hist.alloc(&c, (size_t)256 * nb);
    offs.alloc(&c, (size_t)256 * nb + 1);
    uint64_t *ka = keys, *kb = k2.p;
    int32_t *va = vals, *vb = v2.p;
    int passes = (key_bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        k_digit_hist<<<nb, RS_BS, 0, c.stream>>>(ka, n, shift, hist.p);
        BEM_LAUNCH_CHECK();
        scan_exclusive<int32_t>(c, hist.p, offs.p, (int64_t)256 * nb);
        k_digit_scatter<<<nb, RS_BS, 0, c.stream>>>(ka, va, n, shift, offs.p, kb, vb);
        BEM_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        BEM_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, c.stream));
        BEM_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.stream));
    }
    c.sync();  // temporaries are released on return
}

}  // namespace bem
