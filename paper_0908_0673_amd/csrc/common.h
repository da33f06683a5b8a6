// Internal helpers of the HIP library: errors, device buffers, complex values,
// launch checks.  Included by every translation unit of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <map>
#include <unordered_map>
#include <vector>

#include "../../include/bem.h"

namespace bem {

// Errors travel as exceptions inside the library and become status codes at
// the C interface (api.hip); nothing is thrown across it.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw Error(code, msg); }

#define BEM_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            ::bem::fail(BEM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_) + " (" + \
                                         __FILE__ + ":" + std::to_string(__LINE__) + ")");      \
    } while (0)

#define BEM_LAUNCH_CHECK() BEM_HIP(hipGetLastError())

#define BEM_REQUIRE(cond, code, msg)              \
    do {                                          \
        if (!(cond)) ::bem::fail((code), (msg));  \
    } while (0)

// ---------------------------------------------------------------- context
struct Ctx {
    // Timing with HIP events.  Mode 1 (phases): events between the phases on
    // the context's stream, with every phase on that stream.  Modes 2-4
    // (heavy kernels): event pairs around the M2L product and / or
    // near-field kernels only, each on the stream it runs on, with the usual
    // scheduling.  Events pile up without any synchronisation and are read
    // back when the counters are (collect, after a stream sync), so timing
    // does not stall the host between products; each event carries the
    // sequence number of its product.
    int timing = 0;
    int64_t prod_seq = 0;  // products started on this context
    bool autotune = true;  // tune the launch choices of an untuned shape class on its first product
    double phase_ms[BEM_NPHASE] = {0};
    int64_t phase_n[BEM_NPHASE] = {0};
    std::vector<hipEvent_t> events;
    std::vector<int> ev_phase;      // phase closed by each recorded event
    std::vector<int64_t> ev_prod;   // product of each recorded event
    int ev_used = 0;

    void mark(int phase) {
        if (timing != 1) return;
        if (ev_used == (int)events.size()) {
            hipEvent_t e;
            BEM_HIP(hipEventCreate(&e));
            events.push_back(e);
            ev_phase.push_back(-1);
            ev_prod.push_back(-1);
        }
        BEM_HIP(hipEventRecord(events[ev_used], stream));
        ev_phase[ev_used] = phase;
        ev_prod[ev_used] = prod_seq;
        ev_used++;
    }
    // modes 2-4: an event pair around one kernel on stream st
    std::vector<hipEvent_t> kev;
    std::vector<int> kev_phase;      // phase of each pair
    std::vector<int64_t> kev_prod;   // product of each pair
    int kev_used = 0;                // events used (two per pair)
    hipEvent_t kernel_event() {
        if (kev_used == (int)kev.size()) {
            hipEvent_t e;
            BEM_HIP(hipEventCreate(&e));
            kev.push_back(e);
        }
        return kev[kev_used++];
    }
    // modes 2 (both heavy kernels), 3 (near field only), 4 (M2L products only)
    bool times_kernel(int phase) const {
        return timing == 2 || (timing == 3 && phase == 6) || (timing == 4 && phase == 3);
    }
    int open_phase = -1;
    void kbegin(hipStream_t st, int phase) {
        open_phase = times_kernel(phase) ? phase : -1;
        if (open_phase < 0) return;
        BEM_HIP(hipEventRecord(kernel_event(), st));
        kev_phase.resize(kev_used / 2 + 1);
        kev_prod.resize(kev_used / 2 + 1);
        kev_phase[kev_used / 2] = phase;
        kev_prod[kev_used / 2] = prod_seq;
    }
    void kend(hipStream_t st) {
        if (open_phase < 0) return;
        open_phase = -1;
        hipEvent_t e = kernel_event();
        BEM_HIP(hipEventRecord(e, st));
        if (st == side) side_tail = e;
    }
    // After the streams have been synchronised: folds the recorded intervals
    // into the counters (launches = products in which the phase was timed)
    // and frees the events for reuse.
    void collect() {
        bool seen[BEM_NPHASE] = {false};
        int64_t cur = -1;
        for (int i = 0; i + 1 < kev_used; i += 2) {
            float ms = 0.f;
            BEM_HIP(hipEventElapsedTime(&ms, kev[i], kev[i + 1]));
            const int ph = kev_phase[i / 2];
            if (kev_prod[i / 2] != cur) {
                cur = kev_prod[i / 2];
                for (bool &b : seen) b = false;
            }
            phase_ms[ph] += ms;
            if (!seen[ph]) { phase_n[ph]++; seen[ph] = true; }
        }
        kev_used = 0;
        cur = -1;
        for (int i = 1; i < ev_used; i++) {
            if (ev_prod[i] != ev_prod[i - 1]) continue;  // no interval across products
            if (ev_prod[i] != cur) {
                cur = ev_prod[i];
                for (bool &b : seen) b = false;
            }
            float ms = 0.f;
            BEM_HIP(hipEventElapsedTime(&ms, events[i - 1], events[i]));
            const int ph = ev_phase[i];
            if (ph >= 0 && ph < BEM_NPHASE) {
                phase_ms[ph] += ms;
                if (!seen[ph]) { phase_n[ph]++; seen[ph] = true; }
            }
        }
        ev_used = 0;
    }
    ~Ctx() {
        trim_cache();
        for (auto e : events) (void)hipEventDestroy(e);
        for (auto e : kev) (void)hipEventDestroy(e);
        release_streams();
    }

    int device = 0;
    hipStream_t stream = nullptr;
    bem_allocator alloc{};
    bool has_alloc = false;
    std::string err;

    // Work arena: while set (bem_matvec_noalloc), the per-product work
    // buffers are carved from this device region in order instead of being
    // allocated; a product that needs more than arena_size fails.
    char *arena = nullptr;
    size_t arena_size = 0, arena_used = 0;

    // Device bytes in use by the library through this context (bytes_live)
    // and freed blocks kept for reuse (cached).  Without a caller allocator,
    // freed blocks up to cache_limit bytes in total are kept by size class
    // (four classes per power of two) instead of being returned with
    // hipFree, which waits for the whole device: repeated solves allocate
    // the same work buffers, and a context serving requests beside others
    // must not stall them.
    std::atomic<size_t> bytes_live{0};
    std::atomic<size_t> bytes_peak{0};  // largest bytes_live since creation or the last reset
    std::atomic<size_t> cached{0};
    size_t cache_limit = (size_t)1 << 30;
    // Hard bound on the device bytes this context holds (live plus cached;
    // 0: none): an allocation that would pass it first returns the cached
    // blocks, then fails with BEM_ENOMEM (a serving lane's share of the
    // budget).
    size_t limit = 0;
    std::atomic<size_t> held_peak{0};  // largest bytes_live + cached so far
    std::unordered_map<void *, size_t> sizes;
    std::multimap<size_t, void *> cache;
    static size_t size_class(size_t bytes) {
        if (bytes <= 4096) return 4096;
        int top = 63 - __builtin_clzll((unsigned long long)bytes);
        const size_t step = (size_t)1 << (top - 2);
        return (bytes + step - 1) / step * step;
    }
    void *dmalloc(size_t bytes) {
        if (bytes == 0) bytes = 256;
        void *p = nullptr;
        if (limit) {
            // handing out a cached block of the size class leaves live + cached as it is
            const size_t want = has_alloc ? bytes : size_class(bytes);
            if (has_alloc || cache.find(want) == cache.end()) {
                if (bytes_live + cached + want > limit) trim_cache();
                if (bytes_live + cached + want > limit)
                    fail(BEM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes would pass the " +
                                         std::to_string(limit) + "-byte bound of this context");
            }
        }
        if (has_alloc) {
            p = alloc.alloc(alloc.user, bytes, (void *)stream);
            if (!p) fail(BEM_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        } else {
            bytes = size_class(bytes);
            auto it = cache.find(bytes);
            if (it != cache.end()) {
                p = it->second;
                cache.erase(it);
                cached -= bytes;
            } else {
                hipError_t e = hipMalloc(&p, bytes);
                if (e != hipSuccess && cached) {  // give the cache back and try once more
                    (void)hipGetLastError();
                    trim_cache();
                    e = hipMalloc(&p, bytes);
                }
                if (e != hipSuccess)
                    fail(BEM_ENOMEM, "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
            }
        }
        sizes[p] = bytes;
        const size_t live = bytes_live += bytes;
        if (live > bytes_peak) bytes_peak = live;
        if (live + cached > held_peak) held_peak = live + cached;
        return p;
    }
    void dfree(void *p) {
        if (!p) return;
        size_t bytes = 0;
        auto it = sizes.find(p);
        if (it != sizes.end()) {
            bytes = it->second;
            bytes_live -= bytes;
            sizes.erase(it);
        }
        if (has_alloc) alloc.free(alloc.user, p, (void *)stream);
        else if (bytes && cached + bytes <= cache_limit) {
            cache.emplace(bytes, p);
            cached += bytes;
        } else {
            (void)hipFree(p);
        }
    }
    // returns every cached block to the device
    void trim_cache() {
        for (auto &kv : cache) (void)hipFree(kv.second);
        cache.clear();
        cached = 0;
    }
    void sync() { BEM_HIP(hipStreamSynchronize(stream)); }

    // second stream (default priority) for work that runs concurrently with
    // the main stream inside one call, with its fork / join events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t side_tail = nullptr;  // event recorded last on the side stream, if any (timing)
    hipStream_t side_stream() {
        if (!side) {
            BEM_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
            BEM_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
            BEM_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
        }
        return side;
    }
    // side stream waits for everything issued so far on the main stream
    void fork() {
        BEM_HIP(hipEventRecord(ev_fork, stream));
        BEM_HIP(hipStreamWaitEvent(side, ev_fork, 0));
        side_tail = nullptr;
    }
    // main stream waits for everything issued so far on the side stream (on
    // the timing event that closed the side stream's last kernel, when there
    // is one, rather than on one more event)
    void join() {
        hipEvent_t e = side_tail;
        if (!e) {
            BEM_HIP(hipEventRecord(ev_join, side));
            e = ev_join;
        }
        BEM_HIP(hipStreamWaitEvent(stream, e, 0));
        side_tail = nullptr;
    }
    void release_streams() {
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
        side = nullptr;
        ev_fork = ev_join = nullptr;
    }
};

// Zeroes `bytes` bytes at device address p on the context's stream with a
// fill kernel (no memset node, so the call can sit in a captured graph).
void zero_fill(Ctx &c, void *p, size_t bytes);

// With BEM_SETUP_LOG set in the environment, the wall time of a set-up step
// (its device work synchronised first) goes to stderr when the scope ends.
struct SetupTimer {
    Ctx *c;
    const char *what;
    std::chrono::steady_clock::time_point t0;
    bool on;
    SetupTimer(Ctx &ctx, const char *w) : c(&ctx), what(w), t0(std::chrono::steady_clock::now()) {
        static const bool log = std::getenv("BEM_SETUP_LOG") != nullptr;
        on = log;
    }
    ~SetupTimer() {
        if (!on) return;
        (void)hipStreamSynchronize(c->stream);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        std::fprintf(stderr, "bem setup: %s %.2f ms\n", what, ms);
    }
    // the time since construction or the previous lap, as a sub-step
    void lap(const char *part) {
        if (!on) return;
        (void)hipStreamSynchronize(c->stream);
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "bem setup:   %s: %s %.2f ms\n", what, part,
                     std::chrono::duration<double, std::milli>(now - (tl.time_since_epoch().count() ? tl : t0)).count());
        tl = now;
    }
    std::chrono::steady_clock::time_point tl{};
};

// Device array owned by the library, released through the context's allocator.
template <class T>
struct DBuf {
    Ctx *ctx = nullptr;
    T *p = nullptr;
    size_t n = 0;

    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : ctx(o.ctx), p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); ctx = o.ctx; p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }

    void alloc(Ctx *c, size_t count) {
        release();
        ctx = c;
        n = count;
        p = static_cast<T *>(c->dmalloc(sizeof(T) * (count ? count : 1)));
    }
    void zero() {
        if (n) zero_fill(*ctx, p, sizeof(T) * n);
    }
    void release() {
        if (p && ctx) ctx->dfree(p);
        p = nullptr;
        n = 0;
    }
    // copies from host memory the caller may free on return, so it waits for the copy
    void upload(const T *h, size_t count) {
        BEM_REQUIRE(count <= n, BEM_EINVAL, "upload overflow");
        if (count) {
            BEM_HIP(hipMemcpyAsync(p, h, sizeof(T) * count, hipMemcpyHostToDevice, ctx->stream));
            BEM_HIP(hipStreamSynchronize(ctx->stream));
        }
    }
    std::vector<T> download(size_t count) const {
        std::vector<T> h(count);
        if (count) {
            BEM_HIP(hipMemcpyAsync(h.data(), p, sizeof(T) * count, hipMemcpyDeviceToHost, ctx->stream));
            BEM_HIP(hipStreamSynchronize(ctx->stream));
        }
        return h;
    }
    // makes room for at least `count` elements (contents not kept)
    void ensure(Ctx *c, size_t count) {
        if (p && count <= n) return;
        alloc(c, count);
    }
    // grows to at least `count`, keeping the first `keep` elements
    void grow(size_t count, size_t keep) {
        if (count <= n) return;
        DBuf<T> nb;
        nb.alloc(ctx, count);
        if (keep) BEM_HIP(hipMemcpyAsync(nb.p, p, sizeof(T) * keep, hipMemcpyDeviceToDevice, ctx->stream));
        *this = std::move(nb);
    }
};

template <class T>
inline T read_scalar(Ctx &c, const T *dptr) {
    T v;
    BEM_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, c.stream));
    BEM_HIP(hipStreamSynchronize(c.stream));
    return v;
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------- complex
template <class R>
struct cx {
    R re, im;
    cx() = default;
    __host__ __device__ cx(R r) : re(r), im(0) {}
    __host__ __device__ cx(R r, R i) : re(r), im(i) {}
    __host__ __device__ cx &operator+=(const cx &o) { re += o.re; im += o.im; return *this; }
    __host__ __device__ cx &operator-=(const cx &o) { re -= o.re; im -= o.im; return *this; }
    __host__ __device__ cx &operator*=(R s) { re *= s; im *= s; return *this; }
};
template <class R> __host__ __device__ inline cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R> __host__ __device__ inline cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R> __host__ __device__ inline cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <class R> __host__ __device__ inline cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R> __host__ __device__ inline cx<R> operator*(cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <class R> __host__ __device__ inline cx<R> operator*(R s, cx<R> a) { return {a.re * s, a.im * s}; }
template <class R> __host__ __device__ inline cx<R> conj(cx<R> a) { return {a.re, -a.im}; }

// Value traits: Laplace values are real, Helmholtz values complex.
template <class V> struct real_of { using type = V; };
template <class R> struct real_of<cx<R>> { using type = R; };

template <class V> __host__ __device__ inline V vzero() { return V(0); }

__host__ __device__ inline double re_part(double v) { return v; }
__host__ __device__ inline float re_part(float v) { return v; }
template <class R> __host__ __device__ inline R re_part(cx<R> v) { return v.re; }

template <class To, class From> __host__ __device__ inline To vcast(From v) { return To(v); }
template <> __host__ __device__ inline cx<float> vcast<cx<float>, cx<double>>(cx<double> v) {
    return cx<float>((float)v.re, (float)v.im);
}
template <> __host__ __device__ inline cx<double> vcast<cx<double>, cx<float>>(cx<float> v) {
    return cx<double>((double)v.re, (double)v.im);
}
template <> __host__ __device__ inline cx<double> vcast<cx<double>, cx<double>>(cx<double> v) { return v; }
template <> __host__ __device__ inline cx<float> vcast<cx<float>, cx<float>>(cx<float> v) { return v; }

__device__ inline void vsincos(float x, float *s, float *c) { sincosf(x, s, c); }
__device__ inline void vsincos(double x, double *s, double *c) { sincos(x, s, c); }

// The far-field kernels (P2M, M2M, the M2L steps, L2L) raise their waves'
// issue priority: they run beside the near-field kernel, whose VALU-bound
// waves would otherwise take most of a CU's issue slots from their
// latency-bound ones.  (Wave priority within a CU; the streams keep the
// default priority.)
__device__ inline void far_field_priority() { __builtin_amdgcn_s_setprio(3); }

// Wave-wide (64 lanes) sums by butterfly shuffles: every lane ends with the
// same total, accumulated in a fixed order (deterministic).
__device__ inline double wave_sum(double v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wave_sum(float v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <class R> __device__ inline cx<R> wave_sum(cx<R> v) { return {wave_sum(v.re), wave_sum(v.im)}; }
__device__ inline double wave_max(double v) {
    for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

constexpr int MAXLEV = 21;
constexpr int MAX_ORDER = 10;

}  // namespace bem
