// GPU form of the seeded synthetic session generator.
//
// Each session column value is a pure function of (stream keys, session
// index) computed with the SplitMix64 output function (Steele, Lea and Flood,
// OOPSLA 2014) and integer table interpolation only, identical operation for
// operation to the host form in __init__.py, so the host can regenerate any
// single session of a device-generated day.  This file holds no part of the
// classification or histogram method.
#include <hip/hip_runtime.h>
#include <stdint.h>

extern "C" {

typedef struct {
    uint64_t n_total;   // sessions in the whole stream (stratified time base)
    uint64_t key[6];    // ts, src, src-pick, dst, dst-pick, bytes stream keys
    uint32_t ts_mode;   // 0 uniform, 1 diurnal table, 2 stratified uniform rate
    uint32_t ts_span;   // uniform: range; diurnal: day length T; stratified: W
    uint32_t jitter;    // +-J ms reflected jitter
    uint32_t t_origin;  // added to every timestamp
    uint32_t in_thr;    // src/dst inside a prefix when low word < in_thr
    uint32_t n_prefix;
} sinetgen_params;

}  // extern "C"

namespace {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kQK = 65536;
constexpr int kQFrac = 8;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t key, uint64_t i) {
    return mix64((i + 1) * kGolden + key);
}

__device__ __forceinline__ uint64_t mulhi32(uint64_t x32, uint64_t n) {
    return (x32 * n) >> 32;
}

__device__ uint32_t gen_ts(const sinetgen_params& p, const uint64_t* qtab, uint64_t i) {
    uint64_t r = draw(p.key[0], i) >> 32;
    if (p.ts_mode == 0) return (uint32_t)(mulhi32(r, p.ts_span) + p.t_origin);
    int64_t base;
    if (p.ts_mode == 1) {
        int64_t num = (int64_t)(2 * i + 1) * kQK;
        int64_t den = 2 * (int64_t)p.n_total;
        int64_t k = num / den;
        int64_t frac = num % den;
        int64_t qk = (int64_t)qtab[k];
        int64_t dq = (int64_t)qtab[k + 1] - qk;
        base = (qk + (dq * frac) / den) >> kQFrac;
    } else {
        base = ((int64_t)(2 * i + 1) * (int64_t)p.ts_span) / (2 * (int64_t)p.n_total);
    }
    int64_t J = p.jitter;
    int64_t x = base + (int64_t)mulhi32(r, 2 * (uint64_t)J + 1) - J;
    int64_t T = p.ts_span;
    if (x < 0) x = -x - 1;
    if (x >= T) x = 2 * T - 1 - x;
    return (uint32_t)(x + p.t_origin);
}

__device__ uint32_t gen_addr(const sinetgen_params& p, const uint32_t* pbase,
                             const uint8_t* plen, uint64_t kcol, uint64_t kpick, uint64_t i) {
    uint64_t r = draw(kcol, i);
    uint64_t host = r >> 32;
    if (p.n_prefix == 0) return (uint32_t)host;
    if ((r & 0xFFFFFFFFull) < (uint64_t)p.in_thr) {
        uint64_t q = mulhi32(draw(kpick, i) >> 32, p.n_prefix);
        uint64_t span = (1ull << (32 - (uint64_t)plen[q])) - 1;
        return (uint32_t)((uint64_t)pbase[q] | (host & span));
    }
    return (uint32_t)host;
}

__device__ uint64_t gen_bytes(const sinetgen_params& p, const uint64_t* ltab, uint64_t i) {
    uint64_t u = draw(p.key[5], i) >> 32;
    uint64_t k = u >> 16, f = u & 0xFFFF;
    uint64_t lo = ltab[k];
    return lo + (((ltab[k + 1] - lo) * f) >> 16);
}

__global__ void k_gen(sinetgen_params p, const uint32_t* __restrict__ pbase,
                      const uint8_t* __restrict__ plen, const uint64_t* __restrict__ qtab,
                      const uint64_t* __restrict__ ltab, uint64_t i0, uint64_t n,
                      uint32_t* __restrict__ ts, uint32_t* __restrict__ src,
                      uint32_t* __restrict__ dst, uint64_t* __restrict__ bytes) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        uint64_t i = i0 + j;
        if (ts) ts[j] = gen_ts(p, qtab, i);
        if (src) src[j] = gen_addr(p, pbase, plen, p.key[1], p.key[2], i);
        if (dst) dst[j] = gen_addr(p, pbase, plen, p.key[3], p.key[4], i);
        if (bytes) bytes[j] = gen_bytes(p, ltab, i);
    }
}

// Watch-list overlay: sessions i0 + j whose draw from the source (or
// destination) overlay stream falls below thr get a listed host, picked as
// floor(K * u^2) with u the draw's high word over 2^32.
__global__ void k_watch_overlay(const uint32_t* __restrict__ addrs, uint32_t K, uint64_t key_src,
                        uint64_t key_dst, uint32_t thr, uint64_t i0, uint64_t n,
                        uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
        uint64_t i = i0 + j;
        uint64_t rs = draw(key_src, i), rd = draw(key_dst, i);
        if ((rs & 0xFFFFFFFFull) < thr) {
            uint64_t u = rs >> 32;
            src[j] = addrs[mulhi32((u * u) >> 32, K)];
        }
        if ((rd & 0xFFFFFFFFull) < thr) {
            uint64_t u = rd >> 32;
            dst[j] = addrs[mulhi32((u * u) >> 32, K)];
        }
    }
}

}  // namespace

extern "C" int sinetgen_watch(const uint32_t* addrs, uint32_t K, uint64_t key_src,
                              uint64_t key_dst, uint32_t thr, uint64_t i0, uint64_t n,
                              uint32_t* src, uint32_t* dst, hipStream_t stream) {
    if (!addrs || K == 0 || !src || !dst) return 1;
    if (n == 0) return 0;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_watch_overlay, dim3((unsigned)blocks), dim3(256), 0, stream, addrs, K, key_src,
                       key_dst, thr, i0, n, src, dst);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}

extern "C" int sinetgen_fill(const sinetgen_params* p, const uint32_t* pbase,
                             const uint8_t* plen, const uint64_t* qtab,
                             const uint64_t* ltab, uint64_t i0, uint64_t n,
                             uint32_t* ts, uint32_t* src, uint32_t* dst,
                             uint64_t* bytes, hipStream_t stream) {
    if (!p || !ltab || (p->ts_mode == 1 && !qtab) || (p->n_prefix && (!pbase || !plen)))
        return 1;
    if (p->ts_mode > 2 || p->n_total == 0 || i0 + n > p->n_total) return 1;
    if (n == 0) return 0;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_gen, dim3((unsigned)blocks), dim3(256), 0, stream, *p, pbase, plen,
                       qtab, ltab, i0, n, ts, src, dst, bytes);
    return hipGetLastError() == hipSuccess ? 0 : 2;
}
