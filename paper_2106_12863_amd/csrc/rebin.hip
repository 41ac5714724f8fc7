// Coarser time frames of a histogram (section "All Sessions of SINET",
// Figures 6-7: the sessions grouped into one-hour frames).  out[r][k] is the
// sum of in[r][b] over the k-th group of `factor` consecutive bins of row r
// (the last group may be shorter), modulo 2^64.  HBM bound: every input bin
// is read once.
//   factor <= kRebinSmall: one lane per output frame sums its bins.
//   larger factors: a workgroup takes a tile of consecutive bins of one row;
//   in each step its lanes read consecutive bins (coalesced).  While a wave
//   stays inside one frame its lanes keep running sums, reduced over the
//   wave when the frame changes; a step that straddles frames runs a
//   segmented scan across the wave (frames are non-decreasing across lanes)
//   and the last lane of every frame adds its sum.  Both go to the tile's
//   frames in LDS; the tile's frames are then added to the (cleared)
//   output with device-scope atomics, since the frames at a tile's edges are
//   shared with its neighbours.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sinet.h"
#include "sinet_internal.h"

namespace sinet {
namespace {

constexpr uint32_t kRebinSmall = 32;
constexpr int kRebinBlock = 256;
constexpr uint32_t kRebinSteps = 32;                        // steps of one tile
constexpr uint32_t kRebinTile = kRebinBlock * kRebinSteps;  // 8192 bins
constexpr uint32_t kRebinFrames = kRebinTile / kRebinSmall + 2;  // frames a tile can touch

// floor(x / factor) for 32-bit x with magic = ceil(2^64 / factor), factor >= 2
// (Lemire, Kaser, Kurz, "Faster remainder by direct computation", 2019).
__device__ __forceinline__ uint32_t frame_of(uint32_t x, uint64_t magic) {
    const uint64_t t = (uint64_t)x * (uint32_t)magic;
    const uint64_t u = (uint64_t)x * (uint32_t)(magic >> 32) + (t >> 32);
    return (uint32_t)(u >> 32);
}

__device__ __forceinline__ unsigned long long shfl_up64(unsigned long long v, int d) {
    const int lo = __shfl_up((int)(uint32_t)v, d);
    const int hi = __shfl_up((int)(uint32_t)(v >> 32), d);
    return ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
}

__global__ void __launch_bounds__(kRebinBlock) k_rebin_small(const uint64_t* __restrict__ in,
                                                             uint64_t rows, uint64_t n_bins,
                                                             uint32_t factor, uint64_t n_out,
                                                             uint64_t* __restrict__ out) {
    const uint64_t total = rows * n_out;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t o = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total; o += stride) {
        const uint64_t r = o / n_out, k = o % n_out;
        const uint64_t b0 = k * factor;
        const uint64_t b1 = b0 + factor < n_bins ? b0 + factor : n_bins;
        const uint64_t* row = in + r * n_bins;
        uint64_t sum = 0;
        for (uint64_t b = b0; b < b1; ++b) sum += row[b];
        out[o] = sum;
    }
}

// Sum of every lane's v added to acc[f] by one lane (f the same in all lanes).
__device__ __forceinline__ void flush_wave(unsigned long long* acc, unsigned long long v, uint32_t f) {
    if (__ballot(v != 0ull) == 0ull) return;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int lo = __shfl_xor((int)(uint32_t)v, d);
        const int hi = __shfl_xor((int)(uint32_t)(v >> 32), d);
        v += ((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo;
    }
    if ((threadIdx.x & 63u) == 0) atomicAdd(&acc[f], v);
}

__global__ void __launch_bounds__(kRebinBlock) k_rebin_tiles(const uint64_t* __restrict__ in,
                                                             uint64_t rows, uint32_t n_bins,
                                                             uint64_t magic, uint64_t n_out,
                                                             unsigned long long* __restrict__ out) {
    __shared__ unsigned long long acc[kRebinFrames];
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t tiles_per_row = (n_bins + kRebinTile - 1) / kRebinTile;
    const uint64_t tiles = rows * tiles_per_row;
    for (uint32_t f = threadIdx.x; f < kRebinFrames; f += blockDim.x) acc[f] = 0;
    __syncthreads();
    for (uint64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const uint64_t r = t / tiles_per_row;
        const uint32_t t0 = (uint32_t)((t % tiles_per_row) * kRebinTile);
        const uint32_t t1 = (uint64_t)t0 + kRebinTile < n_bins ? t0 + kRebinTile : n_bins;
        const uint32_t k0 = frame_of(t0, magic);  // first frame of the tile
        const uint64_t* row = in + r * n_bins;
        // while the whole wave stays in one frame its lanes only keep running
        // sums; a step that straddles frames runs the segmented scan
        unsigned long long run = 0;
        uint32_t run_k = k0;  // the running sums' frame (the same in every lane)
#pragma unroll 4
        for (uint32_t i = 0; i < kRebinSteps; ++i) {
            const uint64_t b = (uint64_t)t0 + i * kRebinBlock + threadIdx.x;
            // lanes past the tile's end repeat its last frame with nothing to add
            const uint32_t bb = b < t1 ? (uint32_t)b : t1 - 1;
            unsigned long long v = b < t1 ? (unsigned long long)row[b] : 0ull;
            const uint32_t k = frame_of(bb, magic);
            const uint32_t kf = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
            const uint32_t kl = (uint32_t)__builtin_amdgcn_readlane((int)k, 63);
            if (kf == kl && kf == run_k) {
                run += v;
                continue;
            }
            flush_wave(acc, run, run_k - k0);
            run = 0;
            if (kf == kl) {
                run = v;
                run_k = kf;
                continue;
            }
            // inclusive segmented scan over the wave, segments = equal frames
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const unsigned long long y = shfl_up64(v, d);
                const uint32_t ky = (uint32_t)__shfl_up((int)k, d);
                if (lane >= (uint32_t)d && ky == k) v += y;
            }
            const uint32_t kn = (uint32_t)__shfl_down((int)k, 1);
            if (lane == 63u || kn != k) atomicAdd(&acc[k - k0], v);
            run_k = kl;
        }
        flush_wave(acc, run, run_k - k0);
        __syncthreads();
        const uint32_t k1 = frame_of(t1 - 1, magic);  // last frame of the tile
        for (uint32_t f = threadIdx.x; f <= k1 - k0; f += blockDim.x) {
            const unsigned long long v = acc[f];
            acc[f] = 0;
            if (v)
                __hip_atomic_fetch_add(out + r * n_out + k0 + f, v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

}  // namespace

sinet_status run_rebin(const uint64_t* in, uint64_t rows, uint64_t n_bins, uint32_t factor,
                       uint64_t* out, hipStream_t s) {
    const uint64_t n_out = (n_bins + factor - 1) / factor;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (factor <= kRebinSmall) {
        uint64_t blocks = (rows * n_out + kRebinBlock - 1) / kRebinBlock;
        if (blocks > cap) blocks = cap;
        hipLaunchKernelGGL(k_rebin_small, dim3((unsigned)blocks), dim3(kRebinBlock), 0, s, in, rows,
                           n_bins, factor, n_out, out);
        return check_hip(hipGetLastError(), "rebin launch");
    }
    sinet_status st = launch_zero((unsigned long long*)out, rows * n_out, s);
    if (st != SINET_OK) return st;
    uint64_t blocks = rows * ((n_bins + kRebinTile - 1) / kRebinTile);
    if (blocks > cap) blocks = cap;
    const uint64_t magic = (~0ull) / factor + 1;  // ceil(2^64 / factor), factor > 1
    hipLaunchKernelGGL(k_rebin_tiles, dim3((unsigned)blocks), dim3(kRebinBlock), 0, s, in, rows,
                       (uint32_t)n_bins, magic, n_out, (unsigned long long*)out);
    return check_hip(hipGetLastError(), "rebin launch");
}

}  // namespace sinet

extern "C" sinet_status sinet_rebin(const uint64_t* in, uint32_t rows, uint32_t n_bins,
                                    uint32_t factor, uint64_t* out, hipStream_t stream) {
    using namespace sinet;
    if (!in || !out) return fail(SINET_ERR_INVALID_ARG, "in or out is NULL");
    if (rows == 0 || n_bins == 0 || factor == 0)
        return fail(SINET_ERR_INVALID_ARG, "rows, n_bins and factor must be positive");
    return run_rebin(in, rows, n_bins, factor, out, stream);
}
