// Label runs: the session indices partitioned by label, stably, with wave
// ballots and mbcnt ranks.
//
// Method (Ando et al., arXiv 2106.12863, section "Coordinated Batch
// Processing" and Fig. 3: every chunk of sessions is discriminated before
// the Map stage, so later stages can take the sessions of one direction
// together).  The output idx[n] lists first every index whose label is 0, in
// increasing order, then those labelled 1, 2 and 3; totals[4] counts them.
//
// Design.  Workgroups of 256 lanes take contiguous ranges of kRunChunk
// sessions.  In a tile of 4,096 sessions a lane holds 16 consecutive ones
// (slots s = 0..15, one 16-byte load, the next tile's load in flight).
// Small workgroups keep the tile's phases (ballots, the barrier, placement
// in LDS, the barrier, write-out) of several workgroups per CU overlapped:
// on 1.6e9 labels the scatter and count together took 4.5 ms with 1,024
// lanes, 3.1 ms with 512, 2.85 ms with 256 and 2.96 ms with 128.  For each label L and
// slot s a wave ballot marks the lanes whose slot-s session has label L;
// mbcnt over the 16 masks of L counts the sessions of label L in earlier
// lanes, the lane's own earlier slots complete the rank, and popcounts give
// the wave's class totals.  A count pass writes every
// range's class totals, one workgroup scans them into run offsets, and the
// scatter pass repeats the ballots, places each index of a tile in LDS at
//   label segment start + wave offset + rank
// and writes every label segment to run start + range offset + tile offset
// with consecutive stores.
// Indices are 32-bit, so n < 2^32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pass_common.h"
#include "sinet_internal.h"

namespace sinet {

constexpr uint32_t kRunLanes = 256;
constexpr uint32_t kRunWaves = kRunLanes / 64;
constexpr uint32_t kScanLanes = 1024;                 // the one scan workgroup
constexpr uint32_t kRunSlots = 16;                    // consecutive sessions per lane in a tile
constexpr uint32_t kRunTile = kRunSlots * kRunLanes;  // sessions per tile
constexpr uint32_t kRunTiles = 16;                    // tiles per workgroup range
constexpr uint64_t kRunChunk = (uint64_t)kRunTile * kRunTiles;
constexpr uint32_t kNoLabel = 4u;                     // slots past the end match no label

// The 16 labels of sessions i .. i+15 (low two bits of each byte), one per
// byte; sessions at or past n get kNoLabel.
__device__ __forceinline__ uint4 run_labels16(const uint8_t* label, uint64_t i, uint64_t n, bool vec) {
    if (vec && i + kRunSlots <= n) {
        // read once per pass: nontemporal
        const u32x4_t v = __builtin_nontemporal_load(glob(reinterpret_cast<const u32x4_t*>(label + i)));
        return make_uint4(v.x & 0x03030303u, v.y & 0x03030303u, v.z & 0x03030303u, v.w & 0x03030303u);
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (uint32_t k = 0; k < kRunSlots; ++k)
        w[k >> 2] |= (i + k < n ? (uint32_t)(*glob(label + i + k) & 3u) : kNoLabel) << (8 * (k & 3));
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ uint32_t slot_label(const uint4& v, uint32_t s) {
    const uint32_t w = s < 4 ? v.x : s < 8 ? v.y : s < 12 ? v.z : v.w;
    return (w >> (8 * (s & 3))) & 0xFFu;
}

// Ballots of a wave's tile: for each label, the sessions of that label in
// earlier lanes (mbcnt over the 16 slot masks) and the wave's class totals.
__device__ __forceinline__ void wave_ranks(const uint4& v, uint32_t pre[4], uint32_t wt[4]) {
#pragma unroll
    for (uint32_t L = 0; L < 4; ++L) {
        pre[L] = 0;
        wt[L] = 0;
    }
#pragma unroll
    for (uint32_t s = 0; s < kRunSlots; ++s) {
        const uint32_t l = slot_label(v, s);
#pragma unroll
        for (uint32_t L = 0; L < 4; ++L) {
            const unsigned long long m = __ballot(l == L);
            pre[L] = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                               __builtin_amdgcn_mbcnt_lo((uint32_t)m, pre[L]));
            wt[L] += (uint32_t)__popcll(m);
        }
    }
}

// Count pass: the class totals of every workgroup range.
__global__ void __launch_bounds__(kRunLanes) k_runs_count(const uint8_t* __restrict__ label,
                                                          uint64_t n, uint32_t vec,
                                                          uint32_t* __restrict__ cnt) {
    __shared__ uint32_t s_w[kRunWaves][4];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint64_t r0 = (uint64_t)blockIdx.x * kRunChunk;
    uint32_t tot[4] = {0u, 0u, 0u, 0u};
    uint4 cur = make_uint4(0u, 0u, 0u, 0u);
    if (r0 < n) cur = run_labels16(label, r0 + (uint64_t)kRunSlots * threadIdx.x, n, vec != 0);
    for (uint32_t tl = 0; tl < kRunTiles; ++tl) {
        const uint64_t base = r0 + (uint64_t)tl * kRunTile;
        if (base >= n) break;
        // the next tile's labels are in flight while this one is counted
        const uint64_t nb = base + kRunTile;
        uint4 nxt = make_uint4(0u, 0u, 0u, 0u);
        if (tl + 1 < kRunTiles && nb < n)
            nxt = run_labels16(label, nb + (uint64_t)kRunSlots * threadIdx.x, n, vec != 0);
#pragma unroll
        for (uint32_t s = 0; s < kRunSlots; ++s) {
            const uint32_t l = slot_label(cur, s);
#pragma unroll
            for (uint32_t L = 0; L < 4; ++L) tot[L] += (uint32_t)__popcll(__ballot(l == L));
        }
        cur = nxt;
    }
    if (lane == 0)
        for (uint32_t L = 0; L < 4; ++L) s_w[wave][L] = tot[L];
    __syncthreads();
    if (threadIdx.x < 4) {
        uint32_t s = 0;
        for (uint32_t w = 0; w < kRunWaves; ++w) s += s_w[w][threadIdx.x];
        cnt[4ull * blockIdx.x + threadIdx.x] = s;
    }
}

// Scan: run starts (label-major) plus each range's exclusive prefix, and the
// totals.  One workgroup; lane j takes a contiguous slice of the ranges.
__global__ void __launch_bounds__(kScanLanes) k_runs_scan(const uint32_t* __restrict__ cnt, uint32_t G,
                                                         uint32_t* __restrict__ off,
                                                         unsigned long long* __restrict__ totals) {
    __shared__ uint32_t s_p[4][kScanLanes];
    __shared__ uint32_t s_base[4];
    const uint32_t j = threadIdx.x;
    const uint32_t per = (G + kScanLanes - 1) / kScanLanes;
    const uint32_t g0 = min(G, j * per), g1 = min(G, g0 + per);
    uint32_t loc[4] = {0u, 0u, 0u, 0u};
    for (uint32_t g = g0; g < g1; ++g)
        for (uint32_t L = 0; L < 4; ++L) loc[L] += cnt[4ull * g + L];
    for (uint32_t L = 0; L < 4; ++L) s_p[L][j] = loc[L];
    __syncthreads();
    // inclusive scan of the slices, per label (Hillis-Steele over LDS)
    for (uint32_t d = 1; d < kScanLanes; d <<= 1) {
        uint32_t v[4];
        for (uint32_t L = 0; L < 4; ++L) v[L] = j >= d ? s_p[L][j - d] : 0u;
        __syncthreads();
        for (uint32_t L = 0; L < 4; ++L) s_p[L][j] += v[L];
        __syncthreads();
    }
    if (j == 0) {
        uint32_t b = 0;
        for (uint32_t L = 0; L < 4; ++L) {
            const uint32_t t = s_p[L][kScanLanes - 1];
            s_base[L] = b;
            totals[L] = t;
            b += t;
        }
    }
    __syncthreads();
    uint32_t run[4];
    for (uint32_t L = 0; L < 4; ++L) run[L] = s_base[L] + s_p[L][j] - loc[L];
    for (uint32_t g = g0; g < g1; ++g)
        for (uint32_t L = 0; L < 4; ++L) {
            off[4ull * g + L] = run[L];
            run[L] += cnt[4ull * g + L];
        }
}

// Scatter pass: every index written at its run position.  A tile's indices
// are first placed in LDS in label order (label segments of the tile, then
// waves, then ranks), so that each label's segment leaves the CU as
// consecutive stores.
__global__ void __launch_bounds__(kRunLanes) k_runs_scatter(const uint8_t* __restrict__ label,
                                                            uint64_t n, uint32_t vec,
                                                            const uint32_t* __restrict__ off,
                                                            uint32_t* __restrict__ idx) {
    __shared__ uint4 s_w[kRunWaves];           // each wave's class totals
    __shared__ uint32_t s_idx[kRunTile + 1];   // the last word takes the slots past the end
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    const uint64_t r0 = (uint64_t)blockIdx.x * kRunChunk;
    uint32_t run[4];
#pragma unroll
    for (uint32_t L = 0; L < 4; ++L) run[L] = off[4ull * blockIdx.x + L];
    uint4 cur = make_uint4(0u, 0u, 0u, 0u);
    if (r0 < n) cur = run_labels16(label, r0 + (uint64_t)kRunSlots * threadIdx.x, n, vec != 0);
    for (uint32_t tl = 0; tl < kRunTiles; ++tl) {
        const uint64_t base = r0 + (uint64_t)tl * kRunTile;
        if (base >= n) break;
        const uint64_t nb = base + kRunTile;
        uint4 nxt = make_uint4(0u, 0u, 0u, 0u);
        if (tl + 1 < kRunTiles && nb < n)
            nxt = run_labels16(label, nb + (uint64_t)kRunSlots * threadIdx.x, n, vec != 0);
        uint32_t pre[4], wt[4];
        wave_ranks(cur, pre, wt);
        if (lane == 0) s_w[wave] = make_uint4(wt[0], wt[1], wt[2], wt[3]);
        __syncthreads();   // (1) wave totals visible; the previous tile's write-out is done
        // the wave's offset inside its label segment, the tile's totals, and
        // the segments' starts in the tile (one 16-byte read per wave)
        uint32_t wo[4] = {0u, 0u, 0u, 0u}, tt[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (uint32_t w = 0; w < kRunWaves; ++w) {
            const uint4 x = s_w[w];
            const uint32_t e = w < wave ? 0xFFFFFFFFu : 0u;
            wo[0] += x.x & e;
            wo[1] += x.y & e;
            wo[2] += x.z & e;
            wo[3] += x.w & e;
            tt[0] += x.x;
            tt[1] += x.y;
            tt[2] += x.z;
            tt[3] += x.w;
        }
        const uint32_t tb1 = tt[0], tb2 = tt[0] + tt[1], tb3 = tb2 + tt[2], valid = tb3 + tt[3];
        const uint32_t q0[4] = {wo[0] + pre[0], tb1 + wo[1] + pre[1], tb2 + wo[2] + pre[2],
                                tb3 + wo[3] + pre[3]};
        uint32_t seen[4] = {0u, 0u, 0u, 0u};  // the lane's earlier slots per label
        const uint64_t i = base + (uint64_t)kRunSlots * threadIdx.x;
#pragma unroll
        for (uint32_t s = 0; s < kRunSlots; ++s) {
            const uint32_t l = slot_label(cur, s);
            const uint32_t q = (l == 0 ? q0[0] + seen[0] : l == 1 ? q0[1] + seen[1]
                                : l == 2 ? q0[2] + seen[2] : l == 3 ? q0[3] + seen[3] : kRunTile);
            s_idx[q] = (uint32_t)(i + s);
#pragma unroll
            for (uint32_t M = 0; M < 4; ++M) seen[M] += l == M ? 1u : 0u;
        }
        __syncthreads();   // (2) the tile's indices are in LDS; s_w may be rewritten
        // write-out: LDS slot q of label L goes to run[L] + (q - segment start)
        const uint32_t d1 = run[1] - tb1, d2 = run[2] - tb2, d3 = run[3] - tb3;
        for (uint32_t q = threadIdx.x; q < valid; q += kRunLanes) {
            const uint32_t pos = q + (q < tb1 ? run[0] : q < tb2 ? d1 : q < tb3 ? d2 : d3);
            __builtin_nontemporal_store(s_idx[q], glob(idx + pos));  // written once
        }
#pragma unroll
        for (uint32_t L = 0; L < 4; ++L) run[L] += tt[L];
        cur = nxt;
        // the next tile overwrites s_idx only after its barrier (1), which
        // every wave reaches once its write-out has read s_idx
    }
}

__global__ void k_runs_zero(unsigned long long* totals) {
    if (threadIdx.x < 4) totals[threadIdx.x] = 0ull;
}

}  // namespace sinet

using namespace sinet;

extern "C" sinet_status sinet_label_runs(const uint8_t* label, uint64_t n, uint32_t* idx,
                                         uint64_t* totals, hipStream_t stream) {
    if (!totals) return fail(SINET_ERR_INVALID_ARG, "totals is NULL");
    if (n >= (1ull << 32)) return fail(SINET_ERR_UNSUPPORTED, "2^32 sessions or more (32-bit indices)");
    unsigned long long* tot = reinterpret_cast<unsigned long long*>(totals);
    if (n == 0) {
        hipLaunchKernelGGL(k_runs_zero, dim3(1), dim3(64), 0, stream, tot);
        return check_hip(hipGetLastError(), "label runs launch");
    }
    if (!label || !idx) return fail(SINET_ERR_INVALID_ARG, "label or idx is NULL");
    const uint64_t G = (n + kRunChunk - 1) / kRunChunk;   // < 2^32 / 2^18
    void* ws = nullptr;
    sinet_status st = ws_alloc(&ws, 2 * 16 * G, stream);
    if (st != SINET_OK) return st;
    uint32_t* cnt = static_cast<uint32_t*>(ws);
    uint32_t* off = cnt + 4 * G;
    const uint32_t vec = ((uintptr_t)label & 15u) == 0 ? 1u : 0u;
    hipLaunchKernelGGL(k_runs_count, dim3((uint32_t)G), dim3(kRunLanes), 0, stream, label, n, vec, cnt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_runs_scan, dim3(1), dim3(kScanLanes), 0, stream, cnt, (uint32_t)G, off, tot);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_runs_scatter, dim3((uint32_t)G), dim3(kRunLanes), 0, stream, label, n,
                           vec, off, idx);
        e = hipGetLastError();
    }
    const sinet_status st2 = ws_free(ws, stream);
    st = check_hip(e, "label runs launch");
    return st != SINET_OK ? st : st2;
}
