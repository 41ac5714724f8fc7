// Device helpers shared by the pass kernels (kernels.hip) and the
// sliding-window histogram (window.hip): global-address casts, 16-byte column
// loads, the Map step's key (the bin of a timestamp) and the per-lane
// dropped-session counters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sinet_internal.h"

namespace sinet {

// Column and table pointers always address device (global) memory.  Where the
// kernels read them from a descriptor in memory (the batch kernels), the
// compiler can no longer infer that and falls back to flat accesses, whose
// waits are tied to LDS operations; these casts restore global accesses.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* glob(const T* q) {
    return (const __attribute__((address_space(1))) T*)q;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* glob(T* q) {
    return (__attribute__((address_space(1))) T*)q;
}
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned long long u64x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint4 gload4(const uint32_t* q) {  // q 16-byte aligned
    const u32x4_t v = *glob(reinterpret_cast<const u32x4_t*>(q));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ ulonglong2 gload2(const uint64_t* q) {
    const u64x2_t v = *glob(reinterpret_cast<const u64x2_t*>(q));
    return make_ulonglong2(v.x, v.y);
}
__device__ __forceinline__ void gstore4(uint32_t* q, uint4 v) {
    *glob(reinterpret_cast<u32x4_t*>(q)) = u32x4_t{v.x, v.y, v.z, v.w};
}

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bin_of(uint32_t x, uint32_t width, uint64_t magic) {
    // floor(x / width) for 32-bit x: with c = ceil(2^64 / width) the high 64
    // bits of x * c equal the quotient (Lemire, Kaser, Kurz, "Faster remainder
    // by direct computation", 2019).  width == 1 skips the multiply.
    if (width == 1u) return x;
    uint64_t t = (uint64_t)x * (uint32_t)magic;
    uint64_t u = (uint64_t)x * (uint32_t)(magic >> 32) + (t >> 32);
    return (uint32_t)(u >> 32);
}

// In-window test and bin of one session (the Map step's key).
__device__ __forceinline__ bool in_window(const PassParams& p, uint32_t ts, uint32_t& bin) {
    bin = bin_of(ts - p.t0, p.width, p.magic);
    return ts >= p.t0 && bin < p.n_bins;
}

struct Dropped {
    unsigned long long c[4];
    unsigned long long b[4];
    __device__ __forceinline__ void add(uint32_t lab, uint64_t nbytes) {
#pragma unroll
        for (uint32_t l = 0; l < 4; ++l) {  // constant indices: stays in registers
            const bool h = lab == l;
            c[l] += h ? 1ull : 0ull;
            b[l] += h ? nbytes : 0ull;
        }
    }
    __device__ __forceinline__ void flush(unsigned long long* out) const {
        if (!out) return;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            if (c[l]) {
                atomicAdd(out + 2 * l, c[l]);
                atomicAdd(out + 2 * l + 1, b[l]);
            }
        }
    }
};

// Workgroup barrier for LDS traffic only: waits for this wave's LDS
// operations, then for every wave, but leaves its global loads in flight
// (__syncthreads also waits for every outstanding global load, which empties
// a prefetch queue at each barrier).  The memory clobber keeps the compiler
// from moving memory accesses across it.  Only for barriers that order LDS
// accesses; global memory written before it is not made visible by it.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Minimum over the 64 lanes of a wave by DPP row shifts and row broadcasts
// (lanes a row shift or a masked row leaves without a source keep ~0, the
// identity of min); lane 63 ends with the result.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_min_step(uint32_t x) {
    return min(x, (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFF, (int)x, CTRL, ROW_MASK, 0xF,
                                                         false));
}
__device__ __forceinline__ uint32_t wave_min(uint32_t x) {
    x = dpp_min_step<0x111, 0xF>(x);  // row_shr:1
    x = dpp_min_step<0x112, 0xF>(x);  // row_shr:2
    x = dpp_min_step<0x114, 0xF>(x);  // row_shr:4
    x = dpp_min_step<0x118, 0xF>(x);  // row_shr:8
    x = dpp_min_step<0x142, 0xA>(x);  // row_bcast:15 into rows 1 and 3
    x = dpp_min_step<0x143, 0xC>(x);  // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

}  // namespace sinet
