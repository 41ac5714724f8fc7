// libsinet kernels: per-session discrimination fused with the millisecond
// histogram (one pass over the session columns), for gfx950.
//
// Method (Ando et al., arXiv 2106.12863):
//   * Algorithm 1: an address is inside a CIDR block when
//     bitmask(addr, Z) - bitmask(base, Z) == 0; applied to both endpoints of a
//     session against the whole table, it yields the label
//     in(src) | in(dst) << 1.
//   * Sections "Map" / "Reduce" / "Merge Scatter Pattern": every session maps
//     to key (label, floor((ts - t0) / width)) with value (1, bytes); values
//     merge by unsigned 64-bit addition, associative and commutative, so the
//     order of the device-scope atomic adds below is free and the result is
//     exact.
//
// GPU design (what differs from the paper's Thrust transform + pairwise
// reduction + CPU merge):
//   * one persistent pass; each lane owns 4 consecutive sessions and reads
//     them with 128-bit loads per column (two for the 64-bit byte column) and
//     writes the 4 labels as one 32-bit store;
//   * the table's hot structure (sampled boundaries, membership bits, model
//     parameters, or the prefix rows for the scan) is staged in LDS once per
//     workgroup;
//   * the nearly time-sorted stream is cut into 8 contiguous index ranges,
//     one per XCD (workgroups are dealt to XCDs round-robin), so the bins a
//     range touches stay in that XCD's L2 while its atomics land;
//   * the merge happens in HBM-resident u64 bins with agent-scope atomics
//     executed in L2; no CPU stage.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <tuple>

#include "sinet_device.h"
#include "sinet_internal.h"

namespace sinet {

enum KernelKind : uint32_t {
    KK_SCAN = SINET_LOOKUP_SCAN,
    KK_BSEARCH = SINET_LOOKUP_BSEARCH,
    KK_TRIE = SINET_LOOKUP_TRIE,
    KK_PLA = SINET_LOOKUP_LEARNED_PLA,
    KK_MLP = SINET_LOOKUP_LEARNED_MLP,
    KK_LABEL_IN = 100  // histogram of given labels
};

constexpr int kXcds = 8;
constexpr int kMaxBlock = 1024;

// ---------------------------------------------------------------------------
// searches
// ---------------------------------------------------------------------------
// Learned forms: the model's rounded prediction p is within max_err of the
// true interval for every boundary key; search [p - e, p + e] and confirm the
// bracket B[j] <= a < B[j+1], else fall back to the full search.
__device__ __forceinline__ uint32_t bounded_search(const DevTable& t, uint32_t a, int p) {
    int e = (int)t.max_err;
    int lo = p - e;
    int hi = p + e;
    lo = lo < 0 ? 0 : lo;
    hi = hi > (int)t.m - 1 ? (int)t.m - 1 : hi;
    bool ok = t.B[lo] <= a;
    uint32_t j = 0;
    if (ok) {
        j = (uint32_t)lo + upper_last(t.B + lo, (uint32_t)(hi - lo + 1), a);
        if (j == (uint32_t)hi && (uint32_t)hi + 1 < t.m && t.B[hi + 1] <= a) ok = false;
    }
    if (!ok) {
        atomicAdd(t.fallbacks, 1ull);
        j = upper_last(t.B, t.m, a);
    }
    return j;
}

// Per-workgroup LDS view of the table.
struct LdsView {
    const uint32_t* top;     // BSEARCH
    const uint32_t* member;  // all interval kinds (or global)
    const uint32_t* cb;      // SCAN
    const uint32_t* mask;
    const uint32_t* len;
    const uint32_t* knot;    // PLA
    const float* c;
    const float* g;
    const float* w;          // MLP
};

// Interval index of a (all kinds but SCAN).
template <uint32_t KIND>
__device__ __forceinline__ uint32_t interval_of(const DevTable& t, const LdsView& v, uint32_t a) {
    if constexpr (KIND == KK_BSEARCH) {
        uint32_t i = upper_last(v.top, t.n_top, a);
        if (t.top_log2 == 0) return i;
        uint32_t lo = i << t.top_log2;
        uint32_t cnt = min(1u << t.top_log2, t.m - lo);
        return lo + upper_last(t.B + lo, cnt, a);
    } else if constexpr (KIND == KK_TRIE) {
        uint32_t e = t.trie[a >> 16];
        if (!(e >> 31)) {
            e = t.trie[65536u + e * 256u + ((a >> 8) & 255u)];
            if (!(e >> 31)) e = t.trie[65536u + e * 256u + (a & 255u)];
        }
        return e & 0x7FFFFFFFu;
    } else if constexpr (KIND == KK_PLA) {
        return bounded_search(t, a, clamp_pos(pla_predict(v.knot, v.c, v.g, t.segments, a), t.m));
    } else {  // KK_MLP
        return bounded_search(t, a, clamp_pos(mlp_predict(v.w, t.m_f, a), t.m));
    }
}

// Algorithm 1 over every row: longest match, lowest row on equal length.
// Returns row + 1, or 0 when no row matches.
__device__ __forceinline__ uint32_t scan_owner(const DevTable& t, const LdsView& v, uint32_t a) {
    uint32_t best = 0, best_len = 0;
    for (uint32_t p = 0; p < t.n_prefix; ++p) {
        uint32_t result = (a & v.mask[p]) - v.cb[p];  // SB - CB
        uint32_t l = v.len[p] + 1;                     // 1..33 so that /0 beats "none"
        bool take = (result == 0u) & (l > best_len);
        best = take ? p + 1 : best;
        best_len = take ? l : best_len;
    }
    return best;
}

struct Lookup {
    uint32_t in;     // 0/1
    uint32_t code;   // owner code (row + 1 or 0), valid when want_code
};

template <uint32_t KIND>
__device__ __forceinline__ Lookup lookup(const DevTable& t, const LdsView& v, uint32_t a,
                                         bool want_code) {
    Lookup r;
    if constexpr (KIND == KK_SCAN) {
        r.code = scan_owner(t, v, a);
        r.in = r.code != 0;
    } else {
        uint32_t j = interval_of<KIND>(t, v, a);
        r.in = (v.member[j >> 5] >> (j & 31)) & 1u;
        r.code = want_code ? t.owner[j] : 0u;
    }
    return r;
}

// ---------------------------------------------------------------------------
// the pass kernel
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

struct Dropped {
    unsigned long long c[4];
    unsigned long long b[4];
};

template <bool HIST>
__device__ __forceinline__ void account(const PassParams& p, uint32_t lab, uint32_t ts,
                                        uint64_t nbytes, Dropped& d) {
    if constexpr (HIST) {
        uint32_t x = ts - p.t0;
        uint32_t b = bin_of(x, p.width, p.magic);
        if (ts >= p.t0 && b < p.n_bins) {
            uint64_t k = (uint64_t)lab * p.n_bins + b;
            __hip_atomic_fetch_add(p.count + k, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(p.hbytes + k, (unsigned long long)nbytes, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else {
#pragma unroll
            for (uint32_t l = 0; l < 4; ++l) {  // constant indices: stays in registers
                const bool h = lab == l;
                d.c[l] += h ? 1ull : 0ull;
                d.b[l] += h ? nbytes : 0ull;
            }
        }
    }
}

template <uint32_t KIND, bool HIST>
__device__ __forceinline__ void one_session(const PassParams& p, const LdsView& v, uint64_t i,
                                            Dropped& d) {
    uint32_t lab;
    if (p.pos_out) {
        if constexpr (KIND != KK_SCAN && KIND != KK_LABEL_IN)
            p.pos_out[i] = interval_of<KIND>(p.t, v, p.src[i]);
        return;
    }
    if constexpr (KIND == KK_LABEL_IN) {
        lab = p.label_in[i] & 3u;
    } else {
        bool wc = p.src_inst != nullptr || p.dst_inst != nullptr;
        Lookup ls = lookup<KIND>(p.t, v, p.src[i], wc);
        Lookup ld = lookup<KIND>(p.t, v, p.dst[i], wc);
        lab = ls.in | (ld.in << 1);
        if (p.label_out) p.label_out[i] = (uint8_t)lab;
        if (p.src_inst) p.src_inst[i] = ls.code ? p.t.inst[ls.code - 1] : SINET_NO_INST;
        if (p.dst_inst) p.dst_inst[i] = ld.code ? p.t.inst[ld.code - 1] : SINET_NO_INST;
    }
    if constexpr (HIST) account<HIST>(p, lab, p.ts[i], p.bytes[i], d);
}

template <uint32_t KIND, bool HIST>
__device__ __forceinline__ void four_sessions(const PassParams& p, const LdsView& v, uint64_t g,
                                              Dropped& d) {
    const uint64_t i = g * 4;
    if (p.pos_out) {
        if constexpr (KIND != KK_SCAN && KIND != KK_LABEL_IN) {
            uint4 a = *reinterpret_cast<const uint4*>(p.src + i);
            uint4 o;
            o.x = interval_of<KIND>(p.t, v, a.x);
            o.y = interval_of<KIND>(p.t, v, a.y);
            o.z = interval_of<KIND>(p.t, v, a.z);
            o.w = interval_of<KIND>(p.t, v, a.w);
            *reinterpret_cast<uint4*>(p.pos_out + i) = o;
        }
        return;
    }
    uint32_t lab[4];
    if constexpr (KIND == KK_LABEL_IN) {
        uint32_t l4 = *reinterpret_cast<const uint32_t*>(p.label_in + i);
#pragma unroll
        for (int k = 0; k < 4; ++k) lab[k] = (l4 >> (8 * k)) & 3u;
    } else {
        uint4 s = *reinterpret_cast<const uint4*>(p.src + i);
        uint4 t = *reinterpret_cast<const uint4*>(p.dst + i);
        uint32_t sa[4] = {s.x, s.y, s.z, s.w};
        uint32_t da[4] = {t.x, t.y, t.z, t.w};
        bool wc = p.src_inst != nullptr || p.dst_inst != nullptr;
        uint32_t sc[4], dc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            Lookup ls = lookup<KIND>(p.t, v, sa[k], wc);
            Lookup ld = lookup<KIND>(p.t, v, da[k], wc);
            lab[k] = ls.in | (ld.in << 1);
            sc[k] = ls.code;
            dc[k] = ld.code;
        }
        if (p.label_out) {
            uint32_t packed = lab[0] | (lab[1] << 8) | (lab[2] << 16) | (lab[3] << 24);
            *reinterpret_cast<uint32_t*>(p.label_out + i) = packed;
        }
        if (p.src_inst) {
            uint4 o;
            o.x = sc[0] ? p.t.inst[sc[0] - 1] : SINET_NO_INST;
            o.y = sc[1] ? p.t.inst[sc[1] - 1] : SINET_NO_INST;
            o.z = sc[2] ? p.t.inst[sc[2] - 1] : SINET_NO_INST;
            o.w = sc[3] ? p.t.inst[sc[3] - 1] : SINET_NO_INST;
            *reinterpret_cast<uint4*>(p.src_inst + i) = o;
        }
        if (p.dst_inst) {
            uint4 o;
            o.x = dc[0] ? p.t.inst[dc[0] - 1] : SINET_NO_INST;
            o.y = dc[1] ? p.t.inst[dc[1] - 1] : SINET_NO_INST;
            o.z = dc[2] ? p.t.inst[dc[2] - 1] : SINET_NO_INST;
            o.w = dc[3] ? p.t.inst[dc[3] - 1] : SINET_NO_INST;
            *reinterpret_cast<uint4*>(p.dst_inst + i) = o;
        }
    }
    if constexpr (HIST) {
        uint4 ts = *reinterpret_cast<const uint4*>(p.ts + i);
        ulonglong2 b01 = *reinterpret_cast<const ulonglong2*>(p.bytes + i);
        ulonglong2 b23 = *reinterpret_cast<const ulonglong2*>(p.bytes + i + 2);
        account<HIST>(p, lab[0], ts.x, b01.x, d);
        account<HIST>(p, lab[1], ts.y, b01.y, d);
        account<HIST>(p, lab[2], ts.z, b23.x, d);
        account<HIST>(p, lab[3], ts.w, b23.y, d);
    }
}

// Stage the table's hot arrays into LDS (layout chosen on the host).
template <uint32_t KIND>
__device__ LdsView stage_lds(const DevTable& t, uint32_t* lds) {
    LdsView v{};
    uint32_t off = 0;
    auto copy = [&](const uint32_t* src, uint32_t n) -> const uint32_t* {
        uint32_t* dst = lds + off;
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) dst[k] = src[k];
        off += n;
        return dst;
    };
    if constexpr (KIND == KK_SCAN) {
        v.cb = copy(t.cb, t.n_prefix);
        v.mask = copy(t.mask, t.n_prefix);
        v.len = copy(t.len, t.n_prefix);
    } else if constexpr (KIND != KK_LABEL_IN) {
        if constexpr (KIND == KK_BSEARCH) v.top = copy(t.top, t.n_top);
        if constexpr (KIND == KK_PLA) {
            v.knot = copy(t.knot, t.segments);
            v.c = reinterpret_cast<const float*>(
                copy(reinterpret_cast<const uint32_t*>(t.pla_c), t.segments));
            v.g = reinterpret_cast<const float*>(
                copy(reinterpret_cast<const uint32_t*>(t.pla_g), t.segments));
        }
        if constexpr (KIND == KK_MLP)
            v.w = reinterpret_cast<const float*>(
                copy(reinterpret_cast<const uint32_t*>(t.mlp), SINET_MLP_PARAMS));
        v.member = t.lds_member_words ? copy(t.member, t.lds_member_words) : t.member;
    }
    __syncthreads();
    return v;
}

template <uint32_t KIND, bool HIST, bool VEC>
__global__ void __launch_bounds__(kMaxBlock) k_pass(PassParams p) {
    extern __shared__ uint32_t lds[];
    const LdsView v = stage_lds<KIND>(p.t, lds);

    // XCD-contiguous split of the tiles (one tile = 4 sessions per lane).
    const uint64_t groups = (p.n + 3) / 4;
    const uint64_t tile = blockDim.x;
    const uint64_t n_tiles = (groups + tile - 1) / tile;
    const uint32_t W = gridDim.x;
    const uint32_t xcd = blockIdx.x % kXcds;
    const uint32_t lid = blockIdx.x / kXcds;
    const uint32_t per = W / kXcds, rem = W % kXcds;
    const uint32_t nx = per + (xcd < rem ? 1u : 0u);
    const uint64_t cum = (uint64_t)xcd * per + min(xcd, rem);
    const uint64_t T0 = n_tiles * cum / W;
    const uint64_t T1 = n_tiles * (cum + nx) / W;

    Dropped d{};
    for (uint64_t tl = T0 + lid; tl < T1; tl += nx) {
        const uint64_t g = tl * tile + threadIdx.x;
        if (g >= groups) continue;
        if (VEC && g * 4 + 4 <= p.n) {
            four_sessions<KIND, HIST>(p, v, g, d);
        } else {
            for (uint64_t i = g * 4; i < p.n && i < g * 4 + 4; ++i) one_session<KIND, HIST>(p, v, i, d);
        }
    }
    if constexpr (HIST) {
        if (p.dropped) {
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                if (d.c[l]) {
                    atomicAdd(p.dropped + 2 * l, d.c[l]);
                    atomicAdd(p.dropped + 2 * l + 1, d.b[l]);
                }
            }
        }
    }
}

__global__ void k_zero(unsigned long long* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t head = ((uintptr_t)p & 15) ? 1 : 0;  // p is 8-byte aligned
    if (head && i == 0) p[0] = 0;
    ulonglong2* q = reinterpret_cast<ulonglong2*>(p + head);
    const uint64_t n2 = (n - head) / 2;
    for (uint64_t k = i; k < n2; k += stride) q[k] = make_ulonglong2(0, 0);
    if (i == 0 && ((n - head) & 1)) p[n - 1] = 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using KernelFn = void (*)(PassParams);

template <uint32_t KIND>
static KernelFn pick_fn(bool hist, bool vec) {
    if (hist) return vec ? k_pass<KIND, true, true> : k_pass<KIND, true, false>;
    return vec ? k_pass<KIND, false, true> : k_pass<KIND, false, false>;
}

static KernelFn pick(uint32_t kind, bool hist, bool vec) {
    switch (kind) {
        case KK_SCAN: return pick_fn<KK_SCAN>(hist, vec);
        case KK_BSEARCH: return pick_fn<KK_BSEARCH>(hist, vec);
        case KK_TRIE: return pick_fn<KK_TRIE>(hist, vec);
        case KK_PLA: return pick_fn<KK_PLA>(hist, vec);
        case KK_MLP: return pick_fn<KK_MLP>(hist, vec);
        case KK_LABEL_IN: return pick_fn<KK_LABEL_IN>(hist, vec);
        default: return nullptr;
    }
}

uint32_t device_cu_count() {
    static std::mutex mu;
    static std::map<int, uint32_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    hipDeviceProp_t prop;
    uint32_t cus = 256;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
        cus = (uint32_t)prop.multiProcessorCount;
    cache[dev] = cus;
    return cus;
}

static int blocks_per_cu(KernelFn fn, int block, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<void*, int, size_t, int>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto key = std::make_tuple((void*)fn, block, lds, dev);
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, lds) != hipSuccess || nb < 1)
        nb = 1;
    cache[key] = nb;
    return nb;
}

uint64_t div_magic(uint32_t width) {
    return width >= 2 ? (~0ull) / width + 1 : 0ull;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
static bool aligned4(const void* p) { return ((uintptr_t)p & 3u) == 0; }

sinet_status launch_pass(const PassParams& p, uint32_t mode, hipStream_t s) {
    if (p.n == 0) return SINET_OK;
    const bool hist = (mode & PASS_HIST) != 0;
    uint32_t kind = (mode & PASS_LABEL_IN) ? (uint32_t)KK_LABEL_IN : p.t.kind;
    bool vec = true;
    if (p.pos_out) {
        vec = aligned16(p.src) && aligned16(p.pos_out);
    } else {
        if (kind == KK_LABEL_IN) vec = vec && aligned4(p.label_in);
        else vec = vec && aligned16(p.src) && aligned16(p.dst);
        if (p.label_out) vec = vec && aligned4(p.label_out);
        if (p.src_inst) vec = vec && aligned16(p.src_inst);
        if (p.dst_inst) vec = vec && aligned16(p.dst_inst);
        if (hist) vec = vec && aligned16(p.ts) && aligned16(p.bytes);
    }
    KernelFn fn = pick(kind, hist, vec);
    if (!fn) return fail(SINET_ERR_UNSUPPORTED, "no kernel for this lookup kind");
    const size_t lds = kind == KK_LABEL_IN ? 0 : p.t.lds_bytes;
    const int block = lds > 40 * 1024 ? 1024 : 256;
    if (lds > 160 * 1024) return fail(SINET_ERR_UNSUPPORTED, "table needs more LDS than a CU has");
    const uint64_t tiles = ((p.n + 3) / 4 + block - 1) / block;
    uint64_t grid = (uint64_t)device_cu_count() * blocks_per_cu(fn, block, lds);
    if (grid > tiles) grid = tiles;
    if (grid < 1) grid = 1;
    if (lds > 64 * 1024) (void)hipFuncSetAttribute((const void*)fn,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), lds, s, p);
    return check_hip(hipGetLastError(), "pass kernel launch");
}

sinet_status launch_zero(unsigned long long* p, uint64_t n_words, hipStream_t s) {
    if (n_words == 0) return SINET_OK;
    uint64_t blocks = (n_words / 2 + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n_words);
    return check_hip(hipGetLastError(), "zero kernel launch");
}

}  // namespace sinet
