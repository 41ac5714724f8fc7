// libsinet kernels: per-session discrimination fused with the millisecond
// histogram, for gfx950.
//
// Method (Ando et al., arXiv 2106.12863):
//   * Algorithm 1: an address is inside a CIDR block when
//     bitmask(addr, Z) - bitmask(base, Z) == 0; applied to both endpoints of a
//     session against the whole table, it yields the label
//     in(src) | in(dst) << 1.
//   * Sections "Map" / "Reduce" / "Merge Scatter Pattern": every session maps
//     to key (label, floor((ts - t0) / width)) with value (1, bytes); values
//     merge by unsigned 64-bit addition, associative and commutative, so the
//     order of accumulation is free and the result is exact.
//
// GPU design (what differs from the paper's Thrust transform + pairwise
// reduction + CPU merge):
//   * stage 1 (k_stage1): each lane owns 4 consecutive sessions, read with
//     128-bit loads per column (two for the 64-bit byte column) one chunk
//     ahead; it classifies them against the table staged in LDS, writes the
//     4 labels as one 32-bit store, and counting-sorts the chunk by 1,024-bin
//     block into 4-byte records;
//   * stage 2 (k_stage2): persistent workgroups reduce one block's records in
//     LDS and write every bin of the block once; no zero-fill and no global
//     atomics on the hot path; sessions outside a chunk's block window take
//     a far pass with device-scope atomics, so any input order stays exact;
//   * lookups that walk global memory (trie, learned windows, binary search
//     with a global leaf) run as their own pass that stores the labels first;
//   * the batched form runs the same stages over many streams from device
//     work queues, captured in one graph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string.h>

#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "inout_index.h"
#include "pass_common.h"
#include "sinet_device.h"
#include "sinet_internal.h"

namespace sinet {

enum KernelKind : uint32_t {
    KK_SCAN = SINET_LOOKUP_SCAN,
    KK_BSEARCH = SINET_LOOKUP_BSEARCH,
    KK_TRIE = SINET_LOOKUP_TRIE,
    KK_PLA = SINET_LOOKUP_LEARNED_PLA,
    KK_MLP = SINET_LOOKUP_LEARNED_MLP,
    KK_INOUT = kInoutKind,  // label-only lookups through the in/out index
    KK_LABEL_IN = 100       // histogram of given labels
};
static_assert(KK_LABEL_IN == kLabelInKind && KK_INOUT == kInoutKind, "internal kinds");

constexpr int kXcds = 8;
constexpr int kMaxBlock = 1024;
constexpr int kStage2Block = 512;
constexpr int kSegMax = 256;               // segment descriptors of a block held in LDS
constexpr int kRecUnroll = 8;              // independent record loads per stage-2 lane
constexpr uint32_t kStage2Run = 16;         // consecutive stage-2 blocks per XCD turn (rows off a line)
constexpr uint32_t kSmallMax = 1u << 19;  // byte counts stored inline in a record
constexpr uint64_t kMaxPiece = 1ull << 31;  // sessions per partitioned pass (32-bit slots)

// ---------------------------------------------------------------------------
// searches
//
// A lane looks up several addresses at once (its four sessions' sources and
// destinations).  Every search below advances all of them in lockstep, one
// probe level at a time, so a lane keeps that many independent LDS or global
// loads in flight instead of waiting out one dependent chain per address.
// ---------------------------------------------------------------------------

// Per-workgroup LDS view of the table.
struct LdsView {
    const uint32_t* io;      // in/out index
    const uint32_t* filter;  // 2-bit state of every /16 block (interval kinds)
    const uint32_t* top;     // BSEARCH
    const uint32_t* member;  // all interval kinds (or global)
    const uint32_t* cb;      // SCAN
    const uint32_t* mask;
    const uint32_t* len;
    const uint32_t* knot;    // PLA
    const float* c;
    const float* g;
    const uint32_t* radix;   // PLA: first segment of each radix bucket (u16 pairs)
    const float* w;          // MLP
    uint32_t* queue;         // lookup pass of the interval kinds: this wave's search queue
};

// Entries of a wave's search queue: the searches of the 8 address slots (4
// sessions) of the wave's 64 lanes.
constexpr uint32_t kSearchQueue = 512;

// The window PLA queues the searches of two address slots at a time (128
// entries per wave: the PLA's tables leave little LDS beside them).
constexpr int kPlaGroup = 2;
constexpr uint32_t kPlaQueue = 64u * kPlaGroup;

// Kinds whose lookup pass queues its searches: the binary searches, the trie,
// the MLP and the PLA.  The window PLA reads each queued window with a quad of
// lanes; the kinds whose search ends in a leaf of B in global memory (the
// LDS-sampled binary search, the MLP, a PLA with a wider bound) read each
// queued leaf with a quad of lanes, one round trip instead of a dependent
// binary search (on the 1.6e9-session day: sampled binary search 18.9 -> 11.2
// ms, MLP 23.2 -> 14.4 ms, 256-segment PLA 24.4 -> 13.2 ms; the same PLA queued
// with its leaf binary searches was slower than unqueued, 24.3 -> 37.5 ms).
__host__ __device__ constexpr bool queued_kind(uint32_t kind) {
    return kind == KK_BSEARCH || kind == KK_TRIE || kind == KK_MLP || kind == KK_PLA;
}

// Which queued searches a lookup instantiates (a template flag set): the
// window PLA's, the others' (binary searches, trie, MLP, wider PLA), or both.
constexpr int kQueueWindow = 1;
constexpr int kQueueSearch = 2;
constexpr int kQueueAll = kQueueWindow | kQueueSearch;

// Orders this wave's LDS accesses: the ones before complete before the ones
// after are issued (a wave's LDS requests are served in order; the clobber
// keeps the compiler from moving accesses across).
__device__ __forceinline__ void lds_wave_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// For each q: the last arr[i] <= a[q] among arr[0..n), given arr[0] <= a[q].
template <int N>
__device__ __forceinline__ void upper_last_n(const uint32_t* arr, uint32_t n, const uint32_t* a,
                                             uint32_t* lo) {
#pragma unroll
    for (int q = 0; q < N; ++q) lo[q] = 0;
    while (n > 1) {
        const uint32_t half = n >> 1;
#pragma unroll
        for (int q = 0; q < N; ++q) lo[q] = (arr[lo[q] + half] <= a[q]) ? lo[q] + half : lo[q];
        n -= half;
    }
}

__device__ __forceinline__ uint32_t radix_entry(const uint32_t* radix, uint32_t i) {
    return (radix[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu;
}

// Leaf phase shared by the binary search and the learned kinds: j[q] holds a
// leaf-block index (an index into the sampled boundaries); the leaf's
// 2^top_log2 boundaries (one or two cache lines, padded with 0xFFFFFFFF) are
// searched in global memory.
template <int N>
__device__ __forceinline__ void leaf_search(const DevTable& t, const uint32_t* a, uint32_t* j,
                                            uint32_t need) {
    if (t.top_log2 == 0) return;
#pragma unroll
    for (int q = 0; q < N; ++q) j[q] <<= t.top_log2;
    uint32_t n = 1u << t.top_log2;
    while (n > 1) {
        const uint32_t half = n >> 1;
#pragma unroll
        for (int q = 0; q < N; ++q)
            if ((need >> q) & 1u) j[q] = (t.B[j[q] + half] <= a[q]) ? j[q] + half : j[q];
        n -= half;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) j[q] = min(j[q], t.m - 1);
}

// Learned forms: the model's rounded prediction p is within max_err = e of
// the true interval j for every boundary key.  The leaf blocks that
// [p - e, p + e] can touch are searched in the LDS copy of the sampled
// boundaries (a window of uniform length, shifted inside the array) and the
// bracket top[b] <= a < top[b + 1] is confirmed, giving the leaf block b; the
// leaf is then searched as in the plain binary search.  A failed bracket (a
// wrong model or bound) falls back to the full search over the sample and is
// counted, so results stay exact.
template <int N>
__device__ __forceinline__ void learned_top_n(const DevTable& t, const LdsView& v,
                                              const uint32_t* a, const int* p, uint32_t* j,
                                              uint32_t need) {
    const uint32_t L = t.top_log2;
    const uint32_t nbl = min(((2 * t.max_err) >> L) + 2, t.n_top);
    uint32_t b[N], first[N];
    bool ok[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const int lo = max(p[q] - (int)t.max_err, 0);
        uint32_t b0 = (uint32_t)lo >> L;
        b0 = min(b0, t.n_top - nbl);
        first[q] = b0;
        b[q] = b0;
        ok[q] = v.top[b0] <= a[q];
    }
    uint32_t n = nbl;
    while (n > 1) {
        const uint32_t half = n >> 1;
#pragma unroll
        for (int q = 0; q < N; ++q) b[q] = (v.top[b[q] + half] <= a[q]) ? b[q] + half : b[q];
        n -= half;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        if (!((need >> q) & 1u)) continue;
        const uint32_t last = first[q] + nbl - 1;
        if (ok[q] && b[q] == last && last + 1 < t.n_top && v.top[last + 1] <= a[q]) ok[q] = false;
        if (!ok[q]) {
            atomicAdd(t.fallbacks, 1ull);
            b[q] = upper_last(v.top, t.n_top, a[q]);
        }
        j[q] = b[q];
    }
}

// The learned search: leaf block from the LDS sample, then the leaf.
template <int N>
__device__ __forceinline__ void learned_search_n(const DevTable& t, const LdsView& v,
                                                 const uint32_t* a, const int* p, uint32_t* j,
                                                 uint32_t need) {
    learned_top_n<N>(t, v, a, p, j, need);
    leaf_search<N>(t, a, j, need);
}

// PLA window search (max_err = e <= kPlaWindowErr): the interval of a lies
// within e of the rounded prediction p, so the 16 boundaries from
// s = (p - e) rounded down to a multiple of 4 hold it.  They are read with
// four aligned 16-byte loads, and B[s + 16] with them (two addresses'
// windows in flight at once), and j = s + (the number of them <= a) - 1.  A
// count of 0, or of 16 with B[s + 16] <= a, means the bound was wrong: the
// full search answers, counted.
template <int N>
__device__ __forceinline__ void window_search_n(const DevTable& t, const uint32_t* a, const int* p,
                                                uint32_t* j, uint32_t need) {
    constexpr int G = N < 2 ? N : 2;
    const int e = (int)t.max_err;
#pragma unroll
    for (int q0 = 0; q0 < N; q0 += G) {
        uint4 w[G][4];
        uint32_t s[G], nx[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            s[q] = (uint32_t)max(p[q0 + q] - e, 0) & ~3u;
            if ((need >> (q0 + q)) & 1u) {
                const uint4* b4 = reinterpret_cast<const uint4*>(t.B + s[q]);
#pragma unroll
                for (int v = 0; v < 4; ++v) w[q][v] = b4[v];
                nx[q] = t.B[s[q] + 16u];  // for the bracket check (in the padding at worst)
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) w[q][v] = make_uint4(0u, 0u, 0u, 0u);
                nx[q] = 0xFFFFFFFFu;
            }
        }
#pragma unroll
        for (int q = 0; q < G; ++q) {
            const int qq = q0 + q;
            if (!((need >> qq) & 1u)) continue;
            const uint32_t x = a[qq];
            uint32_t c = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                c += (uint32_t)(w[q][v].x <= x) + (uint32_t)(w[q][v].y <= x) +
                     (uint32_t)(w[q][v].z <= x) + (uint32_t)(w[q][v].w <= x);
            bool ok = c >= 1u;
            if (c == 16u && s[q] + 16u < t.m) ok = x < nx[q];
            uint32_t r = s[q] + c - 1u;
            if (!ok) {
                atomicAdd(t.fallbacks, 1ull);
                r = upper_last(t.B, t.m, x);
            }
            j[qq] = min(r, t.m - 1);
        }
    }
}

// Lane index within the wave.
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Rank of this lane among the lanes set in m.
__device__ __forceinline__ uint32_t rank_in(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// x of lane src (every lane active).
__device__ __forceinline__ uint32_t from_lane(uint32_t src, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)x);
}

// Sum over the four lanes of each quad, in every lane of the quad (DPP quad
// permutations [1,0,3,2] then [2,3,0,1]; every lane active).
__device__ __forceinline__ uint32_t quad_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
    return x;
}

// Membership bits of the addresses in cut /16 blocks by the window PLA, for a
// wave whose 64 lanes are all active.  Unqueued, each address reads its
// 16-boundary window with four 16-byte loads of its own lane, in waves where
// about a third of the lanes need a search, so a wave pays every slot's
// segment search, window loads and compares whichever of its lanes need them.
// Here the addresses that need one, two slots at a time, are ranked with a
// ballot and mbcnt and queued in LDS; each round gives one queued address to
// every lane, which finds its segment, evaluates the line and forms the
// window's first index; then each quad of lanes takes one
// address per step (its address and window start moved over with
// ds_bpermute), each lane loads and compares four of the 16 boundaries, and
// the quad's counts are added with DPP.  One load instruction covers 16
// windows.  The lane at place k of a quad then finishes the quad's address of
// step k: it checks the bracket (falling back to the full search, counted, as
// window_search_n does), reads the interval's membership bit and writes it
// over the queue entry, from which the address's lane reads it back.
template <int N>
__device__ __forceinline__ void pla_window_queued(const DevTable& t, const LdsView& v,
                                                  const uint32_t* a, uint32_t need, uint32_t* in) {
    const uint32_t lane = lane_id();
    const int e = (int)t.max_err;
#pragma unroll
    for (int q0 = 0; q0 < N; q0 += kPlaGroup) {
        uint32_t slot[kPlaGroup], cnt = 0;
#pragma unroll
        for (int k = 0; k < kPlaGroup; ++k) {
            const bool nd = (need >> (q0 + k)) & 1u;
            const unsigned long long m = __ballot(nd);
            slot[k] = cnt + rank_in(m);
            if (nd) v.queue[slot[k]] = a[q0 + k];
            cnt += (uint32_t)__popcll(m);
        }
        if (cnt == 0) continue;  // wave-uniform
        lds_wave_sync();
        for (uint32_t r = 0; r < cnt; r += 64) {
            const uint32_t nr = min(cnt - r, 64u);  // entries this round (wave-uniform)
            const bool mine = lane < nr;
            const uint32_t x = mine ? v.queue[r + lane] : 0u;
            uint32_t wb = 0;
            if (mine) {
                // radix bucket -> candidate segments -> last knot <= x -> line
                const uint32_t rb = x >> (32 - t.radix_bits);
                const uint32_t s0 = radix_entry(v.radix, rb), s1 = radix_entry(v.radix, rb + 1);
                const uint32_t sg = s0 + upper_last(v.knot + s0, s1 - s0 + 1, x);
                const int pp = clamp_pos(pla_eval(v.knot[sg], v.c[sg], v.g[sg], x), t.m);
                wb = (uint32_t)max(pp - e, 0) & ~3u;
            }
            // the round's steps of 16 addresses (at most four; a step past the
            // round's entries is skipped, wave-uniformly): every window load,
            // and the boundary after each window for the bracket check, is
            // issued before any is used
            const uint32_t me = lane & 3u;
            uint32_t xx[4], bb[4], c[4], nx = 0xFFFFFFFFu;
            uint4 w[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                xx[k] = 0u;
                bb[k] = 0u;
                if (16u * k < nr) {
                    const uint32_t src = 16u * k + (lane >> 2);
                    xx[k] = from_lane(src, x);
                    bb[k] = from_lane(src, wb);
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                w[k] = make_uint4(0u, 0u, 0u, 0u);
                if (16u * k + (lane >> 2) < nr) {  // quad-uniform
                    w[k] = *reinterpret_cast<const uint4*>(t.B + bb[k] + 4u * me);
                    if (me == (uint32_t)k) nx = t.B[bb[k] + 16u];  // in the padding at worst
                }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                c[k] = 0u;
                if (16u * k < nr)
                    c[k] = quad_sum((uint32_t)(w[k].x <= xx[k]) + (uint32_t)(w[k].y <= xx[k]) +
                                    (uint32_t)(w[k].z <= xx[k]) + (uint32_t)(w[k].w <= xx[k]));
            }
            // each lane finishes the step of its place in the quad: the bracket
            // check, the interval's membership bit over the queue entry
            const uint32_t cm = me == 0u ? c[0] : me == 1u ? c[1] : me == 2u ? c[2] : c[3];
            const uint32_t xm = me == 0u ? xx[0] : me == 1u ? xx[1] : me == 2u ? xx[2] : xx[3];
            const uint32_t bm = me == 0u ? bb[0] : me == 1u ? bb[1] : me == 2u ? bb[2] : bb[3];
            const uint32_t src = 16u * me + (lane >> 2);
            if (src < nr) {
                bool ok = cm >= 1u;
                if (cm == 16u && bm + 16u < t.m) ok = xm < nx;
                uint32_t j = bm + cm - 1u;
                if (!ok) {
                    atomicAdd(t.fallbacks, 1ull);
                    j = upper_last(t.B, t.m, xm);
                }
                j = min(j, t.m - 1);
                v.queue[r + src] = (v.member[j >> 5] >> (j & 31)) & 1u;
            }
        }
        lds_wave_sync();
#pragma unroll
        for (int k = 0; k < kPlaGroup; ++k)
            if ((need >> (q0 + k)) & 1u) in[q0 + k] = v.queue[slot[k]];
        lds_wave_sync();  // read back before the queue is written again
    }
}

// Leaf block of each address (the binary search over the LDS sample, or the
// learned model and its bracket), for the kinds whose search ends in a leaf of
// B in global memory.
template <uint32_t KIND, int N>
__device__ __forceinline__ void leaf_blocks(const DevTable& t, const LdsView& v, const uint32_t* a,
                                            uint32_t* b, uint32_t need) {
    if constexpr (KIND == KK_BSEARCH) {
        upper_last_n<N>(v.top, t.n_top, a, b);
    } else if constexpr (KIND == KK_MLP) {
        int p[N];
#pragma unroll
        for (int q = 0; q < N; ++q)
            p[q] = (need >> q) & 1u ? clamp_pos(mlp_predict(v.w, t.m_f, a[q]), t.m) : 0;
        learned_top_n<N>(t, v, a, p, b, need);
    } else if constexpr (KIND == KK_PLA) {  // a PLA whose bound is too wide for one window
        int p[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            p[q] = 0;
            if (!((need >> q) & 1u)) continue;
            const uint32_t r = a[q] >> (32 - t.radix_bits);
            const uint32_t s0 = radix_entry(v.radix, r), s1 = radix_entry(v.radix, r + 1);
            const uint32_t sg = s0 + upper_last(v.knot + s0, s1 - s0 + 1, a[q]);
            p[q] = clamp_pos(pla_eval(v.knot[sg], v.c[sg], v.g[sg], a[q]), t.m);
        }
        learned_top_n<N>(t, v, a, p, b, need);
    }
}

// Leaves read by quads of lanes: a wave whose 64 lanes are all active holds up
// to 128 queued addresses x[h] (entry r + 64 h + lane) with their leaf blocks
// b[h].  For each half, four steps of 16 addresses: a quad takes one address
// per step (moved over with ds_bpermute), each of its lanes loads NL 16-byte
// groups of the leaf's 16 NL boundaries and counts those <= the address, and
// the quad adds its counts with DPP; every load of a half is issued before any
// is used.  The interval is the leaf's first index plus the count minus one
// (the leaf's first boundary is <= the address, as the sample said), exactly
// what the leaf's binary search finds.  The lane at place k of a quad then
// writes the membership bit of its quad's address of step k over the entry.
template <int NL>
__device__ __forceinline__ void leaf_quads(const DevTable& t, const LdsView& v, const uint32_t* x,
                                           const uint32_t* b, uint32_t r, uint32_t nr,
                                           uint32_t lane) {
    const uint32_t me = lane & 3u, L = t.top_log2;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (64u * h >= nr) break;  // wave-uniform
        const uint32_t nh = min(nr - 64u * h, 64u);  // entries of this half
        uint32_t xx[4], bb[4], c[4];
        uint4 w[4][NL];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            xx[k] = 0u;
            bb[k] = 0u;
            if (16u * k < nh) {
                const uint32_t src = 16u * k + (lane >> 2);
                xx[k] = from_lane(src, x[h]);
                bb[k] = from_lane(src, b[h]);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int u = 0; u < NL; ++u) w[k][u] = make_uint4(0u, 0u, 0u, 0u);
            if (16u * k + (lane >> 2) < nh) {  // quad-uniform
                const uint4* leaf = reinterpret_cast<const uint4*>(t.B + (bb[k] << L));
#pragma unroll
                for (int u = 0; u < NL; ++u) w[k][u] = leaf[4 * u + me];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c[k] = 0u;
            if (16u * k < nh) {
                uint32_t n = 0;
#pragma unroll
                for (int u = 0; u < NL; ++u)
                    n += (uint32_t)(w[k][u].x <= xx[k]) + (uint32_t)(w[k][u].y <= xx[k]) +
                         (uint32_t)(w[k][u].z <= xx[k]) + (uint32_t)(w[k][u].w <= xx[k]);
                c[k] = quad_sum(n);
            }
        }
        const uint32_t cm = me == 0u ? c[0] : me == 1u ? c[1] : me == 2u ? c[2] : c[3];
        const uint32_t bm = me == 0u ? bb[0] : me == 1u ? bb[1] : me == 2u ? bb[2] : bb[3];
        const uint32_t src = 16u * me + (lane >> 2);
        if (src < nh) {
            const uint32_t j = min((bm << L) + cm - 1u, t.m - 1);
            v.queue[r + 64u * h + src] = (v.member[j >> 5] >> (j & 31)) & 1u;
        }
    }
}

// Interval index of each address (all kinds but SCAN).  Addresses whose bit
// in `need` is clear are skipped (their j is left unspecified); skipped lanes
// issue no memory requests.
template <uint32_t KIND, int N>
__device__ __forceinline__ void intervals(const DevTable& t, const LdsView& v, const uint32_t* a,
                                          uint32_t* j, uint32_t need = 0xFFFFFFFFu) {
    if constexpr (KIND == KK_BSEARCH) {
        upper_last_n<N>(v.top, t.n_top, a, j);
        leaf_search<N>(t, a, j, need);
    } else if constexpr (KIND == KK_TRIE) {
        uint32_t e[N];
#pragma unroll
        for (int q = 0; q < N; ++q) e[q] = (need >> q) & 1u ? t.trie[a[q] >> 16] : 0x80000000u;
#pragma unroll
        for (int q = 0; q < N; ++q)
            if (!(e[q] >> 31)) e[q] = t.trie[65536u + e[q] * 256u + ((a[q] >> 8) & 255u)];
#pragma unroll
        for (int q = 0; q < N; ++q)
            if (!(e[q] >> 31)) e[q] = t.trie[65536u + e[q] * 256u + (a[q] & 255u)];
#pragma unroll
        for (int q = 0; q < N; ++q) j[q] = e[q] & 0x7FFFFFFFu;
    } else if constexpr (KIND == KK_PLA) {
        int p[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            p[q] = 0;
            if (!((need >> q) & 1u)) continue;
            // radix bucket -> candidate segments -> last knot <= a
            const uint32_t r = a[q] >> (32 - t.radix_bits);
            const uint32_t s0 = radix_entry(v.radix, r), s1 = radix_entry(v.radix, r + 1);
            const uint32_t s = s0 + upper_last(v.knot + s0, s1 - s0 + 1, a[q]);
            p[q] = clamp_pos(pla_eval(v.knot[s], v.c[s], v.g[s], a[q]), t.m);
        }
        if (t.pla_window) window_search_n<N>(t, a, p, j, need);
        else learned_search_n<N>(t, v, a, p, j, need);
    } else {  // KK_MLP
        int p[N];
#pragma unroll
        for (int q = 0; q < N; ++q)
            p[q] = (need >> q) & 1u ? clamp_pos(mlp_predict(v.w, t.m_f, a[q]), t.m) : 0;
        learned_search_n<N>(t, v, a, p, j, need);
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

// In/out mark (and, when want_code, the owner code row + 1 or 0) of each
// address.  Label-only lookups first consult the /16 filter: a block that no
// boundary cuts is entirely in or entirely out, which answers most addresses
// from LDS; only addresses in cut blocks run the table's search.
template <uint32_t KIND, int N, int QUEUE = 0>
__device__ __forceinline__ void lookups(const DevTable& t, const LdsView& v, const uint32_t* a,
                                        bool want_code, uint32_t* in, uint32_t* code) {
    if constexpr (KIND == KK_INOUT) {
        inout_lookup<N>(v.io, t.io_slot, t.io_list, a, in);
#pragma unroll
        for (int q = 0; q < N; ++q) code[q] = 0;
    } else if constexpr (KIND == KK_SCAN) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
            code[q] = scan_owner(t, v, a[q]);
            in[q] = code[q] != 0;
        }
    } else {
        uint32_t need = 0xFFFFFFFFu;
        uint32_t st[N];
        if (!want_code && t.filter_lds) {
            need = 0;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                st[q] = (v.filter[a[q] >> 20] >> (((a[q] >> 16) & 15u) * 2)) & 3u;
                need |= (st[q] == 2u ? 1u : 0u) << q;
            }
        }
        if constexpr ((QUEUE & kQueueWindow) && KIND == KK_PLA) {
            if (v.queue && !want_code && t.filter_lds && t.pla_window && __ballot(1) == ~0ull) {
                pla_window_queued<N>(t, v, a, need, in);
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    if (st[q] < 2u) in[q] = st[q];
                    code[q] = 0;
                }
                return;
            }
        }
        if constexpr ((QUEUE & kQueueSearch) != 0) {
            if (v.queue && !want_code && t.filter_lds && (KIND != KK_PLA || !t.pla_window)) {
                // Wave-level compaction of the searches (section "Coordinated Batch
                // Processing": the chunk is discriminated before the Map stage).  Only
                // addresses in cut /16 blocks need one, about a third of them, yet a
                // wave runs a slot's search whenever any of its lanes needs it.  The
                // addresses that need one are ranked with a ballot and mbcnt per slot,
                // queued in LDS, searched two per active lane per round (dense), and
                // their membership bits read back from their queue entries.  Lanes may
                // be inactive (the ragged last tile, the tail), so the active lanes are
                // ranked among themselves.
                const unsigned long long live = __ballot(1);
                const uint32_t me = rank_in(live);
                const uint32_t n_live = (uint32_t)__popcll(live);
                uint32_t slot[N], cnt = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    const bool nd = (need >> q) & 1u;
                    const unsigned long long m = __ballot(nd);
                    slot[q] = cnt + rank_in(m);
                    if (nd) v.queue[slot[q]] = a[q];
                    cnt += (uint32_t)__popcll(m);
                }
                if (cnt) {  // wave-uniform
                    lds_wave_sync();
                    // leaves of 16 or 32 boundaries in global memory, read by quads
                    // of lanes when the whole wave is active
                    const bool quads = KIND != KK_TRIE && n_live == 64u && t.n_top > 1 &&
                                       (t.top_log2 == 4 || t.top_log2 == 5);
                    if (quads) {
                        for (uint32_t r = 0; r < cnt; r += 128) {
                            const uint32_t nr = min(cnt - r, 128u);  // wave-uniform
                            uint32_t x[2] = {me < nr ? v.queue[r + me] : 0u,
                                             me + 64u < nr ? v.queue[r + 64u + me] : 0u};
                            uint32_t b[2] = {0u, 0u};
                            leaf_blocks<KIND, 2>(t, v, x, b,
                                                 (me < nr ? 1u : 0u) | (me + 64u < nr ? 2u : 0u));
                            if (t.top_log2 == 4) leaf_quads<1>(t, v, x, b, r, nr, me);
                            else leaf_quads<2>(t, v, x, b, r, nr, me);
                        }
                    }
                    for (uint32_t r = quads ? cnt : 0u; r < cnt; r += 2 * n_live) {
                        const uint32_t e0 = r + me, e1 = r + n_live + me;
                        uint32_t x[2] = {e0 < cnt ? v.queue[e0] : 0u, e1 < cnt ? v.queue[e1] : 0u};
                        uint32_t j[2] = {0u, 0u};
                        intervals<KIND, 2>(t, v, x, j, (e0 < cnt ? 1u : 0u) | (e1 < cnt ? 2u : 0u));
                        if (e0 < cnt) v.queue[e0] = (v.member[j[0] >> 5] >> (j[0] & 31)) & 1u;
                        if (e1 < cnt) v.queue[e1] = (v.member[j[1] >> 5] >> (j[1] & 31)) & 1u;
                    }
                    lds_wave_sync();
#pragma unroll
                    for (int q = 0; q < N; ++q)
                        if ((need >> q) & 1u) in[q] = v.queue[slot[q]];
                    lds_wave_sync();  // read back before the queue is written again
                }
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    if (st[q] < 2u) in[q] = st[q];
                    code[q] = 0;
                }
                return;
            }
        }
        if (need) {
            uint32_t j[N];
            intervals<KIND, N>(t, v, a, j, need);
#pragma unroll
            for (int q = 0; q < N; ++q) {
                if (!((need >> q) & 1u)) continue;
                in[q] = (v.member[j[q] >> 5] >> (j[q] & 31)) & 1u;
                code[q] = want_code ? t.owner[j[q]] : 0u;
            }
        }
        if (!want_code && t.filter_lds) {
#pragma unroll
            for (int q = 0; q < N; ++q) {
                if (st[q] < 2u) in[q] = st[q];
                code[q] = 0;
            }
        }
    }
}

enum HistMode : int {
    H_NONE = 0,     // labels / institutions / positions only
    H_ATOMIC = 1,   // device-scope atomics into the output bins
    H_PRIVATE = 2   // whole histogram privatised in LDS per workgroup
};

// LDS histogram of the private mode: counts u32 [4][n_bins], bytes u64 [4][n_bins].
struct PrivHist {
    uint32_t* c;
    unsigned long long* b;
};

template <int HM>
__device__ __forceinline__ void account(const PassParams& p, const PrivHist& h, uint32_t lab,
                                        uint32_t ts, uint64_t nbytes, Dropped& d) {
    if constexpr (HM == H_NONE) return;
    uint32_t b;
    if (!in_window(p, ts, b)) {
        d.add(lab, nbytes);
        return;
    }
    const uint64_t k = (uint64_t)lab * p.n_bins + b;
    if constexpr (HM == H_ATOMIC) {
        __hip_atomic_fetch_add(p.count + k, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(p.hbytes + k, (unsigned long long)nbytes, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    } else {
        atomicAdd(h.c + k, 1u);
        atomicAdd(h.b + k, (unsigned long long)nbytes);
    }
}

// 16 bytes read once (the columns of a lookup pass): nontemporal loads.  On
// the 1.6e9-session day the in/out lookup pass took 3.08-3.10 ms with plain
// loads and stores and 2.98-2.99 ms with nontemporal loads of src and dst and
// nontemporal label stores (the stores alone: 3.06-3.07 ms).
__device__ __forceinline__ uint4 gload4_nt(const uint32_t* q) {  // q 16-byte aligned
    const u32x4_t v = __builtin_nontemporal_load(glob(reinterpret_cast<const u32x4_t*>(q)));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Label of session i (scalar path); stores label / institutions when asked.
template <uint32_t KIND, int QUEUE = 0>
__device__ __forceinline__ uint32_t label1(const PassParams& p, const LdsView& v, uint64_t i) {
    const uint32_t a[2] = {*glob(p.src + i), *glob(p.dst + i)};
    const bool wc = p.src_inst != nullptr || p.dst_inst != nullptr;
    uint32_t in[2], code[2];
    lookups<KIND, 2, QUEUE>(p.t, v, a, wc, in, code);
    const uint32_t lab = in[0] | (in[1] << 1);
    if (p.label_out) *glob(p.label_out + i) = (uint8_t)lab;
    if (p.src_inst) *glob(p.src_inst + i) = code[0] ? p.t.inst[code[0] - 1] : SINET_NO_INST;
    if (p.dst_inst) *glob(p.dst_inst + i) = code[1] ? p.t.inst[code[1] - 1] : SINET_NO_INST;
    return lab;
}

template <uint32_t KIND, int HM>
__device__ __forceinline__ void one_session(const PassParams& p, const LdsView& v,
                                            const PrivHist& h, uint64_t i, Dropped& d) {
    if (p.pos_out) {
        if constexpr (KIND != KK_SCAN && KIND != KK_LABEL_IN && KIND != KK_INOUT) {
            const uint32_t a = p.src[i];
            uint32_t j;
            intervals<KIND, 1>(p.t, v, &a, &j);
            p.pos_out[i] = j;
        }
        return;
    }
    uint32_t lab;
    if constexpr (KIND == KK_LABEL_IN) {
        lab = *glob(p.label_in + i) & 3u;
    } else {
        lab = label1<KIND, HM == H_NONE && queued_kind(KIND) ? kQueueAll : 0>(p, v, i);
    }
    if constexpr (HM != H_NONE) account<HM>(p, h, lab, *glob(p.ts + i), *glob(p.bytes + i), d);
}

// Labels of four consecutive sessions starting at i from their loaded source
// and destination words (or the given labels); stores labels / institutions
// when asked.
template <uint32_t KIND, int QUEUE = 0>
__device__ __forceinline__ void labels4_from(const PassParams& p, const LdsView& v, uint64_t i,
                                             uint4 s, uint4 t, uint32_t l4, uint32_t lab[4]) {
    if constexpr (KIND == KK_LABEL_IN) {
#pragma unroll
        for (int k = 0; k < 4; ++k) lab[k] = (l4 >> (8 * k)) & 3u;
    } else {
        // sources and destinations of the four sessions, looked up together
        const uint32_t a[8] = {s.x, s.y, s.z, s.w, t.x, t.y, t.z, t.w};
        const bool wc = p.src_inst != nullptr || p.dst_inst != nullptr;
        uint32_t in[8], code[8];
        lookups<KIND, 8, QUEUE>(p.t, v, a, wc, in, code);
        uint32_t sc[4], dc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lab[k] = in[k] | (in[4 + k] << 1);
            sc[k] = code[k];
            dc[k] = code[4 + k];
        }
        if (p.label_out) {
            const uint32_t packed = lab[0] | (lab[1] << 8) | (lab[2] << 16) | (lab[3] << 24);
            __builtin_nontemporal_store(packed, glob(reinterpret_cast<uint32_t*>(p.label_out + i)));
        }
        if (p.src_inst) {
            uint4 o;
            o.x = sc[0] ? p.t.inst[sc[0] - 1] : SINET_NO_INST;
            o.y = sc[1] ? p.t.inst[sc[1] - 1] : SINET_NO_INST;
            o.z = sc[2] ? p.t.inst[sc[2] - 1] : SINET_NO_INST;
            o.w = sc[3] ? p.t.inst[sc[3] - 1] : SINET_NO_INST;
            gstore4(p.src_inst + i, o);
        }
        if (p.dst_inst) {
            uint4 o;
            o.x = dc[0] ? p.t.inst[dc[0] - 1] : SINET_NO_INST;
            o.y = dc[1] ? p.t.inst[dc[1] - 1] : SINET_NO_INST;
            o.z = dc[2] ? p.t.inst[dc[2] - 1] : SINET_NO_INST;
            o.w = dc[3] ? p.t.inst[dc[3] - 1] : SINET_NO_INST;
            gstore4(p.dst_inst + i, o);
        }
    }
}

template <uint32_t KIND, int QUEUE = 0>
__device__ __forceinline__ void labels4(const PassParams& p, const LdsView& v, uint64_t i,
                                        uint32_t lab[4]) {
    uint4 s = make_uint4(0, 0, 0, 0), t = s;
    uint32_t l4 = 0;
    if constexpr (KIND == KK_LABEL_IN) {
        l4 = *glob(reinterpret_cast<const uint32_t*>(p.label_in + i));
    } else {
        s = gload4(p.src + i);
        t = gload4(p.dst + i);
    }
    labels4_from<KIND, QUEUE>(p, v, i, s, t, l4, lab);
}

template <uint32_t KIND, int HM>
__device__ __forceinline__ void four_sessions(const PassParams& p, const LdsView& v,
                                              const PrivHist& h, uint64_t i, Dropped& d) {
    if (p.pos_out) {
        if constexpr (KIND != KK_SCAN && KIND != KK_LABEL_IN && KIND != KK_INOUT) {
            const uint4 a4 = *reinterpret_cast<const uint4*>(p.src + i);
            const uint32_t a[4] = {a4.x, a4.y, a4.z, a4.w};
            uint32_t j[4];
            intervals<KIND, 4>(p.t, v, a, j);
            *reinterpret_cast<uint4*>(p.pos_out + i) = make_uint4(j[0], j[1], j[2], j[3]);
        }
        return;
    }
    uint32_t lab[4];
    labels4<KIND, HM == H_NONE && queued_kind(KIND) ? kQueueAll : 0>(p, v, i, lab);
    if constexpr (HM != H_NONE) {
        const uint4 ts = gload4(p.ts + i);
        const ulonglong2 b01 = gload2(p.bytes + i);
        const ulonglong2 b23 = gload2(p.bytes + i + 2);
        account<HM>(p, h, lab[0], ts.x, b01.x, d);
        account<HM>(p, h, lab[1], ts.y, b01.y, d);
        account<HM>(p, h, lab[2], ts.z, b23.x, d);
        account<HM>(p, h, lab[3], ts.w, b23.y, d);
    }
}

// Stage the table's hot arrays into LDS (layout chosen on the host).
// Returns the view; *words receives the number of 32-bit words used.
template <uint32_t KIND>
__device__ __forceinline__ LdsView stage_lds(const DevTable& t, uint32_t* lds, uint32_t* words) {
    LdsView v{};
    uint32_t off = 0;
    auto copy = [&](const uint32_t* src, uint32_t n) -> const uint32_t* {
        uint32_t* dst = lds + off;
        for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) dst[k] = *glob(src + k);
        off += n;
        return dst;
    };
    if constexpr (KIND == KK_INOUT) {
        v.io = copy(t.io, t.io_words);
    } else if constexpr (KIND == KK_SCAN) {
        v.cb = copy(t.cb, t.n_prefix);
        v.mask = copy(t.mask, t.n_prefix);
        v.len = copy(t.len, t.n_prefix);
    } else if constexpr (KIND != KK_LABEL_IN) {
        v.filter = t.filter_lds ? copy(t.filter, kFilterWords) : t.filter;
        if constexpr (KIND == KK_BSEARCH || KIND == KK_MLP) v.top = copy(t.top, t.n_top);
        if constexpr (KIND == KK_PLA) v.top = t.pla_window ? nullptr : copy(t.top, t.n_top);
        if constexpr (KIND == KK_PLA) {
            v.knot = copy(t.knot, t.segments);
            v.c = reinterpret_cast<const float*>(
                copy(reinterpret_cast<const uint32_t*>(t.pla_c), t.segments));
            v.g = reinterpret_cast<const float*>(
                copy(reinterpret_cast<const uint32_t*>(t.pla_g), t.segments));
            v.radix = copy(t.radix, radix_words(t.radix_bits));
        }
        if constexpr (KIND == KK_MLP)
            v.w = reinterpret_cast<const float*>(
                copy(reinterpret_cast<const uint32_t*>(t.mlp), SINET_MLP_PARAMS));
        v.member = t.lds_member_words ? copy(t.member, t.lds_member_words) : t.member;
    }
    *words = off;
    __syncthreads();
    return v;
}

// ---------------------------------------------------------------------------
// k_pass: one pass over the sessions.
//   H_NONE    labels / institutions / positions;
//   H_PRIVATE the whole (small) histogram lives in LDS per workgroup and is
//             merged into the output bins with atomics at the end;
//   H_ATOMIC  with far.list: only the sessions the partitioned path flagged
//             as far (see k_stage1), merged with device-scope atomics after
//             the block reduction wrote the bins; without: every session.
// ---------------------------------------------------------------------------
template <uint32_t KIND, int HM, bool VEC>
__device__ __forceinline__ void pass_body(const PassParams& p, const FarList& far) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    uint32_t used = 0;
    LdsView v = stage_lds<KIND>(p.t, lds, &used);
    if constexpr (HM == H_NONE && queued_kind(KIND)) {
        if (p.queue_words) v.queue = lds + used + (threadIdx.x >> 6) * p.queue_words;
    }
    PrivHist h{nullptr, nullptr};
    if constexpr (HM == H_PRIVATE) {
        used = (used + 1) & ~1u;
        h.b = reinterpret_cast<unsigned long long*>(lds + used);
        h.c = lds + used + 2 * 4 * p.n_bins;
        for (uint32_t k = threadIdx.x; k < 4 * p.n_bins; k += blockDim.x) {
            h.b[k] = 0;
            h.c[k] = 0;
        }
        __syncthreads();
    }
    Dropped d{};
    if (HM == H_ATOMIC && far.list) {
        const uint32_t nfar = *far.count;
        for (uint32_t q = blockIdx.x; q < nfar; q += gridDim.x) {
            const uint64_t c = far.list[q];
            for (uint32_t s = threadIdx.x; s < kChunk; s += blockDim.x) {
                const uint64_t i = c * kChunk + s;
                if (i < p.n && ((far.bits[c * (kChunk / 32) + s / 32] >> (s & 31)) & 1u))
                    one_session<KIND, HM>(p, v, h, i, d);
            }
        }
    } else {
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
        if constexpr (HM == H_NONE && VEC && KIND != KK_LABEL_IN) {
            if (!p.pos_out) {
                // labels / institutions only: the next tile's addresses are
                // loaded before the current tile's lookups run
                auto full = [&](uint64_t tl) { return (tl * tile + threadIdx.x) * 4 + 4 <= p.n; };
                uint4 cs = make_uint4(0, 0, 0, 0), cd = cs, ns = cs, nd = cs;
                uint64_t tl = T0 + lid;
                if (tl < T1 && full(tl)) {
                    const uint64_t i = (tl * tile + threadIdx.x) * 4;
                    cs = gload4_nt(p.src + i);
                    cd = gload4_nt(p.dst + i);
                }
                for (; tl < T1; tl += nx) {
                    const uint64_t tn = tl + nx;
                    if (tn < T1 && full(tn)) {
                        const uint64_t i = (tn * tile + threadIdx.x) * 4;
                        ns = gload4_nt(p.src + i);
                        nd = gload4_nt(p.dst + i);
                    }
                    const uint64_t g = tl * tile + threadIdx.x;
                    if (full(tl)) {
                        uint32_t lab[4];
                        constexpr int kQ = HM == H_NONE && queued_kind(KIND) ? kQueueAll : 0;
                        labels4_from<KIND, kQ>(p, v, g * 4, cs, cd, 0u, lab);
                    } else if (g * 4 < p.n) {
                        for (uint64_t i = g * 4; i < p.n && i < g * 4 + 4; ++i)
                            one_session<KIND, HM>(p, v, h, i, d);
                    }
                    cs = ns;
                    cd = nd;
                }
                return;
            }
        }
        for (uint64_t tl = T0 + lid; tl < T1; tl += nx) {
            const uint64_t g = tl * tile + threadIdx.x;
            if (g >= groups) continue;
            if (VEC && g * 4 + 4 <= p.n) {
                four_sessions<KIND, HM>(p, v, h, g * 4, d);
            } else {
                for (uint64_t i = g * 4; i < p.n && i < g * 4 + 4; ++i)
                    one_session<KIND, HM>(p, v, h, i, d);
            }
        }
    }
    if constexpr (HM != H_NONE) d.flush(p.dropped);
    if constexpr (HM == H_PRIVATE) {
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < 4 * p.n_bins; k += blockDim.x) {
            if (h.c[k]) {
                __hip_atomic_fetch_add(p.count + k, (unsigned long long)h.c[k], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(p.hbytes + k, h.b[k], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

template <uint32_t KIND, int HM, bool VEC>
__global__ void __launch_bounds__(kMaxBlock) k_pass(PassParams p, FarList far) {
    pass_body<KIND, HM, VEC>(p, far);
}

// The label pass over the in/out index (the plain form's lookup): its 64 KB
// of LDS lets two 1024-lane workgroups share a CU once the kernel fits in 64
// VGPRs (eight waves per SIMD), twice the waves to hide the column loads.
__global__ void __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(8)))
k_pass_inout(PassParams p, FarList far) {
    pass_body<KK_INOUT, H_NONE, true>(p, far);
}

// ---------------------------------------------------------------------------
// Partitioned histogram: the two-stage map-reduce, both stages on the GPU.
//
// Stage 1 (k_stage1, fused with discrimination): a workgroup takes a chunk of
// kChunk consecutive sessions, labels them and maps each in-window session to
// (block = bin / kBlockBins, offset, label).  Sessions are counting-sorted in
// LDS by block relative to the chunk's first block (a window of kWin blocks)
// and written as 4-byte records, grouped by block, into the chunk's own slot
// range (every block's segment padded with null records to whole 16-byte
// groups); the chunk's directory lists (block, first slot, slots) for every
// block it touched.  Near time-sorted input (the paper's session logs)
// touches few blocks per chunk.
// Segment index: per-block directory counts, an exclusive scan, and a fill
// that groups the directory entries by block (k_fill).
// Stage 2 (k_stage2): persistent workgroups take blocks in turn, accumulate a
// block's segments' records in LDS and write the block's count and byte bins
// once, with coalesced stores, while the next block's segment list is in
// flight; no zero-fill and no global atomics.
// Far path: a session outside its chunk's block window, with bytes >= 2^52,
// or beyond the chunk's extra record slots is flagged and merged afterwards
// by k_pass<H_ATOMIC> with global atomics, so any input stays exact.
//
// Record (self-contained, so stage 2 needs no other read):
//   label (2 bits) | offset in block (10) | 0 | byte count (19)   if bytes < 2^19
//   label (2 bits) | offset in block (10) | 1 | part k (2) | bits 17k..17k+16
//                                              of the byte count  otherwise,
// one record per 17-bit part up to the highest nonzero one (2 to 4 records);
// part 0 carries the session's count.  0xFFFFFFFF is the null record (a part 3
// holds at most bit 51, so no real record has that value).
// ---------------------------------------------------------------------------
// Raw column words of one lane's four sessions (loaded one chunk ahead).
struct Raw4 {
    uint4 src, dst, ts;
    ulonglong2 b01, b23;
    uint32_t l4;
};

template <uint32_t KIND>
__device__ __forceinline__ void load4(const PassParams& p, uint64_t i, Raw4& r) {
    if constexpr (KIND == KK_LABEL_IN) {
        r.l4 = *glob(reinterpret_cast<const uint32_t*>(p.label_in + i));
    } else {
        r.src = gload4(p.src + i);
        r.dst = gload4(p.dst + i);
    }
    r.ts = gload4(p.ts + i);
    r.b01 = gload2(p.bytes + i);
    r.b23 = gload2(p.bytes + i + 2);
}

// LDS scratch of one stage-1 workgroup.
struct Stage1Shared {
    uint32_t cnt[kWin];
    uint32_t base[kWin];
    uint32_t far[kChunk / 32];
    uint32_t wmin[kStage1Block / 64];
    uint32_t nextra, nfar;
};
// Static LDS of a stage-1 workgroup: two alternating Stage1Shared and the
// record buffer (one suffices: a chunk fills it only after its first barrier,
// which every lane reaches after copying the previous chunk out).
constexpr size_t kStage1StaticLds = 2 * sizeof(Stage1Shared) + sizeof(uint4) * (kChunkSlots / 4);

// Records of one session's byte count (see the record format above).
__device__ __forceinline__ uint32_t record_parts(unsigned long long by) {
    if (by < kSmallMax) return 1u;
    return by < (1ull << 34) ? 2u : (by < (1ull << 51) ? 3u : 4u);
}

// Stage 1 on one chunk.  c is the chunk within the stream (sessions
// c * kChunk + ...), g its index in the workspace (slots, directory, far
// bits) and b0 the workspace index of the stream's first block.
template <uint32_t KIND>
__device__ __forceinline__ void stage1_chunk(const PassParams& p, const PartWs& w, const LdsView& v,
                                             Stage1Shared& sh, uint4* srec, uint64_t c, uint64_t g, uint32_t b0,
                                             const Raw4& cur, bool full, Dropped& d) {
    const uint32_t tid = threadIdx.x;
    const uint64_t i0 = c * kChunk + (uint64_t)tid * 4;
    uint32_t lab[4], ts[4], bin[4];
    unsigned long long by[4];
    bool inw[4];
    if (full) {
        labels4_from<KIND>(p, v, i0, cur.src, cur.dst, cur.l4, lab);
        ts[0] = cur.ts.x; ts[1] = cur.ts.y; ts[2] = cur.ts.z; ts[3] = cur.ts.w;
        by[0] = cur.b01.x; by[1] = cur.b01.y; by[2] = cur.b23.x; by[3] = cur.b23.y;
#pragma unroll
        for (int k = 0; k < 4; ++k) inw[k] = in_window(p, ts[k], bin[k]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t i = i0 + k;
            inw[k] = false;
            lab[k] = 0;
            ts[k] = 0;
            by[k] = 0;
            bin[k] = 0;
            if (i < p.n) {
                if constexpr (KIND == KK_LABEL_IN) {
                    lab[k] = *glob(p.label_in + i) & 3u;
                } else {
                    lab[k] = label1<KIND>(p, v, i);
                }
                ts[k] = *glob(p.ts + i);
                by[k] = *glob(p.bytes + i);
                inw[k] = in_window(p, ts[k], bin[k]);
            }
        }
    }
    uint32_t blk[4];
    uint32_t mymin = 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        blk[k] = bin[k] / kBlockBins;
        if (inw[k]) mymin = min(mymin, blk[k]);
        else if (i0 + k < p.n) d.add(lab[k], by[k]);
    }
    // sh alternates between two buffers from chunk to chunk, so clearing this
    // chunk's counters cannot race with lanes still writing the previous one
    mymin = wave_min(mymin);
    if ((tid & 63) == 0) sh.wmin[tid >> 6] = mymin;
    if (tid < kWin) sh.cnt[tid] = 0;
    for (uint32_t k = tid; k < kChunk / 32; k += kStage1Block) sh.far[k] = 0;
    if (tid == 0) {
        sh.nextra = 0;
        sh.nfar = 0;
    }
    __syncthreads();
    uint32_t bmin = 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < kStage1Block / 64; ++k) bmin = min(bmin, sh.wmin[k]);
    uint32_t rank[4], nrec[4];
    bool loc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t r = blk[k] - bmin;
        loc[k] = inw[k] && r < kWin && by[k] < (1ull << 52);
        nrec[k] = record_parts(by[k]);
        if (loc[k] && nrec[k] > 1u) {
            const uint32_t e = atomicAdd(&sh.nextra, nrec[k] - 1u);
            if (e + nrec[k] - 1u > (uint32_t)kExtraRecs) loc[k] = false;
        }
        rank[k] = loc[k] ? atomicAdd(&sh.cnt[r], nrec[k]) : 0u;
        if (inw[k] && !loc[k]) {
            const uint32_t sidx = tid * 4 + k;
            atomicOr(&sh.far[sidx >> 5], 1u << (sidx & 31));
            atomicAdd(&sh.nfar, 1u);
        }
    }
    __syncthreads();
    if (tid < 64) {  // exclusive scan of the kWin (= 64) padded block counts, one wave
        const uint32_t x = (sh.cnt[tid] + 3u) & ~3u;
        uint32_t inc = x;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)inc, o);
            if ((int)tid >= o) inc += y;
        }
        sh.base[tid] = inc - x;
        // null records in the padding of the block's segment
        uint32_t* lpad = reinterpret_cast<uint32_t*>(srec);
        for (uint32_t q = inc - x + sh.cnt[tid]; q < inc; ++q) lpad[q] = 0xFFFFFFFFu;
        // directory entry of every touched block
        const bool nz = x != 0;
        const unsigned long long m = __ballot(nz);
        const uint32_t e = __popcll(m & ((1ull << tid) - 1ull));
        if (nz) {
            const uint32_t b = b0 + bmin + tid;
            w.dir[g * kWin + e] = make_uint4(b, (uint32_t)(g * kChunkSlots) + (inc - x), x, 0u);
            atomicAdd(w.seg_count + b, 1u);
        }
        if (tid == 0) w.nd[g] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    uint32_t* lrec = reinterpret_cast<uint32_t*>(srec);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!loc[k]) continue;
        const uint32_t r = blk[k] - bmin;
        const uint32_t off = bin[k] - blk[k] * kBlockBins;
        const uint32_t key = (lab[k] << 30) | (off << 20);
        const uint32_t at = sh.base[r] + rank[k];
        if (nrec[k] == 1u) {
            lrec[at] = key | (uint32_t)by[k];
        } else {
            for (uint32_t q = 0; q < nrec[k]; ++q)
                lrec[at + q] = key | (1u << 19) | (q << 17) | (uint32_t)((by[k] >> (17 * q)) & 0x1FFFFu);
        }
    }
    __syncthreads();
    {   // the filled slots of the chunk, one 16-byte store per lane
        const uint32_t nloc = sh.base[kWin - 1] + ((sh.cnt[kWin - 1] + 3u) & ~3u);
        uint4* dst = reinterpret_cast<uint4*>(w.rec + g * kChunkSlots);
        for (uint32_t k = tid; k < nloc / 4; k += kStage1Block) dst[k] = srec[k];
    }
    if (sh.nfar) {
        for (uint32_t k = tid; k < kChunk / 32; k += kStage1Block)
            w.farbits[g * (kChunk / 32) + k] = sh.far[k];
        if (tid == 0) w.farlist[atomicAdd(w.farcount, 1u)] = (uint32_t)g;
    }
}

template <uint32_t KIND>
__global__ void __launch_bounds__(kStage1Block, 4) k_stage1(PassParams p, PartWs w) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ Stage1Shared sh[2];
    __shared__ uint4 srec[kChunkSlots / 4];
    __shared__ uint32_t s_run;
    uint32_t used = 0;
    const LdsView v = stage_lds<KIND>(p.t, lds, &used);
    Dropped d{};
    const uint32_t tid = threadIdx.x;
    const uint64_t n_chunks = w.n_chunks;
    uint32_t iter = 0;
    // a chunk is "full" when its kChunk sessions exist and vector loads are allowed
    auto full = [&](uint64_t c) { return w.vec && (c + 1) * kChunk <= p.n; };
    // workgroups take runs of kStage1Run consecutive chunks from a counter, so
    // one that falls behind (a busy XCD, a chunk of far sessions) takes fewer;
    // every lane reads s_run before the chunk's first barrier, tid 0 writes it
    // again only after the run's last one
    for (;;) {
        if (tid == 0) s_run = atomicAdd(w.next_run, 1u);
        __syncthreads();
        const uint64_t c0 = (uint64_t)__builtin_amdgcn_readfirstlane((int)s_run) * kStage1Run;
        if (c0 >= n_chunks) break;
        const uint64_t c1 = c0 + kStage1Run < n_chunks ? c0 + kStage1Run : n_chunks;
        Raw4 cur{}, nxt{};
        if (full(c0)) load4<KIND>(p, c0 * kChunk + (uint64_t)tid * 4, cur);
        for (uint64_t c = c0; c < c1; ++c) {
            if (c + 1 < c1 && full(c + 1)) load4<KIND>(p, (c + 1) * kChunk + (uint64_t)tid * 4, nxt);
            stage1_chunk<KIND>(p, w, v, sh[iter++ & 1u], srec, c, c, 0u, cur, full(c), d);
            cur = nxt;
        }
    }
    d.flush(p.dropped);
}

// Exclusive scan of n u32 counts into out[0..n] (out[n] = total), in three
// launches: per-tile sums, a single-workgroup scan of the tile sums, and the
// per-tile rescan.  kScanTile elements per workgroup of 1024 threads.
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t x, uint32_t* s_w) {
    const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = x;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)inc, o);
        if ((int)lane >= o) inc += y;
    }
    if (lane == 63) s_w[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        const uint32_t nw = blockDim.x >> 6;
        uint32_t v = lane < nw ? s_w[lane] : 0u;
        uint32_t vi = v;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)vi, o);
            if ((int)lane >= o) vi += y;
        }
        if (lane < nw) s_w[lane] = vi - v;
    }
    __syncthreads();
    const uint32_t r = inc + s_w[wid];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(1024) k_scan_tiles(const uint32_t* __restrict__ in, uint32_t n,
                                                     uint32_t* __restrict__ tile_sum) {
    __shared__ uint32_t s_w[16];
    const uint64_t i = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
    const uint32_t x = i < n ? in[i] : 0u;
    const uint32_t inc = block_incl_scan(x, s_w);
    if (threadIdx.x == 1023) tile_sum[blockIdx.x] = inc;
}

__global__ void __launch_bounds__(1024) k_scan_top(uint32_t* __restrict__ tile_sum, uint32_t nt) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nt; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t x = i < nt ? tile_sum[i] : 0u;
        const uint32_t inc = block_incl_scan(x, s_w);
        const uint32_t carry = s_carry;
        if (i < nt) tile_sum[i] = carry + inc - x;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = carry + inc;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(1024) k_scan_final(const uint32_t* __restrict__ in, uint32_t n,
                                                     const uint32_t* __restrict__ tile_off,
                                                     uint32_t* __restrict__ out) {
    __shared__ uint32_t s_w[16];
    const uint64_t i = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
    const uint32_t x = i < n ? in[i] : 0u;
    const uint32_t inc = block_incl_scan(x, s_w);
    const uint32_t exc = tile_off[blockIdx.x] + inc - x;
    if (i < n) out[i] = exc;
    if (i == n) out[n] = exc;  // the total (x = 0 there)
}

// Group the directory entries by block: segs[seg_off[b] ..] = (first slot,
// count).  Consumes seg_count back to zero.
__global__ void k_fill(PartWs w) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < w.n_chunks * kWin;
         q += stride) {
        const uint64_t c = q / kWin;
        const uint32_t e = (uint32_t)(q % kWin);
        if (e >= w.nd[c]) continue;
        const uint4 d = w.dir[q];
        const uint32_t pos = w.seg_off[d.x] + atomicSub(w.seg_count + d.x, 1u) - 1u;
        w.segs[pos] = make_uint2(d.y, d.z);
    }
}

// Stage 2.  Persistent workgroups take their XCD's blocks in turn (stage2_run).
// A block's segment descriptors (first slot, 16-byte groups) sit in LDS,
// double-buffered: while a block's records are accumulated, the next block's
// descriptors and the segment range of the one after it are in flight.
// Each wave walks its segments (w, w + 8, ...) as one stream of 16-byte groups,
// kRecUnroll loads in flight per lane across segment ends.  The accumulators
// are cleared once and then by the write-out that reads them.
struct Stage2Shared {
    unsigned long long b[4 * kBlockBins];
    uint32_t c[4 * kBlockBins];
    uint32_t start[2][kSegMax];  // first slot (a multiple of 4)
    uint32_t nvec[2][kSegMax];   // 16-byte groups
    uint32_t nseg[2];            // described segments
    uint32_t s0[2], s1[2];       // the block's whole segment range
};

// Where a block's bins go.
struct BlockOut {
    unsigned long long* count;
    unsigned long long* hbytes;
    uint32_t n_bins;
    uint32_t blk;  // the block's index in its stream
    int accumulate;
};

__device__ __forceinline__ void add_record(Stage2Shared& sh, uint32_t r) {
    if (r == 0xFFFFFFFFu) return;  // padding
    const uint32_t key = r >> 20;  // label * kBlockBins + offset
    if (!((r >> 19) & 1u)) {
        atomicAdd(&sh.c[key], 1u);
        atomicAdd(&sh.b[key], (unsigned long long)(r & 0x7FFFFu));
    } else {
        const uint32_t q = (r >> 17) & 3u;
        if (q == 0) atomicAdd(&sh.c[key], 1u);
        atomicAdd(&sh.b[key], (unsigned long long)(r & 0x1FFFFu) << (17 * q));
    }
}

// Accumulate the segments described in buffer d.
__device__ __forceinline__ void stage2_segments(const PartWs& w, Stage2Shared& sh, uint32_t d) {
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    constexpr uint32_t kWaves = kStage2Block / 64;
    const uint32_t nseg = sh.nseg[d];
    uint32_t j = wave, o = 0;  // the wave's cursor: segment, group offset (wave-uniform)
    while (j < nseg) {
        uint4 r4[kRecUnroll];
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) {
            r4[u] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
            if (j < nseg) {
                const uint32_t nv = sh.nvec[d][j];
                if (o + lane < nv)
                    r4[u] = reinterpret_cast<const uint4*>(w.rec + sh.start[d][j])[o + lane];
                o += 64;
                if (o >= nv) {
                    o = 0;
                    j += kWaves;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kRecUnroll; ++u) {
            add_record(sh, r4[u].x);
            add_record(sh, r4[u].y);
            add_record(sh, r4[u].z);
            add_record(sh, r4[u].w);
        }
    }
}

// Descriptors of segments [s, s + n) of the current block into buffer d
// (n <= kSegMax), by the whole workgroup.
__device__ __forceinline__ void stage2_describe(const PartWs& w, Stage2Shared& sh, uint32_t d,
                                                uint32_t s, uint32_t n) {
    for (uint32_t k = threadIdx.x; k < n; k += kStage2Block) {
        const uint2 sg = w.segs[s + k];
        sh.start[d][k] = sg.x;
        sh.nvec[d][k] = sg.y >> 2;
    }
    if (threadIdx.x == 0) sh.nseg[d] = n;
}

// Bin pairs are written with non-temporal 16-byte stores: the histogram is
// written once and not read back by this pass.
__device__ __forceinline__ void store_pair(unsigned long long* q, unsigned long long x,
                                           unsigned long long y) {
    __builtin_nontemporal_store(u64x2_t{x, y}, glob(reinterpret_cast<u64x2_t*>(q)));
}

// Bins from an output row's start to its first 128-byte line boundary.  Blocks
// start at multiples of kBlockBins bins (8 KB), so a row's skew is the same in
// every block.
__device__ __forceinline__ uint32_t line_skew(const unsigned long long* row) {
    return (uint32_t)(((128u - ((uintptr_t)row & 127u)) & 127u) >> 3);
}

// Write the block's bins and clear the accumulators it read.  Two consecutive
// bins per lane with 16-byte stores when the label rows are 16-byte aligned
// (n_bins even), else one.  Within every row the lanes start at the row's
// first 128-byte line boundary inside the block and wrap around to the bins
// before it, so each wave store covers whole lines and only the two lines a
// block shares with its neighbours are written in part.  On rows that are not
// line-aligned (n_bins * 8 not a multiple of 128, or an offset buffer) wave
// stores that straddle lines cost about a fifth of the write rate.  A block
// without records (empty) writes zeros without touching the accumulators,
// which are already clear.
__device__ __forceinline__ void stage2_write(Stage2Shared& sh, const BlockOut& t, bool empty) {
    const uint64_t b0 = (uint64_t)t.blk * kBlockBins;
    const bool pairs =
        (t.n_bins & 1u) == 0 && (((uintptr_t)t.count | (uintptr_t)t.hbytes) & 15u) == 0;
    if (pairs) {
        const bool zeros = empty && !t.accumulate;
        for (uint32_t k = threadIdx.x; k < 2 * kBlockBins; k += kStage2Block) {
            const uint32_t lab = k / (kBlockBins / 2), j = k % (kBlockBins / 2);
            const uint64_t row = (uint64_t)lab * t.n_bins;
            // skews are even here: the rows are 16-byte aligned
            const uint32_t oc = (line_skew(t.count + row) + 2 * j) & (kBlockBins - 1);
            const uint32_t ob = (line_skew(t.hbytes + row) + 2 * j) & (kBlockBins - 1);
            const uint32_t ec = lab * kBlockBins + oc, eb = lab * kBlockBins + ob;
            ulonglong2 c = make_ulonglong2(0ull, 0ull), b = make_ulonglong2(0ull, 0ull);
            if (!zeros) {
                c = make_ulonglong2(sh.c[ec], sh.c[ec + 1]);
                b = make_ulonglong2(sh.b[eb], sh.b[eb + 1]);
                sh.c[ec] = 0;
                sh.c[ec + 1] = 0;
                sh.b[eb] = 0;
                sh.b[eb + 1] = 0;
            }
            // n_bins even: bin + 1 is inside whenever bin is
            if (b0 + oc < t.n_bins) {
                unsigned long long* q = t.count + row + b0 + oc;
                if (t.accumulate) {
                    const ulonglong2 o = *reinterpret_cast<const ulonglong2*>(q);
                    c.x += o.x;
                    c.y += o.y;
                }
                store_pair(q, c.x, c.y);
            }
            if (b0 + ob < t.n_bins) {
                unsigned long long* q = t.hbytes + row + b0 + ob;
                if (t.accumulate) {
                    const ulonglong2 o = *reinterpret_cast<const ulonglong2*>(q);
                    b.x += o.x;
                    b.y += o.y;
                }
                store_pair(q, b.x, b.y);
            }
        }
    } else {
        for (uint32_t k = threadIdx.x; k < 4 * kBlockBins; k += kStage2Block) {
            const uint32_t lab = k / kBlockBins, j = k % kBlockBins;
            const uint64_t row = (uint64_t)lab * t.n_bins;
            const uint32_t oc = (line_skew(t.count + row) + j) & (kBlockBins - 1);
            const uint32_t ob = (line_skew(t.hbytes + row) + j) & (kBlockBins - 1);
            unsigned long long c = sh.c[lab * kBlockBins + oc], b = sh.b[lab * kBlockBins + ob];
            sh.c[lab * kBlockBins + oc] = 0;
            sh.b[lab * kBlockBins + ob] = 0;
            if (b0 + oc < t.n_bins) {
                unsigned long long* q = t.count + row + b0 + oc;
                *q = t.accumulate ? *q + c : c;
            }
            if (b0 + ob < t.n_bins) {
                unsigned long long* q = t.hbytes + row + b0 + ob;
                *q = t.accumulate ? *q + b : b;
            }
        }
    }
}

// The persistent block loop; out(g) names where block g's bins go.  Runs of
// `run` consecutive blocks are dealt round-robin over the XCDs (workgroup w
// runs on XCD w % kXcds), and an XCD's S workgroups take its blocks in turn.
// With runs of kStage2Run, neighbouring blocks are written at about the same
// time through the same L2, so a 128-byte line that two blocks share (rows
// whose length is not a multiple of 16 bins) is completed there rather than
// written to HBM in two parts, while every XCD still gets a share of every
// part of the histogram.  On 64 uneven streams the batch's stage 2 took
// 5.33-5.35 ms this way, 5.68-5.72 ms with runs of one block and 5.47-5.48 ms
// with one contiguous range per XCD (which also slowed the day cut into 24
// hourly streams, whose busy hours then fell on a few XCDs: 11.33 -> up to
// 11.83 ms).  Where every row starts on a line, runs of one block are faster
// (the 1e8-session day: 1.19 against 1.23 ms).
template <class Out>
__device__ __forceinline__ void stage2_run(const PartWs& w, Stage2Shared& sh, const Out& out,
                                           uint32_t run) {
    const uint32_t tid = threadIdx.x;
    const uint32_t G = gridDim.x, nb = w.n_blocks;
    const uint32_t X = G < (uint32_t)kXcds ? G : (uint32_t)kXcds;  // XCDs with workgroups
    const uint32_t xcd = blockIdx.x % kXcds, lid = blockIdx.x / kXcds;
    const uint32_t per = G / kXcds, rem = G % kXcds;
    const uint32_t S = per + (xcd < rem ? 1u : 0u);  // workgroups on this XCD
    // the XCD's t-th block (increasing in t; nb once past the last block)
    auto blk = [&](uint32_t t) -> uint32_t {
        const uint64_t b = ((uint64_t)(t / run) * X + xcd) * run + t % run;
        return b < nb ? (uint32_t)b : nb;
    };
    uint32_t t = lid;
    uint32_t g = blk(t);
    if (g >= nb) return;
    for (uint32_t k = tid; k < 4 * kBlockBins; k += kStage2Block) {
        sh.b[k] = 0;
        sh.c[k] = 0;
    }
    {
        const uint32_t s0 = w.seg_off[g], s1 = w.seg_off[g + 1];
        stage2_describe(w, sh, 0, s0, min(s1 - s0, (uint32_t)kSegMax));
        if (tid == 0) {
            sh.s0[0] = s0;
            sh.s1[0] = s1;
        }
    }
    uint32_t gn = blk(t + S);  // next block, and its segment range
    uint32_t n0 = 0, n1 = 0;
    if (gn < nb) {
        n0 = w.seg_off[gn];
        n1 = w.seg_off[gn + 1];
    }
    BlockOut cur = out(g);  // where the current block's bins go (found one block ahead)
    for (uint32_t d = 0; g < nb; t += S, g = gn, gn = blk(t + S), d ^= 1u) {
        __syncthreads();  // descriptors of g in buffer d, accumulators clear
        // in flight during this block: the next block's descriptors and the
        // segment range of the block after it
        const uint32_t nn = gn < nb ? min(n1 - n0, (uint32_t)kSegMax) : 0u;
        uint2 nsg = make_uint2(0u, 0u);
        if (tid < nn) nsg = w.segs[n0 + tid];
        const uint32_t gnn = blk(t + 2 * S);
        uint32_t m0 = 0, m1 = 0;
        if (gnn < nb) {
            m0 = w.seg_off[gnn];
            m1 = w.seg_off[gnn + 1];
        }
        const BlockOut nxt = gn < nb ? out(gn) : cur;  // its lookup overlaps this block
        stage2_segments(w, sh, d);
        // blocks with more than kSegMax segments (unsorted input): further
        // batches through the same buffer
        const uint32_t s0 = sh.s0[d], s1 = sh.s1[d];
        for (uint32_t sb = s0 + kSegMax; sb < s1; sb += kSegMax) {
            __syncthreads();
            stage2_describe(w, sh, d, sb, min(s1 - sb, (uint32_t)kSegMax));
            __syncthreads();
            stage2_segments(w, sh, d);
        }
        __syncthreads();  // accumulation complete
        stage2_write(sh, cur, s0 == s1);
        if (gn < nb) {
            const uint32_t e = d ^ 1u;  // last read before this block's first barrier
            if (tid < nn) {
                sh.start[e][tid] = nsg.x;
                sh.nvec[e][tid] = nsg.y >> 2;
            }
            if (tid == 0) {
                sh.nseg[e] = nn;
                sh.s0[e] = n0;
                sh.s1[e] = n1;
            }
        }
        n0 = m0;
        n1 = m1;
        cur = nxt;
    }
}

struct PlainOut {
    unsigned long long* count;
    unsigned long long* hbytes;
    uint32_t n_bins;
    int accumulate;
    __device__ BlockOut operator()(uint32_t g) const {
        return BlockOut{count, hbytes, n_bins, g, accumulate};
    }
};

__global__ void __launch_bounds__(kStage2Block) k_stage2(PartWs w, unsigned long long* count,
                                                        unsigned long long* hbytes, uint32_t n_bins,
                                                        int accumulate) {
    __shared__ Stage2Shared sh;
    const bool lines = (n_bins & 15u) == 0 && (((uintptr_t)count | (uintptr_t)hbytes) & 127u) == 0;
    stage2_run(w, sh, PlainOut{count, hbytes, n_bins, accumulate}, lines ? 1u : kStage2Run);
}

__global__ void k_zero(unsigned long long* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t head = ((uintptr_t)p & 15) ? 1 : 0;  // p is 8-byte aligned
    if (head && i == 0) p[0] = 0;
    ulonglong2* q = reinterpret_cast<ulonglong2*>(p + head);
    const uint64_t n2 = (n - head) / 2;
    for (uint64_t k = i; k < n2; k += stride) q[k] = make_ulonglong2(0, 0);
    if (i == 0 && ((n - head) & 1)) p[n - 1] = 0;
}

__global__ void k_zero32(uint32_t* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = 0;
}

// ---------------------------------------------------------------------------
// Batched form: many independent streams in one persistent launch.
//
// The paper's coordinated batch processing feeds uneven chunks through a work
// queue so that every worker stays busy (sections "Coordinated Batch
// Processing", "Work Queue", "TASK DECOMPOSITION").  Here the queue is a
// device counter over (stream, chunk range) items that the persistent
// workgroups pull until it is exhausted; a workgroup restages the table in
// LDS only when the stream changes.  Partitioned streams share one workspace
// (chunk and block index spaces concatenated), so one scan, one fill, one
// stage-2 launch and one far pass serve all of them.  Streams with few bins
// keep their whole histogram in LDS for the item and merge it with atomics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

template <uint32_t KIND>
__device__ __forceinline__ void batch_stage1(const BatchArgs& a, const PartWs& w) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ Stage1Shared sh[2];
    __shared__ uint4 srec[kChunkSlots / 4];
    __shared__ uint32_t s_item;
    __shared__ BatchStreamDev s_bs;  // the current stream's descriptor
    const uint32_t tid = threadIdx.x;
    uint32_t staged = 0xFFFFFFFFu;
    LdsView v{};
    uint32_t used = 0;
    uint32_t iter = 0;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(a.counter, 1u);
        __syncthreads();
        const uint32_t it = uniform_u32(s_item);
        if (it >= a.n_items) break;
        const uint4 item = a.items[it];
        const uint32_t si = uniform_u32(item.x);
        if (si != staged) {
            // descriptor to LDS (read there by every lane, never from global
            // memory inside the session loop), then the table
            constexpr uint32_t kWords = sizeof(BatchStreamDev) / 4;
            const uint32_t* src = reinterpret_cast<const uint32_t*>(a.streams + si);
            uint32_t* dst = reinterpret_cast<uint32_t*>(&s_bs);
            for (uint32_t k = tid; k < kWords; k += blockDim.x) dst[k] = src[k];
            __syncthreads();
            v = stage_lds<KIND>(s_bs.p.t, lds, &used);  // ends with a barrier
            staged = si;
        }
        // the descriptor in scalar registers for the item: read from LDS after
        // every barrier it would cost an LDS round trip per use
        BatchStreamDev bs;
        {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(&s_bs);
            uint32_t* dst = reinterpret_cast<uint32_t*>(&bs);
#pragma unroll
            for (uint32_t k = 0; k < sizeof(BatchStreamDev) / 4; ++k) dst[k] = uniform_u32(src[k]);
        }
        const PassParams& p = bs.p;
        Dropped d{};
        if (bs.priv) {
            PrivHist h;
            const uint32_t base = (used + 1) & ~1u;
            h.b = reinterpret_cast<unsigned long long*>(lds + base);
            h.c = lds + base + 2 * 4 * p.n_bins;
            for (uint32_t k = tid; k < 4 * p.n_bins; k += blockDim.x) {
                h.b[k] = 0;
                h.c[k] = 0;
            }
            __syncthreads();
            const bool vec = bs.vec != 0;
            for (uint64_t c = item.y; c < item.z; ++c) {
                const uint64_t g4 = c * (kChunk / 4) + tid;  // group of 4 sessions
                if (vec && g4 * 4 + 4 <= p.n) {
                    four_sessions<KIND, H_PRIVATE>(p, v, h, g4 * 4, d);
                } else {
                    for (uint64_t i = g4 * 4; i < p.n && i < g4 * 4 + 4; ++i)
                        one_session<KIND, H_PRIVATE>(p, v, h, i, d);
                }
            }
            __syncthreads();
            for (uint32_t k = tid; k < 4 * p.n_bins; k += blockDim.x) {
                if (h.c[k]) {
                    __hip_atomic_fetch_add(p.count + k, (unsigned long long)h.c[k], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_add(p.hbytes + k, h.b[k], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
        } else {
            const bool vec = bs.vec != 0;
            auto full = [&](uint64_t c) { return vec && (c + 1) * kChunk <= p.n; };
            Raw4 cur{}, nxt{};
            uint64_t c = item.y;
            if (c < item.z && full(c)) load4<KIND>(p, c * kChunk + (uint64_t)tid * 4, cur);
            for (; c < item.z; ++c) {
                if (c + 1 < item.z && full(c + 1)) load4<KIND>(p, (c + 1) * kChunk + (uint64_t)tid * 4, nxt);
                stage1_chunk<KIND>(p, w, v, sh[iter++ & 1u], srec, c, bs.chunk0 + c, bs.block0, cur,
                                   full(c), d);
                cur = nxt;
            }
        }
        d.flush(p.dropped);
    }
}

// Block g of the shared workspace belongs to the last stream whose first
// block is <= g (streams without blocks share their base with the next one).
struct BatchOut {
    const BatchArgs* a;
    __device__ BlockOut operator()(uint32_t gb) const {
        uint32_t lo = 0, n = a->n_streams;
        while (n > 1) {
            const uint32_t half = n >> 1;
            lo = a->block_base[lo + half] <= gb ? lo + half : lo;
            n -= half;
        }
        while (lo + 1 < a->n_streams && a->block_base[lo + 1] <= gb) ++lo;
        const BatchStreamDev& bs = a->streams[lo];
        return BlockOut{bs.p.count, bs.p.hbytes, bs.p.n_bins, gb - bs.block0, 0};
    }
};

__global__ void __launch_bounds__(kStage2Block) k_batch_stage2(BatchArgs a, PartWs w) {
    __shared__ Stage2Shared sh;
    stage2_run(w, sh, BatchOut{&a}, kStage2Run);
}


// In/out-index lookups fit 128 VGPRs (4 waves per SIMD, two workgroups per CU);
// the interval kinds keep their registers rather than spill.
template <uint32_t KIND>
__global__ void __launch_bounds__(kStage1Block) k_batch_stage1(BatchArgs a, PartWs w) {
    batch_stage1<KIND>(a, w);
}
template <uint32_t KIND>
__global__ void __launch_bounds__(kStage1Block, 4) k_batch_stage1_o4(BatchArgs a, PartWs w) {
    batch_stage1<KIND>(a, w);
}

template <uint32_t KIND>
__global__ void __launch_bounds__(kMaxBlock) k_batch_far(BatchArgs a, PartWs w) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    uint32_t staged = 0xFFFFFFFFu;
    LdsView v{};
    uint32_t used = 0;
    const PrivHist h{nullptr, nullptr};
    const uint32_t nfar = *w.farcount;
    for (uint32_t q = blockIdx.x; q < nfar; q += gridDim.x) {
        const uint64_t g = w.farlist[q];
        uint32_t lo = 0, n = a.n_streams;
        while (n > 1) {
            const uint32_t half = n >> 1;
            lo = a.chunk_base[lo + half] <= g ? lo + half : lo;
            n -= half;
        }
        while (lo + 1 < a.n_streams && a.chunk_base[lo + 1] <= g) ++lo;
        const uint32_t si = uniform_u32(lo);
        const BatchStreamDev& bs = a.streams[si];
        if (bs.priv || bs.p.t.kind != KIND) continue;  // another kind group's chunk
        PassParams p = bs.p;
        p.label_out = nullptr;
        p.src_inst = nullptr;
        p.dst_inst = nullptr;
        p.dropped = nullptr;
        if (si != staged) {
            __syncthreads();
            v = stage_lds<KIND>(p.t, lds, &used);
            staged = si;
        }
        const uint64_t c = g - bs.chunk0;
        Dropped d{};
        for (uint32_t s = threadIdx.x; s < kChunk; s += blockDim.x) {
            const uint64_t i = c * kChunk + s;
            if (i < p.n && ((w.farbits[g * (kChunk / 32) + s / 32] >> (s & 31)) & 1u))
                one_session<KIND, H_ATOMIC>(p, v, h, i, d);
        }
    }
}

// Batched lookup pass: streams whose lookups walk global memory store their
// labels first, as the single-stream path does, and stage 1 reads them (one
// byte per session) instead of stalling its barriers on the lookups.  Work
// items as in batch stage 1; a workgroup restages the table only when the
// stream changes; the next four sessions' addresses are loaded before the
// current ones are looked up.
template <uint32_t KIND>
__global__ void __launch_bounds__(kMaxBlock) k_batch_lookup(BatchArgs a) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    __shared__ uint32_t s_item;
    __shared__ BatchStreamDev s_bs;
    const uint32_t tid = threadIdx.x;
    uint32_t staged = 0xFFFFFFFFu;
    LdsView v{};
    uint32_t used = 0;
    const PrivHist h{nullptr, nullptr};
    for (;;) {
        __syncthreads();  // every lane is done with the previous item
        if (tid == 0) s_item = atomicAdd(a.counter, 1u);
        __syncthreads();
        const uint32_t it = uniform_u32(s_item);
        if (it >= a.n_items) break;
        const uint4 item = a.items[it];
        const uint32_t si = uniform_u32(item.x);
        if (si != staged) {
            constexpr uint32_t kWords = sizeof(BatchStreamDev) / 4;
            const uint32_t* src = reinterpret_cast<const uint32_t*>(a.streams + si);
            uint32_t* dst = reinterpret_cast<uint32_t*>(&s_bs);
            for (uint32_t k = tid; k < kWords; k += blockDim.x) dst[k] = src[k];
            __syncthreads();
            v = stage_lds<KIND>(s_bs.p.t, lds, &used);  // ends with a barrier
            // the window PLA's search queue, after the table (a.queue_words
            // per wave when the launch made room for it)
            if constexpr (KIND == KK_PLA)  // window PLAs only (the wider search needs a larger queue)
                v.queue = a.queue_words && s_bs.p.t.pla_window ? lds + used + (tid >> 6) * a.queue_words
                                                               : nullptr;
            staged = si;
        }
        BatchStreamDev bs;
        {
            const uint32_t* src = reinterpret_cast<const uint32_t*>(&s_bs);
            uint32_t* dst = reinterpret_cast<uint32_t*>(&bs);
#pragma unroll
            for (uint32_t k = 0; k < sizeof(BatchStreamDev) / 4; ++k) dst[k] = uniform_u32(src[k]);
        }
        const PassParams& p = bs.p;
        const uint64_t groups = (p.n + 3) / 4;
        const uint64_t g0 = (uint64_t)item.y * (kChunk / 4);
        const uint64_t g1 = min((uint64_t)item.z * (kChunk / 4), groups);
        auto full = [&](uint64_t g) { return bs.vec && g * 4 + 4 <= p.n; };
        uint4 cs = make_uint4(0, 0, 0, 0), cd = cs, ns = cs, nd = cs;
        uint64_t g = g0 + tid;
        if (g < g1 && full(g)) {
            cs = gload4(p.src + g * 4);
            cd = gload4(p.dst + g * 4);
        }
        for (; g < g1; g += blockDim.x) {
            const uint64_t gn = g + blockDim.x;
            if (gn < g1 && full(gn)) {
                ns = gload4(p.src + gn * 4);
                nd = gload4(p.dst + gn * 4);
            }
            if (full(g)) {
                uint32_t lab[4];
                labels4_from<KIND, KIND == KK_PLA ? kQueueWindow : 0>(p, v, g * 4, cs, cd, 0u, lab);
            } else {
                Dropped d{};
                for (uint64_t i = g * 4; i < p.n && i < g * 4 + 4; ++i)
                    one_session<KIND, H_NONE>(p, v, h, i, d);
            }
            cs = ns;
            cd = nd;
        }
    }
}

__global__ void k_zero_jobs(const ZeroJob* __restrict__ jobs, uint32_t n_jobs) {
    for (uint32_t j = blockIdx.x; j < n_jobs; j += gridDim.x) {
        const ZeroJob z = jobs[j];
        for (uint64_t k = threadIdx.x; k < z.n; k += blockDim.x) z.p[k] = 0;
    }
}

// ---------------------------------------------------------------------------
// Watch-list histograms (sections "AbuseIPDB" and "GRIZZLY STEPPE", Figures
// 8-11): the sessions of listed hosts per time window, in both directions.
// The list is a prefix table whose institution ids are the keys.  Each
// session looks up its source and its destination; a match adds (1, bytes)
// to cell [dir][key][bin] (dir 0: the source matched, 1: the destination),
// or to dropped[dir] outside the window.  Listed sessions are few, so the
// pass is a streaming read of the address columns: the /16 filter in LDS
// rejects most addresses with one LDS read, only addresses in blocks the
// list touches run the interval search, and the timestamps and byte counts
// are loaded only for a lane whose four sessions include a match.  Small
// histograms live in LDS per workgroup (merged with atomics at the end);
// larger ones take device-scope atomics directly.
// ---------------------------------------------------------------------------
constexpr int kWatchBlock = 512;
constexpr uint32_t kWatchPrivCells = 4096;  // [2][n_keys][n_bins] cells kept in LDS
constexpr uint32_t kWatchLdsKeys = 8192;    // intervals whose keys are staged in LDS

struct WatchParams {
    PassParams p;       // list table, columns, window; count/hbytes [2][n_keys][n_bins], dropped [2][2]
    uint32_t n_keys;
    uint32_t vec;       // 16-byte loads allowed
    uint32_t lds_keys;  // 1: key + 1 of every interval staged in LDS (m <= kWatchLdsKeys)
    uint32_t pad;
};

// Longest-match row + 1 (0: no match) of each address.
template <uint32_t KIND, int N>
__device__ __forceinline__ void owners(const DevTable& t, const LdsView& v, const uint32_t* a,
                                       uint32_t* code) {
    if constexpr (KIND == KK_SCAN) {
#pragma unroll
        for (int q = 0; q < N; ++q) code[q] = scan_owner(t, v, a[q]);
    } else {
        uint32_t need = 0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            code[q] = 0;
            const uint32_t st = (v.filter[a[q] >> 20] >> (((a[q] >> 16) & 15u) * 2)) & 3u;
            need |= (st != 0u ? 1u : 0u) << q;
        }
        if (need) {
            uint32_t j[N];
            intervals<KIND, N>(t, v, a, j, need);
#pragma unroll
            for (int q = 0; q < N; ++q)
                if ((need >> q) & 1u) code[q] = *glob(t.owner + j[q]);
        }
    }
}

struct WatchDropped {
    unsigned long long c[2], b[2];
    __device__ __forceinline__ void add(uint32_t dir, uint64_t nbytes) {
        c[dir] += 1;
        b[dir] += nbytes;
    }
    __device__ __forceinline__ void flush(unsigned long long* out) const {
        if (!out) return;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            if (c[d]) {
                atomicAdd(out + 2 * d, c[d]);
                atomicAdd(out + 2 * d + 1, b[d]);
            }
        }
    }
};

// code: key + 1 when is_key, else the owner row + 1 (its key read from the
// table's inst ids).
template <bool PRIV>
__device__ __forceinline__ void watch_add(const WatchParams& w, uint32_t* hc, unsigned long long* hb,
                                          uint32_t dir, uint32_t code, bool is_key, uint32_t ts,
                                          uint64_t nbytes, WatchDropped& d) {
    uint32_t bin;
    if (!in_window(w.p, ts, bin)) {
        d.add(dir, nbytes);
        return;
    }
    const uint32_t key = is_key ? code - 1 : *glob(w.p.t.inst + (code - 1));
    const uint64_t k = ((uint64_t)dir * w.n_keys + key) * w.p.n_bins + bin;
    if constexpr (PRIV) {
        atomicAdd(hc + k, 1u);
        atomicAdd(hb + k, (unsigned long long)nbytes);
    } else {
        __hip_atomic_fetch_add(w.p.count + k, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(w.p.hbytes + k, (unsigned long long)nbytes, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Match codes of the lane's eight addresses (four sources, four
// destinations): key + 1 from the LDS key array when given, else the owner
// row + 1 from device memory, 0 for no match; the interval search is shared
// by the wave: an address whose /16 block
// the list touches goes to the wave's queue in LDS (slots ordered by address
// number, then lane, from ballots), the wave searches the queue 64 entries at
// a time (one entry per lane) and each lane reads its answers back.  Few
// addresses need the search, so a wave runs one round of it rather than
// eight searches in every lane.  Ballots see only the lanes running the call,
// so lanes a branch masked off neither add entries nor take them.  The queue
// is only touched by its own wave,
// whose LDS operations complete in order; the wavefront fences keep the
// compiler from moving them across each other.
template <uint32_t KIND>
__device__ __forceinline__ void owners8_shared(const DevTable& t, const LdsView& v, const uint32_t* a,
                                               uint32_t* queue, const uint32_t* lkey, uint32_t* code) {
    uint32_t need = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        code[q] = 0;
        const uint32_t st = (v.filter[a[q] >> 20] >> (((a[q] >> 16) & 15u) * 2)) & 3u;
        need |= (st != 0u ? 1u : 0u) << q;
    }
    if (__ballot(need != 0u) == 0ull) return;
    uint32_t slot[8];
    uint32_t total = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint64_t m = __ballot((need >> q) & 1u);
        slot[q] = total + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if ((need >> q) & 1u) queue[slot[q]] = a[q];
        total += (uint32_t)__popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // the lanes running this call (a branch may have masked some off) take
    // the queue's entries in turn
    const uint64_t act = __ballot(1);
    const uint32_t n_act = (uint32_t)__popcll(act);
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
    for (uint32_t b = 0; b < total; b += n_act) {
        const uint32_t k = b + rank;
        if (k < total) {
            const uint32_t x = queue[k];
            uint32_t j;
            intervals<KIND, 1>(t, v, &x, &j, 1u);
            queue[k] = lkey ? lkey[j] : *glob(t.owner + j);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if ((need >> q) & 1u) code[q] = queue[slot[q]];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the queue is reused next tile
}

template <uint32_t KIND, bool PRIV>
__global__ void __launch_bounds__(kWatchBlock) k_watch(WatchParams w) {
    extern __shared__ __attribute__((aligned(16))) uint32_t lds[];
    uint32_t used = 0;
    const PassParams& p = w.p;
    const LdsView v = stage_lds<KIND>(p.t, lds, &used);
    // each wave's search queue: eight addresses per lane at most
    uint32_t* queue = lds + used + (threadIdx.x >> 6) * 512u;
    if constexpr (KIND != KK_SCAN) used += (kWatchBlock / 64) * 512u;
    // key + 1 (0: no match) of every interval, when the list is small enough
    uint32_t* lkey = nullptr;
    if constexpr (KIND != KK_SCAN) {
        if (w.lds_keys) {
            lkey = lds + used;
            for (uint32_t j = threadIdx.x; j < p.t.m; j += blockDim.x) {
                const uint32_t o = *glob(p.t.owner + j);
                lkey[j] = o ? *glob(p.t.inst + (o - 1)) + 1u : 0u;
            }
            used += p.t.m;
            __syncthreads();
        }
    }
    uint32_t* hc = nullptr;
    unsigned long long* hb = nullptr;
    const uint32_t cells = 2u * w.n_keys * p.n_bins;  // <= kWatchPrivCells when PRIV
    if constexpr (PRIV) {
        used = (used + 1) & ~1u;
        hb = reinterpret_cast<unsigned long long*>(lds + used);
        hc = lds + used + 2 * cells;
        for (uint32_t k = threadIdx.x; k < cells; k += blockDim.x) {
            hb[k] = 0;
            hc[k] = 0;
        }
        __syncthreads();
    }
    WatchDropped d{};
    const uint64_t groups = (p.n + 3) / 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // the next group's addresses are loaded while this one is looked up
    auto full = [&](uint64_t g) { return w.vec && g * 4 + 4 <= p.n; };
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint4 cs = make_uint4(0, 0, 0, 0), cd = cs;
    if (g < groups && full(g)) {
        cs = gload4(p.src + g * 4);
        cd = gload4(p.dst + g * 4);
    }
    // a group's matches are added one iteration later, so the loads of their
    // times and byte counts overlap the next group's lookups
    uint32_t pcode[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint4 pt = make_uint4(0, 0, 0, 0);
    ulonglong2 pb01 = make_ulonglong2(0, 0), pb23 = pb01;
    bool pend = false;
    auto apply = [&]() {
        if (!pend) return;
        const uint32_t ts[4] = {pt.x, pt.y, pt.z, pt.w};
        const uint64_t by[4] = {pb01.x, pb01.y, pb23.x, pb23.y};
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (pcode[q])
                watch_add<PRIV>(w, hc, hb, q >> 2, pcode[q], lkey != nullptr, ts[q & 3], by[q & 3], d);
        pend = false;
    };
    for (; g < groups; g += stride) {
        const uint64_t i = g * 4;
        uint4 ns = cs, nd = cd;
        if (g + stride < groups && full(g + stride)) {
            ns = gload4(p.src + (g + stride) * 4);
            nd = gload4(p.dst + (g + stride) * 4);
        }
        if (full(g)) {
            const uint4 s4 = cs, d4 = cd;
            const uint32_t a[8] = {s4.x, s4.y, s4.z, s4.w, d4.x, d4.y, d4.z, d4.w};
            uint32_t code[8];
            if constexpr (KIND == KK_SCAN) owners<KIND, 8>(p.t, v, a, code);
            else owners8_shared<KIND>(p.t, v, a, queue, lkey, code);
            uint32_t any = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) any |= code[q];
            apply();  // the previous group's, its loads issued an iteration ago
            if (any) {
                pt = gload4(p.ts + i);
                pb01 = gload2(p.bytes + i);
                pb23 = gload2(p.bytes + i + 2);
#pragma unroll
                for (int q = 0; q < 8; ++q) pcode[q] = code[q];
                pend = true;
            }
        } else {
            apply();
            for (uint64_t e = i; e < p.n && e < i + 4; ++e) {
                const uint32_t a[2] = {*glob(p.src + e), *glob(p.dst + e)};
                uint32_t code[2];
                owners<KIND, 2>(p.t, v, a, code);
                if (code[0] | code[1]) {
                    const uint32_t ts = *glob(p.ts + e);
                    const uint64_t by = *glob(p.bytes + e);
                    for (uint32_t dir = 0; dir < 2; ++dir)
                        if (code[dir]) watch_add<PRIV>(w, hc, hb, dir, code[dir], false, ts, by, d);
                }
            }
        }
        cs = ns;
        cd = nd;
    }
    apply();
    d.flush(p.dropped);
    if constexpr (PRIV) {
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < cells; k += blockDim.x) {
            if (hc[k]) {
                __hip_atomic_fetch_add(p.count + k, (unsigned long long)hc[k], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(p.hbytes + k, hb[k], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using PassFn = void (*)(PassParams, FarList);
using Stage1Fn = void (*)(PassParams, PartWs);

template <uint32_t KIND>
static PassFn pass_fn(int hm, bool vec) {
    if (KIND == KK_INOUT && hm == H_NONE && vec) return k_pass_inout;
    switch (hm) {
        case H_NONE: return vec ? k_pass<KIND, H_NONE, true> : k_pass<KIND, H_NONE, false>;
        case H_ATOMIC: return vec ? k_pass<KIND, H_ATOMIC, true> : k_pass<KIND, H_ATOMIC, false>;
        default: return vec ? k_pass<KIND, H_PRIVATE, true> : k_pass<KIND, H_PRIVATE, false>;
    }
}

static PassFn pick_pass(uint32_t kind, int hm, bool vec) {
    switch (kind) {
        case KK_SCAN: return pass_fn<KK_SCAN>(hm, vec);
        case KK_BSEARCH: return pass_fn<KK_BSEARCH>(hm, vec);
        case KK_TRIE: return pass_fn<KK_TRIE>(hm, vec);
        case KK_PLA: return pass_fn<KK_PLA>(hm, vec);
        case KK_MLP: return pass_fn<KK_MLP>(hm, vec);
        case KK_INOUT: return pass_fn<KK_INOUT>(hm, vec);
        case KK_LABEL_IN: return pass_fn<KK_LABEL_IN>(hm, vec);
        default: return nullptr;
    }
}

static Stage1Fn pick_stage1(uint32_t kind) {
    switch (kind) {
        case KK_SCAN: return k_stage1<KK_SCAN>;
        case KK_BSEARCH: return k_stage1<KK_BSEARCH>;
        case KK_TRIE: return k_stage1<KK_TRIE>;
        case KK_PLA: return k_stage1<KK_PLA>;
        case KK_MLP: return k_stage1<KK_MLP>;
        case KK_INOUT: return k_stage1<KK_INOUT>;
        case KK_LABEL_IN: return k_stage1<KK_LABEL_IN>;
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

static int blocks_per_cu(const void* fn, int block, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<const void*, int, size_t, int>, int> cache;
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto key = std::make_tuple(fn, block, lds, dev);
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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

// Can the 4-session vector loads/stores be used for these pointers?
bool vector_ok(const PassParams& p, uint32_t kind, bool hist) {
    if (p.pos_out) return aligned16(p.src) && aligned16(p.pos_out);
    bool vec = true;
    if (kind == KK_LABEL_IN) vec = aligned4(p.label_in);
    else vec = aligned16(p.src) && aligned16(p.dst);
    if (p.label_out) vec = vec && aligned4(p.label_out);
    if (p.src_inst) vec = vec && aligned16(p.src_inst);
    if (p.dst_inst) vec = vec && aligned16(p.dst_inst);
    if (hist) vec = vec && aligned16(p.ts) && aligned16(p.bytes);
    return vec;
}

static sinet_status launch_k_pass(const PassParams& p, uint32_t kind, int hm, bool vec,
                                  const FarList& far, size_t extra_lds, hipStream_t s) {
    PassFn fn = pick_pass(kind, hm, vec);
    if (!fn) return fail(SINET_ERR_UNSUPPORTED, "no kernel for this lookup kind");
    size_t lds = (kind == KK_LABEL_IN ? 0 : p.t.lds_bytes) + extra_lds + 8;
    if (lds > 160 * 1024) return fail(SINET_ERR_UNSUPPORTED, "table needs more LDS than a CU has");
    const int block = lds > 40 * 1024 ? 1024 : 256;
    // the lookup pass of the queued kinds queues its searches per wave when
    // the queues fit beside the table (labels only: positions and institution
    // ids take the direct path)
    PassParams q = p;
    q.queue_words = 0;
    // (the binary search over all boundaries in global memory, one leaf, is
    // latency-bound like the PLA and keeps the direct path)
    const bool global_search = kind == KK_BSEARCH && p.t.n_top <= 1;
    const uint32_t qw = kind == KK_PLA && p.t.pla_window ? kPlaQueue : kSearchQueue;
    if (hm == H_NONE && queued_kind(kind) && qw && !global_search && !p.pos_out && !p.src_inst &&
        !p.dst_inst && lds + (size_t)(block / 64) * qw * 4 <= 160 * 1024) {
        q.queue_words = qw;
        lds += (size_t)(block / 64) * qw * 4;
    }
    uint64_t grid = (uint64_t)device_cu_count() * blocks_per_cu((const void*)fn, block, lds);
    if (!far.list) {
        const uint64_t tiles = ((p.n + 3) / 4 + block - 1) / block;
        if (grid > tiles) grid = tiles;
    }
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(block), lds, s, q, far);
    return check_hip(hipGetLastError(), "pass kernel launch");
}

sinet_status launch_pass(const PassParams& p, uint32_t mode, hipStream_t s) {
    if (p.n == 0) return SINET_OK;
    const uint32_t kind = (mode & PASS_LABEL_IN) ? (uint32_t)KK_LABEL_IN : p.t.kind;
    const bool hist = (mode & PASS_HIST) != 0;
    FarList none{};
    return launch_k_pass(p, kind, hist ? H_ATOMIC : H_NONE, vector_ok(p, kind, hist), none, 0, s);
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

static sinet_status launch_zero32(uint32_t* p, uint64_t n, hipStream_t s) {
    if (n == 0) return SINET_OK;
    uint64_t blocks = (n + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(k_zero32, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return check_hip(hipGetLastError(), "zero kernel launch");
}

// ---- workspace of the partitioned histogram --------------------------------
static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Persistent stage-2 workgroups: as many as fit on the device at once.
static uint32_t stage2_grid(uint32_t n_blocks) {
    static const uint32_t per_cu = (uint32_t)blocks_per_cu((const void*)k_stage2, kStage2Block, 0);
    const uint64_t g = (uint64_t)device_cu_count() * (per_cu ? per_cu : 1u);
    return (uint32_t)(g < n_blocks ? g : n_blocks);
}

size_t part_ws_bytes(uint64_t n, uint32_t n_bins) {
    const uint64_t nc = (n + kChunk - 1) / kChunk;
    const uint64_t nb = (n_bins + kBlockBins - 1) / kBlockBins;
    const uint64_t nt = (nb + 1 + 1023) / 1024;
    return al256(4 * nc * kChunkSlots) + al256(16 * nc * kWin) +
           al256(4 * nc) + al256(4 * nc * (kChunk / 32)) + al256(4 * (nc + 1)) + al256(4 * nb) +
           al256(4 * (nb + 1)) + al256(8 * nc * kWin) + al256(4 * nt) + 256;
}

PartWs part_ws_carve(void* base, uint64_t n, uint32_t n_bins) {
    PartWs w{};
    const uint64_t nc = (n + kChunk - 1) / kChunk;
    const uint64_t nb = (n_bins + kBlockBins - 1) / kBlockBins;
    const uint64_t nt = (nb + 1 + 1023) / 1024;
    char* a = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) { char* r = a + o; o += al256(bytes); return (void*)r; };
    w.rec = (uint32_t*)take(4 * nc * kChunkSlots);
    w.dir = (uint4*)take(16 * nc * kWin);
    w.nd = (uint32_t*)take(4 * nc);
    w.farbits = (uint32_t*)take(4 * nc * (kChunk / 32));
    w.farlist = (uint32_t*)take(4 * (nc + 1));
    w.seg_count = (uint32_t*)take(4 * nb);
    w.seg_off = (uint32_t*)take(4 * (nb + 1));
    w.segs = (uint2*)take(8 * nc * kWin);
    w.scan_tiles = (uint32_t*)take(4 * nt);
    w.farcount = (uint32_t*)take(256);
    w.next_run = w.farcount + 1;
    w.n_chunks = nc;
    w.n_blocks = (uint32_t)nb;
    return w;
}

// Segment index: exclusive scan of the per-block directory counts, then the
// fill that groups directory entries by block.
sinet_status launch_scan_fill(const PartWs& w, hipStream_t s) {
    const uint32_t nb = w.n_blocks;
    const uint32_t ntiles = (nb + 1 + 1023) / 1024;
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(1024), 0, s, w.seg_count, nb, w.scan_tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, w.scan_tiles, ntiles);
    hipLaunchKernelGGL(k_scan_final, dim3(ntiles), dim3(1024), 0, s, w.seg_count, nb, w.scan_tiles,
                       w.seg_off);
    uint64_t fb = (w.n_chunks * kWin + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 16;
    if (fb > cap) fb = cap;
    if (fb < 1) fb = 1;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)fb), dim3(256), 0, s, w);
    return check_hip(hipGetLastError(), "segment index launch");
}

// ---- phase timing ------------------------------------------------------------
// While enabled, every phase of run_hist is bracketed by two events recorded on
// the launch stream; they are read (and destroyed) by timing_read.
namespace {
struct Mark {
    int phase;
    hipEvent_t a, b;
};
std::mutex g_tm_mu;
bool g_tm_on = false;
std::vector<Mark> g_tm_marks;
uint64_t g_tm_calls = 0;
uint64_t g_tm_window = 0;

class PhaseScope {
   public:
    PhaseScope(int phase, hipStream_t s, bool enabled = true) : phase_(phase), s_(s) {
        if (!enabled) return;
        {
            std::lock_guard<std::mutex> g(g_tm_mu);
            if (!g_tm_on) return;
        }
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        if (hipEventCreate(&a_) != hipSuccess) return;
        if (hipEventCreate(&b_) != hipSuccess) {
            (void)hipEventDestroy(a_);
            return;
        }
        on_ = hipEventRecord(a_, s) == hipSuccess;
        if (!on_) {
            (void)hipEventDestroy(a_);
            (void)hipEventDestroy(b_);
        }
    }
    ~PhaseScope() {
        if (!on_) return;
        (void)hipEventRecord(b_, s_);
        std::lock_guard<std::mutex> g(g_tm_mu);
        g_tm_marks.push_back(Mark{phase_, a_, b_});
    }
    PhaseScope(const PhaseScope&) = delete;
    PhaseScope& operator=(const PhaseScope&) = delete;

   private:
    int phase_;
    hipStream_t s_;
    hipEvent_t a_{}, b_{};
    bool on_ = false;
};

void count_timed_call() {
    std::lock_guard<std::mutex> g(g_tm_mu);
    if (g_tm_on) ++g_tm_calls;
}

void count_window_call() {
    std::lock_guard<std::mutex> g(g_tm_mu);
    if (g_tm_on) ++g_tm_window;
}

void drop_marks_locked() {
    for (const Mark& m : g_tm_marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    g_tm_marks.clear();
    g_tm_calls = 0;
    g_tm_window = 0;
}
}  // namespace

sinet_status timing_enable(int on) {
    std::lock_guard<std::mutex> g(g_tm_mu);
    if (on) drop_marks_locked();
    g_tm_on = on != 0;
    return SINET_OK;
}

sinet_status timing_read(double ms[PH_COUNT], uint64_t* calls, uint64_t* stage1_launches,
                         uint64_t* window_calls) {
    std::lock_guard<std::mutex> g(g_tm_mu);
    for (int k = 0; k < PH_COUNT; ++k) ms[k] = 0.0;
    *stage1_launches = 0;
    for (const Mark& m : g_tm_marks) {
        float t = 0.f;
        sinet_status st = check_hip(hipEventSynchronize(m.b), "timing event");
        if (st == SINET_OK) st = check_hip(hipEventElapsedTime(&t, m.a, m.b), "timing event");
        if (st != SINET_OK) return st;
        ms[m.phase] += t;
        if (m.phase == PH_STAGE1) ++*stage1_launches;
    }
    *calls = g_tm_calls;
    *window_calls = g_tm_window;
    return SINET_OK;
}

// Histogram of one stream by the partitioned path (workspace given).
sinet_status run_partitioned(const PassParams& p0, uint32_t kind, const PartWs& w, int accumulate,
                             hipStream_t s) {
    PassParams p = p0;
    const bool vec = vector_ok(p, kind, true);
    PartWs wv = w;
    wv.vec = vec ? 1u : 0u;
    sinet_status st = launch_zero32(w.seg_count, w.n_blocks, s);
    if (st == SINET_OK) st = launch_zero32(w.farcount, 2, s);  // far count, run counter
    if (st != SINET_OK) return st;
    Stage1Fn f1 = pick_stage1(kind);
    const size_t lds = (kind == KK_LABEL_IN ? 0 : p.t.lds_bytes) + 8;
    if (lds + kStage1StaticLds > 160 * 1024)
        return fail(SINET_ERR_UNSUPPORTED, "table needs more LDS than a CU has");
    uint64_t grid = (uint64_t)device_cu_count() * blocks_per_cu((const void*)f1, kStage1Block, lds);
    if (grid > w.n_chunks) grid = w.n_chunks;
    if (grid < 1) grid = 1;
    {
        PhaseScope ph(PH_STAGE1, s);
        hipLaunchKernelGGL(f1, dim3((unsigned)grid), dim3(kStage1Block), lds, s, p, wv);
        st = check_hip(hipGetLastError(), "stage-1 launch");
    }
    if (st != SINET_OK) return st;
    const uint32_t nb = w.n_blocks;
    {
        PhaseScope ph(PH_INDEX, s);
        st = launch_scan_fill(wv, s);
    }
    if (st != SINET_OK) return st;
    {
        PhaseScope ph(PH_STAGE2, s);
        const uint32_t g2 = stage2_grid(nb);
        hipLaunchKernelGGL(k_stage2, dim3(g2), dim3(kStage2Block), 0, s, wv, p.count, p.hbytes,
                           p.n_bins, accumulate);
        st = check_hip(hipGetLastError(), "stage-2 launch");
    }
    if (st != SINET_OK) return st;
    // far sessions: labels are already stored, do not store them twice
    FarList far{w.farlist, w.farcount, w.farbits};
    PassParams q = p;
    q.label_out = nullptr;
    q.src_inst = nullptr;
    q.dst_inst = nullptr;
    q.dropped = nullptr;
    PhaseScope ph(PH_FAR, s);
    return launch_k_pass(q, kind, H_ATOMIC, false, far, 0, s);
}

// ---- batch launches -----------------------------------------------------------
using BatchFn = void (*)(BatchArgs, PartWs);

static BatchFn pick_batch_stage1(uint32_t kind) {
    switch (kind) {
        case KK_SCAN: return k_batch_stage1<KK_SCAN>;
        case KK_BSEARCH: return k_batch_stage1<KK_BSEARCH>;
        case KK_TRIE: return k_batch_stage1<KK_TRIE>;
        case KK_PLA: return k_batch_stage1<KK_PLA>;
        case KK_MLP: return k_batch_stage1<KK_MLP>;
        case KK_INOUT: return k_batch_stage1_o4<KK_INOUT>;
        case KK_LABEL_IN: return k_batch_stage1_o4<KK_LABEL_IN>;
        default: return nullptr;
    }
}

static BatchFn pick_batch_far(uint32_t kind) {
    switch (kind) {
        case KK_SCAN: return k_batch_far<KK_SCAN>;
        case KK_BSEARCH: return k_batch_far<KK_BSEARCH>;
        case KK_TRIE: return k_batch_far<KK_TRIE>;
        case KK_PLA: return k_batch_far<KK_PLA>;
        case KK_MLP: return k_batch_far<KK_MLP>;
        case KK_INOUT: return k_batch_far<KK_INOUT>;
        case KK_LABEL_IN: return k_batch_far<KK_LABEL_IN>;
        default: return nullptr;
    }
}

using LookupFn = void (*)(BatchArgs);

static LookupFn pick_batch_lookup(uint32_t kind) {
    switch (kind) {
        case KK_BSEARCH: return k_batch_lookup<KK_BSEARCH>;
        case KK_TRIE: return k_batch_lookup<KK_TRIE>;
        case KK_PLA: return k_batch_lookup<KK_PLA>;
        case KK_MLP: return k_batch_lookup<KK_MLP>;
        default: return nullptr;
    }
}

sinet_status launch_batch_lookup(uint32_t kind, const BatchArgs& a, size_t lds, uint32_t grid,
                                 hipStream_t s) {
    LookupFn fn = pick_batch_lookup(kind);
    if (!fn) return fail(SINET_ERR_UNSUPPORTED, "no batch lookup kernel for this kind");
    if (lds + sizeof(BatchStreamDev) + 16 > 160 * 1024)
        return fail(SINET_ERR_UNSUPPORTED, "batch needs more LDS than a CU has");
    const int block = lds > 40 * 1024 ? kMaxBlock : 256;
    // the window PLA's search queues (for a whole block of the largest size)
    // when they fit beside the group's largest table
    BatchArgs b = a;
    b.queue_words = 0;
    const size_t qbytes = (size_t)(kMaxBlock / 64) * kPlaQueue * 4;
    if (kind == KK_PLA && lds + qbytes + sizeof(BatchStreamDev) + 16 <= 160 * 1024) {
        b.queue_words = kPlaQueue;
        lds += qbytes;
    }
    if (grid == 0) grid = device_cu_count() * blocks_per_cu((const void*)fn, block, lds);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, s, b);
    return check_hip(hipGetLastError(), "batch lookup launch");
}

uint32_t batch_stage1_blocks_per_cu(uint32_t kind, size_t lds) {
    BatchFn fn = pick_batch_stage1(kind);
    return fn ? (uint32_t)blocks_per_cu((const void*)fn, kStage1Block, lds) : 1u;
}

sinet_status launch_batch_stage1(uint32_t kind, const BatchArgs& a, const PartWs& w, size_t lds,
                                 uint32_t grid, hipStream_t s) {
    BatchFn fn = pick_batch_stage1(kind);
    if (!fn) return fail(SINET_ERR_UNSUPPORTED, "no batch kernel for this lookup kind");
    if (lds + kStage1StaticLds + sizeof(BatchStreamDev) + 16 > 160 * 1024)
        return fail(SINET_ERR_UNSUPPORTED, "batch needs more LDS than a CU has");
    if (grid == 0) grid = device_cu_count() * blocks_per_cu((const void*)fn, kStage1Block, lds);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kStage1Block), lds, s, a, w);
    return check_hip(hipGetLastError(), "batch stage-1 launch");
}

sinet_status launch_batch_stage2(const BatchArgs& a, const PartWs& w, uint32_t n_blocks,
                                 hipStream_t s) {
    if (n_blocks == 0) return SINET_OK;
    hipLaunchKernelGGL(k_batch_stage2, dim3(stage2_grid(n_blocks)), dim3(kStage2Block), 0, s, a, w);
    return check_hip(hipGetLastError(), "batch stage-2 launch");
}

sinet_status launch_batch_far(uint32_t kind, const BatchArgs& a, const PartWs& w, size_t lds,
                              hipStream_t s) {
    BatchFn fn = pick_batch_far(kind);
    if (!fn) return fail(SINET_ERR_UNSUPPORTED, "no batch kernel for this lookup kind");
    const int block = lds > 40 * 1024 ? 1024 : 256;
    const uint32_t grid = device_cu_count() * blocks_per_cu((const void*)fn, block, lds);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(block), lds, s, a, w);
    return check_hip(hipGetLastError(), "batch far launch");
}

sinet_status launch_zero_jobs(const ZeroJob* jobs, uint32_t n_jobs, hipStream_t s) {
    if (n_jobs == 0) return SINET_OK;
    uint32_t grid = n_jobs < 4096 ? n_jobs : 4096;
    hipLaunchKernelGGL(k_zero_jobs, dim3(grid), dim3(256), 0, s, jobs, n_jobs);
    return check_hip(hipGetLastError(), "zero launch");
}

// ---- per-device pool for the stream-ordered workspace ------------------------
static hipMemPool_t device_pool(int dev) {
    static std::mutex mu;
    static std::map<int, hipMemPool_t> pools;
    std::lock_guard<std::mutex> g(mu);
    auto it = pools.find(dev);
    if (it != pools.end()) return it->second;
    hipMemPoolProps props;
    memset(&props, 0, sizeof(props));
    props.allocType = hipMemAllocationTypePinned;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    if (hipMemPoolCreate(&pool, &props) != hipSuccess) pool = nullptr;
    if (pool) {
        uint64_t thr = ~0ull;  // keep freed blocks for reuse
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    pools[dev] = pool;
    return pool;
}

sinet_status ws_alloc(void** ptr, size_t bytes, hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return check_hip(e, "hipGetDevice");
    hipMemPool_t pool = device_pool(dev);
    e = pool ? hipMallocFromPoolAsync(ptr, bytes, pool, s) : hipMallocAsync(ptr, bytes, s);
    return check_hip(e, "workspace allocation");
}

sinet_status ws_free(void* ptr, hipStream_t s) {
    return check_hip(hipFreeAsync(ptr, s), "workspace free");
}

constexpr int H_WINDOW = 4;

// Which reduce the histogram calls use (sinet_set_reduce).
static std::atomic<int> g_reduce{SINET_REDUCE_AUTO};

sinet_status set_reduce(int mode) {
    if (mode != SINET_REDUCE_AUTO && mode != SINET_REDUCE_RECORDS && mode != SINET_REDUCE_WINDOW)
        return fail(SINET_ERR_INVALID_ARG, "unknown reduce");
    g_reduce.store(mode);
    return SINET_OK;
}

// Histogram strategy for a window: small windows are privatised in LDS; long
// inputs take the sliding-window reduce, the rest the partitioned records.
// The window reduce has about 0.7 ms of fixed cost per call (its pieces'
// boundary fix-up and far pass, and the write-out of bins its few sessions
// leave behind); on the day shape with 86.4 M 1-ms bins it was measured at
// 2.25 ms against 1.82 ms for the records with 1e8 sessions and 3.38 against
// 3.70 ms with 4e8, a crossover near 2.7e8 sessions.
constexpr uint64_t kWindowMinSessions = 1ull << 28;

int hist_strategy(const DevTable& t, uint32_t kind, uint32_t n_bins, uint64_t n) {
    const size_t priv = 12ull * 4 * n_bins;
    const size_t tab = kind == KK_LABEL_IN ? 0 : t.lds_bytes;
    if (n_bins <= 2048 && priv + tab + 64 <= 96 * 1024) return H_PRIVATE;
    const int mode = g_reduce.load();
    if (mode == SINET_REDUCE_WINDOW) return H_WINDOW;
    if (mode == SINET_REDUCE_AUTO && n >= kWindowMinSessions) return H_WINDOW;
    return 3;  // partitioned
}

// Lookups that walk global memory (trie, learned windows, binary searches
// with a global leaf) run as their own pass before stage 1.
bool lookup_splits(const DevTable& t) {
    return t.kind == KK_TRIE || t.kind == KK_PLA || t.kind == KK_MLP ||
           (t.kind == KK_BSEARCH && t.top_log2 > 0);
}

// The columns advanced by off sessions.
static PassParams advance(const PassParams& p, uint64_t off) {
    PassParams q = p;
    q.n = p.n - off;
    auto a32 = [&](const uint32_t* x) { return x ? x + off : x; };
    q.ts = a32(p.ts);
    q.src = a32(p.src);
    q.dst = a32(p.dst);
    q.bytes = p.bytes ? p.bytes + off : nullptr;
    q.label_in = p.label_in ? p.label_in + off : nullptr;
    q.label_out = p.label_out ? p.label_out + off : nullptr;
    q.src_inst = p.src_inst ? p.src_inst + off : nullptr;
    q.dst_inst = p.dst_inst ? p.dst_inst + off : nullptr;
    return q;
}

// Sliding-window reduce (window.hip): the labels first (a lookup pass that
// stores them, unless they are given), then the window pass, the fix-up of
// the bins at the pieces' boundaries and the far path.
// With the workspace given: ws holds win_ws_bytes(n, P) bytes, then (when a
// lookup pass runs and the caller stores no labels) n bytes of labels.
static sinet_status run_window_in(const PassParams& p, uint32_t kind, int accumulate, hipStream_t s,
                                  void* ws, uint32_t P, bool timed) {
    const size_t wsb = win_ws_bytes(p.n, P);
    const bool lookup = kind != KK_LABEL_IN;
    sinet_status st = SINET_OK;
    PassParams q = p;
    if (lookup) {
        PassParams lq = p;
        if (!lq.label_out) lq.label_out = (uint8_t*)ws + wsb;
        lq.pos_out = nullptr;
        FarList none{};
        PhaseScope ph(PH_LOOKUP, s, timed);
        st = launch_k_pass(lq, kind, H_NONE, vector_ok(lq, kind, false), none, 0, s);
        q.label_in = lq.label_out;
    }
    q.label_out = nullptr;
    q.src_inst = nullptr;
    q.dst_inst = nullptr;
    const WinArgs a = win_carve(ws, q, P, accumulate);
    if (st == SINET_OK) {
        PhaseScope ph(PH_INDEX, s, timed);
        st = win_launch_bounds(a, s);
    }
    if (st == SINET_OK) {
        PhaseScope ph(PH_STAGE1, s, timed);
        st = win_launch_main(a, s);
    }
    if (st == SINET_OK) {
        PhaseScope ph(PH_STAGE2, s, timed);
        st = win_launch_fixup(a, s);
    }
    if (st == SINET_OK) {
        PhaseScope ph(PH_FAR, s, timed);
        st = win_launch_far(a, s);
    }
    return st;
}

static size_t window_ws_total(const PassParams& p, uint32_t kind, uint32_t P) {
    const bool lookup = kind != KK_LABEL_IN;
    return win_ws_bytes(p.n, P) + (lookup && !p.label_out ? al256(p.n) : 0);
}

static sinet_status run_window(const PassParams& p, uint32_t kind, int accumulate, hipStream_t s) {
    const uint32_t P = win_pieces(p.n);
    void* ws = nullptr;
    sinet_status st = ws_alloc(&ws, window_ws_total(p, kind, P), s);
    if (st != SINET_OK) return st;
    count_window_call();
    st = run_window_in(p, kind, accumulate, s, ws, P, true);
    const sinet_status st2 = ws_free(ws, s);
    return st != SINET_OK ? st : st2;
}

// The histogram of run_hist with its workspace taken from `scratch` (bytes
// long) instead of allocated: the private pass for small windows (no
// workspace), else the sliding-window reduce with as many pieces as fit.
// Records no timing events.
sinet_status run_hist_in(const PassParams& p, uint32_t mode, int accumulate, hipStream_t s,
                         void* scratch, size_t bytes) {
    const uint32_t kind = (mode & PASS_LABEL_IN) ? (uint32_t)KK_LABEL_IN : p.t.kind;
    if (p.n == 0) return SINET_OK;
    if (hist_strategy(p.t, kind, p.n_bins, p.n) == H_PRIVATE) {
        sinet_status st = SINET_OK;
        if (!accumulate) {
            st = launch_zero(p.count, 4ull * p.n_bins, s);
            if (st == SINET_OK) st = launch_zero(p.hbytes, 4ull * p.n_bins, s);
            if (st != SINET_OK) return st;
        }
        FarList none{};
        return launch_k_pass(p, kind, H_PRIVATE, vector_ok(p, kind, true), none,
                             12ull * 4 * p.n_bins + 8, s);
    }
    uint32_t P = win_pieces(p.n);
    while (P > 1 && window_ws_total(p, kind, P) > bytes) P = P * 3 / 4;
    if (window_ws_total(p, kind, P) > bytes)
        return fail(SINET_ERR_INVALID_ARG, "input too large for the static scratch");
    return run_window_in(p, kind, accumulate, s, scratch, P, false);
}

sinet_status run_hist(const PassParams& p, uint32_t mode, int accumulate, hipStream_t s) {
    const uint32_t kind = (mode & PASS_LABEL_IN) ? (uint32_t)KK_LABEL_IN : p.t.kind;
    if (p.n == 0) return SINET_OK;
    if (!vector_ok(p, kind, true)) {
        // columns that all sit h sessions short of 16-byte alignment (slices of
        // aligned arrays): the aligned rest takes the vector path, then the first
        // h sessions are added by the atomic pass
        for (uint64_t h = 1; h < 4 && h < p.n; ++h) {
            if (!vector_ok(advance(p, h), kind, true)) continue;
            sinet_status st = run_hist(advance(p, h), mode, accumulate, s);
            if (st != SINET_OK) return st;
            PassParams head = p;
            head.n = h;
            FarList none{};
            return launch_k_pass(head, kind, H_ATOMIC, false, none, 0, s);
        }
    }
    count_timed_call();
    const int strat = hist_strategy(p.t, kind, p.n_bins, p.n);
    if (strat == H_PRIVATE) {
        sinet_status st = SINET_OK;
        if (!accumulate) {
            st = launch_zero(p.count, 4ull * p.n_bins, s);
            if (st == SINET_OK) st = launch_zero(p.hbytes, 4ull * p.n_bins, s);
            if (st != SINET_OK) return st;
        }
        FarList none{};
        PhaseScope ph(PH_STAGE1, s);
        return launch_k_pass(p, kind, H_PRIVATE, vector_ok(p, kind, true), none,
                             12ull * 4 * p.n_bins + 8, s);
    }
    if (strat == H_WINDOW) return run_window(p, kind, accumulate, s);
    // partitioned: pieces of at most kMaxPiece sessions (32-bit slot indices)
    int acc = accumulate;
    for (uint64_t lo = 0; lo < p.n; lo += kMaxPiece) {
        PassParams q = p;
        const uint64_t len = p.n - lo < kMaxPiece ? p.n - lo : kMaxPiece;
        q.n = len;
        auto adv32 = [&](const uint32_t* a) { return a ? a + lo : a; };
        q.ts = adv32(p.ts);
        q.src = adv32(p.src);
        q.dst = adv32(p.dst);
        q.bytes = p.bytes ? p.bytes + lo : nullptr;
        q.label_in = p.label_in ? p.label_in + lo : nullptr;
        q.label_out = p.label_out ? p.label_out + lo : nullptr;
        q.src_inst = p.src_inst ? p.src_inst + lo : nullptr;
        q.dst_inst = p.dst_inst ? p.dst_inst + lo : nullptr;
        // Lookups that walk global memory (trie, learned windows, large binary
        // searches) run as their own barrier-free pass; stage 1 then reads the
        // labels (1 byte per session) instead of stalling its barriers on them.
        const bool split = kind != KK_LABEL_IN && lookup_splits(p.t);
        const size_t wsb = part_ws_bytes(len, p.n_bins);
        const size_t lab_bytes = split && !q.label_out ? ((len + 255) & ~(uint64_t)255) : 0;
        void* ws = nullptr;
        sinet_status st = ws_alloc(&ws, wsb + lab_bytes, s);
        if (st != SINET_OK) return st;
        const PartWs w = part_ws_carve(ws, len, p.n_bins);
        uint32_t k2 = kind;
        if (split) {
            PassParams lq = q;
            if (!lq.label_out) lq.label_out = (uint8_t*)ws + wsb;
            lq.pos_out = nullptr;
            FarList none{};
            PhaseScope ph(PH_LOOKUP, s);
            st = launch_k_pass(lq, kind, H_NONE, vector_ok(lq, kind, false), none, 0, s);
            q.label_in = lq.label_out;
            q.label_out = nullptr;
            q.src_inst = nullptr;
            q.dst_inst = nullptr;
            k2 = KK_LABEL_IN;
        }
        if (st == SINET_OK) st = run_partitioned(q, k2, w, acc, s);
        sinet_status st2 = ws_free(ws, s);
        if (st != SINET_OK) return st;
        if (st2 != SINET_OK) return st2;
        acc = 1;
    }
    return SINET_OK;
}


// ---- watch-list histograms ----------------------------------------------------
using WatchFn = void (*)(WatchParams);

template <uint32_t KIND>
static WatchFn watch_fn(bool priv) {
    return priv ? k_watch<KIND, true> : k_watch<KIND, false>;
}

static WatchFn pick_watch(uint32_t kind, bool priv) {
    switch (kind) {
        case KK_SCAN: return watch_fn<KK_SCAN>(priv);
        case KK_BSEARCH: return watch_fn<KK_BSEARCH>(priv);
        case KK_TRIE: return watch_fn<KK_TRIE>(priv);
        case KK_PLA: return watch_fn<KK_PLA>(priv);
        case KK_MLP: return watch_fn<KK_MLP>(priv);
        default: return nullptr;
    }
}

sinet_status run_watch(const PassParams& p, uint32_t n_keys, int accumulate, hipStream_t s) {
    const uint64_t cells = 2ull * n_keys * p.n_bins;
    sinet_status st = SINET_OK;
    if (!accumulate) {
        st = launch_zero(p.count, cells, s);
        if (st == SINET_OK) st = launch_zero(p.hbytes, cells, s);
        if (st == SINET_OK && p.dropped) st = launch_zero(p.dropped, 4, s);
        if (st != SINET_OK) return st;
    }
    if (p.n == 0) return SINET_OK;
    const uint32_t kind = p.t.kind;
    // the table, each wave's search queue and the interval keys (interval
    // kinds), the private cells
    const bool lds_keys = kind != KK_SCAN && p.t.m <= kWatchLdsKeys;
    const size_t table_lds = (size_t)p.t.lds_bytes +
                             (kind == KK_SCAN ? 0 : 4 * 512 * (kWatchBlock / 64)) +
                             (lds_keys ? 4ull * p.t.m : 0) + 8;
    const bool priv = cells <= kWatchPrivCells && table_lds + 12 * cells + 8 <= 64 * 1024;
    WatchFn fn = pick_watch(kind, priv);
    if (!fn) return fail(SINET_ERR_UNSUPPORTED, "no watch kernel for this lookup kind");
    const size_t lds = table_lds + (priv ? 12 * cells + 8 : 0);
    if (lds > 160 * 1024) return fail(SINET_ERR_UNSUPPORTED, "table needs more LDS than a CU has");
    WatchParams w;
    w.p = p;
    w.n_keys = n_keys;
    w.vec = aligned16(p.src) && aligned16(p.dst) && aligned16(p.ts) && aligned16(p.bytes) ? 1u : 0u;
    w.lds_keys = lds_keys ? 1u : 0u;
    w.pad = 0;
    uint64_t grid = (uint64_t)device_cu_count() * blocks_per_cu((const void*)fn, kWatchBlock, lds);
    const uint64_t tiles = ((p.n + 3) / 4 + kWatchBlock - 1) / kWatchBlock;
    if (grid > tiles) grid = tiles;
    if (grid < 1) grid = 1;
    count_timed_call();
    PhaseScope ph(PH_LOOKUP, s);
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(kWatchBlock), lds, s, w);
    return check_hip(hipGetLastError(), "watch kernel launch");
}

}  // namespace sinet
