// Sliding-window histogram: the Map and Reduce steps of the paper in one
// streaming pass over labelled sessions, for gfx950.
//
// Method (Ando et al., arXiv 2106.12863, sections "Map", "Reduce" and "Merge
// Scatter Pattern with CPU"): every session maps to the key (label, bin),
// bin = floor((ts - t0) / width), with the value (1, bytes); values merge by
// unsigned 64-bit addition, which is associative and commutative, so any
// grouping of the additions gives the exact histogram.
//
// Design.  Session logs are nearly sorted by time (a session's timestamp
// lies within a few seconds of its position's time), so a contiguous index
// range of sessions touches a time range of bins that moves forward as the
// range is walked.  Each workgroup takes one such range (a piece) and keeps
// the bins it currently touches in LDS: a ring of kWinBins bins, one 32-bit
// word per (bin, label).  Bins that the window leaves are complete for the
// piece and are written out once; nothing goes through device memory twice.
//   * Ownership.  A pre-pass cuts the time axis at the pieces' boundaries
//     (T[q], the median bin of 64 sessions around the piece's first
//     session, made non-decreasing).  Piece q owns bins [T[q], T[q+1]) and
//     writes every one of them (zeros included), so the histogram needs no
//     zero-fill.  Its sessions that fall into the neighbours' bins (the time
//     jitter around a boundary) are flushed into two spill rows of kWinBins
//     bins (the packed ring words), which a small fix-up pass decodes and
//     adds into the neighbours' bins.
//   * Ring word.  count (5 bits) << 27 | byte sum (27 bits), one LDS atomic
//     add of 2^27 + bytes per session; sessions with 2^22 bytes or more go
//     to the far path, so the byte field cannot carry before the count field
//     wraps.  Every add whose returned old value shows a carry out of the
//     byte field or out of the 32-bit word records an event; with the events
//     the decode (count = w >> 27, bytes = w & (2^27 - 1)) plus (-1, +2^27)
//     per carry and (+32, 0) per wrap is exact for any number of sessions.
//     At most n/32 carries and n/32 + n/1024 wraps can happen, so the event
//     list is bounded.
//   * Sliding.  A lane holds 4 consecutive sessions; a step is 4,096
//     sessions.  A session whose bin is inside the current window is added at
//     once.  The others of a step are pending: the step's largest pending bin
//     decides how far the window moves; the bins it leaves are flushed, and
//     the pending sessions are added into the moved window.  On input whose
//     timestamps lie within +-(kWinBins - 16) / 2 bins of a non-decreasing
//     sequence no session is ever late.
//   * Far path.  Sessions late for the window, outside the piece's reach, or
//     with large byte counts are marked in a per-step bitmap; a last pass
//     re-reads them and adds them, and the events, with device-scope
//     atomics, after every bin has been written.  Any input stays exact.
//   * Issue cost.  A wave64 vector instruction holds a 16-lane SIMD for four
//     cycles, so the per-session path is kept to a few dozen instructions;
//     barriers wait for LDS only (lds_barrier), so the next steps' loads stay
//     in flight across them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pass_common.h"
#include "sinet_internal.h"

namespace sinet {

constexpr uint32_t kWinLanes = 1024;                  // lanes of a window workgroup
constexpr uint32_t kWinWaves = kWinLanes / 64;
constexpr uint32_t kStepWords = kWinStep / 32;        // far-bitmap words of a step
constexpr uint32_t kCountShift = 27;                  // ring word: count << 27 | bytes
constexpr uint32_t kLowMask = (1u << kCountShift) - 1u;
constexpr uint64_t kRingMaxBytes = 1ull << 22;        // larger byte counts take the far path
constexpr uint32_t kWinLead = 160;                    // bins the window's end leads after a move
static_assert(kWinStep == 4 * kWinLanes, "four sessions per lane");
static_assert(kWinBins % 16 == 0, "window moves in steps of 16 bins");
static_assert(32ull * ((1ull << 22) - 1) < (1ull << 27), "no carry before the count wraps");

__device__ __forceinline__ bool win_bin(const WinArgs& a, uint32_t ts, uint32_t& bin) {
    bin = bin_of(ts - a.t0, a.width, a.magic);
    return ts >= a.t0 && bin < a.n_bins;
}

__device__ __forceinline__ uint64_t piece_begin(uint64_t n, uint32_t P, uint32_t q) {
    const uint64_t steps = (n + kWinStep - 1) / kWinStep;
    const uint64_t b = (steps * q / P) * kWinStep;
    return b < n ? b : n;
}

// ---------------------------------------------------------------------------
// Boundaries of the pieces.  est[q] (q > 0) is the median bin of the 64
// sessions around piece q's first session (0 for sessions before the window,
// n_bins after it); piece q then owns [T[q], T[q+1]) with T[q] the running
// maximum of est[0..q] (est[0] = 0) and T[P] = n_bins, so every bin has one
// owner.  One wave per piece; workgroup 0 also clears the counters.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_window_bounds(WinArgs a) {
    const uint32_t lane = threadIdx.x, q = blockIdx.x;
    if (q == 0) {
        if (lane < 4) a.counters[lane] = 0;
        if (lane == 0) a.est[0] = 0;
        return;
    }
    const uint64_t b = piece_begin(a.n, a.pieces, q);
    uint64_t i = b + lane >= 32 ? b + lane - 32 : 0;
    if (i >= a.n) i = a.n - 1;
    const uint32_t ts = *glob(a.ts + i);
    uint32_t bin;
    const uint32_t v = win_bin(a, ts, bin) ? bin : (ts < a.t0 ? 0u : a.n_bins);
    // rank among the 64 values (ties by lane): the lane of rank 32 holds the median
    uint32_t rank = 0;
    for (int k = 0; k < 64; ++k) {
        const uint32_t o = (uint32_t)__shfl((int)v, k);
        rank += (o < v || (o == v && (uint32_t)k < lane)) ? 1u : 0u;
    }
    if (rank == 32u) a.est[q] = v;
}

// T[q + k] for k = -1 .. 2 (running maxima of est; T[P] = n_bins), by wave 0;
// broadcast through LDS.
__device__ __forceinline__ void win_owned(const WinArgs& a, uint32_t q, uint32_t* s_t, uint32_t t[4]) {
    const uint32_t P = a.pieces, lane = threadIdx.x & 63u;
    if (threadIdx.x < 64) {
        uint32_t m[4] = {0u, 0u, 0u, 0u};  // max of est[0..q-1], [0..q], [0..q+1], [0..q+2]
        for (uint32_t j = lane; j <= q + 2 && j < P; j += 64) {
            const uint32_t e = *glob(a.est + j);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (j + 1 <= q + (uint32_t)k) m[k] = max(m[k], e);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t r = ~wave_min(~m[k]);
            const uint32_t idx = q + (uint32_t)k;  // T index q - 1 + k, shifted by one
            if (lane == 0) s_t[k] = idx == 0 ? 0u : (idx - 1 >= P ? a.n_bins : min(r, a.n_bins));
        }
    }
    lds_barrier();
#pragma unroll
    for (int k = 0; k < 4; ++k) t[k] = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_t[k]);  // uniform
}

// ---------------------------------------------------------------------------
// The window pass.
// ---------------------------------------------------------------------------
struct WinPiece {
    uint32_t q, Tq, Tq1;   // the piece, its owned bins [Tq, Tq1)
    uint32_t L, R;         // bins the piece may hold: [L, R)
};

// Write bins [lo, hi): those inside the window [W0, W0 + kWinBins) from the
// ring (clearing their words), the rest as zeros; bins below Tq go to the
// piece's left spill rows, bins from Tq1 on to its right spill rows (the
// packed ring word, 4 bytes per bin and label), the others to the output.  Wave w takes label w % 4 and the bins lo + 64 (w / 4)
// + lane, + 256, ..., so the waves that have no bin return at once.  Called
// by the whole workgroup with uniform arguments.  Accumulation is a template
// parameter: a load here makes the wave wait for every load in flight, the
// prefetched sessions included.
template <bool ACC>
__device__ __forceinline__ void win_flush(const WinArgs& a, const WinPiece& g, uint32_t* ring, bool wset,
                                          uint32_t W0, uint32_t r0, uint64_t lo, uint64_t hi) {
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    const uint64_t x0 = lo + 64ull * (wave >> 2);
    if (x0 >= hi) return;  // wave-uniform
    const uint32_t l = wave & 3u;
    const uint64_t lrow = ((uint64_t)g.q * 2 + 0) * 4 + l;
    const uint64_t rrow = ((uint64_t)g.q * 2 + 1) * 4 + l;
    uint32_t* lw = a.spill + lrow * kWinBins + kWinBins - g.Tq;  // + x, x in [Tq - kWinBins, Tq)
    uint32_t* rw = a.spill + rrow * kWinBins - g.Tq1;            // + x, x in [Tq1, Tq1 + kWinBins)
    unsigned long long* oc = a.count + (uint64_t)l * a.n_bins;
    const uint64_t ob = (uint64_t)(a.hbytes - a.count);  // output byte row - count row
    const uint32_t trips = (uint32_t)((hi - x0 + 255) / 256);
    uint32_t x = (uint32_t)x0 + lane;
    for (uint32_t t = 0; t < trips; ++t, x += 256u) {
        if ((uint64_t)x0 + 256ull * t + lane >= hi) break;
        uint32_t w = 0u;
        const uint32_t off = x - W0;
        if (wset && x >= W0 && off < kWinBins) {
            uint32_t pos = r0 + off;
            pos = pos >= kWinBins ? pos - kWinBins : pos;
            w = ring[pos * 4 + l];
            ring[pos * 4 + l] = 0u;
        }
        if (x >= g.Tq && x < g.Tq1) {  // owned: the bin's count and byte sum
            unsigned long long vc = w >> kCountShift, vb = w & kLowMask;
            unsigned long long* dc = oc + x;
            unsigned long long* db = dc + ob;
            if constexpr (ACC) {
                vc += *glob(dc);
                vb += *glob(db);
            }
            __builtin_nontemporal_store(vc, glob(dc));
            __builtin_nontemporal_store(vb, glob(db));
        } else {  // a neighbour's: the ring word itself, decoded by the fix-up
            __builtin_nontemporal_store(w, glob(x < g.Tq ? lw + x : rw + x));
        }
    }
}

// Carry / wrap events of one add (rare: only a bin with more than 32
// sessions of one label, or 2^27 bytes, in one window).
__device__ __forceinline__ void win_event(const WinArgs& a, uint32_t bin, uint32_t lab, uint32_t carry,
                                          uint32_t wrap) {
    const uint32_t k = carry + wrap;
    const uint32_t e = atomicAdd(a.counters + 1, k);
    const unsigned long long key = ((unsigned long long)bin << 3) | (lab << 1);
    uint32_t j = e;
    if (carry && j < a.ev_cap) a.events[j++] = key;
    if (wrap && j < a.ev_cap) a.events[j] = key | 1ull;
    if (e + k > a.ev_cap) atomicOr(a.counters + 2, 1u);
}

// Events of one add of `add` to a ring word that held `old` (bit 0 carry
// out of the byte field, bit 1 wrap of the word).  The carry into bit 27 of
// old + add is bit 27 of old ^ add ^ sum.  An add of 0 has none.
__device__ __forceinline__ uint32_t win_events(uint32_t old, uint32_t add) {
    const uint32_t sum = old + add;
    const uint32_t carry = ((old ^ add ^ sum) >> kCountShift) & 1u;
    const uint32_t wrap = sum < old ? 2u : 0u;
    return carry | wrap;
}

// Four consecutive sessions of one lane.
struct WinRaw {
    uint4 ts;
    ulonglong2 b01, b23;
    uint32_t l4;
};

// Sessions i .. i + 3 (all below the piece's end): 16-byte loads when the
// columns allow them.
template <bool VEC>
__device__ __forceinline__ void win_load_full(const WinArgs& a, uint64_t i, WinRaw& r) {
    if constexpr (VEC) {  // streamed once: nontemporal loads
        const u32x4_t t = __builtin_nontemporal_load(glob(reinterpret_cast<const u32x4_t*>(a.ts + i)));
        const u64x2_t b0 = __builtin_nontemporal_load(glob(reinterpret_cast<const u64x2_t*>(a.bytes + i)));
        const u64x2_t b1 = __builtin_nontemporal_load(glob(reinterpret_cast<const u64x2_t*>(a.bytes + i + 2)));
        r.ts = make_uint4(t.x, t.y, t.z, t.w);
        r.b01 = make_ulonglong2(b0.x, b0.y);
        r.b23 = make_ulonglong2(b1.x, b1.y);
        r.l4 = __builtin_nontemporal_load(glob(reinterpret_cast<const uint32_t*>(a.label + i)));
    } else {
        r.ts = make_uint4(*glob(a.ts + i), *glob(a.ts + i + 1), *glob(a.ts + i + 2), *glob(a.ts + i + 3));
        r.b01 = make_ulonglong2(*glob(a.bytes + i), *glob(a.bytes + i + 1));
        r.b23 = make_ulonglong2(*glob(a.bytes + i + 2), *glob(a.bytes + i + 3));
        r.l4 = (uint32_t)*glob(a.label + i) | ((uint32_t)*glob(a.label + i + 1) << 8) |
               ((uint32_t)*glob(a.label + i + 2) << 16) | ((uint32_t)*glob(a.label + i + 3) << 24);
    }
}

// The sessions of i .. i + 3 that lie below i1 (the last step of a piece).
__device__ __forceinline__ void win_load_tail(const WinArgs& a, uint64_t i, uint64_t i1, WinRaw& r) {
    uint32_t t[4] = {0u, 0u, 0u, 0u}, l4 = 0u;
    unsigned long long b[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i + k < i1) {
            t[k] = *glob(a.ts + i + k);
            b[k] = *glob(a.bytes + i + k);
            l4 |= (uint32_t)*glob(a.label + i + k) << (8 * k);
        }
    }
    r.ts = make_uint4(t[0], t[1], t[2], t[3]);
    r.b01 = make_ulonglong2(b[0], b[1]);
    r.b23 = make_ulonglong2(b[2], b[3]);
    r.l4 = l4;
}

// Window state of a workgroup (every value uniform).
struct WinState {
    bool wset;                 // the window is placed
    uint32_t W0, r0, V;        // window start, its ring slot, first spill bin written
    uint32_t par;              // exchange buffer of this step
    uint32_t nfar_steps;       // steps listed with far sessions
    unsigned long long prev_far;  // this wave's lanes with far sessions, previous step
    uint32_t prev_word;        // far bits of 32 sessions of the previous step (per 8 lanes)
    uint64_t prev_step;        // first session of the previous step
};

// List the previous step as holding far sessions: every wave writes its 8
// bitmap words (zeros included), lane 0 the list entry.
__device__ __forceinline__ void win_list_far(const WinArgs& a, WinState& st, uint64_t i0) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint64_t sidx = st.prev_step / kWinStep;
    if ((lane & 7u) == 0) a.far_bits[sidx * kStepWords + wave * 8 + (lane >> 3)] = st.prev_word;
    if (tid == 0) a.far_steps[i0 / kWinStep + st.nfar_steps] = (uint32_t)sidx;
    ++st.nfar_steps;
}

// One step: the lane's four sessions from session s0 + 4 * tid on.  FULL:
// every one of them is below the piece's end i1.
template <bool ACC, bool FULL>
__device__ __forceinline__ void win_step(const WinArgs& a, const WinPiece& g, uint32_t* ring,
                                         uint4 (*s_x)[kWinWaves], WinState& st, Dropped& d,
                                         const WinRaw& cur, uint64_t s0, uint64_t i0, uint64_t i1) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint64_t i = s0 + 4ull * tid;
    const uint32_t tsv[4] = {cur.ts.x, cur.ts.y, cur.ts.z, cur.ts.w};
    const unsigned long long byv[4] = {cur.b01.x, cur.b01.y, cur.b23.x, cur.b23.y};
    // the fast path: a session inside the piece's reach whose bin is in the
    // window goes straight into its ring word; one beyond the window's end is
    // pending (added after the window moves); the rest (dropped: outside the
    // histogram; far: outside the piece's reach, large byte counts, or late
    // for the window) take the rare path
    const uint32_t Wn = st.wset ? kWinBins : 0u;
    const uint32_t Wl = st.wset ? st.W0 : 0u;
    const uint32_t delta = st.r0 - st.W0;  // ring slot = bin + delta (mod 2^32), less kWinBins
    uint32_t bin[4], lab[4], word[4], add[4];
    uint32_t rest = 0u, pendm = 0u, evm = 0u;  // bit u: session u; its events at bits 2u, 2u + 1
    uint32_t hi1 = 0u, lo = 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        lab[u] = (cur.l4 >> (8 * u)) & 3u;
        bin[u] = bin_of(tsv[u] - a.t0, a.width, a.magic);
        // bitwise &: no short-circuit branches on the common path
        const bool has = FULL || i + u < i1;
        const bool small = ((uint32_t)(byv[u] >> 32) | ((uint32_t)byv[u] >> 22)) == 0u;
        const bool ranged = has & (tsv[u] >= a.t0) & (bin[u] - g.L < g.R - g.L) & small;
        const bool now = ranged & (bin[u] - st.W0 < Wn);
        const bool pend = ranged & !now & (bin[u] >= Wl);
        // every lane adds (0 outside the window, to a word of its own), so the
        // four atomics of a lane are in flight together
        uint32_t pos = bin[u] + delta;
        pos = pos >= kWinBins ? pos - kWinBins : pos;
        word[u] = now ? pos * 4 + lab[u] : (lane * 4 + (u & 3));
        add[u] = now ? (1u << kCountShift) + (uint32_t)byv[u] : 0u;
        pendm |= pend ? 1u << u : 0u;
        hi1 = max(hi1, pend ? bin[u] + 1u : 0u);
        lo = min(lo, pend ? bin[u] : 0xFFFFFFFFu);
        rest |= (has & !now & !pend) ? 1u << u : 0u;
    }
    {
        uint32_t old[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) old[u] = atomicAdd(ring + word[u], add[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) evm |= win_events(old[u], add[u]) << (2 * u);
    }
    uint32_t farm = 0u;
    if (rest) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (!((rest >> u) & 1u)) continue;
            if (tsv[u] >= a.t0 && bin[u] < a.n_bins) farm |= 1u << u;
            else d.add(lab[u], byv[u]);
        }
    }
    // exchange: the step's pending extent, the previous step's far ballots
    {
        const uint32_t h = wave_min(~hi1);  // ~max(bin + 1)
        const uint32_t m = wave_min(lo);
        if (lane == 0)
            s_x[st.par][wave] = make_uint4(h, m, (uint32_t)st.prev_far, (uint32_t)(st.prev_far >> 32));
    }
    lds_barrier();
    uint32_t H, Lo;
    bool any_far;
    {
        uint4 x = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u);
        if (lane < kWinWaves) x = s_x[st.par][lane];
        any_far = __ballot((x.z | x.w) != 0u) != 0ull;
        // minimum over lanes 0..15 (one DPP row): lane 15 ends with it
        uint32_t xh = x.x, xl = x.y;
        xh = dpp_min_step<0x111, 0xF>(xh);
        xl = dpp_min_step<0x111, 0xF>(xl);
        xh = dpp_min_step<0x112, 0xF>(xh);
        xl = dpp_min_step<0x112, 0xF>(xl);
        xh = dpp_min_step<0x114, 0xF>(xh);
        xl = dpp_min_step<0x114, 0xF>(xl);
        xh = dpp_min_step<0x118, 0xF>(xh);
        xl = dpp_min_step<0x118, 0xF>(xl);
        H = ~(uint32_t)__builtin_amdgcn_readlane((int)xh, 15);
        Lo = (uint32_t)__builtin_amdgcn_readlane((int)xl, 15);
    }
    st.par ^= 1u;
    if (any_far) win_list_far(a, st, i0);  // the previous step had far sessions
    if (H) {  // pending sessions: place or move the window
        const uint32_t M = H - 1u;
        uint32_t lead = kWinLead;
        if (!st.wset) {  // placed at the lowest pending bin, which must stay inside
            st.W0 = max(g.L, Lo & ~15u);
            st.r0 = 0;
            st.V = min(st.W0, g.Tq);
            win_flush<ACC>(a, g, ring, false, st.W0, st.r0, st.V, st.W0);  // below the window: zeros
            st.wset = true;
            lead = 0;
        }
        if ((uint64_t)M >= (uint64_t)st.W0 + kWinBins) {
            // the window's end leads the largest pending bin by kWinLead bins
            // (fewer pending sessions next step); its start stays more than
            // 2 * 5000 bins behind that bin
            const uint64_t nw = ((uint64_t)M + lead - kWinBins + 1 + 15) & ~(uint64_t)15;
            win_flush<ACC>(a, g, ring, true, st.W0, st.r0, st.W0, nw);
            st.r0 = (uint32_t)(((uint64_t)st.r0 + (nw - st.W0)) % kWinBins);
            st.W0 = (uint32_t)nw;
            lds_barrier();  // the flushed words are clear before they are reused
        }
        if (pendm) {
            const uint32_t dl = st.r0 - st.W0;
            uint32_t old[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool p = (pendm >> u) & 1u;
                const bool in = p & (bin[u] >= st.W0) & (bin[u] - st.W0 < kWinBins);
                uint32_t pos = bin[u] + dl;
                pos = pos >= kWinBins ? pos - kWinBins : pos;
                word[u] = in ? pos * 4 + lab[u] : (lane * 4 + (u & 3));
                add[u] = in ? (1u << kCountShift) + (uint32_t)byv[u] : 0u;
                farm |= (p & !in) ? 1u << u : 0u;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) old[u] = atomicAdd(ring + word[u], add[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u) evm |= win_events(old[u], add[u]) << (2 * u);
        }
    }
    if (evm) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t e = (evm >> (2 * u)) & 3u;
            if (e) win_event(a, bin[u], lab[u], e & 1u, e >> 1);
        }
    }
    // far bits: session 4 * tid + u of the step is bit (4 * tid + u) % 32 of
    // word tid / 8; the 8 lanes of a word OR their nibbles together
    {
        uint32_t w = farm << (4u * (lane & 7u));
        w |= (uint32_t)__shfl_xor((int)w, 1);
        w |= (uint32_t)__shfl_xor((int)w, 2);
        w |= (uint32_t)__shfl_xor((int)w, 4);
        st.prev_word = w;
        st.prev_far = __ballot(farm != 0u);
    }
    st.prev_step = s0;
}

template <bool ACC, bool VEC>
__global__ void __launch_bounds__(kWinLanes) k_window(WinArgs a) {
    __shared__ __attribute__((aligned(16))) uint32_t ring[kWinBins * 4];
    __shared__ uint4 s_x[2][kWinWaves];  // per wave: ~max(bin + 1), min bin, far ballot
    uint4* ring4 = reinterpret_cast<uint4*>(ring);
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t P = a.pieces;
    __shared__ uint32_t s_t[4];
    WinPiece g;
    g.q = blockIdx.x;
    {
        uint32_t t[4];  // T[q - 1], T[q], T[q + 1], T[q + 2]
        win_owned(a, g.q, s_t, t);
        g.Tq = t[1];
        g.Tq1 = t[2];
        g.L = max(t[0], g.Tq >= kWinBins ? g.Tq - kWinBins : 0u);
        const uint64_t r = (uint64_t)g.Tq1 + kWinBins;
        g.R = (uint32_t)(r < t[3] ? r : t[3]);
        if (threadIdx.x == 0) {
            a.T[g.q] = g.Tq;
            if (g.q + 1 == P) a.T[P] = g.Tq1;
        }
    }
    const uint64_t i0 = piece_begin(a.n, P, g.q), i1 = piece_begin(a.n, P, g.q + 1);
    for (uint32_t k = tid; k < kWinBins; k += kWinLanes) ring4[k] = make_uint4(0u, 0u, 0u, 0u);
    lds_barrier();

    Dropped d{};
    WinState st{};
    st.V = g.Tq;
    const uint64_t nfull = (i1 - i0) / kWinStep;
    // full steps, two in flight: step s of this lane sits in r[s % 2].  The
    // loads are unconditional (the last two steps load the piece's last full
    // step again), so the compiler can wait for exactly the step it needs.
    WinRaw r[2];
    if (nfull > 0) {
        const uint64_t last = i0 + (nfull - 1) * kWinStep + 4ull * tid;
        win_load_full<VEC>(a, i0 + 4ull * tid, r[0]);
        win_load_full<VEC>(a, min(i0 + kWinStep + 4ull * tid, last), r[1]);
        for (uint64_t s = 0; s < nfull; s += 2) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (s + k >= nfull) break;  // uniform
                const uint64_t s0 = i0 + (s + k) * kWinStep;
                const WinRaw cur = r[k];
                win_load_full<VEC>(a, min(s0 + 2ull * kWinStep + 4ull * tid, last), r[k]);
                win_step<ACC, true>(a, g, ring, s_x, st, d, cur, s0, i0, i1);
            }
        }
    }
    if (i0 + nfull * kWinStep < i1) {  // the piece's last, partial step
        const uint64_t s0 = i0 + nfull * kWinStep;
        WinRaw t;
        win_load_tail(a, s0 + 4ull * tid, i1, t);
        win_step<ACC, false>(a, g, ring, s_x, st, d, t, s0, i0, i1);
    }
    // the last step's far ballots, then the remaining window
    if (lane == 0)
        s_x[st.par][wave] = make_uint4(0u, 0u, (uint32_t)st.prev_far, (uint32_t)(st.prev_far >> 32));
    lds_barrier();
    {
        uint4 x = make_uint4(0u, 0u, 0u, 0u);
        if (lane < kWinWaves) x = s_x[st.par][lane];
        const bool any_far = __ballot((x.z | x.w) != 0u) != 0ull;
        if (any_far && i1 > i0) win_list_far(a, st, i0);
    }
    uint64_t end = g.Tq1;
    if (st.wset) {
        end = (uint64_t)st.W0 + kWinBins;
        if (end > g.R) end = g.R;
        if (end < g.Tq1) end = g.Tq1;
    } else {
        st.W0 = g.Tq;
        st.r0 = 0;
        st.V = g.Tq;
    }
    win_flush<ACC>(a, g, ring, st.wset, st.W0, st.r0, st.W0, end);
    if (tid == 0) {
        a.V[g.q] = st.V;
        a.E[g.q] = (uint32_t)end;
        a.far_n[g.q] = st.nfar_steps;
    }
    d.flush(a.dropped);
}

// ---------------------------------------------------------------------------
// Fix-up: owner q adds piece q-1's right spill ([T[q], E[q-1])) and piece
// q+1's left spill ([V[q+1], T[q+1])) into its bins; one lane per bin, so a
// bin in both ranges is read and written once.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_window_fixup(WinArgs a) {
    const uint32_t q = blockIdx.x, P = a.pieces;
    const uint32_t Tq = a.T[q], Tq1 = a.T[q + 1];
    const uint32_t ea = q > 0 ? min(a.E[q - 1], Tq1) : Tq;         // [Tq, ea) from the left
    const uint32_t vb = q + 1 < P ? max(a.V[q + 1], Tq) : Tq1;     // [vb, Tq1) from the right
    auto one = [&](uint32_t x) {
        const bool fa = x < ea, fb = x >= vb;
#pragma unroll
        for (uint32_t l = 0; l < 4; ++l) {
            unsigned long long vc = 0, vby = 0;  // the spilled ring words, decoded
            if (fa) {
                const uint64_t row = ((uint64_t)(q - 1) * 2 + 1) * 4 + l;
                const uint32_t w = *glob(a.spill + row * kWinBins + (x - Tq));
                vc += w >> kCountShift;
                vby += w & kLowMask;
            }
            if (fb) {
                const uint64_t row = ((uint64_t)(q + 1) * 2 + 0) * 4 + l;
                const uint32_t w = *glob(a.spill + row * kWinBins + (x + kWinBins - Tq1));
                vc += w >> kCountShift;
                vby += w & kLowMask;
            }
            unsigned long long* dc = a.count + (uint64_t)l * a.n_bins + x;
            unsigned long long* db = a.hbytes + (uint64_t)l * a.n_bins + x;
            *glob(dc) = *glob(dc) + vc;
            *glob(db) = *glob(db) + vby;
        }
    };
    if (ea >= vb) {
        for (uint64_t x = (uint64_t)Tq + threadIdx.x; x < Tq1; x += blockDim.x)
            if (x < ea || x >= vb) one((uint32_t)x);
    } else {
        for (uint64_t x = (uint64_t)Tq + threadIdx.x; x < ea; x += blockDim.x) one((uint32_t)x);
        for (uint64_t x = (uint64_t)vb + threadIdx.x; x < Tq1; x += blockDim.x) one((uint32_t)x);
    }
}

// ---------------------------------------------------------------------------
// Far path: the marked sessions and the events, with device-scope atomics,
// after every bin has been written.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_window_far(WinArgs a) {
    // blockIdx.y: the piece; lanes of the x blocks take its listed steps' bitmap
    // words, 32 sessions each
    {
        const uint32_t q = blockIdx.y;
        const uint64_t first = piece_begin(a.n, a.pieces, q) / kWinStep;
        const uint64_t nwords = (uint64_t)a.far_n[q] * kStepWords;
        for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nwords;
             t += (uint64_t)gridDim.x * blockDim.x) {
            const uint64_t st = a.far_steps[first + t / kStepWords];
            const uint32_t wd = (uint32_t)(t % kStepWords);
            uint32_t bits = a.far_bits[st * kStepWords + wd];
            while (bits) {
                const uint32_t b = __builtin_ctz(bits);
                bits &= bits - 1u;
                const uint64_t i = st * kWinStep + wd * 32 + b;
                const uint32_t ts = *glob(a.ts + i);
                const unsigned long long by = *glob(a.bytes + i);
                const uint32_t lab = *glob(a.label + i) & 3u;
                uint32_t bin = 0;
                if (!win_bin(a, ts, bin)) continue;  // marked sessions are inside; kept for safety
                const uint64_t k = (uint64_t)lab * a.n_bins + bin;
                __hip_atomic_fetch_add(a.count + k, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(a.hbytes + k, by, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (blockIdx.y != 0) return;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nev = min(a.counters[1], (uint32_t)a.ev_cap);
    for (uint64_t e = t0; e < nev; e += stride) {
        const unsigned long long key = a.events[e];
        const uint64_t k = ((key >> 1) & 3ull) * a.n_bins + (key >> 3);
        if (key & 1ull) {  // wrap: 32 sessions the count field lost
            __hip_atomic_fetch_add(a.count + k, 32ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {  // carry: 2^27 bytes that went into the count field
            __hip_atomic_fetch_add(a.count + k, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(a.hbytes + k, 1ull << kCountShift, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t al256w(size_t x) { return (x + 255) & ~(size_t)255; }

uint32_t win_pieces(uint64_t n) {
    uint64_t P = device_cu_count();
    const uint64_t steps = (n + kWinStep - 1) / kWinStep;
    if (P > steps) P = steps;
    if (P > 1024) P = 1024;
    return (uint32_t)(P < 1 ? 1 : P);
}

uint64_t win_event_cap(uint64_t n) { return n / 15 + 1024; }

size_t win_ws_bytes(uint64_t n, uint32_t P) {
    const uint64_t steps = (n + kWinStep - 1) / kWinStep;
    return al256w(4ull * (P + 1)) + 4 * al256w(4ull * P) + al256w(16) + al256w(4ull * steps) +
           al256w(4ull * kStepWords * steps) + al256w(8ull * win_event_cap(n)) +
           al256w(4ull * P * 2 * 4 * kWinBins);
}

WinArgs win_carve(void* base, const PassParams& p, uint32_t P, int accumulate) {
    WinArgs a{};
    const uint64_t steps = (p.n + kWinStep - 1) / kWinStep;
    char* c = (char*)base;
    size_t o = 0;
    auto take = [&](size_t bytes) { char* r = c + o; o += al256w(bytes); return (void*)r; };
    a.ts = p.ts;
    a.bytes = p.bytes;
    a.label = p.label_in;
    a.count = p.count;
    a.hbytes = p.hbytes;
    a.dropped = p.dropped;
    a.n = p.n;
    a.magic = p.magic;
    a.t0 = p.t0;
    a.width = p.width;
    a.n_bins = p.n_bins;
    a.T = (uint32_t*)take(4ull * (P + 1));
    a.est = (uint32_t*)take(4ull * P);
    a.V = (uint32_t*)take(4ull * P);
    a.E = (uint32_t*)take(4ull * P);
    a.counters = (uint32_t*)take(16);
    a.far_n = (uint32_t*)take(4ull * P);
    a.far_steps = (uint32_t*)take(4ull * steps);
    a.far_bits = (uint32_t*)take(4ull * kStepWords * steps);
    a.events = (unsigned long long*)take(8ull * win_event_cap(p.n));
    a.spill = (uint32_t*)take(4ull * P * 2 * 4 * kWinBins);
    a.ev_cap = win_event_cap(p.n);
    a.pieces = P;
    a.vec = ((((uintptr_t)p.ts | (uintptr_t)p.bytes) & 15u) == 0 && ((uintptr_t)p.label_in & 3u) == 0)
                ? 1u : 0u;
    a.accumulate = accumulate;
    return a;
}

sinet_status win_launch_bounds(const WinArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_window_bounds, dim3(a.pieces), dim3(64), 0, s, a);
    return check_hip(hipGetLastError(), "window bounds launch");
}

sinet_status win_launch_main(const WinArgs& a, hipStream_t s) {
    auto fn = a.accumulate ? (a.vec ? k_window<true, true> : k_window<true, false>)
                           : (a.vec ? k_window<false, true> : k_window<false, false>);
    hipLaunchKernelGGL(fn, dim3(a.pieces), dim3(kWinLanes), 0, s, a);
    return check_hip(hipGetLastError(), "window pass launch");
}

sinet_status win_launch_fixup(const WinArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_window_fixup, dim3(a.pieces), dim3(1024), 0, s, a);
    return check_hip(hipGetLastError(), "window fix-up launch");
}

sinet_status win_launch_far(const WinArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_window_far, dim3(16, a.pieces), dim3(256), 0, s, a);
    return check_hip(hipGetLastError(), "window far launch");
}

}  // namespace sinet
