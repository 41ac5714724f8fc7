// In/out index: membership of an address in the union of all prefixes of a
// table (the two-way in/out mark of Algorithm 1 without the institution),
// answered from LDS with two 8-byte reads and no data-dependent loop in the
// common case.
//
// Layout (u32 words):
//   [0, 2 * 4096)  per group of 16 consecutive /16 blocks: one word with, in
//                  bits 0..15, block k's membership at its first address and,
//                  in bits 16..31, whether a union boundary cuts block k;
//                  then the byte offset of the group's first cut block's
//                  slot in the slot region (8 x the number of cut blocks in
//                  all earlier groups);
//   slot           one 8-byte slot per cut block, in address order (then a
//                  zero pad slot): the block's union boundaries b (offsets
//                  1..65535 inside the block) stored as b - 1, ascending,
//                  padded with 0xFFFF; a block with more than four boundaries
//                  instead holds 0xFFFF, its boundary count, and the u16
//                  offset of its sorted offsets in the overflow list;
//   list           the overflow list (u16 pairs).
// The membership of a = (block << 16) | x in a cut block is its starting
// state flipped once per boundary b <= x, i.e. by the parity of the number of
// stored offsets b - 1 < x.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace sinet {

constexpr uint32_t kIoGroups = 65536 / 16;
constexpr uint32_t kIoSlotWords = 2;
constexpr uint32_t kIoSlotMax = 4;  // boundaries held in a slot

struct IoLayout {
    uint32_t slot;   // word offset of the slots
    uint32_t list;   // word offset of the overflow list
    uint32_t words;  // total
    uint32_t cut;    // number of cut blocks
};

// Build from the sorted boundaries U of the union (every address where the
// membership changes, in ascending order, starting outside at address 0).
// Returns false when a count does not fit its field.
inline bool build_inout_index(const std::vector<uint32_t>& U, std::vector<uint32_t>& io,
                              IoLayout& lay) {
    std::vector<uint32_t> groups(2 * kIoGroups, 0), slots, list;
    size_t u = 0;
    bool state = false;
    uint32_t cut = 0;
    for (uint64_t k = 0; k < 65536; ++k) {
        if ((k & 15) == 0) groups[2 * (k >> 4) + 1] = 8 * cut;  // bytes into the slot region
        const uint64_t base = k << 16;
        while (u < U.size() && U[u] == base) {  // a boundary at the block's first address
            state = !state;
            ++u;
        }
        const bool s0 = state;
        const size_t u0 = u;
        while (u < U.size() && ((uint64_t)U[u] >> 16) == k) {
            state = !state;
            ++u;
        }
        uint32_t st = s0 ? 1u : 0u;
        if (u != u0) {
            st |= 1u << 16;
            const size_t nb = u - u0;
            if (nb <= kIoSlotMax) {
                uint32_t e[kIoSlotMax];
                for (size_t i = 0; i < kIoSlotMax; ++i)
                    e[i] = i < nb ? (U[u0 + i] & 0xFFFFu) - 1u : 0xFFFFu;
                slots.push_back(e[0] | (e[1] << 16));
                slots.push_back(e[2] | (e[3] << 16));
            } else {
                if (nb > 0xFFFF || list.size() > 0x7FFFFFFF) return false;
                slots.push_back(0xFFFFu | ((uint32_t)nb << 16));
                slots.push_back((uint32_t)list.size());
                for (size_t i = u0; i < u; ++i) list.push_back(U[i] & 0xFFFFu);
            }
            ++cut;
        }
        groups[2 * (k >> 4)] |= st << (k & 15);
    }
    slots.push_back(0u);  // pad slot: read, never used, by uncut blocks past the last cut
    slots.push_back(0u);
    io.assign(groups.begin(), groups.end());
    lay.slot = (uint32_t)io.size();
    io.insert(io.end(), slots.begin(), slots.end());
    lay.list = (uint32_t)io.size();
    for (size_t i = 0; i < list.size(); i += 2)
        io.push_back(list[i] | (i + 1 < list.size() ? list[i + 1] << 16 : 0u));
    lay.words = (uint32_t)io.size();
    lay.cut = cut;
    return true;
}

// Number of entries <= x among the n sorted u16 offsets at list[off..).
__host__ __device__ inline uint32_t io_count_le(const uint32_t* list, uint32_t off, uint32_t n,
                                                uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint32_t i = off + mid;
        const uint32_t b = (list[i >> 1] >> ((i & 1u) * 16)) & 0xFFFFu;
        if (b <= x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Membership (0/1) of N addresses.  io is 8-byte aligned.  The group and
// slot reads of all N addresses are issued before any is used.  Block k of a
// group: in = bit k, cut = bit 16 + k; the slot of a cut block follows the
// group's first slot by the cut blocks before k in the group.  Only the
// parity of the boundaries <= x matters.
template <int N>
__host__ __device__ inline void inout_lookup(const uint32_t* io, uint32_t slot_off,
                                             uint32_t list_off, const uint32_t* a, uint32_t* in) {
    const uint2* grp = reinterpret_cast<const uint2*>(io);
    const uint2* slot = reinterpret_cast<const uint2*>(io + slot_off);
    uint2 g[N], s[N];
    uint32_t t[N];
#pragma unroll
    for (int q = 0; q < N; ++q) g[q] = grp[a[q] >> 20];
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const uint32_t k = (a[q] >> 16) & 15u;
        t[q] = g[q].x >> k;                                   // bit 0: in, bit 16: cut
#ifdef __HIP_DEVICE_COMPILE__
        const uint32_t before = __builtin_amdgcn_ubfe(g[q].x, 16u, k);  // cut blocks before k
#else
        const uint32_t before = (g[q].x >> 16) & ((1u << k) - 1u);
#endif
        s[q] = *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(slot) + g[q].y +
                                               8u * (uint32_t)__builtin_popcount(before));
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const uint32_t x = a[q] & 0xFFFFu;
        uint32_t odd = ((s[q].x & 0xFFFFu) < x) ^ ((s[q].x >> 16) < x) ^ ((s[q].y & 0xFFFFu) < x) ^
                       ((s[q].y >> 16) < x);
        // a slot marking a block with more than four boundaries (read also by
        // uncut lanes whose next cut block it is; the cut bit below masks them)
        if ((s[q].x & 0xFFFFu) == 0xFFFFu)
            odd = io_count_le(io + list_off, s[q].y, s[q].x >> 16, x) & 1u;
        in[q] = (t[q] ^ (odd & (t[q] >> 16))) & 1u;
    }
}

}  // namespace sinet
