// Session text to columns (section "Dataset Description", Table 1: the
// PA-7080 session record, 24 fields).  One record per line, Table 1's fields
// in order separated by ','; the columns come from field 1 (capture_time,
// "YYYY/MM/DD HH:MM:SS.mmm", as milliseconds since midnight of the origin
// day), fields 5 and 8 (source and destination, dotted quads) and field 21
// (bytes).  Every '\n'-ended segment is a line (an empty one too); a last
// segment without '\n' is a line when it is not empty.  A line with fewer
// than 21 fields, an impossible date, a time outside [0, 2^32 - 1) ms of the
// origin, an octet above 255 or a byte count above 2^64 - 1 gives
// ts = 0xFFFFFFFF, src = dst = bytes = 0 and counts as bad.
//
// Three passes over the text:
//   k_count_lines  newlines per 64 KB block (coalesced 16-byte loads);
//   k_scan_counts  one workgroup: exclusive sums of the block counts;
//   k_line_starts  every newline's position + 1 written at its line number;
//   k_parse        a workgroup takes 256 consecutive lines, stages their bytes
//                  in LDS with coalesced loads (as many whole lines at a time
//                  as fit in 64 KB), builds a bitmap of the staged commas
//                  (16 bytes per lane) and each lane finds its line's field
//                  bounds in the bitmap and parses the fields from LDS (a line
//                  longer than the staging is read from device memory
//                  directly).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sinet.h"
#include "sinet_internal.h"

namespace sinet {
namespace {

constexpr int kParseBlock = 256;
constexpr uint64_t kScanBytes = 64 * 1024;    // text bytes per counting block
constexpr uint32_t kStageBytes = 64 * 1024;   // LDS staging of a workgroup's lines
constexpr uint32_t kBadTs = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t nl_in(uint4 v) {
    uint32_t c = 0;
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int b = 0; b < 4; ++b) c += ((w[k] >> (8 * b)) & 0xFFu) == 10u ? 1u : 0u;
    return c;
}

// Newlines of block blockIdx.x ([blk * kScanBytes, +kScanBytes) of the text).
__global__ void __launch_bounds__(kParseBlock) k_count_lines(const uint8_t* __restrict__ text,
                                                             uint64_t len, uint64_t* __restrict__ counts,
                                                             uint32_t vec) {
    __shared__ uint32_t s_sum;
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanBytes;
    const uint64_t b1 = b0 + kScanBytes < len ? b0 + kScanBytes : len;
    uint32_t c = 0;
    if (vec) {
        for (uint64_t p = b0 + 16 * (uint64_t)threadIdx.x; p < b1; p += 16 * kParseBlock) {
            if (p + 16 <= b1) {
                c += nl_in(*reinterpret_cast<const uint4*>(text + p));
            } else {
                for (uint64_t q = p; q < b1; ++q) c += text[q] == 10 ? 1u : 0u;
            }
        }
    } else {
        for (uint64_t p = b0 + threadIdx.x; p < b1; p += kParseBlock) c += text[p] == 10 ? 1u : 0u;
    }
    atomicAdd(&s_sum, c);
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = s_sum;
}

// Exclusive sums of n counts in place, total in counts[n] (one workgroup):
// each 1024-count step scans within waves (shuffles), then adds the totals
// of the waves before and of the steps before.
__global__ void __launch_bounds__(1024) k_scan_counts(uint64_t* __restrict__ counts, uint32_t n) {
    __shared__ uint64_t s_wave[16];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (uint32_t base = 0; base < n; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t x = i < n ? counts[i] : 0ull;
        uint64_t incl = x;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = __shfl_up(incl, d);
            if (lane >= (uint32_t)d) incl += y;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        uint64_t before = s_carry, total = 0;
        for (uint32_t w = 0; w < 16; ++w) {
            if (w < wave) before += s_wave[w];
            total += s_wave[w];
        }
        if (i < n) counts[i] = before + incl - x;
        __syncthreads();  // every lane has read s_wave and s_carry
        if (threadIdx.x == 0) s_carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[n] = s_carry;
}

// starts[k + 1] = position after the k-th newline (starts[0] = 0).  Each step
// of a block reads 64 contiguous bytes per lane (four 16-byte loads); a
// lane's newlines are numbered after the ones of the lanes before it (wave
// scan, then the waves in order).
__device__ __forceinline__ uint64_t nl_bits16(uint4 v) {  // bit i: byte i of v is '\n'
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    uint64_t m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            m |= (uint64_t)(((w[k] >> (8 * q)) & 0xFFu) == 10u ? 1u : 0u) << (4 * k + q);
    return m;
}

__global__ void __launch_bounds__(kParseBlock) k_line_starts(const uint8_t* __restrict__ text,
                                                             uint64_t len,
                                                             const uint64_t* __restrict__ first,
                                                             uint64_t* __restrict__ starts,
                                                             uint32_t vec) {
    __shared__ uint32_t s_wave[kParseBlock / 64];
    __shared__ uint64_t s_base;
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanBytes;
    const uint64_t b1 = b0 + kScanBytes < len ? b0 + kScanBytes : len;
    if (threadIdx.x == 0) {
        s_base = first[blockIdx.x];
        if (blockIdx.x == 0) starts[0] = 0;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (uint64_t st = b0; st < b1; st += 64 * kParseBlock) {
        const uint64_t p = st + 64 * (uint64_t)threadIdx.x;
        uint64_t mask = 0;  // bit q: byte p + q is a newline
        if (vec && p + 64 <= b1) {
            const uint4* v = reinterpret_cast<const uint4*>(text + p);
            const uint4 v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
            mask = nl_bits16(v0) | nl_bits16(v1) << 16 | nl_bits16(v2) << 32 | nl_bits16(v3) << 48;
        } else {
            for (int q = 0; q < 64; ++q)
                if (p + q < b1 && text[p + q] == 10) mask |= 1ull << q;
        }
        const uint32_t c = (uint32_t)__popcll(mask);
        uint32_t incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, d);
            if (lane >= (uint32_t)d) incl += y;
        }
        if (lane == 63) s_wave[wave] = incl;
        __syncthreads();
        uint64_t before = s_base;
        uint32_t step_total = 0;
        for (uint32_t w = 0; w < kParseBlock / 64; ++w) {
            if (w < wave) before += s_wave[w];
            step_total += s_wave[w];
        }
        uint64_t k = before + (incl - c);  // newlines before this lane's first
        while (mask) {
            const uint32_t q = (uint32_t)__builtin_ctzll(mask);
            starts[k + 1] = p + q + 1;
            ++k;
            mask &= mask - 1;
        }
        __syncthreads();  // every lane has read s_wave and s_base
        if (threadIdx.x == 0) s_base += step_total;
        __syncthreads();
    }
}

// days since 1970-01-01 of a proleptic Gregorian date (H. Hinnant's
// days_from_civil)
// (years 0..9999 here: 32-bit arithmetic suffices)
__device__ __forceinline__ int32_t days_from_civil(int32_t y, int32_t m, int32_t d) {
    y -= m <= 2 ? 1 : 0;
    const int32_t era = (y >= 0 ? y : y - 399) / 400;
    const int32_t yoe = y - era * 400;
    const int32_t mp = m > 2 ? m - 3 : m + 9;
    const int32_t doy = (153 * mp + 2) / 5 + d - 1;
    const int32_t doe = yoe * 365 + yoe / 4 - yoe / 100 + doy;
    return era * 146097 + doe - 719468;
}

// Byte access to one line staged in LDS.
struct LdsLine {
    const uint8_t* p;  // the line's first byte
    __device__ __forceinline__ uint32_t operator[](uint32_t i) const { return p[i]; }
    // byte i, or 0xFF at or past e; reads up to 3 bytes past a field's end
    // stay inside the staging (it has 16 bytes of slack), so no branch
    __device__ __forceinline__ uint32_t upto(uint32_t i, uint32_t e) const {
        const uint32_t c = p[i];
        return i < e ? c : 0xFFu;
    }
};

// Byte access to one line in device memory (lines too long for the staging):
// bytes only, never past the line.
struct GlobalLine {
    const uint8_t* p;
    __device__ __forceinline__ uint32_t operator[](uint32_t i) const { return p[i]; }
    __device__ __forceinline__ uint32_t upto(uint32_t i, uint32_t e) const { return i < e ? p[i] : 0xFFu; }
    __device__ __forceinline__ uint32_t comma(uint32_t c, uint32_t n) const {
        while (c < n && p[c] != ',') ++c;
        return c;
    }
};

template <class Bytes>
__device__ __forceinline__ bool dec(const Bytes& b, uint32_t at, int n, int32_t& v) {
    int32_t x = 0;
    for (int i = 0; i < n; ++i) {
        const uint32_t c = b[at + i] - '0';
        if (c > 9u) return false;
        x = x * 10 + c;
    }
    v = x;
    return true;
}

template <class Bytes>
__device__ __forceinline__ bool capture_time(const Bytes& b, uint32_t s, uint32_t e, int64_t origin, uint32_t& ts) {
    if (e - s != 23) return false;
    if (b[s + 4] != '/' || b[s + 7] != '/' || b[s + 10] != ' ' || b[s + 13] != ':' ||
        b[s + 16] != ':' || b[s + 19] != '.')
        return false;
    int32_t y, mo, d, h, mi, se, ms;
    if (!dec(b, s, 4, y) || !dec(b, s + 5, 2, mo) || !dec(b, s + 8, 2, d) || !dec(b, s + 11, 2, h) ||
        !dec(b, s + 14, 2, mi) || !dec(b, s + 17, 2, se) || !dec(b, s + 20, 3, ms))
        return false;
    if (mo < 1 || mo > 12 || d < 1) return false;
    const bool leap = (y % 4 == 0 && y % 100 != 0) || y % 400 == 0;
    // days in month: 31 except April, June, September, November (30) and February
    const int32_t dim = mo == 2 ? (leap ? 29 : 28) : ((mo == 4 || mo == 6 || mo == 9 || mo == 11) ? 30 : 31);
    if (d > dim || h > 23 || mi > 59 || se > 59) return false;
    const int64_t t = ((int64_t)days_from_civil(y, mo, d) - origin) * 86400000 + h * 3600000 +
                      mi * 60000 + se * 1000 + ms;
    if (t < 0 || t >= (int64_t)kBadTs) return false;
    ts = (uint32_t)t;
    return true;
}

template <class Bytes>
__device__ __forceinline__ bool ipv4(const Bytes& b, uint32_t s, uint32_t e, uint32_t& a) {
    if (e - s < 7u || e - s > 15u) return false;  // "1.2.3.4" to "255.255.255.255"
    constexpr uint32_t kDot = (uint32_t)('.' - '0');
    uint32_t v = 0, i = s;
#pragma unroll
    for (int part = 0; part < 4; ++part) {
        // the octet is the digits at i (a fourth one makes it bad); the byte
        // after them must be '.' for parts 0-2 and the field's end for part 3
        const uint32_t d0 = b.upto(i, e) - '0', d1 = b.upto(i + 1, e) - '0';
        const uint32_t d2 = b.upto(i + 2, e) - '0', d3 = b.upto(i + 3, e) - '0';
        if (d0 > 9u) return false;
        const uint32_t nd = d1 > 9u ? 1u : d2 > 9u ? 2u : d3 > 9u ? 3u : 4u;
        if (nd > 3u) return false;
        const uint32_t o = nd == 1u ? d0 : nd == 2u ? d0 * 10 + d1 : d0 * 100 + d1 * 10 + d2;
        if (o > 255u) return false;
        const uint32_t next = nd == 1u ? d1 : nd == 2u ? d2 : d3;
        v = (v << 8) | o;
        i += nd;
        if (part < 3) {
            if (next != kDot) return false;
            ++i;
        }
    }
    if (i != e) return false;
    a = v;
    return true;
}

template <class Bytes>
__device__ __forceinline__ bool count_u64(const Bytes& b, uint32_t s, uint32_t e, uint64_t& out) {
    if (e <= s || e - s > 20) return false;
    // 19 digits stay below 10^19 < 2^64 - 1, so only a 20th digit can
    // overflow; the digits before it are taken four at a time
    const uint32_t last = e - s == 20 ? e - 1 : e;
    uint64_t v = 0;
    for (uint32_t i = s; i < last; i += 4) {
        const uint32_t k = last - i < 4u ? last - i : 4u;  // digits in this group
        const uint32_t d0 = b.upto(i, last) - '0', d1 = b.upto(i + 1, last) - '0';
        const uint32_t d2 = b.upto(i + 2, last) - '0', d3 = b.upto(i + 3, last) - '0';
        if (d0 > 9u || (k > 1u && d1 > 9u) || (k > 2u && d2 > 9u) || (k > 3u && d3 > 9u)) return false;
        const uint32_t g2 = d0 * 10 + d1, g3 = g2 * 10 + d2;
        const uint32_t g = k == 1u ? d0 : k == 2u ? g2 : k == 3u ? g3 : g3 * 10 + d3;
        const uint32_t p10 = k == 1u ? 10u : k == 2u ? 100u : k == 3u ? 1000u : 10000u;
        v = v * p10 + g;
    }
    if (last != e) {
        const uint32_t c = b[last] - '0';
        if (c > 9u) return false;
        // v * 10 + c > 2^64 - 1 = 18446744073709551615 exactly when v exceeds
        // floor((2^64 - 1) / 10), or equals it and c > 5
        if (v > 1844674407370955161ull || (v == 1844674407370955161ull && c > 5u)) return false;
        v = v * 10 + c;
    }
    out = v;
    return true;
}

// Parse the line [0, n) of b; false for a bad line.
template <class Bytes>
__device__ __forceinline__ bool parse_line(const Bytes& b, uint32_t n, int64_t origin, uint32_t& ts, uint32_t& src,
                           uint32_t& dst, uint64_t& nbytes) {
    uint32_t s = 0;
    for (int f = 1; f <= 21; ++f) {
        const uint32_t c = b.comma(s, n);
        // field f is [s, c)
        if (f == 1 && !capture_time(b, s, c, origin, ts)) return false;
        if (f == 5 && !ipv4(b, s, c, src)) return false;
        if (f == 8 && !ipv4(b, s, c, dst)) return false;
        if (f == 21) return count_u64(b, s, c, nbytes);
        if (c >= n) return false;  // the line ended before field 21
        s = c + 1;
    }
    return false;
}

// Bit i of the result: byte i of the 16 bytes v is ','.  The zero-byte test
// is exact per byte: for x = word ^ 0x2C2C2C2C, bit 7 of each byte of
// ((x & 0x7F7F7F7F) + 0x7F7F7F7F) | x is set exactly when that byte of x is
// not zero (the sums stay inside their bytes).  The four words' flags are
// gathered first (bit 8 b + q: byte b of word q), then packed to 16 bits
// (bit 4 b + q) and the 4 x 4 bit matrix is transposed (bit 4 q + b).
__device__ __forceinline__ uint32_t comma_bits16(uint4 v) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t x = w[q] ^ 0x2C2C2C2Cu;
        const uint32_t t = ((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x;  // bit 7 of a byte: not a comma
        s |= (t >> (7 - q)) & (0x01010101u << q);
    }
    s ^= 0x0F0F0F0Fu;
    uint32_t y = (s | (s >> 4)) & 0x00FF00FFu;
    y = (y | (y >> 8)) & 0xFFFFu;
    uint32_t t = (y ^ (y >> 3)) & 0x0A0Au;
    y ^= t ^ (t << 3);
    t = (y ^ (y >> 6)) & 0x00CCu;
    y ^= t ^ (t << 6);
    return y;
}

// Position of the r-th (1-based) set bit of m, r <= popcount(m).
__device__ __forceinline__ uint32_t nth_bit(uint32_t m, uint32_t r) {
    uint32_t pos = 0;
    uint32_t c = (uint32_t)__popc(m & 0xFFFFu);
    if (r > c) { r -= c; m >>= 16; pos += 16; }
    c = (uint32_t)__popc(m & 0xFFu);
    if (r > c) { r -= c; m >>= 8; pos += 8; }
    c = (uint32_t)__popc(m & 0xFu);
    if (r > c) { r -= c; m >>= 4; pos += 4; }
    c = (uint32_t)__popc(m & 0x3u);
    if (r > c) { r -= c; m >>= 2; pos += 2; }
    return pos + (r > (m & 1u) ? 1u : 0u);
}

// parse_line for a line staged in LDS at staging bytes [b0, b1), with the
// staging's comma bitmap (bit i of word j: staged byte 32 j + i is ',').
// The line's bitmap words give its comma count and, for commas 1, 4, 7 and
// 20, the word that holds each and its rank there; commas 5, 8 and 21 are
// the next set bits after 4, 7 and 20 (comma 21 is the line's end when the
// line has exactly 20).  Field f is [comma f-1 + 1, comma f).  Same rules as
// parse_line.
__device__ __forceinline__ bool parse_line_lds(const uint8_t* stage, const uint32_t* bits, uint32_t b0,
                                               uint32_t b1, int64_t origin, uint32_t& ts, uint32_t& src,
                                               uint32_t& dst, uint64_t& nbytes) {
    if (b1 <= b0) return false;  // an empty line has one field
    const uint32_t w0 = b0 >> 5, w1 = (b1 - 1) >> 5;
    const uint32_t lo = 0xFFFFFFFFu << (b0 & 31u);
    const uint32_t hi = 0xFFFFFFFFu >> (31u - ((b1 - 1) & 31u));
    auto word = [&](uint32_t w) {  // the line's commas in bitmap word w
        uint32_t m = bits[w];
        if (w == w0) m &= lo;
        if (w == w1) m &= hi;
        return m;
    };
    uint32_t k = 0;  // commas in the words before w
    uint32_t wa = 0, ra = 0, wb = 0, rb = 0, wc = 0, rc = 0, wd = 0, rd = 0;
    for (uint32_t w = w0; w <= w1; ++w) {
        const uint32_t c = (uint32_t)__popc(word(w));
        // comma t is in word w when k < t <= k + c
        if (0u - k < c) { wa = w; ra = 1u - k; }
        if (3u - k < c) { wb = w; rb = 4u - k; }
        if (6u - k < c) { wc = w; rc = 7u - k; }
        if (19u - k < c) { wd = w; rd = 20u - k; }
        k += c;
    }
    if (k < 20) return false;  // fewer than 21 fields
    // stage position of the first comma after bit q of word w, or b1
    auto after = [&](uint32_t w, uint32_t q) {
        uint32_t m = word(w) & (0xFFFFFFFEu << q);
        while (!m && w < w1) m = word(++w);
        return m ? 32 * w + (uint32_t)__builtin_ctz(m) : b1;
    };
    const uint32_t q1 = nth_bit(word(wa), ra), q4 = nth_bit(word(wb), rb);
    const uint32_t q7 = nth_bit(word(wc), rc), q20 = nth_bit(word(wd), rd);
    const uint32_t c1 = 32 * wa + q1 - b0, c4 = 32 * wb + q4 - b0, c5 = after(wb, q4) - b0;
    const uint32_t c7 = 32 * wc + q7 - b0, c8 = after(wc, q7) - b0;
    const uint32_t c20 = 32 * wd + q20 - b0, c21 = after(wd, q20) - b0;
    const LdsLine b{stage + b0};
    return capture_time(b, 0u, c1, origin, ts) && ipv4(b, c4 + 1, c5, src) &&
           ipv4(b, c7 + 1, c8, dst) && count_u64(b, c20 + 1, c21, nbytes);
}

struct ParseArgs {
    const uint8_t* text;
    uint64_t len;
    const uint64_t* starts;  // [n_nl + 1]
    uint64_t n_nl;           // newlines
    uint64_t n_lines;        // n_nl, + 1 for a last line without newline
    int64_t origin;
    uint32_t* ts;
    uint32_t* src;
    uint32_t* dst;
    uint64_t* bytes;
    unsigned long long* bad;
};

__global__ void __launch_bounds__(kParseBlock) k_parse(ParseArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t stage[kStageBytes + 16];
    __shared__ uint32_t s_comma[kStageBytes / 32];  // bit i of word j: stage[32 j + i] is ','
    __shared__ uint64_t s_start[kParseBlock], s_end[kParseBlock];  // the group's line bytes
    // start and end of the bytes of this lane's line in the group at l0x
    // (0, 0 past the last line); the next group's are loaded while this
    // group is parsed
    auto bounds = [&](uint64_t l0x, uint64_t& xs, uint64_t& xg) {
        const uint64_t lx = l0x + threadIdx.x;
        xs = xg = 0;
        if (lx < a.n_lines) {
            xs = a.starts[lx];
            xg = lx < a.n_nl ? a.starts[lx + 1] : a.len;
        }
    };
    const uint64_t stride = (uint64_t)gridDim.x * kParseBlock;
    uint64_t ns = 0, ng = 0;
    bounds((uint64_t)blockIdx.x * kParseBlock, ns, ng);
    for (uint64_t l0 = (uint64_t)blockIdx.x * kParseBlock; l0 < a.n_lines; l0 += stride) {
        const uint64_t l1 = l0 + kParseBlock < a.n_lines ? l0 + kParseBlock : a.n_lines;
        const uint64_t l = l0 + threadIdx.x;
        // this lane's line [s, e) (without its newline) and the end of its bytes
        const uint64_t s = ns, g = ng;
        const uint64_t e = l < l1 ? (l < a.n_nl ? g - 1 : a.len) : 0;
        if (l0 + stride < a.n_lines) bounds(l0 + stride, ns, ng);
        s_start[threadIdx.x] = s;
        s_end[threadIdx.x] = g;  // read after the first barrier below
        uint32_t ts = kBadTs, src = 0, dst = 0;
        uint64_t nb = 0;
        bool ok = false;
        // lines [next, l1) are left; each step stages the longest prefix of
        // them whose bytes fit in LDS (line ends grow with l, so the lanes
        // that fit are a prefix), or parses one line too long for the
        // staging from device memory
        __syncthreads();
        for (uint64_t next = l0; next < l1;) {
            const uint64_t a0 = s_start[next - l0] & ~15ull;  // 16-byte aligned copy start
            const bool fits = l >= next && l < l1 && g - a0 <= kStageBytes;
            const uint64_t n_fit = (uint64_t)__syncthreads_count(fits ? 1 : 0);
            if (n_fit == 0) {
                if (l == next && e - s < 0xFFFFFFFFull)  // longer lines are bad
                    ok = parse_line(GlobalLine{a.text + s}, (uint32_t)(e - s), a.origin, ts, src, dst, nb);
                next += 1;
                continue;
            }
            const uint64_t m = next + n_fit;  // lines [next, m) are staged
            const uint64_t g1 = s_end[m - 1 - l0];
            const uint64_t full = (g1 - a0) / 16;
            if ((((uintptr_t)a.text) & 15u) == 0) {
                // four 16-byte loads of the lane in flight before its LDS writes
                const uint4* src4 = reinterpret_cast<const uint4*>(a.text + a0);
                uint4* dst4 = reinterpret_cast<uint4*>(stage);
                for (uint64_t k = threadIdx.x; k < full; k += 4 * kParseBlock) {
                    const uint64_t q1 = k + kParseBlock, q2 = k + 2 * kParseBlock,
                                   q3 = k + 3 * kParseBlock;
                    const uint4 r0 = src4[k];
                    const uint4 r1 = q1 < full ? src4[q1] : r0;
                    const uint4 r2 = q2 < full ? src4[q2] : r0;
                    const uint4 r3 = q3 < full ? src4[q3] : r0;
                    dst4[k] = r0;
                    if (q1 < full) dst4[q1] = r1;
                    if (q2 < full) dst4[q2] = r2;
                    if (q3 < full) dst4[q3] = r3;
                }
            } else {
                for (uint64_t k = threadIdx.x; k < 16 * full; k += kParseBlock) stage[k] = a.text[a0 + k];
            }
            for (uint64_t k = a0 + 16 * full + threadIdx.x; k < g1; k += kParseBlock)
                stage[k - a0] = a.text[k];
            __syncthreads();
            // the comma bitmap of the staged bytes, 16 bytes per lane at a time
            // (bits past g1 are stale and lie outside every staged line)
            const uint32_t n_chunk = (uint32_t)((g1 - a0 + 15) / 16);
            for (uint32_t c = threadIdx.x; c < n_chunk; c += kParseBlock) {
                reinterpret_cast<uint16_t*>(s_comma)[c] =
                    (uint16_t)comma_bits16(reinterpret_cast<const uint4*>(stage)[c]);
            }
            __syncthreads();
            if (l >= next && l < m)
                ok = parse_line_lds(stage, s_comma, (uint32_t)(s - a0), (uint32_t)(e - a0), a.origin, ts,
                                    src, dst, nb);
            __syncthreads();  // the staging is free for the next step
            next = m;
        }
        if (l < l1) {
            if (!ok) {
                ts = kBadTs;
                src = dst = 0;
                nb = 0;
            }
            a.ts[l] = ts;
            a.src[l] = src;
            a.dst[l] = dst;
            a.bytes[l] = nb;
        }
        // also keeps s_start / s_end until every lane is past the group
        const int n_bad = __syncthreads_count(l < l1 && !ok ? 1 : 0);
        if (threadIdx.x == 0 && n_bad) atomicAdd(a.bad, (unsigned long long)n_bad);
    }
}

}  // namespace

sinet_status parse_sessions(const uint8_t* text, uint64_t len, int64_t origin, const sinet_columns* out,
                            uint64_t* n_lines, uint64_t* n_bad, hipStream_t s) {
    *n_lines = 0;
    *n_bad = 0;
    if (len == 0) return SINET_OK;
    const uint64_t n_blocks = (len + kScanBytes - 1) / kScanBytes;
    if (n_blocks >= (1ull << 31)) return fail(SINET_ERR_UNSUPPORTED, "text above 2^47 bytes");
    uint64_t* counts = nullptr;
    unsigned long long* bad = nullptr;
    uint64_t* starts = nullptr;
    hipError_t e = hipMallocAsync((void**)&counts, 8 * (n_blocks + 1), s);
    if (e == hipSuccess) e = hipMallocAsync((void**)&bad, 8, s);
    sinet_status st = check_hip(e, "parse workspace");
    auto release = [&]() {
        if (counts) (void)hipFreeAsync(counts, s);
        if (bad) (void)hipFreeAsync(bad, s);
        if (starts) (void)hipFreeAsync(starts, s);
    };
    if (st != SINET_OK) {
        release();
        return st;
    }
    const uint32_t vec = (((uintptr_t)text) & 15u) == 0 ? 1u : 0u;
    hipLaunchKernelGGL(k_count_lines, dim3((unsigned)n_blocks), dim3(kParseBlock), 0, s, text, len,
                       counts, vec);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, counts, (uint32_t)n_blocks);
    uint64_t n_nl = 0;
    uint8_t last = 0;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&n_nl, counts + n_blocks, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&last, text + len - 1, 1, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    st = check_hip(e, "parse line count");
    if (st != SINET_OK) {
        release();
        return st;
    }
    const uint64_t lines = n_nl + (last != 10 ? 1 : 0);
    *n_lines = lines;
    if (lines > out->n) {
        release();
        return fail(SINET_ERR_INVALID_ARG, "output columns hold fewer sessions than the text has lines");
    }
    e = hipMallocAsync((void**)&starts, 8 * (n_nl + 1), s);
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, 8, s);
    st = check_hip(e, "parse workspace");
    if (st == SINET_OK) {
        hipLaunchKernelGGL(k_line_starts, dim3((unsigned)n_blocks), dim3(kParseBlock), 0, s, text, len,
                           counts, starts, vec);
        ParseArgs a{text, len, starts, n_nl, lines, origin,
                    const_cast<uint32_t*>(out->ts), const_cast<uint32_t*>(out->src),
                    const_cast<uint32_t*>(out->dst), const_cast<uint64_t*>(out->bytes), bad};
        uint64_t grid = (lines + kParseBlock - 1) / kParseBlock;
        const uint64_t cap = (uint64_t)device_cu_count() * 8;
        if (grid > cap) grid = cap;
        if (grid < 1) grid = 1;
        hipLaunchKernelGGL(k_parse, dim3((unsigned)grid), dim3(kParseBlock), 0, s, a);
        unsigned long long nb = 0;
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&nb, bad, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        st = check_hip(e, "parse");
        *n_bad = nb;
    }
    release();
    return st;
}

}  // namespace sinet

extern "C" sinet_status sinet_parse_sessions(const uint8_t* text, uint64_t len, int32_t origin_days,
                                             sinet_columns* out, uint64_t* n_lines, uint64_t* n_bad,
                                             hipStream_t stream) {
    using namespace sinet;
    if (!out || !n_lines || !n_bad) return fail(SINET_ERR_INVALID_ARG, "NULL argument");
    if (len && !text) return fail(SINET_ERR_INVALID_ARG, "text is NULL");
    if (!out->ts || !out->src || !out->dst || !out->bytes)
        return fail(SINET_ERR_INVALID_ARG, "output column is NULL");
    return parse_sessions(text, len, origin_days, out, n_lines, n_bad, stream);
}
