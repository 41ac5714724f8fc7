/*
 * CPU oracle for session discrimination and millisecond histogramming.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * statement of what the GPU path must compute, written from the paper
 * (Ando, Kadobayashi, Takakura, "Choice of Parallelism: Multi-GPU Driven
 * Pipeline for Huge Academic Backbone Network", arXiv 2106.12863).  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may call it.
 * It shares no code, header or table with the GPU library.
 *
 * Definitions (section "Threads for traffic direction discrimination with
 * CIDR MATCH", Algorithm 1, Figure 4):
 *   bitmask(x, Z)   x with its low 32-Z bits cleared (the first Z bits kept).
 *   match(a, p)     SB = bitmask(a, Z_p), CB = bitmask(base_p, Z_p),
 *                   result = SB - CB (32-bit wraparound); a match iff 0.
 *   in(a)           some prefix of the CIDR list matches a.
 *   lpm(a)          the matching prefix with the largest Z; equal Z (a
 *                   duplicated prefix) resolves to the lowest row.
 * Label (extension of the paper's two-way in/out mark to both endpoints):
 *   label = in(src) | in(dst) << 1
 *   0 external, 1 egress (the paper's "outgoing": source inside),
 *   2 ingress, 3 internal.
 * Histogram (sections "Map", "Reduce", "Merge Scatter Pattern with CPU"):
 *   key = (label, bin), bin = floor((ts - t0) / width); value = (1, bytes);
 *   one counter per bin, merged by unsigned 64-bit addition (associative and
 *   commutative, so order is free).  Sessions with ts < t0 or
 *   bin >= n_bins are added to dropped[label] instead.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_NO_INST 0xFFFFFFFFu

/* Algorithm 1, "bitmask(X.X.X.X, Z)": keep the Z leading bits.  Z = 0 keeps
 * nothing (a shift by 32 is undefined in C, so it is special-cased). */
uint32_t or_bitmask(uint32_t x, int z) {
    uint32_t m = (z <= 0) ? 0u : (z >= 32 ? 0xFFFFFFFFu : (0xFFFFFFFFu << (32 - z)));
    return x & m;
}

/* Algorithm 1: result = SB - CB; the address is inside the CIDR block iff
 * the result is zero ("outgoing" when tested on the source address). */
int or_match(uint32_t a, uint32_t base, int z) {
    uint32_t sb = or_bitmask(a, z);
    uint32_t cb = or_bitmask(base, z);
    uint32_t result = sb - cb;
    return result == 0u;
}

/* Linear scan of the whole CIDR list (Algorithm 1 applied to every entry).
 * Returns 1 if some prefix matches; *row receives the longest match (lowest
 * row among equal lengths) or -1. */
int or_lookup_scan(const uint32_t* base, const uint8_t* len, uint64_t n_prefix,
                   uint32_t a, int64_t* row) {
    int64_t best = -1;
    int best_len = -1;
    for (uint64_t p = 0; p < n_prefix; ++p) {
        if (or_match(a, base[p], len[p]) && (int)len[p] > best_len) {
            best = (int64_t)p;
            best_len = len[p];
        }
    }
    if (row) *row = best;
    return best >= 0;
}

/* ------------------------------------------------------------------------
 * The same longest-prefix-match definition computed length by length:
 * for Z = 32 down to 0, is bitmask(a, Z) the (masked) base of a /Z prefix?
 * The first Z that answers yes gives the longest match.  One open-addressing
 * hash set per present length maps a masked base to its lowest row.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint64_t cap;      /* power of two */
    uint32_t* key;
    int64_t* row;      /* -1 = empty */
} or_set;

typedef struct {
    or_set by_len[33];
    int present[33];
} or_index;

static uint64_t or_hash(uint32_t k) {
    uint64_t z = (uint64_t)k * 0x9E3779B97F4A7C15ull;
    return z ^ (z >> 29);
}

or_index* or_index_build(const uint32_t* base, const uint8_t* len, uint64_t n_prefix) {
    or_index* ix = (or_index*)calloc(1, sizeof(or_index));
    if (!ix) return NULL;
    uint64_t count[33] = {0};
    for (uint64_t p = 0; p < n_prefix; ++p) count[len[p] > 32 ? 32 : len[p]]++;
    for (int z = 0; z <= 32; ++z) {
        if (!count[z]) continue;
        uint64_t cap = 16;
        while (cap < 2 * count[z]) cap <<= 1;
        ix->present[z] = 1;
        ix->by_len[z].cap = cap;
        ix->by_len[z].key = (uint32_t*)calloc(cap, sizeof(uint32_t));
        ix->by_len[z].row = (int64_t*)malloc(cap * sizeof(int64_t));
        for (uint64_t i = 0; i < cap; ++i) ix->by_len[z].row[i] = -1;
    }
    for (uint64_t p = 0; p < n_prefix; ++p) {
        int z = len[p];
        or_set* s = &ix->by_len[z];
        uint32_t k = or_bitmask(base[p], z);
        uint64_t h = or_hash(k) & (s->cap - 1);
        while (s->row[h] >= 0 && s->key[h] != k) h = (h + 1) & (s->cap - 1);
        if (s->row[h] < 0) { /* first (lowest) row with this prefix wins */
            s->key[h] = k;
            s->row[h] = (int64_t)p;
        }
    }
    return ix;
}

void or_index_free(or_index* ix) {
    if (!ix) return;
    for (int z = 0; z <= 32; ++z) {
        free(ix->by_len[z].key);
        free(ix->by_len[z].row);
    }
    free(ix);
}

int or_index_lookup(const or_index* ix, uint32_t a, int64_t* row) {
    for (int z = 32; z >= 0; --z) {
        if (!ix->present[z]) continue;
        const or_set* s = &ix->by_len[z];
        uint32_t k = or_bitmask(a, z);
        uint64_t h = or_hash(k) & (s->cap - 1);
        while (s->row[h] >= 0) {
            if (s->key[h] == k) {
                if (row) *row = s->row[h];
                return 1;
            }
            h = (h + 1) & (s->cap - 1);
        }
    }
    if (row) *row = -1;
    return 0;
}

/* Per-session discrimination.  mode 0: linear scan; mode 1: per-length hash.
 * label[i] = in(src) | in(dst) << 1; *_inst[i] = inst of the longest match
 * (inst == NULL: the row index) or OR_NO_INST.  Any output may be NULL. */
int or_classify(const uint32_t* base, const uint8_t* len, const uint32_t* inst,
                uint64_t n_prefix, int mode, const uint32_t* src, const uint32_t* dst,
                uint64_t n, uint8_t* label, uint32_t* src_inst, uint32_t* dst_inst) {
    or_index* ix = NULL;
    if (mode == 1) {
        ix = or_index_build(base, len, n_prefix);
        if (!ix) return 1;
    }
    for (uint64_t i = 0; i < n; ++i) {
        int64_t rs, rd;
        int ins = mode ? or_index_lookup(ix, src[i], &rs)
                       : or_lookup_scan(base, len, n_prefix, src[i], &rs);
        int ind = mode ? or_index_lookup(ix, dst[i], &rd)
                       : or_lookup_scan(base, len, n_prefix, dst[i], &rd);
        if (label) label[i] = (uint8_t)(ins | (ind << 1));
        if (src_inst) src_inst[i] = rs < 0 ? OR_NO_INST : (inst ? inst[rs] : (uint32_t)rs);
        if (dst_inst) dst_inst[i] = rd < 0 ? OR_NO_INST : (inst ? inst[rd] : (uint32_t)rd);
    }
    or_index_free(ix);
    return 0;
}

/* Map and reduce with one counter per bin.  count/bytes are [4][n_bins]
 * (label-major), dropped is [4][2] = {count, bytes} per label.  With
 * accumulate == 0 the outputs are cleared first. */
int or_histogram(const uint32_t* ts, const uint64_t* bytes, const uint8_t* label,
                 uint64_t n, uint32_t t0, uint32_t width, uint32_t n_bins,
                 uint64_t* count, uint64_t* bytesh, uint64_t* dropped, int accumulate) {
    if (width == 0 || n_bins == 0) return 1;
    if (!accumulate) {
        memset(count, 0, sizeof(uint64_t) * 4 * (uint64_t)n_bins);
        memset(bytesh, 0, sizeof(uint64_t) * 4 * (uint64_t)n_bins);
        if (dropped) memset(dropped, 0, sizeof(uint64_t) * 8);
    }
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t l = label[i] & 3u;
        if (ts[i] >= t0 && (ts[i] - t0) / width < n_bins) {
            uint64_t b = (ts[i] - t0) / width;
            count[(uint64_t)l * n_bins + b] += 1;
            bytesh[(uint64_t)l * n_bins + b] += bytes[i];
        } else if (dropped) {
            dropped[l * 2 + 0] += 1;
            dropped[l * 2 + 1] += bytes[i];
        }
    }
    return 0;
}

/* Discrimination followed by the histogram (the fused path's definition). */
int or_pipeline(const uint32_t* base, const uint8_t* len, const uint32_t* inst,
                uint64_t n_prefix, int mode, const uint32_t* ts, const uint32_t* src,
                const uint32_t* dst, const uint64_t* bytes, uint64_t n, uint32_t t0,
                uint32_t width, uint32_t n_bins, uint8_t* label, uint64_t* count,
                uint64_t* bytesh, uint64_t* dropped, int accumulate) {
    uint8_t* lab = label ? label : (uint8_t*)malloc(n ? n : 1);
    if (!lab) return 1;
    int rc = or_classify(base, len, inst, n_prefix, mode, src, dst, n, lab, NULL, NULL);
    if (!rc) rc = or_histogram(ts, bytes, lab, n, t0, width, n_bins, count, bytesh, dropped,
                               accumulate);
    if (!label) free(lab);
    return rc;
}

/* ------------------------------------------------------------------------
 * Watch-list histograms (section "AbuseIPDB", section "GRIZZLY STEPPE",
 * Figures 8-11): the sessions that involve a listed host, counted per time
 * window and per direction.  The list is a prefix table (usually /32 hosts);
 * each row carries a key (inst: one key per host, or one per list), and the
 * longest match decides an address's key, as for institutions.
 *   direction 0 (SRC): the source matches the list, key = key(lpm(src));
 *                      for lists of outside hosts, the list's ingoing sessions;
 *   direction 1 (DST): the destination matches, key = key(lpm(dst));
 *                      the list's outgoing sessions.
 * A session whose two endpoints both match counts once in each direction.
 * count/bytes are [2][n_keys][n_bins] (direction-major, then key), dropped
 * is [2][2] = {count, bytes} per direction for matched sessions outside the
 * window.  Keys must be < n_keys (else the call fails with 2).  With
 * accumulate == 0 the outputs are cleared first.
 * ---------------------------------------------------------------------- */
int or_watch(const uint32_t* base, const uint8_t* len, const uint32_t* inst,
             uint64_t n_prefix, int mode, const uint32_t* ts, const uint32_t* src,
             const uint32_t* dst, const uint64_t* bytes, uint64_t n, uint32_t t0,
             uint32_t width, uint32_t n_bins, uint32_t n_keys, uint64_t* count,
             uint64_t* bytesh, uint64_t* dropped, int accumulate) {
    if (width == 0 || n_bins == 0 || n_keys == 0) return 1;
    for (uint64_t p = 0; p < n_prefix; ++p)
        if ((inst ? inst[p] : (uint32_t)p) >= n_keys) return 2;
    const uint64_t cells = 2ull * n_keys * n_bins;
    if (!accumulate) {
        memset(count, 0, sizeof(uint64_t) * cells);
        memset(bytesh, 0, sizeof(uint64_t) * cells);
        if (dropped) memset(dropped, 0, sizeof(uint64_t) * 4);
    }
    or_index* ix = NULL;
    if (mode == 1) {
        ix = or_index_build(base, len, n_prefix);
        if (!ix) return 1;
    }
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t ends[2] = {src[i], dst[i]};
        for (int dir = 0; dir < 2; ++dir) {
            int64_t row;
            int hit = mode ? or_index_lookup(ix, ends[dir], &row)
                           : or_lookup_scan(base, len, n_prefix, ends[dir], &row);
            if (!hit) continue;
            uint64_t key = inst ? inst[row] : (uint64_t)row;
            if (ts[i] >= t0 && (ts[i] - t0) / width < n_bins) {
                uint64_t b = (ts[i] - t0) / width;
                uint64_t c = ((uint64_t)dir * n_keys + key) * n_bins + b;
                count[c] += 1;
                bytesh[c] += bytes[i];
            } else if (dropped) {
                dropped[dir * 2 + 0] += 1;
                dropped[dir * 2 + 1] += bytes[i];
            }
        }
    }
    or_index_free(ix);
    return 0;
}

/* ------------------------------------------------------------------------
 * Coarser time frames (section "All Sessions of SINET", Figures 6-7: the
 * sessions grouped into one-hour frames): out[r][k] is the sum of
 * in[r][b] over b = k * factor .. min((k + 1) * factor, n_bins) - 1, for
 * every row r, k < ceil(n_bins / factor); unsigned 64-bit, modulo 2^64.
 * ---------------------------------------------------------------------- */
int or_rebin(const uint64_t* in, uint64_t rows, uint64_t n_bins, uint64_t factor,
             uint64_t* out) {
    if (rows == 0 || n_bins == 0 || factor == 0) return 1;
    const uint64_t n_out = (n_bins + factor - 1) / factor;
    for (uint64_t r = 0; r < rows; ++r) {
        for (uint64_t k = 0; k < n_out; ++k) {
            uint64_t sum = 0;
            for (uint64_t b = k * factor; b < (k + 1) * factor && b < n_bins; ++b)
                sum += in[r * n_bins + b];
            out[r * n_out + k] = sum;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Elementary intervals of a prefix table (used to state what a position
 * search over sorted boundaries must return).  Every prefix p covers
 * [bitmask(base_p, Z_p), that + 2^(32-Z_p)); the sorted distinct starts and
 * ends, with 0 added, split the address space into intervals inside which
 * the longest match cannot change.  owner[j] is the longest-match row of
 * B[j] plus one, or 0 when no prefix covers it.  Returns m (<= 2 P + 1).
 * ---------------------------------------------------------------------- */
static int or_cmp_u32(const void* a, const void* b) {
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return (x > y) - (x < y);
}

int64_t or_endpoints(const uint32_t* base, const uint8_t* len, uint64_t n_prefix,
                     uint32_t* B, uint32_t* owner) {
    uint32_t* tmp = (uint32_t*)malloc(sizeof(uint32_t) * (2 * n_prefix + 1));
    if (!tmp) return -1;
    uint64_t k = 0;
    tmp[k++] = 0;
    for (uint64_t p = 0; p < n_prefix; ++p) {
        uint64_t s = or_bitmask(base[p], len[p]);
        uint64_t e = s + (1ull << (32 - len[p]));
        tmp[k++] = (uint32_t)s;
        if (e < (1ull << 32)) tmp[k++] = (uint32_t)e;
    }
    qsort(tmp, k, sizeof(uint32_t), or_cmp_u32);
    uint64_t m = 0;
    for (uint64_t i = 0; i < k; ++i)
        if (m == 0 || tmp[i] != B[m - 1]) B[m++] = tmp[i];
    free(tmp);
    or_index* ix = or_index_build(base, len, n_prefix);
    if (!ix) return -1;
    for (uint64_t j = 0; j < m; ++j) {
        int64_t r;
        owner[j] = or_index_lookup(ix, B[j], &r) ? (uint32_t)(r + 1) : 0u;
    }
    or_index_free(ix);
    return (int64_t)m;
}
