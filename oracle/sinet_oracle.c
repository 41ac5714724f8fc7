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
 * Session text to columns (section "Dataset Description", Table 1: the
 * PA-7080 session record, 24 fields).  One record per line, fields in
 * Table 1's order separated by ','.  Every '\n'-ended segment of the text
 * is a line (an empty one included); a last segment without '\n' is a line
 * when it is not empty.  Columns come from four fields:
 *   1  capture_time  exactly "YYYY/MM/DD HH:MM:SS.mmm", a real calendar date
 *                    (proleptic Gregorian), hour < 24, minute and second
 *                    < 60; ts = its milliseconds since midnight of day
 *                    origin_days (days since 1970-01-01), which must lie in
 *                    [0, 2^32 - 1);
 *   5, 8         source and destination: four decimal octets of 1-3 digits,
 *                    each <= 255, separated by '.';
 *   21 bytes         1-20 decimal digits, at most 2^64 - 1.
 * A line with fewer than 21 fields or any of these fields malformed gives
 * ts = 0xFFFFFFFF, src = dst = 0, bytes = 0 and counts as bad.
 * ---------------------------------------------------------------------- */
/* days since 1970-01-01 of a proleptic Gregorian date (H. Hinnant,
 * "chrono-Compatible Low-Level Date Algorithms", days_from_civil) */
static int64_t or_days_from_civil(int64_t y, int64_t m, int64_t d) {
    y -= m <= 2;
    const int64_t era = (y >= 0 ? y : y - 399) / 400;
    const int64_t yoe = y - era * 400;
    const int64_t doy = (153 * (m + (m > 2 ? -3 : 9)) + 2) / 5 + d - 1;
    const int64_t doe = yoe * 365 + yoe / 4 - yoe / 100 + doy;
    return era * 146097 + doe - 719468;
}

static int or_is_leap(int64_t y) { return (y % 4 == 0 && y % 100 != 0) || y % 400 == 0; }

static int or_digits(const char* s, int n, int64_t* v) {
    int64_t x = 0;
    for (int i = 0; i < n; ++i) {
        if (s[i] < '0' || s[i] > '9') return 0;
        x = x * 10 + (s[i] - '0');
    }
    *v = x;
    return 1;
}

static int or_capture_time(const char* f, uint64_t len, int64_t origin_days, uint32_t* ts) {
    if (len != 23) return 0;
    if (f[4] != '/' || f[7] != '/' || f[10] != ' ' || f[13] != ':' || f[16] != ':' || f[19] != '.')
        return 0;
    int64_t y, mo, d, h, mi, se, ms;
    if (!or_digits(f, 4, &y) || !or_digits(f + 5, 2, &mo) || !or_digits(f + 8, 2, &d) ||
        !or_digits(f + 11, 2, &h) || !or_digits(f + 14, 2, &mi) || !or_digits(f + 17, 2, &se) ||
        !or_digits(f + 20, 3, &ms))
        return 0;
    static const int mdays[12] = {31, 28, 31, 30, 31, 30, 31, 31, 30, 31, 30, 31};
    if (mo < 1 || mo > 12 || d < 1) return 0;
    if (d > mdays[mo - 1] + (mo == 2 && or_is_leap(y))) return 0;
    if (h > 23 || mi > 59 || se > 59) return 0;
    const int64_t t = (or_days_from_civil(y, mo, d) - origin_days) * 86400000 + h * 3600000 +
                      mi * 60000 + se * 1000 + ms;
    if (t < 0 || t >= 0xFFFFFFFFll) return 0;
    *ts = (uint32_t)t;
    return 1;
}

static int or_ipv4(const char* f, uint64_t len, uint32_t* a) {
    uint32_t v = 0;
    uint64_t i = 0;
    for (int part = 0; part < 4; ++part) {
        int nd = 0;
        uint32_t o = 0;
        while (i < len && f[i] >= '0' && f[i] <= '9' && nd < 4) {
            o = o * 10 + (uint32_t)(f[i] - '0');
            ++nd;
            ++i;
        }
        if (nd < 1 || nd > 3 || o > 255) return 0;
        v = (v << 8) | o;
        if (part < 3) {
            if (i >= len || f[i] != '.') return 0;
            ++i;
        }
    }
    if (i != len) return 0;
    *a = v;
    return 1;
}

static int or_u64(const char* f, uint64_t len, uint64_t* out) {
    if (len < 1 || len > 20) return 0;
    uint64_t v = 0;
    for (uint64_t i = 0; i < len; ++i) {
        if (f[i] < '0' || f[i] > '9') return 0;
        const uint64_t dg = (uint64_t)(f[i] - '0');
        if (v > (UINT64_MAX - dg) / 10) return 0;
        v = v * 10 + dg;
    }
    *out = v;
    return 1;
}

/* Parse lines of text[len] into ts/src/dst/bytes (capacity cap).  Returns 0,
 * or 1 when there are more lines than cap; *n_lines and *bad are set. */
int or_parse(const char* text, uint64_t len, int64_t origin_days, uint32_t* ts, uint32_t* src,
             uint32_t* dst, uint64_t* bytes, uint64_t cap, uint64_t* n_lines, uint64_t* bad) {
    uint64_t n = 0, nbad = 0, p = 0;
    while (p < len) {
        uint64_t e = p;
        while (e < len && text[e] != '\n') ++e;  /* the line is [p, e) */
        if (n >= cap) return 1;
        /* field boundaries: field k (1-based) is [fs[k], fe[k]) */
        uint64_t fs[22], fe[22];
        int nf = 0;
        uint64_t q = p;
        while (nf < 21) {
            uint64_t c = q;
            while (c < e && text[c] != ',') ++c;
            ++nf;
            fs[nf] = q;
            fe[nf] = c;
            if (c >= e) break;
            q = c + 1;
        }
        uint32_t t = 0, a = 0, b = 0;
        uint64_t by = 0;
        int ok = nf >= 21 && or_capture_time(text + fs[1], fe[1] - fs[1], origin_days, &t) &&
                 or_ipv4(text + fs[5], fe[5] - fs[5], &a) && or_ipv4(text + fs[8], fe[8] - fs[8], &b) &&
                 or_u64(text + fs[21], fe[21] - fs[21], &by);
        if (ok) {
            ts[n] = t;
            src[n] = a;
            dst[n] = b;
            bytes[n] = by;
        } else {
            ts[n] = 0xFFFFFFFFu;
            src[n] = 0;
            dst[n] = 0;
            bytes[n] = 0;
            ++nbad;
        }
        ++n;
        p = e + 1;  /* past the '\n' (or past the end) */
    }
    *n_lines = n;
    *bad = nbad;
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

/* Label runs (section "Coordinated Batch Processing", Fig. 3: the sessions of
 * a chunk are discriminated before the Map stage): the stable partition of
 * the session indices by label.  For L = 0, 1, 2, 3 in turn, every index i
 * with (label[i] & 3) == L is appended in increasing order; totals[L] counts
 * them.  n must be below 2^32 (the indices are 32-bit). */
int or_label_runs(const uint8_t* label, uint64_t n, uint32_t* idx, uint64_t* totals) {
    if (n >= (1ull << 32)) return 1;
    uint64_t k = 0;
    for (uint32_t L = 0; L < 4; ++L) {
        totals[L] = 0;
        for (uint64_t i = 0; i < n; ++i) {
            if ((uint32_t)(label[i] & 3u) == L) {
                idx[k++] = (uint32_t)i;
                totals[L] += 1;
            }
        }
    }
    return 0;
}
