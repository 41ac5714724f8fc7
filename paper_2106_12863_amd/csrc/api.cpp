// libsinet C ABI: argument checks, the host-side table builder and dispatch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "sinet.h"
#include "inout_index.h"
#include "sinet_internal.h"

namespace sinet {

static thread_local std::string g_last_error;

sinet_status fail(sinet_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

sinet_status check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return SINET_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(SINET_ERR_OUT_OF_MEMORY, std::string(what) + ": " + hipGetErrorString(e));
    return fail(SINET_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static constexpr uint32_t kLdsTopMax = 16384;        // sampled boundaries kept in LDS
static constexpr uint32_t kLdsMemberMaxWords = 16384; // membership bits kept in LDS
static constexpr uint32_t kLdsReserveWords = 3328;    // static LDS of the pass kernels
static constexpr uint32_t kMaxSegments = 65535;       // PLA segment index fits 16 bits

static uint32_t prefix_mask(uint32_t z) {
    return z == 0 ? 0u : (z >= 32 ? 0xFFFFFFFFu : (0xFFFFFFFFu << (32 - z)));
}

// Elementary intervals of a laminar set of prefixes (two CIDR blocks are
// either disjoint or nested).  A sweep over the sorted boundaries keeps the
// blocks covering the current point on a stack, innermost on top; a block is
// pushed when the sweep reaches its start and popped at its end.  Blocks
// with the same start are pushed outermost first and, for identical blocks,
// highest row first, so the top is the longest match with the lowest row.
static void build_intervals(const std::vector<uint32_t>& cb, const std::vector<uint32_t>& len,
                            std::vector<uint32_t>& B, std::vector<uint32_t>& owner) {
    const size_t P = cb.size();
    std::vector<uint32_t> order(P);
    for (size_t i = 0; i < P; ++i) order[i] = (uint32_t)i;
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (cb[a] != cb[b]) return cb[a] < cb[b];
        if (len[a] != len[b]) return len[a] < len[b];
        return a > b;
    });
    std::vector<uint32_t> pts;
    pts.reserve(2 * P + 1);
    pts.push_back(0);
    for (size_t i = 0; i < P; ++i) {
        uint64_t e = (uint64_t)cb[i] + (1ull << (32 - len[i]));
        pts.push_back(cb[i]);
        if (e < (1ull << 32)) pts.push_back((uint32_t)e);
    }
    std::sort(pts.begin(), pts.end());
    pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
    B = pts;
    owner.assign(B.size(), 0);
    std::vector<uint32_t> stack;
    stack.reserve(64);
    auto end_of = [&](uint32_t r) { return (uint64_t)cb[r] + (1ull << (32 - len[r])); };
    size_t next = 0;
    for (size_t j = 0; j < B.size(); ++j) {
        const uint64_t x = B[j];
        while (!stack.empty() && end_of(stack.back()) <= x) stack.pop_back();
        while (next < P && cb[order[next]] == x) stack.push_back(order[next++]);
        owner[j] = stack.empty() ? 0u : stack.back() + 1u;
    }
}

// 16-8-8 multibit trie over the intervals: level 1 is indexed by the top 16
// address bits, nodes of 256 entries by the next 8 bits each.  An entry with
// bit 31 set is a leaf holding the interval index; otherwise it is a node
// number (node k occupies entries 65536 + 256 k .. + 255).
static void build_trie(const std::vector<uint32_t>& B, std::vector<uint32_t>& trie) {
    auto pos = [&](uint64_t a) -> uint32_t {
        return (uint32_t)(std::upper_bound(B.begin(), B.end(), (uint32_t)a) - B.begin()) - 1;
    };
    trie.assign(65536, 0);
    uint32_t nodes = 0;
    for (uint64_t k1 = 0; k1 < 65536; ++k1) {
        const uint64_t lo = k1 << 16, hi = lo + 65535;
        const uint32_t j0 = pos(lo), j1 = pos(hi);
        if (j0 == j1) {
            trie[k1] = 0x80000000u | j0;
            continue;
        }
        const uint32_t n2 = nodes++;
        trie[k1] = n2;
        trie.resize(65536 + (size_t)nodes * 256, 0);
        for (uint64_t k2 = 0; k2 < 256; ++k2) {
            const uint64_t lo2 = lo + (k2 << 8), hi2 = lo2 + 255;
            const uint32_t a0 = pos(lo2), a1 = pos(hi2);
            if (a0 == a1) {
                trie[65536 + (size_t)n2 * 256 + k2] = 0x80000000u | a0;
                continue;
            }
            const uint32_t n3 = nodes++;
            trie[65536 + (size_t)n2 * 256 + k2] = n3;
            trie.resize(65536 + (size_t)nodes * 256, 0);
            for (uint64_t k3 = 0; k3 < 256; ++k3)
                trie[65536 + (size_t)n3 * 256 + k3] = 0x80000000u | pos(lo2 + k3);
        }
    }
}

// In/out index of the union of the prefixes (layout in inout_index.h).
static bool build_inout(const std::vector<uint32_t>& B, const std::vector<uint32_t>& owner,
                        std::vector<uint32_t>& io, DevTable& d) {
    std::vector<uint32_t> U;  // where membership of the union changes
    bool prev = false;
    for (size_t j = 0; j < B.size(); ++j) {
        const bool in = owner[j] != 0;
        if (in != prev) U.push_back(B[j]);
        prev = in;
    }
    IoLayout lay{};
    if (!build_inout_index(U, io, lay)) return false;
    d.io_words = lay.words;
    d.io_slot = lay.slot;
    d.io_list = lay.list;
    return true;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static uint32_t lds_bytes_for(const DevTable& t, uint32_t kind) {
    uint32_t words = 0;
    switch (kind) {
        case SINET_LOOKUP_SCAN: return 12u * t.n_prefix;
        case SINET_LOOKUP_BSEARCH: words = t.n_top; break;
        case SINET_LOOKUP_TRIE: break;
        case SINET_LOOKUP_LEARNED_PLA:
            words = (t.pla_window ? 0u : t.n_top) + 3 * t.segments + radix_words(t.radix_bits);
            break;
        case SINET_LOOKUP_LEARNED_MLP: words = t.n_top + SINET_MLP_PARAMS; break;
        default: break;
    }
    return 4u * (words + t.lds_member_words + (t.filter_lds ? kFilterWords : 0u));
}

// LDS words a PLA of S segments needs next to the filter and member bits;
// the window search needs no sample of the boundaries.
static uint32_t pla_lds_words(const DevTable& t, uint32_t S, bool window) {
    return (window ? 0u : t.n_top) + 3 * S + radix_words(t.radix_bits) + t.lds_member_words +
           (t.filter_lds ? kFilterWords : 0u);
}

// 2-bit state of every /16 block: 0 no prefix covers any of it, 1 one interval
// covers all of it and is inside the table, 2 a boundary cuts it.
static void build_filter(const std::vector<uint32_t>& B, const std::vector<uint32_t>& owner,
                         std::vector<uint32_t>& filter) {
    filter.assign(kFilterWords, 0);
    for (uint64_t k = 0; k < 65536; ++k) {
        const uint32_t lo = (uint32_t)(k << 16), hi = lo | 0xFFFFu;
        const uint32_t j0 = (uint32_t)(std::upper_bound(B.begin(), B.end(), lo) - B.begin()) - 1;
        const uint32_t j1 = (uint32_t)(std::upper_bound(B.begin(), B.end(), hi) - B.begin()) - 1;
        const uint32_t st = j0 != j1 ? 2u : (owner[j0] ? 1u : 0u);
        filter[k >> 4] |= st << ((k & 15) * 2);
    }
}

static sinet_status check_device(const sinet_table* t) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return check_hip(e, "hipGetDevice");
    if (dev != t->device) return fail(SINET_ERR_INVALID_ARG, "table belongs to another device");
    return SINET_OK;
}

sinet_status check_usable(const sinet_table* t) {
    if (!t) return fail(SINET_ERR_INVALID_ARG, "table is NULL");
    if ((t->kind == SINET_LOOKUP_LEARNED_PLA || t->kind == SINET_LOOKUP_LEARNED_MLP) && !t->trained)
        return fail(SINET_ERR_INVALID_ARG, "learned table used before sinet_table_train");
    return check_device(t);
}

// The device view a pass uses: label-only passes of a table with an in/out
// index run the index kind (LDS holds the index alone).
DevTable label_view(const sinet_table* t, bool label_only) {
    DevTable d = t->dev;
    if (label_only && d.io) {
        d.kind = kInoutKind;
        d.lds_bytes = 4u * d.io_words;
    }
    return d;
}

sinet_status check_window(const sinet_window* w) {
    if (!w) return fail(SINET_ERR_INVALID_ARG, "window is NULL");
    if (w->width_ms == 0) return fail(SINET_ERR_INVALID_ARG, "width_ms is 0");
    if (w->n_bins == 0) return fail(SINET_ERR_INVALID_ARG, "n_bins is 0");
    return SINET_OK;
}

static sinet_status clear_hist(const sinet_window* w, sinet_hist* h, hipStream_t s) {
    const uint64_t words = 4ull * w->n_bins;
    sinet_status st = launch_zero((unsigned long long*)h->count, words, s);
    if (st == SINET_OK) st = launch_zero((unsigned long long*)h->bytes, words, s);
    if (st == SINET_OK && h->dropped) st = launch_zero((unsigned long long*)h->dropped, 8, s);
    return st;
}

// Argument checks and pass parameters of a pipeline call; *done when nothing
// is left to run (no sessions: the histogram was cleared unless accumulating).
sinet_status pipeline_prepare(const sinet_table* t, const sinet_columns* cols, const sinet_window* win,
                              uint8_t* label, sinet_hist* out, int accumulate, hipStream_t stream,
                              PassParams* pp, bool* done) {
    *done = false;
    sinet_status st = check_usable(t);
    if (st != SINET_OK) return st;
    st = check_window(win);
    if (st != SINET_OK) return st;
    if (!cols) return fail(SINET_ERR_INVALID_ARG, "columns are NULL");
    if (!out || !out->count || !out->bytes) return fail(SINET_ERR_INVALID_ARG, "histogram output is NULL");
    if (cols->n && (!cols->ts || !cols->src || !cols->dst || !cols->bytes))
        return fail(SINET_ERR_INVALID_ARG, "column is NULL");
    if (!accumulate && (cols->n == 0 || out->dropped)) {
        st = cols->n == 0 ? clear_hist(win, out, stream)
                          : launch_zero((unsigned long long*)out->dropped, 8, stream);
        if (st != SINET_OK) return st;
    }
    if (cols->n == 0) {
        *done = true;
        return SINET_OK;
    }
    PassParams& p = *pp;
    memset(&p, 0, sizeof(p));
    p.t = label_view(t, true);
    p.ts = cols->ts;
    p.src = cols->src;
    p.dst = cols->dst;
    p.bytes = cols->bytes;
    p.label_out = label;
    p.count = (unsigned long long*)out->count;
    p.hbytes = (unsigned long long*)out->bytes;
    p.dropped = (unsigned long long*)out->dropped;
    p.n = cols->n;
    p.t0 = win->t0_ms;
    p.width = win->width_ms;
    p.n_bins = win->n_bins;
    p.magic = div_magic(win->width_ms);
    return SINET_OK;
}

}  // namespace sinet

using namespace sinet;

extern "C" {

const char* sinet_status_string(sinet_status s) {
    switch (s) {
        case SINET_OK: return "ok";
        case SINET_ERR_INVALID_ARG: return "invalid argument";
        case SINET_ERR_OUT_OF_MEMORY: return "out of device memory";
        case SINET_ERR_DEVICE: return "device error";
        case SINET_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* sinet_last_error(void) { return g_last_error.c_str(); }

const char* sinet_version(void) { return "libsinet 0.1 gfx950"; }

sinet_status sinet_table_create(const uint32_t* base, const uint8_t* len, const uint32_t* inst,
                                uint64_t n_prefix, sinet_lookup kind, hipStream_t stream,
                                sinet_table** out) {
    if (!out) return fail(SINET_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!base || !len) return fail(SINET_ERR_INVALID_ARG, "base or len is NULL");
    if (n_prefix == 0) return fail(SINET_ERR_INVALID_ARG, "n_prefix is 0");
    if (n_prefix > SINET_MAX_PREFIXES) return fail(SINET_ERR_INVALID_ARG, "too many prefixes");
    const bool want_io = (kind & SINET_TABLE_NO_INOUT_INDEX) == 0;
    const bool global_bsearch = (kind & SINET_TABLE_GLOBAL_BSEARCH) != 0;
    kind = (sinet_lookup)(kind & ~(SINET_TABLE_NO_INOUT_INDEX | SINET_TABLE_GLOBAL_BSEARCH));
    if (kind == SINET_LOOKUP_AUTO) kind = n_prefix <= 64 ? SINET_LOOKUP_SCAN : SINET_LOOKUP_BSEARCH;
    if (kind < SINET_LOOKUP_SCAN || kind > SINET_LOOKUP_LEARNED_MLP)
        return fail(SINET_ERR_INVALID_ARG, "unknown lookup kind");
    if (kind == SINET_LOOKUP_SCAN && n_prefix > 1024)
        return fail(SINET_ERR_INVALID_ARG, "scan tables hold at most 1024 prefixes");
    const size_t P = (size_t)n_prefix;
    std::vector<uint32_t> cb(P), mk(P), ln(P), id(P);
    for (size_t i = 0; i < P; ++i) {
        if (len[i] > 32) return fail(SINET_ERR_INVALID_ARG, "prefix length above 32");
        ln[i] = len[i];
        mk[i] = prefix_mask(len[i]);
        cb[i] = base[i] & mk[i];
        id[i] = inst ? inst[i] : (uint32_t)i;
        if (id[i] == SINET_NO_INST) return fail(SINET_ERR_INVALID_ARG, "inst id 0xFFFFFFFF is reserved");
    }
    sinet_table* t = new sinet_table();
    t->kind = kind;
    t->max_inst = 0;
    for (size_t i = 0; i < P; ++i) t->max_inst = std::max(t->max_inst, id[i]);
    t->n_prefix = n_prefix;
    (void)hipGetDevice(&t->device);
    build_intervals(cb, ln, t->B, t->owner);
    const uint32_t m = (uint32_t)t->B.size();
    const uint32_t mw = (m + 31) / 32;
    std::vector<uint32_t> member(mw, 0);
    for (uint32_t j = 0; j < m; ++j)
        if (t->owner[j]) member[j >> 5] |= 1u << (j & 31);
    // LDS plan: the /16 filter and the membership bits first (every interval
    // kind reads them), then as many sampled boundaries as the per-workgroup
    // LDS limit leaves room for.
    int lds_limit = 65536;
    if (hipDeviceGetAttribute(&lds_limit, hipDeviceAttributeMaxSharedMemoryPerBlock, t->device) !=
            hipSuccess || lds_limit <= 0)
        lds_limit = 65536;
    const uint32_t lds_words = (uint32_t)std::min(lds_limit, 160 * 1024) / 4;
    const bool interval_kind = kind != SINET_LOOKUP_SCAN;
    const uint32_t filter_lds = interval_kind && lds_words >= kFilterWords + 8192 + kLdsReserveWords ? 1u : 0u;
    const uint32_t fw = filter_lds ? kFilterWords : 0u;
    const uint32_t member_lds =
        (mw <= kLdsMemberMaxWords && fw + mw + 1024 + kLdsReserveWords <= lds_words) ? mw : 0;
    // learned kinds keep fewer sampled boundaries, leaving LDS for the model
    const bool learned_kind = kind == SINET_LOOKUP_LEARNED_PLA || kind == SINET_LOOKUP_LEARNED_MLP;
    uint32_t top_cap = std::min<uint32_t>(learned_kind ? kLdsTopMax / 2 : kLdsTopMax,
                                          lds_words - fw - member_lds - kLdsReserveWords);
    if (global_bsearch && kind == SINET_LOOKUP_BSEARCH) top_cap = 1;  // one leaf: all of B
    uint32_t top_log2 = 0;
    while (((uint64_t)m + (1ull << top_log2) - 1) >> top_log2 > top_cap) ++top_log2;
    const uint32_t n_top = (uint32_t)(((uint64_t)m + (1ull << top_log2) - 1) >> top_log2);
    std::vector<uint32_t> top(n_top);
    for (uint32_t i = 0; i < n_top; ++i) top[i] = t->B[(size_t)i << top_log2];
    // boundaries padded with 0xFFFFFFFF to whole leaf blocks of 2^top_log2
    const uint64_t m_pad = (uint64_t)n_top << top_log2;
    std::vector<uint32_t> Bpad(t->B);
    Bpad.resize(m_pad + kBTail, 0xFFFFFFFFu);
    std::vector<uint32_t> filter;
    if (interval_kind) build_filter(t->B, t->owner, filter);
    std::vector<uint32_t> io;
    DevTable iod;
    memset(&iod, 0, sizeof(iod));
    bool io_ok = interval_kind && want_io && build_inout(t->B, t->owner, io, iod) &&
                 io.size() + kLdsReserveWords <= lds_words;
    if (!io_ok) io.clear();
    std::vector<uint32_t> trie;
    if (kind == SINET_LOOKUP_TRIE) build_trie(t->B, trie);
    const bool learned = kind == SINET_LOOKUP_LEARNED_PLA || kind == SINET_LOOKUP_LEARNED_MLP;
    const uint32_t smax = learned ? kMaxSegments : 0;

    // one arena
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const uint32_t rw = learned ? radix_words(kPlaRadixBits) : 0;
    const size_t oB = take(4ull * (m_pad + kBTail)), oOwn = take(4ull * m), oMem = take(4ull * mw),
                 oInst = take(4 * P), oCb = take(4 * P), oMk = take(4 * P), oLn = take(4 * P),
                 oTop = take(4ull * n_top), oTrie = take(4 * trie.size()),
                 oKnot = take(4ull * smax), oC = take(4ull * smax), oG = take(4ull * smax),
                 oMlp = take(4 * SINET_MLP_PARAMS), oFb = take(8), oRadix = take(4ull * rw),
                 oFilter = take(4ull * filter.size()), oIo = take(4ull * io.size());
    void* arena = nullptr;
    hipError_t e = hipMalloc(&arena, off);
    if (e != hipSuccess) {
        delete t;
        return check_hip(e, "table allocation");
    }
    t->arena = arena;
    t->arena_bytes = off;
    char* a = (char*)arena;
    auto up = [&](size_t o, const void* src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(a + o, src, bytes, hipMemcpyHostToDevice, stream);
    };
    hipError_t r = hipSuccess;
    if (r == hipSuccess) r = up(oB, Bpad.data(), 4ull * (m_pad + kBTail));
    if (r == hipSuccess) r = up(oFilter, filter.data(), 4ull * filter.size());
    if (r == hipSuccess) r = up(oIo, io.data(), 4ull * io.size());
    if (r == hipSuccess) r = up(oOwn, t->owner.data(), 4ull * m);
    if (r == hipSuccess) r = up(oMem, member.data(), 4ull * mw);
    if (r == hipSuccess) r = up(oInst, id.data(), 4 * P);
    if (r == hipSuccess) r = up(oCb, cb.data(), 4 * P);
    if (r == hipSuccess) r = up(oMk, mk.data(), 4 * P);
    if (r == hipSuccess) r = up(oLn, ln.data(), 4 * P);
    if (r == hipSuccess) r = up(oTop, top.data(), 4ull * n_top);
    if (r == hipSuccess) r = up(oTrie, trie.data(), 4 * trie.size());
    const unsigned long long zero = 0;
    if (r == hipSuccess) r = up(oFb, &zero, 8);
    if (r == hipSuccess) r = hipStreamSynchronize(stream);
    if (r != hipSuccess) {
        (void)hipFree(arena);
        delete t;
        return check_hip(r, "table upload");
    }
    DevTable& d = t->dev;
    memset(&d, 0, sizeof(d));
    d.kind = kind;
    d.m = m;
    d.B = (const uint32_t*)(a + oB);
    d.owner = (const uint32_t*)(a + oOwn);
    d.member = (const uint32_t*)(a + oMem);
    d.inst = (const uint32_t*)(a + oInst);
    d.n_prefix = (uint32_t)P;
    d.cb = (const uint32_t*)(a + oCb);
    d.mask = (const uint32_t*)(a + oMk);
    d.len = (const uint32_t*)(a + oLn);
    d.top_log2 = top_log2;
    d.n_top = n_top;
    d.top = (const uint32_t*)(a + oTop);
    d.trie = trie.empty() ? nullptr : (const uint32_t*)(a + oTrie);
    d.knot = (const uint32_t*)(a + oKnot);
    d.pla_c = (const float*)(a + oC);
    d.pla_g = (const float*)(a + oG);
    d.mlp = (const float*)(a + oMlp);
    d.radix = (const uint32_t*)(a + oRadix);
    d.radix_bits = kPlaRadixBits;
    d.filter = filter.empty() ? nullptr : (const uint32_t*)(a + oFilter);
    d.filter_lds = filter.empty() ? 0u : filter_lds;
    if (io_ok) {
        d.io = (const uint32_t*)(a + oIo);
        d.io_words = iod.io_words;
        d.io_slot = iod.io_slot;
        d.io_list = iod.io_list;
    }
    d.m_f = (float)m;
    d.fallbacks = (unsigned long long*)(a + oFb);
    d.lds_member_words = member_lds;
    t->lds_words = lds_words;
    d.lds_bytes = lds_bytes_for(d, kind);
    *out = t;
    return SINET_OK;
}

sinet_status sinet_table_train(sinet_table* t, const sinet_train_params* params, hipStream_t stream,
                               sinet_train_report* report) {
    if (!t) return fail(SINET_ERR_INVALID_ARG, "table is NULL");
    sinet_status st = check_device(t);
    if (st != SINET_OK) return st;
    sinet_train_report rep;
    memset(&rep, 0, sizeof(rep));
    if (t->kind == SINET_LOOKUP_LEARNED_PLA) {
        const uint32_t S = params ? params->segments : 0;
        const uint32_t E = params ? params->target_err : 0;
        if (S > kMaxSegments) return fail(SINET_ERR_INVALID_ARG, "segments above 65535");
        if (S && pla_lds_words(t->dev, S, false) + kLdsReserveWords > t->lds_words)
            return fail(SINET_ERR_INVALID_ARG, "segments do not fit in LDS next to the filter and member bits");
        const uint32_t budget = t->lds_words - kLdsReserveWords;
        auto room = [&](bool window) {
            const uint32_t used = pla_lds_words(t->dev, 0, window);
            return used < budget ? (budget - used) / 3 : 0u;
        };
        const uint32_t smax = room(false), smax_window = room(true);
        if (smax_window == 0) return fail(SINET_ERR_UNSUPPORTED, "no LDS left for PLA segments");
        st = train_pla(t, S, E, std::min(smax, kMaxSegments), std::min(smax_window, kMaxSegments),
                       stream, &rep);
    } else if (t->kind == SINET_LOOKUP_LEARNED_MLP) {
        st = train_mlp(t, params, stream, &rep);
    } else {
        return fail(SINET_ERR_INVALID_ARG, "table kind is not learned");
    }
    if (st != SINET_OK) return st;
    t->trained = 1;
    t->dev.lds_bytes = lds_bytes_for(t->dev, t->kind);
    if (report) *report = rep;
    return SINET_OK;
}

sinet_status sinet_table_info(const sinet_table* t, sinet_table_info_t* out) {
    if (!t || !out) return fail(SINET_ERR_INVALID_ARG, "NULL argument");
    memset(out, 0, sizeof(*out));
    out->kind = t->kind;
    out->inout_index = t->dev.io ? 1u : 0u;
    out->n_prefix = t->n_prefix;
    out->m = t->dev.m;
    out->device_bytes = t->arena_bytes;
    out->trained = (uint32_t)t->trained;
    out->max_err = t->dev.max_err;
    out->segments = t->dev.segments;
    out->pla_window = t->dev.pla_window;
    unsigned long long fb = 0;
    hipError_t e = hipMemcpy(&fb, t->dev.fallbacks, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return check_hip(e, "fallback counter read");
    out->fallbacks = fb;
    return SINET_OK;
}

sinet_status sinet_table_get_model(const sinet_table* t, float* params, uint32_t* knot, float* c,
                                   float* g, uint32_t cap, uint32_t* max_err) {
    if (!t) return fail(SINET_ERR_INVALID_ARG, "table is NULL");
    if (!t->trained) return fail(SINET_ERR_INVALID_ARG, "table has no trained model");
    hipError_t e = hipSuccess;
    if (t->kind == SINET_LOOKUP_LEARNED_MLP) {
        if (!params) return fail(SINET_ERR_INVALID_ARG, "params is NULL");
        e = hipMemcpy(params, t->dev.mlp, 4 * SINET_MLP_PARAMS, hipMemcpyDeviceToHost);
    } else {
        const uint32_t S = t->dev.segments;
        if (cap < S) return fail(SINET_ERR_INVALID_ARG, "capacity below the segment count");
        if (knot) e = hipMemcpy(knot, t->dev.knot, 4ull * S, hipMemcpyDeviceToHost);
        if (e == hipSuccess && c) e = hipMemcpy(c, t->dev.pla_c, 4ull * S, hipMemcpyDeviceToHost);
        if (e == hipSuccess && g) e = hipMemcpy(g, t->dev.pla_g, 4ull * S, hipMemcpyDeviceToHost);
    }
    if (max_err) *max_err = t->dev.max_err;
    return check_hip(e, "model download");
}

sinet_status sinet_table_set_model(sinet_table* t, const float* params, const uint32_t* knot,
                                   const float* c, const float* g, uint32_t segments,
                                   uint32_t max_err) {
    if (!t) return fail(SINET_ERR_INVALID_ARG, "table is NULL");
    sinet_status st = check_device(t);
    if (st != SINET_OK) return st;
    hipError_t e = hipSuccess;
    if (t->kind == SINET_LOOKUP_LEARNED_MLP) {
        if (!params) return fail(SINET_ERR_INVALID_ARG, "params is NULL");
        e = hipMemcpy((void*)t->dev.mlp, params, 4 * SINET_MLP_PARAMS, hipMemcpyHostToDevice);
    } else if (t->kind == SINET_LOOKUP_LEARNED_PLA) {
        if (!knot || !c || !g) return fail(SINET_ERR_INVALID_ARG, "PLA arrays are NULL");
        if (segments == 0 || segments > kMaxSegments || segments > t->dev.m)
            return fail(SINET_ERR_INVALID_ARG, "bad segment count");
        if (pla_lds_words(t->dev, segments, true) + kLdsReserveWords > t->lds_words)
            return fail(SINET_ERR_INVALID_ARG, "segments do not fit in LDS next to the filter and member bits");
        if (knot[0] != 0) return fail(SINET_ERR_INVALID_ARG, "knot[0] must be 0");
        for (uint32_t s = 0; s < segments; ++s) {
            if (s && knot[s] <= knot[s - 1]) return fail(SINET_ERR_INVALID_ARG, "knots not ascending");
            if (!(g[s] >= 0.f)) return fail(SINET_ERR_INVALID_ARG, "negative or NaN slope");
        }
        e = hipMemcpy((void*)t->dev.knot, knot, 4ull * segments, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy((void*)t->dev.pla_c, c, 4ull * segments, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy((void*)t->dev.pla_g, g, 4ull * segments, hipMemcpyHostToDevice);
        t->dev.segments = segments;
        t->segments = segments;
        std::vector<uint32_t> kn(knot, knot + segments);
        if (e == hipSuccess) e = upload_radix(t, kn);
    } else {
        return fail(SINET_ERR_INVALID_ARG, "table kind is not learned");
    }
    if (e != hipSuccess) return check_hip(e, "model upload");
    if (max_err == 0xFFFFFFFFu) {
        st = measure_err(t->dev, t->kind == SINET_LOOKUP_LEARNED_MLP, nullptr, &max_err);
        if (st != SINET_OK) return st;
    }
    t->dev.max_err = max_err;
    // the window search needs a bound of at most kPlaWindowErr; otherwise the
    // LDS sample of the boundaries must fit next to the segments
    t->dev.pla_window = 0;
    if (t->kind == SINET_LOOKUP_LEARNED_PLA) {
        if (max_err <= kPlaWindowErr) {
            t->dev.pla_window = 1;
        } else if (pla_lds_words(t->dev, segments, false) + kLdsReserveWords > t->lds_words) {
            t->trained = 0;
            return fail(SINET_ERR_INVALID_ARG,
                        "bound above 6 and the segments leave no LDS for the boundary sample");
        }
    }
    t->trained = 1;
    t->dev.lds_bytes = lds_bytes_for(t->dev, t->kind);
    return SINET_OK;
}

sinet_status sinet_table_intervals(const sinet_table* t, uint32_t* B, uint32_t* owner, uint64_t cap) {
    if (!t || !B || !owner) return fail(SINET_ERR_INVALID_ARG, "NULL argument");
    if (cap < t->B.size()) return fail(SINET_ERR_INVALID_ARG, "capacity below m");
    hipError_t e = hipMemcpy(B, t->dev.B, 4 * t->B.size(), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(owner, t->dev.owner, 4 * t->B.size(), hipMemcpyDeviceToHost);
    return check_hip(e, "interval download");
}

sinet_status sinet_table_destroy(sinet_table* t) {
    if (!t) return fail(SINET_ERR_INVALID_ARG, "table is NULL");
    hipError_t e = hipFree(t->arena);
    delete t;
    return check_hip(e, "table free");
}

sinet_status sinet_table_position(const sinet_table* t, const uint32_t* addr, uint64_t n,
                                  uint32_t* pos, hipStream_t stream) {
    sinet_status st = check_usable(t);
    if (st != SINET_OK) return st;
    if (n == 0) return SINET_OK;
    if (!addr || !pos) return fail(SINET_ERR_INVALID_ARG, "addr or pos is NULL");
    PassParams p;
    memset(&p, 0, sizeof(p));
    p.t = t->dev;
    if (t->kind == SINET_LOOKUP_SCAN) {  // a scan table answers positions by search
        p.t.kind = SINET_LOOKUP_BSEARCH;
        p.t.lds_bytes = lds_bytes_for(p.t, SINET_LOOKUP_BSEARCH);
    }
    p.src = addr;
    p.pos_out = pos;
    p.n = n;
    return launch_pass(p, 0, stream);
}

sinet_status sinet_discriminate(const sinet_table* t, const uint32_t* src, const uint32_t* dst,
                                uint64_t n, uint8_t* label, uint32_t* src_inst, uint32_t* dst_inst,
                                hipStream_t stream) {
    sinet_status st = check_usable(t);
    if (st != SINET_OK) return st;
    if (n == 0) return SINET_OK;
    if (!src || !dst) return fail(SINET_ERR_INVALID_ARG, "src or dst is NULL");
    if (!label && !src_inst && !dst_inst) return SINET_OK;
    PassParams p;
    memset(&p, 0, sizeof(p));
    p.t = label_view(t, !src_inst && !dst_inst);
    p.src = src;
    p.dst = dst;
    p.label_out = label;
    p.src_inst = src_inst;
    p.dst_inst = dst_inst;
    p.n = n;
    return launch_pass(p, PASS_LABEL, stream);
}

sinet_status sinet_histogram(const uint32_t* ts, const uint64_t* bytes, const uint8_t* label,
                             uint64_t n, const sinet_window* win, sinet_hist* out, int accumulate,
                             hipStream_t stream) {
    sinet_status st = check_window(win);
    if (st != SINET_OK) return st;
    if (!out || !out->count || !out->bytes) return fail(SINET_ERR_INVALID_ARG, "histogram output is NULL");
    if (n && (!ts || !bytes || !label)) return fail(SINET_ERR_INVALID_ARG, "column is NULL");
    if (!accumulate && (n == 0 || out->dropped)) {
        st = n == 0 ? clear_hist(win, out, stream)
                    : launch_zero((unsigned long long*)out->dropped, 8, stream);
        if (st != SINET_OK) return st;
    }
    if (n == 0) return SINET_OK;
    PassParams p;
    memset(&p, 0, sizeof(p));
    p.ts = ts;
    p.bytes = bytes;
    p.label_in = label;
    p.count = (unsigned long long*)out->count;
    p.hbytes = (unsigned long long*)out->bytes;
    p.dropped = (unsigned long long*)out->dropped;
    p.n = n;
    p.t0 = win->t0_ms;
    p.width = win->width_ms;
    p.n_bins = win->n_bins;
    p.magic = div_magic(win->width_ms);
    return run_hist(p, PASS_HIST | PASS_LABEL_IN, accumulate, stream);
}

sinet_status sinet_pipeline(const sinet_table* t, const sinet_columns* cols, const sinet_window* win,
                            uint8_t* label, sinet_hist* out, int accumulate, hipStream_t stream) {
    PassParams p;
    bool done = false;
    const sinet_status st = pipeline_prepare(t, cols, win, label, out, accumulate, stream, &p, &done);
    if (st != SINET_OK || done) return st;
    return run_hist(p, PASS_LABEL | PASS_HIST, accumulate, stream);
}

sinet_status sinet_watch_histogram(const sinet_table* list, const sinet_columns* cols,
                                   const sinet_window* win, uint32_t n_keys,
                                   sinet_watch_hist* out, int accumulate, hipStream_t stream) {
    sinet_status st = check_usable(list);
    if (st != SINET_OK) return st;
    st = check_window(win);
    if (st != SINET_OK) return st;
    if (!cols) return fail(SINET_ERR_INVALID_ARG, "columns are NULL");
    if (!out || !out->count || !out->bytes) return fail(SINET_ERR_INVALID_ARG, "watch output is NULL");
    if (n_keys == 0) return fail(SINET_ERR_INVALID_ARG, "n_keys is 0");
    if (list->n_prefix && list->max_inst >= n_keys)
        return fail(SINET_ERR_INVALID_ARG, "a key (inst id) of the list is not below n_keys");
    if (2ull * n_keys * win->n_bins > (1ull << 40))
        return fail(SINET_ERR_INVALID_ARG, "2 * n_keys * n_bins above 2^40");
    if (cols->n && (!cols->ts || !cols->src || !cols->dst || !cols->bytes))
        return fail(SINET_ERR_INVALID_ARG, "column is NULL");
    PassParams p;
    memset(&p, 0, sizeof(p));
    p.t = list->dev;
    p.ts = cols->ts;
    p.src = cols->src;
    p.dst = cols->dst;
    p.bytes = cols->bytes;
    p.count = (unsigned long long*)out->count;
    p.hbytes = (unsigned long long*)out->bytes;
    p.dropped = (unsigned long long*)out->dropped;
    p.n = cols->n;
    p.t0 = win->t0_ms;
    p.width = win->width_ms;
    p.n_bins = win->n_bins;
    p.magic = div_magic(win->width_ms);
    return run_watch(p, n_keys, accumulate, stream);
}

sinet_status sinet_mlp_loss_grad(const float* params, const float* x, const float* y, uint64_t n,
                                 float* loss, float* grad, hipStream_t stream) {
    if (!params || !loss || !grad || (n && (!x || !y)))
        return fail(SINET_ERR_INVALID_ARG, "NULL argument");
    if (n == 0) return fail(SINET_ERR_INVALID_ARG, "n is 0");
    return mlp_loss_grad(params, x, y, n, loss, grad, stream);
}

sinet_status sinet_timing_enable(int on) { return timing_enable(on); }

sinet_status sinet_set_reduce(sinet_reduce mode) { return set_reduce((int)mode); }

sinet_status sinet_timing_read(sinet_timing* out) {
    if (!out) return fail(SINET_ERR_INVALID_ARG, "out is NULL");
    double ms[PH_COUNT];
    uint64_t calls = 0, launches = 0, window = 0;
    const sinet_status st = timing_read(ms, &calls, &launches, &window);
    if (st != SINET_OK) return st;
    out->lookup_ms = ms[PH_LOOKUP];
    out->stage1_ms = ms[PH_STAGE1];
    out->index_ms = ms[PH_INDEX];
    out->stage2_ms = ms[PH_STAGE2];
    out->far_ms = ms[PH_FAR];
    out->calls = calls;
    out->stage1_launches = launches;
    out->window_calls = window;
    return SINET_OK;
}

}  // extern "C"
