// Batched form: many independent, uneven streams (each with its own table,
// window and bin width) processed by one persistent work-queue launch per
// lookup kind, all captured in one hipGraph together with the clears, the
// shared segment index, the block reduction and the far pass.
//
// The paper's coordinated batch processing (sections "Coordinated Batch
// Processing", "Work Queue", "TASK DECOMPOSITION") pulls uneven chunks from a
// queue so that every worker stays busy; its workers were host threads, one
// per GPU.  Here the workers are the GPU's workgroups and the queue is a
// device counter.  The autotuner picks the work-item size and the number of
// persistent workgroups by timing candidates; every candidate computes the
// same exact result.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "sinet_internal.h"

using namespace sinet;

struct sinet_batch_plan {
    int device = 0;
    void* arena = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    sinet_tune tune{};
};

namespace {

constexpr uint32_t kPrivMaxBins = 1024;            // LDS-private histograms up to this size
constexpr size_t kPrivLdsCap = 150 * 1024;         // table + private bins per workgroup

constexpr uint32_t kNoLookup = 0xFFFFFFFFu;

struct Prepared {
    std::vector<BatchStreamDev> desc;
    std::vector<BatchStreamDev> ldesc;  // lookup-pass descriptor of split streams
    std::vector<uint32_t> lkind;        // lookup kind of split streams, else kNoLookup
    std::vector<size_t> lds_look;       // table LDS of the lookup pass
    std::vector<uint64_t> tmp_off;      // offset of a plan-owned label buffer, or ~0
    uint64_t tmp_bytes = 0;
    std::vector<uint32_t> kind;         // kernel kind per stream
    std::vector<size_t> lds_tab;        // table LDS per stream
    std::vector<uint64_t> n_chunks;     // chunks of each stream (sessions / kChunk)
    std::vector<uint64_t> chunk_base;   // workspace chunk of each stream (+ total)
    std::vector<uint32_t> block_base;   // workspace block of each stream (+ total)
    uint64_t c_tot = 0;
    uint32_t k_tot = 0;
};

sinet_status prepare(const sinet_stream* st, uint32_t ns, Prepared& pr) {
    if (!st || ns == 0) return fail(SINET_ERR_INVALID_ARG, "no streams");
    pr.desc.resize(ns);
    pr.ldesc.resize(ns);
    pr.lkind.assign(ns, kNoLookup);
    pr.lds_look.assign(ns, 0);
    pr.tmp_off.assign(ns, ~0ull);
    pr.kind.resize(ns);
    pr.lds_tab.resize(ns);
    pr.n_chunks.resize(ns);
    pr.chunk_base.resize(ns + 1);
    pr.block_base.resize(ns + 1);
    for (uint32_t s = 0; s < ns; ++s) {
        const sinet_stream& x = st[s];
        sinet_status rc = check_usable(x.table);
        if (rc != SINET_OK) return rc;
        rc = check_window(&x.win);
        if (rc != SINET_OK) return rc;
        if (!x.hist.count || !x.hist.bytes) return fail(SINET_ERR_INVALID_ARG, "histogram output is NULL");
        if (x.cols.n && (!x.cols.ts || !x.cols.src || !x.cols.dst || !x.cols.bytes))
            return fail(SINET_ERR_INVALID_ARG, "column is NULL");
        BatchStreamDev& d = pr.desc[s];
        memset(&d, 0, sizeof(d));
        PassParams& p = d.p;
        p.t = label_view(x.table, true);
        p.ts = x.cols.ts;
        p.src = x.cols.src;
        p.dst = x.cols.dst;
        p.bytes = x.cols.bytes;
        p.label_out = x.label;
        p.count = (unsigned long long*)x.hist.count;
        p.hbytes = (unsigned long long*)x.hist.bytes;
        p.dropped = (unsigned long long*)x.hist.dropped;
        p.n = x.cols.n;
        p.t0 = x.win.t0_ms;
        p.width = x.win.width_ms;
        p.n_bins = x.win.n_bins;
        p.magic = div_magic(x.win.width_ms);
        pr.kind[s] = p.t.kind;
        pr.lds_tab[s] = p.t.lds_bytes;
        pr.n_chunks[s] = (p.n + kChunk - 1) / kChunk;
        d.priv = (p.n_bins <= kPrivMaxBins &&
                  pr.lds_tab[s] + 48ull * p.n_bins + 16 <= kPrivLdsCap) ? 1u : 0u;
        d.vec = vector_ok(p, p.t.kind, true) ? 1u : 0u;
        // lookups that walk global memory: a lookup pass stores the labels (in
        // the stream's label output, or a plan-owned buffer when it has none),
        // stage 1 reads them
        if (!d.priv && p.n && lookup_splits(p.t)) {
            pr.lkind[s] = p.t.kind;
            pr.lds_look[s] = p.t.lds_bytes;
            BatchStreamDev& l = pr.ldesc[s];
            l = d;
            if (!x.label) {
                pr.tmp_off[s] = pr.tmp_bytes;
                pr.tmp_bytes += (p.n + 255) & ~255ull;
            }
            pr.kind[s] = kLabelInKind;
            pr.lds_tab[s] = 0;
            d.p.t.kind = kLabelInKind;
            d.p.label_in = x.label;  // or the plan buffer, set when the arena exists
            d.p.label_out = nullptr;
        }
    }
    uint64_t c = 0;
    uint64_t k = 0;
    for (uint32_t s = 0; s < ns; ++s) {
        pr.chunk_base[s] = c;
        pr.block_base[s] = (uint32_t)k;
        BatchStreamDev& d = pr.desc[s];
        d.chunk0 = c;
        d.block0 = (uint32_t)k;
        if (!d.priv) {
            c += pr.n_chunks[s];
            k += (d.p.n_bins + kBlockBins - 1) / kBlockBins;
        }
    }
    pr.chunk_base[ns] = c;
    pr.block_base[ns] = (uint32_t)k;
    if (c * kChunkSlots >= (1ull << 32) || k >= (1ull << 31))
        return fail(SINET_ERR_UNSUPPORTED, "batch too large for one plan (split it)");
    pr.c_tot = c;
    pr.k_tot = (uint32_t)k;
    return SINET_OK;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

sinet_status build_plan(const sinet_stream* st, uint32_t ns, const sinet_tune& tune,
                        sinet_batch_plan* plan) {
    Prepared pr;
    sinet_status rc = prepare(st, ns, pr);
    if (rc != SINET_OK) return rc;
    const uint32_t item_chunks = std::max<uint32_t>(1, tune.chunk / kChunk);

    // kind groups and their work items
    std::vector<uint32_t> kinds;
    for (uint32_t s = 0; s < ns; ++s)
        if (std::find(kinds.begin(), kinds.end(), pr.kind[s]) == kinds.end()) kinds.push_back(pr.kind[s]);
    std::vector<std::vector<uint4>> items(kinds.size());
    std::vector<size_t> group_lds(kinds.size(), 8);
    std::vector<uint32_t> group_priv(kinds.size(), 0);
    for (uint32_t s = 0; s < ns; ++s) {
        const size_t g = std::find(kinds.begin(), kinds.end(), pr.kind[s]) - kinds.begin();
        const BatchStreamDev& d = pr.desc[s];
        size_t need = pr.lds_tab[s] + 16;
        if (d.priv) {
            need += 48ull * d.p.n_bins;
            group_priv[g] = std::max(group_priv[g], d.p.n_bins);
        }
        group_lds[g] = std::max(group_lds[g], need);
        for (uint64_t c0 = 0; c0 < pr.n_chunks[s]; c0 += item_chunks) {
            const uint64_t c1 = std::min<uint64_t>(pr.n_chunks[s], c0 + item_chunks);
            items[g].push_back(make_uint4(s, (uint32_t)c0, (uint32_t)c1, 0u));
        }
    }
    // lookup-pass groups of the split streams
    std::vector<uint32_t> lkinds;
    for (uint32_t s = 0; s < ns; ++s)
        if (pr.lkind[s] != kNoLookup &&
            std::find(lkinds.begin(), lkinds.end(), pr.lkind[s]) == lkinds.end())
            lkinds.push_back(pr.lkind[s]);
    std::vector<std::vector<uint4>> litems(lkinds.size());
    std::vector<size_t> lgroup_lds(lkinds.size(), 8);
    for (uint32_t s = 0; s < ns; ++s) {
        if (pr.lkind[s] == kNoLookup) continue;
        const size_t g = std::find(lkinds.begin(), lkinds.end(), pr.lkind[s]) - lkinds.begin();
        lgroup_lds[g] = std::max(lgroup_lds[g], pr.lds_look[s] + 16);
        for (uint64_t c0 = 0; c0 < pr.n_chunks[s]; c0 += item_chunks) {
            const uint64_t c1 = std::min<uint64_t>(pr.n_chunks[s], c0 + item_chunks);
            litems[g].push_back(make_uint4(s, (uint32_t)c0, (uint32_t)c1, 0u));
        }
    }
    // clears: queue heads, far count, directory counts, dropped, private bins
    std::vector<ZeroJob> jobs;

    // arena layout
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = al256(off + bytes); return o; };
    const size_t oDesc = take(sizeof(BatchStreamDev) * ns);
    std::vector<size_t> oItems(kinds.size());
    for (size_t g = 0; g < kinds.size(); ++g) oItems[g] = take(sizeof(uint4) * std::max<size_t>(1, items[g].size()));
    const size_t oLDesc = take(sizeof(BatchStreamDev) * ns);
    std::vector<size_t> oLItems(lkinds.size());
    for (size_t g = 0; g < lkinds.size(); ++g) oLItems[g] = take(sizeof(uint4) * litems[g].size());
    const size_t oTmp = take(pr.tmp_bytes);
    const size_t oCb = take(8ull * (ns + 1));
    const size_t oBb = take(4ull * (ns + 1));
    const size_t n_ctl = kinds.size() + lkinds.size();  // queue heads: stage 1, then lookups
    const size_t oCtl = take(8ull * n_ctl);
    const size_t ws_bytes = part_ws_bytes(std::max<uint64_t>(1, pr.c_tot) * kChunk,
                                          std::max<uint32_t>(1, pr.k_tot) * kBlockBins);
    const size_t oWs = take(ws_bytes);
    // zero jobs are counted before the arena is final
    size_t n_jobs_max = 4 + 3 * ns;
    const size_t oJobs = take(sizeof(ZeroJob) * n_jobs_max);
    void* arena = nullptr;
    hipError_t e = hipMalloc(&arena, off);
    if (e != hipSuccess) return check_hip(e, "batch plan allocation");
    plan->arena = arena;
    char* a = (char*)arena;
    const PartWs w0 = part_ws_carve(a + oWs, std::max<uint64_t>(1, pr.c_tot) * kChunk,
                                    std::max<uint32_t>(1, pr.k_tot) * kBlockBins);
    PartWs w = w0;
    w.n_chunks = pr.c_tot;
    w.n_blocks = pr.k_tot;
    w.vec = 0;  // unused by the batch kernels: vector loads are chosen per stream
    // label buffers of the split streams, and the vector-load choice now that
    // every address is known
    for (uint32_t s = 0; s < ns; ++s) {
        if (pr.lkind[s] == kNoLookup) continue;
        BatchStreamDev& d = pr.desc[s];
        BatchStreamDev& l = pr.ldesc[s];
        if (pr.tmp_off[s] != ~0ull) d.p.label_in = (const uint8_t*)(a + oTmp + pr.tmp_off[s]);
        l.p.label_out = const_cast<uint8_t*>(d.p.label_in);
        l.vec = vector_ok(l.p, l.p.t.kind, false) ? 1u : 0u;
        d.vec = vector_ok(d.p, kLabelInKind, true) ? 1u : 0u;
    }
    jobs.push_back({(unsigned long long*)(a + oCtl), (uint64_t)n_ctl});
    jobs.push_back({(unsigned long long*)w.farcount, 1});
    if (pr.k_tot) jobs.push_back({(unsigned long long*)w.seg_count, (pr.k_tot + 1) / 2});
    for (uint32_t s = 0; s < ns; ++s) {
        const BatchStreamDev& d = pr.desc[s];
        if (d.p.dropped) jobs.push_back({d.p.dropped, 8});
        if (d.priv) {
            jobs.push_back({d.p.count, 4ull * d.p.n_bins});
            jobs.push_back({d.p.hbytes, 4ull * d.p.n_bins});
        }
    }
    e = hipMemcpy(a + oDesc, pr.desc.data(), sizeof(BatchStreamDev) * ns, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(a + oLDesc, pr.ldesc.data(), sizeof(BatchStreamDev) * ns, hipMemcpyHostToDevice);
    for (size_t g = 0; e == hipSuccess && g < lkinds.size(); ++g)
        e = hipMemcpy(a + oLItems[g], litems[g].data(), sizeof(uint4) * litems[g].size(),
                      hipMemcpyHostToDevice);
    for (size_t g = 0; e == hipSuccess && g < kinds.size(); ++g)
        if (!items[g].empty())
            e = hipMemcpy(a + oItems[g], items[g].data(), sizeof(uint4) * items[g].size(),
                          hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(a + oCb, pr.chunk_base.data(), 8ull * (ns + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(a + oBb, pr.block_base.data(), 4ull * (ns + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(a + oJobs, jobs.data(), sizeof(ZeroJob) * jobs.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return check_hip(e, "batch plan upload");

    std::vector<BatchArgs> args(kinds.size());
    std::vector<uint32_t> grids(kinds.size());
    for (size_t g = 0; g < kinds.size(); ++g) {
        BatchArgs& ba = args[g];
        memset(&ba, 0, sizeof(ba));
        ba.streams = (const BatchStreamDev*)(a + oDesc);
        ba.items = (const uint4*)(a + oItems[g]);
        ba.n_items = (uint32_t)items[g].size();
        ba.n_streams = ns;
        ba.counter = (uint32_t*)(a + oCtl + 8 * g);
        ba.chunk_base = (const uint64_t*)(a + oCb);
        ba.block_base = (const uint32_t*)(a + oBb);
        ba.priv_bins = group_priv[g];
        // occupancy queries before capture
        const uint32_t occ = batch_stage1_blocks_per_cu(kinds[g], group_lds[g]);
        grids[g] = tune.grid ? tune.grid : device_cu_count() * occ;
    }

    std::vector<BatchArgs> largs(lkinds.size());
    for (size_t g = 0; g < lkinds.size(); ++g) {
        BatchArgs& ba = largs[g];
        memset(&ba, 0, sizeof(ba));
        ba.streams = (const BatchStreamDev*)(a + oLDesc);
        ba.items = (const uint4*)(a + oLItems[g]);
        ba.n_items = (uint32_t)litems[g].size();
        ba.n_streams = ns;
        ba.counter = (uint32_t*)(a + oCtl + 8 * (kinds.size() + g));
        ba.chunk_base = (const uint64_t*)(a + oCb);
        ba.block_base = (const uint32_t*)(a + oBb);
    }

    // capture
    e = hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return check_hip(e, "capture stream");
    hipStream_t cs = plan->cap;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return check_hip(e, "begin capture");
    rc = launch_zero_jobs((const ZeroJob*)(a + oJobs), (uint32_t)jobs.size(), cs);
    for (size_t g = 0; rc == SINET_OK && g < lkinds.size(); ++g)
        rc = launch_batch_lookup(lkinds[g], largs[g], lgroup_lds[g], 0, cs);
    for (size_t g = 0; rc == SINET_OK && g < kinds.size(); ++g)
        if (args[g].n_items) rc = launch_batch_stage1(kinds[g], args[g], w, group_lds[g], grids[g], cs);
    if (rc == SINET_OK && pr.k_tot) rc = launch_scan_fill(w, cs);
    if (rc == SINET_OK && pr.k_tot) rc = launch_batch_stage2(args[0], w, pr.k_tot, cs);
    for (size_t g = 0; rc == SINET_OK && pr.k_tot && g < kinds.size(); ++g)
        rc = launch_batch_far(kinds[g], args[g], w, pr.lds_tab.empty() ? 8 : group_lds[g], cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    if (rc != SINET_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return check_hip(e, "end capture");
    plan->graph = graph;
    e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return check_hip(e, "graph instantiate");
    plan->tune = tune;
    plan->tune.block = kStage1Block;
    return SINET_OK;
}

void destroy_plan(sinet_batch_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->arena) (void)hipFree(p->arena);
    delete p;
}

sinet_tune default_tune() {
    sinet_tune t{};
    t.block = kStage1Block;
    t.chunk = 4 * kChunk;
    t.grid = 0;
    return t;
}

std::string signature(const sinet_stream* st, uint32_t ns) {
    uint64_t n = 0, bins = 0, pfx = 0;
    for (uint32_t s = 0; s < ns; ++s) {
        n += st[s].cols.n;
        bins += st[s].win.n_bins;
        pfx += st[s].table ? st[s].table->n_prefix : 0;
    }
    char buf[160];
    snprintf(buf, sizeof(buf), "streams=%u sessions=%llu bins=%llu prefixes=%llu cus=%u", ns,
             (unsigned long long)n, (unsigned long long)bins, (unsigned long long)pfx,
             device_cu_count());
    return buf;
}

bool cache_lookup(const char* path, const std::string& sig, sinet_tune* out) {
    FILE* f = path ? fopen(path, "r") : nullptr;
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        if (!strstr(line, sig.c_str())) continue;
        unsigned b = 0, c = 0, g = 0;
        const char* pb = strstr(line, "\"block\":");
        const char* pc = strstr(line, "\"chunk\":");
        const char* pg = strstr(line, "\"grid\":");
        if (pb && pc && pg && sscanf(pb, "\"block\":%u", &b) == 1 && sscanf(pc, "\"chunk\":%u", &c) == 1 &&
            sscanf(pg, "\"grid\":%u", &g) == 1 && c >= (unsigned)kChunk) {
            out->block = b;
            out->chunk = c;
            out->grid = g;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& sig, const sinet_tune& t, float ms) {
    if (!path) return;
    std::vector<std::string> keep;
    if (FILE* f = fopen(path, "r")) {
        char line[512];
        while (fgets(line, sizeof(line), f))
            if (!strstr(line, sig.c_str())) keep.push_back(line);
        fclose(f);
    }
    FILE* f = fopen(path, "w");
    if (!f) return;
    for (const auto& l : keep) fputs(l.c_str(), f);
    fprintf(f, "{\"sig\": \"%s\", \"block\":%u, \"chunk\":%u, \"grid\":%u, \"ms\": %.4f}\n", sig.c_str(),
            t.block, t.chunk, t.grid, ms);
    fclose(f);
}

}  // namespace

extern "C" {

sinet_status sinet_batch_plan_create(const sinet_stream* streams, uint32_t n_streams,
                                     const sinet_tune* tune, hipStream_t stream,
                                     sinet_batch_plan** out) {
    (void)stream;
    if (!out) return fail(SINET_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    sinet_tune t = tune ? *tune : default_tune();
    if (t.chunk < (uint32_t)kChunk) t.chunk = kChunk;
    sinet_batch_plan* plan = new sinet_batch_plan();
    (void)hipGetDevice(&plan->device);
    sinet_status rc = build_plan(streams, n_streams, t, plan);
    if (rc != SINET_OK) {
        destroy_plan(plan);
        return rc;
    }
    *out = plan;
    return SINET_OK;
}

sinet_status sinet_batch_run(sinet_batch_plan* plan, hipStream_t stream) {
    if (!plan || !plan->exec) return fail(SINET_ERR_INVALID_ARG, "plan is NULL");
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev != plan->device) return fail(SINET_ERR_INVALID_ARG, "plan belongs to another device");
    return check_hip(hipGraphLaunch(plan->exec, stream), "batch graph launch");
}

sinet_status sinet_batch_plan_destroy(sinet_batch_plan* plan) {
    if (!plan) return fail(SINET_ERR_INVALID_ARG, "plan is NULL");
    destroy_plan(plan);
    return SINET_OK;
}

sinet_status sinet_autotune(const sinet_stream* streams, uint32_t n_streams, const char* cache_path,
                            hipStream_t stream, sinet_tune* out) {
    if (!out || !streams || n_streams == 0) return fail(SINET_ERR_INVALID_ARG, "NULL argument");
    const std::string sig = signature(streams, n_streams);
    if (cache_lookup(cache_path, sig, out)) return SINET_OK;
    const uint32_t cus = device_cu_count();
    const uint32_t chunks[] = {(uint32_t)kChunk, 4u * kChunk, 16u * kChunk};
    const uint32_t grids[] = {0u, cus / 2};
    sinet_tune best = default_tune();
    float best_ms = 1e30f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(SINET_ERR_DEVICE, "event creation");
    sinet_status rc = SINET_OK;
    for (uint32_t c : chunks) {
        for (uint32_t g : grids) {
            sinet_tune t{};
            t.block = kStage1Block;
            t.chunk = c;
            t.grid = g;
            sinet_batch_plan* plan = nullptr;
            rc = sinet_batch_plan_create(streams, n_streams, &t, stream, &plan);
            if (rc != SINET_OK) break;
            float ms = 0.f;
            rc = sinet_batch_run(plan, stream);  // warm-up
            if (rc == SINET_OK) {
                (void)hipEventRecord(e0, stream);
                for (int r = 0; r < 3 && rc == SINET_OK; ++r) rc = sinet_batch_run(plan, stream);
                (void)hipEventRecord(e1, stream);
                if (hipEventSynchronize(e1) != hipSuccess) rc = fail(SINET_ERR_DEVICE, "tuning run");
                (void)hipEventElapsedTime(&ms, e0, e1);
            }
            sinet_batch_plan_destroy(plan);
            if (rc != SINET_OK) break;
            if (ms / 3 < best_ms) {
                best_ms = ms / 3;
                best = t;
            }
        }
        if (rc != SINET_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SINET_OK) return rc;
    cache_store(cache_path, sig, best, best_ms);
    *out = best;
    return SINET_OK;
}

}  // extern "C"
