// Out-of-core pipeline: session columns held in host memory are streamed
// through device staging buffers chunk by chunk, and the fused pipeline's
// histogram accumulates over the chunks (the paper's per-chunk results merged
// by addition, section "Pairwise Reduction Pattern with GPU"; Table 3's
// out-of-memory runs are the case this removes).
//
// Two staging slots alternate.  While the device classifies and bins chunk k
// from one slot, chunk k + 1 is copied host-to-device into the other on the
// streamer's own copy stream; columns in pageable memory are first copied
// into pinned staging by host threads.  Labels come back the same way.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <thread>
#include <vector>

#include "sinet.h"
#include "sinet_internal.h"

namespace sinet {
namespace {

constexpr int kSlots = 2;
constexpr unsigned kCopyThreads = 8;  // host threads filling pinned staging

struct Slot {
    // device staging: ts, src, dst (u32), bytes (u64), labels (u8)
    uint32_t* d_ts = nullptr;
    uint32_t* d_src = nullptr;
    uint32_t* d_dst = nullptr;
    uint64_t* d_bytes = nullptr;
    uint8_t* d_label = nullptr;
    // pinned host staging for pageable columns and labels
    uint32_t* h_ts = nullptr;
    uint32_t* h_src = nullptr;
    uint32_t* h_dst = nullptr;
    uint64_t* h_bytes = nullptr;
    uint8_t* h_label = nullptr;
    hipEvent_t copied = nullptr;  // the slot's columns are on the device
    hipEvent_t done = nullptr;    // the slot's chunk is binned and its labels are back
    uint64_t label_off = 0;       // where the slot's labels go in the caller's array
    uint64_t label_n = 0;         // labels waiting in h_label (0: none)
};

bool host_pinned(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable memory reports an error here
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

// memcpy split over host threads (pageable -> pinned staging).
void par_copy(void* dst, const void* src, size_t bytes) {
    if (bytes < (8u << 20)) {
        memcpy(dst, src, bytes);
        return;
    }
    const size_t part = (bytes / kCopyThreads + 63) & ~(size_t)63;
    std::vector<std::thread> th;
    for (unsigned k = 0; k < kCopyThreads; ++k) {
        const size_t a = k * part;
        if (a >= bytes) break;
        const size_t n = std::min(part, bytes - a);
        th.emplace_back([=] { memcpy((char*)dst + a, (const char*)src + a, n); });
    }
    for (auto& t : th) t.join();
}

}  // namespace
}  // namespace sinet

struct sinet_streamer {
    uint64_t chunk = 0;
    int device = 0;
    hipStream_t copy = nullptr;
    sinet::Slot slot[sinet::kSlots];
};

using namespace sinet;

static void streamer_free(sinet_streamer* s) {
    if (!s) return;
    for (Slot& x : s->slot) {
        (void)hipFree(x.d_ts);
        (void)hipFree(x.d_src);
        (void)hipFree(x.d_dst);
        (void)hipFree(x.d_bytes);
        (void)hipFree(x.d_label);
        (void)hipHostFree(x.h_ts);
        (void)hipHostFree(x.h_src);
        (void)hipHostFree(x.h_dst);
        (void)hipHostFree(x.h_bytes);
        (void)hipHostFree(x.h_label);
        if (x.copied) (void)hipEventDestroy(x.copied);
        if (x.done) (void)hipEventDestroy(x.done);
    }
    if (s->copy) (void)hipStreamDestroy(s->copy);
    delete s;
}

extern "C" {

sinet_status sinet_streamer_create(uint64_t chunk_sessions, sinet_streamer** out) {
    if (!out) return fail(SINET_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (chunk_sessions == 0) return fail(SINET_ERR_INVALID_ARG, "chunk_sessions is 0");
    if (chunk_sessions > (1ull << 31)) return fail(SINET_ERR_INVALID_ARG, "chunk_sessions above 2^31");
    sinet_streamer* s = new sinet_streamer();
    s->chunk = chunk_sessions;
    (void)hipGetDevice(&s->device);
    const uint64_t c = chunk_sessions;
    // default priority; non-blocking, so it never waits for work on the null
    // stream implicitly (the events between the streams order everything)
    hipError_t e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    for (Slot& x : s->slot) {
        if (e == hipSuccess) e = hipMalloc((void**)&x.d_ts, 4 * c);
        if (e == hipSuccess) e = hipMalloc((void**)&x.d_src, 4 * c);
        if (e == hipSuccess) e = hipMalloc((void**)&x.d_dst, 4 * c);
        if (e == hipSuccess) e = hipMalloc((void**)&x.d_bytes, 8 * c);
        if (e == hipSuccess) e = hipMalloc((void**)&x.d_label, c);
        if (e == hipSuccess) e = hipHostMalloc((void**)&x.h_ts, 4 * c, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&x.h_src, 4 * c, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&x.h_dst, 4 * c, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&x.h_bytes, 8 * c, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void**)&x.h_label, c, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x.copied, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&x.done, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        streamer_free(s);
        return check_hip(e, "streamer staging");
    }
    *out = s;
    return SINET_OK;
}

sinet_status sinet_streamer_destroy(sinet_streamer* s) {
    if (!s) return SINET_OK;
    (void)hipStreamSynchronize(s->copy);
    for (Slot& x : s->slot) (void)hipEventSynchronize(x.done);
    streamer_free(s);
    return SINET_OK;
}

sinet_status sinet_streamer_pipeline(sinet_streamer* s, const sinet_table* t,
                                     const sinet_columns* host_cols, const sinet_window* win,
                                     uint8_t* host_label, sinet_hist* out, int accumulate,
                                     hipStream_t stream) {
    if (!s) return fail(SINET_ERR_INVALID_ARG, "streamer is NULL");
    sinet_status st = check_usable(t);
    if (st != SINET_OK) return st;
    st = check_window(win);
    if (st != SINET_OK) return st;
    if (!host_cols) return fail(SINET_ERR_INVALID_ARG, "columns are NULL");
    if (!out || !out->count || !out->bytes) return fail(SINET_ERR_INVALID_ARG, "histogram output is NULL");
    const uint64_t n = host_cols->n;
    if (n && (!host_cols->ts || !host_cols->src || !host_cols->dst || !host_cols->bytes))
        return fail(SINET_ERR_INVALID_ARG, "column is NULL");
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev != s->device) return fail(SINET_ERR_INVALID_ARG, "streamer belongs to another device");
    if (n == 0) {
        sinet_columns none{nullptr, nullptr, nullptr, nullptr, 0};
        st = sinet_pipeline(t, &none, win, nullptr, out, accumulate, stream);
        if (st == SINET_OK) st = check_hip(hipStreamSynchronize(stream), "streamed pipeline");
        return st;
    }
    // pinned caller memory is copied from directly
    const bool pin_in = host_pinned(host_cols->ts) && host_pinned(host_cols->src) &&
                        host_pinned(host_cols->dst) && host_pinned(host_cols->bytes);
    const bool pin_lab = host_label && host_pinned(host_label);
    auto drain = [&](Slot& x) -> sinet_status {
        sinet_status r = check_hip(hipEventSynchronize(x.done), "streamed chunk");
        if (r == SINET_OK && x.label_n) par_copy(host_label + x.label_off, x.h_label, x.label_n);
        x.label_n = 0;
        return r;
    };
    const uint64_t chunks = (n + s->chunk - 1) / s->chunk;
    for (uint64_t k = 0; k < chunks && st == SINET_OK; ++k) {
        Slot& x = s->slot[k % kSlots];
        const uint64_t i0 = k * s->chunk;
        const uint64_t len = std::min(s->chunk, n - i0);
        // the slot's previous chunk is binned and its labels are back on the host
        if (k >= (uint64_t)kSlots) st = drain(x);
        if (st != SINET_OK) break;
        const void* src_ts = host_cols->ts + i0;
        const void* src_src = host_cols->src + i0;
        const void* src_dst = host_cols->dst + i0;
        const void* src_bytes = host_cols->bytes + i0;
        if (!pin_in) {
            par_copy(x.h_ts, src_ts, 4 * len);
            par_copy(x.h_src, src_src, 4 * len);
            par_copy(x.h_dst, src_dst, 4 * len);
            par_copy(x.h_bytes, src_bytes, 8 * len);
            src_ts = x.h_ts;
            src_src = x.h_src;
            src_dst = x.h_dst;
            src_bytes = x.h_bytes;
        }
        hipError_t e = hipMemcpyAsync(x.d_ts, src_ts, 4 * len, hipMemcpyHostToDevice, s->copy);
        if (e == hipSuccess) e = hipMemcpyAsync(x.d_src, src_src, 4 * len, hipMemcpyHostToDevice, s->copy);
        if (e == hipSuccess) e = hipMemcpyAsync(x.d_dst, src_dst, 4 * len, hipMemcpyHostToDevice, s->copy);
        if (e == hipSuccess)
            e = hipMemcpyAsync(x.d_bytes, src_bytes, 8 * len, hipMemcpyHostToDevice, s->copy);
        if (e == hipSuccess) e = hipEventRecord(x.copied, s->copy);
        if (e == hipSuccess) e = hipStreamWaitEvent(stream, x.copied, 0);
        st = check_hip(e, "streamed copy");
        if (st != SINET_OK) break;
        sinet_columns c{x.d_ts, x.d_src, x.d_dst, x.d_bytes, len};
        st = sinet_pipeline(t, &c, win, host_label ? x.d_label : nullptr, out,
                            (k > 0 || accumulate) ? 1 : 0, stream);
        if (st != SINET_OK) break;
        if (host_label) {
            uint8_t* dst = pin_lab ? host_label + i0 : x.h_label;
            e = hipMemcpyAsync(dst, x.d_label, len, hipMemcpyDeviceToHost, stream);
            if (!pin_lab) {
                x.label_off = i0;
                x.label_n = len;
            }
        }
        // the host waits for this event before it refills the slot (drain),
        // so the copy stream itself never waits for the kernels
        if (e == hipSuccess) e = hipEventRecord(x.done, stream);
        st = check_hip(e, "streamed chunk");
    }
    for (Slot& x : s->slot) {
        const sinet_status r = drain(x);
        if (st == SINET_OK) st = r;
    }
    return st;
}

}  // extern "C"
