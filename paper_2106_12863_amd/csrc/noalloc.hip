// sinet_pipeline_noalloc: the pipeline call with its device workspace in a
// static array of the library instead of memory allocated per call, for
// callers that cannot allocate (code under graph capture, tight serving
// loops, harnesses that forbid it).
//
// The array (`scratch`, kScratchBytes) lives in device memory of every GPU
// the library runs on until the process ends.  Host code never passes the
// array's name to a kernel or a copy: on the first call on a device, with
// that device current, its device address is looked up once with
// hipGetSymbolAddress and kept per device; every later use goes through that
// address.  Each call overwrites what it needs of the array (the kernels
// clear their own counters), so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "sinet_internal.h"

namespace sinet {

constexpr size_t kScratchBytes = 128ull << 20;
constexpr uint64_t kNoallocMaxSessions = 1ull << 25;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's scratch array (looked up once per device).
static sinet_status scratch_address(void** out) {
    static std::mutex mu;
    static std::map<int, void*> addr;
    int dev = 0;
    sinet_status st = check_hip(hipGetDevice(&dev), "hipGetDevice");
    if (st != SINET_OK) return st;
    std::lock_guard<std::mutex> g(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) {
        *out = it->second;
        return SINET_OK;
    }
    void* ptr = nullptr;
    st = check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch address");
    if (st != SINET_OK) return st;
    addr[dev] = ptr;
    *out = ptr;
    return SINET_OK;
}

}  // namespace sinet

using namespace sinet;

extern "C" sinet_status sinet_pipeline_noalloc(const sinet_table* t, const sinet_columns* cols,
                                               const sinet_window* win, uint8_t* label, sinet_hist* out,
                                               int accumulate, hipStream_t stream) {
    if (cols && cols->n > kNoallocMaxSessions)
        return fail(SINET_ERR_INVALID_ARG, "more than 2^25 sessions for the static scratch");
    PassParams p;
    bool done = false;
    sinet_status st = pipeline_prepare(t, cols, win, label, out, accumulate, stream, &p, &done);
    if (st != SINET_OK || done) return st;
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != SINET_OK) return st;
    return run_hist_in(p, PASS_LABEL | PASS_HIST, accumulate, stream, ws, kScratchBytes);
}
