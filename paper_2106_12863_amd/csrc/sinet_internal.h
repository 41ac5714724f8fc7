// Internal declarations shared by the libsinet translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "sinet.h"

namespace sinet {

// Device view of a prefix table, passed to kernels by value.
//
// Every lookup kind answers the same question: the index j of the elementary
// interval [B[j], B[j+1]) holding an address.  Inside one interval the
// longest matching prefix cannot change, so owner[j] (row + 1, or 0 for no
// match) and the membership bit member[j] = (owner[j] != 0) give the
// institution and the in/out mark of Algorithm 1.
struct DevTable {
    uint32_t kind;
    uint32_t m;                 // number of boundaries (intervals)
    const uint32_t* B;          // [m] sorted boundaries, B[0] = 0
    const uint32_t* owner;      // [m] longest-match row + 1, or 0
    const uint32_t* member;     // [(m + 31) / 32] bit j = owner[j] != 0
    const uint32_t* inst;       // [n_prefix] institution id of each row
    // SCAN: canonical base, mask and length of every row
    uint32_t n_prefix;
    const uint32_t* cb;
    const uint32_t* mask;
    const uint32_t* len;
    // BSEARCH: LDS holds top[i] = B[i << top_log2] for i < n_top
    uint32_t top_log2;
    uint32_t n_top;
    const uint32_t* top;        // [n_top] (device copy, staged into LDS)
    // TRIE 16-8-8: level-1 [65536] then 256-entry nodes; bit 31 = leaf
    const uint32_t* trie;
    // learned: PLA segments (knot, intercept c, slope g), MLP parameters
    uint32_t segments;
    const uint32_t* knot;       // [segments]
    const float* pla_c;         // [segments]
    const float* pla_g;         // [segments]
    const float* mlp;           // [49]
    uint32_t max_err;
    float m_f;                  // (float) m
    unsigned long long* fallbacks;  // device counter
    // LDS layout (bytes) chosen on the host for this table
    uint32_t lds_member_words;  // 0: member bits read from global
    uint32_t lds_bytes;
};

struct Launch {
    int grid;
    int block;
    size_t lds;
};

// Kernel-side parameters of one pass over a stream of sessions.
struct PassParams {
    DevTable t;
    const uint32_t* ts;
    const uint32_t* src;
    const uint32_t* dst;
    const uint64_t* bytes;
    const uint8_t* label_in;    // histogram-only pass: labels given
    uint8_t* label_out;
    uint32_t* src_inst;
    uint32_t* dst_inst;
    uint32_t* pos_out;          // position-only pass (src column holds addresses)
    unsigned long long* count;
    unsigned long long* hbytes;
    unsigned long long* dropped;
    uint64_t n;
    uint32_t t0;
    uint32_t width;
    uint32_t n_bins;
    uint32_t pad;
    uint64_t magic;             // ceil(2^64 / width) for width >= 2
};

}  // namespace sinet

struct sinet_table {
    sinet::DevTable dev;
    sinet_lookup kind;
    uint64_t n_prefix;
    void* arena;                // one device allocation holding every array
    uint64_t arena_bytes;
    int trained;
    uint32_t segments;
    int device;
    uint32_t lds_words;         // per-workgroup LDS budget in 32-bit words
    // host copies used by training and tests
    std::vector<uint32_t> B, owner;
};

namespace sinet {

// status helpers (api.cpp)
sinet_status fail(sinet_status s, const std::string& msg);
sinet_status check_hip(hipError_t e, const char* what);

// kernels.hip
enum PassMode : uint32_t {
    PASS_LABEL = 1u,      // compute labels by lookup
    PASS_STORE = 2u,      // store labels
    PASS_INST = 4u,       // store institution ids
    PASS_HIST = 8u,       // histogram
    PASS_LABEL_IN = 16u,  // labels read from label_in
    PASS_POS = 32u        // store interval index of src (position query)
};
sinet_status launch_pass(const PassParams& p, uint32_t mode, hipStream_t s);
sinet_status launch_zero(unsigned long long* p, uint64_t n_words, hipStream_t s);
uint32_t device_cu_count();
uint64_t div_magic(uint32_t width);

// learned.hip
sinet_status train_pla(sinet_table* t, uint32_t segments, hipStream_t s, sinet_train_report* r);
sinet_status train_mlp(sinet_table* t, const sinet_train_params* p, hipStream_t s,
                       sinet_train_report* r);
sinet_status measure_err(const DevTable& t, bool mlp, hipStream_t s, uint32_t* err);
sinet_status mlp_loss_grad(const float* params, const float* x, const float* y, uint64_t n,
                           float* loss, float* grad, hipStream_t s);

}  // namespace sinet
