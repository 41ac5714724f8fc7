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
    const uint32_t* radix;      // PLA: first segment per radix bucket, u16 pairs
    uint32_t radix_bits;
    uint32_t pla_window;        // PLA: max_err <= kPlaWindowErr, window search in B
    uint32_t filter_lds;        // 1: /16 filter staged in LDS and used
    const uint32_t* filter;     // [kFilterWords] 2-bit state per /16 block:
                                // 0 all out, 1 all in, 2 cut by a boundary
    const float* mlp;           // [49]
    // in/out index (label-only queries): word offsets inside io[]
    const uint32_t* io;         // [io_words] or nullptr
    uint32_t io_words;
    uint32_t io_slot;           // per cut /16 block: up to four boundary offsets
    uint32_t io_list;           // overflow list of blocks with more boundaries
    uint32_t max_err;
    float m_f;                  // (float) m
    unsigned long long* fallbacks;  // device counter
    // LDS layout (bytes) chosen on the host for this table
    uint32_t lds_member_words;  // 0: member bits read from global
    uint32_t lds_bytes;
};

constexpr uint32_t kFilterWords = 65536 / 16;  // 2 bits per /16 block
constexpr uint32_t kPlaRadixBits = 12;          // PLA segment directory: top 12 address bits
constexpr uint32_t kPlaWindowErr = 6;           // largest bound one 16-boundary window serves
constexpr uint32_t kBTail = 20;                 // 0xFFFFFFFF past the padded boundaries
constexpr uint32_t kInoutKind = 6;              // internal kind: label-only via the in/out index
constexpr uint32_t kLabelInKind = 100;          // internal kind: stage 1 on stored labels
__host__ __device__ constexpr uint32_t radix_words(uint32_t bits) {
    return ((1u << bits) + 2) / 2;  // (2^bits + 1) u16 entries
}

// Partitioned histogram geometry.
constexpr int kChunk = 2048;        // sessions per stage-1 chunk
constexpr int kBlockBins = 1024;    // bins per stage-2 block (all four labels)
constexpr int kWin = 64;            // blocks one chunk may touch without the far path
constexpr int kExtraRecs = 384;     // records beyond one per session a chunk may hold
// record slots of a chunk: one per session, the extra part records of large byte
// counts, and the padding of every block's segment to whole 16-byte groups
constexpr int kChunkSlots = kChunk + kExtraRecs + 3 * kWin;
constexpr int kStage1Run = 4;       // chunks a stage-1 workgroup takes at a time
constexpr int kStage1Block = kChunk / 4;  // stage-1 lanes: 4 sessions each

// Device workspace of the partitioned histogram (carved from one allocation).
struct PartWs {
    uint32_t* rec;                  // [n_chunks * kChunkSlots] 4-byte records
    uint4* dir;                     // [n_chunks * kWin] (block, first slot, slots, -)
    uint32_t* nd;                   // [n_chunks] directory entries per chunk
    uint32_t* farbits;              // [n_chunks * kChunk / 32] far sessions (flagged chunks)
    uint32_t* farlist;              // [n_chunks] chunks holding far sessions
    uint32_t* farcount;             // [1]
    uint32_t* next_run;             // [1] next run of kStage1Run chunks to take (k_stage1)
    uint32_t* seg_count;            // [n_blocks] directory entries per block
    uint32_t* seg_off;              // [n_blocks + 1] exclusive scan of seg_count
    uint2* segs;                    // [n_chunks * kWin] (first slot, slots) grouped by block
    uint32_t* scan_tiles;           // scan scratch
    uint64_t n_chunks;
    uint32_t n_blocks;
    uint32_t vec;                   // 16-byte vector loads allowed
};

struct FarList {
    const uint32_t* list;
    const uint32_t* count;
    const uint32_t* bits;
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
    uint32_t queue_words;       // lookup pass: LDS words per wave for the search queue
                                // (0: none; set at launch)
    uint64_t magic;             // ceil(2^64 / width) for width >= 2
};

// Sliding-window histogram (window.hip): one workgroup per piece (a
// contiguous range of sessions), a ring of kWinBins bins x 4 labels in LDS.
constexpr uint32_t kWinBins = 10192;
constexpr uint32_t kWinStep = 4096;  // sessions of one window step (4 per lane)

struct WinArgs {
    const uint32_t* ts;             // session columns (labels given)
    const uint64_t* bytes;
    const uint8_t* label;
    unsigned long long* count;      // [4][n_bins] outputs, dropped [4][2] or NULL
    unsigned long long* hbytes;
    unsigned long long* dropped;
    uint64_t n;
    uint64_t magic;                 // ceil(2^64 / width) for width >= 2
    uint32_t t0, width, n_bins;
    uint32_t pieces;                // P workgroups, one piece of sessions each
    uint32_t* est;                  // [P] median bin around piece q's first session
    uint32_t* T;                    // [P + 1] owned bins of piece q: [T[q], T[q+1])
    uint32_t* V;                    // [P] first bin of piece q's left spill that was written
    uint32_t* E;                    // [P] end of piece q's right spill that was written
    uint32_t* counters;             // [4] -, events, event overflow, -
    uint32_t* far_n;                // [P] steps of piece q holding far sessions
    uint32_t* far_steps;            // [steps] those steps, piece q's listed from its first
                                    // step's slot on
    uint32_t* far_bits;             // [steps * kWinStep / 32] far-session bits of listed steps
    unsigned long long* events;     // [ev_cap] bin << 3 | label << 1 | wrap
    uint32_t* spill;                // [P][left, right][4][kWinBins] ring words (count, byte sum)
    uint64_t ev_cap;
    uint32_t vec;                   // 16-byte column loads allowed
    int accumulate;
};

// One stream of a batch as the batch kernels see it.
struct BatchStreamDev {
    PassParams p;               // label view of its table, columns, outputs, window
    uint64_t chunk0;            // first workspace chunk (partitioned streams)
    uint32_t block0;            // first workspace block (partitioned streams)
    uint32_t priv;              // 1: histogram privatised in LDS, merged by atomics
    uint32_t vec;               // 1: the stream's columns allow 16-byte loads
    uint32_t pad;
};

struct BatchArgs {
    const BatchStreamDev* streams;
    const uint4* items;         // (stream, first chunk, end chunk, -) of one kind group
    uint32_t n_items;
    uint32_t n_streams;
    uint32_t* counter;          // work-queue head of the group
    const uint64_t* chunk_base; // [n_streams + 1] first workspace chunk of each stream
    const uint32_t* block_base; // [n_streams + 1] first workspace block of each stream
    uint32_t priv_bins;         // largest private histogram (bins) of the group
    uint32_t queue_words;       // lookup pass: LDS words per wave for the window PLA's queue
};

struct ZeroJob {
    unsigned long long* p;
    uint64_t n;                 // 64-bit words
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
    uint32_t max_inst;          // largest inst id (watch-list keys must exceed it)
    // host copies used by training and tests
    std::vector<uint32_t> B, owner;
};

namespace sinet {

// status helpers (api.cpp)
sinet_status fail(sinet_status s, const std::string& msg);
sinet_status check_hip(hipError_t e, const char* what);

// api.cpp
sinet_status check_usable(const sinet_table* t);
sinet_status pipeline_prepare(const sinet_table* t, const sinet_columns* cols, const sinet_window* win,
                              uint8_t* label, sinet_hist* out, int accumulate, hipStream_t stream,
                              PassParams* p, bool* done);
sinet_status check_window(const sinet_window* w);
DevTable label_view(const sinet_table* t, bool label_only);

// kernels.hip
bool vector_ok(const PassParams& p, uint32_t kind, bool hist);
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
// histogram passes (labels computed or given) with the strategy chosen per window
sinet_status run_hist(const PassParams& p, uint32_t mode, int accumulate, hipStream_t s);
// run_hist with its workspace in `scratch` (bytes long), nothing allocated
sinet_status run_hist_in(const PassParams& p, uint32_t mode, int accumulate, hipStream_t s,
                         void* scratch, size_t bytes);
// phase timing of run_hist (event pairs on the launch stream)
enum TimedPhase { PH_LOOKUP = 0, PH_STAGE1, PH_INDEX, PH_STAGE2, PH_FAR, PH_COUNT };
sinet_status timing_enable(int on);
sinet_status set_reduce(int mode);
sinet_status timing_read(double ms[PH_COUNT], uint64_t* calls, uint64_t* stage1_launches,
                         uint64_t* window_calls);
size_t part_ws_bytes(uint64_t n, uint32_t n_bins);
PartWs part_ws_carve(void* base, uint64_t n, uint32_t n_bins);
sinet_status run_partitioned(const PassParams& p, uint32_t kind, const PartWs& w, int accumulate,
                             hipStream_t s);
int hist_strategy(const DevTable& t, uint32_t kind, uint32_t n_bins, uint64_t n);
// Watch-list histograms: count/hbytes [2][n_keys][n_bins], dropped [2][2]
// (cleared first unless accumulate); the table's inst ids are the keys.
sinet_status run_watch(const PassParams& p, uint32_t n_keys, int accumulate, hipStream_t s);
// Coarser time frames: out[r][k] = sum of in[r][k * factor ..] (rebin.hip).
sinet_status run_rebin(const uint64_t* in, uint64_t rows, uint64_t n_bins, uint32_t factor,
                       uint64_t* out, hipStream_t s);
// Session text to columns (parse.hip); synchronous, sets the line counts.
sinet_status parse_sessions(const uint8_t* text, uint64_t len, int64_t origin, const sinet_columns* out,
                            uint64_t* n_lines, uint64_t* n_bad, hipStream_t s);
sinet_status ws_alloc(void** ptr, size_t bytes, hipStream_t s);
sinet_status ws_free(void* ptr, hipStream_t s);
uint32_t device_cu_count();
uint64_t div_magic(uint32_t width);

// sliding-window histogram (window.hip)
uint32_t win_pieces(uint64_t n);
size_t win_ws_bytes(uint64_t n, uint32_t pieces);
WinArgs win_carve(void* base, const PassParams& p, uint32_t pieces, int accumulate);
sinet_status win_launch_bounds(const WinArgs& a, hipStream_t s);
sinet_status win_launch_main(const WinArgs& a, hipStream_t s);
sinet_status win_launch_fixup(const WinArgs& a, hipStream_t s);
sinet_status win_launch_far(const WinArgs& a, hipStream_t s);

// batch kernels (kernels.hip)
sinet_status launch_batch_stage1(uint32_t kind, const BatchArgs& a, const PartWs& w, size_t lds,
                                 uint32_t grid, hipStream_t s);
sinet_status launch_batch_stage2(const BatchArgs& a, const PartWs& w, uint32_t n_blocks,
                                 hipStream_t s);
sinet_status launch_batch_far(uint32_t kind, const BatchArgs& a, const PartWs& w, size_t lds,
                              hipStream_t s);
sinet_status launch_zero_jobs(const ZeroJob* jobs, uint32_t n_jobs, hipStream_t s);
sinet_status launch_scan_fill(const PartWs& w, hipStream_t s);
uint32_t batch_stage1_blocks_per_cu(uint32_t kind, size_t lds);
// lookups that run as their own pass before stage 1
bool lookup_splits(const DevTable& t);
sinet_status launch_batch_lookup(uint32_t kind, const BatchArgs& a, size_t lds, uint32_t grid,
                                 hipStream_t s);

// learned.hip
sinet_status train_pla(sinet_table* t, uint32_t segments, uint32_t target_err, uint32_t max_segments,
                       uint32_t max_window, hipStream_t s, sinet_train_report* r);
hipError_t upload_radix(sinet_table* t, const std::vector<uint32_t>& knots);
sinet_status train_mlp(sinet_table* t, const sinet_train_params* p, hipStream_t s,
                       sinet_train_report* r);
sinet_status measure_err(const DevTable& t, bool mlp, hipStream_t s, uint32_t* err);
sinet_status mlp_loss_grad(const float* params, const float* x, const float* y, uint64_t n,
                           float* loss, float* grad, hipStream_t s);

}  // namespace sinet
