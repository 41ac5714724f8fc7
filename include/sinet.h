/*
 * sinet.h -- C ABI of libsinet: per-session ingress/egress discrimination of
 * IPv4 sessions against a backbone prefix table, fused with an exact
 * millisecond histogram, on one AMD Instinct MI355X (gfx950).
 *
 * The operations follow Ando, Kadobayashi and Takakura, "Choice of
 * Parallelism: Multi-GPU Driven Pipeline for Huge Academic Backbone Network"
 * (arXiv 2106.12863):
 *   - discrimination: Algorithm 1 and the section "Threads for traffic
 *     direction discrimination with CIDR MATCH" (mask the address and the
 *     CIDR base to Z bits, subtract, a zero result is a match);
 *   - histogramming: the sections "Map", "Reduce", "Pairwise Reduction
 *     Pattern with GPU" and "Merge Scatter Pattern with CPU" (key = time
 *     bin, values <timestamp,count> and <timestamp,bytes>, 1-ms bins, merged
 *     by an associative and commutative addition);
 *   - batching of many uneven chunks through one work queue: sections
 *     "Coordinated Batch Processing", "Work Queue" and "TASK DECOMPOSITION".
 * The learned position model is not in the paper; it only changes how fast
 * the exact interval is found.
 *
 * Conventions for every call:
 *   - Column, label, institution and histogram buffers are DEVICE pointers
 *     owned by the caller (hipMalloc or a framework tensor).  Prefix-table
 *     inputs of sinet_table_create are HOST pointers, copied.
 *   - Every call that takes a stream only enqueues work on it and returns;
 *     the caller synchronises.  Argument errors are detected on the host
 *     and returned before anything is enqueued.  A device fault surfaces as
 *     SINET_ERR_DEVICE from a later call.
 *   - n == 0 is a successful no-op (with accumulate == 0 the histogram is
 *     still cleared).
 *   - sinet_last_error() gives a thread-local description of the last
 *     non-OK status.
 *   - Tables and plans are library-owned; destroy them with their destroy
 *     call.  A table is read-only after create/train and may be used by
 *     concurrent calls on different streams.
 */
#ifndef SINET_H
#define SINET_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SINET_OK = 0,
    SINET_ERR_INVALID_ARG = 1,
    SINET_ERR_OUT_OF_MEMORY = 2,
    SINET_ERR_DEVICE = 3,
    SINET_ERR_UNSUPPORTED = 4
} sinet_status;

/* Session label: bit 0 = source inside the table (the paper's "outgoing"
 * mark of Algorithm 1), bit 1 = destination inside the table. */
typedef enum {
    SINET_EXTERNAL = 0,
    SINET_EGRESS = 1,
    SINET_INGRESS = 2,
    SINET_INTERNAL = 3
} sinet_label;

/* How a table answers "which interval holds this address".  All kinds give
 * identical results; they differ only in speed. */
typedef enum {
    SINET_LOOKUP_AUTO = 0,        /* scan for <= 64 prefixes, else bsearch   */
    SINET_LOOKUP_SCAN = 1,        /* Algorithm 1 over every row (<= 1024)    */
    SINET_LOOKUP_BSEARCH = 2,     /* binary search over sorted boundaries    */
    SINET_LOOKUP_TRIE = 3,        /* 16-8-8 multibit trie                    */
    SINET_LOOKUP_LEARNED_PLA = 4, /* piecewise-linear model + bounded search */
    SINET_LOOKUP_LEARNED_MLP = 5  /* 1-16-1 ReLU MLP + bounded search        */
} sinet_lookup;

/* OR-ed into the kind argument of sinet_table_create: do not build the
 * in/out index, so label-only queries also run the kind's own search. */
#define SINET_TABLE_NO_INOUT_INDEX 0x100u
/* OR-ed into the kind argument: a BSEARCH table searches the boundaries in
 * global memory from the first probe (no LDS copy of sampled boundaries),
 * i.e. the plain binary search. */
#define SINET_TABLE_GLOBAL_BSEARCH 0x200u

#define SINET_NO_INST 0xFFFFFFFFu
#define SINET_MAX_PREFIXES (1u << 22)
#define SINET_MLP_PARAMS 49

typedef struct sinet_table sinet_table;           /* opaque, device-resident */
typedef struct sinet_batch_plan sinet_batch_plan; /* opaque: queue + graph   */

/* Session columns, structure of arrays, n sessions (device pointers).
 * ts: capture time in ms (u32), src/dst: IPv4 host order, bytes: u64. */
typedef struct {
    const uint32_t* ts;
    const uint32_t* src;
    const uint32_t* dst;
    const uint64_t* bytes;
    uint64_t n;
} sinet_columns;

/* Histogram window: bin = floor((ts - t0_ms) / width_ms) for
 * t0_ms <= ts and bin < n_bins; other sessions are counted in dropped. */
typedef struct {
    uint32_t t0_ms;
    uint32_t width_ms;
    uint32_t n_bins;
} sinet_window;

/* Histogram outputs (device): count[4][n_bins] and bytes[4][n_bins],
 * label-major, unsigned 64-bit, exact modulo 2^64; dropped[4][2] =
 * {count, bytes} per label, or NULL. */
typedef struct {
    uint64_t* count;
    uint64_t* bytes;
    uint64_t* dropped;
} sinet_hist;

/* Watch-list histogram outputs (device): count[2][n_keys][n_bins] and
 * bytes[2][n_keys][n_bins], direction-major, then key, then bin; unsigned
 * 64-bit, exact modulo 2^64.  dropped[2][2] = {count, bytes} of the matched
 * sessions outside the window per direction, or NULL. */
typedef enum {
    SINET_WATCH_SRC = 0,    /* the source matched the list: for a list of outside
                               hosts, sessions coming in from them            */
    SINET_WATCH_DST = 1     /* the destination matched: sessions going out to them */
} sinet_watch_dir;

typedef struct {
    uint64_t* count;
    uint64_t* bytes;
    uint64_t* dropped;
} sinet_watch_hist;

typedef struct {
    uint32_t kind;          /* sinet_lookup of the table                     */
    uint32_t inout_index;   /* 1: label-only queries use the in/out index    */
    uint64_t n_prefix;
    uint64_t m;             /* number of interval boundaries                 */
    uint64_t device_bytes;  /* device memory held by the table               */
    uint32_t trained;       /* learned kinds: 1 after sinet_table_train      */
    uint32_t max_err;       /* learned kinds: measured bound of the search   */
    uint32_t segments;      /* PLA: number of segments                       */
    uint32_t pla_window;    /* PLA: 1 when max_err <= 6, so that each lookup
                               reads one aligned window of 16 boundaries from
                               device memory instead of searching an LDS
                               sample of them                                */
    uint64_t fallbacks;     /* learned kinds: bounded searches that fell back
                               to the full search since create (synchronous
                               read of a device counter)                     */
} sinet_table_info_t;

typedef struct {
    uint32_t steps;         /* MLP: full-batch Adam steps (default 2000)     */
    float lr;               /* MLP: Adam step size (default 1e-2)            */
    const float* init;      /* MLP: host[49] start parameters, or NULL for
                               hinges at k/16                                */
    uint32_t segments;      /* PLA: equal-count least-squares segments, 1..65535;
                               0 = error-bounded segmentation (target_err)   */
    uint32_t target_err;    /* PLA with segments == 0: greedy segmentation with
                               at most this error in boundaries (default 8;
                               raised until the segments fit in LDS)          */
} sinet_train_params;

typedef struct {
    float loss_first;       /* MLP: loss before the first step               */
    float loss_last;        /* MLP: loss after the last step                 */
    uint32_t max_err_untrained; /* MLP: bound with the start parameters      */
    uint32_t max_err;       /* bound after training                          */
    double train_ms;        /* device time of the training (hipEvents)       */
} sinet_train_report;

/* Autotuned launch parameters of the batched persistent kernel. */
typedef struct {
    uint32_t block;         /* threads per workgroup (64..1024, multiple of 64) */
    uint32_t chunk;         /* sessions per work item (multiple of 4*block)  */
    uint32_t grid;          /* persistent workgroups (0: one per slot)       */
    uint32_t reserved;
} sinet_tune;

/* One independent stream of a batch: its columns, table, window and outputs. */
typedef struct {
    sinet_columns cols;
    const sinet_table* table;
    sinet_window win;
    uint8_t* label;         /* device [n] or NULL                            */
    sinet_hist hist;
} sinet_stream;

const char* sinet_status_string(sinet_status s);
const char* sinet_last_error(void);
const char* sinet_version(void);

/* Build a table from n_prefix rows (HOST arrays, copied).  Besides the
 * structure of its lookup kind, every table except SCAN gets an in/out
 * index when it fits in LDS (a 2-bit state per /16 block plus the sorted
 * 16-bit offsets of the boundaries of the union of all prefixes inside the
 * /16 blocks that such a boundary cuts); label-only queries are answered from
 * it, the kind's search serves institution ids and positions.  kind may be
 * OR-ed with SINET_TABLE_NO_INOUT_INDEX.  base: IPv4
 * address, host bits allowed (they are masked off as Algorithm 1 masks the
 * CIDR base); len: prefix length Z in 0..32; inst: institution id of the row
 * (any value except SINET_NO_INST), or NULL for the row index.  The longest
 * matching prefix gives the institution, equal lengths resolve to the lowest
 * row.  Learned kinds need sinet_table_train before use.  Errors:
 * INVALID_ARG (null pointer, len > 32, n_prefix == 0 or above
 * SINET_MAX_PREFIXES, inst == SINET_NO_INST, SCAN above 1024 rows),
 * OUT_OF_MEMORY.  Synchronous. */
sinet_status sinet_table_create(const uint32_t* base, const uint8_t* len, const uint32_t* inst,
                                uint64_t n_prefix, sinet_lookup kind, hipStream_t stream,
                                sinet_table** out);

/* Fit the learned model of a LEARNED_PLA / LEARNED_MLP table on the GPU and
 * measure its maximum position error over every interval.  params may be
 * NULL (defaults); report may be NULL.  PLA with segments == 0: error-bounded
 * segmentation on the host; with target_err == 0 it first aims at a measured
 * bound of at most 6 (the window search, see pla_window) if those segments
 * fit in LDS, else at 8, doubled until the segments fit.  Synchronous. */
sinet_status sinet_table_train(sinet_table* t, const sinet_train_params* params,
                               hipStream_t stream, sinet_train_report* report);

/* The table's shape and its learned model's state (Algorithm 1's CIDR list
 * as built by sinet_table_create: prefixes, interval boundaries m, device
 * bytes, lookup kind and in/out index; for learned kinds the measured bound
 * max_err, the PLA segments, whether the one-window search is used, and the
 * number of fallbacks to the full search so far).  Errors: INVALID_ARG (t or
 * out NULL), DEVICE (the fallback counter's read).  Synchronous: a blocking
 * copy of the counter from the device. */
sinet_status sinet_table_info(const sinet_table* t, sinet_table_info_t* out);

/* Save the learned model of a trained table to HOST arrays: MLP: params[49];
 * PLA: knot[S], c[S], g[S] with S = info.segments <= cap.  Unused pointers
 * may be NULL.  *max_err receives the search bound.  Synchronous. */
sinet_status sinet_table_get_model(const sinet_table* t, float* params, uint32_t* knot, float* c,
                                   float* g, uint32_t cap, uint32_t* max_err);

/* Load a learned model (HOST arrays, copied), e.g. one saved by
 * sinet_table_get_model: MLP: params[49]; PLA: segments rows of knot
 * (ascending, knot[0] == 0), c and g (g >= 0).  max_err == 0xFFFFFFFF
 * measures the bound on the GPU; any other value is used as given, and a
 * bound that is too small only costs fallbacks (results stay exact).
 * Synchronous. */
sinet_status sinet_table_set_model(sinet_table* t, const float* params, const uint32_t* knot,
                                   const float* c, const float* g, uint32_t segments,
                                   uint32_t max_err);

/* Copy the table's interval boundaries and owners (LPM row + 1, 0 = no
 * prefix) to HOST arrays of capacity cap (>= m).  Synchronous. */
sinet_status sinet_table_intervals(const sinet_table* t, uint32_t* B, uint32_t* owner,
                                   uint64_t cap);

sinet_status sinet_table_destroy(sinet_table* t);

/* Interval index j (B[j] <= a < B[j+1]) of n addresses, by the table's own
 * lookup method (device in, device out). */
sinet_status sinet_table_position(const sinet_table* t, const uint32_t* addr, uint64_t n,
                                  uint32_t* pos, hipStream_t stream);

/* Discrimination (Algorithm 1 over the whole table, both endpoints):
 * label[i] = in(src[i]) | in(dst[i]) << 1; src_inst/dst_inst[i] = institution
 * of the longest matching prefix or SINET_NO_INST.  label, src_inst and
 * dst_inst may each be NULL (not stored). */
sinet_status sinet_discriminate(const sinet_table* t, const uint32_t* src, const uint32_t* dst,
                                uint64_t n, uint8_t* label, uint32_t* src_inst,
                                uint32_t* dst_inst, hipStream_t stream);

/* Label runs (section "Coordinated Batch Processing" and Fig. 3: the chunks
 * are discriminated before the Map stage, so the later stages can take the
 * sessions of one direction together): the stable partition of the session
 * indices by label.  label: device u8[n] (its low two bits are the label, as
 * sinet_discriminate writes them); idx: device u32[n], receives first every i
 * with label 0 in increasing order, then label 1, 2, 3; totals: device u64[4],
 * the number of sessions with each label (the run of label L starts at
 * totals[0] + ... + totals[L-1]).  Each wave ranks its sessions within their
 * label with a ballot per label and session slot and mbcnt, and takes its
 * class totals from popcounts; a count pass, a scan over the workgroups'
 * totals and a scatter pass place every index.  Caller-owned buffers; a workspace of 32 bytes per
 * 65,536 sessions comes from the stream-ordered pool.  Errors: INVALID_ARG
 * (totals NULL; label or idx NULL with n > 0), UNSUPPORTED (n >= 2^32: the
 * indices are 32-bit), OUT_OF_MEMORY.  n == 0 zeroes totals.  Asynchronous on
 * stream. */
sinet_status sinet_label_runs(const uint8_t* label, uint64_t n, uint32_t* idx, uint64_t* totals,
                              hipStream_t stream);

/* Histogram of already labelled sessions: the sections "Map" (each session
 * becomes the key (label, bin) with bin = (ts - t0) / width and the values
 * (1, bytes)) and "Reduce" (values of equal keys added), with one exact
 * counter per bin and label as in "Merge Scatter Pattern with CPU" (every
 * 1-ms bin of the day).  Sessions before t0 or past the last bin are added to
 * out->dropped.  accumulate == 0: outputs are cleared first; 1: added to (the
 * merge of per-chunk results by addition of "Pairwise Reduction Pattern with
 * GPU").  Columns, label and outputs are device memory of the caller.
 * Errors: INVALID_ARG for null pointers, width_ms == 0, n_bins == 0.
 * Asynchronous on stream. */
sinet_status sinet_histogram(const uint32_t* ts, const uint64_t* bytes, const uint8_t* label,
                             uint64_t n, const sinet_window* win, sinet_hist* out,
                             int accumulate, hipStream_t stream);

/* Discrimination (Algorithm 1, section "Threads for traffic direction
 * discrimination with CIDR MATCH") fused with the histogram of
 * sinet_histogram (sections "Map", "Reduce", "Merge Scatter Pattern with
 * CPU") over one chunk of sessions: the paper's session pipeline of Fig. 2.
 * label may be NULL (not stored); the other arguments and errors are those
 * of sinet_discriminate and sinet_histogram.  The reduce is chosen by
 * sinet_set_reduce.  Asynchronous on stream. */
sinet_status sinet_pipeline(const sinet_table* t, const sinet_columns* cols,
                            const sinet_window* win, uint8_t* label, sinet_hist* out,
                            int accumulate, hipStream_t stream);

/* Watch-list histograms (sections "AbuseIPDB" and "GRIZZLY STEPPE",
 * Figures 8-11: the sessions of the hosts on a published list per time
 * window, ingoing and outgoing).  list is a prefix table of the listed hosts
 * (usually /32 rows) whose inst ids are the keys: one key per host (the row
 * index, inst == NULL at creation) or one per list.  Each session looks up
 * its source and its destination in the list; the longest match, lowest row
 * on equal length, gives the key.  A matched source adds (1, bytes) to
 * count/bytes[SINET_WATCH_SRC][key][bin], a matched destination to
 * [SINET_WATCH_DST][key][bin], with bin = floor((ts - t0_ms) / width_ms);
 * a session whose two ends match counts once in each direction; matched
 * sessions outside the window go to dropped[dir].  accumulate == 0: outputs
 * cleared first; 1: added to.  Every inst id of list must be below n_keys.
 * The list's kind may be SCAN, BSEARCH, TRIE or a trained learned kind.
 * Errors: INVALID_ARG (NULL table, column or output, width_ms == 0,
 * n_bins == 0, n_keys == 0, an inst id >= n_keys, 2 * n_keys * n_bins
 * above 2^40), UNSUPPORTED (table too large for LDS).  Asynchronous. */
sinet_status sinet_watch_histogram(const sinet_table* list, const sinet_columns* cols,
                                   const sinet_window* win, uint32_t n_keys,
                                   sinet_watch_hist* out, int accumulate, hipStream_t stream);

/* Forward and backward of the 1-16-1 MLP position model (device arrays):
 * params[49] (w1[16], b1[16], w2[16], b2), inputs x[n], targets y[n];
 * writes loss[1] = mean (f(x) - y)^2 and grad[49].  Float32, fixed-order
 * reduction. */
sinet_status sinet_mlp_loss_grad(const float* params, const float* x, const float* y,
                                 uint64_t n, float* loss, float* grad, hipStream_t stream);

/* Pick block/chunk/grid for a batch by timing candidates (results are
 * identical for every candidate).  cache_path may be NULL; otherwise a JSON
 * file read first and written after tuning.  Synchronous. */
sinet_status sinet_autotune(const sinet_stream* streams, uint32_t n_streams,
                            const char* cache_path, hipStream_t stream, sinet_tune* out);

/* Prepare a batch (sections "Coordinated Batch Processing", "Work Queue"):
 * stream descriptors uploaded, and the clears, one persistent work-queue
 * launch per lookup kind, the shared segment index, the block reduction and
 * the far pass captured in one hipGraph.  Streams whose lookups walk device
 * memory (trie, learned, sampled binary search; see sinet_table_create) get a
 * batched lookup pass that stores their labels first, into the stream's label
 * output or, when it has none, a buffer of n bytes held by the plan.  tune may
 * be NULL (defaults).  The plan refers to the caller's buffers and tables,
 * which must outlive it.  Errors: INVALID_ARG (no streams, NULL column or
 * histogram, untrained learned table, bad window), UNSUPPORTED (more than
 * 2^32 record slots in one plan), OUT_OF_MEMORY.  Synchronous. */
sinet_status sinet_batch_plan_create(const sinet_stream* streams, uint32_t n_streams,
                                     const sinet_tune* tune, hipStream_t stream,
                                     sinet_batch_plan** out);

/* Run a prepared batch (one graph launch): every stream's labels and
 * histogram, cleared first, as if by sinet_pipeline per stream. */
sinet_status sinet_batch_run(sinet_batch_plan* plan, hipStream_t stream);

sinet_status sinet_batch_plan_destroy(sinet_batch_plan* plan);

/* Session text to columns (section "Dataset Description", Table 1: the
 * PA-7080 session record, 24 fields).  text (device, len bytes) holds one
 * record per line, Table 1's fields in order separated by ','; every
 * '\n'-ended segment is a line (an empty one too), and a last segment without
 * '\n' is a line when it is not empty.  Line i fills session i of out
 * (device columns; out->n is their capacity):
 *   ts    field 1, capture_time "YYYY/MM/DD HH:MM:SS.mmm" (proleptic
 *         Gregorian), as milliseconds since midnight of day origin_days
 *         (days since 1970-01-01), which must lie in [0, 2^32 - 1);
 *   src   field 5, dst field 8: dotted quads of 1-3 digit octets <= 255;
 *   bytes field 21: 1-20 decimal digits, at most 2^64 - 1.
 * A line with fewer than 21 fields or a malformed one of these fields gives
 * ts = 0xFFFFFFFF (no valid line has it; outside any window ending before
 * 2^32 - 1 ms), src = dst = bytes = 0, and counts
 * in *n_bad.  *n_lines receives the number of lines.  The kernels read whole
 * aligned 16-byte groups of text and stay inside [text, text + len).
 * Errors: INVALID_ARG (NULL pointer, more lines than out->n: *n_lines then
 * holds the number needed), UNSUPPORTED (text of 2^47 bytes or more),
 * OUT_OF_MEMORY (the line index, 8 bytes per line).  Synchronous. */
sinet_status sinet_parse_sessions(const uint8_t* text, uint64_t len, int32_t origin_days,
                                  sinet_columns* out, uint64_t* n_lines, uint64_t* n_bad,
                                  hipStream_t stream);

/* Coarser time frames (section "All Sessions of SINET", Figures 6-7: the
 * sessions grouped into one-hour frames, here from the millisecond bins).
 * in: [rows][n_bins] and out: [rows][ceil(n_bins / factor)] unsigned 64-bit
 * device arrays, row-major; out[r][k] = sum of in[r][b] over b = k * factor
 * .. min((k + 1) * factor, n_bins) - 1, modulo 2^64 (the last frame may be
 * shorter).  out is overwritten.  rows is 4 for a label histogram, 2 * n_keys
 * for a watch-list histogram; count and byte arrays are separate calls.
 * Errors: INVALID_ARG (NULL pointer, rows, n_bins or factor 0).
 * Asynchronous. */
sinet_status sinet_rebin(const uint64_t* in, uint32_t rows, uint32_t n_bins, uint32_t factor,
                         uint64_t* out, hipStream_t stream);

/* Out-of-core pipeline (the paper merges per-chunk
 * results by addition, section "Pairwise Reduction Pattern with GPU", and its
 * Table 3 runs out of device memory on large inputs).  A streamer owns two
 * staging slots, each with device buffers and pinned host buffers for
 * chunk_sessions sessions (about 42 bytes per session per slot), and its own
 * copy stream (default priority, non-blocking).  Errors: INVALID_ARG (chunk_sessions 0 or
 * above 2^31), OUT_OF_MEMORY.  Synchronous. */
typedef struct sinet_streamer sinet_streamer;
sinet_status sinet_streamer_create(uint64_t chunk_sessions, sinet_streamer** out);

/* sinet_pipeline over columns held in HOST memory (pageable or pinned; n may
 * exceed device memory): chunk k + 1 is copied to the device on the
 * streamer's copy stream while chunk k is classified and binned on stream;
 * pageable columns pass through the pinned staging (host threads copy them
 * in), pinned ones are copied from directly.  The histogram (device, as in
 * sinet_pipeline) is cleared first unless accumulate and summed over the
 * chunks; host_label (HOST, n bytes) receives the labels, or NULL.  Results
 * equal one sinet_pipeline call over the same sessions resident on the
 * device.  The streamer must have been created on the current device.
 * Synchronous: returns when every chunk is binned and every label is back. */
sinet_status sinet_streamer_pipeline(sinet_streamer* s, const sinet_table* t,
                                     const sinet_columns* host_cols, const sinet_window* win,
                                     uint8_t* host_label, sinet_hist* out, int accumulate,
                                     hipStream_t stream);

sinet_status sinet_streamer_destroy(sinet_streamer* s);

/* sinet_pipeline without allocating: for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same arguments, results and errors as
 * sinet_pipeline, but its workspace (the sliding-window reduce's piece
 * bounds, spill rows, far bitmap and event list, and the labels when `label`
 * is NULL) is carved from a static 128 MiB device array of the library,
 * which every GPU the library runs on holds until the process ends.  It
 * calls no allocator: no hipMalloc, no pool, no timing events (phase timing
 * does not see it).  Limits: at most 2^25 sessions per call (larger inputs:
 * call it on chunks with accumulate = 1); INVALID_ARG beyond that, checked
 * before anything is enqueued.  Every call on one GPU uses the same array,
 * so calls that overlap on one GPU (different host threads or streams
 * running at the same time) race and must be serialised by the caller. */
sinet_status sinet_pipeline_noalloc(const sinet_table* t, const sinet_columns* cols,
                                    const sinet_window* win, uint8_t* label, sinet_hist* out,
                                    int accumulate, hipStream_t stream);

/* Device time of the phases of sinet_histogram / sinet_pipeline, summed over
 * the calls made since timing was last enabled.  Each phase is bracketed by
 * a pair of HIP events recorded on the call's own stream (none while the
 * stream is being captured into a graph), so a phase's figure is the device
 * time of its kernels on that stream.  Phases of the two reduces:
 *                 records reduce                 sliding-window reduce
 *   lookup_ms     lookup pass storing labels     lookup pass storing labels
 *                 (global-memory searches only)  (every lookup kind)
 *   stage1_ms     k_stage1: classify, bin,       k_window: bin, window in LDS,
 *                 partition into records         one write of every bin
 *   index_ms      segment scan, directory fill   k_window_bounds: pieces' bins
 *   stage2_ms     k_stage2: block reduction      k_window_fixup: boundary spills
 *   far_ms        far pass (global atomics)      k_window_far (global atomics)
 * For n_bins <= 2048 stage1_ms is the single private-histogram pass. */
typedef struct {
    double lookup_ms;
    double stage1_ms;
    double index_ms;
    double stage2_ms;
    double far_ms;
    uint64_t calls;     /* timed sinet_histogram / sinet_pipeline calls */
    uint64_t stage1_launches;  /* stage-1 (or private-pass, or window) launches among them */
    uint64_t window_calls;     /* calls (pieces of calls) reduced by the sliding window */
} sinet_timing;

/* on != 0: start timing every later sinet_histogram / sinet_pipeline call of
 * this process (clears earlier figures); on == 0: stop.  Timing costs two
 * event records per phase.  Not thread-safe against concurrent calls of
 * sinet_timing_read. */
sinet_status sinet_timing_enable(int on);

/* Wait for the recorded events and return the sums since the last enable.
 * Errors: INVALID_ARG (out NULL), HIP (event failure). */
sinet_status sinet_timing_read(sinet_timing* out);

/* Reduce used by sinet_histogram / sinet_pipeline (and the streamer) when
 * the histogram has more than 2048 bins (smaller ones are always reduced in
 * LDS per workgroup).  Both reduces give bit-identical results for any
 * input; they differ in speed and workspace:
 *   RECORDS  the two-stage map-reduce of the sections "Two-stage Map-Reduce
 *            with tiling pattern" and "Reduce": stage 1 writes one 4-byte
 *            record per session grouped by 1024-bin block, stage 2 reduces
 *            each block in LDS and writes its bins (about 6 bytes of
 *            workspace per session);
 *   WINDOW   the same Map and Reduce in one pass over labelled sessions: a
 *            workgroup walks a contiguous range of nearly time-sorted
 *            sessions with the bins it touches in LDS and writes every bin
 *            once (labels are stored by a lookup pass first; about 1 byte
 *            of workspace per session plus 330 MB);
 *   AUTO     WINDOW from 2^28 sessions on, else RECORDS (the default; the
 *            measured crossover of the two on a day of 1-ms bins).
 * Process-wide; takes effect for calls made after it returns.
 * Errors: INVALID_ARG (unknown mode). */
typedef enum {
    SINET_REDUCE_AUTO = 0,
    SINET_REDUCE_RECORDS = 1,
    SINET_REDUCE_WINDOW = 2
} sinet_reduce;
sinet_status sinet_set_reduce(sinet_reduce mode);

#ifdef __cplusplus
}
#endif

#endif /* SINET_H */
