/*
 * rtcdf.h -- C ABI of the Range-Tiled CDF sort (RT-CDF) library for AMD
 * Instinct MI355X (gfx950).
 *
 * RT-CDF is the method of "Shared-Memory Range-Tiled CDF Sort for Small-Range
 * Integer Keys on GPUs" (Sec. 3): an unstable sort of n integer keys known to
 * lie in [minVal, maxVal).  The value range R = maxVal - minVal is split into
 * range tiles of width T; each tile's histogram is built in on-chip memory
 * (Alg. 5), prefix-summed into a local CDF (Alg. 4), offset by the prefix of
 * tile totals (Alg. 6), and every value is written across its output interval
 * (Alg. 7, Lemma 3) without reading the input again.
 *
 * General conventions (apply to every entry point below):
 *  - Pointers named d_* and the key arrays are DEVICE pointers on the current
 *    HIP device; everything else is host memory.  The caller owns all of
 *    them; the library never frees or retains a caller pointer beyond the
 *    call.
 *  - Calls are asynchronous on `stream` (0 = the null stream).  Argument
 *    errors are detected on the host and returned before any GPU work is
 *    enqueued.  HIP launch errors return RTCDF_ERROR_HIP and the HIP code is
 *    available from rtcdf_last_hip_error().  Errors that happen on the GPU
 *    later surface through the usual HIP synchronisation calls.
 *  - The range is half-open: maxVal is exclusive (Sec. 2.1).  minVal and
 *    maxVal are int64 so that maxVal = 2^31 is expressible;
 *    INT32_MIN <= minVal < maxVal <= 2^31 is required.
 *  - Keys must lie in [minVal, maxVal) (a precondition, Sec. 2.1).  A key
 *    outside the range makes the output unspecified (never an out-of-bounds
 *    access by the library).
 *  - The output holds the original key values in nondecreasing order.  The
 *    sort is unstable and carries no payload; since keys are bare integers
 *    the output is unique.
 *  - keys_out may equal keys_in (in place): the output stage never reads the
 *    input.  Partial overlap is rejected.
 *  - Keys need only 4-byte alignment; the kernels peel unaligned heads/tails.
 *  - n <= 2^40.  Below 2^32 every count and output position of the sort is
 *    32-bit, as in the paper's kernels (Sec. 3.2 workspace analysis).  From
 *    n = 2^32 on (not in the paper) the sorts of rtcdf_sort,
 *    rtcdf_sort_with_config, rtcdf_sort_keys, rtcdf_sort_checked and
 *    rtcdf_sort_ws keep the per-value counts in 64 bits: the input is counted
 *    in pieces of 2^31 keys, and the output is written in windows of 2^31
 *    positions by the same local-CDF and output stages, each window from the
 *    counts of its own positions.  The configuration is then the caller's or
 *    the static choice for a 2^31-key piece (no learned pick, no
 *    prefix-maximum output), and the workspace adds 8 bytes per value of the
 *    range.  rtcdf_plan_info and rtcdf_debug_intermediates describe one plain
 *    plan and take n < 2^32 only.
 *  - Functions are thread-safe with respect to different devices; concurrent
 *    calls on one device that use the library's internal workspace are
 *    serialised internally by a mutex but their GPU work is only ordered if
 *    they share a stream.  Use rtcdf_sort_ws with separate workspaces for
 *    concurrent streams.
 */
#ifndef RTCDF_H
#define RTCDF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rtcdf_status {
  RTCDF_SUCCESS = 0,
  RTCDF_ERROR_INVALID_VALUE = 1,    /* NULL with n > 0, maxVal <= minVal, range outside int32, bad config */
  RTCDF_ERROR_SIZE_TOO_LARGE = 2,   /* n > 2^40; n >= 2^32 for the plan-info / intermediates calls */
  RTCDF_ERROR_RANGE_TOO_LARGE = 3,  /* R > RTCDF_MAX_RANGE */
  RTCDF_ERROR_OVERLAP = 4,          /* keys_in and keys_out overlap without being equal */
  RTCDF_ERROR_OUT_OF_MEMORY = 5,    /* device workspace allocation failed */
  RTCDF_ERROR_HIP = 6,              /* a HIP call failed; see rtcdf_last_hip_error() */
  RTCDF_ERROR_WORKSPACE_TOO_SMALL = 7,
  RTCDF_ERROR_NOT_SUPPORTED = 8,    /* device is not gfx950, or feature unavailable */
  RTCDF_ERROR_NO_MODEL = 9,         /* learned mode requested but no model is loaded */
  RTCDF_ERROR_KEY_OUT_OF_RANGE = 10, /* checked mode only: some key lies outside [minVal, maxVal) */
  RTCDF_ERROR_CAPTURE_NEEDS_WORKSPACE = 11 /* rtcdf_sort under stream capture would have to
                                             allocate its workspace (see rtcdf_sort) */
} rtcdf_status_t;

/* Largest supported range.  The workspace grows with R (about 4R + 4m bytes
 * for the histogram/local CDFs and tile offsets, Sec. 3.2), and the
 * histogram stage rescans the input once per LDS pass. */
#define RTCDF_MAX_RANGE (1u << 28)

/* Kernel configuration (the tuning knobs of the method, Sec. 3.3):
 *  tile_width        T, the range-tile width of the local CDFs (Sec. 3).  A
 *                    multiple of 128 in [128, 32768].  The histogram stage
 *                    keeps as many whole tiles per LDS pass as fit.
 *  items_per_thread  keys handled per thread per loop iteration in the
 *                    histogram and output stages: 4, 8 or 16.
 *  blocks_per_tile   co-resident workgroups per compute unit working on a
 *                    range tile: 1, 2 or 4.  Each gets 160 KiB / blocks of
 *                    LDS, so T * 4 * blocks_per_tile <= 160 KiB is required.
 *  flags             an OR of the RTCDF_FLAG_* options below (0: none).
 * Options (none changes the output; each changes how it is computed):
 *  RTCDF_FLAG_OUTPUT_PREFIX_MAX  write the output by the prefix-maximum
 *                    method of Alg. 3 (Sec. 2.2: B = 0, each value stored at
 *                    the first position of its output interval, then the
 *                    running maximum of B) instead of the search of the local
 *                    CDFs of Alg. 7.  It writes B twice and reads it once
 *                    (12 B per key in the output stage instead of 4) but
 *                    writes the steps one value per thread.  The library's
 *                    own choice (every config mode) sets it when R >= 2^14
 *                    and R >= n.
 *  RTCDF_FLAG_COUNTERS_16 / RTCDF_FLAG_COUNTERS_32 / RTCDF_FLAG_COUNTERS_4
 *                    the width of the histogram's LDS counters (Alg. 5): two
 *                    16-bit counters per 32-bit word, one 32-bit counter, or
 *                    eight 4-bit counters, instead of the library's choice
 *                    (32 bits where that needs no more LDS passes than four
 *                    8-bit counters per word, else 8 bits).  At most one of
 *                    the three.  Narrower counters fit more bins per pass
 *                    (4-bit: 2^18 bins in one pass over the keys) but wrap
 *                    (repaired exactly); heavily repeated keys wrap 8-bit
 *                    counters every 256 hits and 4-bit ones every 16, so
 *                    4-bit counters pay only for spread-out keys.  Int32 keys
 *                    only (ignored by rtcdf_sort_keys for narrower keys).
 *  RTCDF_FLAG_WAVE_DEDUPE  before its LDS atomics a wave matches one
 *                    candidate value (its hot value, else its first lane's
 *                    key) against all its keys with ballots and adds the
 *                    copies of a frequent value once: skewed keys no longer
 *                    serialise on one LDS address.
 *  RTCDF_FLAG_CHUNK_4096  4096 output positions per output chunk instead
 *                    of 2048 (fewer chunk boundaries; sparse windows of more
 *                    than 4096 values take the slower global search).
 * A zeroed config (all fields 0) means "let the library choose" (the mode
 * set by rtcdf_set_config_mode).  A config with tile_width, items_per_thread
 * and blocks_per_tile 0 and some flags means the static default table's
 * (tile_width, items_per_thread, blocks_per_tile) for the problem with those
 * flags (the extra points of the tuning grid are such configs). */
#define RTCDF_FLAG_OUTPUT_PREFIX_MAX 0x01u
#define RTCDF_FLAG_COUNTERS_16 0x04u
#define RTCDF_FLAG_COUNTERS_32 0x08u
#define RTCDF_FLAG_COUNTERS_4 0x40u
#define RTCDF_FLAG_COUNTERS_MASK 0x4cu
#define RTCDF_FLAG_WAVE_DEDUPE 0x10u
#define RTCDF_FLAG_CHUNK_4096 0x20u
typedef struct rtcdf_config {
  uint32_t tile_width;
  uint32_t items_per_thread;
  uint32_t blocks_per_tile;
  uint32_t flags;
} rtcdf_config_t;

/* ---- Plain sort ------------------------------------------------------ */

/* Sort n int32 keys from [minVal, maxVal) into keys_out (Sec. 3, Alg. 4).
 * keys_in, keys_out: device arrays of n int32 (may be equal).
 * Uses a workspace cached by the library per (device, stream), allocated on
 * first use and grown as needed: hipMalloc and hipFree (after waiting for
 * `stream`) may run inside this call.
 * The configuration comes from the current config mode.
 * HIP graph capture: rtcdf_sort_ws and rtcdf_sort_batched are the capturable
 * forms.  rtcdf_sort may be captured only when a sort of a problem at least as
 * large (same stream, same plan kind) has run on `stream` before the capture
 * began; otherwise it returns RTCDF_ERROR_CAPTURE_NEEDS_WORKSPACE without
 * enqueuing anything.  Under capture the learned mode's pick (which reads its
 * result back to the host) is skipped and the TUNED/DEFAULT configuration is
 * used.  A workspace that a capture has used is never freed
 * (rtcdf_release_workspaces keeps it; growth retires it), because the graph
 * may be replayed at any time. */
rtcdf_status_t rtcdf_sort(const int32_t* keys_in, int32_t* keys_out, size_t n,
                          int64_t minVal, int64_t maxVal, hipStream_t stream);

/* As rtcdf_sort with an explicit configuration (cfg must be valid, see
 * rtcdf_config_t; NULL or all-zero = library choice).  Every valid config
 * gives a byte-identical output. */
rtcdf_status_t rtcdf_sort_with_config(const int32_t* keys_in, int32_t* keys_out, size_t n,
                                      int64_t minVal, int64_t maxVal,
                                      const rtcdf_config_t* cfg, hipStream_t stream);

/* Keys of other widths.  The sort of 16- and 8-bit keys, signed or not: the
 * histogram reads 16-byte vectors of 8 or 16 keys and widens them, the output
 * stage writes the keys in their own width.  int64 keys: any window
 * [minVal, maxVal) of int64 values with R = maxVal - minVal <=
 * RTCDF_MAX_RANGE (maxVal <= INT64_MAX, so INT64_MAX itself is not a
 * sortable key); every key is normalised to key - minVal in 64-bit
 * arithmetic (counts as for int32 keys, 64-bit from n = 2^32), and the output stage writes
 * minVal + value as 8-byte keys.  key_type is one of rtcdf_key_type_t;
 * keys_in / keys_out are device arrays of n keys of that type, aligned to its
 * size (they may be equal; partial overlap is RTCDF_ERROR_OVERLAP);
 * [minVal, maxVal) must lie within the type's values.
 * cfg as for rtcdf_sort_with_config (NULL = library choice, flags must be 0:
 * the prefix-maximum output is offered for int32 keys only).  RTCDF_KEY_INT32
 * is rtcdf_sort_with_config.  Asynchronous on `stream`; argument errors are
 * returned before any GPU work.  Not in the paper (its keys are 32-bit). */
typedef enum rtcdf_key_type {
  RTCDF_KEY_INT32 = 0,
  RTCDF_KEY_INT16 = 1,
  RTCDF_KEY_UINT16 = 2,
  RTCDF_KEY_INT8 = 3,
  RTCDF_KEY_UINT8 = 4,
  RTCDF_KEY_INT64 = 5
} rtcdf_key_type_t;

rtcdf_status_t rtcdf_sort_keys(const void* keys_in, void* keys_out, size_t n, int key_type,
                               int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                               hipStream_t stream);

/* Checked mode.  The keys lying in [minVal, maxVal) is a precondition of the
 * method (Sec. 2.1) that the sort itself does not test.  These two calls test
 * it, at the price of one more read of the keys (4 B per key):
 *
 * rtcdf_count_out_of_range: writes to *d_count (a device uint64, 8-byte
 * aligned) the number of keys[i], i < n, outside [minVal, maxVal).
 * Asynchronous on `stream`; argument errors as for rtcdf_sort (keys_out is
 * not involved).
 *
 * rtcdf_sort_checked: as rtcdf_sort_with_config (cfg NULL = library choice),
 * but first counts the out-of-range keys and waits for the count (a host
 * synchronisation with `stream`).  If any key is out of range it returns
 * RTCDF_ERROR_KEY_OUT_OF_RANGE and enqueues nothing more (keys_out is left
 * unchanged); otherwise it enqueues the sort and returns without waiting. */
rtcdf_status_t rtcdf_count_out_of_range(const int32_t* keys, size_t n, int64_t minVal, int64_t maxVal,
                                        uint64_t* d_count, hipStream_t stream);
rtcdf_status_t rtcdf_sort_checked(const int32_t* keys_in, int32_t* keys_out, size_t n,
                                  int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                                  hipStream_t stream);

/* Bytes of device workspace rtcdf_sort_ws needs for this problem and
 * configuration (cfg NULL = library choice), written to *bytes.  The
 * requirement depends on n, R, the config and the alignment of keys_out
 * modulo 16 bytes, which is why keys_out is asked for (it is not read).
 * Ranges that need many LDS passes (R above about 1.4 x 10^6, reported by
 * rtcdf_plan_info as partition_buckets > 0) add a copy of the keys,
 * 4 (n + 4 passes + 4) bytes: the keys are first grouped by pass so that each
 * pass reads its own group only. */
rtcdf_status_t rtcdf_workspace_bytes(size_t n, int64_t minVal, int64_t maxVal,
                                     const rtcdf_config_t* cfg, const int32_t* keys_out,
                                     size_t* bytes);

/* As rtcdf_sort_with_config with a caller-owned workspace: d_ws is a device
 * buffer of ws_bytes >= rtcdf_workspace_bytes(...) bytes, 256-byte aligned.
 * Performs no allocation and no host synchronisation, so it may be captured
 * into a HIP graph.  The workspace contents need no initialisation and are
 * scratch after the call; the buffer must not be used concurrently by
 * another call. */
rtcdf_status_t rtcdf_sort_ws(const int32_t* keys_in, int32_t* keys_out, size_t n,
                             int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                             void* d_ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sort of
 * rtcdf_sort_ws with its workspace in a fixed device array of the library,
 * RTCDF_NOALLOC_MAX_WORKSPACE bytes, that each GPU the library runs on holds
 * from the first call on it until the process ends.  Arguments, output and
 * configuration as for rtcdf_sort_ws (cfg NULL = library choice; the learned
 * pick is not consulted).  No hipMalloc, hipFree or other allocation, no host
 * synchronisation.  A problem whose workspace (rtcdf_workspace_bytes) exceeds
 * the array returns RTCDF_ERROR_WORKSPACE_TOO_SMALL before any GPU work (for
 * example n = 10^8 fits up to R = 2^20; ranges that partition the keys by pass
 * need a copy of the keys and fit only for small n).  Every call on one GPU
 * uses that GPU's one array, which keeps the previous call's contents (the
 * sort needs no initialised workspace): calls that may overlap in time on one
 * GPU (unordered streams, or several host threads) race and must be
 * serialised by the caller, e.g. by issuing them on one stream. */
#define RTCDF_NOALLOC_MAX_WORKSPACE (64u << 20)
rtcdf_status_t rtcdf_sort_noalloc(const int32_t* keys_in, int32_t* keys_out, size_t n,
                                  int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                                  hipStream_t stream);

/* Test hook for the intermediate arrays of Alg. 4-6 for tile width
 * cfg->tile_width: d_hist[R] receives the tile histograms (Alg. 5), d_cdf[R]
 * the local CDFs (in-place inclusive scan per tile), d_offsets[m] the tile
 * offsets O (Alg. 6), m = ceil(R / T).  All uint32 device arrays; any may
 * be NULL.  Uses the same kernels as rtcdf_sort_with_config. */
rtcdf_status_t rtcdf_debug_intermediates(const int32_t* keys_in, size_t n, int64_t minVal,
                                         int64_t maxVal, const rtcdf_config_t* cfg,
                                         uint32_t* d_hist, uint32_t* d_cdf,
                                         uint32_t* d_offsets, hipStream_t stream);

/* ---- Batched sort ---------------------------------------------------- */

/* One independent array of a batch (device-resident, 32 bytes): n int32 keys
 * at keys_in from [minVal, minVal + range), sorted into keys_out.  keys_out
 * may equal keys_in (in place) but must not overlap any other segment's
 * output.  1 <= range <= RTCDF_BATCH_MAX_RANGE.  config: the segment's
 * keys per thread per load step of its histogram (the items_per_thread knob
 * of rtcdf_config_t): 4, 8 or 16; 0 (or any other value) means 16.  It
 * changes the speed of the segment's sort, never its output.
 * A descriptor with n = 0, range = 0, range > RTCDF_BATCH_MAX_RANGE (or above
 * the bounds' max_range) or a NULL pointer is skipped and its output left
 * untouched. */
typedef struct rtcdf_segment {
  const int32_t* keys_in;
  int32_t* keys_out;
  uint32_t n;
  int32_t minVal;
  uint32_t range;
  uint32_t config;
} rtcdf_segment_t;

/* Host-side bounds of a batch, used to size the launch and the workspace:
 * total_keys = sum of n, max_n and max_range the largest n and range of any
 * segment.  max_range <= RTCDF_BATCH_MAX_RANGE. */
typedef struct rtcdf_batch_bounds {
  uint64_t total_keys;
  uint32_t max_n;
  uint32_t max_range;
} rtcdf_batch_bounds_t;

#define RTCDF_BATCH_MAX_RANGE (1u << 16)

/* Workspace bytes rtcdf_sort_batched needs for num_segments segments within
 * *bounds, written to *bytes. */
rtcdf_status_t rtcdf_batched_workspace_bytes(uint32_t num_segments,
                                             const rtcdf_batch_bounds_t* bounds, size_t* bytes);

/* Sort every segment of d_segments[num_segments] (a device array) in one
 * persistent launch (Alg. 4 of the paper per range tile of 32768 values: a
 * segment is one or two work items, each handled by one workgroup in LDS,
 * largest first; an in-place segment wider than 32768 values is one item
 * that counts both tiles before it writes any position), preceded by a
 * one-workgroup ordering kernel.  Each
 * segment's output equals rtcdf_sort of that segment.
 * d_ws: caller-owned device workspace of ws_bytes bytes (>=
 * rtcdf_batched_workspace_bytes), 256-byte aligned, no initialisation
 * needed, not shared with a concurrent call.  No allocation and no host
 * synchronisation: capturable into a HIP graph and replayable. */
rtcdf_status_t rtcdf_sort_batched(const rtcdf_segment_t* d_segments, uint32_t num_segments,
                                  const rtcdf_batch_bounds_t* bounds, void* d_ws,
                                  size_t ws_bytes, hipStream_t stream);

/* ---- Configuration source --------------------------------------------- */

typedef enum rtcdf_config_mode {
  RTCDF_CONFIG_DEFAULT = 0,   /* static per-R table (selected by the geometric-mean method of Sec. 4.1) */
  RTCDF_CONFIG_TUNED = 1,     /* nearest entry of a loaded tuning database, else DEFAULT */
  RTCDF_CONFIG_LEARNED = 2    /* the loaded MLP picker (see rtcdf_load_model), else TUNED/DEFAULT */
} rtcdf_config_mode_t;

rtcdf_status_t rtcdf_set_config_mode(int mode);
int rtcdf_get_config_mode(void);

/* The tuning grid, RTCDF_GRID_SIZE points.  Points 0-53: tile width T in
 * {2^10 .. 2^15} x items per thread in {4, 8, 16} x blocks per tile in
 * {1, 2, 4}, flags 0; index i = 9 * log2(T / 1024) + 3 * log2(items / 4) +
 * log2(blocks).  Points with T * 4 * blocks > 160 KiB are invalid (45 of the
 * 54).  Points 54-61, the option points: (0, 0, 0, flags), i.e. the static
 * table's (T, items, blocks) for the problem with the flags
 * PREFIX_MAX, COUNTERS_16, COUNTERS_16 | WAVE_DEDUPE, WAVE_DEDUPE,
 * CHUNK_4096, COUNTERS_16 | CHUNK_4096, COUNTERS_32, COUNTERS_4 (53 valid
 * points in all).
 * configs / valid: host arrays of RTCDF_GRID_SIZE entries, either may be
 * NULL. */
#define RTCDF_GRID_SIZE 62
rtcdf_status_t rtcdf_config_grid(rtcdf_config_t* configs, uint8_t* valid);

/* Exhaustive autotuner: times every valid grid configuration of the plain
 * sort of keys_in into keys_out (device arrays, as rtcdf_sort_with_config)
 * with HIP events on `stream`: `warmup` untimed sorts, then the median of
 * `reps` timed sorts.  times_ms: host array of RTCDF_GRID_SIZE (invalid
 * points get -1); *best (may be NULL) receives the fastest configuration
 * (an option point as its (0, 0, 0, flags) form).  keys_out holds the sorted
 * keys afterwards.  Synchronises the stream. */
rtcdf_status_t rtcdf_autotune(const int32_t* keys_in, int32_t* keys_out, size_t n, int64_t minVal,
                              int64_t maxVal, uint32_t warmup, uint32_t reps, float* times_ms,
                              rtcdf_config_t* best, hipStream_t stream);

/* TUNED mode table: a text file of lines "log2n log2R T items blocks" (the
 * best configuration measured for arrays of that size and range; '#' starts
 * a comment line).  rtcdf_sort then uses the row nearest to (log2 n, log2 R). */
rtcdf_status_t rtcdf_load_tuned_table(const char* path);

/* LEARNED mode model: a file written by paper_2609_00843_amd/learn.py
 * ("RTCDFMLP", version 3, sizes, training ranges of log2 n and log2 R, the
 * decision margin and the trusted feature range zmax, feature mean and sd,
 * the RTCDF_MLP_PARAMS weights, the valid-configuration mask; files whose
 * output count is not RTCDF_GRID_SIZE are refused).  The network predicts a
 * centred log run time per grid point from the keys' sketch.  In LEARNED
 * mode, a sort given no configuration (and rtcdf_pick_config with keys):
 *  - uses the network's fastest point where it predicts at least `margin`
 *    (natural-log units) less than for the configuration TUNED/DEFAULT would
 *    give, else keeps that one;
 *  - where the network is not trusted -- n or R outside its training ranges
 *    by more than half an octave, or a sketch more than zmax standard
 *    deviations from the training mean in some feature (zmax 0: no limit) --
 *    times the whole grid on the keys (rtcdf_autotune, into a scratch buffer
 *    it allocates) and uses the fastest point; that result is kept for the
 *    shape class (n and R to half an octave, the sketch's largest bin fraction
 *    and its position), so later arrays of the class are not timed again
 *    (rtcdf_set_learned_fallback(0) keeps TUNED/DEFAULT there instead);
 *  - keeps every decision for (device, keys_in, n, minVal, maxVal) until the
 *    model changes or rtcdf_clear_pick_cache, so a buffer sorted again costs
 *    no pick (outputs are identical whatever is chosen; only speed differs).
 * A sort never waits for the network: its first call for a buffer enqueues
 * the pick (one small kernel whose result lands in pinned host memory) on
 * `stream` ahead of the sort and sorts with the TUNED/DEFAULT choice; a later
 * call uses the decision once that kernel has finished.  The exhaustive
 * fallback, when it runs, times the grid inside the call that decides.
 * rtcdf_pick_config waits for the pick and decides at once.  Under stream
 * capture the pick is skipped.  rtcdf_unload_model forgets the model. */
rtcdf_status_t rtcdf_load_model(const char* path);
rtcdf_status_t rtcdf_unload_model(void);
rtcdf_status_t rtcdf_set_learned_fallback(int on);
rtcdf_status_t rtcdf_clear_pick_cache(void);

/* How the last configuration choice on this thread was made (by a sort given
 * no configuration, or rtcdf_pick_config), and its grid index (-1 if the
 * configuration is not a grid point). */
typedef enum rtcdf_pick_source {
  RTCDF_PICK_STATIC = 0,               /* TUNED/DEFAULT, the network not consulted */
  RTCDF_PICK_NETWORK = 1,              /* the network's point */
  RTCDF_PICK_NETWORK_KEPT_STATIC = 2,  /* the network predicted less than the margin of gain */
  RTCDF_PICK_AUTOTUNED = 3,            /* exhaustive timing (network not trusted) */
  RTCDF_PICK_CACHED = 4,               /* an earlier decision for the same buffer and problem */
  RTCDF_PICK_PENDING = 5               /* the static choice: the network's pick for this buffer
                                          is still running (a sort never waits for it) */
} rtcdf_pick_source_t;
int rtcdf_last_pick_source(void);
int rtcdf_last_pick_index(void);

/* ---- Learned picker kernels (the network is trained by these) ---------- */

/* Sketch features of an array: [log2 n, log2 R, fraction of S =
 * min(RTCDF_SKETCH_SAMPLES, n) evenly spaced sample keys (key at position
 * floor(i * n / S)) in each of RTCDF_SKETCH_BINS equal-width bins of the
 * range].  d_features: device float[RTCDF_MLP_INPUTS]. */
#define RTCDF_SKETCH_BINS 32
#define RTCDF_SKETCH_SAMPLES 4096
#define RTCDF_MLP_INPUTS 34
#define RTCDF_MLP_HIDDEN 64
#define RTCDF_MLP_OUTPUTS 62
#define RTCDF_MLP_PARAMS 10430
rtcdf_status_t rtcdf_sketch(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                            float* d_features, hipStream_t stream);

/* FP32 MLP y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 (34 -> 64 -> 64 -> 62, one
 * output per grid point).
 * d_params: device float[RTCDF_MLP_PARAMS] laid out W1[64][34] b1 W2[64][64]
 * b2 W3[62][64] b3.  d_X: batch x 34 (row-major), d_Y: batch x 62. */
rtcdf_status_t rtcdf_mlp_forward(const float* d_params, const float* d_X, uint32_t batch, float* d_Y,
                                 hipStream_t stream);

/* Device workspace for rtcdf_mlp_gradient / rtcdf_mlp_train at this batch. */
rtcdf_status_t rtcdf_mlp_workspace_bytes(uint32_t batch, size_t* bytes);

/* Gradient of the masked mean squared error sum(M (Y - T)^2) / sum(M) over
 * the batch (d_T, d_M: batch x 62; M is 0/1) into d_grad[RTCDF_MLP_PARAMS];
 * the loss into d_loss[0] if not NULL.  Deterministic (fixed-order sums).
 * Reads back the mask total (synchronises the stream). */
rtcdf_status_t rtcdf_mlp_gradient(const float* d_params, const float* d_X, const float* d_T,
                                  const float* d_M, uint32_t batch, float* d_grad, float* d_loss,
                                  void* d_ws, size_t ws_bytes, hipStream_t stream);

/* One Adam step (Kingma & Ba) at step t >= 1 on the flat parameter array with
 * moments d_m, d_v (device float[RTCDF_MLP_PARAMS], updated in place). */
rtcdf_status_t rtcdf_mlp_adam_step(float* d_params, const float* d_grad, float* d_m, float* d_v,
                                   uint32_t t, float lr, float beta1, float beta2, float eps,
                                   hipStream_t stream);

/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) numbered
 * t0 + 1 .. t0 + steps; the loss before each step goes to
 * d_loss_history[k] when not NULL. */
rtcdf_status_t rtcdf_mlp_train(float* d_params, float* d_m, float* d_v, uint32_t t0, const float* d_X,
                               const float* d_T, const float* d_M, uint32_t batch, uint32_t steps,
                               float lr, void* d_ws, size_t ws_bytes, float* d_loss_history,
                               hipStream_t stream);

/* Sketch -> standardised features ((f - mean) / sd, d_norm = mean[34] then
 * sd[34]) -> MLP -> index of the smallest prediction among d_valid[62] != 0
 * (lowest index on ties) into d_index[0]; predictions into d_pred[62] if not
 * NULL.  d_params must be 16-byte aligned.  One small launch, no host
 * synchronisation. */
rtcdf_status_t rtcdf_mlp_pick(const int32_t* keys_in, size_t n, int64_t minVal, int64_t maxVal,
                              const float* d_params, const float* d_norm, const uint8_t* d_valid,
                              uint32_t* d_index, float* d_pred, hipStream_t stream);

/* The configuration rtcdf_sort would use for (n, R) under the current mode,
 * written to *cfg, flags included (learned mode needs the keys for its
 * sketch; keys_in may be NULL in the other modes).  Synchronises `stream` in
 * learned mode. */
rtcdf_status_t rtcdf_pick_config(const int32_t* keys_in, size_t n, int64_t minVal,
                                 int64_t maxVal, hipStream_t stream, rtcdf_config_t* cfg);

/* ---- Misc -------------------------------------------------------------- */

const char* rtcdf_status_string(rtcdf_status_t status);
/* The hipError_t of the last RTCDF_ERROR_HIP on this thread (0 if none). */
int rtcdf_last_hip_error(void);
/* Per-stage timing for measurement.  While enabled, every plain sort records
 * HIP events on its stream around its four stages (0 histogram, 1 partial-row
 * reduction, 2 local CDF + tile offsets, 3 output; stages 1 and 2 take no
 * time on the single-tile fast path, whose output stage does both); rtcdf_profile_collect
 * waits for the recorded events, writes the summed milliseconds per stage and
 * the number of sorts to *out, and forgets them.  Disabled by default. */
typedef struct rtcdf_stage_stats {
  uint64_t sorts;
  double ms[4];
} rtcdf_stage_stats_t;

rtcdf_status_t rtcdf_profile_enable(int on);
rtcdf_status_t rtcdf_profile_collect(rtcdf_stage_stats_t* out);

/* Measurement utility: copies `bytes` (a multiple of 16) from d_src to d_dst
 * (16-byte aligned device buffers, not overlapping) with a plain streaming
 * kernel.  Its bandwidth is the attainable-HBM reference the sort kernels are
 * compared with, and its HBM counters calibrate counter-derived traffic. */
rtcdf_status_t rtcdf_stream_copy(const void* d_src, void* d_dst, size_t bytes, hipStream_t stream);

/* The launch plan rtcdf_sort_with_config would use (cfg NULL = library
 * choice; keys_in / keys_out are only inspected for alignment and may be
 * NULL), for measurement and tests. */
typedef struct rtcdf_plan_info {
  uint32_t tile_width;       /* effective T */
  uint32_t tiles;            /* m = ceil(R / T) */
  uint32_t counter_bits;     /* 32, 16 (two per LDS word) or 8 (four per word) */
  uint32_t passes;           /* LDS passes over the input */
  uint32_t pass_bins;        /* bins per pass */
  uint32_t hist_workgroups;  /* passes x chunks */
  uint32_t hist_threads;
  uint32_t items_per_thread;
  uint32_t scan_workgroups;  /* local-CDF workgroups; 0 on the single-tile fast
                                path (one tile, one pass of 32-bit counters, R <= 2048),
                                where the output stage reduces and scans the counts */
  uint32_t out_chunk;        /* output positions per chunk (per wave with the
                                prefix-maximum output) */
  uint32_t out_chunks;
  uint32_t fill_workgroups;  /* output-stage workgroups */
  uint64_t workspace_bytes;
  uint32_t output_flags;     /* RTCDF_FLAG_OUTPUT_PREFIX_MAX when the output is
                                written by Alg. 3, else 0 */
  uint32_t partition_buckets;  /* > 0: the keys are first partitioned by LDS pass
                                  into this many buckets (one more read and write
                                  of the keys; each pass then reads its bucket
                                  only); 0: every pass reads the whole input */
  uint32_t hist_dedupe;        /* 1: the histogram aggregates a wave's duplicates
                                  (RTCDF_FLAG_WAVE_DEDUPE) */
} rtcdf_plan_info_t;

rtcdf_status_t rtcdf_plan_info(size_t n, int64_t minVal, int64_t maxVal, const rtcdf_config_t* cfg,
                               const int32_t* keys_in, const int32_t* keys_out, rtcdf_plan_info_t* out);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int rtcdf_version(void);
/* Frees the library's cached per-device workspaces (not needed before exit). */
rtcdf_status_t rtcdf_release_workspaces(void);

#ifdef __cplusplus
}
#endif
#endif /* RTCDF_H */
