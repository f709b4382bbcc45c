/*
 * ksort.h -- C ABI of the MI355X (gfx950) K-sort library, libksort.so.
 *
 * K-sort (Sundararajan, Pal, Chakraborty, Mahanti, arXiv 1107.3622,
 * Section 1.1) sorts a[left..right] by taking the first element as the key,
 * placing every key that is smaller than it to its left and every key that
 * is larger or equal to its right (Steps 1-4; the key ends at index
 * i = left + number of smaller keys), and repeating on both sides (Steps 5-6)
 * until every side has at most one key (Section 1.2 note).  This library
 * runs each level of that recursion as one pass over all live segments of a
 * device array.
 *
 * Conventions for every entry point below:
 *   - Arrays named d_* are device memory (hipMalloc, or a torch tensor on the
 *     HIP device); the caller owns them and keeps them alive until the work
 *     is complete.  Host pointers are never accepted in a d_* argument.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Keys are IEEE double (KSORT_F64) or float (KSORT_F32), compared in their
 *     own precision exactly as `key <= x`: ties go right; a NaN compares false
 *     and goes left.  The sorted order is unique (bit-exact with any correct
 *     sort) for inputs without NaN and without both +0.0 and -0.0.  With NaNs
 *     the output is still a permutation of the input (every key is kept), in
 *     an order that is not specified.
 *   - Sizes are element counts (int64_t).  n = 0 and n = 1 are valid no-ops.
 *   - Return value: KSORT_OK (0) or a negative KSORT_E* code; nothing is
 *     thrown across the ABI.  ksort_last_error() gives a thread-local detail
 *     string for the most recent failure on the calling thread.
 *   - Completion: the sorting calls return after the work they queued on
 *     `stream` has finished (the level loop reads a completion flag back from
 *     the device), so the output may be read as soon as they return.
 *   - The library keeps one scratch workspace per (device, stream) pair; calls
 *     on the same stream are serialised, calls on different streams run
 *     independently.
 *   - No device wait is unbounded: a partition tile polls for its
 *     predecessors' counts at most 2^22 times (seconds; the environment
 *     variable KSORT_SPIN_LIMIT, a decimal count read whenever a level pass is
 *     enqueued, overrides it) and then ends the pass, which the call reports
 *     as KSORT_EINTERNAL; ksort_last_error() then names the pass, the waiting
 *     tile and the predecessor it waited for.
 *   - Look-back words are tagged with the pass number modulo 2^22 - 1 and
 *     cleared when the tags wrap.  KSORT_EPOCH_SPAN (a decimal count in
 *     [2, 2^22 - 1], read when a sort or a server starts) shortens the span,
 *     so that tests reach the wrap in a few passes.
 *   - Level passes of the plain and batched calls let workgroup b take work
 *     ticket b without an atomic, which assumes the whole grid is dispatched
 *     while its first workgroups wait.  Kernels of other code that keep part
 *     of the device busy at the same time only delay such a pass (for as
 *     long as they hold those slots; the bounded wait above ends it in an
 *     error if that takes seconds).  The server's passes take every ticket
 *     from a counter and do not depend on this.  KSORT_FIXED_FIRST=0 (read
 *     whenever a level pass is enqueued) makes the plain and batched calls
 *     take every ticket from the counter too, for programs that run other
 *     kernels beside the sorts or run them under a counter profiler; it costs
 *     about 14 % at 7e6 keys and 0.5 % at 2^28 (512 claims per pass on one
 *     counter).
 *   - KSORT_VALIDATE=1 (read per call) makes ksort_f64, ksort_f32,
 *     ksort_sort_ex and ksort_segmented first check the whole input buffer
 *     for the inputs outside the bit-exact contract (a NaN, or both +0.0 and
 *     -0.0) and fail with KSORT_EINVAL, no key moved, if it finds one.  It
 *     costs one read of the keys, a small device allocation and a stream
 *     synchronization per call; the server and ksort_sort_static do not
 *     check.
 */
#ifndef KSORT_H
#define KSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define KSORT_API __attribute__((visibility("default")))
#else
#define KSORT_API
#endif

/* error codes */
#define KSORT_OK 0
#define KSORT_EINVAL (-1)      /* bad argument: null pointer with n > 0, n < 0, bad dtype, bad segment */
#define KSORT_ENOMEM (-2)      /* device or host allocation failed */
#define KSORT_EHIP (-3)        /* HIP runtime error (detail in ksort_last_error) */
#define KSORT_EUNSUPPORTED (-4)/* no gfx950 device current */
#define KSORT_ETOOLARGE (-5)   /* request larger than the server's memory budget */
#define KSORT_EAGAIN (-6)      /* server queue full */
#define KSORT_ECANCELLED (-7)  /* request cancelled */
#define KSORT_ETIMEOUT (-8)    /* wait timed out */
#define KSORT_ENOTFOUND (-9)   /* unknown server ticket */
#define KSORT_EINTERNAL (-10)  /* a device check failed: a capacity or count (a library bug), or a look-back wait timed out */

/* key types */
#define KSORT_F64 0
#define KSORT_F32 1

/* Kernel variant: threads per workgroup, keys per thread in a partition tile,
 * and the finish cutoff (segments of at most `cutoff` keys are sorted inside
 * one workgroup's LDS).  All-zero fields mean "library default / autotuned".
 * Only the combinations listed by ksort_variants() exist. */
typedef struct ksort_tuning {
    int32_t block;
    int32_t items;
    int32_t cutoff;
    int32_t reserved;
} ksort_tuning;

/* ------------------------------------------------------------------------
 * Whole-array sort, Steps 1-6 (Section 1.1).
 *
 * ksort_f64 / ksort_f32: sort d_data[0..n-1] ascending, in place.
 *   d_data : device array of n keys (read and overwritten).
 *   n      : number of keys, n >= 0.
 * Scratch: the library uses a device buffer of n keys plus O(n / 2048)
 * descriptors, cached per (device, stream) and grown on demand.
 * Errors: KSORT_EINVAL (d_data NULL with n > 0, n < 0), KSORT_ENOMEM,
 * KSORT_EHIP, KSORT_EUNSUPPORTED.  On error the array content is unspecified
 * but remains a permutation of the input unless the error is KSORT_EHIP or
 * KSORT_EINTERNAL. */
KSORT_API int ksort_f64(double *d_data, int64_t n, void *stream);
KSORT_API int ksort_f32(float *d_data, int64_t n, void *stream);

/* ksort_sort_ex: as above with explicit key type and options.
 *   dtype         : KSORT_F64 or KSORT_F32.
 *   d_first_pivot : device int64, nullable; receives the index i at which the
 *                   first partition call (Step-4 on the whole array) left the
 *                   key a[0]: the number of keys smaller than a[0].  0 for
 *                   n == 1, -1 for n == 0.
 *   tune          : nullable; kernel variant to use (NULL = default/tuned). */
KSORT_API int ksort_sort_ex(int dtype, void *d_data, int64_t n, int64_t *d_first_pivot,
                  const ksort_tuning *tune, void *stream);

/* ------------------------------------------------------------------------
 * One partition level, Steps 1-4 (Section 1.1), on many segments at once.
 *
 * For every segment s, with left = d_seg_left[s], len = d_seg_len[s] and
 * right = left + len - 1, the keys d_in[left..right] are written to
 * d_out[left..right] partitioned around key = d_in[left]:
 *   d_out[left .. i-1]   the keys smaller than the key (some order),
 *   d_out[i]             the key, i = left + #{x in (left, right] : key > x},
 *   d_out[i+1 .. right]  the other keys (some order);
 * and d_pivot[s] = i (absolute index).  The index i is exactly the one the
 * paper's Step-4 produces; the order within each side is this library's
 * (smaller keys in tile order, the others in reverse tile order), not the
 * order Steps 2-3 leave.
 *   d_in, d_out : device arrays of n keys; they must not overlap.  Elements
 *                 of d_out outside every segment are not written.
 *   d_seg_left, d_seg_len : device int64 arrays of nseg entries; segments
 *                 must be disjoint, 1 <= len and left + len <= n.
 *   d_pivot     : device int64 array of nseg entries (output).
 * Errors: KSORT_EINVAL for a bad dtype/pointer/size or any segment outside
 * [0, n) or with len < 1 (such segments are skipped; the others are done).
 * Overlapping segments give unspecified results. */
KSORT_API int ksort_partition_level(int dtype, const void *d_in, void *d_out, int64_t n,
                          const int64_t *d_seg_left, const int64_t *d_seg_len,
                          int64_t nseg, int64_t *d_pivot, void *stream);

/* ------------------------------------------------------------------------
 * The literal arrangement (Section 1.1, Steps 1-4 exactly as the sequential
 * steps leave the array).
 *
 * ksort_partition_level_exact: as ksort_partition_level, except that
 *   d_out[left..right] is exactly the array the paper's Steps 1-4 leave for
 *   each segment, not only the same pivot index and sides: with c the count
 *   of smaller keys, i = left + c and m = i + 1 if i < right and
 *   d_in[i+1] >= key (else m = i), the key goes to i and the first key >= key
 *   in (left, m] (the Step-3.1 temp) to i + 1, a smaller key at x <= m to
 *   x - 1, a larger-or-equal key at x > m stays, and the k-th key >= key in
 *   (left, m] (k >= 2) trades places with the (k-1)-th smaller key in
 *   (m, right] counted from the right (which goes to q_k - 1).
 *   Segments of one key are calls too (d_out[left] = key, pivot left).
 *   Overlapping segments are rejected with KSORT_EINVAL (nothing is
 *   written); invalid segments are skipped as in ksort_partition_level.
 *   n < 2^31.  The segment arrays are read back to the host and the call
 *   synchronizes the stream.  Device scratch of about 25n + 2n *
 *   sizeof(key) bytes is kept per (device, stream) between calls and grown
 *   when a call needs more; ksort_release_workspaces frees it.
 *
 * ksort_sort_exact: Steps 1-6 on d_data[0..n-1], in place, every partition
 *   call leaving the literal arrangement, so every call (its segment, key
 *   and pivot index) is the one the sequential algorithm makes; calls on
 *   the sides of a level run together (breadth-first) instead of depth-first,
 *   which changes no call.  A side is partitioned further when it holds two
 *   or more keys (Steps 5-6).
 *   d_first_pivot : device int64, nullable: i of the call on [0, n-1]
 *                   (0 for n == 1, -1 for n == 0).
 *   d_calls       : device int64 array of 3 * calls_cap entries, nullable;
 *                   receives (left, right, i) of up to calls_cap calls in no
 *                   particular order.
 *   d_ncalls      : device int64, required with d_calls (else nullable):
 *                   the total number of calls (may exceed calls_cap).
 *   The call synchronizes the stream once per eight levels (the level count
 *   is the recursion depth down to sides of 64 keys, which one wave each
 *   finishes: about 2 log2 n on random keys, about n on sorted input).  Its
 *   device scratch, about 33n + 3n * sizeof(key) bytes, is kept per
 *   (device, stream) as for ksort_partition_level_exact.  n < 2^31.
 * Errors: KSORT_EINVAL (bad dtype, n < 0 or >= 2^31, null data with n > 0,
 * d_calls without d_ncalls), KSORT_ENOMEM, KSORT_EHIP, KSORT_EUNSUPPORTED. */
KSORT_API int ksort_partition_level_exact(int dtype, const void *d_in, void *d_out, int64_t n,
                                const int64_t *d_seg_left, const int64_t *d_seg_len,
                                int64_t nseg, int64_t *d_pivot, void *stream);
KSORT_API int ksort_sort_exact(int dtype, void *d_data, int64_t n, int64_t *d_first_pivot,
                     int64_t *d_calls, int64_t calls_cap, int64_t *d_ncalls, void *stream);

/* ------------------------------------------------------------------------
 * Batched sort: Steps 1-6 on each array of a packed batch.
 *
 * Array u is d_packed[d_offsets[u] .. d_offsets[u+1]-1]; each is sorted on
 * its own, in place, all of them in one sequence of level passes.
 *   d_packed        : device array of n_total keys.
 *   d_offsets       : device int64 array of nseg + 1 non-decreasing offsets,
 *                     d_offsets[0] >= 0 and d_offsets[nseg] <= n_total.
 *   d_first_pivots  : device int64 array of nseg entries, nullable; entry u
 *                     receives the first partition's index i relative to the
 *                     array start (0 for one key, -1 for an empty array).
 *   tune            : nullable kernel variant.
 * The level sequence is recorded once per (stream, sizes, pointers) as a HIP
 * graph and replayed on later calls with the same arguments.
 * Errors: KSORT_EINVAL for bad pointers/sizes or offsets that break the rules
 * above (arrays that do are skipped; the others are sorted). */
KSORT_API int ksort_segmented(int dtype, void *d_packed, int64_t n_total,
                    const int64_t *d_offsets, int64_t nseg,
                    int64_t *d_first_pivots, const ksort_tuning *tune,
                    void *stream);

/* ------------------------------------------------------------------------
 * Variants, tuning and profiling (library services, not paper passages).
 *
 * ksort_variants: writes up to `cap` compiled variants for `dtype` to `out`
 *   (host array) and returns how many exist (or a negative error).
 * ksort_get_default / ksort_set_default: the variant used when `tune` is
 *   NULL, per key type (host struct).  Unless a default was set or the size
 *   was tuned, sorts of fewer than 3e6 keys use (512, 16, 1024) instead.
 *   Servers and one-level passes always use the default.
 * ksort_autotune: times every variant (best of five runs) on a seeded input
 *   of n keys on the current device and stores the fastest as the variant
 *   for single arrays of about that size (the same power-of-two bucket, or
 *   the nearest tuned bucket at most two powers of two away); the untuned
 *   default is kept unless another variant is at least 1 % faster.  `out`
 *   (host, nullable) receives the choice.  Uses a temporary device buffer
 *   of 2n keys.
 * ksort_autotune_batch: the same for packed batches (ksort_segmented), timed
 *   on copies of the caller's batch (d_packed is left as it is; arguments as
 *   ksort_segmented), keyed by the batch's total key count.  Uses a
 *   temporary device buffer of n_total keys.
 * ksort_tune_file: choices persist in the JSON file `path` (host string),
 *   one entry per (device architecture, single or batch, key type, size
 *   bucket) with the tuned and the default variant's times: its entries are
 *   read and applied now (those of other architectures are kept, unused),
 *   and every later tuning rewrites it.  NULL stops writing and forgets
 *   every choice (calls take the untuned defaults again).  The environment
 *   variable KSORT_TUNE_FILE names such a file at first use.
 *   A file that cannot be read holds no entries.
 * ksort_tune_count: number of tuning entries known (all architectures).
 * ksort_profile_enable(1) makes every level pass record HIP events on its
 *   stream; ksort_profile_read copies up to `cap` records (host array) and
 *   clears them; ksort_profile_count returns how many are held.
 * Environment: KSORT_TRACE=<path> (read at first use) makes every sorting
 *   call record the same per-pass events and append one JSON line per level
 *   pass to <path> (call, dtype, stage, live_keys, finish_keys, ms, block,
 *   items, cutoff, grid); KSORT_ROCTX=1 puts a roctx range around every
 *   batch of level passes (shown by profilers with host-side markers, for
 *   example rocprofv3 --marker-trace), loading the roctx library at first
 *   use if it is installed. */
typedef struct ksort_level_record {
    int64_t call;         /* sequence number of the sorting call */
    int32_t dtype;
    int32_t stage;        /* pass index within the call (0 = whole arrays) */
    int64_t live_keys;    /* keys partitioned in this pass, counted once per
                             partition call (a chain of one-tile segments run
                             within the pass counts each of its calls) */
    int64_t finish_keys;  /* keys sorted by the LDS finish in this pass */
    double ms;            /* pass duration from HIP events */
    int32_t block, items, cutoff, grid;
} ksort_level_record;

KSORT_API int ksort_variants(int dtype, ksort_tuning *out, int cap);
KSORT_API int ksort_get_default(int dtype, ksort_tuning *out);
KSORT_API int ksort_set_default(int dtype, const ksort_tuning *tune);
KSORT_API int ksort_autotune(int dtype, int64_t n, ksort_tuning *out, void *stream);
KSORT_API int ksort_autotune_batch(int dtype, const void *d_packed, int64_t n_total, const int64_t *d_offsets,
                                   int64_t nseg, ksort_tuning *out, void *stream);
KSORT_API int ksort_tune_file(const char *path);
KSORT_API int ksort_tune_count(void);
KSORT_API int ksort_profile_enable(int on);
KSORT_API int64_t ksort_profile_count(void);
KSORT_API int64_t ksort_profile_read(ksort_level_record *out, int64_t cap);

/* ksort_stream_copy: copies `bytes` bytes from d_src to d_dst (device
 * buffers, 16-byte aligned, not overlapping) with a streaming kernel shaped
 * like a level pass (persistent grid, 16-byte accesses per lane).  It is the
 * measured ceiling a level pass is compared with: a pass reads and writes
 * each live key once, as a copy does.  grid <= 0 takes occupancy x compute
 * units workgroups.  Asynchronous on `stream`.  Errors: KSORT_EINVAL (null or
 * misaligned buffers), KSORT_EHIP. */
KSORT_API int ksort_stream_copy(void *d_dst, const void *d_src, size_t bytes, int grid, void *stream);

/* Bytes of device scratch a sort (ksort_f64/f32, ksort_sort_ex with the
 * default variant, ksort_segmented) or a one-level pass of n keys in nseg
 * arrays or segments needs (host only, no device call).  0 for a bad dtype
 * or a negative size. */
KSORT_API size_t ksort_workspace_bytes(int dtype, int64_t n, int64_t nseg);

/* ksort_set_workspace: the scratch of calls on `stream` of the current
 * device comes from the caller's memory instead of the library's.
 *   d_ws   : device memory, 256-byte aligned, of `bytes` bytes; owned by the
 *            caller, who keeps it alive and leaves it alone until another
 *            ksort_set_workspace on the same stream returns.  NULL hands the
 *            stream back to memory the library allocates itself.
 *   bytes  : size of d_ws, at least 4096.  Size it with ksort_workspace_bytes
 *            for the largest call to come; a call that needs more fails
 *            with KSORT_ENOMEM and allocates nothing.
 *   stream : hipStream_t as void* (NULL = the null stream).
 * Covers ksort_f64/f32, ksort_sort_ex, ksort_segmented and
 * ksort_partition_level on that stream; the literal-arrangement calls and
 * the server allocate their own.  The call waits for the stream's pending
 * work, frees the library's memory of that stream and drops graphs captured
 * for it.  Errors: KSORT_EINVAL (misaligned or smaller than 4096 bytes),
 * KSORT_EHIP. */
KSORT_API int ksort_set_workspace(void *d_ws, size_t bytes, void *stream);

/* ksort_sort_static: ksort_sort_ex (default variant) for callers that cannot
 * allocate memory: code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Its scratch (descriptor lists, counters, flags,
 * look-back words and the ping-pong keys) is a file-scope device array of
 * KSORT_STATIC_SCRATCH_BYTES (64 MiB) that every GPU the library runs on
 * holds until the process ends; the call makes no hipMalloc, hipHostMalloc,
 * hipFree or other allocating call (the first call on a device looks up the
 * array's device address and the device's properties once).
 *   dtype, d_data, n, d_first_pivot, stream: as ksort_sort_ex.
 * Limit: the sort's scratch must fit the array: at most 7,835,072 FP64 or
 * 14,909,568 FP32 keys.  A larger n fails with KSORT_ETOOLARGE before any
 * device work, and ksort_last_error() gives the exact maximum.
 * Calls on one device share the array: the library serializes them (each
 * returns after its work is complete), and a call leaves its contents
 * behind; what must start at zero is cleared by each call.  Work of two
 * processes, or a call recorded into a graph, would race on it: not
 * supported.  Errors: as ksort_sort_ex, and KSORT_ETOOLARGE. */
#define KSORT_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
KSORT_API int ksort_sort_static(int dtype, void *d_data, int64_t n, int64_t *d_first_pivot, void *stream);

/* Releases every cached workspace of the calling process (all devices),
 * the scratch of the literal-arrangement calls included.  Memory given with
 * ksort_set_workspace is not freed (it is the caller's); the streams go back
 * to library-owned memory. */
KSORT_API int ksort_release_workspaces(void);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * A server owns a scheduler thread on one device.  Each submitted request
 * is a device array to sort in place.  Requests are admitted while the sum
 * of their footprints (2 * n * sizeof(key) for data plus ping-pong scratch,
 * plus descriptors) stays within `hbm_budget_bytes` and fewer than
 * `max_inflight` are admitted; every scheduler tick runs one level pass over
 * the live segments of all admitted requests together (one pass per key
 * type), so requests that arrive while others are running join at the next
 * level boundary.  The comparisons and the key rule are those of the plain
 * sort, so each request's output is identical to ksort_f64/ksort_f32 on the
 * same array.
 *
 * ksort_server_create: device = HIP device ordinal.  Returns NULL on error
 *   (see ksort_last_error).
 * ksort_server_submit: d_data is borrowed until the request completes or is
 *   cancelled; *ticket receives its id.  The server runs on streams of its
 *   own, so every write of d_data must be complete when the call is made
 *   (synchronize the producing stream first).  KSORT_ETOOLARGE if the
 *   request can never fit the budget, KSORT_EAGAIN if the pending queue is
 *   full.
 * ksort_server_poll: *state = 0 pending/running, 1 done, or a negative error.
 * ksort_server_wait: blocks up to timeout_s seconds (negative = forever);
 *   returns KSORT_OK when done, KSORT_ETIMEOUT, or the request's error.
 * ksort_server_cancel: a request not yet admitted is dropped
 *   (KSORT_ECANCELLED is then its state); an admitted one runs to completion.
 * ksort_server_result: first pivot (relative index) and timings of a done
 *   request.
 * ksort_server_stats: aggregate counters and latency percentiles.
 * ksort_server_destroy: stops admitting, lets admitted requests finish,
 *   cancels queued ones, joins the thread and frees the server.
 * Request producers may run their own kernels on other streams while the
 * server runs (the server's passes take every work ticket from a counter, so
 * no pass waits for a workgroup that those kernels keep from starting).
 * Each pass runs every finish task it lists (no finish work is deferred to a
 * later pass).  A failed device check fails every request of that key
 * type's lane with KSORT_EINTERNAL (ksort_server_wait then sets
 * ksort_last_error() to the check's detail); the lane clears its state and
 * goes on serving. */
typedef struct ksort_server ksort_server;

typedef struct ksort_request_info {
    int64_t n;
    int32_t dtype;
    int32_t state;          /* as ksort_server_poll */
    int64_t first_pivot;
    double t_submit_s;      /* host steady clock, seconds */
    double t_admit_s;
    double t_done_s;
    int32_t levels;         /* level passes the request took part in */
    int32_t pad;
} ksort_request_info;

typedef struct ksort_server_stats_t {
    int64_t submitted, admitted, completed, rejected, cancelled, failed;
    int64_t keys_completed;
    int64_t ticks;
    double busy_s;          /* wall time with at least one admitted request */
    double p50_latency_s, p99_latency_s, mean_latency_s;
    int64_t inflight_now, queued_now;
    int64_t budget_used_bytes;
} ksort_server_stats_t;

KSORT_API ksort_server *ksort_server_create(size_t hbm_budget_bytes, int max_inflight, int device);
KSORT_API int ksort_server_submit(ksort_server *srv, int dtype, void *d_data, int64_t n, uint64_t *ticket);
KSORT_API int ksort_server_poll(ksort_server *srv, uint64_t ticket, int *state);
KSORT_API int ksort_server_wait(ksort_server *srv, uint64_t ticket, double timeout_s);
KSORT_API int ksort_server_cancel(ksort_server *srv, uint64_t ticket);
KSORT_API int ksort_server_result(ksort_server *srv, uint64_t ticket, ksort_request_info *out);
KSORT_API int ksort_server_stats(ksort_server *srv, ksort_server_stats_t *out);
KSORT_API void ksort_server_destroy(ksort_server *srv);

/* ------------------------------------------------------------------------ */
KSORT_API const char *ksort_strerror(int code);
KSORT_API const char *ksort_last_error(void);
/* Library version string. */
KSORT_API const char *ksort_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KSORT_H */
