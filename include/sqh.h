/*
 * sqh -- segmented QuickHull for planar point sets on AMD MI355X (gfx950).
 *
 * C ABI of libsqh.so. Every entry point takes plain pointers and sizes; no
 * C++ exception crosses this boundary. Device pointers refer to memory on
 * the context's HIP device; "host" pointers to ordinary process memory.
 *
 * What is computed (paper: Zhang, Mei, Xu, Zhao, "A Novel Implementation of
 * QuickHull Algorithm on the GPU", arXiv 1501.04706). Section 1 states the
 * problem: the convex hull of a planar point set. Sections 3-4 give the
 * method this library follows: the points are split by the line through
 * the leftmost and rightmost points (section 4.3, "The First Split"); then,
 * for all segments at once, the farthest point of every segment is found by
 * a segmented reduction (section 4.4.1), points inside the triangle it forms
 * with the segment's end points are discarded and the rest are compacted by
 * a stable partition into the two new segments (sections 4.4.2-4.4.4),
 * until no segment has points left. Segments and their head flags / keys
 * follow section 2 and Table 1.
 *
 * Result convention (exact, independent of rounding): the hull is the list
 * of input indices of the extreme points of conv(points) in counter-
 * clockwise order, starting at the lexicographically smallest position
 * (min x, then min y). Positions are compared by value (-0.0 == +0.0); each
 * vertex is reported by the lowest index at its position; points in the
 * interior of a hull edge are not vertices. n == 0 gives h = 0; a single
 * distinct position gives [lowest index]; collinear input gives
 * [lexmin, lexmax]. All orientation decisions are exact: a float32 filter
 * with a proven error bound, and an exact float64 expansion where the filter
 * cannot decide.
 *
 * Streams and synchronisation: work is enqueued on the caller's stream. The
 * single-hull and batched calls return after the work has finished (they
 * read small status words back to the host); the engine calls are
 * documented one by one below.
 *
 * Threading: a context may be used by one host thread at a time.
 */
#ifndef SQH_H
#define SQH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define SQH_OK          0
#define SQH_EINVAL     -1  /* null pointer, negative size, non-finite coordinate */
#define SQH_ENOMEM     -2  /* workspace smaller than sqh_workspace_bytes() */
#define SQH_ECAPACITY  -3  /* hull larger than the output capacity */
#define SQH_EDEVICE    -4  /* HIP runtime error or device-side fault report */
#define SQH_EBUSY      -5  /* engine: no room for the request right now */
#define SQH_ENOTFOUND  -6  /* engine: nothing finished yet */

/* Predicate precision modes (sqh_set_precision). */
#define SQH_FP32_FILTER     0  /* float32 filters, exact float64 expansion on failure */
#define SQH_FP64_ONLY       1  /* every predicate evaluated exactly in float64 */
#define SQH_FP32_SEMISTATIC 2  /* as SQH_FP32_FILTER without the static line filter */

/* Pre-filter of single hulls (sqh_set_prefilter). */
#define SQH_PREFILTER_NONE    0  /* the plain method */
#define SQH_PREFILTER_QUAD    1  /* the paper's first mode: extremes in x and y */
#define SQH_PREFILTER_OCTAGON 2  /* also the extremes of x + y and x - y */

/* Data layout of the passes of single hulls (sqh_set_variant). */
#define SQH_VARIANT_PARTITION 0  /* each pass partitions a segment into its children */
#define SQH_VARIANT_SORTED    1  /* the paper's x-sorted chains: sort once, then only remove */

typedef struct sqh_ctx sqh_ctx;

#define SQH_MAX_TIMED_PASSES 64

/* Per-call counters of the last sqh_hull / sqh_hull_batched call.
 * ms_total and ms_kernel come from HIP events recorded on the call's stream;
 * the phase times are differences of the device's constant 100 MHz clock read
 * by workgroup 0 at the end of each phase of the persistent kernel (each
 * phase ends at a grid-wide barrier, so they partition ms_kernel). */
typedef struct sqh_stats {
    int64_t passes;           /* segmented passes after the first compaction */
    int64_t points;           /* input points */
    int64_t first_survivors;  /* points kept by the first compaction */
    int64_t survivors_total;  /* sum over passes of points entering the pass */
    int64_t orient_evals;     /* orientation predicates evaluated */
    int64_t orient_exact;     /* ... of which took the exact float64 path */
    int64_t cmp_exact;        /* farthest-point comparisons decided exactly */
    int64_t hull_size;        /* total hull vertices (all sets) */
    int64_t max_segments;     /* largest number of active segments in a pass */
    double  ms_total;         /* device time of the whole call: workspace reset + the cooperative launches */
    double  ms_kernel;        /* the cooperative launches alone (pre-filter, hull kernel; sorted variant:
                                 first phases, sort, passes) */
    double  ms_seed, ms_split, ms_first, ms_pass, ms_emit;  /* phases of the hull kernel (its own clock) */
    double  ms_prefilter;     /* the pre-filter's two phases (extremes, compaction) */
    int64_t prefilter_points; /* points kept by the pre-filter plus its corners; -1: not run */
    int64_t pass_points[SQH_MAX_TIMED_PASSES];    /* points entering pass k */
    int64_t pass_segments[SQH_MAX_TIMED_PASSES];  /* segments in pass k */
    double  pass_ms[SQH_MAX_TIMED_PASSES];        /* kernel time of pass k */
    double  ms_sort;          /* sorted-chain variant: the sort of the first segments */
    int64_t sorted_points;    /* sorted-chain variant: points sorted; -1: no sort ran */
    int64_t sort_violations;  /* sorted-chain variant: neighbours found out of order after the sort (0) */
    int64_t stream_path;      /* 0: general path; 1: the streaming kernels finished the hull;
                                 2: ... and the passes kernel took over (more than 256 segments) */
    int64_t line_filter;      /* 1: the streaming path used the static line filter */
} sqh_stats;

/*
 * Create a context on HIP device `device` (the device becomes current on
 * the calling thread). The context owns only small host/device state
 * (counters, tuning). Returns SQH_OK, SQH_EINVAL (null ctx or bad device)
 * or SQH_EDEVICE.
 */
int sqh_create(sqh_ctx **ctx, int device);

/* Destroy a context created by sqh_create. NULL is ignored. */
void sqh_destroy(sqh_ctx *ctx);

/*
 * Select the predicate precision. SQH_FP32_FILTER (default): each
 * orientation test first takes a float32 filter with a certified error
 * bound (the semi-static bound of the points' offsets, or, on the streaming
 * path when every |coordinate| is at most 2^60 and the input is not far
 * from the origin compared with its extent, a static bound fixed per edge
 * from the input's extent: two FMAs a test); undecided tests take the
 * exact float64 expansion. SQH_FP32_SEMISTATIC: the semi-static filter
 * only. SQH_FP64_ONLY: every test exact. Outputs are identical; only speed
 * and the exact-path counters differ. Returns SQH_OK or SQH_EINVAL.
 */
int sqh_set_precision(sqh_ctx *ctx, int mode);

/*
 * Streaming path on (on != 0, the default) or off. On, a call on one set of
 * at least 2^16 points (no pre-filter, partition variant, 16-byte aligned
 * input) runs its first phases and passes over few large segments as
 * ordinary launches that never wait for one another, and the cooperative
 * passes kernel only for what they leave. The output is identical either
 * way. Returns SQH_OK or SQH_EINVAL.
 */
int sqh_set_streaming(sqh_ctx *ctx, int on);

/*
 * Pre-filter for calls on one set (sqh_hull, or a batch of one set; the
 * engine ignores it): the paper's first mode (section 4.2, Table 2's
 * Mode 1) takes extreme points in x and y and discards the points inside
 * their quadrilateral before the first split; SQH_PREFILTER_OCTAGON adds
 * the extremes of x + y and x - y (rounded to float32). The corners are
 * input points; a point is discarded only when a float32 test certifies it
 * strictly inside every edge of their polygon, which makes it an interior
 * point of the hull. The method then runs on the remaining points, in an
 * unspecified order, carrying their input indices, so the output is
 * identical to the plain method's. Returns SQH_OK or SQH_EINVAL.
 */
int sqh_set_prefilter(sqh_ctx *ctx, int mode);

/*
 * Layout of the passes for calls on one set (sqh_hull, or a batch of one
 * set; other batches and the engine ignore it). SQH_VARIANT_PARTITION
 * (default): every pass moves each segment's points into its two children
 * (a stable three-way partition). SQH_VARIANT_SORTED: the paper's layout
 * (sections 3, 4.3 and 4.4): after the first split the points of each
 * first segment are sorted by x, ascending on the lower chain and
 * descending on the upper one, with a radix sort; every later pass then
 * only removes points, the children staying in order. The output is
 * identical; the stats report the sort's time, the points sorted and a
 * check of the order (sort_violations, 0). Returns SQH_OK or SQH_EINVAL.
 */
int sqh_set_variant(sqh_ctx *ctx, int variant);

/*
 * Device workspace, in bytes, needed by sqh_hull (n_sets = 1) or
 * sqh_hull_batched for n_total points in n_sets sets. The workspace holds
 * two survivor buffers (x, y float32 and index int32 per point), the
 * segment tables, the vertex bitmap and the look-back status words. It is
 * caller-owned device memory, reused across calls, 256-byte aligned.
 * Returns 0 if n_total or n_sets is out of range (n_total > 2^31 - 2).
 */
size_t sqh_workspace_bytes(int64_t n_total, int64_t n_sets);

/*
 * Convex hull of one point set.
 *   d_xy     device, n interleaved (x, y) float32 pairs (array of
 *            structures, 8 bytes per point); read only.
 *   n        number of points, 0 <= n <= 2^31 - 2.
 *   d_out    device, out_cap int32; receives the hull indices (0-based into
 *            d_xy) in counter-clockwise order from the lexmin point.
 *   h_count  host; receives the hull size h (also when h > out_cap).
 *   d_ws     device workspace of ws_bytes >= sqh_workspace_bytes(n, 1).
 *   stream   HIP stream (hipStream_t; NULL = default stream).
 * Returns SQH_OK; SQH_EINVAL for null pointers, n out of range or any
 * NaN/Inf coordinate; SQH_ENOMEM for a small workspace; SQH_ECAPACITY when
 * h > out_cap (d_out then holds the first out_cap vertices); SQH_EDEVICE.
 * Synchronises the stream before returning.
 */
int sqh_hull(sqh_ctx *ctx, const float *d_xy, int64_t n, int32_t *d_out, int64_t out_cap,
             int64_t *h_count, void *d_ws, size_t ws_bytes, void *stream);

/*
 * The same hull from separate coordinate arrays (structure of arrays):
 * d_x[i], d_y[i] (device, float32, n each) are point i. One streaming kernel
 * interleaves them into the front of the workspace (8 bytes per point,
 * 16-byte aligned), then the call runs as sqh_hull on that copy, so indices,
 * order, errors and synchronisation are those of sqh_hull. The workspace
 * needs ws_bytes >= sqh_workspace_bytes_soa(n) (0 when n is out of range).
 */
size_t sqh_workspace_bytes_soa(int64_t n);
int sqh_hull_soa(sqh_ctx *ctx, const float *d_x, const float *d_y, int64_t n, int32_t *d_out, int64_t out_cap,
                 int64_t *h_count, void *d_ws, size_t ws_bytes, void *stream);

/*
 * sqh_hull without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). The library keeps one static scratch
 * array per device (40 MiB, held until the process ends); the call allocates
 * nothing. Arguments, result convention and return codes are those of
 * sqh_hull, plus SQH_ENOMEM when n > SQH_NOALLOC_MAX_POINTS, and
 * SQH_EDEVICE when the scratch array's device address could not be obtained
 * by sqh_create. Every call on a device shares that device's array: calls
 * that overlap on one device (several streams, threads or contexts) race
 * and must be serialised by the caller. Synchronises the stream.
 */
#define SQH_NOALLOC_MAX_POINTS 262144
int sqh_hull_noalloc(sqh_ctx *ctx, const float *d_xy, int64_t n, int32_t *d_out, int64_t out_cap,
                     int64_t *h_count, void *stream);

/*
 * Convex hulls of n_sets independent point sets stored back to back.
 *   d_xy       device, n_total (x, y) float32 pairs.
 *   d_set_off  device, n_sets + 1 int64, non-decreasing, d_set_off[0] = 0,
 *              d_set_off[n_sets] = n_total; set s owns points
 *              [d_set_off[s], d_set_off[s+1]). Empty sets are allowed.
 *   d_out      device, out_cap int32; set s's hull (indices local to the
 *              set) is written at d_out[d_out_off[s] .. d_out_off[s+1]).
 *   d_out_off  device, n_sets + 1 int64, written by the call.
 *   h_total    host; receives d_out_off[n_sets] (total vertices).
 * All sets are processed together: the per-set first split and every pass
 * run over the segments of all sets in one launch sequence. Returns as
 * sqh_hull (SQH_ECAPACITY if the total exceeds out_cap; then no hull is
 * written past out_cap). Synchronises the stream before returning.
 */
int sqh_hull_batched(sqh_ctx *ctx, const float *d_xy, const int64_t *d_set_off, int64_t n_sets,
                     int64_t n_total, int32_t *d_out, int64_t *d_out_off, int64_t out_cap,
                     int64_t *h_total, void *d_ws, size_t ws_bytes, void *stream);

/*
 * Launch-shape autotuner (not part of the paper's method; it chooses how the
 * same computation is laid out on the device). Runs the batched problem
 * described by the arguments (as sqh_hull_batched; d_set_off and d_out_off
 * may be NULL when n_sets == 1) once per candidate shape plus `reps` timed
 * repetitions (1..100), and stores the fastest shape in the context for
 * this problem's size class, floor(log2(n_total)). Candidates: the number of
 * workgroups of the persistent kernel (all co-resident ones, 3/4, 1/2, 1/4)
 * times the tail threshold (0, 2^13, 2^16 points; at most 256 segments) below which one
 * workgroup finishes the remaining passes; for one set of at least 2^16
 * points (streaming on) also the streaming path with 1024, 512 or 256
 * workgroups per kernel. Later calls of any size use the
 * entry of the nearest class. The output of every shape is identical; only
 * time differs. Leaves the last candidate's result in d_out. Returns as
 * sqh_hull_batched, or SQH_ENOMEM when the context's table (40 classes) is
 * full. Synchronises the stream.
 */
int sqh_autotune(sqh_ctx *ctx, const float *d_xy, const int64_t *d_set_off, int64_t n_sets, int64_t n_total,
                 int32_t *d_out, int64_t *d_out_off, int64_t out_cap, void *d_ws, size_t ws_bytes,
                 void *stream, int reps);

/*
 * The context's tuning table as JSON,
 *   {"entries": [{"log2n": K, "grid": G, "tail": T, "stream": S, "sgrid": W}, ...], "engine_grid": E}
 * (S = 1: large single hulls may take the streaming path; W = its kernels'
 * workgroups, 0 = the default of twice the co-resident grid, at most 1024)
 * ("engine_grid", present when set, is the number of workgroups of a serving
 * engine step; by default a step leaves 1/8 of the compute units free so
 * that the copies of the next step's admissions can run beside it)
 * written NUL-terminated into host buffer `buf` of `len` bytes (truncated
 * if short; buf may be NULL). Returns the length the full text needs,
 * including the NUL, or SQH_EINVAL.
 */
int sqh_get_tuning(const sqh_ctx *ctx, char *buf, size_t len);

/*
 * Replace the context's tuning table with the entries of `json` (the format
 * of sqh_get_tuning; an empty list restores the built-in shape; a missing
 * "engine_grid" restores the engine default). Rejects the whole text with
 * SQH_EINVAL if an entry lacks a key or has grid outside [1, co-resident
 * workgroups of this device], a negative tail, stream not 0 or 1, or sgrid
 * outside [0, 1024], or engine_grid is outside [1, co-resident workgroups].
 * "stream" and "sgrid" are optional (defaults 1 and 0).
 */
int sqh_set_tuning(sqh_ctx *ctx, const char *json);

/*
 * A HIP graph of one batched hull on fixed buffers: a kernel node that
 * resets the workspace and the persistent kernel's node (launched as a
 * cooperative kernel), with the launch shape chosen by the context's tuning
 * table when the graph is created. The arguments are those of
 * sqh_hull_batched (d_set_off and d_out_off may be NULL when n_sets == 1);
 * the buffers must outlive the graph, and their contents (points, set
 * offsets) are read at every launch, so the caller may refill them between
 * launches with the same sizes. The graph captures the precision mode at
 * creation. Returns SQH_OK and *graph, or the codes of sqh_hull_batched.
 */
typedef struct sqh_graph sqh_graph;
int sqh_graph_create(sqh_ctx *ctx, const float *d_xy, const int64_t *d_set_off, int64_t n_sets,
                     int64_t n_total, int32_t *d_out, int64_t *d_out_off, int64_t out_cap, void *d_ws,
                     size_t ws_bytes, sqh_graph **graph);

/* Enqueue one replay of the graph on `stream`. Does not synchronise;
 * d_out / d_out_off are valid once the stream reaches this point. Launches
 * of one graph (or of anything sharing its workspace) must not overlap. */
int sqh_graph_launch(sqh_graph *graph, void *stream);

/* Synchronise `stream`, then read the status of the graph's last replay:
 * *h_total (host, may be NULL) receives the total hull vertices, and the
 * context's counters (sqh_get_stats) are filled, except the event times.
 * Returns as sqh_hull_batched. */
int sqh_graph_result(sqh_graph *graph, int64_t *h_total, void *stream);

/* Destroy a graph. NULL is ignored. */
void sqh_graph_destroy(sqh_graph *graph);

/*
 * Serving engine: continuous batching of hull requests over one device
 * arena (an extension beyond the paper: the paper's segments -- section 2,
 * Table 1 -- of many independent requests share one segment table).
 *
 * The arena is caller-owned device memory of sqh_engine_bytes(slots,
 * max_requests, stage_points) bytes. A request of n points occupies n slots
 * (rounded up to 64) from admission until its hull has been collected:
 * admission is by this footprint. Admitted points wait in a staging area of
 * stage_points points until the next step. Every step
 *   - runs the seed, first split and first compaction (sections 4.3-4.4) of
 *     the requests admitted since the last step and appends their segments to
 *     the resident segment table,
 *   - runs up to max_passes passes (section 4.4) over the segments of every
 *     resident request at once, so new and old requests share each launch,
 *   - emits the hulls of the requests left without segments (same result
 *     convention as sqh_hull, indices local to the request) and frees their
 *     slots.
 * An engine is used by one host thread. Admissions may use their own stream
 * (a copy stream) and overlap a launched step.
 */
typedef struct sqh_engine sqh_engine;

/* Arena bytes for `slots` (a multiple of 64, 64 <= slots <= 2^31 - 128)
 * point slots, up to max_requests (1 .. 2^20) requests in flight and two
 * staging halves of stage_points (1 .. slots) points each (admissions fill
 * one half while a launched step reads the other). 0 if out of range. */
size_t sqh_engine_bytes(int64_t slots, int64_t max_requests, int64_t stage_points);

/* Create an engine over device arena d_arena of arena_bytes bytes
 * (>= sqh_engine_bytes). The context supplies the device, the precision
 * mode and the launch-shape tuning; it must outlive the engine. Returns
 * SQH_OK, SQH_EINVAL, SQH_ENOMEM (arena too small) or SQH_EDEVICE. */
int sqh_engine_create(sqh_ctx *ctx, void *d_arena, size_t arena_bytes, int64_t slots, int64_t max_requests,
                      int64_t stage_points, sqh_engine **engine);

/* Destroy an engine (the arena stays the caller's). NULL is ignored. */
void sqh_engine_destroy(sqh_engine *engine);

/*
 * Admit one request of n (x, y) float32 points, copied from `xy` (host
 * memory if on_device == 0, else device memory) into the staging area on
 * `stream`; `tag` identifies it in sqh_engine_poll. Returns SQH_OK;
 * SQH_EBUSY when its slots, the staging area or the request table have no
 * room now (retry after a step); SQH_EINVAL for a null pointer, n < 0 or n
 * larger than the slots or the staging area; SQH_EDEVICE. n == 0 finishes
 * at once with an empty hull. Non-finite coordinates are reported by
 * sqh_engine_poll for that request only.
 */
int sqh_engine_admit(sqh_engine *engine, const float *xy, int64_t n, uint64_t tag, int on_device,
                     void *stream);

/*
 * Enqueue one step (see above) with at most max_passes (1 .. 65536) passes
 * on `stream` and return without waiting. The step takes every request
 * admitted so far (it waits on the device for their copies, whatever stream
 * they were admitted on); requests admitted while it runs go to the other
 * staging half and join the next step. Returns SQH_OK; SQH_ENOTFOUND if no
 * request is staged or resident; SQH_EBUSY if a step is already in flight;
 * SQH_EINVAL; SQH_EDEVICE.
 */
int sqh_engine_launch(sqh_engine *engine, int max_passes, void *stream);

/*
 * Wait for the launched step and collect it: returns the number of requests
 * that finished in it (their hulls then wait for sqh_engine_poll; their
 * slots are free again), 0 if no step is in flight, or SQH_EDEVICE (the
 * engine is unusable afterwards).
 */
int sqh_engine_finish(sqh_engine *engine);

/* sqh_engine_launch followed by sqh_engine_finish (0 if there is nothing to
 * do). */
int sqh_engine_step(sqh_engine *engine, int max_passes, void *stream);

/*
 * Take the oldest finished request: *tag receives its tag and *h its hull
 * size; up to cap indices go to host array h_out. Returns SQH_OK;
 * SQH_ENOTFOUND if none is finished; SQH_ECAPACITY if h > cap (the result
 * stays queued: call again with a larger buffer); SQH_EINVAL if the
 * request had a non-finite coordinate (the request is consumed, h = 0).
 */
int sqh_engine_poll(sqh_engine *engine, uint64_t *tag, int32_t *h_out, int64_t cap, int64_t *h);

/* Counts of resident (in the segment table), staged (admitted, not yet
 * stepped) and finished-but-not-polled requests, and free slots; any
 * pointer may be NULL. Returns SQH_OK, or SQH_EDEVICE after a failed step. */
int sqh_engine_status(const sqh_engine *engine, int64_t *resident, int64_t *staged, int64_t *finished,
                      int64_t *free_slots);

/* Counters of the last hull call on this context. */
int sqh_get_stats(const sqh_ctx *ctx, sqh_stats *out);

/*
 * Per-launch device times. With on != 0, every later sqh_hull or
 * sqh_hull_batched call on this context records a HIP event on its stream
 * before and after each kernel it launches (the workspace reset included),
 * or, when `only` names a kernel (as sqh_get_launch_times reports it), only
 * around that kernel's launches (each event costs device time between the
 * kernels). Returns SQH_OK, SQH_EINVAL (null ctx, name of 32 characters or
 * more) or SQH_EDEVICE.
 */
int sqh_set_launch_timing(sqh_ctx *ctx, int on, const char *only);

/*
 * The kernels of the last call (launch timing on), in launch order: up to
 * cap entries of a static name and the milliseconds between its two events.
 * A kernel that found nothing to do still appears. Returns the number of
 * entries, or SQH_EINVAL / SQH_EDEVICE.
 */
int sqh_get_launch_times(const sqh_ctx *ctx, const char **names, double *ms, int cap);

/* Diagnostics: with the environment variable SQH_TRACE=1 set before
 * sqh_create, every call records per-workgroup timestamps (100 MHz device
 * clock) at phase boundaries; this copies up to max_entries of them
 * (8 per workgroup, workgroup-major) into host array `out` and returns the
 * number copied (0 when tracing is off), or SQH_EINVAL. */
int sqh_get_trace(const sqh_ctx *ctx, uint64_t *out, int max_entries);

/*
 * Test hooks (they run the device code of the hull path on caller-given
 * cases; no hull call uses them). Device pointers; each call synchronises
 * `stream` and returns SQH_OK, SQH_EINVAL (bad size or null pointer) or
 * SQH_EDEVICE.
 *
 * sqh_diag_orient: for each of n cases of 6 floats (ox, oy, ex, ey, px, py),
 * d_sign[i] = the sign of orient(o, e, p) = (ex-ox)(py-oy) - (ey-oy)(px-ox)
 * as the kernels decide it (float32 semi-static filter, then the exact
 * path; every test exact if fp64_only), d_flags[i] bit 0 = the filter
 * decided, and d_vals[4i..4i+3] = d, es (the filter's value and bound:
 * certified when |d| > es, |d - orient| <= 2 es) and t, m (the static line
 * filter of section 4.4.3's edge tests with Mx, My taken from the case's
 * own coordinates: |t - orient| < m; m = -1 where it does not apply).
 */
int sqh_diag_orient(const float *d_tri, int64_t n, int fp64_only, int32_t *d_sign, float *d_vals, int32_t *d_flags,
                    void *stream);

/*
 * sqh_diag_compare: for each of n cases of 8 floats (ox, oy, ex, ey, px, py,
 * qx, qy) with indices d_ids[2i], d_ids[2i+1], d_out[i] bit 0 = P comes
 * before Q in the farthest-point order for edge o -> e (section 4.4.1:
 * larger area right of the edge; equal areas: earlier along the edge; the
 * same position: lower index), bit 1 = Q before P, both as the kernels
 * decide from float32 intervals and the exact path.
 */
int sqh_diag_compare(const float *d_cases, const int32_t *d_ids, int64_t n, int fp64_only, int32_t *d_out,
                     void *stream);

/*
 * sqh_diag_scan: the workgroup scan of the kernels (section 2's scan over
 * 1024-value runs): d_ex_a[i] = sum of d_in over the run before i, d_ex_b[i]
 * = i's position in its run, d_tot[2r], d_tot[2r+1] = run r's totals.
 */
int sqh_diag_scan(const int32_t *d_in, int64_t n, int32_t *d_ex_a, int32_t *d_ex_b, int32_t *d_tot, void *stream);

/* Static description of a return code. */
const char *sqh_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SQH_H */
