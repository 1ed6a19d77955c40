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
#define SQH_FP32_FILTER 0  /* float32 filter, exact float64 expansion on failure */
#define SQH_FP64_ONLY   1  /* every predicate evaluated exactly in float64 */

typedef struct sqh_ctx sqh_ctx;

#define SQH_MAX_TIMED_PASSES 64

/* Per-call counters of the last sqh_hull / sqh_hull_batched call. Kernel
 * times come from HIP events recorded on the call's stream around each
 * launch. */
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
    double  ms_total;         /* device time of the whole call */
    double  ms_seed, ms_split, ms_first, ms_pass, ms_table, ms_emit;  /* kernel times */
    int64_t pass_points[SQH_MAX_TIMED_PASSES];    /* points entering pass k */
    int64_t pass_segments[SQH_MAX_TIMED_PASSES];  /* segments in pass k */
    double  pass_ms[SQH_MAX_TIMED_PASSES];        /* kernel time of pass k */
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

/* Select SQH_FP32_FILTER (default) or SQH_FP64_ONLY. Outputs are identical;
 * only speed and the exact-path counters differ. */
int sqh_set_precision(sqh_ctx *ctx, int mode);

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

/* Counters of the last hull call on this context. */
int sqh_get_stats(const sqh_ctx *ctx, sqh_stats *out);

/* Diagnostics: with the environment variable SQH_TRACE=1 set before
 * sqh_create, every call records per-workgroup timestamps (100 MHz device
 * clock) at phase boundaries; this copies up to max_entries of them
 * (8 per workgroup, workgroup-major) into host array `out` and returns the
 * number copied (0 when tracing is off), or SQH_EINVAL. */
int sqh_get_trace(const sqh_ctx *ctx, uint64_t *out, int max_entries);

/* Static description of a return code. */
const char *sqh_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SQH_H */
