/*
 * CPU oracle for the planar convex hull, in plain C -- TEST INFRASTRUCTURE
 * ONLY. It is the timed CPU baseline and the large-n parity reference; only
 * tests/, the smoke check and the benchmark's cpu_baseline leg load it. It
 * shares no code, header or constant with the HIP library.
 *
 * Result (the plain definition, problem stated in the paper's section 1):
 * the counter-clockwise list of input indices of the extreme points of the
 * hull, starting at the lexicographically smallest position, each vertex
 * represented by the lowest index at its position, collinear points on hull
 * edges excluded. n == 0 gives an empty list, one distinct position gives
 * one index, collinear input gives [lexmin, lexmax].
 *
 * Method: Andrew's monotone chain (the sort-then-remove-concave-vertices
 * idea the paper builds on in section 3): sort indices by (x, y, index),
 * drop repeated positions keeping the first, build the lower chain left to
 * right and the upper chain right to left, popping while the last turn is
 * not strictly left.
 *
 * Exact orientation: for float32 inputs each product of two coordinates is
 * exact in binary64 (24+24 significand bits, exponents within range), so
 *   orient(a,b,c) = bx*cy - bx*ay - ax*cy - by*cx + by*ax + ay*cx
 * is a sum of six exact doubles. Its sign is taken from a nonoverlapping
 * expansion built with Knuth's TwoSum and Shewchuk's Grow-Expansion
 * (Shewchuk 1997): the sign of the most significant nonzero component is
 * the sign of the exact sum. Partial sums are multiples of 2^-298, so no
 * step underflows. Build without -ffast-math and without FMA contraction.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_ECAPACITY -3

/* a + b == *s + *e exactly, any magnitudes (Knuth). */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *e = (a - av) + (b - bv);
    *s = x;
}

/* Exact sign of t[0] + ... + t[k-1]. */
static int sum_sign(const double *t, int k)
{
    double e[16];
    int m = 0;
    for (int i = 0; i < k; i++) {
        double q = t[i];
        for (int j = 0; j < m; j++) {
            double s, h;
            two_sum(q, e[j], &s, &h);
            e[j] = h;
            q = s;
        }
        e[m++] = q;
    }
    for (int j = m - 1; j >= 0; j--) {
        if (e[j] > 0.0) return 1;
        if (e[j] < 0.0) return -1;
    }
    return 0;
}

static int orient_sign(const float *xy, int32_t a, int32_t b, int32_t c)
{
    double ax = xy[2 * (int64_t)a], ay = xy[2 * (int64_t)a + 1];
    double bx = xy[2 * (int64_t)b], by = xy[2 * (int64_t)b + 1];
    double cx = xy[2 * (int64_t)c], cy = xy[2 * (int64_t)c + 1];
    double t[6];
    t[0] = bx * cy;
    t[1] = -(bx * ay);
    t[2] = -(ax * cy);
    t[3] = -(by * cx);
    t[4] = by * ax;
    t[5] = ay * cx;
    return sum_sign(t, 6);
}

/* Exposed for the predicate tests. */
int oracle_orient_sign(float ax, float ay, float bx, float by, float cx, float cy)
{
    float p[6] = {ax, ay, bx, by, cx, cy};
    return orient_sign(p, 0, 1, 2);
}

/* ---- sort by (x, y, index): bottom-up merge sort of an index array ---- */

static inline int lex_less(const float *xy, int32_t i, int32_t j)
{
    float xi = xy[2 * (int64_t)i], xj = xy[2 * (int64_t)j];
    if (xi < xj) return 1;
    if (xi > xj) return 0;
    float yi = xy[2 * (int64_t)i + 1], yj = xy[2 * (int64_t)j + 1];
    if (yi < yj) return 1;
    if (yi > yj) return 0;
    return i < j;
}

static void merge_sort(const float *xy, int32_t *a, int32_t *tmp, int64_t n)
{
    for (int64_t w = 1; w < n; w *= 2) {
        for (int64_t lo = 0; lo < n; lo += 2 * w) {
            int64_t mid = lo + w < n ? lo + w : n;
            int64_t hi = lo + 2 * w < n ? lo + 2 * w : n;
            int64_t i = lo, j = mid, k = lo;
            while (i < mid && j < hi) tmp[k++] = lex_less(xy, a[j], a[i]) ? a[j++] : a[i++];
            while (i < mid) tmp[k++] = a[i++];
            while (j < hi) tmp[k++] = a[j++];
        }
        memcpy(a, tmp, (size_t)n * sizeof(int32_t));
    }
}

/*
 * xy: n interleaved (x, y) float32 pairs (host memory, not modified).
 * out: capacity out_cap int32; *h receives the hull size even when it
 * exceeds out_cap (then ORC_ECAPACITY is returned and out holds the first
 * out_cap vertices). Returns ORC_EINVAL for n < 0, n > INT32_MAX or a
 * non-finite coordinate, ORC_ENOMEM if scratch allocation fails.
 */
int oracle_hull(const float *xy, int64_t n, int32_t *out, int64_t out_cap, int64_t *h)
{
    *h = 0;
    if (n < 0 || n > INT32_MAX) return ORC_EINVAL;
    for (int64_t i = 0; i < 2 * n; i++)
        if (!isfinite(xy[i])) return ORC_EINVAL;
    if (n == 0) return ORC_OK;

    int32_t *idx = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int32_t *chain = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t) * 2);
    if (!idx || !tmp || !chain) {
        free(idx); free(tmp); free(chain);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; i++) idx[i] = (int32_t)i;
    merge_sort(xy, idx, tmp, n);

    /* deduplicate positions (value comparison, so -0 == +0), keep first */
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++) {
        if (m > 0) {
            int32_t p = idx[m - 1], q = idx[i];
            if (xy[2 * (int64_t)p] == xy[2 * (int64_t)q] &&
                xy[2 * (int64_t)p + 1] == xy[2 * (int64_t)q + 1])
                continue;
        }
        idx[m++] = idx[i];
    }

    int64_t k = 0;
    if (m == 1) {
        chain[k++] = idx[0];
    } else {
        /* lower chain */
        for (int64_t i = 0; i < m; i++) {
            while (k >= 2 && orient_sign(xy, chain[k - 2], chain[k - 1], idx[i]) <= 0) k--;
            chain[k++] = idx[i];
        }
        /* upper chain; the lower chain's last point starts it */
        int64_t base = k;
        for (int64_t i = m - 2; i >= 0; i--) {
            while (k >= base + 1 && orient_sign(xy, chain[k - 2], chain[k - 1], idx[i]) <= 0) k--;
            chain[k++] = idx[i];
        }
        k--; /* the last point repeats the first */
    }
    *h = k;
    int64_t c = k < out_cap ? k : out_cap;
    for (int64_t i = 0; i < c; i++) out[i] = chain[i];
    free(idx); free(tmp); free(chain);
    return k > out_cap ? ORC_ECAPACITY : ORC_OK;
}
