/*
 * Host sanitizer harness for the C oracle (test infrastructure): built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_oracle_sanitized.py, it reads n and n float32 (x, y) pairs
 * from a file, runs the oracle's hull with the full capacity and with a
 * capacity one short of the hull, and prints the hull indices (one line).
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_hull(const float *xy, int64_t n, int32_t *out, int64_t out_cap, int64_t *h);

int main(int argc, char **argv)
{
    if (argc != 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int64_t n = 0;
    if (fread(&n, sizeof n, 1, f) != 1 || n < 0) return 2;
    float *xy = (float *)malloc((size_t)(2 * n + 1) * sizeof(float));
    int32_t *out = (int32_t *)malloc((size_t)(n + 1) * sizeof(int32_t));
    if (!xy || !out) return 3;
    if (n > 0 && fread(xy, sizeof(float), (size_t)(2 * n), f) != (size_t)(2 * n)) return 2;
    fclose(f);
    int64_t h = 0;
    int rc = oracle_hull(xy, n, out, n, &h);
    if (rc != 0) return 4;
    for (int64_t i = 0; i < h; i++) printf(i ? " %d" : "%d", out[i]);
    printf("\n");
    if (h > 0) {
        /* capacity one short: the first h - 1 vertices and the full count */
        int64_t h2 = 0;
        int32_t *small = (int32_t *)malloc((size_t)h * sizeof(int32_t));
        if (!small) return 3;
        rc = oracle_hull(xy, n, small, h - 1, &h2);
        if (rc == 0 || h2 != h) return 5;
        for (int64_t i = 0; i + 1 < h; i++)
            if (small[i] != out[i]) return 6;
        free(small);
    }
    free(xy);
    free(out);
    return 0;
}
