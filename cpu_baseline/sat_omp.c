/*
 * Multi-core CPU baseline for the integral-image sliding-window path: the uint64 integral image
 * of an 8-bit image (Sec. II-B) built in row bands on all host cores, then the sums of every window
 * of the valid region (Sec. III-A) by the four-corner lookup, one band of output rows per thread.
 *
 * This is a comparison point for the benchmark, written for speed on a multi-core host in the
 * manner of the paper's CPU runs (Sec. IV-A): it is neither the oracle (whose serial code stays the
 * definition the tests check against) nor the product path.  It shares no code with either.
 *
 * Build in three passes over the bands of rows b = 0 .. T-1 (T threads):
 *   1. column totals of each band, in parallel;
 *   2. carry[b][x] = the column totals of every band above b (a running sum down the bands);
 *   3. each band swept row by row from its carry: acc[x] += I[y][x]; S[y][x] = sum_{j<=x} acc[j].
 * Window sums: one thread per band of output rows, each reading four table entries per output.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define HOT __attribute__((target_clones("avx2", "default")))

HOT static void add_row(uint64_t *restrict acc, const uint8_t *restrict row, int64_t W) {
    for (int64_t x = 0; x < W; ++x) acc[x] += row[x];
}

HOT static void prefix_row(uint64_t *restrict out, const uint64_t *restrict acc, int64_t W) {
    uint64_t run = 0;
    for (int64_t x = 0; x < W; ++x) {
        run += acc[x];
        out[x] = run;
    }
}

HOT static void corner_row(uint32_t *restrict out, const uint64_t *restrict top, const uint64_t *restrict bot,
                           int64_t ow, int64_t w, int64_t s) {
    /* top == NULL: the window starts on row 0 (the row above contributes zero) */
    for (int64_t l = 0; l < ow; ++l) {
        const int64_t x0 = l * s, x1 = x0 + w - 1;
        uint64_t v = bot[x1] - (x0 ? bot[x0 - 1] : 0);
        if (top) v -= top[x1] - (x0 ? top[x0 - 1] : 0);
        out[l] = (uint32_t)v;
    }
}

/* Table of an H x W 8-bit image (pitch ipitch) into S (pitch spitch), on `threads` threads
 * (<= 0: OpenMP's default).  Returns the thread count used, or -1 if scratch memory ran out. */
int omp_sat_build_u8(const uint8_t *img, int64_t H, int64_t W, int64_t ipitch, uint64_t *S, int64_t spitch,
                     int threads) {
    if (threads <= 0) threads = omp_get_max_threads();
    if (threads > H) threads = (int)H;
    uint64_t *tot = calloc((size_t)threads * (size_t)W, sizeof(uint64_t));
    uint64_t *run = calloc((size_t)W, sizeof(uint64_t));
    if (!tot || !run) {
        free(tot);
        free(run);
        return -1;
    }
#pragma omp parallel num_threads(threads)
    {
        const int b = omp_get_thread_num(), T = omp_get_num_threads();
        const int64_t y0 = H * b / T, y1 = H * (b + 1) / T;
        uint64_t *acc = tot + (size_t)b * W;
        for (int64_t y = y0; y < y1; ++y) add_row(acc, img + y * ipitch, W);
#pragma omp barrier
#pragma omp single
        {
            /* turn band totals into carries from the bands above: running sum down the bands */
            for (int t = 0; t < T; ++t) {
                uint64_t *c = tot + (size_t)t * W;
                for (int64_t x = 0; x < W; ++x) {
                    const uint64_t own = c[x];
                    c[x] = run[x];
                    run[x] += own;
                }
            }
        }
        for (int64_t y = y0; y < y1; ++y) {
            add_row(acc, img + y * ipitch, W);
            prefix_row(S + y * spitch, acc, W);
        }
    }
    free(tot);
    free(run);
    return threads;
}

/* Sums of every win_h x win_w window at `stride` from table S (H x W, pitch spitch) into out
 * (uint32, pitch opitch), output rows spread over `threads` threads. */
int omp_window_sum_u32(const uint64_t *S, int64_t H, int64_t W, int64_t spitch, int64_t win_h, int64_t win_w,
                       int64_t stride, uint32_t *out, int64_t opitch, int threads) {
    if (win_h < 1 || win_w < 1 || stride < 1 || win_h > H || win_w > W) return -1;
    if (threads <= 0) threads = omp_get_max_threads();
    const int64_t oh = (H - win_h) / stride + 1, ow = (W - win_w) / stride + 1;
#pragma omp parallel for num_threads(threads) schedule(static)
    for (int64_t k = 0; k < oh; ++k) {
        const int64_t y0 = k * stride, y1 = y0 + win_h - 1;
        corner_row(out + k * opitch, y0 ? S + (y0 - 1) * spitch : NULL, S + y1 * spitch, ow, win_w, stride);
    }
    return threads;
}
