/*
 * sat_oracle.c -- plain, serial CPU oracle for the integral-image sliding-window method.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  The product path (the HIP library) never links or calls it,
 * and this file shares no code, header, table or helper with that path.
 *
 * What it computes (Ockerman, Klamer, Haab, "Accelerating Biological Spatial Cluster Analysis
 * with the Parallel Integral Image Technique"):
 *   - the integral image / summed-area table: each entry is the sum of every pixel above and to
 *     the left of it, the entry's own pixel included (Sec. II-B);
 *   - the window sum at every window position, stored in a new array with one entry per
 *     position of the valid region, (r-w+1)(c-w+1) of them for stride 1 (Sec. II-A, Sec. III-A);
 *   - the same window sum by the four-corner lookup into the table (Sec. II-B, Sec. III-B);
 *   - the integral-image window average and standard deviation (Sec. II-A).
 * Readings where the paper is silent (inclusive table, population deviation, stride, non-square
 * windows, 64-bit wrap-around) are listed in the design notes of this repository.
 *
 * Everything is single-threaded, integer arithmetic in uint64_t (wrapping mod 2^64) unless
 * stated.  Images are row-major with a row pitch given in elements; pixel types are 8- or 16-bit
 * unsigned (bpp = 1 or 2).  Tables written here are dense (row pitch == W).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Pixel (y, x) of an image with `bpp` bytes per pixel and a pitch in elements. */
static uint64_t pixel(const void *img, int bpp, int64_t pitch, int64_t y, int64_t x) {
    if (bpp == 1) return ((const uint8_t *)img)[y * pitch + x];
    return ((const uint16_t *)img)[y * pitch + x];
}

/* Number of window positions along one axis of length n for window length k and stride s:
 * positions 0, s, 2s, ... whose window stays inside the image (valid region only). */
int oracle_window_shape(int64_t H, int64_t W, int64_t h, int64_t w, int64_t s,
                        int64_t *out_h, int64_t *out_w) {
    if (H < 1 || W < 1 || h < 1 || w < 1 || s < 1 || h > H || w > W) return 1;
    *out_h = (H - h) / s + 1;
    *out_w = (W - w) / s + 1;
    return 0;
}

/* Integral image, serial (Sec. II-B, Sec. III-B "O(r*c)").  For each row a running row sum is
 * kept; the table entry is the entry directly above plus that running sum:
 *   S[y][x] = S[y-1][x] + sum_{j<=x} I[y][j],  S[-1][x] = 0.
 * Q is the same table over the squared pixels; either output may be NULL. */
int oracle_sat(const void *img, int bpp, int64_t H, int64_t W, int64_t pitch,
               uint64_t *S, uint64_t *Q) {
    if (!img || H < 1 || W < 1 || pitch < W || (bpp != 1 && bpp != 2)) return 1;
    for (int64_t y = 0; y < H; ++y) {
        uint64_t run = 0, run_sq = 0;
        for (int64_t x = 0; x < W; ++x) {
            uint64_t v = pixel(img, bpp, pitch, y, x);
            run += v;
            run_sq += v * v;
            if (S) S[y * W + x] = (y > 0 ? S[(y - 1) * W + x] : 0) + run;
            if (Q) Q[y * W + x] = (y > 0 ? Q[(y - 1) * W + x] : 0) + run_sq;
        }
    }
    return 0;
}

/* Column totals of an image (the column direction of the table of Sec. II-B): entry x is the
 * sum of column x over all H rows, added to carry[x] (zero where carry is NULL); T2 likewise over
 * the squared pixels (may be NULL).  Row r0 + y of a taller image's table is then the table of
 * its rows r0 .. r0 + H' - 1 plus the running sum along x of the totals of rows 0 .. r0 - 1. */
int oracle_column_totals(const void *img, int bpp, int64_t H, int64_t W, int64_t pitch,
                         const uint64_t *carry, const uint64_t *carry_sq, uint64_t *T, uint64_t *T2) {
    if (!img || !T || H < 1 || W < 1 || pitch < W || (bpp != 1 && bpp != 2)) return 1;
    for (int64_t x = 0; x < W; ++x) {
        T[x] = carry ? carry[x] : 0;
        if (T2) T2[x] = carry_sq ? carry_sq[x] : 0;
    }
    for (int64_t y = 0; y < H; ++y) {       /* row by row, in memory order */
        for (int64_t x = 0; x < W; ++x) {
            uint64_t v = pixel(img, bpp, pitch, y, x);
            T[x] += v;
            if (T2) T2[x] += v * v;
        }
    }
    return 0;
}

/* Table entry with the convention that row -1 and column -1 are zero. */
static uint64_t sat_at(const uint64_t *S, int64_t W, int64_t y, int64_t x) {
    if (y < 0 || x < 0) return 0;
    return S[y * W + x];
}

/* Window sums by the four-corner lookup (Sec. II-B, Sec. III-B "4(r*c)"): the value at the
 * bottom-right corner, minus the value just above the window at its right edge, minus the value
 * just left of the window at its bottom edge, plus the value diagonally above-left, which was
 * subtracted twice.  Window k,l covers rows k*s .. k*s+h-1 and columns l*s .. l*s+w-1.
 * Arithmetic wraps mod 2^64; the result is exact whenever the true window sum is below 2^64. */
int oracle_window_sum_sat(const uint64_t *S, int64_t H, int64_t W, int64_t h, int64_t w,
                          int64_t s, uint64_t *out) {
    int64_t oh, ow;
    if (!S || !out || oracle_window_shape(H, W, h, w, s, &oh, &ow)) return 1;
    for (int64_t k = 0; k < oh; ++k) {
        int64_t y0 = k * s, y1 = y0 + h - 1;
        for (int64_t l = 0; l < ow; ++l) {
            int64_t x0 = l * s, x1 = x0 + w - 1;
            out[k * ow + l] = sat_at(S, W, y1, x1) - sat_at(S, W, y0 - 1, x1)
                            - sat_at(S, W, y1, x0 - 1) + sat_at(S, W, y0 - 1, x0 - 1);
        }
    }
    return 0;
}

/* One window summed directly, pixel by pixel: the naive analysis of Sec. II-A at one position.
 * Returns the sum and the sum of squares. */
void oracle_window_at(const void *img, int bpp, int64_t pitch, int64_t y0, int64_t x0,
                      int64_t h, int64_t w, uint64_t *sum, uint64_t *sum_sq) {
    uint64_t a = 0, b = 0;
    for (int64_t y = y0; y < y0 + h; ++y)
        for (int64_t x = x0; x < x0 + w; ++x) {
            uint64_t v = pixel(img, bpp, pitch, y, x);
            a += v;
            b += v * v;
        }
    if (sum) *sum = a;
    if (sum_sq) *sum_sq = b;
}

/* Naive sliding-window analysis (Sec. II-A, cost O((r-w+1)(c-w+1)w^2) of Sec. III-A): every
 * window position is summed directly.  `squares` selects the sum of squared pixels instead. */
int oracle_window_sum_direct(const void *img, int bpp, int64_t H, int64_t W, int64_t pitch,
                             int64_t h, int64_t w, int64_t s, int squares, uint64_t *out) {
    int64_t oh, ow;
    if (!img || !out || pitch < W || (bpp != 1 && bpp != 2)) return 1;
    if (oracle_window_shape(H, W, h, w, s, &oh, &ow)) return 1;
    for (int64_t k = 0; k < oh; ++k)
        for (int64_t l = 0; l < ow; ++l) {
            uint64_t a, b;
            oracle_window_at(img, bpp, pitch, k * s, l * s, h, w, &a, &b);
            out[k * ow + l] = squares ? b : a;
        }
    return 0;
}

/* Window average and population standard deviation from the exact integer window sum S1 and sum
 * of squares Q1 over n pixels (Sec. II-A names both statistics; the formulas are the textbook
 * ones):  mean = S1 / n;  variance = (n*Q1 - S1^2) / n^2, so std = sqrt(n*Q1 - S1^2) / n.
 * The numerator is formed exactly in 128-bit integers (it is >= 0 by Cauchy-Schwarz) and rounded
 * to double once; then one correctly rounded square root and one division follow. */
void oracle_mean_std(const uint64_t *sums, const uint64_t *sum_sqs, int64_t count, uint64_t n,
                     double *mean, double *std_dev) {
    for (int64_t i = 0; i < count; ++i) {
        u128 num = (u128)n * sum_sqs[i] - (u128)sums[i] * sums[i];
        mean[i] = (double)sums[i] / (double)n;
        std_dev[i] = sqrt((double)num) / (double)n;
    }
}

/* Sum over all window positions of the window sums, computed the other way round: every pixel
 * weighted by the number of window positions that contain it.  Wraps mod 2^64.  This is an
 * identity that holds at any size, used to check full-scale outputs without storing them. */
uint64_t oracle_coverage_total(const void *img, int bpp, int64_t H, int64_t W, int64_t pitch,
                               int64_t h, int64_t w, int64_t s) {
    int64_t oh, ow;
    if (oracle_window_shape(H, W, h, w, s, &oh, &ow)) return 0;
    uint64_t *cy = (uint64_t *)calloc((size_t)H, sizeof(uint64_t));
    uint64_t *cx = (uint64_t *)calloc((size_t)W, sizeof(uint64_t));
    if (!cy || !cx) { free(cy); free(cx); return 0; }
    for (int64_t k = 0; k < oh; ++k)
        for (int64_t y = k * s; y < k * s + h; ++y) cy[y] += 1;
    for (int64_t l = 0; l < ow; ++l)
        for (int64_t x = l * s; x < l * s + w; ++x) cx[x] += 1;
    uint64_t total = 0;
    for (int64_t y = 0; y < H; ++y) {
        if (!cy[y]) continue;
        uint64_t row = 0;
        for (int64_t x = 0; x < W; ++x) row += pixel(img, bpp, pitch, y, x) * cx[x];
        total += row * cy[y];
    }
    free(cy);
    free(cx);
    return total;
}

/* The serial integral image of oracle_sat, run over an image too large to hold its table: only
 * the last hmax+1 table rows are kept (a ring).  While the table is built row by row the routine
 * copies out requested table rows and, for each requested window, the requested output rows,
 * each by the four-corner lookup of oracle_window_sum_sat.  Nothing is reordered: row y of the
 * table is produced exactly as in oracle_sat, and an output row is emitted as soon as the last
 * table row it needs exists.
 *
 *   nwin windows (win_h[i], win_w[i]) share stride s; window i requests n_rows[i] output rows,
 *   listed consecutively in rows[] (each list ascending), and receives them consecutively in
 *   out[] (each row ow_i entries).  sat_rows (ascending, n_sat entries) are copied to sat_out
 *   (W entries each).  *total receives the last table entry (the image total mod 2^64).
 *   `squares` builds the table of squared pixels instead.  Returns 0 on success. */
int oracle_stream(const void *img, int bpp, int64_t H, int64_t W, int64_t pitch, int squares,
                  int64_t nwin, const int64_t *win_h, const int64_t *win_w, int64_t s,
                  const int64_t *n_rows, const int64_t *rows, uint64_t *out,
                  int64_t n_sat, const int64_t *sat_rows, uint64_t *sat_out, uint64_t *total) {
    if (!img || H < 1 || W < 1 || pitch < W || (bpp != 1 && bpp != 2) || s < 1) return 1;
    int64_t hmax = 1;
    for (int64_t i = 0; i < nwin; ++i) {
        int64_t oh, ow;
        if (oracle_window_shape(H, W, win_h[i], win_w[i], s, &oh, &ow)) return 1;
        if (win_h[i] > hmax) hmax = win_h[i];
    }
    int64_t ring = hmax + 1;
    uint64_t *T = (uint64_t *)malloc((size_t)(ring * W) * sizeof(uint64_t));
    int64_t *next = (int64_t *)calloc((size_t)(nwin > 0 ? nwin : 1), sizeof(int64_t));
    int64_t *row_base = (int64_t *)calloc((size_t)(nwin > 0 ? nwin : 1), sizeof(int64_t));
    int64_t *out_base = (int64_t *)calloc((size_t)(nwin > 0 ? nwin : 1), sizeof(int64_t));
    if (!T || !next || !row_base || !out_base) {
        free(T); free(next); free(row_base); free(out_base);
        return 2;
    }
    for (int64_t i = 1; i < nwin; ++i) {
        int64_t oh, ow;
        oracle_window_shape(H, W, win_h[i - 1], win_w[i - 1], s, &oh, &ow);
        row_base[i] = row_base[i - 1] + n_rows[i - 1];
        out_base[i] = out_base[i - 1] + n_rows[i - 1] * ow;
    }
    int64_t next_sat = 0;
    for (int64_t y = 0; y < H; ++y) {
        uint64_t *cur = T + (y % ring) * W;
        const uint64_t *up = y > 0 ? T + ((y - 1) % ring) * W : NULL;
        uint64_t run = 0;
        for (int64_t x = 0; x < W; ++x) {
            uint64_t v = pixel(img, bpp, pitch, y, x);
            run += squares ? v * v : v;
            cur[x] = (up ? up[x] : 0) + run;
        }
        while (next_sat < n_sat && sat_rows[next_sat] == y) {
            memcpy(sat_out + next_sat * W, cur, (size_t)W * sizeof(uint64_t));
            ++next_sat;
        }
        for (int64_t i = 0; i < nwin; ++i) {
            int64_t h = win_h[i], w = win_w[i], oh, ow;
            oracle_window_shape(H, W, h, w, s, &oh, &ow);
            while (next[i] < n_rows[i]) {
                int64_t k = rows[row_base[i] + next[i]];
                if (k < 0 || k >= oh) { next[i] = n_rows[i]; break; }
                int64_t y0 = k * s, y1 = y0 + h - 1;
                if (y1 != y) break;
                const uint64_t *bot = T + (y1 % ring) * W;
                const uint64_t *top = y0 > 0 ? T + ((y0 - 1) % ring) * W : NULL;
                uint64_t *o = out + out_base[i] + next[i] * ow;
                for (int64_t l = 0; l < ow; ++l) {
                    int64_t x0 = l * s, x1 = x0 + w - 1;
                    uint64_t b1 = bot[x1], b0 = x0 > 0 ? bot[x0 - 1] : 0;
                    uint64_t t1 = top ? top[x1] : 0, t0 = (top && x0 > 0) ? top[x0 - 1] : 0;
                    o[l] = b1 - t1 - b0 + t0;
                }
                ++next[i];
            }
        }
    }
    if (total) *total = T[((H - 1) % ring) * W + (W - 1)];
    free(T); free(next); free(row_base); free(out_base);
    return 0;
}

/* ---- The streamed integral image, resumable and started part-way down the image.
 *
 * The same serial recurrence as oracle_sat / oracle_stream, begun at image row r0 instead of row
 * 0.  The rows above r0 enter only through their column totals carry[x] = sum_{y<r0} I[y][x]: by
 * the definition of the table (Sec. II-B) the table row just above the start is
 *   S[r0-1][x] = sum_{j<=x} carry[j],
 * and every later row follows from it by the recurrence S[y][x] = S[y-1][x] + sum_{j<=x} I[y][j].
 * The stream keeps that recurrence's last hmax+1 rows (a ring) between calls, so a caller walks
 * the image in bands of rows; several streams started at different rows cover one image in
 * parallel, each from the column totals of the rows above its start.
 *
 * Window sums are emitted by the four-corner lookup of oracle_window_sum_sat as soon as the
 * bottom row of a window exists, for every window whose rows all lie at or below r0 (the row
 * above such a window, r0-1 at the highest, is in the ring). */
typedef struct {
    const void *img;
    int bpp, squares;
    int64_t H, W, pitch, s, r0, cur, ring, nwin;
    int64_t win_h[8], win_w[8], next_k[8];
    uint64_t *T;       /* ring of table rows: row y lives at slot y % ring */
} oracle_stream_state;

/* Start a stream at image row r0 (0 <= r0 <= H; r0 == H gives a stream with nothing to do).
 * img points at row 0 of the whole H x W image (pitch in elements).  carry: column totals of rows
 * 0..r0-1 (of the squared pixels when `squares`), W entries, required when r0 > 0 and ignored
 * otherwise.  Up to 8 windows (win_h[i], win_w[i]) sharing stride s, each fitting the image.
 * Returns NULL on bad arguments or allocation failure. */
void *oracle_stream_open(const void *img, int bpp, int64_t H, int64_t W, int64_t pitch, int squares,
                         int64_t nwin, const int64_t *win_h, const int64_t *win_w, int64_t s, int64_t r0,
                         const uint64_t *carry) {
    if (!img || H < 1 || W < 1 || pitch < W || (bpp != 1 && bpp != 2) || s < 1) return NULL;
    if (nwin < 0 || nwin > 8 || r0 < 0 || r0 > H || (r0 > 0 && !carry)) return NULL;
    oracle_stream_state *st = (oracle_stream_state *)calloc(1, sizeof(oracle_stream_state));
    if (!st) return NULL;
    int64_t hmax = 1;
    for (int64_t i = 0; i < nwin; ++i) {
        int64_t oh, ow;
        if (oracle_window_shape(H, W, win_h[i], win_w[i], s, &oh, &ow)) {
            free(st);
            return NULL;
        }
        st->win_h[i] = win_h[i];
        st->win_w[i] = win_w[i];
        st->next_k[i] = (r0 + s - 1) / s;      /* first window whose top row is at or below r0 */
        if (win_h[i] > hmax) hmax = win_h[i];
    }
    st->img = img;
    st->bpp = bpp;
    st->squares = squares;
    st->H = H;
    st->W = W;
    st->pitch = pitch;
    st->s = s;
    st->r0 = r0;
    st->cur = r0;
    st->nwin = nwin;
    st->ring = hmax + 1;
    st->T = (uint64_t *)malloc((size_t)(st->ring * W) * sizeof(uint64_t));
    if (!st->T) {
        free(st);
        return NULL;
    }
    if (r0 > 0) {      /* table row r0 - 1: the running sum along x of the totals above */
        uint64_t *above = st->T + ((r0 - 1) % st->ring) * W, run = 0;
        for (int64_t x = 0; x < W; ++x) {
            run += carry[x];
            above[x] = run;
        }
    }
    return st;
}

/* Continue the stream through image row r1 - 1 (st's current row <= r1 <= H).  Table rows
 * cur .. r1-1 are copied to sat_out (W entries each) when it is non-NULL.  For window i, the output
 * rows k whose window lies in rows r0 .. r1-1 and was not emitted before are written to outs[i]
 * consecutively (ow_i entries each; outs may be NULL when there are no windows); k_first[i] and
 * n_out[i] (may be NULL) receive the first such row index and their number.  Returns 0, or 1 on
 * bad arguments. */
int oracle_stream_next(void *handle, int64_t r1, uint64_t *sat_out, uint64_t *const *outs, int64_t *k_first,
                       int64_t *n_out) {
    oracle_stream_state *st = (oracle_stream_state *)handle;
    if (!st || r1 < st->cur || r1 > st->H || (st->nwin > 0 && !outs)) return 1;
    const int64_t W = st->W, s = st->s;
    int64_t emitted[8] = {0};
    for (int64_t i = 0; i < st->nwin; ++i)
        if (k_first) k_first[i] = st->next_k[i];
    for (int64_t y = st->cur; y < r1; ++y) {
        uint64_t *cur = st->T + (y % st->ring) * W;
        const uint64_t *up = y > 0 ? st->T + ((y - 1) % st->ring) * W : NULL;
        uint64_t run = 0;
        for (int64_t x = 0; x < W; ++x) {
            uint64_t v = pixel(st->img, st->bpp, st->pitch, y, x);
            run += st->squares ? v * v : v;
            cur[x] = (up ? up[x] : 0) + run;
        }
        if (sat_out) memcpy(sat_out + (y - st->cur) * W, cur, (size_t)W * sizeof(uint64_t));
        for (int64_t i = 0; i < st->nwin; ++i) {
            int64_t h = st->win_h[i], w = st->win_w[i], oh, ow;
            oracle_window_shape(st->H, W, h, w, s, &oh, &ow);
            int64_t k = st->next_k[i];
            if (k >= oh || k * s + h - 1 != y) continue;   /* window k ends on a later row */
            int64_t y0 = k * s, y1 = y;
            const uint64_t *bot = st->T + (y1 % st->ring) * W;
            const uint64_t *top = y0 > 0 ? st->T + ((y0 - 1) % st->ring) * W : NULL;
            uint64_t *o = outs[i] + emitted[i] * ow;
            for (int64_t l = 0; l < ow; ++l) {
                int64_t x0 = l * s, x1 = x0 + w - 1;
                uint64_t b1 = bot[x1], b0 = x0 > 0 ? bot[x0 - 1] : 0;
                uint64_t t1 = top ? top[x1] : 0, t0 = (top && x0 > 0) ? top[x0 - 1] : 0;
                o[l] = b1 - t1 - b0 + t0;
            }
            ++emitted[i];
            st->next_k[i] = k + 1;
        }
    }
    for (int64_t i = 0; i < st->nwin; ++i)
        if (n_out) n_out[i] = emitted[i];
    st->cur = r1;
    return 0;
}

void oracle_stream_close(void *handle) {
    oracle_stream_state *st = (oracle_stream_state *)handle;
    if (!st) return;
    free(st->T);
    free(st);
}

/* ---- Higher window moments from tables of pixel powers (the method applied to I^k).
 *
 * The paper lists further sliding-window statistics as future work (Sec. V) and builds every
 * statistic it has from window sums (Sec. II-A, II-B).  The third and fourth moments are sums
 * too: with S_k the window sum of pixel^k over n pixels, the central moments expand into the raw
 * sums by the binomial theorem.  Readings: population moments (divisor n), skewness
 * g1 = m3 / m2^(3/2), excess kurtosis g2 = m4 / m2^2 - 3, both undefined (NaN) when m2 = 0. */

typedef __int128 i128;

/* Integral image of pixel^k, k = 1..4 (k = 1, 2 give the tables of oracle_sat).  Wraps mod
 * 2^64 exactly like oracle_sat.  Returns 0 on success. */
int oracle_sat_power(const void *img, int bpp, int64_t H, int64_t W, int64_t pitch, int k, uint64_t *T) {
    if (!img || !T || H < 1 || W < 1 || pitch < W || (bpp != 1 && bpp != 2) || k < 1 || k > 4) return 1;
    for (int64_t y = 0; y < H; ++y) {
        uint64_t run = 0;
        for (int64_t x = 0; x < W; ++x) {
            uint64_t v = pixel(img, bpp, pitch, y, x), p = v;
            for (int j = 1; j < k; ++j) p *= v;
            run += p;
            T[y * W + x] = (y > 0 ? T[(y - 1) * W + x] : 0) + run;
        }
    }
    return 0;
}

/* sums[j] = sum over the h x w window at (y0, x0) of pixel^(j+1), j < k, summed directly. */
void oracle_window_powers(const void *img, int bpp, int64_t pitch, int64_t y0, int64_t x0, int64_t h,
                          int64_t w, int k, uint64_t *sums) {
    for (int j = 0; j < k; ++j) sums[j] = 0;
    for (int64_t y = y0; y < y0 + h; ++y)
        for (int64_t x = x0; x < x0 + w; ++x) {
            uint64_t v = pixel(img, bpp, pitch, y, x), p = 1;
            for (int j = 0; j < k; ++j) {
                p *= v;
                sums[j] += p;
            }
        }
}

/* Mean, std, skewness and excess kurtosis of `count` windows of n pixels from their exact power
 * sums s1..s4 (s3, s4 may be NULL: skewness / kurtosis not computed).  With
 *   A = n*S2 - S1^2                                   (= n^2 m2),
 *   B = n^2*S3 - 3n*S1*S2 + 2*S1^3                    (= n^3 m3),
 *   C = n^3*S4 - 4n^2*S1*S3 + 6n*S1^2*S2 - 3*S1^4     (= n^4 m4),
 * formed exactly in 128-bit integers, each rounded to double once:
 *   mean = S1/n,  std = sqrt(A)/n,  skew = B / (A*sqrt(A)),  kurt = (C - 3A^2) / (A*A).
 * The caller keeps n and the pixel range small enough for the 128-bit terms. */
void oracle_moments(const uint64_t *s1, const uint64_t *s2, const uint64_t *s3, const uint64_t *s4, int64_t count,
                    uint64_t n, double *mean, double *std_dev, double *skew, double *kurt) {
    const i128 N = (i128)n;
    for (int64_t i = 0; i < count; ++i) {
        const i128 a1 = (i128)s1[i], a2 = (i128)s2[i];
        const i128 A = N * a2 - a1 * a1;
        const double a = (double)A;
        mean[i] = (double)s1[i] / (double)n;
        std_dev[i] = sqrt(a) / (double)n;
        if (skew) {
            const i128 a3 = (i128)s3[i];
            const i128 B = N * N * a3 - 3 * N * a1 * a2 + 2 * a1 * a1 * a1;
            skew[i] = A == 0 ? NAN : (double)B / (a * sqrt(a));
        }
        if (kurt) {
            const i128 a3 = (i128)s3[i], a4 = (i128)s4[i];
            const i128 C = N * N * N * a4 - 4 * N * N * a1 * a3 + 6 * N * a1 * a1 * a2 - 3 * a1 * a1 * a1 * a1;
            kurt[i] = A == 0 ? NAN : (double)(C - 3 * A * A) / (a * a);
        }
    }
}
