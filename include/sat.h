/*
 * sat.h -- C ABI of libsat.so: integral image (summed-area table) and sliding-window statistics
 * on an AMD Instinct MI355X (gfx950).
 *
 * The operations are those of Ockerman, Klamer, Haab, "Accelerating Biological Spatial Cluster
 * Analysis with the Parallel Integral Image Technique":
 *   sat_build        the integral image: entry (y, x) is the sum of every pixel above and to the
 *                    left of (y, x), pixel (y, x) included (Sec. II-B; cost O(r*c), Sec. III-B);
 *                    optionally the same table over squared pixels;
 *   window_sum       the sum of every window position of the valid region, one output per
 *                    position, (r-w+1)(c-w+1) of them at stride 1 (Sec. II-A, Sec. III-A), each by
 *                    the four-corner lookup into the table (Sec. II-B; cost 4(r*c), Sec. III-B);
 *   window_mean_std  the window average and standard deviation from the two tables (Sec. II-A);
 *   window_sum_multi several window sizes from one table in one pass (Sec. I, Sec. V);
 *   *_batched        the same over many images in one launch;
 *   sat_build_band   the table of a band of rows of a taller image, from the band and the column
 *                    totals of the rows above it (sat_column_totals);
 *   sat_build_powers the tables of pixel^1 .. pixel^k in one pass, and window_moments the window
 *                    mean, deviation, skewness and excess kurtosis from them (further
 *                    sliding-window statistics, left to future work in Sec. V).
 *
 * Conventions shared by every call:
 *   - Images are row-major, 8- or 16-bit unsigned, with a row pitch in ELEMENTS (>= width; the
 *     base may have any alignment).  Widths and pitches are at most 2^24 elements, heights at
 *     most 2^31-1 rows.  Tables are uint64_t, row-major, pitch in
 *     elements.  Outputs are row-major with a pitch in elements.
 *   - Every data pointer (image, tables, outputs, workspace) is a DEVICE pointer owned by the
 *     caller; the library never allocates or frees device memory.  The one piece it keeps is the
 *     fixed scratch array of sat_build_noalloc, part of its code object on each device.
 *   - Every compute call is asynchronous on `stream` (a hipStream_t passed as void*; NULL is the
 *     default stream).  Results are valid once the stream has been synchronised.
 *   - Arguments are validated completely, on the host, before any HIP call.  On any error the
 *     call enqueues nothing and touches no output; the return value says why and
 *     sat_last_error() gives a message.  No call throws, aborts or exits.
 *   - Table arithmetic wraps modulo 2^64.  A window sum is exact whenever its true value is below
 *     2^64 (every 8-bit window, and every 16-bit window of fewer than 2^32 pixels, squared or not).
 *   - Window (k, l) covers rows k*stride .. k*stride+win_h-1 and columns l*stride ..
 *     l*stride+win_w-1; only windows that fit entirely inside the image exist (valid region).
 *   - Inputs and outputs must not overlap.  Calls on different streams may run concurrently
 *     provided their outputs and workspaces are distinct.
 */
#ifndef SAT_H
#define SAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SAT_OK = 0,
    SAT_ERR_ARG = 1,       /* NULL pointer, size < 1, pitch < width, bad dtype, overlap, ... */
    SAT_ERR_WINDOW = 2,    /* win_h > H or win_w > W: the valid region is empty (Sec. III-A)    */
    SAT_ERR_OVERFLOW = 3,  /* uint32 output asked for but win_h*win_w*max_pixel > UINT32_MAX,
                              or an image too tall for exact 62-bit column totals                */
    SAT_ERR_WORKSPACE = 4, /* workspace NULL or smaller than the matching *_workspace_bytes()   */
    SAT_ERR_HIP = 5,       /* the HIP runtime refused a launch or a query                       */
    SAT_ERR_DEVICE = 6     /* a kernel reported a protocol fault (see sat_workspace_check)      */
} sat_status;

typedef enum {
    SAT_U8 = 1,   /* uint8_t pixels                                     */
    SAT_U16 = 2,  /* uint16_t pixels                                    */
    SAT_U32 = 3,  /* uint32_t window sums (or per-pixel maximum 2^32-1) */
    SAT_U64 = 4,  /* uint64_t window sums                               */
    SAT_F64 = 5   /* double                                             */
} sat_dtype;

/* Output shape of the valid region: out_h = (H - win_h) / stride + 1, out_w likewise
 * (Sec. III-A gives (r-w+1)(c-w+1) positions for stride 1).  Pure host arithmetic.
 * Errors: SAT_ERR_ARG (NULL out pointer, any size or the stride < 1), SAT_ERR_WINDOW. */
sat_status window_out_shape(int64_t H, int64_t W, int64_t win_h, int64_t win_w, int64_t stride,
                            int64_t *out_h, int64_t *out_w);

/* Bytes of device workspace sat_build needs for an H x W image (with_sq != 0: also the squared
 * table), for the kernel variant a sat_build on the calling thread would use (the built-in choice
 * for this size, whatever the alignment of the image's rows, or the one sat_force_variant set).
 * Returns 0 for invalid sizes.  The workspace
 * holds one lookback word per column per strip of rows for the column scan and a control block;
 * its contents need no initialisation and are scratch after the call returns, but the workspace
 * must not be shared by two builds in flight. */
size_t sat_build_workspace_bytes(int64_t H, int64_t W, sat_dtype pixel_type, int with_sq);

/* Integral image of an H x W image (Sec. II-B, Sec. III-B):
 *   sat[y*sat_pitch + x]    = sum_{i<=y, j<=x} image[i*image_pitch + j]           (mod 2^64)
 *   sat_sq[y*sat_pitch + x] = sum_{i<=y, j<=x} image[i*image_pitch + j]^2        (mod 2^64)
 * image: device, pixel_type SAT_U8 or SAT_U16, pitch image_pitch >= W elements, any alignment;
 * rows that start 16-byte aligned (base and pitch) let the build stage image tiles with 16-byte
 * loads, its fastest form.
 * sat: device, H rows of sat_pitch >= W uint64_t; sat_sq: same shape and pitch, or NULL to skip
 * the squared table.  Entries beyond column W-1 of each row are not written.
 * workspace: device, >= sat_build_workspace_bytes(H, W, pixel_type, sat_sq != NULL) bytes.
 * Errors: SAT_ERR_ARG, SAT_ERR_OVERFLOW (H * max_pixel^2 >= 2^62 with sat_sq, H * max_pixel
 * >= 2^62 without), SAT_ERR_WORKSPACE, SAT_ERR_HIP. */
sat_status sat_build(const void *image, sat_dtype pixel_type, int64_t H, int64_t W,
                     int64_t image_pitch, uint64_t *sat, uint64_t *sat_sq, int64_t sat_pitch,
                     void *workspace, size_t workspace_bytes, void *stream);

/* sat_build for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same table, from the same kernels, with
 * the workspace taken from a fixed scratch array inside the library (128 MiB per device, held
 * from the first call on a device until the process ends) instead of an argument.  The caller
 * still passes the image and the tables.  The call allocates and frees nothing.
 * Builds whose sat_build_workspace_bytes(H, W, pixel_type, sat_sq != NULL) exceeds 128 MiB (e.g.
 * 8-bit images beyond about 16000 x 16000, or 16-bit ones with squares beyond about 11500 x 11500)
 * are refused with SAT_ERR_WORKSPACE before anything is enqueued.  Every call on one device uses
 * that device's one scratch array: calls that overlap on a device (two streams, or two threads)
 * race and may corrupt each other's tables; calls in order on one stream are safe.  The scratch
 * array lives on the device of `stream` (the current device for NULL).  Other arguments and
 * errors as sat_build. */
sat_status sat_build_noalloc(const void *image, sat_dtype pixel_type, int64_t H, int64_t W,
                             int64_t image_pitch, uint64_t *sat, uint64_t *sat_sq, int64_t sat_pitch,
                             void *stream);

/* ---- Bands of a taller image.  The integral image is a prefix sum down the columns of the
 * row-wise prefix sums (Sec. II-B), so the table rows of a band of image rows r0 .. r0+H-1 follow
 * from the band alone plus one vector: the column totals of the rows above it,
 *   carry[x] = sum_{i<r0} I[i][x],
 * which contributes sum_{j<=x} carry[j] to every table entry of the band.  Building an image in
 * bands (streamed from the host, or one band per GPU) therefore needs only these W-word vectors
 * passed between bands. */

/* Column totals of an H x W image added to a carry:
 *   out[x]    = carry[x]    + sum_{y<H} image[y*image_pitch + x]                 (mod 2^64)
 *   out_sq[x] = carry_sq[x] + sum_{y<H} image[y*image_pitch + x]^2               (mod 2^64)
 * The carry of the next band, or (with carry = NULL) one band's own totals, for a caller that
 * needs the totals of the rows above a band before that band's rows exist as a table.
 * image: device, SAT_U8 or SAT_U16, as sat_build.  carry / carry_sq: device, W uint64_t, or NULL
 * for zero; each may equal its output (accumulate in place) or must overlap no output.
 * out: device, W uint64_t, 8-byte aligned; out_sq: device, W uint64_t, or NULL to skip the
 * squares (carry_sq must then be NULL; with out_sq and a carry, carry_sq is required).
 * Needs no workspace.  Errors: SAT_ERR_ARG, SAT_ERR_HIP. */
sat_status sat_column_totals(const void *image, sat_dtype pixel_type, int64_t H, int64_t W,
                             int64_t image_pitch, const uint64_t *carry, const uint64_t *carry_sq,
                             uint64_t *out, uint64_t *out_sq, void *stream);

/* Integral image of a band of rows of a taller image, given the column totals of the rows above
 * it (Sec. II-B, as above).  With `image` the band's H rows and carry the column totals of the
 * rows_above rows above it:
 *   sat[y*sat_pitch + x] = sum_{j<=x} carry[j] + sum_{i<=y, j<=x} image[i*image_pitch + j],
 * which is row rows_above + y of the whole image's table; sat_sq likewise from carry_sq and the
 * squared pixels.  carry = NULL means no rows above (rows_above must be 0): then this is
 * sat_build.
 * total_out / total_sq_out: device, W uint64_t, or NULL: receive carry + this band's column
 * totals (carry_sq + squared totals), the carry of the band below.  Each may equal its carry
 * (advance a carry in place) or must overlap nothing else.
 * rows_above bounds the carry: every carry[x] must be at most rows_above * max_pixel (and
 * carry_sq[x] at most rows_above * max_pixel^2), as column totals of rows_above rows are.  The
 * host refuses (rows_above + H) * max_pixel(^2) >= 2^62 with SAT_ERR_OVERFLOW; a carry beyond
 * 2^62 - 1 - H * max_pixel(^2) makes sat_workspace_check report SAT_ERR_DEVICE.  A build without
 * sat_sq whose (rows_above + H) * max_pixel is below 2^30 keeps its lookback words in 32 bits,
 * and there the bound is 2^30 - 1 - H * max_pixel.
 * Other arguments, workspace (sat_build_workspace_bytes(H, W, ...)) and errors as sat_build;
 * a carry with sat_sq needs carry_sq; carries and totals 8-byte aligned. */
sat_status sat_build_band(const void *image, sat_dtype pixel_type, int64_t H, int64_t W,
                          int64_t image_pitch, const uint64_t *carry, const uint64_t *carry_sq,
                          int64_t rows_above, uint64_t *sat, uint64_t *sat_sq, int64_t sat_pitch,
                          uint64_t *total_out, uint64_t *total_sq_out, void *workspace,
                          size_t workspace_bytes, void *stream);

/* Sum of every window of the valid region by the four-corner lookup (Sec. II-B):
 *   out[k*out_pitch + l] = T(y1, x1) - T(y0-1, x1) - T(y1, x0-1) + T(y0-1, x0-1),
 *   y0 = k*stride, y1 = y0+win_h-1, x0 = l*stride, x1 = x0+win_w-1, T(-1, .) = T(., -1) = 0.
 * sat: device table of an H x W image (pitch sat_pitch).  pixel_type gives the largest pixel the
 * table may hold (SAT_U8: 255, SAT_U16: 65535, SAT_U32: 2^32-1 e.g. a table of squared 16-bit
 * pixels) and is used only to refuse a uint32 output that could overflow.
 * out: device, out_h rows (window_out_shape) of out_pitch >= out_w elements of out_type
 * (SAT_U32 or SAT_U64).
 * Errors: SAT_ERR_ARG, SAT_ERR_WINDOW, SAT_ERR_OVERFLOW, SAT_ERR_HIP. */
sat_status window_sum(const uint64_t *sat, sat_dtype pixel_type, int64_t H, int64_t W,
                      int64_t sat_pitch, int64_t win_h, int64_t win_w, int64_t stride,
                      void *out, sat_dtype out_type, int64_t out_pitch, void *stream);

/* Window mean and population standard deviation (Sec. II-A) from the table of pixels and the
 * table of squared pixels, n = win_h*win_w:
 *   S1 = window sum of sat, Q1 = window sum of sat_sq (both by the corner lookup, exact);
 *   mean = (double)S1 / n;  std = sqrt((double)(n*Q1 - S1^2)) / n, the numerator formed
 *   exactly in 128-bit integers and rounded to double once.
 * sat_sq may equal sat for 0/1 images.  sum_out (uint64_t S1) may be NULL; mean_out and
 * std_out are required.  All three share out_pitch (>= out_w elements).
 * Errors: SAT_ERR_ARG, SAT_ERR_WINDOW, SAT_ERR_HIP. */
sat_status window_mean_std(const uint64_t *sat, const uint64_t *sat_sq, int64_t H, int64_t W,
                           int64_t sat_pitch, int64_t win_h, int64_t win_w, int64_t stride,
                           uint64_t *sum_out, double *mean_out, double *std_out,
                           int64_t out_pitch, void *stream);

/* Several window sizes from one table in one pass over it (Sec. I: variable window sizes in
 * constant time; Sec. V: multiple window sizes from a single integral image).  Window i is
 * win_h[i] x win_w[i]; all share `stride`; outs[i] (device, out_type elements, pitch
 * out_pitch[i]) receives exactly what window_sum would write for it.  1 <= n_windows <= 8.
 * win_h, win_w, outs and out_pitch are host arrays read before the call returns.
 * Errors: as window_sum, for any window. */
sat_status window_sum_multi(const uint64_t *sat, sat_dtype pixel_type, int64_t H, int64_t W,
                            int64_t sat_pitch, int32_t n_windows, const int64_t *win_h,
                            const int64_t *win_w, int64_t stride, void *const *outs,
                            sat_dtype out_type, const int64_t *out_pitch, void *stream);

/* One image of a batch (host struct; the pointers in it are device pointers).  For
 * sat_build_batched: image, H, W, image_pitch, sat, sat_sq (may be NULL), sat_pitch.  For
 * window_mean_std_batched additionally sum_out (may be NULL), mean_out, std_out, out_pitch. */
typedef struct {
    const void *image;
    int64_t H, W, image_pitch;
    uint64_t *sat;
    uint64_t *sat_sq;
    int64_t sat_pitch;
    uint64_t *sum_out;
    double *mean_out;
    double *std_out;
    int64_t out_pitch;
} sat_batch_item;

/* Workspace bytes for sat_build_batched / window_mean_std_batched over these items. */
size_t sat_batch_workspace_bytes(const sat_batch_item *items, int32_t n, sat_dtype pixel_type,
                                 int with_sq);

/* The integral images of n images of uneven sizes in ONE persistent launch: workgroups take
 * (image, strip) work items from one queue; each image gets its own column lookback state.
 * Same per-image contract as sat_build.  items is a host array copied before the call returns.
 * Errors: as sat_build, for any item (index in the message), SAT_ERR_ARG for n < 1. */
sat_status sat_build_batched(const sat_batch_item *items, int32_t n, sat_dtype pixel_type,
                             void *workspace, size_t workspace_bytes, void *stream);

/* window_mean_std over n images in one launch, one window size and stride for all.  Items
 * whose image is smaller than the window are an error (SAT_ERR_WINDOW, index in the message).
 * workspace: device, 256-byte aligned, at least 256 + 256 * n bytes (sat_batch_workspace_bytes
 * of the same items is enough); the call writes its descriptor table after the first 256 bytes,
 * so a workspace shared with a preceding build keeps that build's fault word for
 * sat_workspace_check.  items is a host array read before the call returns. */
sat_status window_mean_std_batched(const sat_batch_item *items, int32_t n, int64_t win_h,
                                   int64_t win_w, int64_t stride, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* Workspace bytes for sat_build_stats_batched over these items (0 for invalid sizes). */
size_t sat_build_stats_workspace_bytes(const sat_batch_item *items, int32_t n, sat_dtype pixel_type);

/* The tables of pixels and squares of n images AND the window sum, mean and standard deviation of
 * every image's windows in ONE persistent launch: sat_build_batched followed by
 * window_mean_std_batched, fused.  Workgroups take work items from one queue: first every
 * (image, strip) item of the build, then every statistics item; a statistics item of image i
 * waits until all of image i's strips are stored (a per-image counter; bounded wait, reported by
 * sat_workspace_check), so the statistics of early images overlap the builds of later ones.
 * Items: as sat_build_batched (sat_sq required on every item) plus sum_out (may be NULL),
 * mean_out, std_out and out_pitch as window_mean_std_batched; one window size and stride for all
 * (Sec. II-A statistics of the Sec. II-B tables).  Results equal those of the two calls.  Windows
 * whose height is not a multiple of the stride, and build variants forced outside the fused
 * kernel's set, run as the two launches instead.
 * workspace: device, 256-byte aligned, >= sat_build_stats_workspace_bytes(items, n, pixel_type).
 * Errors: as sat_build_batched and window_mean_std_batched, for any item. */
sat_status sat_build_stats_batched(const sat_batch_item *items, int32_t n, sat_dtype pixel_type, int64_t win_h,
                                   int64_t win_w, int64_t stride, void *workspace, size_t workspace_bytes,
                                   void *stream);

/* Synchronises `stream` and reads the fault word a build left in `workspace`: SAT_OK, or
 * SAT_ERR_DEVICE if a column-lookback wait hit its spin bound, a band build's carry exceeded
 * the bound its rows_above sets, or a fused statistics item's wait for its image's tables hit its
 * spin bound (the results of that call are then unreliable), or SAT_ERR_HIP.
 * Meant for tests and debugging; the fast path never waits. */
sat_status sat_workspace_check(void *workspace, void *stream);

/* Copy nbytes from pinned host memory to device memory with a kernel on `stream`, for callers
 * that feed images from host buffers while other streams compute (the serving loop's uploads).
 * The enqueue is a kernel launch: it returns without waiting for copies in flight elsewhere, where
 * a DMA copy enqueue (hipMemcpyAsync) can hold the calling thread for milliseconds.  The kernel
 * reads the host pages over the bus and writes dst with 16-byte stores.
 * host: memory from hipHostMalloc (torch's pin_memory), valid until the copy has run on the
 * stream; dst: device, nbytes bytes; both 16-byte aligned; they must not overlap.
 * Errors: SAT_ERR_ARG (NULL, nbytes 0, misaligned, or host memory the device cannot address:
 * checked with hipHostGetDevicePointer, which leaves no error pending); SAT_ERR_HIP. */
sat_status sat_upload(const void *host, void *dst, size_t nbytes, void *stream);

/* Message for the last error returned on the calling thread (static storage, never NULL). */
const char *sat_last_error(void);

/* ---- Higher window moments: tables of pixel powers (the integral image of Sec. II-B applied to
 * I^k) and sliding-window statistics beyond the mean and deviation, which the paper leaves to
 * future work (Sec. V).  Every statistic here is a function of window sums of pixel^k. */

/* Bytes of device workspace sat_build_powers needs (0 for invalid sizes, pixel types or k). */
size_t sat_powers_workspace_bytes(int64_t H, int64_t W, sat_dtype pixel_type, int32_t k);

/* Tables of pixel^1 .. pixel^k of an H x W image in one pass over it:
 *   tables[p-1][y*sat_pitch + x] = sum_{i<=y, j<=x} image[i*image_pitch + j]^p      (mod 2^64),
 * so k = 1 gives sat_build's sat and k = 2 its sat_sq.
 * image: device, pixel_type SAT_U8 or SAT_U16, pitch image_pitch >= W elements.
 * tables: HOST array of k device pointers, each H rows of sat_pitch >= W uint64_t; no two may
 * overlap each other or the image.  k = 1..4.
 * workspace: device, >= sat_powers_workspace_bytes(H, W, pixel_type, k) bytes, 16-byte aligned,
 * scratch after the call (not shared by two builds in flight).
 * Errors: SAT_ERR_ARG; SAT_ERR_OVERFLOW when a column total of some pixel^p can reach 2^62
 * (H * max_pixel^p >= 2^62: always for 16-bit pixels and k = 4, above 16384 rows for k = 3);
 * SAT_ERR_WORKSPACE; SAT_ERR_HIP. */
sat_status sat_build_powers(const void *image, sat_dtype pixel_type, int64_t H, int64_t W, int64_t image_pitch,
                            int32_t k, uint64_t *const *tables, int64_t sat_pitch, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Window mean, population standard deviation, skewness and excess kurtosis of every window of
 * the valid region from the tables of pixel^1..pixel^k (n = win_h*win_w, S_p = window sum of
 * tables[p-1] by the corner lookup, exact):
 *   A = n*S2 - S1^2,  B = n^2*S3 - 3n*S1*S2 + 2*S1^3,
 *   C = n^3*S4 - 4n^2*S1*S3 + 6n*S1^2*S2 - 3*S1^4,
 * exact in 128-bit integers, each rounded to double once;
 *   mean = S1/n,  std = sqrt(A)/n,  skew = B / (A*sqrt(A)),  kurt = (C - 3*A^2) / (A*A),
 * with skew and kurt NaN where A = 0 (a constant window).
 * tables: HOST array of k device pointers (H x W, pitch sat_pitch); pixel_type (SAT_U8 or
 * SAT_U16) bounds the pixels for the overflow checks.  Outputs: device doubles, out_h rows of
 * out_pitch >= out_w, each may be NULL but not all; mean needs k >= 1, std 2, skew 3, kurt 4.
 * Errors: SAT_ERR_ARG; SAT_ERR_WINDOW; SAT_ERR_OVERFLOW when a window sum of pixel^p could reach
 * 2^64 or a numerator 2^127 (for 16-bit pixels, skewness needs n <= 65536); SAT_ERR_HIP. */
sat_status window_moments(const uint64_t *const *tables, int32_t k, sat_dtype pixel_type, int64_t H, int64_t W,
                          int64_t sat_pitch, int64_t win_h, int64_t win_w, int64_t stride, double *mean_out,
                          double *std_out, double *skew_out, double *kurt_out, int64_t out_pitch, void *stream);

/* Build and tuning introspection: number of compiled kernel variants of kind 0 (table build)
 * or 1 (window gather), the name of variant i, and the variant a later call on this thread
 * will use (-1 restores the built-in choice).  Kind 2 sets the strip height (rows, 1..1024) of
 * the batched builds on this thread, capped at the variant's own height and used only by
 * variants that take shorter strips (-1 restores the variant's height; sat_batch_workspace_bytes
 * follows it).  Kind 3 (tests only) sets a nonzero seed on this thread that makes later builds
 * sleep a pseudo-random time before every lookback publication, to perturb the order in which
 * strips finish; 0 turns it off.  Kind 4 sets the number of column segments (1..8; 0 restores
 * the built-in choice) that later helper-wave builds of one image of at most 32768 rows on this
 * thread split each strip into, each segment a separate work item (capped at one per block).
 * Results are unchanged.  Used by the tile-shape tuner and the tests. */
int32_t sat_variant_count(int32_t kind);
const char *sat_variant_name(int32_t kind, int32_t index);
sat_status sat_force_variant(int32_t kind, int32_t index);

/* 1 if variant `index` of `kind` runs on images of pixel_type (with_sq != 0: with the squared
 * table), else 0.  Gather variants run on every table; a build variant whose workgroup state
 * does not fit the 160 KiB of LDS for that pixel type is not compiled for it, and a build forced
 * to it fails with SAT_ERR_ARG.  0 for an out-of-range kind, index or pixel type.  Needs no
 * device. */
int32_t sat_variant_supported(int32_t kind, int32_t index, sat_dtype pixel_type, int32_t with_sq);

#ifdef __cplusplus
}
#endif

#endif /* SAT_H */
