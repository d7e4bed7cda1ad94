// sat_internal.h -- descriptors and launchers shared by the C-ABI front end and the kernels.
// Internal to libsat.so; the public interface is include/sat.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace satk {

// ---------------------------------------------------------------- table build

// One image to build.  All pointers are device pointers; pitches are in elements.
struct BuildDesc {
    const void *img;
    uint64_t *S;          // table of pixels
    uint64_t *Q;          // table of squared pixels, or nullptr
    uint64_t *T3, *T4;    // power builds: tables of pixel^3 and pixel^4, or nullptr
    const uint64_t *carry, *carry_q;   // band builds: column totals of the rows above the image
                                       // (W words each), or nullptr (no rows above)
    uint64_t *total, *total_q;         // band builds: column totals through the image's last row
                                       // including the carry (W words each), or nullptr
    int64_t H, W, ipitch, spitch;
    int64_t Wp;           // state row length: nblocks * block width
    int64_t state_off;    // first lookback word of this image in the state array (S part)
    int64_t state_q_off;  // first lookback word of the squared table's state (Q part)
    int64_t first_item;   // first work item (strip) of this image in the batch
    int32_t nstrips, nblocks;
    int32_t strip_h;      // rows per strip (<= the variant's strip height; chosen to balance rounds)
    int32_t wave_rows;    // rows per wave: ceil(strip_h / waves)
    int32_t img_vb;       // widest aligned load (16, 8 or 4 bytes) every image row start allows;
                          // -4: rows not 4-byte aligned (unaligned 4-byte loads, no LDS DMA)
    int32_t sat_vec;      // 1: table rows allow 16-byte vector stores
    uint32_t stress;      // nonzero (tests only): seed of pseudo-random delays before every lookback
                          // publish and fused ready count, to perturb the order strips finish in
    uint32_t narrow;      // 1: the lookback keeps 32-bit state words (no squared table and every
                          // column total, carry included, below 2^30); the same for every image
                          // of a launch, and only for variants whose strips run the lookback
    int32_t nseg;         // column segments per strip (helper-wave builds of one image; else 1):
                          // work item i is strip i / nseg, segment i % nseg
    int32_t seg_blocks;   // blocks per segment (nblocks when nseg == 1)
    const uint64_t *seg_pre, *seg_pre_q;   // nseg > 1: for segment k >= 1, H + 1 words from
                          // (k - 1) * (H + 1): word y + 1 is the table value at row y, column
                          // k * seg_blocks * block width - 1, word 0 the carry's part of it (the
                          // rows above a band); squares likewise
};

// Workspace layout: 256-byte control header, then the lookback state.
struct BuildCtrl {
    unsigned long long ticket;   // next work item
    unsigned int fault;          // bit 0: a lookback wait hit its spin bound; bit 1: a carried
                                 // column total reached 2^62 (band builds); bit 2: a statistics
                                 // item's wait for its image's tables hit its spin bound (fused)
    unsigned int pad0;
    BuildDesc one;               // descriptor of a single-image build (written by the clear kernel)
    unsigned char pad[256 - 16 - sizeof(BuildDesc)];
};
static_assert(sizeof(BuildCtrl) == 256, "control header is 256 bytes");

// MODE_HELPER: helper wave stages tiles and forms column sums and lookback one block ahead (one
// barrier per block, two tile buffers).  MODE_HELPER3: the compute waves form their own column
// sums and the helper runs the lookback of block b+1 while they compute block b (two barriers
// per block, three tile buffers): more LDS, shorter helper path per block.
enum BuildMode { MODE_LOOKBACK = 0, MODE_REDUCE_SCAN = 1, MODE_HELPER = 2, MODE_HELPER3 = 3 };

struct BuildVariant {
    const char *name;
    int px;       // pixels per lane along a row
    int rw;       // rows per wave
    int nw;       // waves per workgroup
    int mode;     // BuildMode
    int win;      // strips read this many lookback words per round trip (0: totals from a pre-pass)
    int th() const { return rw * nw; }       // strip height
    int bw() const { return 64 * px; }        // block width
    // The strips run the decoupled lookback (and may keep 32-bit state words, BuildDesc::narrow).
    bool lookback() const { return mode != MODE_REDUCE_SCAN && win > 0; }
};

int build_variant_count();
const BuildVariant &build_variant(int v);
// Workgroups of variant v that can be resident on the current device at once (pixel type, squares).
int build_variant_capacity(int v, int bpp, bool sq);
// 1 if variant v accepts a strip height below its maximum (strip_h / wave_rows at run time).
int build_variant_adaptive(int v);

// Enqueue the whole build (state clear + kernels) of n images sharing pixel type and squared
// flag.  `dev_descs` is a device copy of `descs` when n > 1 (nullptr when n == 1: the single
// descriptor is passed by value).  Returns the HIP error of the first failing launch.
hipError_t launch_build(int variant, int bpp, bool sq, const BuildDesc *descs, int n,
                        const BuildDesc *dev_descs, int64_t total_items, void *workspace,
                        int64_t state_words, hipStream_t stream);

// The library's own device scratch for callers that cannot allocate (sat_build_noalloc): a
// fixed array in the code object, one copy per device.  noalloc_scratch returns the address of
// the copy on the device `stream` belongs to (the current device for the null stream), looked up
// once per device with that device current and kept; it allocates nothing.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
hipError_t noalloc_scratch(hipStream_t stream, void **ptr);

// Copy `bytes` (a multiple of 8) of host data to the 8-byte aligned device address `dst`, in
// stream order, by kernels that take the data as by-value arguments: the host buffer may be
// released as soon as the call returns, and nothing is staged through pageable memory.
hipError_t upload_words(const void *src, size_t bytes, void *dst, hipStream_t stream);

// Tables of pixel^1..pixel^np of one image (S, Q, T3, T4 of the descriptor) in one pass: the
// helper-wave build with np lookback planes of nstrips * Wp words each (state_off: the first).
constexpr int kPowBlockW = 256;   // block width (columns) of the power build
constexpr int kPowStripH = 64;    // its largest strip height
int power_build_capacity(int bpp, int np);
hipError_t launch_build_powers(int bpp, int np, const BuildDesc &d, void *workspace, int64_t state_words,
                               hipStream_t stream);

// out = carry + column totals of an H x W image (pixels of bpp bytes, pitch in elements), and
// out_q = carry_q + totals of its squares when out_q is non-null.  carry / carry_q may be null
// (zero) or equal to out / out_q.  vec16: the image's rows start 16-byte aligned.
hipError_t launch_column_totals(int bpp, const void *img, int64_t H, int64_t W, int64_t pitch, int vec16,
                                const uint64_t *carry, const uint64_t *carry_q, uint64_t *out, uint64_t *out_q,
                                hipStream_t stream);

// ---------------------------------------------------------------- window gathers

struct GatherDesc {
    const uint64_t *S;
    const uint64_t *Q;       // mean/std only
    int64_t spitch;
    int64_t oh, ow;
    int64_t win_h, win_w, stride;
    void *out;               // window sums (u32 or u64), may be nullptr for mean/std
    double *mean;
    double *stdv;
    int64_t opitch;
    int64_t chunks;          // column chunks per output row
    int64_t first_item;      // batched: first work item of this image
    int64_t q;               // chain gathers: output rows between two reads of one table row
    int64_t seg;             // chain gathers: chain positions per work item
};

// Window moments from tables of pixel powers: up to four tables, any subset of the outputs.
struct MomentDesc {
    const uint64_t *T[4];    // tables of pixel^1 .. pixel^order
    int64_t spitch;
    int64_t oh, ow;
    int64_t win_h, win_w, stride;
    double *mean, *stdv, *skew, *kurt;   // outputs, nullptr where not wanted
    int64_t opitch;
    int64_t chunks;          // column chunks per output row (filled by the launcher)
};
// order: number of tables read (1 mean, 2 std, 3 skewness, 4 excess kurtosis).  variant: a
// gather variant; chain variants walk chains where the window height is a multiple of the stride.
hipError_t launch_window_moments(int variant, int order, MomentDesc d, hipStream_t stream);

int gather_variant_count();
const char *gather_variant_name(int v);

// Window sums of one window (variant: a gather variant; chain variants fall back to the row-pair
// kernel when the window height is not a multiple of the stride).
hipError_t launch_window_sum(int variant, const GatherDesc &d, bool out64, hipStream_t stream);
// Window sums of n <= 8 windows of one table, sharing table reads where the windows allow.
hipError_t launch_window_sum_multi(int variant, const GatherDesc *d, int n, bool out64, hipStream_t stream);
// Mean/std of one image (n == 1, dev_descs == nullptr) or of a batch: `descs` (host) and
// `dev_descs` (device copy made by the caller after this plans them) hold one descriptor per
// image; plan_mean_std fills the work split of every descriptor and returns the total items.
int64_t plan_mean_std(int variant, GatherDesc *descs, int n);
hipError_t launch_mean_std(int variant, const GatherDesc *descs, int n, const GatherDesc *dev_descs,
                           int64_t total_items, hipStream_t stream);
// Outputs per thread (1, 2 or 4) of the chain-walk mean/std items of gather variant `variant`.
int mean_std_chain_v(int variant, int64_t stride);

// Batched tables of pixels and squares and the window mean/std of every image in ONE persistent
// launch (build variant `variant`, one of those fused_build_variant accepts; `v` the chain
// outputs per thread).  bdescs / dev_bdescs: one build descriptor per image (host / device copy),
// build_items strips in all; gdescs: the images' chain mean/std descriptors (planned by
// plan_mean_std, q > 0), gather_items items in all, device copy dev_gdescs.  ready: n counters
// inside the cleared state words (the launch zeroes them with the lookback state).
bool fused_build_variant(int variant);
// Column segments of the helper-wave build: at most kMaxSeg per strip, each at least
// kMinSegBlocks blocks wide (built-in choice), for images of at most kSegMaxRows rows.  The pre-pass writes, after the lookback state, per-row totals of
// the segments and the boundary columns of the table (seg_pre) that let a segment start mid-row.
constexpr int kMaxSeg = 8;
constexpr int kMinSegBlocks = 2;
constexpr int64_t kSegMaxRows = 32768;
// Bytes of the pre-pass area for an H-row image (squares: twice).
inline size_t seg_area_bytes(int64_t H, bool sq) {
    return static_cast<size_t>(kMaxSeg - 1) * static_cast<size_t>(2 * H + 1) * 8 * (sq ? 2 : 1);
}
// Enqueue the pre-pass of a segmented build (d.nseg > 1): sums (nseg - 1) * H words (and as many
// for squares) of scratch, then d.seg_pre / d.seg_pre_q.
hipError_t launch_seg_prepass(int bpp, bool sq, const BuildDesc &d, uint64_t *sums, uint64_t *sums_q,
                              hipStream_t stream);

// Host-to-device copy by a kernel reading pinned host memory at its device address src_dev.
hipError_t launch_upload(const void *src_dev, void *dst, size_t nbytes, hipStream_t stream);

hipError_t launch_fused(int variant, int bpp, int v, const BuildDesc *bdescs, int n, const BuildDesc *dev_bdescs,
                        int64_t build_items, const GatherDesc *dev_gdescs, int64_t gather_items, void *workspace,
                        int64_t state_words, unsigned int *ready, hipStream_t stream);

}  // namespace satk
