// sat_api.cpp -- the C ABI of libsat.so (declared in include/sat.h): argument validation, shape
// and workspace arithmetic, kernel-variant choice and launch.  Validation is complete and
// synchronous before the first HIP call, so every error path is testable without a GPU.
#include "sat.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sat_internal.h"

namespace {

thread_local std::string g_err = "no error";
// build variant, gather variant, batch strip height, lookback stress seed (0: off), column
// segments of a helper-wave build (0: the built-in choice)
thread_local int g_force[5] = {-1, -1, -1, 0, 0};

sat_status fail(sat_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

sat_status ok() {
    g_err = "no error";
    return SAT_OK;
}

sat_status hip_fail(hipError_t e, const char *what) {
    return fail(SAT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr int64_t kMaxDim = (1ll << 31) - 1;
constexpr int64_t kMaxRowElems = 1ll << 24;   // 32-bit buffer offsets over a strip of rows stay in range

int bytes_of(sat_dtype t) {
    switch (t) {
        case SAT_U8: return 1;
        case SAT_U16: return 2;
        case SAT_U32: return 4;
        case SAT_U64: return 8;
        case SAT_F64: return 8;
    }
    return 0;
}

uint64_t max_pixel(sat_dtype t) {
    switch (t) {
        case SAT_U8: return 255u;
        case SAT_U16: return 65535u;
        case SAT_U32: return 4294967295u;
        default: return 0;
    }
}

// Byte extent [p, p + bytes) of a row-major 2-D array.
struct Span {
    uintptr_t lo = 0, hi = 0;
};
Span span(const void *p, int64_t rows, int64_t pitch, int64_t cols, int elem) {
    Span s;
    if (!p) return s;
    s.lo = reinterpret_cast<uintptr_t>(p);
    s.hi = s.lo + static_cast<uintptr_t>(((rows - 1) * pitch + cols) * elem);
    return s;
}
bool overlap(const Span &a, const Span &b) {
    return a.lo != a.hi && b.lo != b.hi && a.lo < b.hi && b.lo < a.hi;
}

sat_status check_dims(int64_t H, int64_t W, const char *who) {
    if (H < 1 || W < 1) return fail(SAT_ERR_ARG, "%s: image size %lld x %lld must be at least 1 x 1", who,
                                    (long long)H, (long long)W);
    if (H > kMaxDim || W > kMaxRowElems)
        return fail(SAT_ERR_ARG, "%s: image height above 2^31-1 or width above 2^24", who);
    return SAT_OK;
}

sat_status check_pitch(int64_t pitch, int64_t W, int64_t H, int elem, const char *who, const char *what) {
    if (pitch < W) return fail(SAT_ERR_ARG, "%s: %s pitch %lld is below the width %lld", who, what,
                               (long long)pitch, (long long)W);
    // Buffer resources span at most 64 rows of a strip (one wave's 16 rows for stores), so 32-bit
    // byte offsets stay in range for pitches up to 2^24 elements; rows * pitch * elem stays far
    // from int64 overflow
    if (pitch > kMaxRowElems || H > ((1ll << 60) / (pitch * elem)))
        return fail(SAT_ERR_ARG, "%s: %s pitch above 2^24 elements or extent too large", who, what);
    return SAT_OK;
}

// ------------------------------------------------------------------ build planning

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

// Gather variant of a call on this thread: the forced one, else the automatic chain walk (the
// LDS-staged kernel where it applies; chain and row-pair kernels otherwise, chosen per launch).
int gather_variant() {
    const int v = g_force[1];
    return v >= 0 && v < satk::gather_variant_count() ? v : 0;
}

// Variants the built-in choice uses (indices into the compiled table).
constexpr int kVarNtPx8 = 8;        // lookback, non-temporal stores, 8 pixels per lane
constexpr int kVarNtPx4 = 9;        // lookback, non-temporal stores, 4 pixels per lane
constexpr int kVarHelperPx4 = 10;   // helper wave (DMA tiles, lookback a block ahead), 4 pixels per lane
constexpr int kVarHelperPx8 = 11;   // helper wave, 8 pixels per lane, 48-row strips
constexpr int kVarShort = 2;        // lookback, 32-row strips
constexpr int kVarHelper3Px4 = 12;  // helper wave, lookback only (column sums on the compute waves), 4 pixels per lane
constexpr int kVarHelper3Px8 = 13;  // the same, 8 pixels per lane, 48-row strips

bool helper_variant(int v) {
    return v == kVarHelperPx4 || v == kVarHelperPx8 || v == kVarHelper3Px4 || v == kVarHelper3Px8;
}

// Row alignment class of an image: 16 when every row start allows 16-byte loads, 4 when it
// allows 4-byte loads, else 1.  The helper wave's LDS DMA needs 4; below 16 it moves a dword
// per lane and instruction, a quarter of what it moves with 16-byte rows.
int row_align(const void *image, int64_t ipitch, int bpp) {
    const uintptr_t a = reinterpret_cast<uintptr_t>(image);
    const int64_t pb = ipitch * bpp;
    if (a % 16 == 0 && pb % 16 == 0) return 16;
    if (a % 4 == 0 && pb % 4 == 0) return 4;
    return 1;
}

// Strip height of at most th rows for one image: th unless the strips would not fit the `cap`
// resident workgroups in whole rounds; then the height that spreads them evenly over the fewest
// rounds (a last round with few strips costs a whole strip sweep).
int balanced_strip_h(int64_t H, int th, int64_t cap) {
    const int64_t strips = (H + th - 1) / th;
    if (cap < 1 || strips <= cap) return th;
    const int64_t rounds = (strips + cap - 1) / cap;
    int64_t h = (H + rounds * cap - 1) / (rounds * cap);
    if (h < 1) h = 1;
    return static_cast<int>(h < th ? h : th);
}

// Plan of the helper-wave build of one image with 16-byte aligned rows.  Where its strips are no
// more than the compute units, each workgroup sweeps the width alone, block by block, and blocks
// of eight pixels per lane (512 columns) take half the steps of blocks of four.  So: eight pixels
// per lane at 48-row strips, or 24-row strips where 48-row ones would leave three quarters of the
// CUs idle.  Where 48-row strips outnumber the CUs but 64-row strips
// do not, one 64-row strip per CU at four pixels per lane beats two 48-row strips on some CUs.
// Taller images take eight pixels per lane at 48 rows, balanced over rounds of resident
// workgroups once they fill one.  Images narrower than eight 512-column blocks, and 16-bit images
// with squares (whose eight-pixel tiles do not fit the LDS), take four pixels per lane at the
// least of 32, 48 or 64 rows that gives at most one strip per CU.
// Measured (ms per build, previous choice -> this one, bit-exact throughout): 8750 x 85000 u8
// 2.43 -> 1.79; 17500 x 85000 u8 4.56 -> 3.39; 20000^2 u8 1.28 -> 1.00; 16000^2 u8 0.81 -> 0.63;
// 2000 x 16000 u8 0.30 -> 0.25; 8192^2 u16 0.24 -> 0.21; 12000^2 u16 with squares 0.83 -> 0.72.
struct BuildPlan {
    int v;
    int strip_h;
};

// Images of at most this many rows split helper-wave strips into column segments (choose_segments).
constexpr int64_t kSegAutoRows = 4096;

int helper_strip_h(int v, int64_t H, int bpp, bool sq) {
    const int64_t ncu = device_cus();
    const int64_t cap = satk::build_variant_capacity(v, bpp, sq);
    const int th = satk::build_variant(v).th();
    if (v == kVarHelper3Px8 && H > kSegAutoRows && (H + th - 1) / th <= ncu) {
        // One round: the shortest strips (at least half a tile) that still fit on the CUs.
        // Measured (ms per build): 4375 x 85000 u8 1.06-1.10 at 48 rows -> 0.93-0.98 at 24; 8750
        // x 85000 u8 1.465-1.475 at 48 rows, 1.456-1.463 at 36-44, 1.73-1.88 at 24-32 (two
        // rounds).  Shorter images split their strips into column segments instead (below), and
        // there 24-row strips lost: 3200 x 4100 u8 0.091 -> 0.097.
        const int64_t h = (H + ncu - 1) / ncu;
        return static_cast<int>(h < th / 2 ? th / 2 : h);
    }
    if (v == kVarHelperPx8 || v == kVarHelper3Px8) {
        if (4 * ((H + th - 1) / th) <= ncu) return th / 2;
        return balanced_strip_h(H, th, cap);
    }
    for (int h = th / 2; h < th; h += th / 4)
        if ((H + h - 1) / h <= ncu) return h;
    return balanced_strip_h(H, th, cap);
}

BuildPlan helper_plan(int64_t H, int64_t W, int bpp, bool sq) {
    const int64_t ncu = device_cus();
    int v = kVarHelperPx4;
    if (W >= 8 * satk::build_variant(kVarHelperPx8).bw() && satk::build_variant_capacity(kVarHelperPx8, bpp, sq) > 0) {
        const int64_t n48 = (H + 47) / 48, n64 = (H + 63) / 64;
        v = (n48 > ncu && n64 <= ncu) ? kVarHelperPx4 : kVarHelperPx8;
    }
    // The three-stage helper pipeline (column sums on the compute waves, the helper's lookback
    // overlapping their block and the DMA of the tile after next) shortens each block where the
    // helper's path sets the pace, at the cost of a third tile buffer (one workgroup per CU for
    // 8-bit 512-column tiles).  Measured (ms, two-stage -> three-stage, one GPU, bit-exact):
    // 8192^2 u16 with squares 0.346 -> 0.311, 12000^2 0.712 -> 0.682, 16000^2 u8 0.594 -> 0.552,
    // 2000 x 16000 u8 0.255 -> 0.227, 20000^2 u8 0.969 -> 0.928.  Wider rows gained once the
    // helper's barrier after the DMA stopped waiting for it: 85000-pixel rows, 8750 rows 1.52 ->
    // 1.27, 17500 rows 3.13 -> 2.68, 4375 rows 1.26 -> 1.07; 8192 x 40000 u16 with squares 1.52 ->
    // 1.22.  Tall wide images, where the two-stage pipeline keeps two workgroups on every CU over
    // several rounds, stay with it: 70000 x 85000 tied alone (10.99 vs 10.95) and was 2-8 % slower
    // in three stages right after a gather.
    const int v3 = v == kVarHelperPx4 ? kVarHelper3Px4 : kVarHelper3Px8;
    const bool tall_wide = W > 32768 && (H + 47) / 48 > 2 * ncu;
    if (!tall_wide && satk::build_variant_capacity(v3, bpp, sq) > 0) v = v3;
    return {v, helper_strip_h(v, H, bpp, sq)};
}

// align: the least row alignment class over the images (row_align).
int choose_build_variant(int64_t total_rows, int64_t W, int n_images, int bpp, bool sq, int align) {
    const int v = g_force[0];
    if (v >= 0) return v;
    // Each work item is one strip swept across the full width, so the number of strips is the
    // parallelism.  Measured choices (ms per build; 2000 x 16000 to 70000 x 85000):
    //  - one image with 16-byte aligned rows: the helper wave, which stages tiles by 16-byte DMA
    //    and runs the lookback one block ahead of the compute waves (helper_plan below);
    //  - otherwise, with two 64-row strips per CU or more: lookback with non-temporal table
    //    stores (the table is read back only after it has left the caches), eight pixels per
    //    lane for 8-bit images without squares (elsewhere that variant holds one wave per SIMD);
    //  - with fewer strips each workgroup's own latency decides: the helper wave when rows allow
    //    its DMA, else 32-row strips.
    if (n_images == 1 && align == 16) return helper_plan(total_rows, W, bpp, sq).v;
    const int64_t want = 2ll * device_cus();
    const int64_t strips64 = (total_rows + 63 * n_images) / 64;
    if (strips64 >= want) return (bpp == 1 && !sq) ? kVarNtPx8 : kVarNtPx4;
    return align >= 4 ? kVarHelperPx4 : kVarShort;
}

// Strip height for variant v on one image of H rows with row alignment class `align`.
int choose_strip_h(int v, int64_t H, int bpp, bool sq, int align) {
    const satk::BuildVariant &var = satk::build_variant(v);
    if (!satk::build_variant_adaptive(v)) return var.th();
    if (align == 16 && helper_variant(v)) return helper_strip_h(v, H, bpp, sq);
    const int64_t cap = satk::build_variant_capacity(v, bpp, sq);
    // Few strips (at most half the resident workgroups): 32-row strips, twice as many, all in one
    // round.  Measured at 4096-12000 rows: 3-11 % faster than 64-row strips; 16- and 24-row strips
    // were slower, and so were 32-row strips once 64-row ones filled a round.
    if (var.th() >= 64 && cap > 0 && 2 * ((H + var.th() - 1) / var.th()) <= cap) return var.th() / 2;
    return balanced_strip_h(H, var.th(), cap);
}

// Lower bound of the strip height any variant may pick (for workspace sizing): with at least two
// rounds the balanced height exceeds half the full height, and images with few strips take half.
int min_strip_h(const satk::BuildVariant &v, int adaptive) {
    return adaptive ? (v.th() + 1) / 2 : v.th();
}

// A forced variant must exist and have an instantiation for this pixel type (its workgroup state
// fits the LDS).
sat_status check_build_variant(int v, int bpp, bool sq, const char *who) {
    if (v < 0 || v >= satk::build_variant_count()) return fail(SAT_ERR_ARG, "%s: forced variant out of range", who);
    if (satk::build_variant_capacity(v, bpp, sq) < 1)
        return fail(SAT_ERR_ARG, "%s: build variant %s does not fit the LDS for %d-byte pixels%s", who,
                    satk::build_variant(v).name, bpp, sq ? " with squares" : "");
    return SAT_OK;
}

// Column segments per strip of a helper-wave build of one image (1: each strip sweeps whole rows).
// The strips are the build's parallelism.  On images of at most kSegAutoRows rows each strip is
// split into segments of at least kMinSegBlocks blocks that separate workgroups build (a
// pre-pass supplies the row totals left of each segment), about two rounds of resident
// workgroups' worth.  Measured with the helper pipelines (ms, whole rows -> built-in segments):
// 8-bit 2000 x 4000 0.096 -> 0.079, 2000 x 16000 0.218 -> 0.131, 3000 x 12000 0.207 -> 0.147,
// 4096 x 16000 0.262 -> 0.170-0.186, 2048 x 32768 0.336 -> 0.173, 1500 x 85000 0.818 -> 0.292;
// 16-bit with squares 4096 x 8192 0.250 -> 0.178.  Taller images take three segments where
// their strips are at their least height (below); elsewhere they gained nothing or lost.  A
// forced count (sat_force_variant kind 4) applies up to kSegMaxRows rows, for which the
// workspace reserves the pre-pass area.
int choose_segments(int v, const satk::BuildDesc &d, int bpp, bool sq) {
    const satk::BuildVariant &var = satk::build_variant(v);
    if ((var.mode != satk::MODE_HELPER && var.mode != satk::MODE_HELPER3) || !var.lookback() ||
        d.H > satk::kSegMaxRows)
        return 1;
    const int forced = g_force[4];
    // Taller images are split only where the plan's strips are at their least height (half a
    // tile): the image is then too short to give every CU a strip of a useful height.  Measured
    // on one GPU (ms, whole rows -> 3 segments): 6000^2 u16 with squares 0.252 -> 0.219, 8192^2
    // 0.316 -> 0.308, 7000 x 16000 0.558 -> 0.539; u8 at 24-row strips 5000 x 12000 0.237 ->
    // 0.204, 6000 x 20000 0.336 -> 0.296, 6000 x 40000 0.579 -> 0.518.  Taller strips lost:
    // 12000^2 0.66 -> 0.78, 16000^2 0.48 -> 0.57, 8750 x 85000 1.48 -> 1.56, 8192 x 85000 at
    // 32-row strips 1.39 -> 1.44.
    const bool tall = d.H > kSegAutoRows;
    if (forced <= 0 && tall && 2 * d.strip_h > var.th()) return 1;
    const int64_t most = std::min<int64_t>(satk::kMaxSeg, forced > 0 ? d.nblocks : d.nblocks / satk::kMinSegBlocks);
    if (most < 2) return 1;
    int64_t want = forced;
    if (forced <= 0) {
        const int64_t cap = satk::build_variant_capacity(v, bpp, sq);
        want = tall ? 3 : (cap > 0 ? std::max<int64_t>(2, 2 * cap / d.nstrips) : 1);
    }
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, most)));
}

int64_t state_words_for(const satk::BuildVariant &v, int64_t H, int64_t W, bool sq, int strip_h) {
    const int64_t strips = (H + strip_h - 1) / strip_h;
    const int64_t wp = (W + v.bw() - 1) / v.bw() * v.bw();
    int64_t words = strips * wp * (sq ? 2 : 1);
    return (words + 1) & ~1ll;
}

// Lookback words a build of one image with variant v may need (any strip height it may pick).
int64_t build_state_words(int v, int64_t H, int64_t W, bool sq) {
    const satk::BuildVariant &var = satk::build_variant(v);
    return state_words_for(var, H, W, sq, min_strip_h(var, satk::build_variant_adaptive(v)));
}

// Lookback words a build of one H x W image needs whichever row alignment it turns out to have
// (the built-in choice depends on it).
int64_t build_state_words_any(int64_t H, int64_t W, int bpp, bool sq) {
    int64_t words = 0;
    for (int align : {16, 4, 1}) {
        const int64_t w = build_state_words(choose_build_variant(H, W, 1, bpp, sq, align), H, W, sq);
        if (w > words) words = w;
    }
    return words;
}

// Offset of the segment pre-pass area in a single-image build's workspace: after the largest
// lookback state any variant may use, on a 256-byte boundary.
size_t seg_area_offset(int64_t H, int64_t W, int bpp, bool sq) {
    const size_t end = sizeof(satk::BuildCtrl) + 8 * static_cast<size_t>(build_state_words_any(H, W, bpp, sq));
    return (end + 255) / 256 * 256;
}

void fill_desc(satk::BuildDesc &d, const satk::BuildVariant &v, const void *image, int bpp, int64_t H,
               int64_t W, int64_t ipitch, uint64_t *sat, uint64_t *sat_sq, int64_t spitch, int strip_h) {
    d.img = image;
    d.S = sat;
    d.Q = sat_sq;
    d.H = H;
    d.W = W;
    d.ipitch = ipitch;
    d.spitch = spitch;
    d.strip_h = strip_h;
    d.wave_rows = (strip_h + v.nw - 1) / v.nw;
    d.nstrips = static_cast<int32_t>((H + strip_h - 1) / strip_h);
    d.nblocks = static_cast<int32_t>((W + v.bw() - 1) / v.bw());
    d.Wp = static_cast<int64_t>(d.nblocks) * v.bw();
    const uintptr_t ia = reinterpret_cast<uintptr_t>(image);
    const int64_t row_bytes = ipitch * bpp;
    // Rows whose starts are not 4-byte aligned still take 4-byte loads into registers (the
    // hardware serves unaligned dword buffer loads); only the LDS DMA path needs alignment.
    d.img_vb = -4;
    for (int vb = 16; vb >= 4; vb /= 2)
        if (ia % vb == 0 && row_bytes % vb == 0 && vb <= v.bw() * bpp) {
            d.img_vb = vb;
            break;
        }
    const bool sa = reinterpret_cast<uintptr_t>(sat) % 16 == 0 &&
                    (!sat_sq || reinterpret_cast<uintptr_t>(sat_sq) % 16 == 0);
    d.sat_vec = (sa && spitch % 2 == 0) ? 1 : 0;
    d.stress = static_cast<uint32_t>(g_force[3]);
    d.nseg = 1;
    d.seg_blocks = d.nblocks;
}

// Whether a build of `rows` rows in all (rows above included) may keep 32-bit lookback state
// words: a variant whose strips run the lookback, no squared table, and every column total below
// 2^30.
bool narrow_state(const satk::BuildVariant &v, bool sq, int64_t rows, int bpp) {
    const uint64_t maxpix = bpp == 1 ? 255u : 65535u;
    return v.lookback() && !sq && rows >= 0 && static_cast<uint64_t>(rows) * maxpix < (uint64_t(1) << 30);
}

sat_status validate_build_item(const void *image, sat_dtype pixel_type, int64_t H, int64_t W, int64_t ipitch,
                               const uint64_t *sat, const uint64_t *sat_sq, int64_t spitch, const char *who) {
    if (!image || !sat) return fail(SAT_ERR_ARG, "%s: image and sat must be non-NULL", who);
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16)
        return fail(SAT_ERR_ARG, "%s: pixel_type must be SAT_U8 or SAT_U16", who);
    sat_status st = check_dims(H, W, who);
    if (st) return st;
    const int bpp = bytes_of(pixel_type);
    if ((st = check_pitch(ipitch, W, H, bpp, who, "image"))) return st;
    if ((st = check_pitch(spitch, W, H, 8, who, "table"))) return st;
    if (sat == sat_sq) return fail(SAT_ERR_ARG, "%s: sat and sat_sq must be distinct", who);
    const unsigned __int128 m = max_pixel(pixel_type);
    const unsigned __int128 col = static_cast<unsigned __int128>(H) * (sat_sq ? m * m : m);
    if (col >= (static_cast<unsigned __int128>(1) << 62))
        return fail(SAT_ERR_OVERFLOW, "%s: %lld rows are too many for exact 62-bit column totals", who,
                    (long long)H);
    const Span si = span(image, H, ipitch, W, bpp), ss = span(sat, H, spitch, W, 8),
               sq = span(sat_sq, H, spitch, W, 8);
    if (overlap(si, ss) || overlap(si, sq) || overlap(ss, sq))
        return fail(SAT_ERR_ARG, "%s: image, sat and sat_sq must not overlap", who);
    return SAT_OK;
}

// ------------------------------------------------------------------ gather planning

sat_status validate_window(const uint64_t *sat, int64_t H, int64_t W, int64_t spitch, int64_t win_h,
                           int64_t win_w, int64_t stride, const char *who, int64_t *oh, int64_t *ow) {
    if (!sat) return fail(SAT_ERR_ARG, "%s: sat must be non-NULL", who);
    sat_status st = check_dims(H, W, who);
    if (st) return st;
    if ((st = check_pitch(spitch, W, H, 8, who, "table"))) return st;
    if (win_h < 1 || win_w < 1 || stride < 1)
        return fail(SAT_ERR_ARG, "%s: window %lld x %lld and stride %lld must be >= 1", who, (long long)win_h,
                    (long long)win_w, (long long)stride);
    if (win_h > H || win_w > W)
        return fail(SAT_ERR_WINDOW, "%s: window %lld x %lld does not fit the %lld x %lld image", who,
                    (long long)win_h, (long long)win_w, (long long)H, (long long)W);
    *oh = (H - win_h) / stride + 1;
    *ow = (W - win_w) / stride + 1;
    return SAT_OK;
}

satk::GatherDesc gather_desc(const uint64_t *sat, const uint64_t *sat_sq, int64_t spitch, int64_t oh, int64_t ow,
                             int64_t win_h, int64_t win_w, int64_t stride, void *out, double *mean, double *stdv,
                             int64_t opitch) {
    satk::GatherDesc d{};
    d.S = sat;
    d.Q = sat_sq;
    d.spitch = spitch;
    d.oh = oh;
    d.ow = ow;
    d.win_h = win_h;
    d.win_w = win_w;
    d.stride = stride;
    d.out = out;
    d.mean = mean;
    d.stdv = stdv;
    d.opitch = opitch;
    return d;
}


// sat_build and sat_build_band: one image, optionally seeded with the column totals of the rows
// above it (carry, rows_above) and emitting its own column totals through its last row (total).
sat_status build_one(const void *image, sat_dtype pixel_type, int64_t H, int64_t W, int64_t image_pitch,
                     const uint64_t *carry, const uint64_t *carry_sq, int64_t rows_above, uint64_t *sat,
                     uint64_t *sat_sq, int64_t sat_pitch, uint64_t *total, uint64_t *total_sq, void *workspace,
                     size_t workspace_bytes, void *stream, const char *who) {
    sat_status st = validate_build_item(image, pixel_type, H, W, image_pitch, sat, sat_sq, sat_pitch, who);
    if (st) return st;
    const bool sq = sat_sq != nullptr;
    const int bpp = bytes_of(pixel_type);
    if (rows_above < 0 || rows_above > kMaxDim)
        return fail(SAT_ERR_ARG, "%s: rows_above %lld out of range", who, (long long)rows_above);
    if (rows_above > 0 && !carry) return fail(SAT_ERR_ARG, "%s: rows_above > 0 needs a carry", who);
    if (carry && sq && !carry_sq) return fail(SAT_ERR_ARG, "%s: a carry with sat_sq needs carry_sq", who);
    if (carry_sq && (!carry || !sq)) return fail(SAT_ERR_ARG, "%s: carry_sq needs carry and sat_sq", who);
    if (total_sq && !sq) return fail(SAT_ERR_ARG, "%s: total_sq_out needs sat_sq", who);
    {
        // every column total of the band, carry included, must stay below 2^62
        const unsigned __int128 m = max_pixel(pixel_type);
        const unsigned __int128 col = static_cast<unsigned __int128>(rows_above + H) * (sq ? m * m : m);
        if (col >= (static_cast<unsigned __int128>(1) << 62))
            return fail(SAT_ERR_OVERFLOW, "%s: %lld rows above and %lld rows are too many for exact 62-bit column "
                        "totals", who, (long long)rows_above, (long long)H);
    }
    const Span si = span(image, H, image_pitch, W, bpp), ss = span(sat, H, sat_pitch, W, 8),
               sqs = span(sat_sq, H, sat_pitch, W, 8);
    const Span sc = span(carry, 1, W, W, 8), scq = span(carry_sq, 1, W, W, 8);
    const Span st_ = span(total, 1, W, W, 8), stq = span(total_sq, 1, W, W, 8);
    for (const Span *o : {&st_, &stq})
        if (overlap(*o, si) || overlap(*o, ss) || overlap(*o, sqs))
            return fail(SAT_ERR_ARG, "%s: a total output overlaps the image or a table", who);
    if (overlap(st_, stq)) return fail(SAT_ERR_ARG, "%s: total_out and total_sq_out overlap", who);
    for (const Span *c : {&sc, &scq})
        if (overlap(*c, ss) || overlap(*c, sqs)) return fail(SAT_ERR_ARG, "%s: a carry overlaps a table", who);
    // a carry is either its own total output (in place) or apart from both totals
    if ((carry != total && (overlap(sc, st_) || overlap(sc, stq))) ||
        (carry_sq != total_sq && (overlap(scq, st_) || overlap(scq, stq))))
        return fail(SAT_ERR_ARG, "%s: a carry must equal its total output or overlap no total", who);
    if (reinterpret_cast<uintptr_t>(carry) % 8 || reinterpret_cast<uintptr_t>(carry_sq) % 8 ||
        reinterpret_cast<uintptr_t>(total) % 8 || reinterpret_cast<uintptr_t>(total_sq) % 8)
        return fail(SAT_ERR_ARG, "%s: carries and totals must be 8-byte aligned", who);
    const size_t need = sat_build_workspace_bytes(H, W, pixel_type, sq);
    if (!workspace || workspace_bytes < need)
        return fail(SAT_ERR_WORKSPACE, "%s: workspace of %zu bytes is below the %zu needed", who, workspace_bytes,
                    need);
    if (reinterpret_cast<uintptr_t>(workspace) % 16)
        return fail(SAT_ERR_ARG, "%s: workspace must be 16-byte aligned", who);
    const Span sw{reinterpret_cast<uintptr_t>(workspace), reinterpret_cast<uintptr_t>(workspace) + workspace_bytes};
    for (const Span *o : {&si, &ss, &sqs, &sc, &scq, &st_, &stq})
        if (overlap(sw, *o)) return fail(SAT_ERR_ARG, "%s: workspace overlaps an input or output", who);
    const int align = row_align(image, image_pitch, bpp);
    const int v = choose_build_variant(H, W, 1, bpp, sq, align);
    if ((st = check_build_variant(v, bpp, sq, who))) return st;
    const satk::BuildVariant &var = satk::build_variant(v);
    satk::BuildDesc d{};
    const int strip_h = choose_strip_h(v, H, bpp, sq, align);
    fill_desc(d, var, image, bpp, H, W, image_pitch, sat, sat_sq, sat_pitch, strip_h);
    d.state_off = 0;
    d.state_q_off = static_cast<int64_t>(d.nstrips) * d.Wp;
    d.first_item = 0;
    d.carry = carry;
    d.carry_q = carry_sq;
    d.total = total;
    d.total_q = total_sq;
    d.narrow = narrow_state(var, sq, rows_above + H, bpp) ? 1u : 0u;
    const int64_t words = state_words_for(var, H, W, sq, strip_h);
    const int nseg = choose_segments(v, d, bpp, sq);
    if (nseg > 1) {
        d.seg_blocks = (d.nblocks + nseg - 1) / nseg;
        d.nseg = (d.nblocks + d.seg_blocks - 1) / d.seg_blocks;
        // pre-pass area: row sums of segments 0 .. kMaxSeg - 2 (then of squares), then the
        // boundary columns (then of squares)
        const int64_t ns = (satk::kMaxSeg - 1) * H, np = (satk::kMaxSeg - 1) * (H + 1);
        uint64_t *sums = reinterpret_cast<uint64_t *>(static_cast<char *>(workspace) + seg_area_offset(H, W, bpp, sq));
        uint64_t *sums_q = sq ? sums + ns : nullptr;
        uint64_t *pre = sums + ns * (sq ? 2 : 1);
        d.seg_pre = pre;
        d.seg_pre_q = sq ? pre + np : nullptr;
        const hipError_t e = satk::launch_seg_prepass(bpp, sq, d, sums, sums_q, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return hip_fail(e, who);
    }
    hipError_t e = satk::launch_build(v, bpp, sq, &d, 1, nullptr, static_cast<int64_t>(d.nstrips) * d.nseg,
                                      workspace, words, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

}  // namespace

extern "C" {

const char *sat_last_error(void) { return g_err.c_str(); }

sat_status window_out_shape(int64_t H, int64_t W, int64_t win_h, int64_t win_w, int64_t stride, int64_t *out_h,
                            int64_t *out_w) {
    if (!out_h || !out_w) return fail(SAT_ERR_ARG, "window_out_shape: output pointers must be non-NULL");
    if (H < 1 || W < 1 || win_h < 1 || win_w < 1 || stride < 1)
        return fail(SAT_ERR_ARG, "window_out_shape: sizes and stride must be >= 1");
    if (win_h > H || win_w > W) return fail(SAT_ERR_WINDOW, "window_out_shape: window larger than image");
    *out_h = (H - win_h) / stride + 1;
    *out_w = (W - win_w) / stride + 1;
    return ok();
}

size_t sat_build_workspace_bytes(int64_t H, int64_t W, sat_dtype pixel_type, int with_sq) {
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return 0;
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16) return 0;
    const int v = choose_build_variant(H, W, 1, bytes_of(pixel_type), with_sq != 0, 16);
    if (v < 0 || v >= satk::build_variant_count()) return 0;
    const int bpp = bytes_of(pixel_type);
    if (H <= satk::kSegMaxRows) return seg_area_offset(H, W, bpp, with_sq != 0) + satk::seg_area_bytes(H, with_sq != 0);
    return sizeof(satk::BuildCtrl) + 8 * static_cast<size_t>(build_state_words_any(H, W, bpp, with_sq != 0));
}

sat_status sat_build(const void *image, sat_dtype pixel_type, int64_t H, int64_t W, int64_t image_pitch,
                     uint64_t *sat, uint64_t *sat_sq, int64_t sat_pitch, void *workspace, size_t workspace_bytes,
                     void *stream) {
    return build_one(image, pixel_type, H, W, image_pitch, nullptr, nullptr, 0, sat, sat_sq, sat_pitch, nullptr,
                     nullptr, workspace, workspace_bytes, stream, "sat_build");
}

sat_status sat_build_noalloc(const void *image, sat_dtype pixel_type, int64_t H, int64_t W, int64_t image_pitch,
                             uint64_t *sat, uint64_t *sat_sq, int64_t sat_pitch, void *stream) {
    const char *who = "sat_build_noalloc";
    sat_status st = validate_build_item(image, pixel_type, H, W, image_pitch, sat, sat_sq, sat_pitch, who);
    if (st) return st;
    const size_t need = sat_build_workspace_bytes(H, W, pixel_type, sat_sq != nullptr);
    if (need == 0 || need > satk::kNoAllocScratchBytes)
        return fail(SAT_ERR_WORKSPACE, "%s: a %lld x %lld build%s needs %zu bytes of scratch, above the library's "
                    "fixed %zu; call sat_build with a workspace", who, (long long)H, (long long)W,
                    sat_sq ? " with squares" : "", need, satk::kNoAllocScratchBytes);
    void *ws = nullptr;
    const hipError_t e = satk::noalloc_scratch(static_cast<hipStream_t>(stream), &ws);
    if (e != hipSuccess) return hip_fail(e, who);
    return build_one(image, pixel_type, H, W, image_pitch, nullptr, nullptr, 0, sat, sat_sq, sat_pitch, nullptr,
                     nullptr, ws, satk::kNoAllocScratchBytes, stream, who);
}

sat_status sat_build_band(const void *image, sat_dtype pixel_type, int64_t H, int64_t W, int64_t image_pitch,
                          const uint64_t *carry, const uint64_t *carry_sq, int64_t rows_above, uint64_t *sat,
                          uint64_t *sat_sq, int64_t sat_pitch, uint64_t *total_out, uint64_t *total_sq_out,
                          void *workspace, size_t workspace_bytes, void *stream) {
    return build_one(image, pixel_type, H, W, image_pitch, carry, carry_sq, rows_above, sat, sat_sq, sat_pitch,
                     total_out, total_sq_out, workspace, workspace_bytes, stream, "sat_build_band");
}

sat_status sat_column_totals(const void *image, sat_dtype pixel_type, int64_t H, int64_t W, int64_t image_pitch,
                             const uint64_t *carry, const uint64_t *carry_sq, uint64_t *out, uint64_t *out_sq,
                             void *stream) {
    const char *who = "sat_column_totals";
    if (!image || !out) return fail(SAT_ERR_ARG, "%s: image and out must be non-NULL", who);
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16)
        return fail(SAT_ERR_ARG, "%s: pixel_type must be SAT_U8 or SAT_U16", who);
    sat_status st = check_dims(H, W, who);
    if (st) return st;
    const int bpp = bytes_of(pixel_type);
    if ((st = check_pitch(image_pitch, W, H, bpp, who, "image"))) return st;
    if (carry_sq && !out_sq) return fail(SAT_ERR_ARG, "%s: carry_sq needs out_sq", who);
    if (out_sq && carry && !carry_sq)
        return fail(SAT_ERR_ARG, "%s: with a carry and out_sq, carry_sq must be non-NULL", who);
    const Span si = span(image, H, image_pitch, W, bpp);
    const Span so = span(out, 1, W, W, 8), soq = span(out_sq, 1, W, W, 8);
    const Span sc = span(carry, 1, W, W, 8), scq = span(carry_sq, 1, W, W, 8);
    if (overlap(si, so) || overlap(si, soq) || overlap(so, soq))
        return fail(SAT_ERR_ARG, "%s: image, out and out_sq must not overlap", who);
    // a carry is either the output itself (in place) or apart from both outputs
    if ((carry != out && (overlap(sc, so) || overlap(sc, soq))) ||
        (carry_sq != out_sq && (overlap(scq, so) || overlap(scq, soq))))
        return fail(SAT_ERR_ARG, "%s: a carry must equal its output or overlap no output", who);
    if (reinterpret_cast<uintptr_t>(out) % 8 || reinterpret_cast<uintptr_t>(out_sq) % 8 ||
        reinterpret_cast<uintptr_t>(carry) % 8 || reinterpret_cast<uintptr_t>(carry_sq) % 8)
        return fail(SAT_ERR_ARG, "%s: totals and carries must be 8-byte aligned", who);
    const int vec16 = row_align(image, image_pitch, bpp) == 16 ? 1 : 0;
    hipError_t e = satk::launch_column_totals(bpp, image, H, W, image_pitch, vec16, carry, carry_sq, out, out_sq,
                                              static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

sat_status window_sum(const uint64_t *sat, sat_dtype pixel_type, int64_t H, int64_t W, int64_t sat_pitch,
                      int64_t win_h, int64_t win_w, int64_t stride, void *out, sat_dtype out_type, int64_t out_pitch,
                      void *stream) {
    const char *who = "window_sum";
    int64_t oh = 0, ow = 0;
    sat_status st = validate_window(sat, H, W, sat_pitch, win_h, win_w, stride, who, &oh, &ow);
    if (st) return st;
    if (!out) return fail(SAT_ERR_ARG, "%s: out must be non-NULL", who);
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16 && pixel_type != SAT_U32)
        return fail(SAT_ERR_ARG, "%s: pixel_type must be SAT_U8, SAT_U16 or SAT_U32", who);
    if (out_type != SAT_U32 && out_type != SAT_U64)
        return fail(SAT_ERR_ARG, "%s: out_type must be SAT_U32 or SAT_U64", who);
    if (out_type == SAT_U32) {
        const unsigned __int128 worst = static_cast<unsigned __int128>(win_h) * static_cast<unsigned __int128>(win_w) *
                                        max_pixel(pixel_type);
        if (worst > 0xffffffffu)
            return fail(SAT_ERR_OVERFLOW, "%s: a %lld x %lld window of this pixel type can exceed uint32", who,
                        (long long)win_h, (long long)win_w);
    }
    if ((st = check_pitch(out_pitch, ow, oh, bytes_of(out_type), who, "output"))) return st;
    if (overlap(span(out, oh, out_pitch, ow, bytes_of(out_type)), span(sat, H, sat_pitch, W, 8)))
        return fail(SAT_ERR_ARG, "%s: out overlaps the table", who);
    const int v = gather_variant();
    satk::GatherDesc d = gather_desc(sat, nullptr, sat_pitch, oh, ow, win_h, win_w, stride, out, nullptr, nullptr,
                                     out_pitch);
    hipError_t e = satk::launch_window_sum(v, d, out_type == SAT_U64, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

sat_status window_sum_multi(const uint64_t *sat, sat_dtype pixel_type, int64_t H, int64_t W, int64_t sat_pitch,
                            int32_t n_windows, const int64_t *win_h, const int64_t *win_w, int64_t stride,
                            void *const *outs, sat_dtype out_type, const int64_t *out_pitch, void *stream) {
    const char *who = "window_sum_multi";
    if (n_windows < 1 || n_windows > 8) return fail(SAT_ERR_ARG, "%s: n_windows must be 1..8", who);
    if (!win_h || !win_w || !outs || !out_pitch) return fail(SAT_ERR_ARG, "%s: NULL array argument", who);
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16 && pixel_type != SAT_U32)
        return fail(SAT_ERR_ARG, "%s: pixel_type must be SAT_U8, SAT_U16 or SAT_U32", who);
    if (out_type != SAT_U32 && out_type != SAT_U64)
        return fail(SAT_ERR_ARG, "%s: out_type must be SAT_U32 or SAT_U64", who);
    satk::GatherDesc d[8];
    Span spans[8];
    const Span ssat = span(sat, H, sat_pitch, W, 8);
    for (int i = 0; i < n_windows; ++i) {
        int64_t oh = 0, ow = 0;
        sat_status st = validate_window(sat, H, W, sat_pitch, win_h[i], win_w[i], stride, who, &oh, &ow);
        if (st) return st;
        if (!outs[i]) return fail(SAT_ERR_ARG, "%s: outs[%d] is NULL", who, i);
        if (out_type == SAT_U32) {
            const unsigned __int128 worst = static_cast<unsigned __int128>(win_h[i]) *
                                            static_cast<unsigned __int128>(win_w[i]) * max_pixel(pixel_type);
            if (worst > 0xffffffffu)
                return fail(SAT_ERR_OVERFLOW, "%s: window %d can exceed uint32", who, i);
        }
        if ((st = check_pitch(out_pitch[i], ow, oh, bytes_of(out_type), who, "output"))) return st;
        spans[i] = span(outs[i], oh, out_pitch[i], ow, bytes_of(out_type));
        if (overlap(spans[i], ssat)) return fail(SAT_ERR_ARG, "%s: outs[%d] overlaps the table", who, i);
        for (int j = 0; j < i; ++j)
            if (overlap(spans[i], spans[j])) return fail(SAT_ERR_ARG, "%s: outs[%d] and outs[%d] overlap", who, j, i);
        d[i] = gather_desc(sat, nullptr, sat_pitch, oh, ow, win_h[i], win_w[i], stride, outs[i], nullptr, nullptr,
                           out_pitch[i]);
    }
    hipError_t e = satk::launch_window_sum_multi(gather_variant(), d, n_windows, out_type == SAT_U64,
                                                 static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

sat_status window_mean_std(const uint64_t *sat, const uint64_t *sat_sq, int64_t H, int64_t W, int64_t sat_pitch,
                           int64_t win_h, int64_t win_w, int64_t stride, uint64_t *sum_out, double *mean_out,
                           double *std_out, int64_t out_pitch, void *stream) {
    const char *who = "window_mean_std";
    int64_t oh = 0, ow = 0;
    sat_status st = validate_window(sat, H, W, sat_pitch, win_h, win_w, stride, who, &oh, &ow);
    if (st) return st;
    if (!sat_sq || !mean_out || !std_out)
        return fail(SAT_ERR_ARG, "%s: sat_sq, mean_out and std_out must be non-NULL", who);
    if ((st = check_pitch(out_pitch, ow, oh, 8, who, "output"))) return st;
    const Span ssat = span(sat, H, sat_pitch, W, 8), ssq = span(sat_sq, H, sat_pitch, W, 8);
    const Span so[3] = {span(sum_out, oh, out_pitch, ow, 8), span(mean_out, oh, out_pitch, ow, 8),
                        span(std_out, oh, out_pitch, ow, 8)};
    for (int i = 0; i < 3; ++i) {
        if (overlap(so[i], ssat) || overlap(so[i], ssq))
            return fail(SAT_ERR_ARG, "%s: an output overlaps a table", who);
        for (int j = 0; j < i; ++j)
            if (overlap(so[i], so[j])) return fail(SAT_ERR_ARG, "%s: outputs overlap each other", who);
    }
    satk::GatherDesc d = gather_desc(sat, sat_sq, sat_pitch, oh, ow, win_h, win_w, stride, sum_out, mean_out,
                                     std_out, out_pitch);
    const int v = gather_variant();
    const int64_t items = satk::plan_mean_std(v, &d, 1);
    if (items > 0xffffffffll) return fail(SAT_ERR_ARG, "%s: too many work items", who);
    hipError_t e = satk::launch_mean_std(v, &d, 1, nullptr, items, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

// ------------------------------------------------------------------ tables of pixel powers, moments

namespace {

// Geometry of the power build (for strip heights and state sizes): 4 pixels per lane, 16 rows per
// wave, 4 compute waves.
const satk::BuildVariant kPowVariant{"power_px4_rw16_nw4", 4, 16, 4, satk::MODE_HELPER, 1};
static_assert(4 * 64 == satk::kPowBlockW && 16 * 4 == satk::kPowStripH, "power build geometry");

int64_t power_state_words(int64_t H, int64_t W, int k, int strip_h) {
    const int64_t strips = (H + strip_h - 1) / strip_h;
    const int64_t wp = (W + satk::kPowBlockW - 1) / satk::kPowBlockW * satk::kPowBlockW;
    return (strips * wp * k + 1) & ~1ll;
}

// Largest pixel^p of the pixel type (p <= 4 fits 128 bits).
unsigned __int128 max_pow(sat_dtype t, int p) {
    unsigned __int128 r = 1;
    for (int i = 0; i < p; ++i) r *= max_pixel(t);
    return r;
}

}  // namespace

size_t sat_powers_workspace_bytes(int64_t H, int64_t W, sat_dtype pixel_type, int32_t k) {
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return 0;
    if ((pixel_type != SAT_U8 && pixel_type != SAT_U16) || k < 1 || k > 4) return 0;
    // the shortest strips the balanced height may pick are half the full height
    return sizeof(satk::BuildCtrl) + 8 * static_cast<size_t>(power_state_words(H, W, k, satk::kPowStripH / 2));
}

sat_status sat_build_powers(const void *image, sat_dtype pixel_type, int64_t H, int64_t W, int64_t image_pitch,
                            int32_t k, uint64_t *const *tables, int64_t sat_pitch, void *workspace,
                            size_t workspace_bytes, void *stream) {
    const char *who = "sat_build_powers";
    if (!image || !tables) return fail(SAT_ERR_ARG, "%s: image and tables must be non-NULL", who);
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16)
        return fail(SAT_ERR_ARG, "%s: pixel_type must be SAT_U8 or SAT_U16", who);
    if (k < 1 || k > 4) return fail(SAT_ERR_ARG, "%s: k = %d must be 1..4", who, k);
    sat_status st = check_dims(H, W, who);
    if (st) return st;
    const int bpp = bytes_of(pixel_type);
    if ((st = check_pitch(image_pitch, W, H, bpp, who, "image"))) return st;
    if ((st = check_pitch(sat_pitch, W, H, 8, who, "table"))) return st;
    for (int p = 1; p <= k; ++p)
        if (static_cast<unsigned __int128>(H) * max_pow(pixel_type, p) >= (static_cast<unsigned __int128>(1) << 62))
            return fail(SAT_ERR_OVERFLOW, "%s: %lld rows of pixel^%d are too many for exact 62-bit column totals", who,
                        (long long)H, p);
    Span sp[5];
    sp[0] = span(image, H, image_pitch, W, bpp);
    for (int p = 0; p < k; ++p) {
        if (!tables[p]) return fail(SAT_ERR_ARG, "%s: tables[%d] must be non-NULL", who, p);
        sp[p + 1] = span(tables[p], H, sat_pitch, W, 8);
        for (int q = 0; q <= p; ++q)
            if (overlap(sp[p + 1], sp[q])) return fail(SAT_ERR_ARG, "%s: the image and tables must not overlap", who);
    }
    const size_t need = sat_powers_workspace_bytes(H, W, pixel_type, k);
    if (!workspace || workspace_bytes < need)
        return fail(SAT_ERR_WORKSPACE, "%s: workspace of %zu bytes is below the %zu needed", who, workspace_bytes,
                    need);
    if (reinterpret_cast<uintptr_t>(workspace) % 16) return fail(SAT_ERR_ARG, "%s: workspace must be 16-byte aligned", who);
    const Span sw{reinterpret_cast<uintptr_t>(workspace), reinterpret_cast<uintptr_t>(workspace) + workspace_bytes};
    for (int p = 0; p <= k; ++p)
        if (overlap(sw, sp[p])) return fail(SAT_ERR_ARG, "%s: workspace overlaps an input or output", who);
    const int cap = satk::power_build_capacity(bpp, k);
    const int strip_h = balanced_strip_h(H, satk::kPowStripH, cap);
    satk::BuildDesc d{};
    fill_desc(d, kPowVariant, image, bpp, H, W, image_pitch, tables[0], k >= 2 ? tables[1] : nullptr, sat_pitch,
              strip_h);
    d.T3 = k >= 3 ? tables[2] : nullptr;
    d.T4 = k >= 4 ? tables[3] : nullptr;
    bool aligned = sat_pitch % 2 == 0;
    for (int p = 0; p < k; ++p) aligned = aligned && reinterpret_cast<uintptr_t>(tables[p]) % 16 == 0;
    d.sat_vec = aligned ? 1 : 0;
    d.state_off = 0;
    d.first_item = 0;
    const int64_t words = power_state_words(H, W, k, strip_h);
    hipError_t e = satk::launch_build_powers(bpp, k, d, workspace, words, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

sat_status window_moments(const uint64_t *const *tables, int32_t k, sat_dtype pixel_type, int64_t H, int64_t W,
                          int64_t sat_pitch, int64_t win_h, int64_t win_w, int64_t stride, double *mean_out,
                          double *std_out, double *skew_out, double *kurt_out, int64_t out_pitch, void *stream) {
    const char *who = "window_moments";
    if (!tables) return fail(SAT_ERR_ARG, "%s: tables must be non-NULL", who);
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16)
        return fail(SAT_ERR_ARG, "%s: pixel_type must be SAT_U8 or SAT_U16", who);
    const int order = kurt_out ? 4 : skew_out ? 3 : std_out ? 2 : mean_out ? 1 : 0;
    if (order == 0) return fail(SAT_ERR_ARG, "%s: at least one output must be non-NULL", who);
    if (k < order || k > 4)
        return fail(SAT_ERR_ARG, "%s: %d tables given, the requested statistics need %d (at most 4)", who, k, order);
    int64_t oh = 0, ow = 0;
    sat_status st = validate_window(tables[0], H, W, sat_pitch, win_h, win_w, stride, who, &oh, &ow);
    if (st) return st;
    for (int p = 0; p < order; ++p)
        if (!tables[p]) return fail(SAT_ERR_ARG, "%s: tables[%d] must be non-NULL", who, p);
    // Window sums must be exact (below 2^64), and the 128-bit numerators must not overflow: their
    // terms are bounded by 6 (n*m)^3 for the skewness and 17 (n*m)^4 for the kurtosis.
    const uint64_t n = static_cast<uint64_t>(win_h) * static_cast<uint64_t>(win_w);
    for (int p = 1; p <= order; ++p)
        if (static_cast<unsigned __int128>(n) * max_pow(pixel_type, p) >= (static_cast<unsigned __int128>(1) << 64))
            return fail(SAT_ERR_OVERFLOW, "%s: window sums of pixel^%d over %llu pixels can exceed 64 bits", who, p,
                        (unsigned long long)n);
    const double nm = static_cast<double>(n) * static_cast<double>(max_pixel(pixel_type));
    const double lim = std::ldexp(1.0, 127) * 0.999;
    if ((order >= 3 && 6.0 * nm * nm * nm >= lim) || (order >= 4 && 17.0 * nm * nm * nm * nm >= lim))
        return fail(SAT_ERR_OVERFLOW, "%s: the moment numerators of %llu-pixel windows can exceed 128 bits", who,
                    (unsigned long long)n);
    if ((st = check_pitch(out_pitch, ow, oh, 8, who, "output"))) return st;
    double *outs[4] = {mean_out, std_out, skew_out, kurt_out};
    Span so[4], stab[4];
    for (int p = 0; p < order; ++p) stab[p] = span(tables[p], H, sat_pitch, W, 8);
    for (int i = 0; i < 4; ++i) {
        so[i] = span(outs[i], oh, out_pitch, ow, 8);
        for (int p = 0; p < order; ++p)
            if (overlap(so[i], stab[p])) return fail(SAT_ERR_ARG, "%s: an output overlaps a table", who);
        for (int j = 0; j < i; ++j)
            if (overlap(so[i], so[j])) return fail(SAT_ERR_ARG, "%s: outputs overlap each other", who);
    }
    satk::MomentDesc d{};
    for (int p = 0; p < order; ++p) d.T[p] = tables[p];
    d.spitch = sat_pitch;
    d.oh = oh;
    d.ow = ow;
    d.win_h = win_h;
    d.win_w = win_w;
    d.stride = stride;
    d.mean = mean_out;
    d.stdv = std_out;
    d.skew = skew_out;
    d.kurt = kurt_out;
    d.opitch = out_pitch;
    const int64_t chunks = (ow + 255) / 256;
    if (oh * chunks > 0xffffffffll) return fail(SAT_ERR_ARG, "%s: too many work items", who);
    hipError_t e = satk::launch_window_moments(gather_variant(), order, d, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

// ------------------------------------------------------------------ batches

static size_t round256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Strip height of the images of a batch under variant v: the variant's full height, or the height
// sat_force_variant(2, rows) set on this thread (tuning), capped at the full height for variants
// whose waves take fewer rows (adaptive) and ignored for the others.
static int batch_strip_h(int v) {
    const satk::BuildVariant &var = satk::build_variant(v);
    const int f = g_force[2];
    if (f < 1 || !satk::build_variant_adaptive(v)) return var.th();
    return f < var.th() ? f : var.th();
}

// Validation and descriptors of a batch of builds (sat_build_batched and sat_build_stats_batched):
// every item valid, squared tables on all items or none, the variant for the batch's rows and
// alignment, one descriptor per item with its lookback words (state_words in all, even) and its
// first work item (items_total in all).
static sat_status plan_build_batch(const sat_batch_item *items, int32_t n, sat_dtype pixel_type, const char *who,
                                   std::vector<satk::BuildDesc> &d, int *variant, int64_t *state_words,
                                   int64_t *items_total) {
    if (!items || n < 1) return fail(SAT_ERR_ARG, "%s: need at least one item", who);
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16)
        return fail(SAT_ERR_ARG, "%s: pixel_type must be SAT_U8 or SAT_U16", who);
    const bool sq = items[0].sat_sq != nullptr;
    int64_t rows = 0;
    for (int i = 0; i < n; ++i) {
        char tag[64];
        snprintf(tag, sizeof tag, "%s item %d", who, i);
        const sat_batch_item &it = items[i];
        sat_status st = validate_build_item(it.image, pixel_type, it.H, it.W, it.image_pitch, it.sat, it.sat_sq,
                                            it.sat_pitch, tag);
        if (st) return st;
        if ((it.sat_sq != nullptr) != sq)
            return fail(SAT_ERR_ARG, "%s: item %d: every item or none must have sat_sq", who, i);
        rows += it.H;
    }
    const int bpp = bytes_of(pixel_type);
    int align = 16;
    for (int i = 0; i < n; ++i) {
        const int a = row_align(items[i].image, items[i].image_pitch, bpp);
        if (a < align) align = a;
    }
    const int v = choose_build_variant(rows, 0, n, bpp, sq, align);
    if (sat_status st = check_build_variant(v, bpp, sq, who)) return st;
    const satk::BuildVariant &var = satk::build_variant(v);
    d.assign(n, satk::BuildDesc{});
    int64_t off = 0, total = 0;
    for (int i = 0; i < n; ++i) {
        const sat_batch_item &it = items[i];
        fill_desc(d[i], var, it.image, bpp, it.H, it.W, it.image_pitch, it.sat, it.sat_sq, it.sat_pitch,
                  batch_strip_h(v));
        const int64_t plane = static_cast<int64_t>(d[i].nstrips) * d[i].Wp;
        d[i].state_off = off;
        d[i].state_q_off = off + plane;
        off += plane * (sq ? 2 : 1);
        d[i].first_item = total;
        total += d[i].nstrips;
    }
    bool narrow = true;
    for (int i = 0; i < n; ++i) narrow = narrow && narrow_state(var, sq, items[i].H, bpp);
    for (int i = 0; i < n; ++i) d[i].narrow = narrow ? 1u : 0u;
    *variant = v;
    *state_words = (off + 1) & ~1ll;
    *items_total = total;
    return SAT_OK;
}

// Tables and images of a batch must not overlap the workspace, and no two items' tables overlap.
static sat_status check_batch_workspace(const sat_batch_item *items, int32_t n, sat_dtype pixel_type, void *workspace,
                                        size_t workspace_bytes, const char *who) {
    const Span sw{reinterpret_cast<uintptr_t>(workspace), reinterpret_cast<uintptr_t>(workspace) + workspace_bytes};
    const int bpp = bytes_of(pixel_type);
    std::vector<Span> outs;
    for (int i = 0; i < n; ++i) {
        const sat_batch_item &it = items[i];
        const Span a = span(it.sat, it.H, it.sat_pitch, it.W, 8), b = span(it.sat_sq, it.H, it.sat_pitch, it.W, 8);
        if (overlap(a, sw) || overlap(b, sw) || overlap(span(it.image, it.H, it.image_pitch, it.W, bpp), sw))
            return fail(SAT_ERR_ARG, "%s: item %d overlaps the workspace", who, i);
        for (const Span &o : outs)
            if (overlap(o, a) || overlap(o, b)) return fail(SAT_ERR_ARG, "%s: item %d tables overlap another", who, i);
        outs.push_back(a);
        if (b.lo != b.hi) outs.push_back(b);
    }
    return SAT_OK;
}

// Validation and chain/row-pair plan of the window statistics of a batch (window_mean_std_batched
// and sat_build_stats_batched): every window fits its image, sat_sq, mean_out and std_out given,
// outputs inside their pitch and apart from each other, the workspace and every table.
static sat_status plan_stats_batch(const sat_batch_item *items, int32_t n, int64_t win_h, int64_t win_w,
                                   int64_t stride, void *workspace, size_t workspace_bytes, const char *who,
                                   std::vector<satk::GatherDesc> &d, int *gvariant, int64_t *total_items) {
    if (!items || n < 1) return fail(SAT_ERR_ARG, "%s: need at least one item", who);
    d.assign(n, satk::GatherDesc{});
    const Span sw{reinterpret_cast<uintptr_t>(workspace), reinterpret_cast<uintptr_t>(workspace) + workspace_bytes};
    std::vector<Span> outs;
    for (int i = 0; i < n; ++i) {
        char tag[64];
        snprintf(tag, sizeof tag, "%s item %d", who, i);
        const sat_batch_item &it = items[i];
        int64_t oh = 0, ow = 0;
        sat_status st = validate_window(it.sat, it.H, it.W, it.sat_pitch, win_h, win_w, stride, tag, &oh, &ow);
        if (st) return st;
        if (!it.sat_sq || !it.mean_out || !it.std_out)
            return fail(SAT_ERR_ARG, "%s: sat_sq, mean_out and std_out must be non-NULL", tag);
        if ((st = check_pitch(it.out_pitch, ow, oh, 8, tag, "output"))) return st;
        const Span so[3] = {span(it.sum_out, oh, it.out_pitch, ow, 8), span(it.mean_out, oh, it.out_pitch, ow, 8),
                            span(it.std_out, oh, it.out_pitch, ow, 8)};
        for (int a = 0; a < 3; ++a) {
            if (overlap(so[a], sw)) return fail(SAT_ERR_ARG, "%s: output overlaps the workspace", tag);
            for (const Span &o : outs)
                if (overlap(o, so[a])) return fail(SAT_ERR_ARG, "%s: outputs overlap", tag);
        }
        for (int a = 0; a < 3; ++a)
            if (so[a].lo != so[a].hi) outs.push_back(so[a]);
        d[i] = gather_desc(it.sat, it.sat_sq, it.sat_pitch, oh, ow, win_h, win_w, stride, it.sum_out, it.mean_out,
                           it.std_out, it.out_pitch);
    }
    const int v = gather_variant();
    const int64_t total = satk::plan_mean_std(v, d.data(), n);
    for (int i = 0; i < n; ++i) {
        const Span a = span(items[i].sat, items[i].H, items[i].sat_pitch, items[i].W, 8);
        const Span b = span(items[i].sat_sq, items[i].H, items[i].sat_pitch, items[i].W, 8);
        for (const Span &o : outs)
            if (overlap(o, a) || overlap(o, b)) return fail(SAT_ERR_ARG, "%s: an output overlaps a table", who);
    }
    if (total > 0xffffffffll) return fail(SAT_ERR_ARG, "%s: too many work items", who);
    *gvariant = v;
    *total_items = total;
    return SAT_OK;
}

size_t sat_batch_workspace_bytes(const sat_batch_item *items, int32_t n, sat_dtype pixel_type, int with_sq) {
    if (!items || n < 1) return 0;
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16) return 0;
    size_t words = 0;
    int64_t rows = 0;
    for (int i = 0; i < n; ++i) {
        if (items[i].H < 1 || items[i].W < 1 || items[i].H > kMaxDim || items[i].W > kMaxDim) return 0;
        rows += items[i].H;
    }
    for (int align : {16, 4, 1}) {   // whichever variant the rows' alignment selects
        const int v = choose_build_variant(rows, 0, n, bytes_of(pixel_type), with_sq != 0, align);
        if (v < 0 || v >= satk::build_variant_count()) return 0;
        const satk::BuildVariant &var = satk::build_variant(v);
        size_t w = 0;
        for (int i = 0; i < n; ++i)
            w += static_cast<size_t>(state_words_for(var, items[i].H, items[i].W, with_sq != 0, batch_strip_h(v)));
        if (w > words) words = w;
    }
    const size_t descs = round256(static_cast<size_t>(n) *
                                  (sizeof(satk::BuildDesc) > sizeof(satk::GatherDesc) ? sizeof(satk::BuildDesc)
                                                                                      : sizeof(satk::GatherDesc)));
    return sizeof(satk::BuildCtrl) + descs + 8 * words + 256;   // 256: alignment slack
}

sat_status sat_build_batched(const sat_batch_item *items, int32_t n, sat_dtype pixel_type, void *workspace,
                             size_t workspace_bytes, void *stream) {
    const char *who = "sat_build_batched";
    std::vector<satk::BuildDesc> d;
    int v = 0;
    int64_t off = 0, items_total = 0;
    sat_status st = plan_build_batch(items, n, pixel_type, who, d, &v, &off, &items_total);
    if (st) return st;
    const bool with_sq = items[0].sat_sq != nullptr;
    const size_t need = sat_batch_workspace_bytes(items, n, pixel_type, with_sq);
    if (!workspace || workspace_bytes < need)
        return fail(SAT_ERR_WORKSPACE, "%s: workspace of %zu bytes is below the %zu needed", who, workspace_bytes,
                    need);
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(SAT_ERR_ARG, "%s: workspace must be 256-byte aligned", who);
    if ((st = check_batch_workspace(items, n, pixel_type, workspace, workspace_bytes, who))) return st;
    // Layout: [control 256 B][state][descriptors]; the kernels see the state right after the
    // control header, so the descriptors go at the end of the used state.
    char *base = static_cast<char *>(workspace);
    const size_t desc_bytes = round256(static_cast<size_t>(n) * sizeof(satk::BuildDesc));
    char *dev_desc = base + sizeof(satk::BuildCtrl) + 8 * static_cast<size_t>(off);
    dev_desc = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(dev_desc) + 255) & ~static_cast<uintptr_t>(255));
    if (dev_desc + desc_bytes > base + workspace_bytes)
        return fail(SAT_ERR_WORKSPACE, "%s: workspace too small for the descriptor table", who);
    hipStream_t s = static_cast<hipStream_t>(stream);
    static_assert(sizeof(satk::BuildDesc) % 8 == 0, "descriptors move as 64-bit words");
    hipError_t e = satk::upload_words(d.data(), static_cast<size_t>(n) * sizeof(satk::BuildDesc), dev_desc, s);
    if (e != hipSuccess) return hip_fail(e, who);
    e = satk::launch_build(v, bytes_of(pixel_type), with_sq, d.data(), n, reinterpret_cast<satk::BuildDesc *>(dev_desc),
                           items_total, workspace, off, s);
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

sat_status window_mean_std_batched(const sat_batch_item *items, int32_t n, int64_t win_h, int64_t win_w,
                                   int64_t stride, void *workspace, size_t workspace_bytes, void *stream) {
    const char *who = "window_mean_std_batched";
    if (!items || n < 1) return fail(SAT_ERR_ARG, "%s: need at least one item", who);
    if (!workspace) return fail(SAT_ERR_WORKSPACE, "%s: workspace must be non-NULL", who);
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(SAT_ERR_ARG, "%s: workspace must be 256-byte aligned", who);
    // the descriptor table goes after the control header, which keeps the fault word of a build
    // that shared this workspace intact for sat_workspace_check
    const size_t desc_bytes = round256(static_cast<size_t>(n) * sizeof(satk::GatherDesc));
    if (workspace_bytes < sizeof(satk::BuildCtrl) + desc_bytes)
        return fail(SAT_ERR_WORKSPACE, "%s: workspace of %zu bytes is below the %zu needed", who, workspace_bytes,
                    sizeof(satk::BuildCtrl) + desc_bytes);
    std::vector<satk::GatherDesc> d;
    int v = 0;
    int64_t total = 0;
    sat_status st = plan_stats_batch(items, n, win_h, win_w, stride, workspace, workspace_bytes, who, d, &v, &total);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    static_assert(sizeof(satk::GatherDesc) % 8 == 0, "descriptors move as 64-bit words");
    auto *dev_desc = reinterpret_cast<satk::GatherDesc *>(static_cast<char *>(workspace) + sizeof(satk::BuildCtrl));
    hipError_t e = satk::upload_words(d.data(), static_cast<size_t>(n) * sizeof(satk::GatherDesc), dev_desc, s);
    if (e != hipSuccess) return hip_fail(e, who);
    e = satk::launch_mean_std(v, d.data(), n, dev_desc, total, s);
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

size_t sat_build_stats_workspace_bytes(const sat_batch_item *items, int32_t n, sat_dtype pixel_type) {
    const size_t b = sat_batch_workspace_bytes(items, n, pixel_type, 1);
    if (b == 0) return 0;
    // the build's workspace, then the per-image ready counters and the statistics descriptors
    return b + round256(4 * static_cast<size_t>(n) + 8) + round256(static_cast<size_t>(n) * sizeof(satk::GatherDesc));
}

sat_status sat_build_stats_batched(const sat_batch_item *items, int32_t n, sat_dtype pixel_type, int64_t win_h,
                                   int64_t win_w, int64_t stride, void *workspace, size_t workspace_bytes,
                                   void *stream) {
    const char *who = "sat_build_stats_batched";
    std::vector<satk::BuildDesc> bd;
    int bv = 0;
    int64_t state_words = 0, build_items = 0;
    sat_status st = plan_build_batch(items, n, pixel_type, who, bd, &bv, &state_words, &build_items);
    if (st) return st;
    if (!items[0].sat_sq) return fail(SAT_ERR_ARG, "%s: every item needs sat_sq", who);
    const size_t need = sat_build_stats_workspace_bytes(items, n, pixel_type);
    if (!workspace || workspace_bytes < need)
        return fail(SAT_ERR_WORKSPACE, "%s: workspace of %zu bytes is below the %zu needed", who, workspace_bytes,
                    need);
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(SAT_ERR_ARG, "%s: workspace must be 256-byte aligned", who);
    if ((st = check_batch_workspace(items, n, pixel_type, workspace, workspace_bytes, who))) return st;
    std::vector<satk::GatherDesc> gd;
    int gv = 0;
    int64_t gather_items = 0;
    if ((st = plan_stats_batch(items, n, win_h, win_w, stride, workspace, workspace_bytes, who, gd, &gv,
                               &gather_items)))
        return st;
    if (!satk::fused_build_variant(bv) || gd[0].q == 0) {
        // no fused kernel for this build variant or window (row-pair statistics): two launches
        if ((st = sat_build_batched(items, n, pixel_type, workspace, workspace_bytes, stream))) return st;
        return window_mean_std_batched(items, n, win_h, win_w, stride, workspace, workspace_bytes, stream);
    }
    // Layout: [control 256 B][lookback words][ready counters][build descriptors][statistics
    // descriptors]; the launch clears the lookback words and the counters together.
    const int64_t ready_words = (n + 1) / 2;
    const int64_t cleared = (state_words + ready_words + 1) & ~1ll;
    char *base = static_cast<char *>(workspace);
    auto *ready = reinterpret_cast<unsigned int *>(base + sizeof(satk::BuildCtrl) + 8 * static_cast<size_t>(state_words));
    char *dev_b = base + sizeof(satk::BuildCtrl) + 8 * static_cast<size_t>(cleared);
    dev_b = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(dev_b) + 255) & ~static_cast<uintptr_t>(255));
    char *dev_g = dev_b + round256(static_cast<size_t>(n) * sizeof(satk::BuildDesc));
    if (dev_g + static_cast<size_t>(n) * sizeof(satk::GatherDesc) > base + workspace_bytes)
        return fail(SAT_ERR_WORKSPACE, "%s: workspace too small for the descriptor tables", who);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = satk::upload_words(bd.data(), static_cast<size_t>(n) * sizeof(satk::BuildDesc), dev_b, s);
    if (e == hipSuccess)
        e = satk::upload_words(gd.data(), static_cast<size_t>(n) * sizeof(satk::GatherDesc), dev_g, s);
    if (e == hipSuccess)
        e = satk::launch_fused(bv, bytes_of(pixel_type), satk::mean_std_chain_v(gv, stride), bd.data(), n,
                               reinterpret_cast<satk::BuildDesc *>(dev_b), build_items,
                               reinterpret_cast<satk::GatherDesc *>(dev_g), gather_items, workspace, cleared, ready, s);
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

sat_status sat_workspace_check(void *workspace, void *stream) {
    if (!workspace) return fail(SAT_ERR_ARG, "sat_workspace_check: workspace must be non-NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "sat_workspace_check");
    satk::BuildCtrl ctrl;
    e = hipMemcpy(&ctrl, workspace, sizeof ctrl, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "sat_workspace_check");
    if (ctrl.fault & 1u) return fail(SAT_ERR_DEVICE, "sat_workspace_check: a lookback wait exceeded its spin bound");
    if (ctrl.fault & 2u)
        return fail(SAT_ERR_DEVICE, "sat_workspace_check: a carried column total leaves no room below 2^62 for "
                    "the band (a carry above its rows_above bound)");
    if (ctrl.fault & 4u)
        return fail(SAT_ERR_DEVICE, "sat_workspace_check: a statistics item's wait for its image's tables exceeded "
                    "its spin bound");
    return ok();
}

sat_status sat_upload(const void *host, void *dst, size_t nbytes, void *stream) {
    const char *who = "sat_upload";
    if (!host || !dst) return fail(SAT_ERR_ARG, "%s: host and dst must be non-NULL", who);
    if (nbytes == 0) return fail(SAT_ERR_ARG, "%s: nbytes must be at least 1", who);
    if ((reinterpret_cast<uintptr_t>(host) | reinterpret_cast<uintptr_t>(dst)) & 15u)
        return fail(SAT_ERR_ARG, "%s: host and dst must be 16-byte aligned", who);
    // the device's address of the pinned pages (the same address on a unified address space)
    void *src = nullptr;
    hipError_t e = hipHostGetDevicePointer(&src, const_cast<void *>(host), 0);
    if (e != hipSuccess || !src) {
        (void)hipGetLastError();     // leave no sticky error behind for the caller's next check
        return fail(SAT_ERR_ARG, "%s: host is not pinned, device-accessible host memory (hipHostMalloc)", who);
    }
    e = satk::launch_upload(src, dst, nbytes, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, who);
    return ok();
}

int32_t sat_variant_count(int32_t kind) {
    if (kind == 0) return satk::build_variant_count();
    if (kind == 1) return satk::gather_variant_count();
    return 0;
}

const char *sat_variant_name(int32_t kind, int32_t index) {
    if (kind == 0 && index >= 0 && index < satk::build_variant_count()) return satk::build_variant(index).name;
    if (kind == 1 && index >= 0 && index < satk::gather_variant_count()) return satk::gather_variant_name(index);
    return "";
}

int32_t sat_variant_supported(int32_t kind, int32_t index, sat_dtype pixel_type, int32_t with_sq) {
    if (index < 0 || index >= sat_variant_count(kind)) return 0;
    if (pixel_type != SAT_U8 && pixel_type != SAT_U16) return 0;
    if (kind == 1) return 1;
    return satk::build_variant_capacity(index, bytes_of(pixel_type), with_sq != 0) > 0 ? 1 : 0;
}

sat_status sat_force_variant(int32_t kind, int32_t index) {
    if (kind == 4) {
        if (index < 0 || index > satk::kMaxSeg)
            return fail(SAT_ERR_ARG, "sat_force_variant: column segments must be 0 (built-in) .. %d", satk::kMaxSeg);
        g_force[4] = index;
        return ok();
    }
    if (kind == 3) {
        if (index < 0) return fail(SAT_ERR_ARG, "sat_force_variant: stress seed must be >= 0");
        g_force[3] = index;
        return ok();
    }
    if (kind == 2) {
        if (index != -1 && (index < 1 || index > 1024))
            return fail(SAT_ERR_ARG, "sat_force_variant: strip height out of range");
        g_force[2] = index;
        return ok();
    }
    if (kind != 0 && kind != 1) return fail(SAT_ERR_ARG, "sat_force_variant: kind must be 0 .. 4");
    if (index < -1 || index >= sat_variant_count(kind))
        return fail(SAT_ERR_ARG, "sat_force_variant: index out of range");
    g_force[kind] = index;
    return ok();
}

}  // extern "C"
