// sat_gather.hip -- window statistics from integral images by the four-corner lookup.
//
// A window sum is the table value at the window's bottom-right corner, minus the value just above
// the window at its right edge, minus the value just left of it at its bottom edge, plus the
// value diagonally above-left (Sec. II-B); one output per window position of the valid region
// (Sec. II-A, Sec. III-A), four lookups each (the 4(r*c) term of Sec. III-B).
//
// The kernels are bound by HBM bandwidth.  A work item is one output row segment of `chunk`
// consecutive outputs; a thread handles V outputs spaced 256 apart so that every load and store
// instruction of a wave touches 64 consecutive elements.  Of the two table rows an output row
// reads, the upper one was the lower one of the output row win_h/stride rows earlier; items are
// ordered row by row inside column bands so that this reuse distance stays inside the
// memory-side cache (band width chosen by the host from win_h).
#include "sat_internal.h"

namespace satk {
namespace {

struct ItemMap {
    int64_t k;    // output row
    int64_t c;    // column chunk
};

// Band-major, then row-major traversal of (output row, chunk) items.
__device__ __forceinline__ ItemMap map_item(int64_t item, int64_t oh, int64_t chunks, int64_t band) {
    const int64_t full = chunks / band;                 // number of full bands
    const int64_t per_full = oh * band;
    ItemMap m;
    const int64_t b = item / per_full;
    if (b < full) {
        const int64_t r = item - b * per_full;
        m.k = r / band;
        m.c = b * band + (r - m.k * band);
    } else {
        const int64_t last = chunks - full * band;      // width of the ragged last band
        const int64_t r = item - full * per_full;
        m.k = r / last;
        m.c = full * band + (r - m.k * last);
    }
    return m;
}

// The four corner values of output l of an output row: bottom-right, bottom-left-outside,
// top-right-outside, top-left-outside.  Loads are issued for every l (indices clamped into the
// row) so that all of a thread's loads are in flight before the first use; terms that fall
// outside the table (row y0-1 < 0 or column x0-1 < 0) are masked to zero afterwards.
struct Corners {
    uint64_t b1, b0, t1, t0;
};

__device__ __forceinline__ Corners load_corners(const uint64_t *__restrict__ top, const uint64_t *__restrict__ bot,
                                                int64_t l, const GatherDesc &d) {
    const int64_t lc = l < d.ow ? l : d.ow - 1;
    const int64_t x0 = lc * d.stride;
    const int64_t x1 = x0 + d.win_w - 1;
    const int64_t xm = x0 > 0 ? x0 - 1 : 0;
    Corners c;
    c.b1 = bot[x1];
    c.b0 = bot[xm];
    c.t1 = top[x1];
    c.t0 = top[xm];
    return c;
}

__device__ __forceinline__ uint64_t corner_sum(const Corners &c, int64_t l, const GatherDesc &d, bool has_top) {
    const bool has_left = l * d.stride > 0;
    const uint64_t b0 = has_left ? c.b0 : 0;
    const uint64_t t1 = has_top ? c.t1 : 0;
    const uint64_t t0 = (has_top && has_left) ? c.t0 : 0;
    return c.b1 - t1 - b0 + t0;
}

template <typename OutT, int V>
__global__ __launch_bounds__(256) void window_sum_kernel(GatherDesc d, int64_t band) {
    const ItemMap m = map_item(blockIdx.x, d.oh, d.chunks, band);
    const int64_t y0 = m.k * d.stride;
    const int64_t y1 = y0 + d.win_h - 1;
    const bool has_top = y0 > 0;
    const uint64_t *bot = d.S + y1 * d.spitch;
    const uint64_t *top = d.S + (has_top ? y0 - 1 : 0) * d.spitch;
    OutT *out = static_cast<OutT *>(d.out) + m.k * d.opitch;
    const int64_t l0 = m.c * (256 * V) + threadIdx.x;
    Corners c[V];
#pragma unroll
    for (int v = 0; v < V; ++v) c[v] = load_corners(top, bot, l0 + v * 256, d);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t l = l0 + v * 256;
        if (l < d.ow) out[l] = static_cast<OutT>(corner_sum(c[v], l, d, has_top));
    }
}

// Several windows of one table, one pass: all windows share the row above the window (y0 - 1)
// and the column left of it (x0 - 1) for a given output position, so the upper row segment is
// read once for all of them.  Windows are sorted by height by the host; items follow the rows
// and bands of the tallest window.
constexpr int kMaxMulti = 8;
struct MultiArgs {
    GatherDesc d[kMaxMulti];
    int n;
    int64_t oh_max;       // rows of the shortest window's output (the largest oh)
    int64_t chunks;       // chunks of the widest output row
};

template <typename OutT, int V>
__global__ __launch_bounds__(256) void window_sum_multi_kernel(MultiArgs a, int64_t band) {
    const ItemMap m = map_item(blockIdx.x, a.oh_max, a.chunks, band);
    const int64_t stride = a.d[0].stride;
    const int64_t y0 = m.k * stride;
    const bool has_top = y0 > 0;
    const uint64_t *S = a.d[0].S;
    const int64_t spitch = a.d[0].spitch;
    const uint64_t *top = S + (has_top ? y0 - 1 : 0) * spitch;
    const int64_t l0 = m.c * (256 * V) + threadIdx.x;
    for (int i = 0; i < a.n; ++i) {
        const GatherDesc &d = a.d[i];
        if (m.k >= d.oh) continue;
        const uint64_t *bot = S + (y0 + d.win_h - 1) * spitch;
        OutT *out = static_cast<OutT *>(d.out) + m.k * d.opitch;
        Corners c[V];
#pragma unroll
        for (int v = 0; v < V; ++v) c[v] = load_corners(top, bot, l0 + v * 256, d);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int64_t l = l0 + v * 256;
            if (l < d.ow) out[l] = static_cast<OutT>(corner_sum(c[v], l, d, has_top));
        }
    }
}

// Correctly rounded conversion of an unsigned 128-bit integer to double: the top 64 significant
// bits (the lowest of them made sticky for any nonzero remainder) are converted with one
// round-to-nearest, then scaled by an exact power of two.
__device__ __forceinline__ double u128_to_double(uint64_t hi, uint64_t lo) {
    if (hi == 0) return static_cast<double>(lo);
    const int lz = __clzll(static_cast<long long>(hi));
    uint64_t top = lz ? ((hi << lz) | (lo >> (64 - lz))) : hi;
    const uint64_t rest = lz ? (lo << lz) : lo;
    top |= (rest != 0) ? 1u : 0u;
    return ldexp(static_cast<double>(top), 64 - lz);
}

template <int V>
__device__ __forceinline__ void mean_std_row(const GatherDesc &d, int64_t k, int64_t c) {
    const int64_t y0 = k * d.stride;
    const int64_t y1 = y0 + d.win_h - 1;
    const bool has_top = y0 > 0;
    const uint64_t *botS = d.S + y1 * d.spitch;
    const uint64_t *topS = d.S + (has_top ? y0 - 1 : 0) * d.spitch;
    const uint64_t *botQ = d.Q + y1 * d.spitch;
    const uint64_t *topQ = d.Q + (has_top ? y0 - 1 : 0) * d.spitch;
    const uint64_t n = static_cast<uint64_t>(d.win_h) * static_cast<uint64_t>(d.win_w);
    const double dn = static_cast<double>(n);
    uint64_t *sum = static_cast<uint64_t *>(d.out);
    const int64_t l0 = c * (256 * V) + threadIdx.x;
    Corners cs[V], cq[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        cs[v] = load_corners(topS, botS, l0 + v * 256, d);
        cq[v] = load_corners(topQ, botQ, l0 + v * 256, d);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t l = l0 + v * 256;
        if (l < d.ow) {
            const uint64_t s1 = corner_sum(cs[v], l, d, has_top);
            const uint64_t q1 = corner_sum(cq[v], l, d, has_top);
            // n*q1 - s1*s1 exactly, in 128 bits (non-negative by Cauchy-Schwarz).
            const uint64_t a_lo = n * q1, a_hi = __umul64hi(n, q1);
            const uint64_t b_lo = s1 * s1, b_hi = __umul64hi(s1, s1);
            const uint64_t num_lo = a_lo - b_lo;
            const uint64_t num_hi = a_hi - b_hi - (a_lo < b_lo ? 1u : 0u);
            const int64_t o = k * d.opitch + l;
            if (sum) sum[o] = s1;
            d.mean[o] = static_cast<double>(s1) / dn;
            d.stdv[o] = sqrt(u128_to_double(num_hi, num_lo)) / dn;
        }
    }
}

template <int V>
__global__ __launch_bounds__(256) void mean_std_kernel(GatherDesc one, const GatherDesc *__restrict__ many,
                                                       int n, int64_t band) {
    const int64_t item = blockIdx.x;
    if (many == nullptr) {
        const ItemMap m = map_item(item, one.oh, one.chunks, band);
        mean_std_row<V>(one, m.k, m.c);
        return;
    }
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (many[mid].first_item <= item) lo = mid;
        else hi = mid - 1;
    }
    const GatherDesc d = many[lo];
    const int64_t r = item - d.first_item;
    const int64_t k = r / d.chunks;
    mean_std_row<V>(d, k, r - k * d.chunks);
}

struct GatherVariant {
    const char *name;
    int v;          // outputs per thread
    int banded;     // 1: column bands sized to the window height; 0: plain row-major
};
const GatherVariant kGather[] = {
    {"v4_banded", 4, 1},
    {"v2_banded", 2, 1},
    {"v8_banded", 8, 1},
    {"v4_rowmajor", 4, 0},
};
constexpr int kNumGather = sizeof(kGather) / sizeof(kGather[0]);

// Column band (in chunks) such that win_h table rows of the band stay within a budget of the
// memory-side cache: rows * band_columns * 8 B <= budget.
int64_t band_chunks(const GatherDesc &d, int v, bool banded, int64_t rows_reused) {
    if (!banded) return d.chunks;
    const int64_t budget = 96ll << 20;
    const int64_t cols = budget / (8 * (rows_reused > 0 ? rows_reused : 1));
    const int64_t chunk_cols = 256ll * v * d.stride;
    int64_t band = cols / chunk_cols;
    if (band < 1) band = 1;
    if (band > d.chunks) band = d.chunks;
    return band;
}

template <typename OutT>
hipError_t launch_sum_typed(int v, const GatherDesc &d0, bool banded, hipStream_t s) {
    GatherDesc d = d0;
    d.chunks = (d.ow + 256 * v - 1) / (256 * v);
    const int64_t band = band_chunks(d, v, banded, d.win_h);
    const int64_t items = d.oh * d.chunks;
    const dim3 grid(static_cast<unsigned>(items));
    switch (v) {
        case 2: hipLaunchKernelGGL((window_sum_kernel<OutT, 2>), grid, dim3(256), 0, s, d, band); break;
        case 8: hipLaunchKernelGGL((window_sum_kernel<OutT, 8>), grid, dim3(256), 0, s, d, band); break;
        default: hipLaunchKernelGGL((window_sum_kernel<OutT, 4>), grid, dim3(256), 0, s, d, band); break;
    }
    return hipGetLastError();
}

}  // namespace

int gather_variant_count() { return kNumGather; }
const char *gather_variant_name(int v) { return kGather[v].name; }
int64_t gather_chunk_outputs(int v) { return 256ll * kGather[v].v; }

hipError_t launch_window_sum(int variant, const GatherDesc &d, bool out64, hipStream_t stream) {
    const GatherVariant &g = kGather[variant];
    return out64 ? launch_sum_typed<uint64_t>(g.v, d, g.banded != 0, stream)
                 : launch_sum_typed<uint32_t>(g.v, d, g.banded != 0, stream);
}

hipError_t launch_window_sum_multi(const GatherDesc *descs, int n, bool out64, hipStream_t stream) {
    constexpr int V = 4;
    MultiArgs a{};
    a.n = n;
    a.oh_max = 0;
    int64_t ow_max = 0, h_max = 0;
    for (int i = 0; i < n; ++i) {
        a.d[i] = descs[i];
        if (descs[i].oh > a.oh_max) a.oh_max = descs[i].oh;
        if (descs[i].ow > ow_max) ow_max = descs[i].ow;
        if (descs[i].win_h > h_max) h_max = descs[i].win_h;
    }
    a.chunks = (ow_max + 256 * V - 1) / (256 * V);
    GatherDesc shape = descs[0];
    shape.chunks = a.chunks;
    const int64_t band = band_chunks(shape, V, true, h_max);
    const dim3 grid(static_cast<unsigned>(a.oh_max * a.chunks));
    if (out64) hipLaunchKernelGGL((window_sum_multi_kernel<uint64_t, V>), grid, dim3(256), 0, stream, a, band);
    else hipLaunchKernelGGL((window_sum_multi_kernel<uint32_t, V>), grid, dim3(256), 0, stream, a, band);
    return hipGetLastError();
}

hipError_t launch_mean_std(const GatherDesc *descs, int n, const GatherDesc *dev_descs, int64_t total_items,
                           hipStream_t stream) {
    constexpr int V = 2;
    if (n == 1) {
        GatherDesc d = descs[0];
        d.chunks = (d.ow + 256 * V - 1) / (256 * V);
        const int64_t band = band_chunks(d, V, true, d.win_h);
        hipLaunchKernelGGL((mean_std_kernel<V>), dim3(static_cast<unsigned>(d.oh * d.chunks)), dim3(256), 0,
                           stream, d, nullptr, 1, band);
    } else {
        hipLaunchKernelGGL((mean_std_kernel<V>), dim3(static_cast<unsigned>(total_items)), dim3(256), 0, stream,
                           descs[0], dev_descs, n, int64_t(1));
    }
    return hipGetLastError();
}

}  // namespace satk
