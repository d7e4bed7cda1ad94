// sat_gather.hip -- window statistics from integral images by the four-corner lookup.
//
// A window sum is the table value at the window's bottom-right corner, minus the value just above
// the window at its right edge, minus the value just left of it at its bottom edge, plus the
// value diagonally above-left (Sec. II-B); one output per window position of the valid region
// (Sec. II-A, Sec. III-A), four lookups each (the 4(r*c) term of Sec. III-B).
//
// The kernels are bound by HBM bandwidth, and what they cost is how often each table row is
// read.  Two families:
//
//   chain gathers (the default): output rows k and k + q of a window of height h share a table
//     row when q * stride == h -- the row just above output row k + q is the bottom row of
//     output row k.  For windows of heights h_1..h_n that are all multiples of the stride and
//     q = gcd(h_i / stride), every row that output rows r, r + q, r + 2q, ... of ANY of the
//     windows read is one of the rows (r + jq) * stride - 1.  A work item walks one such chain
//     down a chunk of output columns and reads each of those rows once; per row t and window i
//     it forms the difference of the window's two corner columns
//         D_i(t)[l] = T(t, l*stride + w_i - 1) - T(t, l*stride - 1),
//     and the sum of the window at chain position p is D_i at step p + L_i minus D_i at step
//     p, L_i = h_i / (q * stride).  The table is read about once per gather, for all windows
//     together, instead of twice per window.
//   row-pair gathers: one output row segment per work item, reading its two table rows; used
//     when a window height is not a multiple of the stride (no two output rows share a row).
#include "sat_internal.h"
#include "sat_chain_stats.h"

namespace satk {
namespace {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

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
// The four corner entries of one window, as E: 32-bit outputs (sums mod 2^32) need only the low
// word of each table entry, so they load half the bytes.
template <typename E>
struct Corners {
    E b1, b0, t1, t0;
};

template <typename E>
__device__ __forceinline__ Corners<E> load_corners(const uint64_t *__restrict__ top, const uint64_t *__restrict__ bot,
                                                   int64_t l, const GatherDesc &d) {
    const int64_t lc = l < d.ow ? l : d.ow - 1;
    const int64_t x0 = lc * d.stride;
    const int64_t x1 = x0 + d.win_w - 1;
    const int64_t xm = x0 > 0 ? x0 - 1 : 0;
    Corners<E> c;
    if constexpr (sizeof(E) == 4) {
        const uint32_t *b32 = reinterpret_cast<const uint32_t *>(bot), *t32 = reinterpret_cast<const uint32_t *>(top);
        c.b1 = b32[2 * x1];
        c.b0 = b32[2 * xm];
        c.t1 = t32[2 * x1];
        c.t0 = t32[2 * xm];
    } else {
        c.b1 = bot[x1];
        c.b0 = bot[xm];
        c.t1 = top[x1];
        c.t0 = top[xm];
    }
    return c;
}

template <typename E>
__device__ __forceinline__ E corner_sum(const Corners<E> &c, int64_t l, const GatherDesc &d, bool has_top) {
    const bool has_left = l * d.stride > 0;
    const E b0 = has_left ? c.b0 : E(0);
    const E t1 = has_top ? c.t1 : E(0);
    const E t0 = (has_top && has_left) ? c.t0 : E(0);
    return static_cast<E>(c.b1 - t1 - b0 + t0);
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
    Corners<OutT> c[V];
#pragma unroll
    for (int v = 0; v < V; ++v) c[v] = load_corners<OutT>(top, bot, l0 + v * 256, d);
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
        Corners<OutT> c[V];
#pragma unroll
        for (int v = 0; v < V; ++v) c[v] = load_corners<OutT>(top, bot, l0 + v * 256, d);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int64_t l = l0 + v * 256;
            if (l < d.ow) out[l] = static_cast<OutT>(corner_sum(c[v], l, d, has_top));
        }
    }
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
    const int64_t l0 = c * (256 * V) + threadIdx.x;
    Corners<uint64_t> cs[V], cq[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        cs[v] = load_corners<uint64_t>(topS, botS, l0 + v * 256, d);
        cq[v] = load_corners<uint64_t>(topQ, botQ, l0 + v * 256, d);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t l = l0 + v * 256;
        if (l < d.ow) {
            stats_store(d, k * d.opitch + l, corner_sum(cs[v], l, d, has_top), corner_sum(cq[v], l, d, has_top), n,
                        dn);
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

// ------------------------------------------------------------------ chain gathers

constexpr int kChainMaxWin = 4;       // windows per chain launch (more are split into groups)
constexpr int kRingBytes = 48 << 10;  // LDS ring budget per workgroup

// Work item -> (XCD slice, position): workgroup b is dispatched to XCD b mod 8, so consecutive
// work items are given to consecutive workgroups of one XCD; neighbouring column chunks, which
// read overlapping table columns of the same rows at the same time, then share that XCD's L2.
__device__ __forceinline__ int64_t xcd_item(int64_t per_xcd) {
    const int64_t b = blockIdx.x;
    return per_xcd > 0 ? (b & 7) * per_xcd + (b >> 3) : b;
}

struct ChainWin {
    void *out;
    int64_t opitch;
    int64_t oh, ow;
    int32_t w;        // window width
    int32_t L;        // chain steps from a window's top row to its bottom row
    int32_t ring0;    // first ring slot of this window
    int32_t pad;
};

struct ChainArgs {
    const uint64_t *S;
    int64_t spitch;
    int64_t stride;
    int64_t q, seg, chunks, items, per_xcd;
    int64_t ow_max;
    ChainWin win[kChainMaxWin];
};

// Table entries of one chain row, in the output type: sums mod 2^32 need only the low word of
// each entry, so 32-bit outputs load half the bytes.
template <typename E, int V, int N>
struct ChainRow {
    E left[V];
    E right[N][V];
};

template <typename OutT, int V, int N>
__global__ __launch_bounds__(256) void chain_sum_kernel(ChainArgs a) {
    extern __shared__ __align__(16) unsigned char ring_raw[];   // N > 1: sum(L_i) slots x V x 256 OutT
    OutT *ring = reinterpret_cast<OutT *>(ring_raw);
    const int64_t item = xcd_item(a.per_xcd);
    if (item >= a.items) return;
    const ChainItem it = chain_item(item, a.chunks, a.q, a.seg);
    int64_t pend[N];
    int64_t jlast = -1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        pend[i] = chain_end(a.win[i].oh, it.r, a.q, it.j0, a.seg);
        if (pend[i] >= it.j0 && pend[i] + a.win[i].L > jlast) jlast = pend[i] + a.win[i].L;
    }
    if (jlast < it.j0) return;

    const int tid = threadIdx.x;
    const int32_t s = static_cast<int32_t>(a.stride);
    int32_t lx[V], xl[V], xr[N][V];
    bool has_left[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        lx[v] = static_cast<int32_t>(it.c * (256 * V)) + v * 256 + tid;
        const int32_t lc = lx[v] < a.ow_max ? lx[v] : static_cast<int32_t>(a.ow_max) - 1;
        has_left[v] = lc > 0;
        xl[v] = lc > 0 ? lc * s - 1 : 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int32_t li = lx[v] < a.win[i].ow ? lx[v] : static_cast<int32_t>(a.win[i].ow) - 1;
            xr[i][v] = li * s + a.win[i].w - 1;
        }
    }
    auto load = [&](int64_t j, ChainRow<OutT, V, N> &row) {
        const int64_t t = (it.r + j * a.q) * a.stride - 1;
        const uint64_t *p = a.S + (t > 0 ? t : 0) * a.spitch;
        if constexpr (sizeof(OutT) == 4) {
            const uint32_t *p32 = reinterpret_cast<const uint32_t *>(p);     // low words
#pragma unroll
            for (int v = 0; v < V; ++v) row.left[v] = p32[2 * static_cast<int64_t>(xl[v])];
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int v = 0; v < V; ++v) row.right[i][v] = p32[2 * static_cast<int64_t>(xr[i][v])];
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) row.left[v] = p[xl[v]];
#pragma unroll
            for (int i = 0; i < N; ++i)
#pragma unroll
                for (int v = 0; v < V; ++v) row.right[i][v] = p[xr[i][v]];
        }
    };

    ChainRow<OutT, V, N> cur, nxt;
    OutT prev[V];
    int slot[N];
#pragma unroll
    for (int i = 0; i < N; ++i) slot[i] = 0;
    load(it.j0, cur);
#pragma unroll 1
    for (int64_t j = it.j0; j <= jlast; ++j) {
        if (j < jlast) load(j + 1, nxt);
        const bool row_ok = it.r + j * a.q > 0;     // row (r + jq) * stride - 1 exists
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const ChainWin &cw = a.win[i];
            OutT D[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const OutT lv = has_left[v] ? cur.left[v] : OutT(0);
                D[v] = row_ok ? static_cast<OutT>(cur.right[i][v] - lv) : OutT(0);
            }
            const int64_t p = j - cw.L;
            OutT *rs = N > 1 ? ring + static_cast<int64_t>(cw.ring0 + slot[i]) * (V * 256) : nullptr;
            if (p >= it.j0 && p <= pend[i]) {
                OutT *o = static_cast<OutT *>(cw.out) + (it.r + p * a.q) * cw.opitch;
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const OutT top = N > 1 ? rs[v * 256 + tid] : prev[v];
                    if (lx[v] < cw.ow) __builtin_nontemporal_store(static_cast<OutT>(D[v] - top), o + lx[v]);
                }
            }
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (N > 1) rs[v * 256 + tid] = D[v];
                else prev[v] = D[v];
            }
            if (N > 1) slot[i] = slot[i] + 1 == cw.L ? 0 : slot[i] + 1;
        }
        cur = nxt;
    }
}

// Mean and standard deviation (single image, or a batch through a descriptor table) by chain
// walks over both tables: one read of each table row of S and Q per gather.
template <int V>
__global__ __launch_bounds__(256) void chain_stats_kernel(GatherDesc one, const GatherDesc *__restrict__ many,
                                                          int n, int64_t total, int64_t per_xcd) {
    int64_t item = xcd_item(per_xcd);
    if (item >= total) return;
    GatherDesc d;
    if (many == nullptr) {
        d = one;
    } else {
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (many[mid].first_item <= item) lo = mid;
            else hi = mid - 1;
        }
        d = many[lo];
        item -= d.first_item;
    }
    chain_stats_item<V>(d, item);
}

// Stride-1 chain walk with the row span staged in LDS.  A work item owns kLdsC consecutive
// outputs; at every chain step its workgroup loads the table row's span of columns
// [x0 - 1, x0 + kLdsC + w_max - 1) once, keeps it (in the output type: sums mod 2^32 for 32-bit
// outputs) in a ring of L_max + 1 rows shared by all windows, and forms each output as
//     (T_j[l + w - 1] - T_{j-L}[l + w - 1]) - (T_j[l - 1] - T_{j-L}[l - 1]),
// the vertical difference over the window's lag taken at the window's two corner columns.  One
// chunk reads its span once, so the corner columns reaching past the chunk cost w_max / kLdsC
// extra instead of a second read by the neighbouring chunk.  Two rows are in flight (the loop is
// unrolled by two with unconditional, clamped loads) and every output store is issued through a
// range-checked buffer resource, so the wait counts the compiler derives stay exact.
constexpr int kLdsBS = 256;
constexpr int kLdsV = 4;
constexpr int kLdsC = kLdsBS * kLdsV;
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer resource, 32-bit data format

template <typename OutT, int N, int NL>
__global__ __launch_bounds__(kLdsBS) void chain_lds_kernel(ChainArgs a, int32_t span, int32_t nslot) {
    extern __shared__ __align__(16) unsigned char ring_raw[];
    OutT *ring = reinterpret_cast<OutT *>(ring_raw);
    const int64_t item = xcd_item(a.per_xcd);
    if (item >= a.items) return;
    const ChainItem it = chain_item(item, a.chunks, a.q, a.seg);
    int64_t pend[N];
    int64_t jlast = -1;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        pend[i] = chain_end(a.win[i].oh, it.r, a.q, it.j0, a.seg);
        if (pend[i] >= it.j0 && pend[i] + a.win[i].L > jlast) jlast = pend[i] + a.win[i].L;
    }
    if (jlast < it.j0) return;
    const int tid = threadIdx.x;
    const int64_t x0 = it.c * kLdsC;
    const int64_t W = a.win[0].ow + a.win[0].w - 1;       // table width (stride 1)
    int32_t colk[NL];
    bool inside[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int kk = k * kLdsBS + tid;
        const int64_t col = x0 - 1 + kk;
        inside[k] = kk < span && col >= 0 && col < W;
        colk[k] = static_cast<int32_t>(col < 0 ? 0 : (col > W - 1 ? W - 1 : col));
    }
    // The ring keeps table values in the output type (sums mod 2^32 for 32-bit outputs need only
    // the low word of each entry), so 32-bit outputs load only low words: the dead high halves of
    // 64-bit loads were reused as registers for the LDS reads, which then had to wait for the
    // table row loaded ahead, and the prefetch bought nothing.
    auto gload = [&](int64_t j, OutT (&pre)[NL]) {
        const int64_t jj = j <= jlast ? j : jlast;
        const int64_t t = it.r + jj * a.q - 1;
        const uint64_t *p = a.S + (t > 0 ? t : 0) * a.spitch;
        if constexpr (sizeof(OutT) == 4) {
            const uint32_t *p32 = reinterpret_cast<const uint32_t *>(p);
#pragma unroll
            for (int k = 0; k < NL; ++k) pre[k] = p32[2 * static_cast<int64_t>(colk[k])];
        } else {
#pragma unroll
            for (int k = 0; k < NL; ++k) pre[k] = p[colk[k]];
        }
    };
    int slot = static_cast<int>(it.j0 % nslot);
    auto step = [&](int64_t j, const OutT (&pre)[NL]) {
        __syncthreads();                                   // the slot reused now was last read a step ago
        const bool rowok = it.r + j * a.q > 0;             // row -1 is all zero
        OutT *dst = ring + slot * span;
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const int kk = k * kLdsBS + tid;
            if (kk < span) dst[kk] = (rowok && inside[k]) ? pre[k] : OutT(0);
        }
        __syncthreads();
        const OutT *cur = dst;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const ChainWin &cw = a.win[i];
            const int64_t p = j - cw.L;
            const bool emit = p >= it.j0 && p <= pend[i];
            int so = slot - cw.L;
            so += so < 0 ? nslot : 0;
            const OutT *old = ring + so * span;
            const int64_t prow = emit ? p : it.j0;
            OutT *rowp = static_cast<OutT *>(cw.out) + (it.r + prow * a.q) * cw.opitch + x0;
            const int64_t remain = cw.ow - x0;
            const int nrec = emit ? static_cast<int>((remain > 0 ? (remain < kLdsC ? remain : kLdsC) : 0) *
                                                     static_cast<int64_t>(sizeof(OutT)))
                                  : 0;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(rowp, 0, nrec, kRsrcWord3);
#pragma unroll
            for (int v = 0; v < kLdsV; ++v) {
                const int u = v * kLdsBS + tid;
                const OutT val = static_cast<OutT>((cur[u + cw.w] - old[u + cw.w]) - (cur[u] - old[u]));
                if constexpr (sizeof(OutT) == 8)
                    __builtin_amdgcn_raw_buffer_store_b64(u32x2{static_cast<uint32_t>(val),
                                                                static_cast<uint32_t>(static_cast<uint64_t>(val) >> 32)},
                                                          rs, u * 8, 0, 2);
                else
                    __builtin_amdgcn_raw_buffer_store_b32(static_cast<uint32_t>(val), rs, u * 4, 0, 2);
            }
        }
        slot = slot + 1 == nslot ? 0 : slot + 1;
    };
    OutT pre0[NL], pre1[NL];
    gload(it.j0, pre0);
    gload(it.j0 + 1, pre1);
#pragma unroll 1
    for (int64_t j = it.j0; j <= jlast; j += 2) {
        step(j, pre0);
        gload(j + 2, pre0);
        if (j + 1 > jlast) break;
        step(j + 1, pre1);
        gload(j + 3, pre1);
    }
}

// ------------------------------------------------------------------ variants and launch

enum GatherKind { G_CHAIN = 0, G_ROWPAIR = 1 };
struct GatherVariant {
    const char *name;
    int kind;       // GatherKind
    int v;          // outputs per thread per step
    int banded;     // row-pair: 1 = column bands sized to the window height; 0 = row-major
};
const GatherVariant kGather[] = {
    {"chain_auto", G_CHAIN, 0, 0},     // LDS-staged where it applies, else the ring of corner differences
    {"chain_v2", G_CHAIN, 2, 0},
    {"chain_v1", G_CHAIN, 1, 0},
    {"chain_v4", G_CHAIN, 4, 0},
    {"rowpair_v4_banded", G_ROWPAIR, 4, 1},
    {"rowpair_v2_banded", G_ROWPAIR, 2, 1},
    {"rowpair_v8_banded", G_ROWPAIR, 8, 1},
    {"rowpair_v4_rowmajor", G_ROWPAIR, 4, 0},
};
constexpr int kNumGather = sizeof(kGather) / sizeof(kGather[0]);
constexpr int kRowPairFallback = 4;

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

int device_cus() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0, v = 0;
        cus = (hipGetDevice(&dev) == hipSuccess &&
               hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
                  ? v
                  : 256;
    }
    return cus;
}

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// Split of a chain gather into work items: `base` = residues x column chunks of the launch, P =
// chain positions of the longest chain.  Chains are cut into segments only as far as needed for
// about 32 workgroups per CU, and never below 16 steps per slowest-window lag (a segment re-reads
// the L rows before its first output).
int64_t chain_segments(int64_t base, int64_t P, int Lmax) {
    const int64_t target = 32ll * device_cus();
    int64_t nseg = (target + base - 1) / base;
    const int64_t min_seg = 16ll * (Lmax > 1 ? Lmax : 1);
    int64_t cap = P / min_seg;
    if (cap < 1) cap = 1;
    if (nseg > cap) nseg = cap;
    if (nseg < 1) nseg = 1;
    return (P + nseg - 1) / nseg;    // segment length
}

void xcd_grid(int64_t items, int64_t *grid, int64_t *per_xcd) {
    const int64_t per = (items + 7) / 8;
    *grid = per * 8;
    *per_xcd = per;
}

template <typename OutT, int V, int N>
hipError_t launch_chain_typed(ChainArgs &a, size_t lds, hipStream_t s) {
    int64_t grid = 0;
    xcd_grid(a.items, &grid, &a.per_xcd);
    hipLaunchKernelGGL((chain_sum_kernel<OutT, V, N>), dim3(static_cast<unsigned>(grid)), dim3(256), lds, s, a);
    return hipGetLastError();
}

template <typename OutT, int V>
hipError_t launch_chain_n(ChainArgs &a, int n, size_t lds, hipStream_t s) {
    switch (n) {
        case 1: return launch_chain_typed<OutT, V, 1>(a, 0, s);
        case 2: return launch_chain_typed<OutT, V, 2>(a, lds, s);
        case 3: return launch_chain_typed<OutT, V, 3>(a, lds, s);
        default: return launch_chain_typed<OutT, V, 4>(a, lds, s);
    }
}

// Outputs per thread of a chain launch: the variant's, or for the automatic variant one per
// thread without a lag ring and two with one (measured fastest on 70000 x 85000 tables).
int chain_v(const GatherVariant &g, int n_windows) { return g.v > 0 ? g.v : (n_windows > 1 ? 2 : 1); }

// Outputs per thread of a mean/std chain launch: with a stride above one each output reads a
// fraction of a cache line, and four outputs per thread keep more lines in flight (measured on
// 64 uneven 16-bit images at stride 4); one at stride 1.
// Outputs per thread of the mean/std chain walk: four, at every stride (at 32768^2 and stride 1
// 8.9 ms against 9.4-9.7 ms with one; equal at 8192^2).
int stats_v(const GatherVariant &g, int64_t) { return g.v > 0 ? g.v : 4; }

// LDS-staged chain launches: spans of up to NL * 256 columns are compiled for these NL.
constexpr int kLdsNL[] = {5, 6, 8, 12};
constexpr size_t kLdsMaxBytes = 150 << 10;

// Loads per thread, span and LDS bytes of an LDS-staged launch, or false where it does not apply.
bool lds_plan(int64_t stride, int64_t wmax, int Lmax, bool out64, int *nl, int *span, size_t *lds) {
    if (stride != 1) return false;
    const int64_t sp = kLdsC + wmax;
    const int64_t need = (sp + kLdsBS - 1) / kLdsBS;
    int pick = 0;
    for (int c : kLdsNL)
        if (c >= need) {
            pick = c;
            break;
        }
    if (pick == 0) return false;
    const size_t bytes = static_cast<size_t>(Lmax + 1) * static_cast<size_t>(sp) * (out64 ? 8 : 4);
    if (bytes > kLdsMaxBytes) return false;
    *nl = pick;
    *span = static_cast<int>(sp);
    *lds = bytes;
    return true;
}

template <typename OutT, int N, int NL>
hipError_t launch_lds_typed(ChainArgs &a, int span, int nslot, size_t lds, hipStream_t s) {
    static bool attr_set = false;      // the maximum is set once per instantiation
    const void *fn = reinterpret_cast<const void *>(&chain_lds_kernel<OutT, N, NL>);
    if (!attr_set && lds > (64u << 10)) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsMaxBytes));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int64_t grid = 0;
    xcd_grid(a.items, &grid, &a.per_xcd);
    hipLaunchKernelGGL((chain_lds_kernel<OutT, N, NL>), dim3(static_cast<unsigned>(grid)), dim3(kLdsBS), lds, s, a,
                       static_cast<int32_t>(span), static_cast<int32_t>(nslot));
    return hipGetLastError();
}

template <typename OutT, int N>
hipError_t launch_lds_n(ChainArgs &a, int nl, int span, int nslot, size_t lds, hipStream_t s) {
    switch (nl) {
        case 5: return launch_lds_typed<OutT, N, 5>(a, span, nslot, lds, s);
        case 6: return launch_lds_typed<OutT, N, 6>(a, span, nslot, lds, s);
        case 8: return launch_lds_typed<OutT, N, 8>(a, span, nslot, lds, s);
        default: return launch_lds_typed<OutT, N, 12>(a, span, nslot, lds, s);
    }
}

template <typename OutT>
hipError_t launch_lds(ChainArgs &a, int n, int nl, int span, int nslot, size_t lds, hipStream_t s) {
    switch (n) {
        case 1: return launch_lds_n<OutT, 1>(a, nl, span, nslot, lds, s);
        case 2: return launch_lds_n<OutT, 2>(a, nl, span, nslot, lds, s);
        case 3: return launch_lds_n<OutT, 3>(a, nl, span, nslot, lds, s);
        default: return launch_lds_n<OutT, 4>(a, nl, span, nslot, lds, s);
    }
}

// One chain launch over windows idx[0..n) of d (all heights multiples of the stride, ring fits).
// allow_lds: use the LDS-staged kernel where it applies (stride 1, span within the LDS budget).
hipError_t launch_chain_group(int V, const GatherDesc *d, const int *idx, int n, bool out64, hipStream_t s,
                              bool allow_lds = false) {
    ChainArgs a{};
    a.S = d[idx[0]].S;
    a.spitch = d[idx[0]].spitch;
    a.stride = d[idx[0]].stride;
    int64_t q = 0, oh_max = 0, ow_max = 0;
    for (int i = 0; i < n; ++i) q = gcd64(q, d[idx[i]].win_h / a.stride);
    int slots = 0, Lmax = 1;
    for (int i = 0; i < n; ++i) {
        const GatherDesc &g = d[idx[i]];
        ChainWin &w = a.win[i];
        w.out = g.out;
        w.opitch = g.opitch;
        w.oh = g.oh;
        w.ow = g.ow;
        w.w = static_cast<int32_t>(g.win_w);
        w.L = static_cast<int32_t>(g.win_h / (a.stride * q));
        w.ring0 = slots;
        slots += w.L;
        if (w.L > Lmax) Lmax = w.L;
        if (g.oh > oh_max) oh_max = g.oh;
        if (g.ow > ow_max) ow_max = g.ow;
    }
    a.q = q;
    a.ow_max = ow_max;
    int64_t wmax = 0;
    for (int i = 0; i < n; ++i) wmax = d[idx[i]].win_w > wmax ? d[idx[i]].win_w : wmax;
    int nl = 0, span = 0;
    size_t lds_bytes = 0;
    if (allow_lds && lds_plan(a.stride, wmax, Lmax, out64, &nl, &span, &lds_bytes)) {
        a.chunks = (ow_max + kLdsC - 1) / kLdsC;
        const int64_t P = (oh_max + q - 1) / q;
        a.seg = chain_segments(q * a.chunks, P, Lmax);
        a.items = q * a.chunks * ((P + a.seg - 1) / a.seg);
        return out64 ? launch_lds<uint64_t>(a, n, nl, span, Lmax + 1, lds_bytes, s)
                     : launch_lds<uint32_t>(a, n, nl, span, Lmax + 1, lds_bytes, s);
    }
    a.chunks = (ow_max + 256 * V - 1) / (256 * V);
    const int64_t P = (oh_max + q - 1) / q;
    a.seg = chain_segments(q * a.chunks, P, Lmax);
    a.items = q * a.chunks * ((P + a.seg - 1) / a.seg);
    const size_t lds = static_cast<size_t>(slots) * V * 256 * (out64 ? 8 : 4);
    switch (V) {
        case 1: return out64 ? launch_chain_n<uint64_t, 1>(a, n, lds, s) : launch_chain_n<uint32_t, 1>(a, n, lds, s);
        case 4: return out64 ? launch_chain_n<uint64_t, 4>(a, n, lds, s) : launch_chain_n<uint32_t, 4>(a, n, lds, s);
        default: return out64 ? launch_chain_n<uint64_t, 2>(a, n, lds, s) : launch_chain_n<uint32_t, 2>(a, n, lds, s);
    }
}

template <typename OutT>
hipError_t launch_rowpair_typed(int v, const GatherDesc &d0, bool banded, hipStream_t s) {
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

// Row-pair pass over several windows sharing the upper row (any heights).
hipError_t launch_rowpair_multi(const GatherDesc *descs, const int *idx, int n, bool out64, hipStream_t stream) {
    constexpr int V = 4;
    MultiArgs a{};
    a.n = n;
    a.oh_max = 0;
    int64_t ow_max = 0, h_max = 0;
    for (int i = 0; i < n; ++i) {
        const GatherDesc &g = descs[idx[i]];
        a.d[i] = g;
        if (g.oh > a.oh_max) a.oh_max = g.oh;
        if (g.ow > ow_max) ow_max = g.ow;
        if (g.win_h > h_max) h_max = g.win_h;
    }
    a.chunks = (ow_max + 256 * V - 1) / (256 * V);
    GatherDesc shape = descs[idx[0]];
    shape.chunks = a.chunks;
    const int64_t band = band_chunks(shape, V, true, h_max);
    const dim3 grid(static_cast<unsigned>(a.oh_max * a.chunks));
    if (out64) hipLaunchKernelGGL((window_sum_multi_kernel<uint64_t, V>), grid, dim3(256), 0, stream, a, band);
    else hipLaunchKernelGGL((window_sum_multi_kernel<uint32_t, V>), grid, dim3(256), 0, stream, a, band);
    return hipGetLastError();
}

bool chain_ok(const GatherDesc &d) { return d.win_h % d.stride == 0; }

}  // namespace

int mean_std_chain_v(int variant, int64_t stride) { return stats_v(kGather[variant], stride); }

int gather_variant_count() { return kNumGather; }
const char *gather_variant_name(int v) { return kGather[v].name; }

hipError_t launch_window_sum(int variant, const GatherDesc &d, bool out64, hipStream_t stream) {
    const GatherVariant *g = &kGather[variant];
    if (g->kind == G_CHAIN && chain_ok(d)) {
        const int idx = 0;
        return launch_chain_group(chain_v(*g, 1), &d, &idx, 1, out64, stream, g->v == 0);
    }
    if (g->kind == G_CHAIN) g = &kGather[kRowPairFallback];
    return out64 ? launch_rowpair_typed<uint64_t>(g->v, d, g->banded != 0, stream)
                 : launch_rowpair_typed<uint32_t>(g->v, d, g->banded != 0, stream);
}

hipError_t launch_window_sum_multi(int variant, const GatherDesc *descs, int n, bool out64, hipStream_t stream) {
    const GatherVariant &g = kGather[variant];
    int order[8], nc = 0, rest[8], nr = 0;
    for (int i = 0; i < n; ++i) {
        if (g.kind == G_CHAIN && chain_ok(descs[i])) order[nc++] = i;
        else rest[nr++] = i;
    }
    // chain groups: windows by height, greedily while the lag rings fit the LDS budget
    for (int a = 1; a < nc; ++a)
        for (int b = a; b > 0 && descs[order[b]].win_h < descs[order[b - 1]].win_h; --b) {
            const int t = order[b];
            order[b] = order[b - 1];
            order[b - 1] = t;
        }
    const int64_t slot_bytes = static_cast<int64_t>(chain_v(g, 2)) * 256 * (out64 ? 8 : 4);
    int i = 0;
    while (i < nc) {
        int m = 1;
        while (i + m < nc && m < kChainMaxWin) {
            const int64_t s = descs[order[i]].stride;
            int64_t q = 0;
            for (int k = 0; k <= m; ++k) q = gcd64(q, descs[order[i + k]].win_h / s);
            int64_t slots = 0;
            for (int k = 0; k <= m; ++k) slots += descs[order[i + k]].win_h / (s * q);
            if (slots * slot_bytes > kRingBytes) break;
            ++m;
        }
        hipError_t e = launch_chain_group(chain_v(g, m), descs, order + i, m, out64, stream, g.v == 0);
        if (e != hipSuccess) return e;
        i += m;
    }
    if (nr > 0) return launch_rowpair_multi(descs, rest, nr, out64, stream);
    return hipSuccess;
}

int64_t plan_mean_std(int variant, GatherDesc *descs, int n) {
    const GatherVariant &g = kGather[variant];
    const bool chain = g.kind == G_CHAIN && chain_ok(descs[0]);
    int64_t total = 0;
    if (!chain) {
        for (int i = 0; i < n; ++i) {
            descs[i].chunks = (descs[i].ow + 511) / 512;
            descs[i].q = 0;
            descs[i].seg = 0;
            descs[i].first_item = total;
            total += descs[i].oh * descs[i].chunks;
        }
        return total;
    }
    const int V = stats_v(g, descs[0].stride);
    const int64_t q = descs[0].win_h / descs[0].stride;
    int64_t base = 0, P = 0;
    for (int i = 0; i < n; ++i) {
        descs[i].chunks = (descs[i].ow + 256 * V - 1) / (256 * V);
        base += q * descs[i].chunks;
        const int64_t Pi = (descs[i].oh + q - 1) / q;
        if (Pi > P) P = Pi;
    }
    const int64_t seg = chain_segments(base, P, 1);
    for (int i = 0; i < n; ++i) {
        const int64_t Pi = (descs[i].oh + q - 1) / q;
        descs[i].q = q;
        descs[i].seg = seg;
        descs[i].first_item = total;
        total += q * descs[i].chunks * ((Pi + seg - 1) / seg);
    }
    return total;
}

hipError_t launch_mean_std(int variant, const GatherDesc *descs, int n, const GatherDesc *dev_descs,
                           int64_t total_items, hipStream_t stream) {
    const GatherVariant &g = kGather[variant];
    const bool chain = descs[0].q > 0;
    if (chain) {
        int64_t grid = 0, per = 0;
        xcd_grid(total_items, &grid, &per);
        const dim3 gr(static_cast<unsigned>(grid));
        const GatherDesc *many = n == 1 ? nullptr : dev_descs;
        switch (stats_v(g, descs[0].stride)) {
            case 1: hipLaunchKernelGGL((chain_stats_kernel<1>), gr, dim3(256), 0, stream, descs[0], many, n, total_items, per); break;
            case 4: hipLaunchKernelGGL((chain_stats_kernel<4>), gr, dim3(256), 0, stream, descs[0], many, n, total_items, per); break;
            default: hipLaunchKernelGGL((chain_stats_kernel<2>), gr, dim3(256), 0, stream, descs[0], many, n, total_items, per); break;
        }
        return hipGetLastError();
    }
    constexpr int V = 2;
    if (n == 1) {
        GatherDesc d = descs[0];
        const int64_t band = band_chunks(d, V, true, d.win_h);
        hipLaunchKernelGGL((mean_std_kernel<V>), dim3(static_cast<unsigned>(d.oh * d.chunks)), dim3(256), 0,
                           stream, d, nullptr, 1, band);
    } else {
        hipLaunchKernelGGL((mean_std_kernel<V>), dim3(static_cast<unsigned>(total_items)), dim3(256), 0, stream,
                           descs[0], dev_descs, n, int64_t(1));
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ higher window moments
//
// Window statistics beyond mean and std from tables of pixel powers (the method applied to
// I^k): with S_k the window sum of pixel^k over n pixels (four-corner lookups, exact), the
// central moments expand into the raw sums by the binomial theorem,
//   A = n*S2 - S1^2 = n^2 m2,   B = n^2*S3 - 3n*S1*S2 + 2*S1^3 = n^3 m3,
//   C = n^3*S4 - 4n^2*S1*S3 + 6n*S1^2*S2 - 3*S1^4 = n^4 m4,
// formed exactly in signed 128-bit integers (the host bounds n and the pixel range so that no
// term overflows) and rounded to double once each:
//   mean = S1/n, std = sqrt(A)/n, skewness = B / (A*sqrt(A)), excess kurtosis = (C - 3A^2)/(A*A),
// population moments; skewness and kurtosis are NaN where A = 0.  Where the window height is a
// multiple of the stride the outputs come from chain walks (each table row of every power read
// once, as for the mean and deviation); otherwise one output row segment per work item reads
// the two table rows of each power (row pairs, banded for L2 reuse).

namespace {

typedef __int128 i128;

__device__ __forceinline__ double i128_to_double(i128 x) {
    const bool neg = x < 0;
    const unsigned __int128 u = neg ? static_cast<unsigned __int128>(-x) : static_cast<unsigned __int128>(x);
    const double r = u128_to_double(static_cast<uint64_t>(u >> 64), static_cast<uint64_t>(u));
    return neg ? -r : r;
}

// 64 x 64 -> 128-bit products, the only wide multiplications below.
__device__ __forceinline__ i128 mul64(uint64_t x, uint64_t y) {
    return static_cast<i128>(static_cast<unsigned __int128>(x) * y);
}

// The numerators in factored forms with few wide products (the same integers as the expansions
// above): with D = n*S3 - S1*S2 and F = n*S4 - 4*S1*S3 + 3*S2^2,
//   B = n*D - 2*S1*A,    C - 3A^2 = n^2*F - 6*A^2.
// n <= 2^32, so n^2 fits 64 bits; where the kurtosis is allowed, A < 2^63.
template <int K>
__device__ __forceinline__ void moments_store(const MomentDesc &d, int64_t o, const uint64_t (&s)[K], uint64_t n,
                                              double dn) {
    if (d.mean) __builtin_nontemporal_store(static_cast<double>(s[0]) / dn, d.mean + o);
    if constexpr (K >= 2) {
        const i128 A = mul64(n, s[1]) - mul64(s[0], s[0]);
        const double a = i128_to_double(A);
        const double ra = sqrt(a);
        if (d.stdv) __builtin_nontemporal_store(ra / dn, d.stdv + o);
        if constexpr (K >= 3) {
            if (d.skew) {
                const i128 D = mul64(n, s[2]) - mul64(s[0], s[1]);
                const i128 B = static_cast<i128>(n) * D - 2 * static_cast<i128>(s[0]) * A;
                __builtin_nontemporal_store(A == 0 ? __builtin_nan("") : i128_to_double(B) / (a * ra), d.skew + o);
            }
            if constexpr (K >= 4) {
                if (d.kurt) {
                    const i128 F = mul64(n, s[3]) - 4 * mul64(s[0], s[2]) + 3 * mul64(s[1], s[1]);
                    const uint64_t a64 = static_cast<uint64_t>(A);
                    const i128 E = static_cast<i128>(n * n) * F - 6 * mul64(a64, a64);
                    __builtin_nontemporal_store(A == 0 ? __builtin_nan("") : i128_to_double(E) / (a * a), d.kurt + o);
                }
            }
        }
    }
}

template <int K, int V>
__global__ __launch_bounds__(256) void moments_kernel(MomentDesc d, int64_t band) {
    const ItemMap m = map_item(blockIdx.x, d.oh, d.chunks, band);
    GatherDesc g{};
    g.ow = d.ow;
    g.stride = d.stride;
    g.win_w = d.win_w;
    const int64_t y0 = m.k * d.stride;
    const int64_t y1 = y0 + d.win_h - 1;
    const bool has_top = y0 > 0;
    const uint64_t n = static_cast<uint64_t>(d.win_h) * static_cast<uint64_t>(d.win_w);
    const double dn = static_cast<double>(n);
    const int64_t l0 = m.c * (256 * V) + threadIdx.x;
    Corners<uint64_t> c[K][V];
#pragma unroll
    for (int p = 0; p < K; ++p) {
        const uint64_t *bot = d.T[p] + y1 * d.spitch;
        const uint64_t *top = d.T[p] + (has_top ? y0 - 1 : 0) * d.spitch;
#pragma unroll
        for (int v = 0; v < V; ++v) c[p][v] = load_corners<uint64_t>(top, bot, l0 + v * 256, g);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t l = l0 + v * 256;
        if (l < d.ow) {
            uint64_t s[K];
#pragma unroll
            for (int p = 0; p < K; ++p) s[p] = corner_sum(c[p][v], l, g, has_top);
            moments_store<K>(d, m.k * d.opitch + l, s, n, dn);
        }
    }
}

// Chain walk over K tables: chain position j reads table row (r + j*q)*stride - 1 of every power
// once; output row r + (j-1)*q is the difference of the corner differences at positions j and
// j-1 (q*stride = win_h).
template <int K, int V>
__global__ __launch_bounds__(256) void chain_moments_kernel(MomentDesc d, int64_t q, int64_t seg, int64_t total,
                                                            int64_t per_xcd) {
    const int64_t item = xcd_item(per_xcd);
    if (item >= total) return;
    const ChainItem it = chain_item(item, d.chunks, q, seg);
    const int64_t pend = chain_end(d.oh, it.r, q, it.j0, seg);
    if (pend < it.j0) return;
    const int64_t jlast = pend + 1;
    const int tid = threadIdx.x;
    const int32_t s = static_cast<int32_t>(d.stride);
    int32_t lx[V], xl[V], xr[V];
    bool has_left[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        lx[v] = static_cast<int32_t>(it.c * (256 * V)) + v * 256 + tid;
        const int32_t lc = lx[v] < d.ow ? lx[v] : static_cast<int32_t>(d.ow) - 1;
        has_left[v] = lc > 0;
        xl[v] = lc > 0 ? lc * s - 1 : 0;
        xr[v] = lc * s + static_cast<int32_t>(d.win_w) - 1;
    }
    const uint64_t nn = static_cast<uint64_t>(d.win_h) * static_cast<uint64_t>(d.win_w);
    const double dn = static_cast<double>(nn);
    auto load = [&](int64_t j, uint64_t (&rows)[2 * K][V]) {
        const int64_t t = (it.r + j * q) * d.stride - 1;
        const int64_t off = (t > 0 ? t : 0) * d.spitch;
#pragma unroll
        for (int p = 0; p < K; ++p) {
            const uint64_t *pt = d.T[p] + off;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                rows[2 * p][v] = pt[xl[v]];
                rows[2 * p + 1][v] = pt[xr[v]];
            }
        }
    };
    uint64_t cur[2 * K][V], nxt[2 * K][V], prev[K][V];
    load(it.j0, cur);
#pragma unroll 1
    for (int64_t j = it.j0; j <= jlast; ++j) {
        if (j < jlast) load(j + 1, nxt);
        const bool row_ok = it.r + j * q > 0;
        const int64_t orow = (it.r + (j - 1) * q) * d.opitch;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            uint64_t dd[K];
#pragma unroll
            for (int p = 0; p < K; ++p) dd[p] = row_ok ? cur[2 * p + 1][v] - (has_left[v] ? cur[2 * p][v] : 0) : 0;
            if (j > it.j0 && lx[v] < d.ow) {
                uint64_t sums[K];
#pragma unroll
                for (int p = 0; p < K; ++p) sums[p] = dd[p] - prev[p][v];
                moments_store<K>(d, orow + lx[v], sums, nn, dn);
            }
#pragma unroll
            for (int p = 0; p < K; ++p) prev[p][v] = dd[p];
        }
#pragma unroll
        for (int k = 0; k < 2 * K; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) cur[k][v] = nxt[k][v];
    }
}

// Stride-1 chain walk with the row spans of all K tables staged in LDS (the scheme of
// chain_lds_kernel for one window, lag 1): a work item owns kLdsC consecutive outputs; at every
// chain step its workgroup loads the table rows' columns [x0 - 1, x0 + kLdsC + w - 1) of each
// power once into a two-slot ring, and forms each output's power sums as
//     (T_j[l + w - 1] - T_{j-1}[l + w - 1]) - (T_j[l - 1] - T_{j-1}[l - 1]).
// Two steps' loads are in flight (unrolled by two, unconditional clamped loads); the epilogue
// loop over a thread's outputs is not unrolled, to bound register use.
template <int K, int NL>
__global__ __launch_bounds__(kLdsBS) void chain_lds_moments_kernel(MomentDesc d, int64_t q, int64_t seg, int64_t total,
                                                                   int64_t per_xcd, int32_t span) {
    extern __shared__ __align__(16) unsigned char ring_raw[];
    uint64_t *ring = reinterpret_cast<uint64_t *>(ring_raw);        // [slot][power][span]
    const int64_t item = xcd_item(per_xcd);
    if (item >= total) return;
    const ChainItem it = chain_item(item, d.chunks, q, seg);
    const int64_t pend = chain_end(d.oh, it.r, q, it.j0, seg);
    if (pend < it.j0) return;
    const int64_t jlast = pend + 1;
    const int tid = threadIdx.x;
    const int64_t x0 = it.c * kLdsC;
    const int64_t W = d.ow + d.win_w - 1;                          // table width (stride 1)
    const int32_t w = static_cast<int32_t>(d.win_w);
    const uint64_t nn = static_cast<uint64_t>(d.win_h) * static_cast<uint64_t>(d.win_w);
    const double dn = static_cast<double>(nn);
    int32_t colk[NL];
    bool inside[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int kk = k * kLdsBS + tid;
        const int64_t col = x0 - 1 + kk;
        inside[k] = kk < span && col >= 0 && col < W;
        colk[k] = static_cast<int32_t>(col < 0 ? 0 : (col > W - 1 ? W - 1 : col));
    }
    auto gload = [&](int64_t j, uint64_t (&pre)[K][NL]) {
        const int64_t jj = j <= jlast ? j : jlast;
        const int64_t t = it.r + jj * q - 1;
        const int64_t off = (t > 0 ? t : 0) * d.spitch;
#pragma unroll
        for (int p = 0; p < K; ++p) {
            const uint64_t *row = d.T[p] + off;
#pragma unroll
            for (int k = 0; k < NL; ++k) pre[p][k] = row[colk[k]];
        }
    };
    int slot = static_cast<int>(it.j0 & 1);
    auto step = [&](int64_t j, const uint64_t (&pre)[K][NL]) {
        __syncthreads();                                   // the slot reused now was last read a step ago
        const bool rowok = it.r + j * q > 0;               // row -1 is all zero
        uint64_t *dst = ring + static_cast<int64_t>(slot) * K * span;
#pragma unroll
        for (int p = 0; p < K; ++p)
#pragma unroll
            for (int k = 0; k < NL; ++k) {
                const int kk = k * kLdsBS + tid;
                if (kk < span) dst[p * span + kk] = (rowok && inside[k]) ? pre[p][k] : 0;
            }
        __syncthreads();
        const int64_t prow = j - 1;                        // output position emitted at this step
        if (prow >= it.j0 && prow <= pend) {
            const uint64_t *cur = dst;
            const uint64_t *old = ring + static_cast<int64_t>(slot ^ 1) * K * span;
            const int64_t orow = (it.r + prow * q) * d.opitch + x0;
#pragma unroll 1
            for (int v = 0; v < kLdsV; ++v) {
                const int u = v * kLdsBS + tid;
                if (x0 + u < d.ow) {
                    uint64_t sums[K];
#pragma unroll
                    for (int p = 0; p < K; ++p)
                        sums[p] = (cur[p * span + u + w] - old[p * span + u + w]) - (cur[p * span + u] - old[p * span + u]);
                    moments_store<K>(d, orow + u, sums, nn, dn);
                }
            }
        }
        slot ^= 1;
    };
    uint64_t pre0[K][NL], pre1[K][NL];
    gload(it.j0, pre0);
    gload(it.j0 + 1, pre1);
#pragma unroll 1
    for (int64_t j = it.j0; j <= jlast; j += 2) {
        step(j, pre0);
        gload(j + 2, pre0);
        if (j + 1 > jlast) break;
        step(j + 1, pre1);
        gload(j + 3, pre1);
    }
}

template <int K, int NL>
hipError_t launch_lds_moments_typed(const MomentDesc &d, int64_t q, int64_t seg, int64_t total, int span, size_t lds,
                                    hipStream_t s) {
    static bool attr_set = false;      // the maximum is set once per instantiation
    const void *fn = reinterpret_cast<const void *>(&chain_lds_moments_kernel<K, NL>);
    if (!attr_set && lds > (64u << 10)) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsMaxBytes));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    int64_t grid = 0, per = 0;
    xcd_grid(total, &grid, &per);
    hipLaunchKernelGGL((chain_lds_moments_kernel<K, NL>), dim3(static_cast<unsigned>(grid)), dim3(kLdsBS), lds, s, d, q,
                       seg, total, per, static_cast<int32_t>(span));
    return hipGetLastError();
}

template <int K>
hipError_t launch_lds_moments(const MomentDesc &d, int64_t q, int64_t seg, int64_t total, int nl, int span, size_t lds,
                              hipStream_t s) {
    switch (nl) {
        case 5: return launch_lds_moments_typed<K, 5>(d, q, seg, total, span, lds, s);
        case 6: return launch_lds_moments_typed<K, 6>(d, q, seg, total, span, lds, s);
        case 8: return launch_lds_moments_typed<K, 8>(d, q, seg, total, span, lds, s);
        default: return launch_lds_moments_typed<K, 12>(d, q, seg, total, span, lds, s);
    }
}

template <int K>
void launch_chain_moments(const MomentDesc &d, int V, int64_t q, int64_t seg, int64_t total, hipStream_t stream) {
    int64_t grid = 0, per = 0;
    xcd_grid(total, &grid, &per);
    if (V == 4)
        hipLaunchKernelGGL((chain_moments_kernel<K, 4>), dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, d, q,
                           seg, total, per);
    else if (V == 2)
        hipLaunchKernelGGL((chain_moments_kernel<K, 2>), dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, d, q,
                           seg, total, per);
    else
        hipLaunchKernelGGL((chain_moments_kernel<K, 1>), dim3(static_cast<unsigned>(grid)), dim3(256), 0, stream, d, q,
                           seg, total, per);
}

}  // namespace

hipError_t launch_window_moments(int variant, int order, MomentDesc d, hipStream_t stream) {
    if (order < 1 || order > 4) return hipErrorInvalidValue;
    const GatherVariant &gv = kGather[variant];
    int nl = 0, span = 0;
    size_t lds = 0;
    // Built-in chain choice at stride 1: the LDS-staged walk for up to three tables when its ring
    // (two slots of each table's span) fits, and for three tables only up to 6 * 256 loaded
    // columns.  At 32768^2, 64 x 64 it took 3.48 / 5.23 / 7.64 ms for one / two / three tables
    // against 3.60 / 5.64 / 8.15 ms for the register walk; with four tables it holds 198 VGPRs,
    // two waves per SIMD, and lost (15.24 against 14.78 ms), so four take the register walk.
    if (gv.kind == G_CHAIN && gv.v == 0 && d.stride == 1 && order <= 3 &&
        lds_plan(1, d.win_w, 2 * order - 1, true, &nl, &span, &lds) && (order <= 2 || nl <= 6)) {
        const int64_t q = d.win_h;
        d.chunks = (d.ow + kLdsC - 1) / kLdsC;
        const int64_t P = (d.oh + q - 1) / q;
        const int64_t seg = chain_segments(q * d.chunks, P, 1);
        const int64_t total = q * d.chunks * ((P + seg - 1) / seg);
        switch (order) {
            case 1: return launch_lds_moments<1>(d, q, seg, total, nl, span, lds, stream);
            case 2: return launch_lds_moments<2>(d, q, seg, total, nl, span, lds, stream);
            default: return launch_lds_moments<3>(d, q, seg, total, nl, span, lds, stream);
        }
    }
    if (gv.kind == G_CHAIN && d.win_h % d.stride == 0) {
        // outputs per thread: four at stride 1 keep 32 loads per thread in flight (15.5 ms against
        // 16.6 ms with one at 32768^2, 64 x 64, four statistics); strides above 1 are insensitive
        const int V = gv.v > 0 ? gv.v : (d.stride > 1 ? 2 : 4);
        const int64_t q = d.win_h / d.stride;
        d.chunks = (d.ow + 256 * V - 1) / (256 * V);
        const int64_t P = (d.oh + q - 1) / q;                 // chain positions with outputs
        const int64_t seg = chain_segments(q * d.chunks, P, 1);
        const int64_t total = q * d.chunks * ((P + seg - 1) / seg);
        switch (order) {
            case 1: launch_chain_moments<1>(d, V, q, seg, total, stream); break;
            case 2: launch_chain_moments<2>(d, V, q, seg, total, stream); break;
            case 3: launch_chain_moments<3>(d, V, q, seg, total, stream); break;
            default: launch_chain_moments<4>(d, V, q, seg, total, stream); break;
        }
        return hipGetLastError();
    }
    constexpr int V = 2;
    d.chunks = (d.ow + 256 * V - 1) / (256 * V);
    GatherDesc g{};
    g.chunks = d.chunks;
    g.stride = d.stride;
    const int64_t band = band_chunks(g, V, true, d.win_h * order);
    const dim3 grid(static_cast<unsigned>(d.oh * d.chunks));
    switch (order) {
        case 1: hipLaunchKernelGGL((moments_kernel<1, V>), grid, dim3(256), 0, stream, d, band); break;
        case 2: hipLaunchKernelGGL((moments_kernel<2, V>), grid, dim3(256), 0, stream, d, band); break;
        case 3: hipLaunchKernelGGL((moments_kernel<3, V>), grid, dim3(256), 0, stream, d, band); break;
        case 4: hipLaunchKernelGGL((moments_kernel<4, V>), grid, dim3(256), 0, stream, d, band); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace satk
