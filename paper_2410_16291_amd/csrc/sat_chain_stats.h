// sat_chain_stats.h -- device code of the chain-walk mean/std gather, shared by the gather kernels
// (sat_gather.hip) and the fused batched build-and-statistics kernel (sat_build.hip).
// Internal to libsat.so.
#pragma once

#include "sat_internal.h"

namespace satk {
namespace {

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

// Sum, mean and population standard deviation of one window from its exact sums S1, Q1.
__device__ __forceinline__ void stats_store(const GatherDesc &d, int64_t o, uint64_t s1, uint64_t q1, uint64_t n,
                                            double dn) {
    // n*q1 - s1*s1 exactly, in 128 bits (non-negative by Cauchy-Schwarz).
    const uint64_t a_lo = n * q1, a_hi = __umul64hi(n, q1);
    const uint64_t b_lo = s1 * s1, b_hi = __umul64hi(s1, s1);
    const uint64_t num_lo = a_lo - b_lo;
    const uint64_t num_hi = a_hi - b_hi - (a_lo < b_lo ? 1u : 0u);
    uint64_t *sum = static_cast<uint64_t *>(d.out);
    if (sum) __builtin_nontemporal_store(s1, sum + o);
    __builtin_nontemporal_store(static_cast<double>(s1) / dn, d.mean + o);
    __builtin_nontemporal_store(sqrt(u128_to_double(num_hi, num_lo)) / dn, d.stdv + o);
}

// Position of one work item: column chunk c, chain residue r, chain positions [j0, j0 + seg).
struct ChainItem {
    int64_t c, r, j0;
};

__device__ __forceinline__ ChainItem chain_item(int64_t item, int64_t chunks, int64_t q, int64_t seg) {
    ChainItem it;
    it.c = item % chunks;
    const int64_t rs = item / chunks;
    it.r = rs % q;
    it.j0 = (rs / q) * seg;
    return it;
}

// Last chain position of residue r inside [j0, j0 + seg) with an output row below oh, or -1.
__device__ __forceinline__ int64_t chain_end(int64_t oh, int64_t r, int64_t q, int64_t j0, int64_t seg) {
    const int64_t lastk = oh - 1 - r;
    if (lastk < 0) return -1;
    const int64_t pm = lastk / q;
    return pm < j0 + seg - 1 ? pm : j0 + seg - 1;
}

// One work item of the chain-walk mean/std gather of descriptor d (256 threads): column chunk,
// chain residue and chain positions from the item index (chain_item), one read of each table row
// of S and Q on the chain, window sums as differences of the corner columns, then sum, mean and
// standard deviation per output.
template <int V>
__device__ __forceinline__ void chain_stats_item(const GatherDesc &d, int64_t item) {
    const ChainItem it = chain_item(item, d.chunks, d.q, d.seg);
    const int64_t pend = chain_end(d.oh, it.r, d.q, it.j0, d.seg);
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
    auto load = [&](int64_t j, uint64_t (&rows)[4][V]) {
        const int64_t t = (it.r + j * d.q) * d.stride - 1;
        const int64_t off = (t > 0 ? t : 0) * d.spitch;
        const uint64_t *ps = d.S + off, *pq = d.Q + off;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            rows[0][v] = ps[xl[v]];
            rows[1][v] = ps[xr[v]];
            rows[2][v] = pq[xl[v]];
            rows[3][v] = pq[xr[v]];
        }
    };
    uint64_t cur[4][V], nxt[4][V], prev_s[V], prev_q[V];
    load(it.j0, cur);
#pragma unroll 1
    for (int64_t j = it.j0; j <= jlast; ++j) {
        if (j < jlast) load(j + 1, nxt);
        const bool row_ok = it.r + j * d.q > 0;
        const int64_t orow = (it.r + (j - 1) * d.q) * d.opitch;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint64_t ds = row_ok ? cur[1][v] - (has_left[v] ? cur[0][v] : 0) : 0;
            const uint64_t dq = row_ok ? cur[3][v] - (has_left[v] ? cur[2][v] : 0) : 0;
            if (j > it.j0 && lx[v] < d.ow) stats_store(d, orow + lx[v], ds - prev_s[v], dq - prev_q[v], nn, dn);
            prev_s[v] = ds;
            prev_q[v] = dq;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int v = 0; v < V; ++v) cur[k][v] = nxt[k][v];
    }
}

}  // namespace
}  // namespace satk
