// sat_build.hip -- integral-image (summed-area table) construction for gfx950.
//
// The table is the inclusive 2-D prefix sum of the image (Sec. II-B); its cost is one pass over
// the image (the O(r*c) term of Sec. III-B).  Decomposition used here:
//
//   S[y][x] = U_w[x] + sum_{y' = y0_w .. y} R[y'][x]
//   R[y][x] = L[y] + (prefix of row y inside the current column block)
//   U_w[x]  = S[y0_w - 1][x] = sum_{x' <= x} C_w[x']
//   C_w[x]  = sum of column x above row y0_w  (strip column totals from the lookback, plus the
//             rows of the waves above this one inside the strip)
//
// A workgroup owns one strip of up to TH = RW*NW rows and sweeps it left to right in blocks of
// BW = 64*PX columns; wave w owns a band of the strip's rows and lane l owns the column pair
// (2l, 2l+1) of every 128-column sub-block of a block.  The row direction is handled by the sweep
// itself (the left carry L of each row is a register); the column direction crosses strips, and
// the totals of the strips above come from a decoupled lookback down each column:
//   - for block b the strip publishes its column totals A (status "aggregate"),
//   - reads the state of the strip above: an inclusive total P ends the walk, an aggregate is
//     added and the walk continues one strip higher,
//   - publishes P = (totals above) + A (status "prefix").
// Each lookback word is a single 64-bit value, status in bits 62-63 and the column total in
// bits 0-61, so a relaxed agent-scope atomic store or load moves a complete, self-describing
// state and no fence is needed.  Strips are handed out by an atomic ticket, so a workgroup only
// ever waits for strips whose workgroups have already started: forward progress does not depend
// on dispatch order.  Every wait is bounded; a wait that exceeds the bound sets a fault word in
// the workspace and the kernel still completes.
//
// Three strip workers share this scheme:
//   Build     every wave computes; wave 0 runs the lookback between two workgroup barriers.  The
//             same code also runs in a reduce-then-scan mode (an ablation): one kernel writes the
//             strip column totals, a second scans them down each column, and the strip kernel
//             then reads its totals instead of looking back.
//   Build2    four compute waves and a helper wave that stages tiles by LDS DMA and runs the
//             lookback ahead of the compute waves, so that the lookback's memory round trip is
//             never on their path (two pipelines, see the struct).
//   BuildPow  Build2 for the tables of pixel^1..pixel^k (k lookback planes, one pass over the
//             LDS tile per power).
//
// Per-row work: the 64 lanes of a wave scan a row of BW pixels with DPP (row_shr 1/2/4/8 within
// rows of 16 lanes, then row_bcast 15 and 31 across them) in 32-bit integers, which cannot
// overflow for a block (BW * 65535 < 2^32; squares of 16-bit pixels are scanned as their two
// 16-bit halves); the 64-bit carries are added once per pixel.
#include "sat_internal.h"
#include "sat_chain_stats.h"

#include <mutex>
#include <type_traits>

namespace satk {
namespace {

constexpr uint64_t kStAggregate = 1ull << 62;
constexpr uint64_t kStPrefix = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 22;

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ cross-lane helpers

template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return static_cast<uint32_t>(
        __builtin_amdgcn_update_dpp(0, static_cast<int>(v), CTRL, ROW_MASK, 0xf, BOUND_ZERO));
}

// One step of a 64-bit scan as two 32-bit DPP moves and a 32-bit add with carry.  The step is
// kept in 32-bit operations on purpose: with a fused 64-bit add the compiler placed the next DPP
// read of the sum one instruction after its write, below the two wait states a DPP source
// needs, and the upper lanes of each row read stale values.
template <int CTRL, int ROW_MASK, bool BOUND_ZERO>
__device__ __forceinline__ void dpp_add64(uint32_t &lo, uint32_t &hi) {
    const uint32_t dlo = dpp<CTRL, ROW_MASK, BOUND_ZERO>(lo);
    const uint32_t dhi = dpp<CTRL, ROW_MASK, BOUND_ZERO>(hi);
    const uint32_t nlo = lo + dlo;
    hi = hi + dhi + (nlo < lo ? 1u : 0u);
    lo = nlo;
}

// 64-bit sum in 32-bit operations, for values that feed a DPP scan (see dpp_add64).
__device__ __forceinline__ uint64_t add64(uint64_t a, uint64_t b) {
    const uint32_t lo = static_cast<uint32_t>(a) + static_cast<uint32_t>(b);
    const uint32_t hi = static_cast<uint32_t>(a >> 32) + static_cast<uint32_t>(b >> 32) +
                        (lo < static_cast<uint32_t>(a) ? 1u : 0u);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}
__device__ __forceinline__ uint32_t add64(uint32_t a, uint32_t b) { return a + b; }

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_scan(uint32_t v) {
    v += dpp<0x111, 0xf, true>(v);   // row_shr:1
    v += dpp<0x112, 0xf, true>(v);   // row_shr:2
    v += dpp<0x114, 0xf, true>(v);   // row_shr:4
    v += dpp<0x118, 0xf, true>(v);   // row_shr:8   -> prefix within each row of 16 lanes
    v += dpp<0x142, 0xa, false>(v);  // row_bcast:15 -> rows 1 and 3 add lane 15 / 47
    v += dpp<0x143, 0xc, false>(v);  // row_bcast:31 -> rows 2 and 3 add lane 31
    return v;
}

__device__ __forceinline__ uint64_t wave_scan(uint64_t v) {
    uint32_t lo = static_cast<uint32_t>(v), hi = static_cast<uint32_t>(v >> 32);
    dpp_add64<0x111, 0xf, true>(lo, hi);
    dpp_add64<0x112, 0xf, true>(lo, hi);
    dpp_add64<0x114, 0xf, true>(lo, hi);
    dpp_add64<0x118, 0xf, true>(lo, hi);
    dpp_add64<0x142, 0xa, false>(lo, hi);
    dpp_add64<0x143, 0xc, false>(lo, hi);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
}
__device__ __forceinline__ uint64_t readlane(uint64_t v, int l) {
    return (static_cast<uint64_t>(readlane(static_cast<uint32_t>(v >> 32), l)) << 32) |
           readlane(static_cast<uint32_t>(v), l);
}

// Test-only perturbation of the lookback: with a nonzero seed (BuildDesc::stress) a wave sleeps a
// pseudo-random number of steps (0..31 x 512 cycles, hashed from the seed, strip, block and phase)
// before it publishes a lookback word or a fused ready count.  Publication order then varies
// from run to run while every wait stays bounded and ticket order keeps progress guaranteed.
__device__ __forceinline__ void stress_delay(uint32_t seed, int strip, int64_t xb, uint32_t phase) {
    if (seed == 0) return;
    uint32_t h = seed ^ (static_cast<uint32_t>(strip) * 0x9E3779B1u) ^ (static_cast<uint32_t>(xb) * 0x85EBCA77u) ^
                 (phase * 0xC2B2AE3Du);
    h ^= h >> 15;
    h *= 0x2C1B3C6Du;
    h ^= h >> 12;
    h *= 0x297A2D39u;
    h ^= h >> 15;
    const uint32_t n = h & 31u;
    for (uint32_t i = 0; i < n; ++i) __builtin_amdgcn_s_sleep(8);
}

// Lookback state words: the value in the low bits, the status in the top two (0: not yet
// published, kAggregate: the strip's own column total, kPrefix: the inclusive column total of
// every strip through this one).  64-bit words hold any total a build can reach; 32-bit words
// serve builds whose column totals stay below 2^30 (no squared table and (rows above + H) *
// max_pixel < 2^30, decided by the host per launch): half the lookback's traffic and half the
// state to clear.
constexpr uint32_t kAggregate = 1u;
constexpr uint32_t kPrefix = 2u;

template <typename SW>
struct StateWord {
    static constexpr int kShift = 8 * static_cast<int>(sizeof(SW)) - 2;
    static constexpr SW kMask = (static_cast<SW>(1) << kShift) - 1;
    static __device__ __forceinline__ SW make(uint32_t status, uint64_t value) {
        return (static_cast<SW>(status) << kShift) | static_cast<SW>(value);
    }
    static __device__ __forceinline__ uint32_t status(SW w) { return static_cast<uint32_t>(w >> kShift); }
    static __device__ __forceinline__ uint64_t value(SW w) { return static_cast<uint64_t>(w & kMask); }
    static __device__ __forceinline__ void store(SW *p, SW v) {
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ __forceinline__ SW load(const SW *p) {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

__device__ __forceinline__ void store_state(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_state(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ the strip worker

constexpr int kRsrcWord3 = 0x00020000;   // raw buffer resource, 32-bit data format (gfx9 family)

typedef int i32x4 __attribute__((ext_vector_type(4)));

// Raw buffer resource (base, stride 0, num_records bytes) as four scalar dwords.
__device__ __forceinline__ i32x4 make_rsrc(const void *base, uint32_t num_records) {
    const uint64_t a = reinterpret_cast<uint64_t>(base);
    return i32x4{static_cast<int>(static_cast<uint32_t>(a)), static_cast<int>(static_cast<uint32_t>(a >> 32) & 0xffffu),
                 static_cast<int>(num_records), kRsrcWord3};
}

// 16-byte buffer store with the two wait states the hardware needs before any VALU may
// overwrite the store's data VGPRs (a store of more than 8 bytes reads its data after issue).
// The compiler does not insert them for gfx950: an overwrite in the next cycle was seen to
// corrupt lanes 12-15 of every 16-lane group.  Keeping the s_nop inside the same asm block
// makes the gap independent of scheduling and register allocation.  The asm has no outputs.
// Store policies of table rows: bit 0 non-temporal (the table is read back only after it has
// left the caches); bit 1 device-coherent (written through this XCD's L2, so that a reader on
// another XCD sees it once the store has completed, with no write-back of the whole L2).
constexpr int kStNT = 1;
constexpr int kStCoherent = 2;
// Cache-policy bits of the buffer-store builtins: slc (nt) = 2, scc (sc1) = 16.
constexpr int store_aux(int pol) { return ((pol & kStNT) ? 2 : 0) | ((pol & kStCoherent) ? 16 : 0); }

template <int POL = 0>
__device__ __forceinline__ void store16_rsrc(u32x4 data, i32x4 rsrc, uint32_t voff, uint32_t soff) {
    if constexpr (POL == (kStNT | kStCoherent))
        asm volatile("buffer_store_dwordx4 %0, %1, %2, %3 offen sc1 nt\n\ts_nop 1"
                     :
                     : "v"(data), "v"(voff), "s"(rsrc), "s"(soff)
                     : "memory");
    else if constexpr (POL == kStCoherent)
        asm volatile("buffer_store_dwordx4 %0, %1, %2, %3 offen sc1\n\ts_nop 1"
                     :
                     : "v"(data), "v"(voff), "s"(rsrc), "s"(soff)
                     : "memory");
    else if constexpr (POL == kStNT)
        asm volatile("buffer_store_dwordx4 %0, %1, %2, %3 offen nt\n\ts_nop 1"
                     :
                     : "v"(data), "v"(voff), "s"(rsrc), "s"(soff)
                     : "memory");
    else
        asm volatile("buffer_store_dwordx4 %0, %1, %2, %3 offen\n\ts_nop 1"
                     :
                     : "v"(data), "v"(voff), "s"(rsrc), "s"(soff)
                     : "memory");
}

// LDS-only workgroup barrier: orders LDS accesses between the waves of a workgroup and leaves
// each wave's global stores in flight.  (A full __syncthreads() makes every wave wait until its
// table stores have reached memory before the barrier: on gfx9 the vector memory counter covers
// stores too, so each block of a strip would end in a drain of its stores.)
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Barrier for the helper wave just after it issued a tile's LDS DMA that no wave reads before a
// later barrier.  The release fence of lds_barrier would make the helper wait for that DMA here
// (LDS DMA writes LDS and is counted on the vector memory counter), so the tile's load latency
// would be paid before the barrier instead of overlapping the lookback that follows.  Only the
// helper's own LDS accesses are waited for; the DMA is waited for at the next barrier.
__device__ __forceinline__ void dma_barrier() {
    __builtin_amdgcn_s_waitcnt(0xc07f);          // lgkmcnt(0); vmcnt and expcnt at their maximum
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------------ rows of one table block
//
// A wave's rows of one block of one table: for every row, the lane's pixel pair of each 128-column
// sub-block (or their squares), a DPP scan of pair sums across the wave, the row's left carry and
// the running column sums down the wave's rows, then one 16-byte store per lane (contiguous
// across the wave).  Rows are taken G at a time: their LDS reads go out together and their G
// scans are independent, so one wave keeps G dependency chains in flight instead of one (with one
// or two waves per SIMD nothing else hides the DPP and LDS latencies).  The running column sums
// are then advanced row by row, in order.

// Inclusive scan across the wave of the pair sums a0 + a1, exact in 64 bits.  WIDE (pixel values
// up to 2^32 - 1, the squares of 16-bit pixels): both halves of each value (bits 0-15 and 16-31)
// are scanned as separate 32-bit sums, each at most 128 * 65535 < 2^32, and recombined.
template <bool WIDE>
__device__ __forceinline__ void scan_pair(uint32_t a0, uint32_t a1, uint64_t &pair, uint64_t &incl) {
    if constexpr (WIDE) {
        const uint32_t lo = (a0 & 0xffffu) + (a1 & 0xffffu);
        const uint32_t hi = (a0 >> 16) + (a1 >> 16);
        const uint32_t slo = wave_scan(lo);
        const uint32_t shi = wave_scan(hi);
        pair = static_cast<uint64_t>(a0) + a1;
        incl = (static_cast<uint64_t>(shi) << 16) + slo;
    } else {
        const uint32_t p = a0 + a1;
        pair = p;
        incl = wave_scan(p);
    }
}

// G rows starting at wave row r0 (all valid).  trow: the lane's pixel pair of sub-block 0 of the
// wave's first row in the LDS tile (rows BW pixels apart).
template <typename T, int PX, int G, bool SQUARE, bool WIDE, bool VEC, int POL>
__device__ __forceinline__ void row_group(const T *trow, int r0, int lane, const uint64_t (&u)[PX],
                                          uint64_t (&acc)[PX], uint64_t lcarry, uint64_t &tvec, const i32x4 &rs_blk,
                                          const char *blk0, uint32_t row_recs, uint32_t pitch_bytes) {
    constexpr int NS = PX / 2, BW = 64 * PX;
    uint32_t pv[G][NS];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int sb = 0; sb < NS; ++sb) {
            const T *src = trow + (r0 + g) * BW + 128 * sb;
            if (sizeof(T) == 1) pv[g][sb] = *reinterpret_cast<const uint16_t *>(src);
            else pv[g][sb] = *reinterpret_cast<const uint32_t *>(src);
        }
    uint64_t base[G];
#pragma unroll
    for (int g = 0; g < G; ++g) base[g] = readlane(lcarry, r0 + g);
#pragma unroll
    for (int sb = 0; sb < NS; ++sb) {
        uint32_t a0[G], a1[G];
        uint64_t pair[G], incl[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t v0 = sizeof(T) == 1 ? (pv[g][sb] & 0xffu) : (pv[g][sb] & 0xffffu);
            const uint32_t v1 = sizeof(T) == 1 ? ((pv[g][sb] >> 8) & 0xffu) : (pv[g][sb] >> 16);
            a0[g] = SQUARE ? v0 * v0 : v0;
            a1[g] = SQUARE ? v1 * v1 : v1;
            scan_pair<WIDE>(a0[g], a1[g], pair[g], incl[g]);
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint64_t b = base[g] + (incl[g] - pair[g]);
            acc[2 * sb] += b + a0[g];
            acc[2 * sb + 1] += b + pair[g];
            const uint64_t o0 = u[2 * sb] + acc[2 * sb], o1 = u[2 * sb + 1] + acc[2 * sb + 1];
            const uint32_t roff = static_cast<uint32_t>(r0 + g) * pitch_bytes;
            if (VEC) {
                store16_rsrc<POL>(u32x4{static_cast<uint32_t>(o0), static_cast<uint32_t>(o0 >> 32),
                                        static_cast<uint32_t>(o1), static_cast<uint32_t>(o1 >> 32)},
                                  rs_blk, static_cast<uint32_t>(lane) * 16 + sb * 1024, roff);
            } else {
                const __amdgpu_buffer_rsrc_t rs_row = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<char *>(blk0 + roff), 0, static_cast<int>(row_recs), kRsrcWord3);
                const uint32_t voff = static_cast<uint32_t>(lane) * 16 + sb * 1024;
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{static_cast<uint32_t>(o0), static_cast<uint32_t>(o0 >> 32)},
                                                      rs_row, voff, 0, store_aux(POL));
                __builtin_amdgcn_raw_buffer_store_b64(u32x2{static_cast<uint32_t>(o1), static_cast<uint32_t>(o1 >> 32)},
                                                      rs_row, voff + 8, 0, store_aux(POL));
            }
            base[g] += readlane(incl[g], 63);
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
        if (lane == r0 + g) tvec = base[g] - readlane(lcarry, r0 + g);
}

// All rows_ok rows of the wave for one table of one block; returns the row totals of the block
// (lane r holds row r's) to add to the left carries.  Stores go through buffer resources so that
// the hardware range check, not a branch per row, drops what lies outside the image:
//   VEC (block wholly inside the image width, 16-byte aligned table rows): one resource spanning
//     the wave's rows from the block start, records ending at the last valid row's width; row r
//     is addressed by the scalar offset r * pitch;
//   ragged: one resource per row covering exactly [block start, W) of that row, 8-byte stores.
template <typename T, int PX, bool SQUARE, bool WIDE, bool VEC, int POL>
__device__ __forceinline__ uint64_t block_rows(const T *trow, int lane, const uint64_t (&u)[PX], uint64_t lcarry,
                                               uint64_t *blk0, int rows_ok, uint32_t row_recs, uint32_t pitch_bytes) {
    constexpr int G = 4;
    uint64_t acc[PX];
#pragma unroll
    for (int p = 0; p < PX; ++p) acc[p] = 0;
    uint64_t tvec = 0;
    const int nvalid = rows_ok > 0 ? rows_ok : 0;
    const uint32_t blk_recs = nvalid > 0 ? (nvalid - 1) * pitch_bytes + row_recs : 0;
    const i32x4 rs_blk = make_rsrc(blk0, VEC ? blk_recs : 0);
    const char *b0 = reinterpret_cast<const char *>(blk0);
    int r = 0;
#pragma unroll 1
    for (; r + G <= nvalid; r += G)
        row_group<T, PX, G, SQUARE, WIDE, VEC, POL>(trow, r, lane, u, acc, lcarry, tvec, rs_blk, b0, row_recs,
                                                    pitch_bytes);
#pragma unroll 1
    for (; r < nvalid; ++r)
        row_group<T, PX, 1, SQUARE, WIDE, VEC, POL>(trow, r, lane, u, acc, lcarry, tvec, rs_blk, b0, row_recs,
                                                    pitch_bytes);
    return tvec;
}

template <typename T, bool SQ, int PX, int RW, int NW, int MODE, bool NTS = false, bool COH = false>
struct Build {
    static constexpr int POL = (NTS ? kStNT : 0) | (COH ? kStCoherent : 0);   // table store policy
    static constexpr int TH = RW * NW;                       // strip height
    static constexpr int BW = 64 * PX;                       // block width
    static constexpr int NT = NW * 64;                       // threads per workgroup
    static constexpr int NS = PX / 2;                        // 128-column sub-blocks per block
    static constexpr int PXB = PX * static_cast<int>(sizeof(T));   // bytes a lane owns in a row
    static constexpr int ROWB = BW * static_cast<int>(sizeof(T));  // bytes of one tile row
    static constexpr int TILEB = TH * ROWB;                  // bytes of one image tile
    static constexpr int PFW = TILEB / NT / 4;               // prefetch dwords per thread
    static_assert(PX % 2 == 0 && PFW >= 4 && PFW % 4 == 0, "lanes own column pairs; 16-byte chunks");

    // Lane l owns, in every 128-column sub-block s of a block, the adjacent columns 2l and 2l+1;
    // its p-th pixel (p = 2s + j) is column 128s + 2l + j of the block.  A table row segment of
    // a sub-block is then one contiguous 1 KiB wave store (16 bytes per lane).
    static __device__ __forceinline__ int col(int lane, int p) { return (p >> 1) * 128 + 2 * lane + (p & 1); }
    // Squared partial sums: 8-bit squares fit 32 bits for a whole block, 16-bit ones do not.
    using QT = typename std::conditional<sizeof(T) == 1, uint32_t, uint64_t>::type;
    // Squares of 16-bit pixels need the split scan of scan_pair.
    static constexpr bool WIDE_SQ = sizeof(T) == 2;

    struct Smem {
        uint32_t tile[TILEB / 4];                            // image tile of the current block
        uint32_t cs[2][NW][BW];                              // per-wave column sums (2 buffers)
        QT csq[SQ ? 2 : 1][SQ ? NW : 1][SQ ? BW : 1];
        uint64_t v[BW];                                      // column totals above the strip
        uint64_t vq[SQ ? BW : 1];
        long long ticket;
    };

    // raw[s] holds the lane's pixel pair of sub-block s (two bytes or two halves).
    static __device__ __forceinline__ uint32_t pix(const uint32_t (&raw)[NS], int p) {
        if (sizeof(T) == 1) return (raw[p >> 1] >> (8 * (p & 1))) & 0xffu;
        return (raw[p >> 1] >> (16 * (p & 1))) & 0xffffu;
    }

    // This lane's PX pixels of tile row `row` (LDS).
    static __device__ __forceinline__ void tile_px(const Smem &sm, int row, int lane, uint32_t (&raw)[NS]) {
        const T *src = reinterpret_cast<const T *>(sm.tile) + row * BW + 2 * lane;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (sizeof(T) == 1) raw[s] = *reinterpret_cast<const uint16_t *>(src + 128 * s);
            else raw[s] = *reinterpret_cast<const uint32_t *>(src + 128 * s);
        }
    }

    // ---- image tile staging.  Fast path: a tile wholly inside the image whose rows allow
    // VB-byte loads; every thread loads PFW dwords of it as VB-byte chunks (consecutive threads,
    // consecutive chunks of a row) into registers, committed to LDS later.
    template <int VB>
    static __device__ __forceinline__ void fetch(const BuildDesc &d, int64_t ys, int64_t xb, int nvalid,
                                                 uint32_t (&pf)[PFW]) {
        constexpr int CPR = ROWB / VB;                       // chunks per tile row
        constexpr int WPC = VB / 4;                          // dwords per chunk
        constexpr int NCH = PFW / WPC;                       // chunks per thread
        constexpr int RPI = NT / CPR;                        // tile rows advanced per chunk index
        static_assert(NT % CPR == 0, "a workgroup covers whole tile rows per step");
        const int64_t pitchb = d.ipitch * static_cast<int64_t>(sizeof(T));
        const unsigned char *base = static_cast<const unsigned char *>(d.img) +
                                    (ys * d.ipitch + xb) * static_cast<int64_t>(sizeof(T));
        // The resource ends after the strip's last valid row: rows past it read as zero.
        const uint32_t recs = static_cast<uint32_t>(nvalid - 1) * static_cast<uint32_t>(pitchb) + ROWB;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char *>(base), 0, static_cast<int>(recs), kRsrcWord3);
        const uint32_t voff = static_cast<uint32_t>((threadIdx.x / CPR) * pitchb + (threadIdx.x % CPR) * VB);
        const uint32_t step = static_cast<uint32_t>(RPI * pitchb);
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int so = static_cast<int>(i * step);
            if (VB == 16) {
                const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, so, 0);
                pf[i * WPC] = t.x; pf[i * WPC + (WPC > 1 ? 1 : 0)] = t.y;
                pf[i * WPC + (WPC > 2 ? 2 : 0)] = t.z; pf[i * WPC + (WPC > 3 ? 3 : 0)] = t.w;
            } else if (VB == 8) {
                const u32x2 t = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, so, 0);
                pf[i * WPC] = t.x; pf[i * WPC + (WPC > 1 ? 1 : 0)] = t.y;
            } else {
                pf[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, voff, so, 0);
            }
        }
    }

    template <int VB>
    static __device__ __forceinline__ void commit(Smem &sm, const uint32_t (&pf)[PFW]) {
        constexpr int CPR = ROWB / VB;
        constexpr int WPC = VB / 4;
        constexpr int NCH = PFW / WPC;
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int c = i * NT + static_cast<int>(threadIdx.x);
            const int row = c / CPR, off = (c % CPR) * VB;
            uint32_t *dst = sm.tile + (row * ROWB + off) / 4;
#pragma unroll
            for (int k = 0; k < WPC; ++k) dst[k] = pf[i * WPC + k];
        }
    }

    static __device__ __forceinline__ bool fast_tile(const BuildDesc &d, int64_t xb) {
        return d.img_vb != 0 && xb + BW <= d.W;
    }

    static __device__ __forceinline__ void fetch_any(const BuildDesc &d, int64_t ys, int64_t xb, int nvalid,
                                                     uint32_t (&pf)[PFW]) {
        if (d.img_vb == 16) fetch<16>(d, ys, xb, nvalid, pf);
        else if (d.img_vb == 8) fetch<8>(d, ys, xb, nvalid, pf);
        else fetch<4>(d, ys, xb, nvalid, pf);
    }
    static __device__ __forceinline__ void commit_any(const BuildDesc &d, Smem &sm, const uint32_t (&pf)[PFW]) {
        if (d.img_vb == 16) commit<16>(sm, pf);
        else if (d.img_vb == 8) commit<8>(sm, pf);
        else commit<4>(sm, pf);
    }

    // Slow path (ragged or unaligned tiles): element by element, zeros outside the strip's
    // valid rows and the image width.
    static __device__ void load_tile_slow(const BuildDesc &d, Smem &sm, int64_t ys, int64_t xb, int nvalid) {
        const T *img = static_cast<const T *>(d.img);
        T *tile = reinterpret_cast<T *>(sm.tile);
#pragma unroll 4
        for (int e = threadIdx.x; e < TH * BW; e += NT) {
            const int row = e / BW, col = e % BW;
            const int64_t y = ys + row, x = xb + col;
            tile[e] = (row < nvalid && x < d.W) ? img[y * d.ipitch + x] : static_cast<T>(0);
        }
    }

    // Column totals of all strips above `strip` for this lane's PX columns (decoupled lookback),
    // after publishing this strip's own totals a / aq.  Run by one full wave.
    // Offset of the lane's p-th column from its first column (2 * lane) inside a block.
    static __device__ __forceinline__ int soff(int p) { return (p >> 1) * 128 + (p & 1); }
    // Lookback word of lane l's p-th column in a block's state row: p * 64 + l.  Only the lookback
    // writes and reads these words, so any fixed permutation of the block's columns serves; this
    // one makes every 64-lane access 512 contiguous bytes (whole cache lines), where the column
    // order (soff) would touch every line half.
    static __device__ __forceinline__ int lslot(int p) { return p * 64; }

    // Strip 0 of a band build: the column totals above the strip are the carried totals of the
    // rows above the image (zero without a carry).  Every lookback value of the band is then a
    // carry plus at most H maximal pixels, which must stay below the state word's value range
    // (2^62, or 2^30 for 32-bit words; the host has checked that H * max_pixel fits): a carry
    // above that range less H * max_pixel sets fault bit 1.
    template <typename SW>
    static __device__ __forceinline__ void seed(const BuildDesc &d, int64_t xb, int lane, uint64_t (&v)[PX],
                                                uint64_t (&vq)[PX], unsigned int *fault) {
        if (!d.carry) return;
        constexpr uint64_t kMaxPix = sizeof(T) == 1 ? 255u : 65535u;
        constexpr uint64_t kRange = static_cast<uint64_t>(StateWord<SW>::kMask);
        const uint64_t room = kRange - static_cast<uint64_t>(d.H) * kMaxPix;
        const uint64_t room_q = kRange - static_cast<uint64_t>(d.H) * kMaxPix * kMaxPix;
        bool big = false;
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            const int64_t x = xb + col(lane, p);
            v[p] = x < d.W ? d.carry[x] : 0;
            big = big || v[p] > room;
            if (SQ) {
                vq[p] = x < d.W ? d.carry_q[x] : 0;
                big = big || vq[p] > room_q;
            }
        }
        if (big) atomicOr(fault, 2u);
    }

    // The last strip's inclusive totals (totals above + its own) are the column totals through
    // the image's last row: the carry of the next band.
    static __device__ __forceinline__ void emit_total(const BuildDesc &d, int strip, int64_t xb, int lane,
                                                      const uint64_t (&v)[PX], const uint64_t (&a)[PX],
                                                      const uint64_t (&vq)[PX], const uint64_t (&aq)[PX]) {
        if (strip != d.nstrips - 1) return;
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            const int64_t x = xb + col(lane, p);
            if (x < d.W) {
                if (d.total) d.total[x] = v[p] + a[p];
                if (SQ && d.total_q) d.total_q[x] = vq[p] + aq[p];
            }
        }
    }

    // Column totals of all strips above `strip` for this lane's PX columns by decoupled lookback
    // over the state words of the strips above (32-bit words when the build's descriptor says its
    // totals fit them).  Run by one full wave.
    static __device__ __forceinline__ void lookback(const BuildDesc &d, int strip, int64_t xb, int lane,
                                                    const uint64_t (&a)[PX], const uint64_t (&aq)[PX],
                                                    uint64_t (&v)[PX], uint64_t (&vq)[PX], uint64_t *state,
                                                    unsigned int *fault) {
        if constexpr (!SQ) {
            if (d.narrow) {
                lookback_win_t<1, uint32_t>(d, strip, xb, lane, a, aq, v, vq, state, fault);
                return;
            }
        }
        lookback_win_t<1, uint64_t>(d, strip, xb, lane, a, aq, v, vq, state, fault);
    }

    template <int WIN>
    static __device__ __forceinline__ void lookback_win(const BuildDesc &d, int strip, int64_t xb, int lane,
                                                        const uint64_t (&a)[PX], const uint64_t (&aq)[PX],
                                                        uint64_t (&v)[PX], uint64_t (&vq)[PX], uint64_t *state,
                                                        unsigned int *fault) {
        if constexpr (!SQ) {
            if (d.narrow) {
                lookback_win_t<WIN, uint32_t>(d, strip, xb, lane, a, aq, v, vq, state, fault);
                return;
            }
        }
        lookback_win_t<WIN, uint64_t>(d, strip, xb, lane, a, aq, v, vq, state, fault);
    }

    // Decoupled lookback that reads the states of WIN strips per round trip (j, j-1, ...,
    // j-WIN+1) and consumes them in order while every still-open column of the wave is ready:
    // aggregates are added and the walk goes on, an inclusive prefix (or strip 0) closes the
    // column.  When all strips are in flight together, prefixes propagate one strip per memory
    // round trip; the window lets a walk cover WIN strips per round trip instead.
    // A strip publishes its aggregates before it reads anything.  (Publishing them only for the
    // columns that the strip above had not yet closed saves a store per column where it had, but
    // holding them back for one round trip slowed the whole build by a third: strips below wait
    // on them.)
    template <int WIN, typename SW>
    static __device__ __forceinline__ void lookback_win_t(const BuildDesc &d, int strip, int64_t xb, int lane,
                                          const uint64_t (&a)[PX], const uint64_t (&aq)[PX],
                                          uint64_t (&v)[PX], uint64_t (&vq)[PX], uint64_t *state_words,
                                          unsigned int *fault) {
        using SWd = StateWord<SW>;
        SW *state = reinterpret_cast<SW *>(state_words);
        const int64_t col0 = xb + lane;
        SW *mine = state + d.state_off + static_cast<int64_t>(strip) * d.Wp + col0;
        SW *mine_q = state + d.state_q_off + static_cast<int64_t>(strip) * d.Wp + col0;
#pragma unroll
        for (int p = 0; p < PX; ++p) { v[p] = 0; vq[p] = 0; }
        if (strip == 0) {
            seed<SW>(d, xb, lane, v, vq, fault);
            stress_delay(d.stress, strip, xb, 0);
#pragma unroll
            for (int p = 0; p < PX; ++p) {
                SWd::store(mine + lslot(p), SWd::make(kPrefix, v[p] + a[p]));
                if (SQ) SWd::store(mine_q + lslot(p), SWd::make(kPrefix, vq[p] + aq[p]));
            }
            emit_total(d, strip, xb, lane, v, a, vq, aq);
            return;
        }
        stress_delay(d.stress, strip, xb, 1);
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            SWd::store(mine + lslot(p), SWd::make(kAggregate, a[p]));
            if (SQ) SWd::store(mine_q + lslot(p), SWd::make(kAggregate, aq[p]));
        }
        constexpr uint32_t kAll = SQ ? ((1u << (2 * PX)) - 1u) : ((1u << PX) - 1u);
        uint32_t done = 0;
        uint32_t spins = 0;
        int j = strip - 1;
        for (;;) {
            SW w[WIN][PX], wq[WIN][PX];
#pragma unroll
            for (int k = 0; k < WIN; ++k) {
                const int jj = j - k;
                const SW *up = state + d.state_off + static_cast<int64_t>(jj) * d.Wp + col0;
                const SW *up_q = state + d.state_q_off + static_cast<int64_t>(jj) * d.Wp + col0;
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    w[k][p] = 0;
                    wq[k][p] = 0;
                    if (jj >= 0 && !(done & (1u << p))) w[k][p] = SWd::load(up + lslot(p));
                    if (SQ && jj >= 0 && !(done & (1u << (PX + p)))) wq[k][p] = SWd::load(up_q + lslot(p));
                }
            }
            int consumed = 0;
            bool stalled = false;
#pragma unroll
            for (int k = 0; k < WIN; ++k) {
                const int jj = j - k;
                if (stalled || jj < 0 || __all(done == kAll)) break;
                bool ready = true;
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    if (!(done & (1u << p))) ready = ready && SWd::status(w[k][p]) != 0;
                    if (SQ && !(done & (1u << (PX + p)))) ready = ready && SWd::status(wq[k][p]) != 0;
                }
                if (!__all(ready)) {
                    stalled = true;
                    break;
                }
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    if (!(done & (1u << p))) {
                        v[p] += SWd::value(w[k][p]);
                        if (SWd::status(w[k][p]) == kPrefix || jj == 0) done |= 1u << p;
                    }
                    if (SQ && !(done & (1u << (PX + p)))) {
                        vq[p] += SWd::value(wq[k][p]);
                        if (SWd::status(wq[k][p]) == kPrefix || jj == 0) done |= 1u << (PX + p);
                    }
                }
                ++consumed;
            }
            if (__all(done == kAll)) break;
            j -= consumed;
            if (stalled) {
                if (++spins > kSpinLimit) {
                    atomicOr(fault, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        stress_delay(d.stress, strip, xb, 2);
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            SWd::store(mine + lslot(p), SWd::make(kPrefix, v[p] + a[p]));
            if (SQ) SWd::store(mine_q + lslot(p), SWd::make(kPrefix, vq[p] + aq[p]));
        }
        emit_total(d, strip, xb, lane, v, a, vq, aq);
    }

    static __device__ void strip(const BuildDesc &d, int strip_idx, uint64_t *state, unsigned int *fault, Smem &sm) {
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
        const int th = d.strip_h, rw = d.wave_rows;                      // th <= TH, rw <= RW
        const int64_t ys = static_cast<int64_t>(strip_idx) * th;       // first row of the strip
        const int nvalid = static_cast<int>(d.H - ys < th ? d.H - ys : th);
        const int row0 = wave * rw;                                       // first strip row of this wave
        const int64_t yw = ys + row0;
        const int rows_ok = nvalid - row0 < rw ? (nvalid - row0 > 0 ? nvalid - row0 : 0) : rw;
        uint64_t *S_w = d.S + yw * d.spitch;
        uint64_t *Q_w = SQ ? d.Q + yw * d.spitch : nullptr;
        const uint32_t pitch_bytes = static_cast<uint32_t>(d.spitch * 8);

        uint64_t lrow = 0, lrow_q = 0;       // lane r: sum of row yw+r left of the block
        uint64_t ucarry = 0, ucarry_q = 0;   // table value at (yw-1, block start - 1)

        // Stage block 0.
        uint32_t pf[PFW];
        if (fast_tile(d, 0)) {
            fetch_any(d, ys, 0, nvalid, pf);
            commit_any(d, sm, pf);
        } else {
            load_tile_slow(d, sm, ys, 0, nvalid);
        }
        lds_barrier();

        for (int b = 0; b < d.nblocks; ++b) {
            const int buf = b & 1;
            const int64_t xb = static_cast<int64_t>(b) * BW;

            // Column sums of this wave's rows.
            {
                uint32_t cs[PX];
                QT csq[PX];
#pragma unroll
                for (int p = 0; p < PX; ++p) { cs[p] = 0; csq[p] = 0; }
#pragma unroll 8
                for (int r = 0; r < rows_ok; ++r) {
                    uint32_t raw[NS];
                    tile_px(sm, row0 + r, lane, raw);
#pragma unroll
                    for (int p = 0; p < PX; ++p) {
                        const uint32_t v = pix(raw, p);
                        cs[p] += v;
                        if (SQ) csq[p] += static_cast<QT>(v) * v;
                    }
                }
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    sm.cs[buf][wave][lane * PX + p] = cs[p];
                    if (SQ) sm.csq[buf][wave][lane * PX + p] = csq[p];
                }
            }
            // Prefetch the next block's tile while this block's lookback and rows run.
            const bool next_fast = b + 1 < d.nblocks && fast_tile(d, xb + BW);
            if (next_fast) fetch_any(d, ys, xb + BW, nvalid, pf);
            lds_barrier();

            if (wave == 0) {
                uint64_t a[PX], aq[PX], v[PX], vq[PX];
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    a[p] = 0;
                    aq[p] = 0;
#pragma unroll
                    for (int w = 0; w < NW; ++w) {
                        a[p] += sm.cs[buf][w][lane * PX + p];
                        if (SQ) aq[p] += sm.csq[buf][w][lane * PX + p];
                    }
                }
                if (MODE == MODE_LOOKBACK) {
                    lookback(d, strip_idx, xb, lane, a, aq, v, vq, state, fault);
                } else {
                    const uint64_t *tot = state + d.state_off + static_cast<int64_t>(strip_idx) * d.Wp + xb + 2 * lane;
                    const uint64_t *tot_q = state + d.state_q_off + static_cast<int64_t>(strip_idx) * d.Wp + xb + 2 * lane;
#pragma unroll
                    for (int p = 0; p < PX; ++p) {
                        v[p] = tot[soff(p)];
                        vq[p] = SQ ? tot_q[soff(p)] : 0;
                    }
                }
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    sm.v[lane * PX + p] = v[p];
                    if (SQ) sm.vq[lane * PX + p] = vq[p];
                }
            }
            lds_barrier();

            // Table row just above this wave's rows: prefix along x of the column totals above.
            uint64_t u[PX], uq[PX];
            {
                uint64_t c[PX], cq[PX];
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    c[p] = sm.v[lane * PX + p];
                    cq[p] = SQ ? sm.vq[lane * PX + p] : 0;
                }
                for (int w = 0; w < wave; ++w)
#pragma unroll
                    for (int p = 0; p < PX; ++p) {
                        c[p] += sm.cs[buf][w][lane * PX + p];
                        if (SQ) cq[p] += sm.csq[buf][w][lane * PX + p];
                    }
                // Sub-block by sub-block: pair prefix in the lane, DPP scan of pair totals.
#pragma unroll
                for (int sb = 0; sb < NS; ++sb) {
                    const uint64_t pair = add64(c[2 * sb], c[2 * sb + 1]);
                    const uint64_t incl = wave_scan(pair);
                    const uint64_t b = ucarry + (incl - pair);
                    u[2 * sb] = b + c[2 * sb];
                    u[2 * sb + 1] = b + pair;
                    ucarry += readlane(incl, 63);
                    if (SQ) {
                        const uint64_t pair_q = add64(cq[2 * sb], cq[2 * sb + 1]);
                        const uint64_t incl_q = wave_scan(pair_q);
                        const uint64_t b_q = ucarry_q + (incl_q - pair_q);
                        uq[2 * sb] = b_q + cq[2 * sb];
                        uq[2 * sb + 1] = b_q + pair_q;
                        ucarry_q += readlane(incl_q, 63);
                    }
                }
            }

            // Rows: row prefix (lane-serial, then DPP across lanes) plus the row's left carry,
            // accumulated down the wave's rows and offset by the table row above.  The squared
            // table is a second pass over the same tile to keep live ranges short.
            const bool vec = d.sat_vec && xb + BW <= d.W;
            const uint32_t row_recs = static_cast<uint32_t>((d.W - xb) * 8);   // bytes from block start to W
            const T *trow = reinterpret_cast<const T *>(sm.tile) + row0 * BW + 2 * lane;
            if (vec) {
                lrow += block_rows<T, PX, false, false, true, POL>(trow, lane, u, lrow, S_w + xb, rows_ok, row_recs, pitch_bytes);
                if (SQ) lrow_q += block_rows<T, PX, true, WIDE_SQ, true, POL>(trow, lane, uq, lrow_q, Q_w + xb, rows_ok, row_recs, pitch_bytes);
            } else {
                lrow += block_rows<T, PX, false, false, false, POL>(trow, lane, u, lrow, S_w + xb, rows_ok, row_recs, pitch_bytes);
                if (SQ) lrow_q += block_rows<T, PX, true, WIDE_SQ, false, POL>(trow, lane, uq, lrow_q, Q_w + xb, rows_ok, row_recs, pitch_bytes);
            }

            // Replace the tile with the next block's.
            if (b + 1 < d.nblocks) {
                lds_barrier();
                if (next_fast) commit_any(d, sm, pf);
                else load_tile_slow(d, sm, ys, xb + BW, nvalid);
                lds_barrier();
            }
        }
    }
};

// Helper-wave tile staging: the tile at columns [xb, xb+BW) of a strip's rows [ys, ys+nvalid)
// into one LDS tile buffer (TH rows of BW pixels, row-major).
template <typename T, int PX, int TH>
struct TileStage {
    static constexpr int BW = 64 * PX;
    static constexpr int ROWB = BW * static_cast<int>(sizeof(T));
    static constexpr int TILEB = TH * ROWB;
    static_assert(TILEB % 1024 == 0, "tile is a whole number of 1 KiB wave loads");

    // Fast path (tile inside the image width, rows 4- or 16-byte aligned): wave
    // loads of 256 B (a dword per lane) or 1 KiB (dwordx4 per lane) from a buffer resource
    // straight into LDS.  The resource ends after the last valid row, so rows past the image read
    // as zero without a branch; the lane part of the address is one VGPR, the chunk part a scalar
    // offset.  Otherwise element by element, zeros outside the image.
    template <int VB, bool FULL = false>
    static __device__ __forceinline__ void dma(const BuildDesc &d, uint32_t *tile, int64_t ys, int64_t xb, int nvalid,
                                               int lane) {
        constexpr int CB = 64 * VB;                         // bytes per wave load
        const unsigned char *base = static_cast<const unsigned char *>(d.img) +
                                    (ys * d.ipitch + xb) * static_cast<int64_t>(sizeof(T));
        const uint32_t pitchb = static_cast<uint32_t>(d.ipitch * static_cast<int64_t>(sizeof(T)));
        const uint32_t recs = static_cast<uint32_t>(nvalid - 1) * pitchb + ROWB;
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned char *>(base), 0, static_cast<int>(recs), kRsrcWord3);
        const uint32_t lb = static_cast<uint32_t>(lane) * VB;
        const uint32_t voff = (lb / ROWB) * pitchb + lb % ROWB;
        auto chunk = [&](int c) {
            const uint32_t cb = static_cast<uint32_t>(c) * CB;
            const uint32_t so = (cb / ROWB) * pitchb + cb % ROWB;
            auto *dst = (__attribute__((address_space(3))) void *)(tile + c * (CB / 4));
            if constexpr (VB == 16)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dst, 16, voff, static_cast<int>(so), 0, 0);
            else
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dst, 4, voff, static_cast<int>(so), 0, 0);
        };
        if constexpr (FULL) {
            // Every chunk of the tile, so that each tile load is at least kFullLoads vector memory
            // instructions and a wait may leave the next tile's loads in flight (kFullLoads).
            // Rows past nvalid lie past the resource and read as zero.
#pragma unroll
            for (int c = 0; c < TILEB / CB; ++c) chunk(c);
        } else {
            const int nch = (nvalid * ROWB + CB - 1) / CB;      // chunks holding valid rows
#pragma unroll 4
            for (int c = 0; c < nch; ++c) chunk(c);
        }
    }

    // Vector memory instructions a FULL tile load issues at least (16-byte chunks; 4-byte chunks
    // issue four times as many); the element path instead waits for its own loads.
    static constexpr int kFullLoads = TILEB / 1024 < 63 ? TILEB / 1024 : 63;

    template <bool FULL = false>
    static __device__ void load(const BuildDesc &d, uint32_t *tile_buf, int64_t ys, int64_t xb, int nvalid,
                                int lane) {
        if (d.img_vb >= 4 && xb + BW <= d.W) {
            if (d.img_vb >= 16) dma<16, FULL>(d, tile_buf, ys, xb, nvalid, lane);
            else dma<4, FULL>(d, tile_buf, ys, xb, nvalid, lane);
        } else {
            const T *img = static_cast<const T *>(d.img);
            T *tile = reinterpret_cast<T *>(tile_buf);
#pragma unroll 4
            for (int e = lane; e < nvalid * BW; e += 64) {
                const int row = e / BW, col = e % BW;
                const int64_t y = ys + row, x = xb + col;
                tile[e] = (row < nvalid && x < d.W) ? img[y * d.ipitch + x] : static_cast<T>(0);
            }
        }
    }

};

// ------------------------------------------------------------------ helper-wave strip worker
//
// Same arithmetic and lookback protocol as Build, with the global loads and the lookback kept off
// the compute waves' path.  A workgroup has NW compute waves and one helper wave; the compute
// waves only read LDS, scan and store.  Two pipelines:
//   P3 = false (two tile buffers, one barrier per block): the helper stages the next tile straight
//     into LDS (global_load_lds, no VGPRs), forms its column sums for every compute wave and runs
//     the decoupled lookback for it, one block ahead of the compute waves.  Least LDS: two
//     workgroups per CU for 8-bit tiles, which tall images need to reach the write ceiling.
//   P3 = true (three tile buffers, two barriers per block): the helper stages tiles two blocks
//     ahead; each compute wave forms the column sums of its own rows of tile b+1, and the helper
//     runs only the lookback of block b+1 while the compute waves work on block b.  The helper's
//     path per block is a fraction of P3 = false's, which matters where each CU holds one strip
//     and the helper's latency sets the pace.
//     Barriers: X_b ("column sums of b+1 are in LDS") and Y_b ("block b is done, the lookback of
//     b+1 is in LDS, tile b+2 has landed").
// The helper and the compute waves run separate loops with the same barriers, so the compute
// waves' barriers wait only for their LDS accesses, never for the helper's DMA or for their own
// table stores (gfx9 counts stores and loads on one vector memory counter).
template <typename T, bool SQ, int PX, int RW, int NW, int WIN, bool NTS = false, bool P3 = false>
struct Build2 {
    using B1 = Build<T, SQ, PX, RW, NW, MODE_LOOKBACK>;   // shared helpers (column map, lookback)
    static constexpr int TH = RW * NW;
    static constexpr int BW = 64 * PX;
    static constexpr int NS = PX / 2;
    static constexpr int NT = (NW + 1) * 64;
    static constexpr int HELPER = NW;                     // wave index of the helper
    static constexpr int ROWB = BW * static_cast<int>(sizeof(T));
    static constexpr int TILEB = TH * ROWB;
    static constexpr int NTILE = P3 ? 3 : 2;              // tile buffers: blocks b, b+1 (, b+2)
    static_assert(TILEB % 1024 == 0, "tile is a whole number of 1 KiB wave loads");
    using QT = typename B1::QT;

    struct Smem {
        uint32_t tile[NTILE][TILEB / 4];                  // image tiles of blocks b, b+1 (, b+2)
        uint32_t cs[2][NW][BW];                           // per compute wave column sums (blocks b, b+1)
        QT csq[SQ ? 2 : 1][SQ ? NW : 1][SQ ? BW : 1];
        uint64_t v[2][BW];                                // column totals above the strip
        uint64_t vq[SQ ? 2 : 1][SQ ? BW : 1];
        long long ticket;
    };

    static __device__ void load_tile(const BuildDesc &d, Smem &sm, int tb, int64_t ys, int64_t xb, int nvalid,
                                     int lane) {
        TileStage<T, PX, TH>::load(d, sm.tile[tb], ys, xb, nvalid, lane);
    }

    // Wait for this wave's outstanding global loads (the tile DMA) and LDS traffic.
    static __device__ __forceinline__ void wait_loads() { __builtin_amdgcn_s_waitcnt(0x0070); }

    // Helper wave (P3 = false): column sums of tile tb for every compute wave into column-sum
    // buffer buf, then the lookback of block xb (lookback_block).
    static __device__ void prepare(const BuildDesc &d, Smem &sm, int tb, int buf, int64_t xb, int strip, int nvalid,
                                   int rw, int lane, uint64_t *state, unsigned int *fault) {
        for (int w = 0; w < NW; ++w) {
            const int left = nvalid - w * rw;
            colsums(sm, tb, buf, w, w * rw, left < rw ? (left > 0 ? left : 0) : rw, lane);
        }
        lookback_block(d, sm, buf, xb, strip, lane, state, fault);
    }

    // Compute wave: column sums of its own rows (rows_ok from wave row row0) of tile tb into
    // column-sum buffer buf.
    static __device__ void colsums(Smem &sm, int tb, int buf, int wave, int row0, int rows_ok, int lane) {
        uint32_t cs[PX];
        QT csq[PX];
#pragma unroll
        for (int p = 0; p < PX; ++p) { cs[p] = 0; csq[p] = 0; }
        const T *tile = reinterpret_cast<const T *>(sm.tile[tb]) + 2 * lane + row0 * BW;
#pragma unroll 8
        for (int r = 0; r < rows_ok; ++r) {
            const T *row = tile + r * BW;
#pragma unroll
            for (int sb = 0; sb < NS; ++sb) {
                uint32_t pair;
                if (sizeof(T) == 1) pair = *reinterpret_cast<const uint16_t *>(row + 128 * sb);
                else pair = *reinterpret_cast<const uint32_t *>(row + 128 * sb);
                const uint32_t v0 = sizeof(T) == 1 ? (pair & 0xffu) : (pair & 0xffffu);
                const uint32_t v1 = sizeof(T) == 1 ? ((pair >> 8) & 0xffu) : (pair >> 16);
                cs[2 * sb] += v0;
                cs[2 * sb + 1] += v1;
                if (SQ) {
                    csq[2 * sb] += static_cast<QT>(v0 * v0);
                    csq[2 * sb + 1] += static_cast<QT>(v1 * v1);
                }
            }
        }
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            sm.cs[buf][wave][lane * PX + p] = cs[p];
            if (SQ) sm.csq[buf][wave][lane * PX + p] = csq[p];
        }
    }

    // Helper wave: the strip's column sums of block xb (the compute waves' sums in buffer buf),
    // the lookback for it, and the column totals above the strip into v[buf] / vq[buf].
    static __device__ void lookback_block(const BuildDesc &d, Smem &sm, int buf, int64_t xb, int strip, int lane,
                                          uint64_t *state, unsigned int *fault) {
        uint64_t a[PX], aq[PX];
#pragma unroll
        for (int p = 0; p < PX; ++p) { a[p] = 0; aq[p] = 0; }
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int p = 0; p < PX; ++p) {
                a[p] += sm.cs[buf][w][lane * PX + p];
                if (SQ) aq[p] += sm.csq[buf][w][lane * PX + p];
            }
        uint64_t v[PX], vq[PX];
        if constexpr (WIN > 0) {
            B1::template lookback_win<WIN>(d, strip, xb, lane, a, aq, v, vq, state, fault);
        } else {
            const uint64_t *tot = state + d.state_off + static_cast<int64_t>(strip) * d.Wp + xb + 2 * lane;
            const uint64_t *tot_q = state + d.state_q_off + static_cast<int64_t>(strip) * d.Wp + xb + 2 * lane;
#pragma unroll
            for (int p = 0; p < PX; ++p) {
                v[p] = tot[B1::soff(p)];
                vq[p] = SQ ? tot_q[B1::soff(p)] : 0;
            }
        }
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            sm.v[buf][lane * PX + p] = v[p];
            if (SQ) sm.vq[buf][lane * PX + p] = vq[p];
        }
    }

    // Compute wave: the rows of block xb (tile buffer tb, column sums and totals buffer buf).
    static __device__ void compute(const BuildDesc &d, const Smem &sm, int tb, int buf, int64_t xb, int wave, int rw,
                                   int lane, int rows_ok, uint64_t *S_w, uint64_t *Q_w, uint32_t pitch_bytes,
                                   uint64_t &lrow, uint64_t &lrow_q, uint64_t &ucarry, uint64_t &ucarry_q) {
        uint64_t u[PX], uq[PX];
        {
            uint64_t c[PX], cq[PX];
#pragma unroll
            for (int p = 0; p < PX; ++p) {
                c[p] = sm.v[buf][lane * PX + p];
                cq[p] = SQ ? sm.vq[buf][lane * PX + p] : 0;
            }
            for (int w = 0; w < wave; ++w)
#pragma unroll
                for (int p = 0; p < PX; ++p) {
                    c[p] += sm.cs[buf][w][lane * PX + p];
                    if (SQ) cq[p] += sm.csq[buf][w][lane * PX + p];
                }
#pragma unroll
            for (int sb = 0; sb < NS; ++sb) {
                const uint64_t pair = add64(c[2 * sb], c[2 * sb + 1]);
                const uint64_t incl = wave_scan(pair);
                const uint64_t b = ucarry + (incl - pair);
                u[2 * sb] = b + c[2 * sb];
                u[2 * sb + 1] = b + pair;
                ucarry += readlane(incl, 63);
                if (SQ) {
                    const uint64_t pair_q = add64(cq[2 * sb], cq[2 * sb + 1]);
                    const uint64_t incl_q = wave_scan(pair_q);
                    const uint64_t b_q = ucarry_q + (incl_q - pair_q);
                    uq[2 * sb] = b_q + cq[2 * sb];
                    uq[2 * sb + 1] = b_q + pair_q;
                    ucarry_q += readlane(incl_q, 63);
                }
            }
        }
        const bool vec = d.sat_vec && xb + BW <= d.W;
        const uint32_t row_recs = static_cast<uint32_t>((d.W - xb) * 8);
        const T *trow = reinterpret_cast<const T *>(sm.tile[tb] + wave * rw * ROWB / 4) + 2 * lane;
        if (vec) {
            lrow += block_rows<T, PX, false, false, true, NTS ? kStNT : 0>(trow, lane, u, lrow, S_w + xb, rows_ok, row_recs, pitch_bytes);
            if (SQ) lrow_q += block_rows<T, PX, true, B1::WIDE_SQ, true, NTS ? kStNT : 0>(trow, lane, uq, lrow_q, Q_w + xb, rows_ok, row_recs, pitch_bytes);
        } else {
            lrow += block_rows<T, PX, false, false, false, NTS ? kStNT : 0>(trow, lane, u, lrow, S_w + xb, rows_ok, row_recs, pitch_bytes);
            if (SQ) lrow_q += block_rows<T, PX, true, B1::WIDE_SQ, false, NTS ? kStNT : 0>(trow, lane, uq, lrow_q, Q_w + xb, rows_ok, row_recs, pitch_bytes);
        }
    }

    // Compute wave of a segment that starts mid-row (segment k >= 1 at column x0): the row totals
    // left of x0 for its rows (lane r: row yw + r) and the table value at (yw - 1, x0 - 1), from
    // the boundary column the pre-pass wrote.
    static __device__ __forceinline__ void seg_carries(const BuildDesc &d, int seg, int64_t yw, int lane, int rows_ok,
                                                       uint64_t &lrow, uint64_t &lrow_q, uint64_t &ucarry,
                                                       uint64_t &ucarry_q) {
        const int64_t off = static_cast<int64_t>(seg - 1) * (d.H + 1);
        const uint64_t *P = d.seg_pre + off;
        ucarry = P[yw];
        if (lane < rows_ok) lrow = P[yw + lane + 1] - P[yw + lane];
        if constexpr (SQ) {
            const uint64_t *PQ = d.seg_pre_q + off;
            ucarry_q = PQ[yw];
            if (lane < rows_ok) lrow_q = PQ[yw + lane + 1] - PQ[yw + lane];
        }
    }

    // One work item: strip item / nseg, its column segment item % nseg (blocks b0 .. b0 + nb - 1).
    static __device__ void strip(const BuildDesc &d, int item, uint64_t *state, unsigned int *fault, Smem &sm) {
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
        const bool helper = wave == HELPER;
        const int nseg = d.nseg;
        const int strip_idx = nseg > 1 ? item / nseg : item;
        const int seg = nseg > 1 ? item - strip_idx * nseg : 0;
        const int b0 = seg * d.seg_blocks;
        const int nb = d.nblocks - b0 < d.seg_blocks ? d.nblocks - b0 : d.seg_blocks;
        const int64_t x0 = static_cast<int64_t>(b0) * BW;
        const int th = d.strip_h, rw = d.wave_rows;                       // th <= TH, rw <= RW
        const int64_t ys = static_cast<int64_t>(strip_idx) * th;
        const int nvalid = static_cast<int>(d.H - ys < th ? d.H - ys : th);
        const int64_t yw = ys + (helper ? 0 : wave) * rw;
        const int left = nvalid - wave * rw;
        const int rows_ok = helper ? 0 : (left < rw ? (left > 0 ? left : 0) : rw);
        uint64_t *S_w = d.S + yw * d.spitch;
        uint64_t *Q_w = SQ ? d.Q + yw * d.spitch : nullptr;
        const uint32_t pitch_bytes = static_cast<uint32_t>(d.spitch * 8);
        uint64_t lrow = 0, lrow_q = 0, ucarry = 0, ucarry_q = 0;
        if (seg > 0 && rows_ok > 0) seg_carries(d, seg, yw, lane, rows_ok, lrow, lrow_q, ucarry, ucarry_q);

        if constexpr (!P3) {
            // One loop for all waves, one barrier per block.  Measured on tall 8-bit images (two
            // workgroups per CU): the joined loop, whose barrier also drains the compute waves'
            // table stores of the block, is 5-7 % faster than separate helper and compute loops.
            if (helper) {
                __builtin_amdgcn_s_setprio(3);   // see below
                load_tile(d, sm, 0, ys, x0, nvalid, lane);
                wait_loads();
                prepare(d, sm, 0, 0, x0, strip_idx, nvalid, rw, lane, state, fault);
            }
            lds_barrier();
            if (helper && nb > 1) load_tile(d, sm, 1, ys, x0 + BW, nvalid, lane);
            for (int i = 0; i < nb; ++i) {
                const int buf = i & 1;
                const int64_t xb = x0 + static_cast<int64_t>(i) * BW;
                if (!helper) {
                    compute(d, sm, buf, buf, xb, wave, rw, lane, rows_ok, S_w, Q_w, pitch_bytes, lrow, lrow_q,
                            ucarry, ucarry_q);
                } else if (i + 1 < nb) {
                    wait_loads();
                    prepare(d, sm, buf ^ 1, buf ^ 1, xb + BW, strip_idx, nvalid, rw, lane, state, fault);
                }
                lds_barrier();
                if (helper && i + 2 < nb) load_tile(d, sm, buf, ys, xb + 2 * BW, nvalid, lane);
            }
            return;
        }
        // Barriers: Z (tiles 0 and 1 landed), X' / Y' (column sums, then lookback, of block 0),
        // then X_b / Y_b per block; the same count in both loops.
        if (helper) {
            // The helper shares a SIMD with a compute wave that has VALU work ready nearly every
            // cycle; at the default (age-ordered) priority the helper, the youngest wave, got only
            // the leftover issue slots and its short lookback and DMA steps became the critical
            // path.  Its work is a few instructions per block, so it goes first.
            __builtin_amdgcn_s_setprio(3);
            load_tile(d, sm, 0, ys, x0, nvalid, lane);
            if (nb > 1) load_tile(d, sm, 1, ys, x0 + BW, nvalid, lane);
            wait_loads();
            lds_barrier();                                                        // Z
            lds_barrier();                                                        // X'
            lookback_block(d, sm, 0, x0, strip_idx, lane, state, fault);
            lds_barrier();                                                        // Y'
            for (int i = 0; i < nb; ++i) {
                const int64_t xb = x0 + static_cast<int64_t>(i) * BW;
                if (i + 2 < nb) load_tile(d, sm, (i + 2) % NTILE, ys, xb + 2 * BW, nvalid, lane);
                dma_barrier();                                                    // X_b: tile b+2 in flight
                if (i + 1 < nb) lookback_block(d, sm, (i + 1) & 1, xb + BW, strip_idx, lane, state, fault);
                wait_loads();
                lds_barrier();                                                    // Y_b
            }
        } else {
            const int row0 = wave * rw;
            lds_barrier();                                                        // Z
            colsums(sm, 0, 0, wave, row0, rows_ok, lane);
            lds_barrier();                                                        // X'
            lds_barrier();                                                        // Y'
            for (int i = 0; i < nb; ++i) {
                const int64_t xb = x0 + static_cast<int64_t>(i) * BW;
                if (i + 1 < nb) colsums(sm, (i + 1) % NTILE, (i + 1) & 1, wave, row0, rows_ok, lane);
                lds_barrier();                                                    // X_b
                compute(d, sm, i % NTILE, i & 1, xb, wave, rw, lane, rows_ok, S_w, Q_w, pitch_bytes, lrow, lrow_q,
                        ucarry, ucarry_q);
                lds_barrier();                                                    // Y_b
            }
        }
    }
};

// ------------------------------------------------------------------ tables of pixel powers
//
// The helper-wave build of Build2 for NP tables at once: the tables of pixel^1 .. pixel^NP (the
// integral image of Sec. II-B applied to I^k), from one read of the image.  The helper wave forms
// per-wave column sums of every power and runs one decoupled lookback over NP state planes; the
// compute waves make one pass over the LDS tile per power, each with the scan type the power
// needs (32-bit while a wave's 128 pixel powers sum below 2^32, else 64-bit).

// Largest value of pixel^P, saturated at 2^64 - 1.
template <typename T, int P>
constexpr uint64_t max_pow() {
    const uint64_t m = sizeof(T) == 1 ? 255u : 65535u;
    uint64_t r = 1;
    for (int i = 0; i < P; ++i) r = r > ~0ull / m ? ~0ull : r * m;
    return r;
}

// Narrowest exact types: one pixel's power, a sum of up to 16 of them (a wave's rows), and the
// scan of a wave's 128 pixel powers.
template <typename T, int P>
using PowT = typename std::conditional<(max_pow<T, P>() <= 0xffffffffull), uint32_t, uint64_t>::type;
template <typename T, int P>
using SumT = typename std::conditional<(max_pow<T, P>() <= 0xffffffffull / 16), uint32_t, uint64_t>::type;
template <typename T, int P>
using PowScan = typename std::conditional<(max_pow<T, P>() <= 0xffffffffull / 128), uint32_t, uint64_t>::type;

// Sum of two values that feed a DPP scan.  In 64 bits: two 32-bit adds (with carry) and then the
// two wait states a DPP read of a fresh VALU result needs, in one asm block.  Written as plain
// code, the two halves may be fused into one 64-bit add (v_lshl_add_u64) whose result the
// compiler does not guard for a following DPP read.
__device__ __forceinline__ uint32_t dpp_src_sum(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ uint64_t dpp_src_sum(uint64_t a, uint64_t b) {
    uint32_t lo, hi;
    asm volatile("v_add_co_u32 %0, vcc, %2, %3\n\tv_addc_co_u32 %1, vcc, %4, %5, vcc\n\ts_nop 1"
                 : "=&v"(lo), "=v"(hi)
                 : "v"(static_cast<uint32_t>(a)), "v"(static_cast<uint32_t>(b)), "v"(static_cast<uint32_t>(a >> 32)),
                   "v"(static_cast<uint32_t>(b >> 32))
                 : "vcc");
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// pixel^P, each product in the narrowest type that holds it exactly (8-bit pixels: all 32-bit).
template <typename T, int P>
__device__ __forceinline__ PowT<T, P> pow_of(uint32_t v) {
    if constexpr (P == 1) return v;
    else return static_cast<PowT<T, P>>(pow_of<T, P - 1>(v)) * v;
}

template <typename T, int NP, int PX, int RW, int NW, bool NTS>
struct BuildPow {
    using B1 = Build<T, false, PX, RW, NW, MODE_LOOKBACK>;   // lookback word map (lslot)
    static constexpr int TH = RW * NW;
    static constexpr int BW = 64 * PX;
    static constexpr int NS = PX / 2;
    static constexpr int HELPER = NW;
    static constexpr int ROWB = BW * static_cast<int>(sizeof(T));
    static constexpr int TILEB = TH * ROWB;
    static_assert(NP >= 1 && NP <= 4 && NP * PX <= 32, "power count and lane pixels fit the done mask");
    // Tile buffers: two, or three where the state with two already takes more than half of the
    // 160 KiB of LDS (one workgroup per CU) and a third still fits.  With three the DMA of block
    // b+3 is issued as block b's buffer frees, so a tile has a whole block step to land.
    static constexpr size_t kLds2 = 2 * static_cast<size_t>(TILEB) + 2 * NP * NW * BW * 8 + 2 * NP * BW * 8 + 8;
    static constexpr int NTILE = kLds2 > 80 * 1024 && kLds2 + TILEB <= 156 * 1024 ? 3 : 2;
    using Stage = TileStage<T, PX, TH>;

    struct Smem {
        uint32_t tile[NTILE][TILEB / 4];                  // image tiles of blocks b, b+1 (, b+2)
        uint64_t cs[2][NP][NW][BW];                       // per compute wave column sums of pixel^p
        uint64_t v[2][NP][BW];                            // column totals above the strip
        long long ticket;
    };

    static __device__ __forceinline__ uint64_t *table(const BuildDesc &d, int p) {
        return p == 0 ? d.S : p == 1 ? d.Q : p == 2 ? d.T3 : d.T4;
    }

    // Decoupled lookback over NP planes of nstrips * Wp words (the protocol of Build::lookback).
    static __device__ void lookback(const BuildDesc &d, int strip, int64_t xb, int lane, const uint64_t (&a)[NP][PX],
                                    uint64_t (&v)[NP][PX], uint64_t *state, unsigned int *fault) {
        const int64_t plane = static_cast<int64_t>(d.nstrips) * d.Wp;
        const int64_t col0 = xb + lane;
        uint64_t *mine = state + d.state_off + static_cast<int64_t>(strip) * d.Wp + col0;
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < PX; ++i) v[p][i] = 0;
        const uint64_t first = strip == 0 ? kStPrefix : kStAggregate;
        stress_delay(d.stress, strip, xb, 1);
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < PX; ++i) store_state(mine + p * plane + B1::lslot(i), first | a[p][i]);
        if (strip == 0) return;
        constexpr uint32_t kAll = NP * PX == 32 ? 0xffffffffu : ((1u << (NP * PX)) - 1u);
        uint32_t done = 0, spins = 0;
        int j = strip - 1;
        for (;;) {
            const uint64_t *up = state + d.state_off + static_cast<int64_t>(j) * d.Wp + col0;
            uint64_t w[NP][PX];
            bool ready = true;
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    w[p][i] = 0;
                    if (!(done & (1u << (p * PX + i)))) {
                        w[p][i] = load_state(up + p * plane + B1::lslot(i));
                        ready = ready && (w[p][i] >> 62) != 0;
                    }
                }
            if (!__all(ready)) {
                if (++spins > kSpinLimit) {
                    atomicOr(fault, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
                continue;
            }
#pragma unroll
            for (int p = 0; p < NP; ++p)
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    const uint32_t bit = 1u << (p * PX + i);
                    if (!(done & bit)) {
                        v[p][i] += w[p][i] & kValueMask;
                        if ((w[p][i] >> 62) == 2 || j == 0) done |= bit;
                    }
                }
            if (__all(done == kAll)) break;
            --j;
        }
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < PX; ++i) {
                if (p == 0 && i == 0) stress_delay(d.stress, strip, xb, 2);
                store_state(mine + p * plane + B1::lslot(i), kStPrefix | (v[p][i] + a[p][i]));
            }
    }

    // Helper wave: per-wave column sums of every power of tile tb into buffer buf, the lookback,
    // and the column totals above the strip for the compute waves.
    static __device__ void prepare(const BuildDesc &d, Smem &sm, int tb, int buf, int64_t xb, int strip, int nvalid,
                                   int rw, int lane, uint64_t *state, unsigned int *fault) {
        uint64_t a[NP][PX];
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < PX; ++i) a[p][i] = 0;
        const T *tile = reinterpret_cast<const T *>(sm.tile[tb]) + 2 * lane;
        for (int w = 0; w < NW; ++w) {
            SumT<T, 1> c1[PX];
            SumT<T, 2> c2[PX];
            SumT<T, 3> c3[PX];
            SumT<T, 4> c4[PX];
#pragma unroll
            for (int i = 0; i < PX; ++i) { c1[i] = 0; c2[i] = 0; c3[i] = 0; c4[i] = 0; }
            const int r_end = nvalid - w * rw < rw ? nvalid - w * rw : rw;
            for (int r = 0; r < r_end; ++r) {
                const T *row = tile + (w * rw + r) * BW;
#pragma unroll
                for (int sb = 0; sb < NS; ++sb) {
                    uint32_t pair;
                    if (sizeof(T) == 1) pair = *reinterpret_cast<const uint16_t *>(row + 128 * sb);
                    else pair = *reinterpret_cast<const uint32_t *>(row + 128 * sb);
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const uint32_t v = sizeof(T) == 1 ? ((pair >> (8 * j)) & 0xffu) : ((pair >> (16 * j)) & 0xffffu);
                        const int i = 2 * sb + j;
                        c1[i] += v;
                        if constexpr (NP >= 2) {
                            const PowT<T, 2> q2 = pow_of<T, 2>(v);
                            c2[i] += q2;
                            if constexpr (NP >= 3) {
                                const PowT<T, 3> q3 = static_cast<PowT<T, 3>>(q2) * v;
                                c3[i] += q3;
                                if constexpr (NP >= 4) c4[i] += static_cast<PowT<T, 4>>(q3) * v;
                            }
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < PX; ++i) {
                const uint64_t cw[4] = {c1[i], c2[i], c3[i], c4[i]};
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    sm.cs[buf][p][w][lane * PX + i] = cw[p];
                    a[p][i] += cw[p];
                }
            }
        }
        uint64_t v[NP][PX];
        lookback(d, strip, xb, lane, a, v, state, fault);
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int i = 0; i < PX; ++i) sm.v[buf][p][lane * PX + i] = v[p][i];
    }

    // Compute wave: the rows of power P (table P-1) of block xb (tile tb, sums and totals buf).
    template <int P>
    static __device__ __forceinline__ void power_rows(const BuildDesc &d, const Smem &sm, int tb, int buf, int64_t xb, int wave,
                                                      int rw, int lane, int rows_ok, int64_t yw, uint32_t pitch_bytes,
                                                      uint64_t &lrow, uint64_t &ucarry) {
        using ST = PowScan<T, P>;
        uint64_t u[PX];
        {
            uint64_t c[PX];
#pragma unroll
            for (int i = 0; i < PX; ++i) c[i] = sm.v[buf][P - 1][lane * PX + i];
            for (int w = 0; w < wave; ++w)
#pragma unroll
                for (int i = 0; i < PX; ++i) c[i] += sm.cs[buf][P - 1][w][lane * PX + i];
#pragma unroll
            for (int sb = 0; sb < NS; ++sb) {
                const uint64_t pair = dpp_src_sum(c[2 * sb], c[2 * sb + 1]);
                const uint64_t incl = wave_scan(pair);
                const uint64_t b = ucarry + (incl - pair);
                u[2 * sb] = b + c[2 * sb];
                u[2 * sb + 1] = b + pair;
                ucarry += readlane(incl, 63);
            }
        }
        uint64_t *blk0 = table(d, P - 1) + yw * d.spitch + xb;
        const bool vec = d.sat_vec && xb + BW <= d.W;
        const uint32_t row_recs = static_cast<uint32_t>((d.W - xb) * 8);
        const T *trow = reinterpret_cast<const T *>(sm.tile[tb] + wave * rw * ROWB / 4) + 2 * lane;
        uint64_t acc[PX];
#pragma unroll
        for (int i = 0; i < PX; ++i) acc[i] = 0;
        uint64_t tvec = 0;
        const uint32_t voff = static_cast<uint32_t>(lane) * 16;
        const uint32_t blk_recs = rows_ok > 0 ? (rows_ok - 1) * pitch_bytes + row_recs : 0;
        const i32x4 rs_blk = make_rsrc(blk0, vec ? blk_recs : 0);
        const char *rowp = reinterpret_cast<const char *>(blk0);
        uint32_t roff = 0;
#pragma unroll 1
        for (int r = 0; r < rows_ok; ++r) {
            uint64_t base = readlane(lrow, r);
            const __amdgpu_buffer_rsrc_t rs_row = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<char *>(rowp), 0, vec ? 0 : static_cast<int>(row_recs), kRsrcWord3);
#pragma unroll
            for (int sb = 0; sb < NS; ++sb) {
                uint32_t pairv;
                if (sizeof(T) == 1) pairv = *reinterpret_cast<const uint16_t *>(trow + 128 * sb);
                else pairv = *reinterpret_cast<const uint32_t *>(trow + 128 * sb);
                const uint32_t v0 = sizeof(T) == 1 ? (pairv & 0xffu) : (pairv & 0xffffu);
                const uint32_t v1 = sizeof(T) == 1 ? ((pairv >> 8) & 0xffu) : (pairv >> 16);
                const ST a0 = pow_of<T, P>(v0), a1 = pow_of<T, P>(v1);
                const ST pair = dpp_src_sum(a0, a1);
                const ST incl = wave_scan(pair);
                const uint64_t b = base + (incl - pair);
                acc[2 * sb] += b + a0;
                acc[2 * sb + 1] += b + pair;
                const uint64_t o0 = u[2 * sb] + acc[2 * sb], o1 = u[2 * sb + 1] + acc[2 * sb + 1];
                if (vec) {
                    store16_rsrc<NTS ? kStNT : 0>(u32x4{static_cast<uint32_t>(o0), static_cast<uint32_t>(o0 >> 32),
                                            static_cast<uint32_t>(o1), static_cast<uint32_t>(o1 >> 32)},
                                      rs_blk, voff + sb * 1024, roff);
                } else {
                    __builtin_amdgcn_raw_buffer_store_b64(u32x2{static_cast<uint32_t>(o0), static_cast<uint32_t>(o0 >> 32)},
                                                          rs_row, voff + sb * 1024, 0, store_aux(NTS ? kStNT : 0));
                    __builtin_amdgcn_raw_buffer_store_b64(u32x2{static_cast<uint32_t>(o1), static_cast<uint32_t>(o1 >> 32)},
                                                          rs_row, voff + sb * 1024 + 8, 0, store_aux(NTS ? kStNT : 0));
                }
                base += readlane(incl, 63);
            }
            if (lane == r) tvec = base - readlane(lrow, r);
            trow += BW;
            rowp += pitch_bytes;
            roff += pitch_bytes;
        }
        lrow += tvec;
    }

    static __device__ void strip(const BuildDesc &d, int strip_idx, uint64_t *state, unsigned int *fault, Smem &sm) {
        const int lane = threadIdx.x & 63;
        const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
        const bool helper = wave == HELPER;
        const int th = d.strip_h, rw = d.wave_rows;                       // th <= TH, rw <= RW
        const int64_t ys = static_cast<int64_t>(strip_idx) * th;
        const int nvalid = static_cast<int>(d.H - ys < th ? d.H - ys : th);
        const int64_t yw = ys + (helper ? 0 : wave) * rw;
        const int left = nvalid - wave * rw;
        const int rows_ok = helper ? 0 : (left < rw ? (left > 0 ? left : 0) : rw);
        const uint32_t pitch_bytes = static_cast<uint32_t>(d.spitch * 8);
        uint64_t lrow[NP], ucarry[NP];       // lane r: row yw+r left of the block; table above, left of it
#pragma unroll
        for (int p = 0; p < NP; ++p) { lrow[p] = 0; ucarry[p] = 0; }

        // Separate helper and compute loops, as in Build2::strip.  Tile loads are FULL: with
        // three buffers the helper waits for tile b+1 while tile b+2, issued after it, stays in
        // flight (vector memory instructions complete in order, and tile b+2 is at least
        // kFullLoads of them); with two, or when no later tile was issued, it waits for all.
        if (helper) {
            const int nb = d.nblocks;
            Stage::template load<true>(d, sm.tile[0], ys, 0, nvalid, lane);
            __builtin_amdgcn_s_waitcnt(0x0070);
            prepare(d, sm, 0, 0, 0, strip_idx, nvalid, rw, lane, state, fault);
            lds_barrier();
            if (nb > 1) Stage::template load<true>(d, sm.tile[1], ys, BW, nvalid, lane);
            if (NTILE == 3 && nb > 2) Stage::template load<true>(d, sm.tile[2 % NTILE], ys, 2 * BW, nvalid, lane);
            for (int b = 0; b < nb; ++b) {
                const int buf = b & 1;
                const int64_t xb = static_cast<int64_t>(b) * BW;
                if (b + 1 < nb) {
                    constexpr int K = Stage::kFullLoads;
                    if (NTILE == 3 && b + 2 < nb)
                        __builtin_amdgcn_s_waitcnt((K & 15) | ((K >> 4) << 14) | (7 << 4));   // vmcnt(K) lgkmcnt(0)
                    else
                        __builtin_amdgcn_s_waitcnt(0x0070);
                    prepare(d, sm, (b + 1) % NTILE, buf ^ 1, xb + BW, strip_idx, nvalid, rw, lane, state, fault);
                }
                lds_barrier();
                if (b + NTILE < nb)
                    Stage::template load<true>(d, sm.tile[b % NTILE], ys, xb + NTILE * BW, nvalid, lane);
            }
        } else {
            lds_barrier();
            for (int b = 0; b < d.nblocks; ++b) {
                const int buf = b & 1, tb = b % NTILE;
                const int64_t xb = static_cast<int64_t>(b) * BW;
                power_rows<1>(d, sm, tb, buf, xb, wave, rw, lane, rows_ok, yw, pitch_bytes, lrow[0], ucarry[0]);
                if constexpr (NP >= 2) power_rows<2>(d, sm, tb, buf, xb, wave, rw, lane, rows_ok, yw, pitch_bytes, lrow[1], ucarry[1]);
                if constexpr (NP >= 3) power_rows<3>(d, sm, tb, buf, xb, wave, rw, lane, rows_ok, yw, pitch_bytes, lrow[2], ucarry[2]);
                if constexpr (NP >= 4) power_rows<4>(d, sm, tb, buf, xb, wave, rw, lane, rows_ok, yw, pitch_bytes, lrow[3], ucarry[3]);
                lds_barrier();
            }
        }
    }
};

template <typename T, int NP, int PX, int RW, int NW, bool NTS>
__global__ __launch_bounds__((NW + 1) * 64) void build_pow_kernel(BuildDesc d, long long total_items, uint64_t *state,
                                                                  BuildCtrl *ctrl) {
    using B = BuildPow<T, NP, PX, RW, NW, NTS>;
    __shared__ typename B::Smem sm;
    for (;;) {
        if (threadIdx.x == 0) sm.ticket = static_cast<long long>(atomicAdd(&ctrl->ticket, 1ull));
        __syncthreads();
        const long long t = static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(sm.ticket))) |
                            (static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(sm.ticket >> 32))) << 32);
        __syncthreads();
        if (t >= total_items) return;
        B::strip(d, __builtin_amdgcn_readfirstlane(static_cast<int>(t)), state, &ctrl->fault, sm);
    }
}

template <typename T, bool SQ, int PX, int RW, int NW, int WIN, bool NTS, bool P3>
__global__ __launch_bounds__((NW + 1) * 64) void build2_kernel(const BuildDesc *__restrict__ many, int n,
                                                               long long total_items, uint64_t *state, BuildCtrl *ctrl) {
    using B = Build2<T, SQ, PX, RW, NW, WIN, NTS, P3>;
    __shared__ typename B::Smem sm;
    for (;;) {
        if (threadIdx.x == 0) sm.ticket = static_cast<long long>(atomicAdd(&ctrl->ticket, 1ull));
        __syncthreads();
        const long long t = static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(sm.ticket))) |
                            (static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(sm.ticket >> 32))) << 32);
        __syncthreads();
        if (t >= total_items) return;
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (many[mid].first_item <= t) lo = mid;
            else hi = mid - 1;
        }
        const BuildDesc d = many[lo];   // by value: kept in registers, not reloaded after every store
        B::strip(d, __builtin_amdgcn_readfirstlane(static_cast<int>(t - d.first_item)), state, &ctrl->fault, sm);
    }
}

// Persistent strip kernel: each workgroup takes strips (of one image, or of a batch) from the
// ticket counter until none are left.  The occupancy hint holds the variants that can to 128
// VGPRs (four waves per SIMD, e.g. 4 pixels per lane on 8-bit images); the others (8 pixels per
// lane, or 16-bit pixels with squares) need more and stay at two or one wave per SIMD, for which
// the compiler reports the hint as not met (-Wpass-failed), as expected.
template <typename T, bool SQ, int PX, int RW, int NW, int MODE, bool NTS>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(16 / NW > 4 ? 4 : 16 / NW)))
void build_kernel(const BuildDesc *__restrict__ many, int n, long long total_items, uint64_t *state,
                  BuildCtrl *ctrl) {
    using B = Build<T, SQ, PX, RW, NW, MODE, NTS>;
    __shared__ typename B::Smem sm;
    for (;;) {
        if (threadIdx.x == 0) sm.ticket = static_cast<long long>(atomicAdd(&ctrl->ticket, 1ull));
        __syncthreads();
        const long long t = static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(sm.ticket))) |
                            (static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(sm.ticket >> 32))) << 32);
        __syncthreads();
        if (t >= total_items) return;
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (many[mid].first_item <= t) lo = mid;
            else hi = mid - 1;
        }
        const BuildDesc d = many[lo];   // by value: kept in registers, not reloaded after every store
        B::strip(d, __builtin_amdgcn_readfirstlane(static_cast<int>(t - d.first_item)), state, &ctrl->fault, sm);
    }
}

// Batched tables and window statistics in one persistent launch.  Tickets 0 .. build_items-1 are
// the (image, strip) items of the table build, image by image; the tickets after them are the
// chain-walk mean/std items of the images' windows, image by image.  A build item, once its
// strip's table rows are stored, releases them at agent scope and counts the strip in its image's
// ready counter.  A statistics item of image i first waits (bounded; bit 2 of the fault word on
// timeout) until every strip of image i is counted, then acquires; a workgroup acquires each image
// once, as its items come in ticket order.  Every wait is on items with smaller tickets, handed out
// before it, so progress never depends on dispatch order, and the statistics of early images run
// while the last strips of later ones are still being built.
template <typename T, int PX, int RW, int NW, bool NTS, int V>
__global__ __launch_bounds__(NW * 64) void fused_kernel(const BuildDesc *__restrict__ bd,
                                                        const GatherDesc *__restrict__ gd, int n,
                                                        long long build_items, long long total_items, uint64_t *state,
                                                        BuildCtrl *ctrl, unsigned int *ready) {
    static_assert(NW * 64 == 256, "statistics items run on 256 threads");
    using B = Build<T, true, PX, RW, NW, MODE_LOOKBACK, NTS, true>;   // device-coherent table stores
    __shared__ typename B::Smem sm;
    int acquired = -1;
    for (;;) {
        if (threadIdx.x == 0) sm.ticket = static_cast<long long>(atomicAdd(&ctrl->ticket, 1ull));
        __syncthreads();
        const long long t = static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(sm.ticket))) |
                            (static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(sm.ticket >> 32))) << 32);
        __syncthreads();
        if (t >= total_items) return;
        if (t < build_items) {
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (bd[mid].first_item <= t) lo = mid;
                else hi = mid - 1;
            }
            const BuildDesc d = bd[lo];
            B::strip(d, __builtin_amdgcn_readfirstlane(static_cast<int>(t - d.first_item)), state, &ctrl->fault, sm);
            // Release: the strip's table stores are device-coherent (written through the L2), so
            // once each wave has seen its stores complete they are visible on every XCD; no
            // write-back of the whole L2 (an agent-scope release fence) is needed, which per strip
            // cost a quarter of the launch.
            __builtin_amdgcn_s_waitcnt(0x0070);                  // vmcnt(0), lgkmcnt(0)
            __syncthreads();
            if (threadIdx.x == 0) {
                stress_delay(d.stress, static_cast<int>(t), 0, 3);
                __hip_atomic_fetch_add(ready + lo, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            const long long item = t - build_items;
            int lo = 0, hi = n - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (gd[mid].first_item <= item) lo = mid;
                else hi = mid - 1;
            }
            if (lo != acquired) {
                if (threadIdx.x == 0) {
                    const unsigned int need = static_cast<unsigned int>(bd[lo].nstrips);
                    uint32_t spins = 0;
                    while (__hip_atomic_load(ready + lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        if (++spins > kSpinLimit) {
                            atomicOr(&ctrl->fault, 4u);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                    }
                }
                __syncthreads();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                acquired = lo;
            }
            const GatherDesc d = gd[lo];
            chain_stats_item<V>(d, item - d.first_item);
        }
    }
}

// A few KiB of host data (descriptor tables) written to device memory from kernel arguments:
// the launch copies the arguments when it is enqueued, so the caller's host buffer is free once
// the launch returns (an asynchronous copy from pageable memory gives no such guarantee).
constexpr int kChunkWords = 448;   // 3.5 KiB per launch, inside the kernel-argument limit
struct WordChunk {
    uint64_t w[kChunkWords];
};

__global__ __launch_bounds__(512) void words_write_kernel(WordChunk c, uint64_t *dst, int nwords) {
    const int i = static_cast<int>(threadIdx.x);
    if (i < nwords) dst[i] = c.w[i];
}

// Zero the lookback words and reset the control header.
// When `slot` is non-null the single-image descriptor `one` is written there as well.
__global__ void clear_kernel(uint64_t *state, long long nwords, BuildCtrl *ctrl, BuildDesc one, BuildDesc *slot) {
    const long long i0 = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i0 == 0) {
        ctrl->ticket = 0;
        ctrl->fault = 0;
        if (slot) *slot = one;
    }
    const long long step = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long i = i0; 2 * i < nwords; i += step) {   // 8-byte stores: see store16_rsrc
        state[2 * i] = 0;
        state[2 * i + 1] = 0;
    }
}

// Pre-pass of a build split into column segments (BuildDesc::nseg > 1).  A segment that starts at
// column x0 > 0 needs, for each row of its strip, the row's total left of x0, and the table value
// just above its strip at column x0 - 1: both come from the table's column x0 - 1, which this
// pass computes for every segment boundary from one read of the image left of the last segment.
//
// segsum_kernel: sums[k * H + y] = sum of row y over segment k's columns (k < nseg - 1), and of the
// squared pixels; one wave per row, 16-byte loads where the rows allow them.
template <typename T, bool SQ>
__global__ __launch_bounds__(256) void segsum_kernel(BuildDesc d, long long segw, uint64_t *sums, uint64_t *sums_q) {
    const int wave = static_cast<int>(threadIdx.x >> 6), lane = static_cast<int>(threadIdx.x & 63);
    const int64_t y = static_cast<int64_t>(blockIdx.x) * 4 + wave;
    const int k = static_cast<int>(blockIdx.y);
    if (y >= d.H) return;
    const int64_t xb = static_cast<int64_t>(k) * segw;
    const int64_t xe = xb + segw < d.W ? xb + segw : d.W;
    const T *row = static_cast<const T *>(d.img) + y * d.ipitch;
    uint64_t acc = 0, accq = 0;
    if (d.img_vb >= 16) {
        constexpr int E = 16 / static_cast<int>(sizeof(T));      // pixels per 16-byte load
        for (int64_t x = xb + static_cast<int64_t>(lane) * E; x < xe; x += 64 * E) {
            if (x + E <= xe) {
                const u32x4 v = *reinterpret_cast<const u32x4 *>(row + x);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
#pragma unroll
                    for (int e = 0; e < 4 / static_cast<int>(sizeof(T)); ++e) {
                        const uint64_t px = (v[w] >> (8 * sizeof(T) * e)) & (sizeof(T) == 1 ? 0xffu : 0xffffu);
                        acc += px;
                        if (SQ) accq += px * px;
                    }
                }
            } else {
                for (int64_t xx = x; xx < xe; ++xx) {
                    const uint64_t px = row[xx];
                    acc += px;
                    if (SQ) accq += px * px;
                }
            }
        }
    } else {
        for (int64_t x = xb + lane; x < xe; x += 64) {
            const uint64_t px = row[x];
            acc += px;
            if (SQ) accq += px * px;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o);
        if (SQ) accq += __shfl_xor(accq, o);
    }
    if (lane == 0) {
        sums[static_cast<int64_t>(k) * d.H + y] = acc;
        if (SQ) sums_q[static_cast<int64_t>(k) * d.H + y] = accq;
    }
}

// Exclusive scan of one value per thread over a 1024-thread block (Hillis-Steele in LDS), and the
// block's sum; `buf` is 1024 words of LDS, free again on return.
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *buf) {
    const int t = static_cast<int>(threadIdx.x);
    buf[t] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint64_t add = t >= o ? buf[t - o] : 0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    const uint64_t incl = buf[t];
    __syncthreads();
    return incl - v;
}
__device__ __forceinline__ uint64_t block_sum(uint64_t v, uint64_t *buf) {
    const uint64_t ex = block_exclusive_scan(v, buf);
    buf[threadIdx.x] = ex + v;
    __syncthreads();
    const uint64_t total = buf[1023];
    __syncthreads();
    return total;
}

// segscan_kernel: for segment k = blockIdx.x + 1, its boundary column x0 - 1 (x0 = k * segw):
// word 0 the carried column totals left of x0 (zero without a carry), word y + 1 = word y + the
// total of row y left of x0 (sums of segments 0 .. k - 1).  Each thread takes a run of consecutive
// rows: run totals, a scan of the runs across the block, then the run's words.
template <bool SQ>
__global__ __launch_bounds__(1024) void segscan_kernel(BuildDesc d, long long segw, const uint64_t *sums,
                                                       const uint64_t *sums_q, uint64_t *pre, uint64_t *pre_q) {
    __shared__ uint64_t part[1024], part_q[1024];
    const int k = static_cast<int>(blockIdx.x) + 1;
    const int t = static_cast<int>(threadIdx.x);
    const int64_t x0 = static_cast<int64_t>(k) * segw;
    uint64_t c = 0, cq = 0;
    if (d.carry) {
        for (int64_t x = t; x < x0; x += 1024) {
            c += d.carry[x];
            if (SQ) cq += d.carry_q[x];
        }
    }
    const uint64_t K = block_sum(c, part), KQ = SQ ? block_sum(cq, part_q) : 0;
    const int64_t run = (d.H + 1023) / 1024;
    const int64_t r0 = static_cast<int64_t>(t) * run;
    const int64_t r1 = r0 + run < d.H ? r0 + run : d.H;
    uint64_t tot = 0, tot_q = 0;
    for (int64_t y = r0; y < r1; ++y)
        for (int j = 0; j < k; ++j) {
            tot += sums[static_cast<int64_t>(j) * d.H + y];
            if (SQ) tot_q += sums_q[static_cast<int64_t>(j) * d.H + y];
        }
    uint64_t *P = pre + static_cast<int64_t>(k - 1) * (d.H + 1);
    uint64_t *PQ = SQ ? pre_q + static_cast<int64_t>(k - 1) * (d.H + 1) : nullptr;
    uint64_t base = K + block_exclusive_scan(tot, part), base_q = SQ ? KQ + block_exclusive_scan(tot_q, part_q) : 0;
    if (t == 0) {
        P[0] = K;
        if (SQ) PQ[0] = KQ;
    }
    for (int64_t y = r0; y < r1; ++y) {
        for (int j = 0; j < k; ++j) {
            base += sums[static_cast<int64_t>(j) * d.H + y];
            if (SQ) base_q += sums_q[static_cast<int64_t>(j) * d.H + y];
        }
        P[y + 1] = base;
        if (SQ) PQ[y + 1] = base_q;
    }
}

// Reduce-then-scan ablation, phase 1: column totals of every strip (TH rows) of one image.
template <typename T, bool SQ, int PX, int TH>
__global__ __launch_bounds__(256) void colsum_kernel(BuildDesc d, uint64_t *state) {
    const int64_t xcol = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * PX;
    if (xcol >= d.Wp) return;
    const int64_t strip = blockIdx.y;
    uint64_t cs[PX], csq[PX];
#pragma unroll
    for (int p = 0; p < PX; ++p) { cs[p] = 0; csq[p] = 0; }
    const T *img = static_cast<const T *>(d.img);
    for (int r = 0; r < TH; ++r) {
        const int64_t y = strip * TH + r;
        if (y >= d.H) break;
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            if (xcol + p < d.W) {
                const uint64_t v = img[y * d.ipitch + xcol + p];
                cs[p] += v;
                csq[p] += v * v;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < PX; ++p) {
        state[d.state_off + strip * d.Wp + xcol + p] = cs[p];
        if (SQ) state[d.state_q_off + strip * d.Wp + xcol + p] = csq[p];
    }
}

// Reduce-then-scan ablation, phase 2: exclusive scan of the strip totals down each column,
// starting from the carried column totals of a band build (zero without them); the inclusive
// end of the scan is the band's total output.
__global__ __launch_bounds__(256) void colscan_kernel(uint64_t *state, long long off, long long Wp,
                                                      int nstrips, const uint64_t *carry, uint64_t *total,
                                                      long long W) {
    const long long x = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (x >= Wp) return;
    uint64_t run = (carry && x < W) ? carry[x] : 0;
    for (int i = 0; i < nstrips; ++i) {
        uint64_t *p = state + off + static_cast<long long>(i) * Wp + x;
        const uint64_t t = *p;
        *p = run;
        run += t;
    }
    if (total && x < W) total[x] = run;
}

// ------------------------------------------------------------------ column totals

// out[x] = carry[x] (zero without a carry); the squared output likewise.  A fill kernel, not a
// memset, so that a captured graph replays it correctly.
__global__ __launch_bounds__(256) void totals_init_kernel(const uint64_t *carry, const uint64_t *carry_q,
                                                          uint64_t *out, uint64_t *out_q, long long W) {
    const long long x = static_cast<long long>(blockIdx.x) * 256 + threadIdx.x;
    if (x >= W) return;
    out[x] = carry ? carry[x] : 0;
    if (out_q) out_q[x] = carry_q ? carry_q[x] : 0;
}

// Column totals of an image added to out (and of its squares to out_q): the prepass a band of
// rows needs before its build when the rows above it are built elsewhere.  A workgroup is four
// waves over a tile of kTotRowBytes-byte columns and rows_per rows; wave w sums the rows
// y0 + w, y0 + w + 4, ... of the tile in registers, kTotBatch rows' loads in flight at a time.  A
// wave sums at most 16384 rows, so its 32-bit sums of pixels and of 8-bit squares are exact; the
// four waves' sums meet in LDS, and each column's total goes to out with one 64-bit atomic add.
// Tiles wholly inside the image with 16-byte aligned rows give each lane 16 contiguous bytes of a
// row; other tiles give lane l the columns l, l + 64, ... (coalesced element loads).
constexpr int kTotRowBytes = 1024;
constexpr int kTotWaves = 4;
constexpr int kTotBatch = 8;
constexpr long long kTotMaxRows = 65536;   // rows per tile: 16384 per wave

template <typename T, bool SQ>
__global__ __launch_bounds__(64 * kTotWaves) void column_totals_kernel(const T *__restrict__ img, long long H,
                                                                       long long W, long long pitch,
                                                                       long long rows_per, long long ncol, int vec16,
                                                                       uint64_t *out, uint64_t *out_q) {
    constexpr int VEC = 16 / static_cast<int>(sizeof(T));            // columns per lane
    constexpr int CW = kTotRowBytes / static_cast<int>(sizeof(T));   // columns per tile
    using QT = typename std::conditional<sizeof(T) == 1, uint32_t, uint64_t>::type;
    __shared__ uint32_t red[kTotWaves * CW];
    __shared__ QT red_q[SQ ? kTotWaves * CW : 1];
    const long long cb = static_cast<long long>(blockIdx.x) % ncol, rb = static_cast<long long>(blockIdx.x) / ncol;
    const long long y0 = rb * rows_per;
    const long long y1 = y0 + rows_per < H ? y0 + rows_per : H;
    const long long xw = cb * CW;
    const int lane = static_cast<int>(threadIdx.x) & 63, wave = static_cast<int>(threadIdx.x) >> 6;
    uint32_t sum[VEC];
    QT sq[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) { sum[k] = 0; sq[k] = 0; }
    auto add16 = [&](const u32x4 t) {
        const uint32_t wd[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const uint32_t v = sizeof(T) == 1 ? (wd[k >> 2] >> (8 * (k & 3))) & 0xffu
                                              : (wd[k >> 1] >> (16 * (k & 1))) & 0xffffu;
            sum[k] += v;
            if (SQ) sq[k] += static_cast<QT>(v) * v;
        }
    };
    const bool fast = vec16 && xw + CW <= W;   // uniform over the workgroup
    long long y = y0 + wave;
    if (fast) {
        const T *base = img + xw + lane * VEC;
        for (; y + (kTotBatch - 1) * kTotWaves < y1; y += kTotBatch * kTotWaves) {
            u32x4 t[kTotBatch];
#pragma unroll
            for (int b = 0; b < kTotBatch; ++b)
                t[b] = *reinterpret_cast<const u32x4 *>(base + (y + b * kTotWaves) * pitch);
#pragma unroll
            for (int b = 0; b < kTotBatch; ++b) add16(t[b]);
        }
        for (; y < y1; y += kTotWaves) add16(*reinterpret_cast<const u32x4 *>(base + y * pitch));
    } else {
        for (; y < y1; y += kTotWaves) {
            const T *row = img + y * pitch + xw + lane;
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                const uint32_t v = xw + lane + 64 * k < W ? static_cast<uint32_t>(row[64 * k]) : 0u;
                sum[k] += v;
                if (SQ) sq[k] += static_cast<QT>(v) * v;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        const int c = fast ? lane * VEC + k : lane + 64 * k;   // column within the tile
        red[wave * CW + c] = sum[k];
        if (SQ) red_q[wave * CW + c] = sq[k];
    }
    __syncthreads();
    for (int c = static_cast<int>(threadIdx.x); c < CW; c += 64 * kTotWaves) {
        const long long x = xw + c;
        if (x < W) {
            uint64_t s = 0, q = 0;
#pragma unroll
            for (int w = 0; w < kTotWaves; ++w) {
                s += red[w * CW + c];
                if (SQ) q += red_q[w * CW + c];
            }
            atomicAdd(reinterpret_cast<unsigned long long *>(out + x), static_cast<unsigned long long>(s));
            if (SQ) atomicAdd(reinterpret_cast<unsigned long long *>(out_q + x), static_cast<unsigned long long>(q));
        }
    }
}

template <typename T, bool SQ>
hipError_t launch_totals_typed(const void *img, int64_t H, int64_t W, int64_t pitch, int vec16,
                               const uint64_t *carry, const uint64_t *carry_q, uint64_t *out, uint64_t *out_q,
                               hipStream_t stream) {
    hipLaunchKernelGGL(totals_init_kernel, dim3(static_cast<unsigned>((W + 255) / 256)), dim3(256), 0, stream, carry,
                       carry_q, out, out_q, static_cast<long long>(W));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int CW = kTotRowBytes / static_cast<int>(sizeof(T));
    constexpr int64_t kStep = kTotWaves * kTotBatch;
    const int64_t ncol = (W + CW - 1) / CW;
    // About 2048 workgroups (eight per compute unit, two rounds of four-wave groups): rows per
    // tile from that, a whole number of load batches, at most kTotMaxRows.
    int64_t rows_per = (H * ncol + 2047) / 2048;
    rows_per = (rows_per + kStep - 1) / kStep * kStep;
    if (rows_per > kTotMaxRows) rows_per = kTotMaxRows;
    const int64_t nrow = (H + rows_per - 1) / rows_per;
    hipLaunchKernelGGL((column_totals_kernel<T, SQ>), dim3(static_cast<unsigned>(ncol * nrow)), dim3(64 * kTotWaves),
                       0, stream, static_cast<const T *>(img), static_cast<long long>(H), static_cast<long long>(W),
                       static_cast<long long>(pitch), static_cast<long long>(rows_per), static_cast<long long>(ncol),
                       vec16, out, out_q);
    return hipGetLastError();
}

// ------------------------------------------------------------------ variants and launch

// Compiled variants: index, name, pixels per lane, rows per wave, waves, mode, lookback window
// (helper mode; 0 = column totals precomputed), adaptive strip height, non-temporal table stores.
#define SAT_BUILD_VARIANTS(X)                                                      \
    X(0, "lookback_px8_rw16_nw4", 8, 16, 4, MODE_LOOKBACK, 1, 1, false)            \
    X(1, "lookback_px4_rw16_nw4", 4, 16, 4, MODE_LOOKBACK, 1, 1, false)            \
    X(2, "lookback_px4_rw8_nw4", 4, 8, 4, MODE_LOOKBACK, 1, 1, false)              \
    X(3, "lookback_px4_rw8_nw8", 4, 8, 8, MODE_LOOKBACK, 1, 1, false)              \
    X(4, "reduce_scan_px4_rw16_nw4", 4, 16, 4, MODE_REDUCE_SCAN, 1, 0, false)      \
    X(5, "helper_px2_rw16_nw4", 2, 16, 4, MODE_HELPER, 1, 0, false)                \
    X(6, "helper_px4_rw16_nw4", 4, 16, 4, MODE_HELPER, 1, 0, false)                \
    X(7, "helper_reduce_scan_px4_rw16_nw4", 4, 16, 4, MODE_HELPER, 0, 0, false)    \
    X(8, "lookback_nt_px8_rw16_nw4", 8, 16, 4, MODE_LOOKBACK, 1, 1, true)          \
    X(9, "lookback_nt_px4_rw16_nw4", 4, 16, 4, MODE_LOOKBACK, 1, 1, true)          \
    X(10, "helper_nt_px4_rw16_nw4", 4, 16, 4, MODE_HELPER, 1, 1, true)             \
    X(11, "helper_nt_px8_rw12_nw4", 8, 12, 4, MODE_HELPER, 1, 1, true)            \
    X(12, "helper3_nt_px4_rw16_nw4", 4, 16, 4, MODE_HELPER3, 1, 1, true)           \
    X(13, "helper3_nt_px8_rw12_nw4", 8, 12, 4, MODE_HELPER3, 1, 1, true)

const BuildVariant kVariants[] = {
#define SAT_X(i, name, px, rw, nw, mode, win, adapt, nt) {name, px, rw, nw, mode, win},
    SAT_BUILD_VARIANTS(SAT_X)
#undef SAT_X
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);
const int kAdaptive[] = {
#define SAT_X(i, name, px, rw, nw, mode, win, adapt, nt) adapt,
    SAT_BUILD_VARIANTS(SAT_X)
#undef SAT_X
};

int resident_capacity(const void *kernel, int threads) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

// Static LDS of a variant for one pixel type; a variant whose workgroup state exceeds the 160 KiB
// of a compute unit is not instantiated for that pixel type (capacity 0, launch refused).
constexpr size_t kLdsBytes = 160 * 1024;
template <typename T, bool SQ, int PX, int RW, int NW, int MODE, int WIN, bool NT>
constexpr bool lds_fits() {
    if constexpr (MODE == MODE_HELPER || MODE == MODE_HELPER3)
        return sizeof(typename Build2<T, SQ, PX, RW, NW, WIN, NT, MODE == MODE_HELPER3>::Smem) <= kLdsBytes;
    else return sizeof(typename Build<T, SQ, PX, RW, NW, MODE, NT>::Smem) <= kLdsBytes;
}

template <typename T, bool SQ, int PX, int RW, int NW, int MODE, int WIN, bool NT>
int capacity_typed() {
    if constexpr (!lds_fits<T, SQ, PX, RW, NW, MODE, WIN, NT>()) {
        return 0;
    } else {
        static int cap = 0;   // per instantiation; the library drives one device model
        if (cap == 0) {
            if constexpr (MODE == MODE_HELPER || MODE == MODE_HELPER3)
                cap = resident_capacity(
                    reinterpret_cast<const void *>(&build2_kernel<T, SQ, PX, RW, NW, WIN, NT, MODE == MODE_HELPER3>),
                    (NW + 1) * 64);
            else
                cap = resident_capacity(reinterpret_cast<const void *>(&build_kernel<T, SQ, PX, RW, NW, MODE, NT>),
                                        NW * 64);
        }
        return cap;
    }
}

template <typename T, bool SQ, int PX, int RW, int NW, int MODE, int WIN, bool NT>
hipError_t launch_typed(const BuildDesc *descs, int n, const BuildDesc *dev_descs, int64_t total_items,
                        void *workspace, int64_t state_words, hipStream_t stream) {
    if constexpr (!lds_fits<T, SQ, PX, RW, NW, MODE, WIN, NT>()) {
        return hipErrorInvalidConfiguration;
    } else {
        BuildCtrl *ctrl = static_cast<BuildCtrl *>(workspace);
        uint64_t *state = reinterpret_cast<uint64_t *>(static_cast<char *>(workspace) + sizeof(BuildCtrl));
        BuildDesc *slot = n == 1 ? &ctrl->one : nullptr;
        const BuildDesc *table = n == 1 ? slot : dev_descs;
        constexpr int TH = RW * NW;
        constexpr bool kPrepass = MODE == MODE_REDUCE_SCAN || ((MODE == MODE_HELPER || MODE == MODE_HELPER3) && WIN == 0);
        if (!kPrepass) {
            // 32-bit state words fill the first half of the state (the offsets count words)
            const long long words = descs[0].narrow ? (state_words + 1) / 2 : state_words;
            const long long pairs = (words + 1) / 2;
            const long long blocks = pairs > 0 ? (pairs + 255) / 256 : 1;
            const unsigned grid = static_cast<unsigned>(blocks < 8192 ? blocks : 8192);
            hipLaunchKernelGGL(clear_kernel, dim3(grid), dim3(256), 0, stream, state, words, ctrl, descs[0], slot);
        } else {
            hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(256), 0, stream, state, 0ll, ctrl, descs[0], slot);
            for (int i = 0; i < n; ++i) {
                const BuildDesc &d = descs[i];
                const int64_t xb = (d.Wp / PX + 255) / 256;
                hipLaunchKernelGGL((colsum_kernel<T, SQ, PX, TH>), dim3(static_cast<unsigned>(xb), d.nstrips),
                                   dim3(256), 0, stream, d, state);
                const unsigned cb = static_cast<unsigned>((d.Wp + 255) / 256);
                hipLaunchKernelGGL(colscan_kernel, dim3(cb), dim3(256), 0, stream, state,
                                   static_cast<long long>(d.state_off), static_cast<long long>(d.Wp), d.nstrips,
                                   d.carry, d.total, static_cast<long long>(d.W));
                if (SQ)
                    hipLaunchKernelGGL(colscan_kernel, dim3(cb), dim3(256), 0, stream, state,
                                       static_cast<long long>(d.state_q_off), static_cast<long long>(d.Wp),
                                       d.nstrips, d.carry_q, d.total_q, static_cast<long long>(d.W));
            }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int cap = capacity_typed<T, SQ, PX, RW, NW, MODE, WIN, NT>();
        const int64_t grid = total_items < cap ? total_items : cap;
        if constexpr (MODE == MODE_HELPER || MODE == MODE_HELPER3)
            hipLaunchKernelGGL((build2_kernel<T, SQ, PX, RW, NW, WIN, NT, MODE == MODE_HELPER3>), dim3(static_cast<unsigned>(grid)),
                               dim3((NW + 1) * 64), 0, stream, table, n, static_cast<long long>(total_items), state, ctrl);
        else
            hipLaunchKernelGGL((build_kernel<T, SQ, PX, RW, NW, MODE, NT>), dim3(static_cast<unsigned>(grid)),
                               dim3(NW * 64), 0, stream, table, n, static_cast<long long>(total_items), state, ctrl);
        return hipGetLastError();
    }
}

template <typename T, bool SQ>
hipError_t launch_variant(int v, const BuildDesc *descs, int n, const BuildDesc *dev_descs, int64_t total,
                          void *ws, int64_t words, hipStream_t s) {
    switch (v) {
#define SAT_X(i, name, px, rw, nw, mode, win, adapt, nt) \
        case i: return launch_typed<T, SQ, px, rw, nw, mode, win, nt>(descs, n, dev_descs, total, ws, words, s);
        SAT_BUILD_VARIANTS(SAT_X)
#undef SAT_X
        default: return hipErrorInvalidValue;
    }
}

template <typename T, bool SQ>
int capacity_variant(int v) {
    switch (v) {
#define SAT_X(i, name, px, rw, nw, mode, win, adapt, nt) \
        case i: return capacity_typed<T, SQ, px, rw, nw, mode, win, nt>();
        SAT_BUILD_VARIANTS(SAT_X)
#undef SAT_X
        default: return 1;
    }
}

// Power builds: 4 pixels per lane (256-column blocks), 16 rows per wave, 4 compute waves and the
// helper, non-temporal table stores.  With four 8-bit tables the workgroup state is 112 KiB of
// LDS, one workgroup per CU: 17 % faster at 32768^2 than 2 pixels per lane with two workgroups
// per CU, and 32-row strips were slower still.
template <typename T, int NP>
const void *pow_kernel() {
    return reinterpret_cast<const void *>(&build_pow_kernel<T, NP, 4, 16, 4, true>);
}
static_assert(64 * 4 == kPowBlockW && 16 * 4 == kPowStripH, "power build geometry");

template <typename T, int NP>
int pow_capacity_typed() {
    static int cap = 0;
    if (cap == 0) cap = resident_capacity(pow_kernel<T, NP>(), 5 * 64);
    return cap;
}

template <typename T, int NP>
hipError_t launch_pow_typed(const BuildDesc &d, void *workspace, int64_t state_words, hipStream_t stream) {
    BuildCtrl *ctrl = static_cast<BuildCtrl *>(workspace);
    uint64_t *state = reinterpret_cast<uint64_t *>(static_cast<char *>(workspace) + sizeof(BuildCtrl));
    const long long pairs = (state_words + 1) / 2;
    const long long blocks = pairs > 0 ? (pairs + 255) / 256 : 1;
    const unsigned cgrid = static_cast<unsigned>(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(clear_kernel, dim3(cgrid), dim3(256), 0, stream, state, static_cast<long long>(state_words), ctrl,
                       d, static_cast<BuildDesc *>(nullptr));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int cap = pow_capacity_typed<T, NP>();
    const int64_t grid = d.nstrips < cap ? d.nstrips : cap;
    hipLaunchKernelGGL((build_pow_kernel<T, NP, 4, 16, 4, true>), dim3(static_cast<unsigned>(grid)), dim3(5 * 64), 0,
                       stream, d, static_cast<long long>(d.nstrips), state, ctrl);
    return hipGetLastError();
}

template <typename T, bool SQ>
hipError_t launch_seg_typed(const BuildDesc &d, uint64_t *sums, uint64_t *sums_q, hipStream_t stream) {
    const long long segw = static_cast<long long>(d.seg_blocks) * (d.Wp / d.nblocks);
    hipLaunchKernelGGL((segsum_kernel<T, SQ>), dim3(static_cast<unsigned>((d.H + 3) / 4), d.nseg - 1), dim3(256), 0,
                       stream, d, segw, sums, sums_q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((segscan_kernel<SQ>), dim3(d.nseg - 1), dim3(1024), 0, stream, d, segw, sums, sums_q,
                       const_cast<uint64_t *>(d.seg_pre), const_cast<uint64_t *>(d.seg_pre_q));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_seg_prepass(int bpp, bool sq, const BuildDesc &d, uint64_t *sums, uint64_t *sums_q,
                              hipStream_t stream) {
    if (d.nseg < 2) return hipSuccess;
    if (bpp == 1) return sq ? launch_seg_typed<uint8_t, true>(d, sums, sums_q, stream)
                            : launch_seg_typed<uint8_t, false>(d, sums, sums_q, stream);
    return sq ? launch_seg_typed<uint16_t, true>(d, sums, sums_q, stream)
              : launch_seg_typed<uint16_t, false>(d, sums, sums_q, stream);
}

int power_build_capacity(int bpp, int np) {
    if (bpp == 1) {
        switch (np) {
            case 1: return pow_capacity_typed<uint8_t, 1>();
            case 2: return pow_capacity_typed<uint8_t, 2>();
            case 3: return pow_capacity_typed<uint8_t, 3>();
            case 4: return pow_capacity_typed<uint8_t, 4>();
        }
    } else {
        switch (np) {
            case 1: return pow_capacity_typed<uint16_t, 1>();
            case 2: return pow_capacity_typed<uint16_t, 2>();
            case 3: return pow_capacity_typed<uint16_t, 3>();
        }
    }
    return 0;
}

hipError_t launch_build_powers(int bpp, int np, const BuildDesc &d, void *workspace, int64_t state_words,
                               hipStream_t stream) {
    if (bpp == 1) {
        switch (np) {
            case 1: return launch_pow_typed<uint8_t, 1>(d, workspace, state_words, stream);
            case 2: return launch_pow_typed<uint8_t, 2>(d, workspace, state_words, stream);
            case 3: return launch_pow_typed<uint8_t, 3>(d, workspace, state_words, stream);
            case 4: return launch_pow_typed<uint8_t, 4>(d, workspace, state_words, stream);
        }
    } else {
        switch (np) {
            case 1: return launch_pow_typed<uint16_t, 1>(d, workspace, state_words, stream);
            case 2: return launch_pow_typed<uint16_t, 2>(d, workspace, state_words, stream);
            case 3: return launch_pow_typed<uint16_t, 3>(d, workspace, state_words, stream);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_column_totals(int bpp, const void *img, int64_t H, int64_t W, int64_t pitch, int vec16,
                                const uint64_t *carry, const uint64_t *carry_q, uint64_t *out, uint64_t *out_q,
                                hipStream_t stream) {
    if (bpp == 1)
        return out_q ? launch_totals_typed<uint8_t, true>(img, H, W, pitch, vec16, carry, carry_q, out, out_q, stream)
                     : launch_totals_typed<uint8_t, false>(img, H, W, pitch, vec16, carry, carry_q, out, out_q, stream);
    return out_q ? launch_totals_typed<uint16_t, true>(img, H, W, pitch, vec16, carry, carry_q, out, out_q, stream)
                 : launch_totals_typed<uint16_t, false>(img, H, W, pitch, vec16, carry, carry_q, out, out_q, stream);
}

}  // namespace satk

// Workspace of sat_build_noalloc: lookback words and the control header of one build at a time per
// device.  Host code never passes this name to a kernel or a copy (on the host it stands for the
// symbol, not for device memory): it takes the device address from hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[satk::kNoAllocScratchBytes];

namespace satk {

hipError_t noalloc_scratch(hipStream_t stream, void **ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int cur = 0, dev = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    dev = cur;
    if (stream) {
        hipDevice_t sd;
        if ((e = hipStreamGetDevice(stream, &sd)) != hipSuccess) return e;
        dev = static_cast<int>(sd);
    }
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // the symbol's address on `dev`: looked up with that device current
        if (dev != cur && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (dev != cur) {
            const hipError_t r = hipSetDevice(cur);
            if (e == hipSuccess) e = r;
        }
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t upload_words(const void *src, size_t bytes, void *dst, hipStream_t stream) {
    if (bytes % 8 || reinterpret_cast<uintptr_t>(dst) % 8) return hipErrorInvalidValue;
    const uint64_t *w = static_cast<const uint64_t *>(src);
    uint64_t *d = static_cast<uint64_t *>(dst);
    const size_t n = bytes / 8;
    for (size_t i = 0; i < n; i += kChunkWords) {
        WordChunk c{};
        const int k = static_cast<int>(n - i < static_cast<size_t>(kChunkWords) ? n - i : kChunkWords);
        for (int j = 0; j < k; ++j) c.w[j] = w[i + j];
        hipLaunchKernelGGL(words_write_kernel, dim3(1), dim3(512), 0, stream, c, d + i, k);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

int build_variant_count() { return kNumVariants; }
const BuildVariant &build_variant(int v) { return kVariants[v]; }
int build_variant_adaptive(int v) { return (v >= 0 && v < kNumVariants) ? kAdaptive[v] : 0; }

int build_variant_capacity(int v, int bpp, bool sq) {
    if (bpp == 1) return sq ? capacity_variant<uint8_t, true>(v) : capacity_variant<uint8_t, false>(v);
    return sq ? capacity_variant<uint16_t, true>(v) : capacity_variant<uint16_t, false>(v);
}

bool fused_build_variant(int variant) { return variant == 9 || variant == 1 || variant == 2; }

namespace {

template <typename T, int PX, int RW, int NW, bool NTS>
hipError_t launch_fused_typed(int v, const BuildDesc *bdescs, const BuildDesc *dev_bdescs, int n, int64_t build_items,
                              const GatherDesc *dev_gdescs, int64_t gather_items, void *workspace, int64_t state_words,
                              unsigned int *ready, hipStream_t stream) {
    BuildCtrl *ctrl = static_cast<BuildCtrl *>(workspace);
    uint64_t *state = reinterpret_cast<uint64_t *>(static_cast<char *>(workspace) + sizeof(BuildCtrl));
    const long long pairs = (state_words + 1) / 2;
    const long long blocks = pairs > 0 ? (pairs + 255) / 256 : 1;
    const unsigned cgrid = static_cast<unsigned>(blocks < 8192 ? blocks : 8192);
    hipLaunchKernelGGL(clear_kernel, dim3(cgrid), dim3(256), 0, stream, state, static_cast<long long>(state_words),
                       ctrl, bdescs[0], static_cast<BuildDesc *>(nullptr));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const void *k1 = reinterpret_cast<const void *>(&fused_kernel<T, PX, RW, NW, NTS, 1>);
    const void *k2 = reinterpret_cast<const void *>(&fused_kernel<T, PX, RW, NW, NTS, 2>);
    const void *k4 = reinterpret_cast<const void *>(&fused_kernel<T, PX, RW, NW, NTS, 4>);
    const void *k = v == 1 ? k1 : v == 4 ? k4 : k2;
    static int cap[3] = {0, 0, 0};
    const int ci = v == 1 ? 0 : v == 4 ? 2 : 1;
    if (cap[ci] == 0) cap[ci] = resident_capacity(k, NW * 64);
    const long long total = static_cast<long long>(build_items + gather_items);
    const unsigned grid = static_cast<unsigned>(total < cap[ci] ? total : cap[ci]);
    if (v == 1)
        hipLaunchKernelGGL((fused_kernel<T, PX, RW, NW, NTS, 1>), dim3(grid), dim3(NW * 64), 0, stream, dev_bdescs,
                           dev_gdescs, n, static_cast<long long>(build_items), total, state, ctrl, ready);
    else if (v == 4)
        hipLaunchKernelGGL((fused_kernel<T, PX, RW, NW, NTS, 4>), dim3(grid), dim3(NW * 64), 0, stream, dev_bdescs,
                           dev_gdescs, n, static_cast<long long>(build_items), total, state, ctrl, ready);
    else
        hipLaunchKernelGGL((fused_kernel<T, PX, RW, NW, NTS, 2>), dim3(grid), dim3(NW * 64), 0, stream, dev_bdescs,
                           dev_gdescs, n, static_cast<long long>(build_items), total, state, ctrl, ready);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fused_t(int variant, int v, const BuildDesc *bdescs, const BuildDesc *dev_bdescs, int n,
                          int64_t build_items, const GatherDesc *dev_gdescs, int64_t gather_items, void *workspace,
                          int64_t state_words, unsigned int *ready, hipStream_t stream) {
    switch (variant) {
        case 9: return launch_fused_typed<T, 4, 16, 4, true>(v, bdescs, dev_bdescs, n, build_items, dev_gdescs,
                                                             gather_items, workspace, state_words, ready, stream);
        case 1: return launch_fused_typed<T, 4, 16, 4, false>(v, bdescs, dev_bdescs, n, build_items, dev_gdescs,
                                                              gather_items, workspace, state_words, ready, stream);
        case 2: return launch_fused_typed<T, 4, 8, 4, false>(v, bdescs, dev_bdescs, n, build_items, dev_gdescs,
                                                             gather_items, workspace, state_words, ready, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fused(int variant, int bpp, int v, const BuildDesc *bdescs, int n, const BuildDesc *dev_bdescs,
                        int64_t build_items, const GatherDesc *dev_gdescs, int64_t gather_items, void *workspace,
                        int64_t state_words, unsigned int *ready, hipStream_t stream) {
    if (bpp == 1)
        return launch_fused_t<uint8_t>(variant, v, bdescs, dev_bdescs, n, build_items, dev_gdescs, gather_items,
                                       workspace, state_words, ready, stream);
    return launch_fused_t<uint16_t>(variant, v, bdescs, dev_bdescs, n, build_items, dev_gdescs, gather_items,
                                    workspace, state_words, ready, stream);
}

hipError_t launch_build(int variant, int bpp, bool sq, const BuildDesc *descs, int n,
                        const BuildDesc *dev_descs, int64_t total_items, void *workspace,
                        int64_t state_words, hipStream_t stream) {
    if (bpp == 1)
        return sq ? launch_variant<uint8_t, true>(variant, descs, n, dev_descs, total_items, workspace, state_words, stream)
                  : launch_variant<uint8_t, false>(variant, descs, n, dev_descs, total_items, workspace, state_words, stream);
    return sq ? launch_variant<uint16_t, true>(variant, descs, n, dev_descs, total_items, workspace, state_words, stream)
              : launch_variant<uint16_t, false>(variant, descs, n, dev_descs, total_items, workspace, state_words, stream);
}

}  // namespace satk
