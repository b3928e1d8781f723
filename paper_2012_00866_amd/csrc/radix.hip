// Step 2 of Huskysort on the GPU: a stable LSD radix sort of (u64 key, u32
// value) pairs inside independent segments.
//
// The paper sorts the codes with introsort while swapping the objects
// alongside (Sec. 3.1 Step 2).  On a GPU the same role is filled by a
// least-significant-digit radix sort that carries the 32-bit index with every
// 64-bit code: integer comparisons only, and stable, so equal codes keep index
// order and the permutation is unique.
//
// Layout of one sort:
//  * segments: contiguous position ranges sorted independently (one for a
//    single sort, one per instance for the batched form, one per long run of
//    equal codes for the device-wide fix-up);
//  * the multi-tile passes take their digits over the bits that vary, packed,
//    when that needs fewer passes than fixed-width digits: a key bit that has
//    the same value in every key of a segment cannot change the segment's
//    order, so the varying bits, kept in order and packed from the least
//    significant up, are sorted instead of the whole key (digits vary in 4 of
//    every 7 bits, lowercase letters in 5, when no string stops inside the
//    coded prefix);
//  * a segment of at most one tile (256 threads x ITEMS keys) is sorted
//    entirely in LDS by one workgroup (k_tile_sort), digit passes whose digit
//    is the same in every key of the segment skipped (packing pays less
//    there than the extra work of building digits from several runs);
//  * longer ("big") segments: one reduction finds the bits that vary inside
//    each segment (OR and AND of its keys); the digit programs pack the bits
//    that vary in any big segment, and a pass that takes no bit varying
//    inside a segment is skipped for it.  Every remaining pass is
//    reduce-then-scan with no dependency chain between tiles:
//      k_count      digit counts of every tile (a segment's first pass
//                   reads the keys, every later pass one byte per key),
//      k_group_scan exclusive scan of the counts over groups of 64 tiles,
//      k_seg_scan   scan over a segment's groups, and the digit starts,
//      k_scatter    every tile ranks its keys with wavefront ballots, adds
//                   its offsets and scatters through LDS so that
//                   neighbouring lanes write neighbouring addresses; beside
//                   each key it writes the key's digit of the next pass,
//                   which is that pass's count input.
//    A decoupled look-back (one kernel per pass) would save the count pass's
//    read, but its chain of per-tile flags and its per-tile ticket atomic
//    cost more than that read on this GPU.
//  * each big segment's skipped passes are tracked with a bit mask; the
//    ping-pong buffer holding its data after pass p is the parity of the
//    passes it ran before p, and a final copy returns odd-parity segments to
//    the primary buffers.

#include <hip/hip_ext.h>

#include <algorithm>

#include "common.h"
#include "internal.h"
#include "rank.h"

namespace husky {

// ------------------------------------------------------------------ setup
struct SrcOffsets {
    const uint64_t* off;
    uint32_t n;
    __device__ uint32_t count() const { return n; }
    __device__ void get(uint32_t i, uint32_t& s, uint32_t& l) const {
        s = (uint32_t)off[i];
        l = (uint32_t)(off[i + 1] - off[i]);
    }
};
struct SrcSingle {
    uint32_t n;
    __device__ uint32_t count() const { return 1; }
    __device__ void get(uint32_t, uint32_t& s, uint32_t& l) const {
        s = 0;
        l = n;
    }
};
struct SrcItems {
    const RunItem* items;
    const uint32_t* cnt;
    uint32_t cap;
    __device__ uint32_t count() const {
        uint32_t c = *cnt;
        return c < cap ? c : cap;
    }
    __device__ void get(uint32_t i, uint32_t& s, uint32_t& l) const {
        s = items[i].start;
        l = items[i].len;
    }
};

// One workgroup: segment descriptors, the two tile spaces, the big list and
// its scan groups.  Each thread takes SEG_K consecutive segments per round, so
// a round of four block scans covers BLOCK * SEG_K segments.
constexpr uint32_t SEG_K = 8;
// z0[0..nz0) and z1[0..nz1) are cleared on the way (a sort's status and
// Step 3's counters, without a launch of their own).
template <typename Src>
__global__ __launch_bounds__(BLOCK) void k_seg_setup(Src src, SegDesc* segs, BigDesc* bigs,
                                                     uint32_t* counters, uint32_t tile,
                                                     uint32_t* __restrict__ z0, uint32_t nz0,
                                                     uint32_t* __restrict__ z1, uint32_t nz1) {
    __shared__ uint32_t scratch[NWAVES];
    for (uint32_t i = threadIdx.x; i < nz0; i += BLOCK) z0[i] = 0;
    for (uint32_t i = threadIdx.x; i < nz1; i += BLOCK) z1[i] = 0;
    const uint32_t S = src.count();
    uint32_t carry_all = 0, carry_big = 0, carry_nbig = 0, carry_grp = 0;
    for (uint32_t base = 0; base < S; base += BLOCK * SEG_K) {
        const uint32_t i0 = base + threadIdx.x * SEG_K;
        uint32_t st[SEG_K], ln[SEG_K];
        uint32_t s_all = 0, s_big = 0, s_nbig = 0, s_grp = 0;
#pragma unroll
        for (uint32_t j = 0; j < SEG_K; ++j) {
            st[j] = ln[j] = 0;
            if (i0 + j < S) src.get(i0 + j, st[j], ln[j]);
            const uint32_t nt = (ln[j] + tile - 1) / tile;
            const bool big = ln[j] > tile;
            s_all += nt;
            s_big += big ? nt : 0u;
            s_nbig += big ? 1u : 0u;
            s_grp += big ? (nt + GROUP_TILES - 1) / GROUP_TILES : 0u;
        }
        uint32_t tot_all, tot_big, tot_nbig, tot_grp;
        uint32_t ex_all = block_exclusive_sum(s_all, scratch, &tot_all);
        uint32_t ex_big = block_exclusive_sum(s_big, scratch, &tot_big);
        uint32_t ex_nbig = block_exclusive_sum(s_nbig, scratch, &tot_nbig);
        uint32_t ex_grp = block_exclusive_sum(s_grp, scratch, &tot_grp);
#pragma unroll
        for (uint32_t j = 0; j < SEG_K; ++j) {
            const uint32_t i = i0 + j;
            const uint32_t nt = (ln[j] + tile - 1) / tile;
            const bool big = ln[j] > tile;
            const uint32_t ng = big ? (nt + GROUP_TILES - 1) / GROUP_TILES : 0u;
            if (i < S) {
                SegDesc d;
                d.start = st[j];
                d.len = ln[j];
                d.first_tile = carry_all + ex_all;
                d.aux = big ? carry_nbig + ex_nbig : NOT_BIG;
                segs[i] = d;
                if (big) {
                    BigDesc b;
                    b.start = st[j];
                    b.len = ln[j];
                    b.first_tile = carry_big + ex_big;
                    b.exec = 0;  // written once the varying bits are known
                    b.first_group = carry_grp + ex_grp;
                    b.ntiles = nt;
                    b.ngroups = ng;
                    b.pad = 0;
                    bigs[carry_nbig + ex_nbig] = b;
                }
            }
            ex_all += nt;
            ex_big += big ? nt : 0u;
            ex_nbig += big ? 1u : 0u;
            ex_grp += ng;
        }
        carry_all += tot_all;
        carry_big += tot_big;
        carry_nbig += tot_nbig;
        carry_grp += tot_grp;
    }
    if (threadIdx.x == 0) {
        counters[C_ALL_TILES] = carry_all;
        counters[C_BIG_TILES] = carry_big;
        counters[C_NUM_BIG] = carry_nbig;
        counters[C_NUM_SEGS] = S;
        counters[C_NUM_GROUPS] = carry_grp;
        counters[C_EXEC_UNION] = 0;
        counters[C_VARY_LO] = 0;
        counters[C_VARY_HI] = 0;
        counters[C_EXEC_DONE] = 0;
        counters[C_PERFECT_OFF] = 0;
    }
}

hipError_t radix_segments_from_offsets(const uint64_t* seg_offsets, uint32_t n_segs,
                                       const RadixScratch& sc, const RadixConfig& cfg,
                                       hipStream_t s, uint32_t* z0, uint32_t nz0, uint32_t* z1,
                                       uint32_t nz1) {
    SrcOffsets src{seg_offsets, n_segs};
    ProfScope ps(P_SETUP, s);
    hipLaunchKernelGGL(k_seg_setup<SrcOffsets>, dim3(1), dim3(BLOCK), 0, s, src, sc.segs,
                       sc.bigs, sc.counters, (uint32_t)cfg.tile(), z0, nz0, z1, nz1);
    return hipGetLastError();
}
hipError_t radix_segments_single(uint32_t n, const RadixScratch& sc, const RadixConfig& cfg,
                                 hipStream_t s, uint32_t* z0, uint32_t nz0, uint32_t* z1,
                                 uint32_t nz1) {
    SrcSingle src{n};
    ProfScope ps(P_SETUP, s);
    hipLaunchKernelGGL(k_seg_setup<SrcSingle>, dim3(1), dim3(BLOCK), 0, s, src, sc.segs,
                       sc.bigs, sc.counters, (uint32_t)cfg.tile(), z0, nz0, z1, nz1);
    return hipGetLastError();
}
hipError_t radix_segments_from_items(const RunItem* items, const uint32_t* count,
                                     uint32_t max_items, const RadixScratch& sc,
                                     const RadixConfig& cfg, hipStream_t s) {
    SrcItems src{items, count, max_items};
    ProfScope ps(P_SETUP, s);
    hipLaunchKernelGGL(k_seg_setup<SrcItems>, dim3(1), dim3(BLOCK), 0, s, src, sc.segs,
                       sc.bigs, sc.counters, (uint32_t)cfg.tile(), (uint32_t*)nullptr, 0u,
                       (uint32_t*)nullptr, 0u);
    return hipGetLastError();
}

// ------------------------------------------------------------------ big-segment passes
// OR / AND over the workgroup; the result is valid in thread 0.
__device__ __forceinline__ void block_or_and(uint64_t& o, uint64_t& a, uint64_t* s_o, uint64_t* s_a) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        o |= (uint64_t)__shfl_xor((unsigned long long)o, d, WAVE);
        a &= (uint64_t)__shfl_xor((unsigned long long)a, d, WAVE);
    }
    const uint32_t w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        s_o[w] = o;
        s_a[w] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NWAVES; ++i) {
            o |= s_o[i];
            a &= s_a[i];
        }
    }
}

template <typename F>
__device__ __forceinline__ uint32_t find_big(const BigDesc* bigs, uint32_t nb, uint32_t x, F key) {
    uint32_t lo = 0, hi = nb;  // largest b with key(bigs[b]) <= x
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (key(bigs[mid]) <= x)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}
__device__ __forceinline__ uint32_t big_of_tile(const BigDesc* bigs, uint32_t nb, uint32_t t) {
    return find_big(bigs, nb, t, [](const BigDesc& b) { return b.first_tile; });
}
__device__ __forceinline__ uint32_t big_of_group(const BigDesc* bigs, uint32_t nb, uint32_t g) {
    return find_big(bigs, nb, g, [](const BigDesc& b) { return b.first_group; });
}

// OR and AND of the keys of every big tile (bits that vary = OR ^ AND).
template <int ITEMS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_orand(const uint64_t* __restrict__ keys,
                                                 const BigDesc* __restrict__ bigs,
                                                 const uint32_t* __restrict__ counters,
                                                 uint64_t* __restrict__ korand) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_o[NWAVES], s_a[NWAVES];
    HUSKY_UNITS_P(PS, t, counters[C_BIG_TILES]) {
        const BigDesc B = bigs[big_of_tile(bigs, counters[C_NUM_BIG], t)];
        const uint32_t lt = t - B.first_tile;
        const uint32_t base = B.start + lt * TILE;
        const uint32_t nvalid = min(TILE, B.len - lt * TILE);
        uint64_t o = 0, a = ~0ull;
        for (uint32_t i = threadIdx.x; i < nvalid; i += BLOCK) {
            const uint64_t k = keys[base + i];
            o |= k;
            a &= k;
        }
        block_or_and(o, a, s_o, s_a);
        if (threadIdx.x == 0) {
            korand[2 * (size_t)t] = o;
            korand[2 * (size_t)t + 1] = a;
        }
        if (PS) __syncthreads();
    }
}

// The digit programs over the union of the varying bits, and every big
// segment's mask of passes (run by one workgroup, the last of k_exec):
// packed bit c is key bit number c among the union's bits, pass c / BITS,
// digit bit c % BITS -- or, when packing saves no pass, BITS-wide windows from
// begin_bit that hold a varying bit.  A segment runs the passes that take a
// bit varying inside it.  Packing keeps the order of the bits, and a bit
// outside the union is constant inside every segment, so the passes sort
// each segment by its keys.
// With perfect_lsb (keys are ASCII codes with the perfect bit in bit 0), bit 0
// is left out of every digit when that saves a pass, and C_PERFECT_OFF tells
// run detection to compare keys without it (the order of the remaining bits
// is the order of the codes, so runs of equal codes are still contiguous).
template <int BITS>
__device__ __forceinline__ int passes_for(uint64_t u, int begin_bit, int end_bit) {
    int nw = 0;
    for (int sh = begin_bit; sh < end_bit; sh += BITS) nw += ((u >> sh) & ((1ull << BITS) - 1ull)) ? 1 : 0;
    const int np = (__popcll(u) + BITS - 1) / BITS;
    return np < nw ? np : nw;
}

template <int BITS>
__device__ void build_programs(BigDesc* __restrict__ bigs, uint32_t* __restrict__ counters,
                               const uint64_t* __restrict__ segvary, uint32_t* __restrict__ prog,
                               int begin_bit, int end_bit, uint32_t nb, uint32_t* s_prog,
                               uint64_t* s_pm, uint32_t* s_or, bool perfect_lsb) {
    for (int i = threadIdx.x; i < MAX_PASSES * PROG_WORDS; i += BLOCK) s_prog[i] = 0;
    for (int p = threadIdx.x; p < MAX_PASSES; p += BLOCK) s_pm[p] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t u = (uint64_t)__hip_atomic_load(&counters[C_VARY_LO], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) |
                     ((uint64_t)__hip_atomic_load(&counters[C_VARY_HI], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) << 32);
        const uint64_t range = (end_bit >= 64 ? ~0ull : (1ull << end_bit) - 1ull);
        const bool drop = perfect_lsb && begin_bit == 0 && (u & 1ull) &&
                          passes_for<BITS>(u & ~1ull, begin_bit, end_bit) < passes_for<BITS>(u, begin_bit, end_bit);
        if (drop) u &= ~1ull;
        counters[C_PERFECT_OFF] = drop ? 1u : 0u;
        int nw = 0;
        for (int sh = begin_bit; sh < end_bit; sh += BITS) nw += ((u >> sh) & ((1ull << BITS) - 1ull)) ? 1 : 0;
        const bool packed = (__popcll(u) + BITS - 1) / BITS < nw;
        int c = 0, prev = -2;
        for (int sh = begin_bit; sh < end_bit && !packed; sh += BITS) {
            const uint64_t wm = (((1ull << BITS) - 1ull) << sh) & range;
            if (!(u & wm)) continue;
            const int len = end_bit - sh < BITS ? end_bit - sh : BITS;
            s_prog[c * PROG_WORDS] = 1;
            s_prog[c * PROG_WORDS + 1] = (uint32_t)sh | ((uint32_t)len << 8);
            s_pm[c] = wm;
            ++c;
        }
        for (int b = 0; b < 64 && packed; ++b) {
            if (!((u >> b) & 1ull)) continue;
            const int p = c / BITS, db = c % BITS;
            uint32_t* pp = s_prog + p * PROG_WORDS;
            if (db > 0 && prev == b - 1) {
                pp[pp[0]] += 1u << 8;  // one more bit in the pass's last run
            } else {
                pp[0] += 1u;
                pp[pp[0]] = (uint32_t)b | (1u << 8) | ((uint32_t)db << 16);
            }
            s_pm[p] |= 1ull << b;
            prev = b;
            ++c;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < MAX_PASSES * PROG_WORDS; i += BLOCK) prog[i] = s_prog[i];
    uint32_t all = 0;
    for (uint32_t b = threadIdx.x; b < nb; b += BLOCK) {
        const uint64_t v = load_agent(&segvary[b]);  // written by other workgroups
        uint32_t m = 0;
#pragma unroll
        for (int p = 0; p < MAX_PASSES; ++p) m |= (v & s_pm[p]) ? 1u << p : 0u;
        bigs[b].exec = m;
        all |= m;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) all |= __shfl_xor(all, d, WAVE);
    if (lane_id() == 0) s_or[threadIdx.x / WAVE] = all;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t u = 0;
        for (int w = 0; w < NWAVES; ++w) u |= s_or[w];
        counters[C_EXEC_UNION] = u;
    }
}

// The workgroup that finished the last big segment: the digit programs.
template <int BITS>
__device__ void exec_last(BigDesc* __restrict__ bigs, uint32_t* __restrict__ counters,
                          uint64_t* __restrict__ segvary, uint32_t* __restrict__ prog, int begin_bit,
                          int end_bit, uint32_t nb, uint32_t* s_prog, uint64_t* s_pm, uint32_t* s_or,
                          bool perfect_lsb) {
    __threadfence();
    build_programs<BITS>(bigs, counters, segvary, prog, begin_bit, end_bit, nb, s_prog, s_pm, s_or,
                         perfect_lsb);
}

// Bits that vary inside every big segment (within [begin_bit, end_bit)) and
// their union; the workgroup that finishes last builds the digit programs.
template <int BITS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_exec(BigDesc* __restrict__ bigs,
                                                uint32_t* __restrict__ counters,
                                                const uint64_t* __restrict__ korand,
                                                uint64_t* __restrict__ segvary,
                                                uint32_t* __restrict__ prog, int begin_bit,
                                                int end_bit, bool perfect_lsb) {
    __shared__ uint64_t s_o[NWAVES], s_a[NWAVES];
    __shared__ uint32_t s_prog[MAX_PASSES * PROG_WORDS];
    __shared__ uint64_t s_pm[MAX_PASSES];
    __shared__ uint32_t s_or[NWAVES];
    __shared__ uint32_t s_last;
    const uint32_t nb = counters[C_NUM_BIG];
    HUSKY_UNITS_P(PS, b, nb) {
        const BigDesc B = bigs[b];
        uint64_t o = 0, a = ~0ull;
        // four tiles' words in flight per thread
        for (uint32_t t0 = threadIdx.x; t0 < B.ntiles; t0 += 4 * BLOCK) {
            uint64_t vo[4], va[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t t = t0 + u * BLOCK;
                vo[u] = t < B.ntiles ? korand[2 * (size_t)(B.first_tile + t)] : 0ull;
                va[u] = t < B.ntiles ? korand[2 * (size_t)(B.first_tile + t) + 1] : ~0ull;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                o |= vo[u];
                a &= va[u];
            }
        }
        block_or_and(o, a, s_o, s_a);
        if (threadIdx.x == 0) {
            const uint64_t range = (end_bit >= 64 ? ~0ull : (1ull << end_bit) - 1ull) & ~((1ull << begin_bit) - 1ull);
            const uint64_t vary = (o ^ a) & range;
            store_agent(&segvary[b], vary);
            if ((uint32_t)vary) atomicOr(&counters[C_VARY_LO], (uint32_t)vary);
            if (vary >> 32) atomicOr(&counters[C_VARY_HI], (uint32_t)(vary >> 32));
            __threadfence();
            s_last = atomicAdd(&counters[C_EXEC_DONE], 1u) == nb - 1 ? 1u : 0u;
        }
        __syncthreads();
        const bool last = s_last != 0;
        __syncthreads();
        if (last) exec_last<BITS>(bigs, counters, segvary, prog, begin_bit, end_bit, nb, s_prog, s_pm, s_or,
                                  perfect_lsb);
    }
}

__device__ __forceinline__ bool pass_runs(const BigDesc& B, int pass, bool& flip) {
    if (!((B.exec >> pass) & 1u)) return false;
    flip = __popc(B.exec & ((1u << pass) - 1u)) & 1u;
    return true;
}

// Where a pass finds the digits the previous scatter left (see k_scatter).
enum : int { DIG_NONE = 0, DIG_BYTES = 1, DIG_IN_VALS = 2 };
constexpr uint32_t VAL_MASK = 0x00FFFFFFu;

// Digit counts of one tile -> cnt[tile][digit].  After a segment's first
// pass the digits come from what the previous scatter left: one byte per
// key (DIG_BYTES) or the values' top bytes (DIG_IN_VALS), instead of the
// 8-byte keys.
template <int BITS, int ITEMS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_count(const uint64_t* __restrict__ keysA,
                                                 const uint64_t* __restrict__ keysB,
                                                 const uint32_t* __restrict__ valsA,
                                                 const uint32_t* __restrict__ valsB,
                                                 const BigDesc* __restrict__ bigs,
                                                 const uint32_t* __restrict__ counters,
                                                 uint32_t* __restrict__ cnt, int pass,
                                                 const uint32_t* __restrict__ prog,
                                                 const uint8_t* __restrict__ dig, int dmode, bool low8) {
    static_assert(BITS <= 8, "cnt holds 256 digits per tile");
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint32_t s_h[HIST_WORDS];
    if (!((counters[C_EXEC_UNION] >> pass) & 1u)) return;  // no segment runs this pass
    const uint32_t nbt = counters[C_BIG_TILES];
    HUSKY_UNITS_P(PS, bx, nbt) {
    const uint32_t t = xcd_remap(bx, nbt);
    const BigDesc B = bigs[big_of_tile(bigs, counters[C_NUM_BIG], t)];
    bool flip;
    if (!pass_runs(B, pass, flip)) continue;
    const uint64_t* src = flip ? keysB : keysA;
    DigitProg dp;
    dp.load(prog, pass);
    // a program of one run (the usual case) needs no run loop
    const bool single = dp.nr <= 1;
    const uint32_t s0 = dp.run[0] & 63u, m0 = (1u << ((dp.run[0] >> 8) & 15u)) - 1u;
    const uint32_t lt = t - B.first_tile;
    const uint32_t base = B.start + lt * TILE;
    const uint32_t nvalid = min(TILE, B.len - lt * TILE);
    const bool later_pass = (B.exec & ((1u << pass) - 1u)) != 0;
    // the values' top bytes already hold the keys' low bytes (vals_low8)
    const bool low8_digit = low8 && pass == 0 && dp.nr == 1 && dp.run[0] == (8u << 8);
    if (dmode == DIG_BYTES && later_pass) {
        uint8_t d[ITEMS];
        load_tile<ITEMS>(dig + base, nvalid, d);
        tile_histogram<ITEMS>([&](int i) { return (uint32_t)d[i]; }, nvalid, s_h, cnt + (size_t)t * 256);
    } else if (dmode == DIG_IN_VALS && (later_pass || low8_digit)) {
        uint32_t v[ITEMS];
        load_tile<ITEMS>((flip ? valsB : valsA) + base, nvalid, v);
        tile_histogram<ITEMS>([&](int i) { return v[i] >> 24; }, nvalid, s_h, cnt + (size_t)t * 256);
    } else {
        uint64_t k[ITEMS];
        load_tile<ITEMS>(src + base, nvalid, k);
        tile_histogram<ITEMS>(
            [&](int i) { return single ? (uint32_t)(k[i] >> s0) & m0 : dp.digit(k[i]); }, nvalid, s_h,
            cnt + (size_t)t * 256);
    }
    if (PS) __syncthreads();
    }
}

// Exclusive scan of the tile counts inside each group of GROUP_TILES tiles
// (in place); the group's totals go to gtot[group][digit].
template <int BITS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_group_scan(const BigDesc* __restrict__ bigs,
                                                      const uint32_t* __restrict__ counters,
                                                      uint32_t* __restrict__ cnt,
                                                      uint32_t* __restrict__ gtot, int pass) {
    constexpr int R = 1 << BITS;
    if (!((counters[C_EXEC_UNION] >> pass) & 1u)) return;  // no segment runs this pass
    HUSKY_UNITS_P(PS, g, counters[C_NUM_GROUPS]) {
    const BigDesc B = bigs[big_of_group(bigs, counters[C_NUM_BIG], g)];
    bool flip;
    if (!pass_runs(B, pass, flip)) continue;
    const uint32_t t0 = B.first_tile + (g - B.first_group) * GROUP_TILES;
    const uint32_t nt = min((uint32_t)GROUP_TILES, B.first_tile + B.ntiles - t0);
    for (uint32_t d = threadIdx.x; d < (uint32_t)R; d += BLOCK) {
        uint32_t v[GROUP_TILES];
#pragma unroll
        for (int i = 0; i < GROUP_TILES; ++i) v[i] = (uint32_t)i < nt ? cnt[(size_t)(t0 + i) * 256 + d] : 0u;
        uint32_t run = 0;
#pragma unroll
        for (int i = 0; i < GROUP_TILES; ++i) {
            if ((uint32_t)i < nt) cnt[(size_t)(t0 + i) * 256 + d] = run;
            run += v[i];
        }
        gtot[(size_t)g * 256 + d] = run;
    }
    }
}

// Scan of the group totals of one big segment (in place) and the absolute
// start of every digit: binstart[segment][digit].
template <int BITS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_seg_scan(const BigDesc* __restrict__ bigs,
                                                    const uint32_t* __restrict__ counters,
                                                    uint32_t* __restrict__ gtot,
                                                    uint32_t* __restrict__ binstart, int pass) {
    constexpr int R = 1 << BITS;
    __shared__ uint32_t scratch[NWAVES];
    if (!((counters[C_EXEC_UNION] >> pass) & 1u)) return;  // no segment runs this pass
    HUSKY_UNITS_P(PS, b, counters[C_NUM_BIG]) {
    const BigDesc B = bigs[b];
    bool flip;
    if (!pass_runs(B, pass, flip)) continue;
    const uint32_t d = threadIdx.x;
    uint32_t run = 0;
    if (d < (uint32_t)R) {
        // up to 64 group totals in flight per thread (2^24 keys in one pass)
        constexpr int U = 64;
        for (uint32_t g0 = 0; g0 < B.ngroups; g0 += U) {
            uint32_t v[U];
#pragma unroll
            for (int i = 0; i < U; ++i)
                v[i] = g0 + i < B.ngroups ? gtot[(size_t)(B.first_group + g0 + i) * 256 + d] : 0u;
#pragma unroll
            for (int i = 0; i < U; ++i) {
                if (g0 + i < B.ngroups) gtot[(size_t)(B.first_group + g0 + i) * 256 + d] = run;
                run += v[i];
            }
        }
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_sum(d < (uint32_t)R ? run : 0u, scratch, &tot);
    if (d < (uint32_t)R) binstart[(size_t)b * 256 + d] = B.start + ex;
    }
}

// The two scans in one launch, for the device-wide fix-up's sorts (whose
// every pass is launched whether or not a group needs it): each group's
// workgroup scans its tiles' counts as k_group_scan does; a segment of one
// group gets its digit starts from that same workgroup, and in a longer
// segment the workgroup that completes its last group scans the group totals
// as k_seg_scan does.  Each group's workgroup publishes its totals with a
// device-scope release and counts itself in the segment's BigDesc::pad
// (which grows by ngroups per pass, so the count that reaches a multiple of
// ngroups is the pass's last).
template <int BITS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_scans(BigDesc* __restrict__ bigs,
                                                 const uint32_t* __restrict__ counters,
                                                 uint32_t* __restrict__ cnt, uint32_t* __restrict__ gtot,
                                                 uint32_t* __restrict__ binstart, int pass) {
    constexpr int R = 1 << BITS;
    static_assert(R <= BLOCK, "one thread per digit");
    __shared__ uint32_t scratch[NWAVES];
    __shared__ uint32_t s_last;
    if (!((counters[C_EXEC_UNION] >> pass) & 1u)) return;  // no segment runs this pass
    HUSKY_UNITS_P(PS, g, counters[C_NUM_GROUPS]) {
    const uint32_t b = big_of_group(bigs, counters[C_NUM_BIG], g);
    const BigDesc B = bigs[b];
    bool flip;
    if (!pass_runs(B, pass, flip)) continue;
    const uint32_t d = threadIdx.x;
    const uint32_t t0 = B.first_tile + (g - B.first_group) * GROUP_TILES;
    const uint32_t nt = min((uint32_t)GROUP_TILES, B.first_tile + B.ntiles - t0);
    uint32_t run = 0;
    if (d < (uint32_t)R) {
        uint32_t v[GROUP_TILES];
#pragma unroll
        for (int i = 0; i < GROUP_TILES; ++i) v[i] = (uint32_t)i < nt ? cnt[(size_t)(t0 + i) * 256 + d] : 0u;
#pragma unroll
        for (int i = 0; i < GROUP_TILES; ++i) {
            if ((uint32_t)i < nt) cnt[(size_t)(t0 + i) * 256 + d] = run;
            run += v[i];
        }
    }
    if (B.ngroups == 1) {
        uint32_t tot;
        const uint32_t ex = block_exclusive_sum(d < (uint32_t)R ? run : 0u, scratch, &tot);
        if (d < (uint32_t)R) {
            gtot[(size_t)g * 256 + d] = 0;
            binstart[(size_t)b * 256 + d] = B.start + ex;
        }
        continue;
    }
    if (d < (uint32_t)R) gtot[(size_t)g * 256 + d] = run;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&bigs[b].pad, 1u) + 1u) % B.ngroups == 0u ? 1u : 0u;
    __syncthreads();
    if (s_last) {
        __threadfence();
        // the segment's group totals (written by other workgroups) -> exclusive
        // over groups, in place; the digit starts from the segment totals
        uint32_t srun = 0;
        if (d < (uint32_t)R) {
            constexpr int U = 64;
            for (uint32_t g0 = 0; g0 < B.ngroups; g0 += U) {
                uint32_t v[U];
#pragma unroll
                for (int i = 0; i < U; ++i)
                    v[i] = g0 + i < B.ngroups
                               ? __hip_atomic_load(&gtot[(size_t)(B.first_group + g0 + i) * 256 + d],
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : 0u;
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    if (g0 + i < B.ngroups) gtot[(size_t)(B.first_group + g0 + i) * 256 + d] = srun;
                    srun += v[i];
                }
            }
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_sum(d < (uint32_t)R ? srun : 0u, scratch, &tot);
        if (d < (uint32_t)R) binstart[(size_t)b * 256 + d] = B.start + ex;
    }
    __syncthreads();  // s_last is reused by the next unit
    }
}

// Rank and scatter one tile.  The tile is staged through LDS twice, keys
// first and then indices in the same buffer, which halves the LDS a
// workgroup needs and lets more workgroups share a compute unit.  Each key
// also leaves, at its new position, its digit of the segment's next pass for
// that pass's count kernel: in dig (DIG_BYTES), or in the top byte of the
// value moved with it (DIG_IN_VALS: values and positions below 2^24; the
// value's low 24 bits are the value, and a segment's last pass leaves the
// top byte zero).
template <int BITS, int ITEMS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_scatter(
    uint64_t* __restrict__ keysA, uint32_t* __restrict__ valsA, uint64_t* __restrict__ keysB,
    uint32_t* __restrict__ valsB, const BigDesc* __restrict__ bigs,
    const uint32_t* __restrict__ counters, const uint32_t* __restrict__ cnt,
    const uint32_t* __restrict__ gtot, const uint32_t* __restrict__ binstart, int pass,
    const uint32_t* __restrict__ prog, uint8_t* __restrict__ dig, int dmode) {
    constexpr int R = 1 << BITS;
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_buf[TILE];
    __shared__ uint32_t s_whist[NWAVES * R];
    __shared__ uint32_t s_binstart[R];
    __shared__ uint32_t s_gbase[R];
    __shared__ uint32_t s_scan[NWAVES];
    if (!((counters[C_EXEC_UNION] >> pass) & 1u)) return;  // no segment runs this pass
    const uint32_t nbt = counters[C_BIG_TILES];
    HUSKY_UNITS_P(PS, bx, nbt) {
    const uint32_t t = xcd_remap(bx, nbt), tid = threadIdx.x;
    const uint32_t b = big_of_tile(bigs, counters[C_NUM_BIG], t);
    const BigDesc B = bigs[b];
    bool flip;
    if (!pass_runs(B, pass, flip)) continue;
    const uint64_t* ksrc = flip ? keysB : keysA;
    const uint32_t* vsrc = flip ? valsB : valsA;
    uint64_t* kdst = flip ? keysA : keysB;
    uint32_t* vdst = flip ? valsA : valsB;
    const uint32_t lt = t - B.first_tile;
    const uint32_t base = B.start + lt * TILE;
    const uint32_t nvalid = min(TILE, B.len - lt * TILE);

    DigitProg dp;
    dp.load(prog, pass);
    uint64_t k[ITEMS];
    uint32_t v[ITEMS];
    load_striped<ITEMS>(ksrc, vsrc, base, nvalid, k, v);
    // a program of one run (the usual case) needs no run loop
    const bool single = dp.nr <= 1;
    const uint32_t s0 = dp.run[0] & 63u, m0 = (1u << ((dp.run[0] >> 8) & 15u)) - 1u;
    uint32_t pos[ITEMS], dg[ITEMS];
    if (single) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) dg[i] = (uint32_t)(k[i] >> s0) & m0;
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) dg[i] = dp.digit(k[i]);
    }
    // the segment's next pass, if any, and its program
    const uint32_t later = dmode != DIG_NONE ? B.exec & ~((2u << pass) - 1u) : 0u;
    DigitProg dq;
    dq.load(prog, later ? __ffs(later) - 1 : pass);
    const bool single_q = dq.nr <= 1;
    const uint32_t sq = dq.run[0] & 63u, mq = (1u << ((dq.run[0] >> 8) & 15u)) - 1u;
    uint32_t bc = 0;
    rank_digits<BITS, ITEMS>(dg, nvalid, pos, s_whist, s_binstart, s_scan, &bc);
    if (tid < (uint32_t)R) {
        const uint32_t g = B.first_group + lt / GROUP_TILES;
        s_gbase[tid] = binstart[(size_t)b * 256 + tid] + gtot[(size_t)g * 256 + tid] +
                       cnt[(size_t)t * 256 + tid] - s_binstart[tid];
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s_buf[pos[i]] = k[i];
    __syncthreads();
    uint32_t dst[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = i * BLOCK + tid;
        dst[i] = 0;
        if (p < nvalid) {
            const uint64_t key = s_buf[p];
            dst[i] = s_gbase[single ? (uint32_t)(key >> s0) & m0 : dp.digit(key)] + p;
            kdst[dst[i]] = key;
            if (later) {
                const uint32_t nd = single_q ? (uint32_t)(key >> sq) & mq : dq.digit(key);
                if (dmode == DIG_BYTES)
                    dig[dst[i]] = (uint8_t)nd;
                else
                    dst[i] |= nd << 24;  // positions are below 2^24 here
            }
        }
    }
    __syncthreads();
    uint32_t* s_v = (uint32_t*)s_buf;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s_v[pos[i]] = dmode == DIG_IN_VALS ? v[i] & VAL_MASK : v[i];
    __syncthreads();
    if (dmode == DIG_IN_VALS) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = i * BLOCK + tid;
            if (p < nvalid) vdst[dst[i] & VAL_MASK] = s_v[p] | (dst[i] & ~VAL_MASK);
        }
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = i * BLOCK + tid;
            if (p < nvalid) vdst[dst[i]] = s_v[p];
        }
    }
    if (PS) __syncthreads();
    }
}

// Return odd-parity big segments from the alternate buffers.
template <bool PS>
__global__ __launch_bounds__(BLOCK) void k_copy_back(uint64_t* __restrict__ keysA,
                                                     uint32_t* __restrict__ valsA,
                                                     const uint64_t* __restrict__ keysB,
                                                     const uint32_t* __restrict__ valsB,
                                                     const BigDesc* __restrict__ bigs,
                                                     const uint32_t* __restrict__ counters,
                                                     uint32_t tile, bool clean) {
    HUSKY_UNITS_P(PS, t, counters[C_BIG_TILES]) {
        const BigDesc B = bigs[big_of_tile(bigs, counters[C_NUM_BIG], t)];
        if (clean && B.exec == 0) {
            // no pass ran: the values still carry the low bytes in their top bytes
            const uint32_t lt = t - B.first_tile;
            const uint32_t base = B.start + lt * tile;
            const uint32_t cnt = min(tile, B.len - lt * tile);
            for (uint32_t i = threadIdx.x; i < cnt; i += BLOCK) valsA[base + i] &= VAL_MASK;
            continue;
        }
        if (!(__popc(B.exec) & 1)) continue;
        const uint32_t lt = t - B.first_tile;
        const uint32_t base = B.start + lt * tile;
        const uint32_t cnt = min(tile, B.len - lt * tile);
        for (uint32_t i = threadIdx.x; i < cnt; i += BLOCK) {
            keysA[base + i] = keysB[base + i];
            valsA[base + i] = valsB[base + i];
        }
    }
}

// ------------------------------------------------------------------ single-tile segments
// One workgroup sorts a segment of 2..TILE keys entirely in LDS: every pass
// whose digit varies inside the segment ranks and scatters through LDS.
template <int BITS, int ITEMS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_tile_sort(uint64_t* __restrict__ keys,
                                                     uint32_t* __restrict__ vals,
                                                     const SegDesc* __restrict__ segs,
                                                     const uint32_t* __restrict__ counters,
                                                     int begin_bit, int end_bit) {
    constexpr int R = 1 << BITS;
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_whist[NWAVES * R];
    __shared__ uint32_t s_binstart[R];
    __shared__ uint32_t s_scan[NWAVES];
    __shared__ uint64_t s_or[NWAVES], s_and[NWAVES];

    HUSKY_UNITS_P(PS, sidx, counters[C_NUM_SEGS]) {
    const SegDesc d = segs[sidx];
    if (d.len < 2 || d.len > TILE) continue;
    const uint32_t nvalid = d.len;
    uint64_t k[ITEMS];
    uint32_t v[ITEMS];
    load_striped<ITEMS>(keys, vals, d.start, nvalid, k, v);

    // bits that vary inside the segment
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    uint64_t o = 0, a = ~0ull;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        if (p < nvalid) {
            o |= k[i];
            a &= k[i];
        }
    }
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) {
        o |= (uint64_t)__shfl_xor((unsigned long long)o, dd, WAVE);
        a &= (uint64_t)__shfl_xor((unsigned long long)a, dd, WAVE);
    }
    if (lane == 0) {
        s_or[w] = o;
        s_and[w] = a;
    }
    __syncthreads();
    uint64_t vary = 0;
    {
        uint64_t oo = 0, aa = ~0ull;
#pragma unroll
        for (int ww = 0; ww < NWAVES; ++ww) {
            oo |= s_or[ww];
            aa &= s_and[ww];
        }
        vary = oo ^ aa;
    }
    for (int shift = begin_bit; shift < end_bit; shift += BITS) {
        const int width = min(BITS, end_bit - shift);
        const uint32_t dmask = (1u << width) - 1u;
        if (!((uint32_t)(vary >> shift) & dmask)) continue;  // digit constant in the segment
        uint32_t pos[ITEMS];
        uint32_t cnt;
        rank_tile<BITS, ITEMS>(k, shift, dmask, nvalid, pos, s_whist, s_binstart, s_scan, &cnt);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            s_keys[pos[i]] = k[i];
            s_vals[pos[i]] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
            k[i] = s_keys[p];
            v[i] = s_vals[p];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        if (p < nvalid) {
            keys[d.start + p] = k[i];
            vals[d.start + p] = v[i];
        }
    }
    if (PS) __syncthreads();
    }
}

// Zero-fill (kept as a kernel so that captured graphs hold no memset nodes).
__global__ void k_zero_u64(uint64_t* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * BLOCK)
        p[i] = 0;
}
__global__ void k_zero_u32(uint32_t* __restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * BLOCK)
        p[i] = 0;
}

hipError_t zero_u64(uint64_t* p, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<size_t>((n + BLOCK - 1) / BLOCK, 4096);
    hipLaunchKernelGGL(k_zero_u64, dim3(blocks), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}
hipError_t zero_u32(uint32_t* p, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    const uint32_t blocks = (uint32_t)std::min<size_t>((n + BLOCK - 1) / BLOCK, 4096);
    hipLaunchKernelGGL(k_zero_u32, dim3(blocks), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ driver
template <int BITS, int ITEMS>
static hipError_t exec_impl(int begin_bit, int end_bit, uint32_t max_segs, uint32_t max_tiles,
                            const RadixScratch& sc, hipStream_t s, bool perfect_lsb) {
    const bool walk = sc.grid_cap != ~0u;
    max_tiles = std::min(max_tiles, sc.big_tile_cap);
    const uint32_t max_big = std::min(std::min(sc.big_cap, max_tiles / 2 + 1), std::max(max_segs, 1u));
    ProfScope ps(P_VARY, s);
    if (walk)
        hipLaunchKernelGGL((k_exec<BITS, true>), dim3(sc.grid(max_big)), dim3(BLOCK), 0, s, sc.bigs,
                           sc.counters, sc.korand, sc.segvary, sc.prog, begin_bit, end_bit, perfect_lsb);
    else
        hipLaunchKernelGGL((k_exec<BITS, false>), dim3(sc.grid(max_big)), dim3(BLOCK), 0, s, sc.bigs,
                           sc.counters, sc.korand, sc.segvary, sc.prog, begin_bit, end_bit, perfect_lsb);
    return hipGetLastError();
}

template <int BITS, int ITEMS, bool PS>
static hipError_t sort_impl(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                            uint32_t* vals_alt, int begin_bit, int end_bit, uint32_t max_segs,
                            uint32_t max_tiles, uint32_t pass_union, const RadixScratch& sc,
                            int pclass, bool tile_segments, hipStream_t s) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    const int npasses = (end_bit - begin_bit + BITS - 1) / BITS;
    BigDesc* bigs = sc.bigs;
    // single-tile segments (unless the caller sorts them itself)
    if (max_segs && tile_segments) {
        ProfScope ps(P_TILE_SORT, s);
        hipLaunchKernelGGL((k_tile_sort<BITS, ITEMS, PS>), dim3(sc.grid(max_segs)), dim3(BLOCK), 0, s, keys,
                           vals, sc.segs, sc.counters, begin_bit, end_bit);
    }
    max_tiles = std::min(max_tiles, sc.big_tile_cap);
    if (max_tiles == 0 || pass_union == 0) return hipGetLastError();
    // every big segment spans two or more tiles, and there are at most
    // max_segs segments
    const uint32_t max_big = std::min(std::min(sc.big_cap, max_tiles / 2 + 1), std::max(max_segs, 1u));
    const uint32_t max_groups = std::min(sc.group_cap, max_tiles / GROUP_TILES + max_big + 1);
    const int dmode = sc.dig_in_vals ? DIG_IN_VALS : sc.dig ? DIG_BYTES : DIG_NONE;
    // packed varying bits never outnumber the key bits in [begin_bit, end_bit)
    for (int p = 0; p < npasses; ++p) {
        if (!((pass_union >> p) & 1u)) continue;
        {
            ProfScope ps(pclass == P_SCATTER_FIX ? P_COUNT_SCAN_FIX : P_COUNT_SCAN, s);
            hipLaunchKernelGGL((k_count<BITS, ITEMS, PS>), dim3(sc.grid(max_tiles)), dim3(BLOCK), 0, s, keys,
                               keys_alt, vals, vals_alt, bigs, sc.counters, sc.cnt, p, sc.prog,
                               (const uint8_t*)sc.dig, dmode, sc.vals_low8 && dmode == DIG_IN_VALS);
            // one launch where segments are mostly of one scan group (the
            // fix-up's groups, batched instances); a single long instance
            // keeps the two launches (its groups' release fences cost more)
            if (PS || max_segs > 1) {
                hipLaunchKernelGGL((k_scans<BITS, PS>), dim3(sc.grid(max_groups)), dim3(BLOCK), 0, s, bigs,
                                   sc.counters, sc.cnt, sc.gtot, sc.binstart, p);
            } else {
                hipLaunchKernelGGL((k_group_scan<BITS, PS>), dim3(sc.grid(max_groups)), dim3(BLOCK), 0, s,
                                   bigs, sc.counters, sc.cnt, sc.gtot, p);
                hipLaunchKernelGGL((k_seg_scan<BITS, PS>), dim3(sc.grid(max_big)), dim3(BLOCK), 0, s, bigs,
                                   sc.counters, sc.gtot, sc.binstart, p);
            }
        }
        // timed (when profiling) by events that the dispatch itself records
        hipEvent_t ev0, ev1;
        ProfScope ps(pclass, s, &ev0, &ev1);
        hipExtLaunchKernelGGL((k_scatter<BITS, ITEMS, PS>), dim3(sc.grid(max_tiles)), dim3(BLOCK), 0, s, ev0, ev1, 0u,
                              keys, vals, keys_alt, vals_alt, (const BigDesc*)bigs,
                              (const uint32_t*)sc.counters, (const uint32_t*)sc.cnt,
                              (const uint32_t*)sc.gtot, (const uint32_t*)sc.binstart, p,
                              (const uint32_t*)sc.prog, sc.dig, dmode);
    }
    ProfScope ps(P_COPY_BACK, s);
    hipLaunchKernelGGL(k_copy_back<PS>, dim3(sc.grid(max_tiles)), dim3(BLOCK), 0, s, keys, vals, keys_alt,
                       vals_alt, bigs, sc.counters, TILE, sc.vals_low8);
    return hipGetLastError();
}

template <int ITEMS>
static void orand_launch(const uint64_t* keys, uint32_t max_tiles, const RadixScratch& sc, hipStream_t s) {
    if (sc.grid_cap != ~0u)
        hipLaunchKernelGGL((k_orand<ITEMS, true>), dim3(sc.grid(max_tiles)), dim3(BLOCK), 0, s, keys, sc.bigs,
                           sc.counters, sc.korand);
    else
        hipLaunchKernelGGL((k_orand<ITEMS, false>), dim3(sc.grid(max_tiles)), dim3(BLOCK), 0, s, keys, sc.bigs,
                           sc.counters, sc.korand);
}

hipError_t radix_reduce_tiles(const uint64_t* keys, uint32_t max_tiles, const RadixScratch& sc,
                              const RadixConfig& cfg, hipStream_t s) {
    max_tiles = std::min(max_tiles, sc.big_tile_cap);
    if (!max_tiles) return hipSuccess;
    ProfScope ps(P_VARY, s);
    if (cfg.items == 16)
        orand_launch<16>(keys, max_tiles, sc, s);
    else if (cfg.items == 12)
        orand_launch<12>(keys, max_tiles, sc, s);
    else
        orand_launch<8>(keys, max_tiles, sc, s);
    return hipGetLastError();
}

hipError_t radix_exec_masks(int begin_bit, int end_bit, uint32_t max_segs, uint32_t max_tiles,
                            const RadixScratch& sc, const RadixConfig& cfg, hipStream_t s,
                            bool perfect_lsb) {
    if (cfg.bits == 8) return exec_impl<8, 16>(begin_bit, end_bit, max_segs, max_tiles, sc, s, perfect_lsb);
    if (cfg.bits == 7) return exec_impl<7, 16>(begin_bit, end_bit, max_segs, max_tiles, sc, s, perfect_lsb);
    if (cfg.bits == 6) return exec_impl<6, 16>(begin_bit, end_bit, max_segs, max_tiles, sc, s, perfect_lsb);
    return hipErrorInvalidValue;
}

hipError_t radix_sort_segments(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                               uint32_t* vals_alt, int begin_bit, int end_bit,
                               uint32_t max_segs, uint32_t max_tiles, uint32_t pass_union,
                               const RadixScratch& sc, const RadixConfig& cfg, int pclass,
                               hipStream_t s, bool tile_segments) {
#define HUSKY_SORT_CASE(B, I)                                                                      \
    if (cfg.bits == B && cfg.items == I)                                                           \
        return sc.grid_cap != ~0u                                                                  \
                   ? sort_impl<B, I, true>(keys, vals, keys_alt, vals_alt, begin_bit, end_bit,     \
                                           max_segs, max_tiles, pass_union, sc, pclass,            \
                                           tile_segments, s)                                       \
                   : sort_impl<B, I, false>(keys, vals, keys_alt, vals_alt, begin_bit, end_bit,    \
                                            max_segs, max_tiles, pass_union, sc, pclass,           \
                                            tile_segments, s);
    HUSKY_SORT_CASE(8, 16)
    HUSKY_SORT_CASE(8, 12)
    HUSKY_SORT_CASE(8, 8)
    HUSKY_SORT_CASE(7, 16)
    HUSKY_SORT_CASE(7, 12)
    HUSKY_SORT_CASE(7, 8)
    HUSKY_SORT_CASE(6, 16)
    HUSKY_SORT_CASE(6, 12)
    HUSKY_SORT_CASE(6, 8)
#undef HUSKY_SORT_CASE
    return hipErrorInvalidValue;
}

}  // namespace husky
