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
//  * a segment of at most one tile (256 threads x ITEMS keys) is sorted
//    entirely in LDS by one workgroup (k_tile_sort), digit passes whose digit
//    is the same in every key of the segment skipped;
//  * longer ("big") segments go through one histogram kernel that counts the
//    digits of every pass at once, one scan kernel per segment (which also
//    marks passes whose digit is constant across the whole segment), then one
//    onesweep kernel per digit pass: every tile ranks its keys locally with
//    wavefront ballots, publishes its per-digit counts, finds its global
//    offsets by decoupled look-back over earlier tiles of the same segment and
//    scatters through LDS so that neighbouring lanes write neighbouring
//    addresses.  Tiles take their index from an atomic counter, so a tile
//    only ever waits on tiles that are already running.
//  * each big segment's skipped passes are tracked with a bit mask; the
//    ping-pong buffer holding its data after pass p is the parity of the
//    passes it ran before p, and a final copy returns odd-parity segments to
//    the primary buffers.

#include <algorithm>

#include "common.h"
#include "internal.h"

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

// One workgroup: segment descriptors, the two tile spaces and the big list.
template <typename Src>
__global__ __launch_bounds__(BLOCK) void k_seg_setup(Src src, SegDesc* segs, SegDesc* bigs,
                                                     uint32_t* counters, uint32_t tile) {
    __shared__ uint32_t scratch[NWAVES];
    const uint32_t S = src.count();
    uint32_t carry_all = 0, carry_big = 0, carry_nbig = 0;
    for (uint32_t base = 0; base < S; base += BLOCK) {
        const uint32_t i = base + threadIdx.x;
        uint32_t st = 0, ln = 0;
        if (i < S) src.get(i, st, ln);
        const uint32_t nt = (ln + tile - 1) / tile;
        const bool big = ln > tile;
        uint32_t tot_all, tot_big, tot_nbig;
        const uint32_t ex_all = block_exclusive_sum(nt, scratch, &tot_all);
        const uint32_t ex_big = block_exclusive_sum(big ? nt : 0u, scratch, &tot_big);
        const uint32_t ex_nbig = block_exclusive_sum(big ? 1u : 0u, scratch, &tot_nbig);
        if (i < S) {
            SegDesc d;
            d.start = st;
            d.len = ln;
            d.first_tile = carry_all + ex_all;
            d.aux = big ? carry_nbig + ex_nbig : NOT_BIG;
            segs[i] = d;
            if (big) {
                SegDesc b;
                b.start = st;
                b.len = ln;
                b.first_tile = carry_big + ex_big;
                b.aux = 0;  // exec mask, written by the scan kernel
                bigs[carry_nbig + ex_nbig] = b;
            }
        }
        carry_all += tot_all;
        carry_big += tot_big;
        carry_nbig += tot_nbig;
    }
    if (threadIdx.x == 0) {
        counters[C_ALL_TILES] = carry_all;
        counters[C_BIG_TILES] = carry_big;
        counters[C_NUM_BIG] = carry_nbig;
        counters[C_NUM_SEGS] = S;
    }
    if (threadIdx.x < MAX_PASSES) counters[C_TILE0 + threadIdx.x] = 0;
}

// Bigs are stored after segs in the descriptor array: segs[0, seg_cap),
// bigs[seg_cap, seg_cap + big_cap).
static inline SegDesc* bigs_of(const RadixScratch& sc) { return sc.segs + sc.seg_cap; }

hipError_t radix_segments_from_offsets(const uint64_t* seg_offsets, uint32_t n_segs,
                                       const RadixScratch& sc, const RadixConfig& cfg,
                                       hipStream_t s) {
    SrcOffsets src{seg_offsets, n_segs};
    ProfScope ps(P_SETUP, s);
    hipLaunchKernelGGL(k_seg_setup<SrcOffsets>, dim3(1), dim3(BLOCK), 0, s, src, sc.segs,
                       bigs_of(sc), sc.counters, (uint32_t)cfg.tile());
    return hipGetLastError();
}
hipError_t radix_segments_single(uint32_t n, const RadixScratch& sc, const RadixConfig& cfg,
                                 hipStream_t s) {
    SrcSingle src{n};
    ProfScope ps(P_SETUP, s);
    hipLaunchKernelGGL(k_seg_setup<SrcSingle>, dim3(1), dim3(BLOCK), 0, s, src, sc.segs,
                       bigs_of(sc), sc.counters, (uint32_t)cfg.tile());
    return hipGetLastError();
}
hipError_t radix_segments_from_items(const RunItem* items, const uint32_t* count,
                                     uint32_t max_items, const RadixScratch& sc,
                                     const RadixConfig& cfg, hipStream_t s) {
    SrcItems src{items, count, max_items};
    ProfScope ps(P_SETUP, s);
    hipLaunchKernelGGL(k_seg_setup<SrcItems>, dim3(1), dim3(BLOCK), 0, s, src, sc.segs,
                       bigs_of(sc), sc.counters, (uint32_t)cfg.tile());
    return hipGetLastError();
}

// ------------------------------------------------------------------ histogram
// Counts the digit of every pass for the keys of big segments.  Workgroup b
// covers big-space tiles [b*G, (b+1)*G) and flushes its LDS counts to the
// segment's row whenever the segment changes.
template <int BITS>
__global__ __launch_bounds__(BLOCK) void k_hist(const uint64_t* __restrict__ keys,
                                                const SegDesc* __restrict__ bigs,
                                                const uint32_t* __restrict__ counters,
                                                uint32_t* __restrict__ hist, uint32_t tile,
                                                uint32_t G, int begin_bit, int end_bit,
                                                int npasses) {
    constexpr int R = 1 << BITS;
    constexpr int ROW = MAX_PASSES * R;
    // one row of counters per wavefront keeps the LDS atomics of different
    // wavefronts apart; a wavefront whose 64 digits agree adds 64 once
    __shared__ uint32_t s_h[NWAVES * ROW];
    const uint32_t total = counters[C_BIG_TILES], nb = counters[C_NUM_BIG];
    const uint32_t t0 = blockIdx.x * G;
    if (t0 >= total) return;
    const uint32_t t1 = min(total, t0 + G);
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    uint32_t* my = s_h + w * ROW;
    for (uint32_t i = threadIdx.x; i < (uint32_t)(NWAVES * ROW); i += BLOCK) s_h[i] = 0;
    uint32_t b = find_seg(bigs, nb, t0);
    SegDesc d = bigs[b];
    __syncthreads();
    auto flush = [&](uint32_t seg) {
        for (uint32_t i = threadIdx.x; i < (uint32_t)(npasses * R); i += BLOCK) {
            uint32_t v = 0;
#pragma unroll
            for (int ww = 0; ww < NWAVES; ++ww) {
                v += s_h[ww * ROW + i];
                s_h[ww * ROW + i] = 0;
            }
            if (v) atomicAdd(&hist[(size_t)seg * MAX_PASSES * 256 + (i / R) * 256 + (i % R)], v);
        }
    };
    for (uint32_t t = t0; t < t1; ++t) {
        if (b + 1 < nb && bigs[b + 1].first_tile <= t) {
            __syncthreads();
            flush(b);  // segment changes
            ++b;
            d = bigs[b];
            __syncthreads();
        }
        const uint32_t lt = t - d.first_tile;
        const uint32_t pos0 = d.start + lt * tile;
        const uint32_t cnt = min(tile, d.len - lt * tile);
        // whole wavefronts walk the tile so that ballots see all 64 lanes
        for (uint32_t i0 = w * WAVE; i0 < cnt; i0 += BLOCK) {
            const uint32_t i = i0 + lane;
            const bool ok = i < cnt;
            const uint64_t k = ok ? keys[pos0 + i] : 0ull;
            const bool full = ballot(ok) == ~0ull;
            for (int p = 0; p < npasses; ++p) {
                const int sh = begin_bit + p * BITS;
                const int wd = min(BITS, end_bit - sh);
                const uint32_t dg = (uint32_t)(k >> sh) & ((1u << wd) - 1u);
                const uint32_t d0 = readlane(dg, 0);
                if (full && ballot(dg == d0) == ~0ull) {
                    if (lane == 0) my[p * R + d0] += WAVE;
                } else if (ok) {
                    atomicAdd(&my[p * R + dg], 1u);
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();
    flush(b);
}

// Exclusive scan of every pass's counts of one big segment (in place) and
// the mask of passes whose digit varies inside the segment.
template <int BITS>
__global__ __launch_bounds__(BLOCK) void k_hist_scan(SegDesc* __restrict__ bigs,
                                                     const uint32_t* __restrict__ counters,
                                                     uint32_t* __restrict__ hist, int npasses) {
    constexpr int R = 1 << BITS;
    __shared__ uint32_t scratch[NWAVES];
    const uint32_t b = blockIdx.x;
    if (b >= counters[C_NUM_BIG]) return;
    const uint32_t len = bigs[b].len;
    uint32_t mask = 0;
    for (int p = 0; p < npasses; ++p) {
        uint32_t* row = hist + (size_t)b * MAX_PASSES * 256 + p * 256;
        const uint32_t v = threadIdx.x < (uint32_t)R ? row[threadIdx.x] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_sum(v, scratch, &tot);
        const int constant = __syncthreads_or(v == len);
        if (threadIdx.x < (uint32_t)R) row[threadIdx.x] = ex;
        if (!constant) mask |= 1u << p;
    }
    if (threadIdx.x == 0) bigs[b].aux = mask;
}

// ------------------------------------------------------------------ tile ranking
// Ranks the ITEMS keys of every thread of one tile by their digit
// (key >> shift) & dmask, dmask < 2^BITS.
// Keys sit in "wave-striped" order: item k of lane l of wave w is tile
// position w*64*ITEMS + k*64 + l; positions >= nvalid are padding and rank
// last.  On return pos[k] is the key's position in the digit-sorted tile
// (stable in tile position) and, for tid < R, *bin_count holds the number of
// valid keys with digit tid and s_binstart[tid] its first position.
template <int BITS, int ITEMS>
__device__ __forceinline__ void rank_tile(const uint64_t (&keys)[ITEMS], int shift,
                                          uint32_t dmask, uint32_t nvalid, uint32_t (&pos)[ITEMS],
                                          uint32_t* s_whist, uint32_t* s_binstart,
                                          uint32_t* s_scan, uint32_t* bin_count) {
    constexpr int R = 1 << BITS;
    const uint32_t tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
    for (uint32_t i = tid; i < (uint32_t)(NWAVES * R); i += BLOCK) s_whist[i] = 0;
    __syncthreads();
    // Each wavefront owns one histogram row.  Within an iteration every lane
    // reads its digit's count before the one lane per digit updates it; LDS
    // operations of one wavefront complete in order, and the empty asm with a
    // memory clobber keeps the compiler from reusing a count across
    // iterations.
    uint32_t* wh = s_whist + w * R;
    uint32_t rank[ITEMS], dig[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t p = w * WAVE * ITEMS + k * WAVE + lane;
        const uint32_t d = p < nvalid ? ((uint32_t)(keys[k] >> shift) & dmask) : (uint32_t)(R - 1);
        dig[k] = d;
        // lanes holding the same digit: for every digit bit keep the lanes
        // whose bit agrees (ballot, inverted where this lane's bit is 0)
        uint32_t plo = ~0u, phi = ~0u;
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const uint32_t bit = (d >> b) & 1u;
            const uint64_t bal = ballot(bit != 0);
            const uint32_t flip = bit - 1u;  // 0 when set, all ones when clear
            plo &= (uint32_t)bal ^ flip;
            phi &= (uint32_t)(bal >> 32) ^ flip;
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
        const uint32_t cnt = (uint32_t)__popc(plo) + (uint32_t)__popc(phi);
        const uint32_t base = wh[d];
        __asm__ volatile("" ::: "memory");
        if (below == cnt - 1) wh[d] = base + cnt;
        __asm__ volatile("" ::: "memory");
        rank[k] = base + below;
    }
    __syncthreads();
    uint32_t tot = 0;
    if (tid < (uint32_t)R) {
#pragma unroll
        for (int ww = 0; ww < NWAVES; ++ww) {
            const uint32_t c = s_whist[ww * R + tid];
            s_whist[ww * R + tid] = tot;
            tot += c;
        }
    }
    uint32_t all;
    const uint32_t ex = block_exclusive_sum(tid < (uint32_t)R ? tot : 0u, s_scan, &all);
    if (tid < (uint32_t)R) {
        s_binstart[tid] = ex;
        const uint32_t pad = (uint32_t)(BLOCK * ITEMS) - nvalid;
        *bin_count = (tid == (uint32_t)(R - 1)) ? tot - pad : tot;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) pos[k] = s_binstart[dig[k]] + s_whist[w * R + dig[k]] + rank[k];
}

template <int ITEMS>
__device__ __forceinline__ void load_striped(const uint64_t* __restrict__ keys,
                                             const uint32_t* __restrict__ vals, uint32_t base,
                                             uint32_t nvalid, uint64_t (&k)[ITEMS],
                                             uint32_t (&v)[ITEMS]) {
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        if (p < nvalid) {
            k[i] = keys[base + p];
            v[i] = vals[base + p];
        } else {
            k[i] = ~0ull;
            v[i] = 0;
        }
    }
}

// ------------------------------------------------------------------ onesweep pass
template <int BITS, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_onesweep(
    uint64_t* __restrict__ keysA, uint32_t* __restrict__ valsA, uint64_t* __restrict__ keysB,
    uint32_t* __restrict__ valsB, const SegDesc* __restrict__ bigs,
    uint32_t* __restrict__ counters, const uint32_t* __restrict__ hist,
    uint64_t* __restrict__ status, int pass, int shift, uint32_t dmask) {
    constexpr int R = 1 << BITS;
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_whist[NWAVES * R];
    __shared__ uint32_t s_binstart[R];
    __shared__ uint32_t s_gbase[R];
    __shared__ uint32_t s_scan[NWAVES];
    __shared__ uint32_t s_tile;

    const uint32_t tid = threadIdx.x;
    // workgroups beyond the tile count leave before taking a tile id, so the
    // ids handed out are exactly 0 .. tiles-1
    const uint32_t n_tiles = counters[C_BIG_TILES];
    if (blockIdx.x >= n_tiles) return;
    if (tid == 0) s_tile = atomicAdd(&counters[C_TILE0 + pass], 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t b = find_seg(bigs, counters[C_NUM_BIG], tile);
    const SegDesc d = bigs[b];
    const uint32_t exec = d.aux;
    if (!((exec >> pass) & 1u)) return;  // every tile of this segment skips the pass
    const bool flip = __popc(exec & ((1u << pass) - 1u)) & 1u;
    const uint64_t* ksrc = flip ? keysB : keysA;
    const uint32_t* vsrc = flip ? valsB : valsA;
    uint64_t* kdst = flip ? keysA : keysB;
    uint32_t* vdst = flip ? valsA : valsB;

    const uint32_t lt = tile - d.first_tile;
    const uint32_t base = d.start + lt * TILE;
    const uint32_t nvalid = min(TILE, d.len - lt * TILE);

    uint64_t k[ITEMS];
    uint32_t v[ITEMS];
    load_striped<ITEMS>(ksrc, vsrc, base, nvalid, k, v);
    uint32_t pos[ITEMS];
    uint32_t cnt = 0;
    rank_tile<BITS, ITEMS>(k, shift, dmask, nvalid, pos, s_whist, s_binstart, s_scan, &cnt);

    // decoupled look-back, one bin per thread
    if (tid < (uint32_t)R) {
        const uint64_t FA = (uint64_t)(2 * pass + 1) << 32;  // aggregate of this tile
        const uint64_t FI = (uint64_t)(2 * pass + 2) << 32;  // inclusive prefix
        uint64_t* st = status + (size_t)tile * 256 + tid;
        uint32_t excl = 0;
        if (lt == 0) {
            store_agent(st, FI | cnt);
        } else {
            store_agent(st, FA | cnt);
            uint32_t j = tile - 1;
            for (;;) {
                const uint64_t sv = load_agent(status + (size_t)j * 256 + tid);
                const uint64_t f = sv & 0xFFFFFFFF00000000ull;
                if (f < FA) {
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += (uint32_t)sv;
                if (f == FI) break;
                --j;
            }
            store_agent(st, FI | (excl + cnt));
        }
        const uint32_t gstart = hist[(size_t)b * MAX_PASSES * 256 + pass * 256 + tid];
        s_gbase[tid] = d.start + gstart + excl - s_binstart[tid];
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        s_keys[pos[i]] = k[i];
        s_vals[pos[i]] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = i * BLOCK + tid;
        if (p < nvalid) {
            const uint64_t key = s_keys[p];
            const uint32_t dg = (uint32_t)(key >> shift) & dmask;
            const uint32_t dst = s_gbase[dg] + p;
            kdst[dst] = key;
            vdst[dst] = s_vals[p];
        }
    }
}

// Return odd-parity big segments from the alternate buffers.
__global__ __launch_bounds__(BLOCK) void k_copy_back(uint64_t* __restrict__ keysA,
                                                     uint32_t* __restrict__ valsA,
                                                     const uint64_t* __restrict__ keysB,
                                                     const uint32_t* __restrict__ valsB,
                                                     const SegDesc* __restrict__ bigs,
                                                     const uint32_t* __restrict__ counters,
                                                     uint32_t tile) {
    const uint32_t t = blockIdx.x;
    if (t >= counters[C_BIG_TILES]) return;
    const uint32_t b = find_seg(bigs, counters[C_NUM_BIG], t);
    const SegDesc d = bigs[b];
    if (!(__popc(d.aux) & 1)) return;
    const uint32_t lt = t - d.first_tile;
    const uint32_t base = d.start + lt * tile;
    const uint32_t cnt = min(tile, d.len - lt * tile);
    for (uint32_t i = threadIdx.x; i < cnt; i += BLOCK) {
        keysA[base + i] = keysB[base + i];
        valsA[base + i] = valsB[base + i];
    }
}

// ------------------------------------------------------------------ single-tile segments
// One workgroup sorts a segment of 2..TILE keys entirely in LDS: every pass
// whose digit varies inside the segment ranks and scatters through LDS.
template <int BITS, int ITEMS>
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

    const uint32_t sidx = blockIdx.x;
    if (sidx >= counters[C_NUM_SEGS]) return;
    const SegDesc d = segs[sidx];
    if (d.len < 2 || d.len > TILE) return;
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
static hipError_t sort_impl(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                            uint32_t* vals_alt, int begin_bit, int end_bit, uint32_t max_segs,
                            uint32_t max_tiles, const RadixScratch& sc, int pclass,
                            hipStream_t s) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    const int npasses = (end_bit - begin_bit + BITS - 1) / BITS;
    SegDesc* bigs = bigs_of(sc);
    // single-tile segments
    if (max_segs) {
        ProfScope ps(P_TILE_SORT, s);
        hipLaunchKernelGGL((k_tile_sort<BITS, ITEMS>), dim3(max_segs), dim3(BLOCK), 0, s, keys,
                           vals, sc.segs, sc.counters, begin_bit, end_bit);
    }
    if (max_tiles == 0) return hipGetLastError();
    // big segments
    // every multi-tile segment spans two or more tiles, and there are at most
    // max_segs segments
    const uint32_t max_big = std::min(std::min(sc.big_cap, max_tiles / 2 + 1), std::max(max_segs, 1u));
    hipError_t e = zero_u32(sc.hist, (size_t)max_big * MAX_PASSES * 256, s);
    if (e != hipSuccess) return e;
    e = zero_u64(sc.status, (size_t)std::min(max_tiles, sc.lookback_cap) * 256, s);
    if (e != hipSuccess) return e;
    e = zero_u32(sc.counters + C_TILE0, MAX_PASSES, s);
    if (e != hipSuccess) return e;
    const uint32_t G = 8;
    {
        ProfScope ps(P_HIST, s);
        hipLaunchKernelGGL((k_hist<BITS>), dim3((max_tiles + G - 1) / G), dim3(BLOCK), 0, s, keys,
                           bigs, sc.counters, sc.hist, TILE, G, begin_bit, end_bit, npasses);
    }
    {
        ProfScope ps(P_HIST_SCAN, s);
        hipLaunchKernelGGL((k_hist_scan<BITS>), dim3(max_big), dim3(BLOCK), 0, s, bigs,
                           sc.counters, sc.hist, npasses);
    }
    for (int p = 0; p < npasses; ++p) {
        const int shift = begin_bit + p * BITS;
        const uint32_t dmask = (1u << min(BITS, end_bit - shift)) - 1u;  // top digit may be narrower
        ProfScope ps(pclass, s);
        hipLaunchKernelGGL((k_onesweep<BITS, ITEMS>), dim3(max_tiles), dim3(BLOCK), 0, s, keys,
                           vals, keys_alt, vals_alt, bigs, sc.counters, sc.hist, sc.status, p,
                           shift, dmask);
    }
    ProfScope ps(P_COPY_BACK, s);
    hipLaunchKernelGGL(k_copy_back, dim3(max_tiles), dim3(BLOCK), 0, s, keys, vals, keys_alt,
                       vals_alt, bigs, sc.counters, TILE);
    return hipGetLastError();
}

hipError_t radix_sort_segments(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                               uint32_t* vals_alt, int begin_bit, int end_bit,
                               uint32_t max_segs, uint32_t max_tiles, const RadixScratch& sc,
                               const RadixConfig& cfg, int pclass, hipStream_t s) {
#define HUSKY_SORT_CASE(B, I)                                                                 \
    if (cfg.bits == B && cfg.items == I)                                                      \
        return sort_impl<B, I>(keys, vals, keys_alt, vals_alt, begin_bit, end_bit, max_segs, \
                               max_tiles, sc, pclass, s);
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
