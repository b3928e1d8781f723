// Stable ranking of one tile of keys by one digit (wavefront ballots) and a
// running maximum over a tile, shared by the radix sort, the LDS fix-up tier
// and the learned bucket passes.
#pragma once

#include "common.h"

namespace husky {

// ------------------------------------------------------------------ tile ranking
// m & ~(bal ^ f) in one three-input bit operation: the truth table takes the
// operands as the columns 0xF0, 0xCC and 0xAA, so this function's table is
// 0xF0 & ~(0xCC ^ 0xAA) = 0x90.
__device__ __forceinline__ uint32_t bit_agree(uint32_t m, uint32_t bal, uint32_t f) {
    return __builtin_amdgcn_bitop3_b32(m, bal, f, 0x90);
}

// Ranks the ITEMS digits (< 2^BITS) of every thread of one tile of a
// workgroup of NW wavefronts (NW * 64 >= 2^BITS threads).  Digits sit in
// "wave-striped" order: item k of lane l of wave w is tile position
// w*64*ITEMS + k*64 + l; positions >= nvalid are padding and rank last.  On
// return pos[k] is the item's position in the digit-sorted tile (stable in
// tile position) and, for tid < R, *bin_count holds the number of valid items
// with digit tid and s_binstart[tid] its first position.  s_whist: NW * R
// words; s_scan: NW words.
template <int BITS, int ITEMS, int NW = NWAVES>
__device__ __forceinline__ void rank_digits(uint32_t (&dig)[ITEMS], uint32_t nvalid,
                                            uint32_t (&pos)[ITEMS], uint32_t* s_whist,
                                            uint32_t* s_binstart, uint32_t* s_scan,
                                            uint32_t* bin_count) {
    constexpr int R = 1 << BITS;
    constexpr uint32_t NT = NW * WAVE;
    const uint32_t tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
    for (uint32_t i = tid; i < (uint32_t)(NW * R); i += NT) s_whist[i] = 0;
    __syncthreads();
    // Each wavefront owns one histogram row.  For every item, the lanes
    // holding the same digit find each other with one ballot per digit bit;
    // all of them read the row's count for that digit, then the highest of
    // them adds the group's size with an LDS atomic.  LDS operations of one
    // wavefront execute in order, so each read sees every earlier item's
    // add, and no item waits for the previous one's result.
    uint32_t* wh = s_whist + w * R;
    uint32_t base[ITEMS], bl[(ITEMS + 4) / 5];  // counts read; ranks in the group, 6 bits each
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t p = w * WAVE * ITEMS + k * WAVE + lane;
        const uint32_t d = p < nvalid ? dig[k] : (uint32_t)(R - 1);
        dig[k] = d;
        // lanes holding the same digit: for every digit bit keep the lanes
        // whose bit agrees (the ballot, inverted where this lane's bit is 0)
        uint32_t plo = ~0u, phi = ~0u;
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            // the bit as all ones or all zeros (one signed bit-field extract),
            // its ballot, and one three-input bit operation per mask half
            const uint32_t f = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
            const uint64_t bal = ballot((int32_t)f < 0);
            plo = bit_agree(plo, (uint32_t)bal, f);
            phi = bit_agree(phi, (uint32_t)(bal >> 32), f);
        }
        const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
        const uint32_t cnt = (uint32_t)__popc(plo) + (uint32_t)__popc(phi);
        base[k] = wh[d];
        if (below == cnt - 1)
            __hip_atomic_fetch_add(&wh[d], cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        bl[k / 5] = (k % 5 ? bl[k / 5] : 0u) | below << (6 * (k % 5));
    }
    uint32_t rank[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) rank[k] = base[k] + ((bl[k / 5] >> (6 * (k % 5))) & 63u);
    __syncthreads();
    uint32_t tot = 0;
    if (tid < (uint32_t)R) {
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            const uint32_t c = s_whist[ww * R + tid];
            s_whist[ww * R + tid] = tot;
            tot += c;
        }
    }
    uint32_t all;
    const uint32_t ex = block_exclusive_sum<NW>(tid < (uint32_t)R ? tot : 0u, s_scan, &all);
    if (tid < (uint32_t)R) {
        s_binstart[tid] = ex;
        const uint32_t pad = NT * ITEMS - nvalid;
        *bin_count = (tid == (uint32_t)(R - 1)) ? tot - pad : tot;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) pos[k] = s_binstart[dig[k]] + s_whist[w * R + dig[k]] + rank[k];
}

// ------------------------------------------------------------------ tile histogram
// One tile of src in the wave-striped layout, positions >= nvalid zero.  A
// whole tile loads without per-item conditions, so that every load is in
// flight before the first is used.
template <int ITEMS, typename T>
__device__ __forceinline__ void load_tile(const T* __restrict__ src, uint32_t nvalid, T (&x)[ITEMS]) {
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    if (nvalid == (uint32_t)(BLOCK * ITEMS)) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) x[i] = src[w * WAVE * ITEMS + i * WAVE + lane];
    } else {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
            x[i] = p < nvalid ? src[p] : T(0);
        }
    }
}


// Counts of the 8-bit digits of one tile (wave-striped layout as above,
// positions >= nvalid skipped): out[d] = number of items with digit d.
// dig_of(i) gives item i's digit.  The workgroup keeps HIST_COPIES
// histograms, lane l of every wavefront adding to copy l % HIST_COPIES, so
// lanes holding the same digit (skewed digits, or keys grouped by earlier
// passes) collide at most 64 / HIST_COPIES ways on one LDS address inside
// one instruction; rows are HIST_STRIDE = 257 words apart, so the copies of
// one digit sit in different banks.  s_h: HIST_COPIES * HIST_STRIDE words.
// The caller issues its loads first: the clearing here overlaps them.
constexpr int HIST_COPIES = 16, HIST_STRIDE = 257, HIST_WORDS = HIST_COPIES * HIST_STRIDE;
template <int ITEMS, typename F>
__device__ __forceinline__ void tile_histogram(F dig_of, uint32_t nvalid, uint32_t* s_h,
                                               uint32_t* __restrict__ out) {
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    for (uint32_t i = threadIdx.x; i < (uint32_t)HIST_WORDS; i += BLOCK) s_h[i] = 0;
    __syncthreads();
    uint32_t* my = s_h + (lane % HIST_COPIES) * HIST_STRIDE;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        if (p < nvalid)
            __hip_atomic_fetch_add(&my[dig_of(i)], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < 256u; d += BLOCK) {
        uint32_t v = 0;
#pragma unroll
        for (int r = 0; r < HIST_COPIES; ++r) v += s_h[r * HIST_STRIDE + d];
        out[d] = v;
    }
}

// The same ranking by the digit (key >> shift) & dmask, dmask < 2^BITS.
template <int BITS, int ITEMS>
__device__ __forceinline__ void rank_tile(const uint64_t (&keys)[ITEMS], int shift,
                                          uint32_t dmask, uint32_t nvalid, uint32_t (&pos)[ITEMS],
                                          uint32_t* s_whist, uint32_t* s_binstart,
                                          uint32_t* s_scan, uint32_t* bin_count) {
    uint32_t dig[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) dig[k] = (uint32_t)(keys[k] >> shift) & dmask;
    rank_digits<BITS, ITEMS>(dig, nvalid, pos, s_whist, s_binstart, s_scan, bin_count);
}

// Running maximum over the tile in position order, with positions held in the
// wave-striped layout of rank_digits: every position's value replaced by the
// maximum of the values at or before it.  s_tmp: NW * 64 * ITEMS words.
template <int ITEMS, int NW>
__device__ __forceinline__ void tile_running_max(uint32_t (&v)[ITEMS], uint32_t* s_tmp,
                                                 uint32_t* s_scan) {
    const uint32_t tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s_tmp[w * WAVE * ITEMS + i * WAVE + lane] = v[i];
    __syncthreads();
    // thread t owns positions [ITEMS t, ITEMS t + ITEMS)
    uint32_t m = 0, loc[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        m = max(m, s_tmp[tid * ITEMS + i]);
        loc[i] = m;
    }
    uint32_t inc = m;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const uint32_t t = __shfl_up(inc, d, WAVE);
        if (lane >= (uint32_t)d) inc = max(inc, t);
    }
    if (lane == WAVE - 1) s_scan[w] = inc;
    uint32_t prev = __shfl_up(inc, 1, WAVE);
    if (lane == 0) prev = 0;
    __syncthreads();
    for (uint32_t ww = 0; ww < w; ++ww) prev = max(prev, s_scan[ww]);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) s_tmp[tid * ITEMS + i] = max(prev, loc[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) v[i] = s_tmp[w * WAVE * ITEMS + i * WAVE + lane];
    __syncthreads();
}

// One pass's digit program (common.h), held in scalar registers.
struct DigitProg {
    uint32_t nr;
    uint32_t run[PROG_WORDS - 1];
    __device__ __forceinline__ void load(const uint32_t* __restrict__ prog, int pass) {
        const uint32_t* p = prog + pass * PROG_WORDS;
        nr = p[0];
#pragma unroll
        for (int r = 0; r < PROG_WORDS - 1; ++r) run[r] = (uint32_t)r < nr ? p[1 + r] : 0u;
    }
    __device__ __forceinline__ uint32_t digit(uint64_t key) const {
        // the first run starts at digit bit 0
        uint32_t d = (uint32_t)(key >> (run[0] & 63u)) & ((1u << ((run[0] >> 8) & 15u)) - 1u);
#pragma unroll
        for (int r = 1; r < PROG_WORDS - 1; ++r) {
            if ((uint32_t)r >= nr) break;
            const uint32_t w = run[r];
            const uint32_t len = (w >> 8) & 15u;
            d |= ((uint32_t)(key >> (w & 63u)) & ((1u << len) - 1u)) << ((w >> 16) & 15u);
        }
        return d;
    }
};

// A 64-bit value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// For a sort inside one workgroup: packs the bits of every key that vary
// (`vary`, the same in every lane) into the key's low bits, in order, when
// that saves an 8-bit digit pass, and returns the bits that vary afterwards.
// Bits that do not vary cannot change the order of the keys or which keys
// are equal, so the packed keys sort and compare like the keys.
template <int ITEMS>
__device__ __forceinline__ uint64_t pack_varying(uint64_t (&k)[ITEMS], uint64_t vary) {
    vary = uniform64(vary);
    int windows = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) windows += ((vary >> (8 * j)) & 0xFFull) ? 1 : 0;
    const int bits = __popcll(vary);
    if ((bits + 7) / 8 >= windows) return vary;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        uint64_t m = vary, out = 0;
        int dst = 0;
        while (m) {  // runs of adjacent varying bits
            const int s = __builtin_ctzll(m);
            const uint64_t rest = ~(m >> s);
            const int len = rest ? __builtin_ctzll(rest) : 64 - s;
            const uint64_t run = len >= 64 ? ~0ull : (1ull << len) - 1ull;
            out |= ((k[i] >> s) & run) << dst;
            dst += len;
            m &= ~(run << s);
        }
        k[i] = out;
    }
    return bits >= 64 ? ~0ull : (1ull << bits) - 1ull;
}

// The bits of x selected by m (the same in every lane), packed in order from
// bit 0 up: bit order is kept, so packed values compare like the selected
// bits.  unpack1 puts them back (unselected bits 0).
__device__ __forceinline__ uint64_t pack1(uint64_t x, uint64_t m) {
    uint64_t out = 0;
    int dst = 0;
    while (m) {  // runs of adjacent selected bits
        const int s = __builtin_ctzll(m);
        const uint64_t rest = ~(m >> s);
        const int len = rest ? __builtin_ctzll(rest) : 64 - s;
        const uint64_t run = len >= 64 ? ~0ull : (1ull << len) - 1ull;
        out |= ((x >> s) & run) << dst;
        dst += len;
        m &= ~(run << s);
    }
    return out;
}
__device__ __forceinline__ uint64_t unpack1(uint64_t p, uint64_t m) {
    uint64_t out = 0;
    int src = 0;
    while (m) {
        const int s = __builtin_ctzll(m);
        const uint64_t rest = ~(m >> s);
        const int len = rest ? __builtin_ctzll(rest) : 64 - s;
        const uint64_t run = len >= 64 ? ~0ull : (1ull << len) - 1ull;
        out |= ((p >> src) & run) << s;
        src += len;
        m &= ~(run << s);
    }
    return out;
}

// pack1 over every item, in place (one item at a time, so that only one
// packed value is live besides the inputs).
template <int ITEMS>
__device__ __forceinline__ void pack_bits(uint64_t (&x)[ITEMS], uint64_t m) {
    m = uniform64(m);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) x[i] = pack1(x[i], m);
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

}  // namespace husky
