// Device-side helpers shared by the Huskysort HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace husky {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;  // threads of every tiled kernel (4 wavefronts)
constexpr int NWAVES = BLOCK / WAVE;
constexpr int MAX_PASSES = 11;  // 64-bit keys with 6-bit digits

// Segment descriptor: a contiguous range of positions sorted on its own.
struct SegDesc {
    uint32_t start;       // first position
    uint32_t len;         // positions in the segment
    uint32_t first_tile;  // global index of its first tile
    uint32_t aux;         // all segments: row in the big list or NOT_BIG;
                          // big list: mask of the digit passes it runs
};
constexpr uint32_t NOT_BIG = 0xFFFFFFFFu;

// A segment that spans two or more radix tiles.
struct BigDesc {
    uint32_t start, len;
    uint32_t first_tile;   // first tile in the multi-tile tile space
    uint32_t exec;         // mask of the digit passes it runs
    uint32_t first_group;  // first scan group (GROUP_TILES tiles each)
    uint32_t ntiles, ngroups, pad;
};
constexpr int GROUP_TILES = 64;

// Slots of the segment-sort counter block (device uint32[64]).
enum : uint32_t {
    C_TILE0 = 0,       // [MAX_PASSES] dynamic tile ids, one per digit pass
    C_ALL_TILES = 16,  // tiles over every segment (run detection / key tile space)
    C_BIG_TILES = 17,  // tiles over multi-tile segments (onesweep tile space)
    C_NUM_BIG = 18,    // number of multi-tile segments
    C_NUM_SEGS = 19,   // number of segments
    C_NUM_GROUPS = 20, // scan groups over the multi-tile segments
    C_EXEC_UNION = 21, // OR of the pass masks of all multi-tile segments
    C_VARY_LO = 22,    // OR of the varying bits of all multi-tile segments,
    C_VARY_HI = 23,    //   low and high words
    C_EXEC_DONE = 24,  // big segments whose varying bits are known
    C_PERFECT_OFF = 25,// 1 when the multi-tile passes leave out key bit 0
                       // (the perfect bit of ASCII codes) because it would
                       // cost a digit pass; run detection then ignores it
};

// Digit programs of the multi-tile passes: the bits that vary in any
// multi-tile segment, packed from the least significant up, form the digits
// (pass p takes packed bits [p * BITS, p * BITS + BITS)).  Per pass PROG_WORDS
// words: the number of runs, then one word per run of key bits that are
// adjacent both in the key and in the digit: source shift | length << 8 |
// destination shift << 16.
constexpr int PROG_WORDS = 9;

// Largest s < ns with segs[s].first_tile <= tile (segments in tile order).
__device__ __forceinline__ uint32_t find_seg(const SegDesc* segs, uint32_t ns, uint32_t tile) {
    uint32_t lo = 0, hi = ns;  // invariant: answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (segs[mid].first_tile <= tile)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Entry of a fix-up work list: `len` members starting at `start`, to be
// compared from refinement round `round` on.
struct RunItem {
    uint32_t start;
    uint32_t len;
    uint32_t round;
    // Device-wide tier: a position (in elements) before which every member
    // equals the group's first member, found by its common-prefix pass
    // (LCP_NONE, the value items are created with, after that pass: every
    // member is the same string).
    uint32_t lcp;
};
constexpr uint32_t LCP_NONE = ~0u;

// The round a device-wide group is keyed in: its own, or the later round
// whose chunk holds the position its members first differ at (every chunk
// before that one is the same in all of them).
__device__ __forceinline__ uint32_t keyed_round(const RunItem& r, uint32_t origin, uint32_t chunk) {
    if (r.lcp == LCP_NONE || r.lcp < origin) return r.round;
    const uint32_t j = (r.lcp - origin) / chunk;
    return j > r.round ? j : r.round;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of m in lanes strictly below this lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
    uint32_t lo = readlane((uint32_t)v, lane), hi = readlane((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        uint32_t t = __shfl_up(v, d, WAVE);
        if (lane >= (uint32_t)d) v += t;
    }
    return v;
}

// Workgroups of a launch are dispatched to the 8 XCDs round-robin (block b
// on XCD b % 8), each XCD behind its own L2.  xcd_remap(b, G) hands each XCD a
// contiguous range of the G tiles instead, so that neighbouring tiles -- whose
// scattered writes share cache lines -- complete their lines in one L2.  It is
// a bijection of [0, G), so it only changes which workgroup runs which tile.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t G) {
    constexpr uint32_t X = 8;
    const uint32_t q = G / X, r = G % X, x = b % X, i = b / X;
    return x * q + (x < r ? x : r) + i;
}

// Work units of a kernel whose grid comes from a host bound: units u =
// blockIdx.x, blockIdx.x + gridDim.x, ... below the device-side `count`.  A
// grid of at least `count` workgroups runs each unit in its own workgroup; a
// capped grid (a multiple of 8, so every unit stays on its workgroup's XCD
// in xcd_remap) walks several.  The body ends with a barrier when it uses
// LDS, so the next unit may reuse it; units skipped with `continue` are
// skipped by the whole workgroup.
// HUSKY_UNITS_P(PS, ...) walks only when PS (a compile-time flag) is set;
// otherwise a workgroup runs the one unit of its own index, as straight-line
// code (grids launched with a unit per workgroup).
#define HUSKY_UNITS_P(PS, u, count) \
    for (uint32_t u = blockIdx.x, u##_end = (count); u < u##_end; u = (PS) ? u + gridDim.x : u##_end)
#define HUSKY_UNITS(u, count) HUSKY_UNITS_P(true, u, count)

// Exclusive prefix sum over the NW * 64 threads of a workgroup.// Exclusive prefix sum over the NW * 64 threads of a workgroup.  `scratch`
// holds NW words of LDS.  Returns the exclusive prefix; *total gets the block
// total.  Every thread of the block must call it.
template <int NW = NWAVES>
__device__ __forceinline__ uint32_t block_exclusive_sum(uint32_t v, uint32_t* scratch,
                                                        uint32_t* total) {
    const uint32_t lane = lane_id(), wid = threadIdx.x / WAVE;
    uint32_t inc = wave_inclusive_sum(v);
    if (lane == WAVE - 1) scratch[wid] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        uint32_t s = scratch[w];
        before += (w < (int)wid) ? s : 0u;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// Coherent (device-scope) 64-bit loads and stores for cross-workgroup flags.
__device__ __forceinline__ uint64_t load_agent(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bytes [addr, addr + 8) of a byte buffer of `total` bytes, little-endian in
// the returned word, bytes past `total` read as zero.  Two aligned 8-byte
// loads when they stay inside the buffer, byte loads otherwise.
__device__ __forceinline__ uint64_t load8_unaligned(const uint8_t* buf, uint64_t total,
                                                    uint64_t addr) {
    const uint64_t base = addr & ~7ull;
    const uint32_t sh = (uint32_t)(addr & 7ull) * 8u;
    if (base + 16 <= total) {
        const uint64_t* w = (const uint64_t*)(buf + base);
        uint64_t w0 = w[0], w1 = w[1];
        return sh ? ((w0 >> sh) | (w1 << (64 - sh))) : w0;
    }
    uint64_t r = 0;
    for (int k = 0; k < 8; ++k) {
        uint64_t a = addr + k;
        if (a < total) r |= (uint64_t)buf[a] << (8 * k);
    }
    return r;
}

// Byte-reverse of a 64-bit word.
__device__ __forceinline__ uint64_t bswap64(uint64_t x) { return __builtin_bswap64(x); }

}  // namespace husky
