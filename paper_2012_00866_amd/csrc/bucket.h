// The learned form's bucket function, evaluated per key: shared by the encode
// kernel (which computes each code's bucket as soon as it has the code) and
// the fit (which builds the tables it reads).
//
// Tables of a fitted model (device memory):
//   cellinfo[W], one u64 per 24-bit cell W:
//     bits  0..15  b0, the cell's first bucket
//     bits 16..31  b1, its end bucket (the cell owns [b0, b1))
//   and, for a heavy cell (b1 >= b0 + 2), whose k = b1 - b0 - 1 splitters
//   share their top P bits:
//     bits 32..38  P
//     bits 39..43  s, the sub-cell bits below P
//     bits 44..62  the e = P - cp - 24 prefix bits right below the cell,
//                  right-aligned (used when e <= 19)
//     bit  63      set when e > 19 or P = 64: P, s and the whole prefix are
//                  then read from the cell's subtab header
//   subtab[16 b0 ..] of a heavy cell: a 16-byte header {u16 P, u16 s, u32 0,
//     u64 prefix}, then 2^s u16 entries, entry v = the cell's splitters below
//     the first code whose s bits below the prefix equal v;
//   splitters[b0 .. b0 + k - 2]: the cell's equal-depth splitters.
// A key of a heavy cell counts the splitters not above it: 0 if its top P
// bits are below the prefix, k - 1 if above, else those below its sub-cell
// plus a search among the sub-cell's own splitters (rarely more than one).
#pragma once

#include "../../include/husky.h"
#include "common.h"

namespace husky {

constexpr uint32_t LUT_CELLS = 1u << 24;
constexpr uint32_t SUB_SLOT = 16;  // sub-cell table entries per bucket
constexpr int INLINE_PREFIX_BITS = 19;

struct BucketArgs {
    const husky_learned_header* hdr;
    const uint64_t* cellinfo;
    const uint64_t* splitters;
    const uint16_t* subtab;
    uint16_t* bid;
};

// The 24-bit cell of a code: clamp to [lo, hi], then the 24 bits right below
// the cp-bit common prefix of lo and hi (never decreases as the code grows).
__device__ __forceinline__ uint32_t window_of(uint64_t code, uint64_t lo, uint64_t hi, uint32_t cp) {
    const uint64_t c = code < lo ? lo : (code > hi ? hi : code);
    return cp >= 64 ? 0u : (uint32_t)((c << cp) >> 40);
}

__device__ __forceinline__ uint32_t bucket_of(const BucketArgs& a, uint64_t code, uint64_t lo,
                                              uint64_t hi, uint32_t cp) {
    const uint64_t ci = a.cellinfo[window_of(code, lo, hi, cp)];
    const uint32_t b0 = (uint32_t)ci & 0xFFFFu, b1 = (uint32_t)(ci >> 16) & 0xFFFFu;
    if (b1 < b0 + 2) return b0;
    const uint64_t c = code < lo ? lo : (code > hi ? hi : code);
    const uint32_t k = b1 - b0;
    uint32_t P, s;
    bool below, above;
    if (ci >> 63) {
        const uint4 h = *reinterpret_cast<const uint4*>(a.subtab + SUB_SLOT * b0);
        P = h.x & 0xFFFFu;
        s = h.x >> 16;
        const uint64_t prefix = (uint64_t)h.z | ((uint64_t)h.w << 32);
        const uint64_t ct = P >= 64 ? c : (P ? c >> (64 - P) : 0ull);
        const uint64_t pt = P >= 64 ? prefix : (P ? prefix >> (64 - P) : 0ull);
        below = ct < pt;
        above = ct > pt;
    } else {
        P = (uint32_t)(ci >> 32) & 127u;
        s = (uint32_t)(ci >> 39) & 31u;
        const uint32_t e = P - cp - 24u;  // prefix bits below the cell, <= 19
        const uint32_t extra = (uint32_t)(ci >> 44) & ((1u << INLINE_PREFIX_BITS) - 1u);
        const uint32_t kx = e ? (uint32_t)((c << (cp + 24)) >> (64 - e)) : 0u;
        below = kx < extra;
        above = kx > extra;
    }
    uint32_t x, y;
    if (below) {
        x = y = 0;
    } else if (above) {
        x = y = k - 1;
    } else if (s) {
        const uint32_t v = (uint32_t)((c << P) >> (64 - s));
        const uint16_t* t = a.subtab + SUB_SLOT * b0 + 8;
        x = t[v];
        y = v + 1 < (1u << s) ? t[v + 1] : k - 1;
    } else {
        x = 0;
        y = k - 1;
    }
    while (x < y) {  // splitters[b0 + .] <= c
        const uint32_t mid = (x + y) >> 1;
        if (a.splitters[b0 + mid] <= c) x = mid + 1; else y = mid;
    }
    return b0 + x;
}

}  // namespace husky
