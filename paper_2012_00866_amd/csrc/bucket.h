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
constexpr int LEARNED_K = 4;  // keys whose bucket lookups one thread of the encode kernel overlaps

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

// The buckets of K keys at once (ok[j] false: no key, out[j] left 0).  The
// steps run side by side over the K keys so that each step's table reads for
// all of them are in flight together.
template <int K>
__device__ __forceinline__ void bucket_of(const BucketArgs& a, const uint64_t (&code)[K],
                                          const bool (&ok)[K], uint64_t lo, uint64_t hi, uint32_t cp,
                                          uint32_t (&out)[K]) {
    uint64_t c[K], ci[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        c[j] = code[j] < lo ? lo : (code[j] > hi ? hi : code[j]);
        ci[j] = ok[j] ? a.cellinfo[window_of(code[j], lo, hi, cp)] : 0ull;
    }
    uint32_t b0[K], kk[K];
    bool heavy[K];
    uint4 h[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        b0[j] = (uint32_t)ci[j] & 0xFFFFu;
        const uint32_t b1 = (uint32_t)(ci[j] >> 16) & 0xFFFFu;
        heavy[j] = ok[j] && b1 >= b0[j] + 2;
        kk[j] = b1 - b0[j];
        h[j] = heavy[j] && (ci[j] >> 63) ? *reinterpret_cast<const uint4*>(a.subtab + SUB_SLOT * b0[j])
                                         : make_uint4(0, 0, 0, 0);
    }
    uint32_t x[K], y[K], v[K], P[K], s[K];
    bool look[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        bool below = false, above = false;
        P[j] = s[j] = 0;
        if (!heavy[j]) {
            // a cell of one bucket
        } else if (ci[j] >> 63) {
            P[j] = h[j].x & 0xFFFFu;
            s[j] = h[j].x >> 16;
            const uint64_t prefix = (uint64_t)h[j].z | ((uint64_t)h[j].w << 32);
            const uint64_t ct = P[j] >= 64 ? c[j] : (P[j] ? c[j] >> (64 - P[j]) : 0ull);
            const uint64_t pt = P[j] >= 64 ? prefix : (P[j] ? prefix >> (64 - P[j]) : 0ull);
            below = ct < pt;
            above = ct > pt;
        } else {
            P[j] = (uint32_t)(ci[j] >> 32) & 127u;
            s[j] = (uint32_t)(ci[j] >> 39) & 31u;
            const uint32_t e = P[j] - cp - 24u;  // prefix bits below the cell, <= 19
            const uint32_t extra = (uint32_t)(ci[j] >> 44) & ((1u << INLINE_PREFIX_BITS) - 1u);
            const uint32_t kx = e ? (uint32_t)((c[j] << (cp + 24)) >> (64 - e)) : 0u;
            below = kx < extra;
            above = kx > extra;
        }
        look[j] = heavy[j] && !below && !above && s[j];
        v[j] = look[j] ? (uint32_t)((c[j] << P[j]) >> (64 - s[j])) : 0u;
        x[j] = below ? 0u : (above ? kk[j] - 1 : 0u);
        y[j] = below ? 0u : (above ? kk[j] - 1 : kk[j] - 1);
        if (!heavy[j]) x[j] = y[j] = 0;
    }
    // the sub-cell's splitter range
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (look[j]) {
            const uint16_t* t = a.subtab + SUB_SLOT * b0[j] + 8;
            const uint32_t tx = t[v[j]];
            const uint32_t ty = v[j] + 1 < (1u << s[j]) ? t[v[j] + 1] : kk[j] - 1;
            x[j] = tx;
            y[j] = ty;
        }
    }
    // splitters[b0 + .] <= c, all K searches advancing together
    for (;;) {
        bool any = false;
        uint32_t mid[K];
        uint64_t sp[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            mid[j] = (x[j] + y[j]) >> 1;
            sp[j] = x[j] < y[j] ? a.splitters[b0[j] + mid[j]] : 0ull;
            any = any || x[j] < y[j];
        }
        if (!any) break;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (x[j] < y[j]) {
                if (sp[j] <= c[j]) x[j] = mid[j] + 1; else y[j] = mid[j];
            }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) out[j] = ok[j] ? b0[j] + (heavy[j] ? x[j] : 0u) : 0u;
}

}  // namespace husky
