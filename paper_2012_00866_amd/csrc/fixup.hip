// Step 3 of Huskysort on the GPU: re-sort every run of equal codes by the
// full comparator (the role the paper gives to the final Timsort pass,
// Sec. 3.1 Step 3; Sec. 3.3 expects few remaining inversions, so this pass is
// close to linear).
//
// Inside a run all codes are equal, so (given the coder's domain) every
// member agrees on its first min(len, m) elements (m = 9 bytes for ASCII7,
// 4 units for UTF16).  The run is ordered by "refinement keys": round r looks
// at the chunk of C elements starting at p = m + C*r (C = 7 bytes / 3 units)
// and packs it into one 64-bit key
//     [63:60] min(len, m)       -- members shorter than m order by length
//     [59: 4] the chunk, big-endian, zero past the string end
//             (ASCII: 7 bytes in [59:4]; UTF16: 3 units in [59:12])
//     [ 3: 0] elements of the chunk present, or C+1 when the string goes on.
// Comparing these keys is comparing the strings on [p, p + C) with a proper
// prefix first; members tied on a key whose last field is C+1 continue to
// round r+1, members tied otherwise are identical strings and keep index
// order.  Each tier sorts (group, key, position) so ties keep the order the
// stable code sort left them in, i.e. ascending index.
//
// Tiers by run length:
//   small  (<= t_small, <= 64)  one wavefront per run, rank by counting over
//                               the wavefront's lanes;
//   medium (<= t_medium)        one workgroup per run, bitonic sort in LDS;
//   large                       device-wide: refinement keys for every member
//                               (k_large_keys), a segmented radix sort, and
//                               run detection on the keys for the next round.

#include "common.h"
#include "internal.h"

namespace husky {

template <int CODER>
__device__ __forceinline__ uint64_t chunk_key(const uint8_t* __restrict__ bytes, uint64_t total_bytes,
                                              uint64_t off, uint64_t len, uint32_t round) {
    if (CODER == 0) {
        const uint64_t p = (uint64_t)ascii_m + (uint64_t)ascii_chunk * round;
        const uint64_t top = len < (uint64_t)ascii_m ? len : (uint64_t)ascii_m;
        const uint64_t rem = len > p ? len - p : 0;
        const uint64_t clen = rem > (uint64_t)ascii_chunk ? (uint64_t)ascii_chunk + 1 : rem;
        const uint64_t nb = rem < (uint64_t)ascii_chunk ? rem : (uint64_t)ascii_chunk;
        uint64_t w = nb ? load8_unaligned(bytes, total_bytes, off + p) : 0ull;
        w &= nb ? ((1ull << (8 * nb)) - 1ull) : 0ull;
        const uint64_t chunk = bswap64(w) >> 8;  // byte p in bits 55..48
        return (top << 60) | (chunk << 4) | clen;
    } else {
        const uint64_t p = (uint64_t)utf16_m + (uint64_t)utf16_chunk * round;
        const uint64_t top = len < (uint64_t)utf16_m ? len : (uint64_t)utf16_m;
        const uint64_t rem = len > p ? len - p : 0;
        const uint64_t clen = rem > (uint64_t)utf16_chunk ? (uint64_t)utf16_chunk + 1 : rem;
        const uint64_t nu = rem < (uint64_t)utf16_chunk ? rem : (uint64_t)utf16_chunk;
        uint64_t w = nu ? load8_unaligned(bytes, total_bytes, (off + p) * 2) : 0ull;
        w &= nu ? ((1ull << (16 * nu)) - 1ull) : 0ull;
        const uint64_t chunk = ((w & 0xFFFFull) << 32) | (((w >> 16) & 0xFFFFull) << 16) |
                               ((w >> 32) & 0xFFFFull);
        return (top << 60) | (chunk << 12) | clen;
    }
}

// ------------------------------------------------------------------ small tier
template <int CODER>
__global__ __launch_bounds__(BLOCK) void k_fix_small(const RunItem* __restrict__ items,
                                                     const uint32_t* __restrict__ count,
                                                     uint32_t cap, const uint8_t* __restrict__ bytes,
                                                     const uint64_t* __restrict__ offsets,
                                                     uint32_t n, uint32_t* __restrict__ idx,
                                                     const uint64_t* __restrict__ key0) {
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    const uint32_t n_items = min(*count, cap);
    const uint32_t lane = lane_id();
    const uint32_t nw = gridDim.x * NWAVES;
    for (uint32_t it = blockIdx.x * NWAVES + threadIdx.x / WAVE; it < n_items; it += nw) {
        const RunItem r = items[it];
        const uint32_t L = r.len;  // 2..64
        const bool mine = lane < L;
        uint32_t member = 0;
        uint64_t off = 0, len = 0;
        bool have_ol = false;
        if (mine) member = idx[r.start + lane];
        uint32_t g = 0, lt = 0;
        bool active = mine;
        uint32_t round = r.round;
        for (;;) {
            uint64_t key = 0;
            if (active) {
                if (round == 0 && key0) {
                    key = key0[member];
                } else {
                    if (!have_ol) {
                        off = offsets[member];
                        len = offsets[member + 1] - off;
                        have_ol = true;
                    }
                    key = chunk_key<CODER>(bytes, total_bytes, off, len, round);
                }
            }
            uint32_t first = 0, eq = 0;
            lt = 0;
            for (uint32_t q = 0; q < L; ++q) {
                const uint32_t gq = readlane(g, (int)q);
                const uint64_t kq = readlane64(key, (int)q);
                const bool less = gq < g || (gq == g && kq < key);
                const bool same = gq == g && kq == key;
                first += less ? 1u : 0u;
                eq += same ? 1u : 0u;
                lt += (less || (same && q < lane)) ? 1u : 0u;
            }
            const bool cont = active && key_continues<CODER>(key) && eq > 1;
            g = first;
            active = cont;
            if (!ballot(cont)) break;
            ++round;
        }
        if (mine) idx[r.start + lt] = member;
    }
}

// ------------------------------------------------------------------ medium tier
// LDS per run of up to MAXL members: keys, (group << 16 | position),
// member offsets / lengths / indices, scan scratch, continue flags.
template <int MAXL>
struct MediumLds {
    uint64_t key[MAXL];
    uint64_t off[MAXL];
    uint32_t gj[MAXL];
    uint32_t len[MAXL];
    uint32_t mem[MAXL];
    uint32_t tmp[MAXL];
    uint8_t act[MAXL];
    uint32_t scan[NWAVES];
    uint32_t flag;
};

__device__ __forceinline__ bool gjk_less(uint32_t ga, uint64_t ka, uint32_t gb, uint64_t kb) {
    const uint32_t g1 = ga >> 16, g2 = gb >> 16;
    if (g1 != g2) return g1 < g2;
    if (ka != kb) return ka < kb;
    return (ga & 0xFFFFu) < (gb & 0xFFFFu);
}

template <int CODER, int MAXL>
__global__ __launch_bounds__(BLOCK) void k_fix_medium(const RunItem* __restrict__ items,
                                                      const uint32_t* __restrict__ count,
                                                      uint32_t cap, const uint8_t* __restrict__ bytes,
                                                      const uint64_t* __restrict__ offsets,
                                                      uint32_t n, uint32_t* __restrict__ idx,
                                                      const uint64_t* __restrict__ key0,
                                                      uint32_t lmin, uint32_t lmax) {
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    extern __shared__ __align__(16) uint8_t lds_raw[];
    MediumLds<MAXL>& S = *reinterpret_cast<MediumLds<MAXL>*>(lds_raw);
    const uint32_t n_items = min(*count, cap);
    const uint32_t tid = threadIdx.x;
    for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
        const RunItem r = items[it];
        const uint32_t L = r.len;
        if (L <= lmin || L > lmax || L > (uint32_t)MAXL) continue;  // another size class's launch
        uint32_t L2 = 1;
        while (L2 < L) L2 <<= 1;
        for (uint32_t j = tid; j < L2; j += BLOCK) {
            if (j < L) {
                S.mem[j] = idx[r.start + j];
                S.act[j] = 1;
                S.gj[j] = j;  // group 0
            } else {
                S.gj[j] = 0xFFFFFFFFu;
                S.key[j] = ~0ull;
                S.act[j] = 0;
            }
        }
        __syncthreads();
        uint32_t round = r.round;
        bool have_ol = false;
        for (;;) {
            if (round == 0 && key0) {
                for (uint32_t q = tid; q < L; q += BLOCK)
                    S.key[q] = S.act[q] ? key0[S.mem[S.gj[q] & 0xFFFFu]] : 0ull;
            } else {
                if (!have_ol) {  // string offsets and lengths, once a round needs bytes
                    for (uint32_t j = tid; j < L; j += BLOCK) {
                        const uint32_t m = S.mem[j];
                        const uint64_t o = offsets[m];
                        S.off[j] = o;
                        S.len[j] = (uint32_t)(offsets[m + 1] - o);
                    }
                    have_ol = true;
                    __syncthreads();
                }
                for (uint32_t q = tid; q < L; q += BLOCK) {
                    const uint32_t j = S.gj[q] & 0xFFFFu;
                    S.key[q] = S.act[q] ? chunk_key<CODER>(bytes, total_bytes, S.off[j], S.len[j], round)
                                        : 0ull;
                }
            }
            __syncthreads();
            // already in (group, key, position) order -- e.g. a run of
            // identical strings -- needs no sort
            bool unsorted = false;
            for (uint32_t q = tid + 1; q < L; q += BLOCK)
                unsorted = unsorted || gjk_less(S.gj[q], S.key[q], S.gj[q - 1], S.key[q - 1]);
            const bool need_sort = __syncthreads_or(unsorted);
            // bitonic sort of (group, key, position) over L2 slots
            for (uint32_t k = 2; need_sort && k <= L2; k <<= 1) {
                for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
                    for (uint32_t i = tid; i < L2 / 2; i += BLOCK) {
                        const uint32_t lo = 2 * i - (i & (jj - 1));
                        const uint32_t hi = lo + jj;
                        const bool up = (lo & k) == 0;
                        const uint32_t ga = S.gj[lo], gb = S.gj[hi];
                        const uint64_t ka = S.key[lo], kb = S.key[hi];
                        const bool swap = up ? gjk_less(gb, kb, ga, ka) : gjk_less(ga, ka, gb, kb);
                        if (swap) {
                            S.gj[lo] = gb;
                            S.gj[hi] = ga;
                            S.key[lo] = kb;
                            S.key[hi] = ka;
                        }
                    }
                    __syncthreads();
                }
            }
            // heads and continue flags from the sorted (group, key); members
            // that finished earlier carry key 0, which never continues
            bool any = false;
            for (uint32_t q = tid; q < L; q += BLOCK) {
                const uint32_t gq = S.gj[q] >> 16;
                const uint64_t kq = S.key[q];
                const bool same_prev = q > 0 && (S.gj[q - 1] >> 16) == gq && S.key[q - 1] == kq;
                const bool same_next = q + 1 < L && (S.gj[q + 1] >> 16) == gq && S.key[q + 1] == kq;
                S.tmp[q] = same_prev ? 0u : q;
                const bool c = key_continues<CODER>(kq) && (same_prev || same_next);
                S.act[q] = c ? 1 : 0;
                any = any || c;
            }
            if (!__syncthreads_or(any)) break;
            // new group id = position of the group's first member (running max)
            uint32_t carry = 0;
            const uint32_t lane = lane_id();
            for (uint32_t b = 0; b < L; b += BLOCK) {
                const uint32_t q = b + tid;
                uint32_t m = q < L ? S.tmp[q] : 0u;
#pragma unroll
                for (int d = 1; d < WAVE; d <<= 1) {
                    const uint32_t t = __shfl_up(m, d, WAVE);
                    if (lane >= (uint32_t)d) m = max(m, t);
                }
                if (lane == WAVE - 1) S.scan[tid / WAVE] = m;
                __syncthreads();
                uint32_t before = carry, all = carry;
                for (int w = 0; w < NWAVES; ++w) {
                    const uint32_t v = S.scan[w];
                    if (w < (int)(tid / WAVE)) before = max(before, v);
                    all = max(all, v);
                }
                if (q < L) S.gj[q] = (max(before, m) << 16) | (S.gj[q] & 0xFFFFu);
                carry = all;
                __syncthreads();
            }
            ++round;
        }
        // position q holds original member j
        for (uint32_t q = tid; q < L; q += BLOCK) idx[r.start + q] = S.mem[S.gj[q] & 0xFFFFu];
        __syncthreads();
    }
}

// ------------------------------------------------------------------ large tier keys
template <int CODER, int ITEMS>
__global__ __launch_bounds__(BLOCK) void k_large_keys(const RunItem* __restrict__ items,
                                                      const SegDesc* __restrict__ segs,
                                                      const uint32_t* __restrict__ counters,
                                                      const uint8_t* __restrict__ bytes,
                                                      const uint64_t* __restrict__ offsets,
                                                      uint32_t n,
                                                      const uint32_t* __restrict__ idx,
                                                      const uint64_t* __restrict__ key0,
                                                      uint64_t* __restrict__ keys) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    const uint32_t t = blockIdx.x;
    if (t >= counters[C_ALL_TILES]) return;
    const uint32_t sidx = find_seg(segs, counters[C_NUM_SEGS], t);
    const SegDesc d = segs[sidx];
    const uint32_t round = items[sidx].round;
    const uint32_t lt = t - d.first_tile;
    const uint32_t base = d.start + lt * TILE;
    const uint32_t nvalid = min(TILE, d.len - lt * TILE);
    if (round == 0 && key0) {
        for (uint32_t i = threadIdx.x; i < nvalid; i += BLOCK) keys[base + i] = key0[idx[base + i]];
        return;
    }
    for (uint32_t i = threadIdx.x; i < nvalid; i += BLOCK) {
        const uint32_t m = idx[base + i];
        const uint64_t o = offsets[m];
        keys[base + i] = chunk_key<CODER>(bytes, total_bytes, o, offsets[m + 1] - o, round);
    }
}

// ------------------------------------------------------------------ launchers
static uint32_t persistent_blocks() {
    static uint32_t cached = 0;
    if (!cached) {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cus > 0)
            cached = (uint32_t)cus;
        else
            cached = 256;
    }
    return cached;
}

hipError_t fixup_small(const FixupArgs& a, const TierLists& tl, uint32_t, hipStream_t s) {
    const uint32_t blocks = persistent_blocks() * 8;
    ProfScope ps(P_FIX_SMALL, s);
    if (a.coder == 0)
        hipLaunchKernelGGL(k_fix_small<0>, dim3(blocks), dim3(BLOCK), 0, s, tl.small, tl.small_count,
                           tl.small_cap, (const uint8_t*)a.elems, a.offsets, a.n, a.idx, a.key0);
    else
        hipLaunchKernelGGL(k_fix_small<1>, dim3(blocks), dim3(BLOCK), 0, s, tl.small, tl.small_count,
                           tl.small_cap, (const uint8_t*)a.elems, a.offsets, a.n, a.idx, a.key0);
    return hipGetLastError();
}

// One launch per size class of the medium list, each sized for its longest
// run: a class of short runs needs little LDS, so many workgroups share a CU
// and hide the latency of the idx / key / string gathers.
template <int CODER, int MAXL>
static hipError_t medium_impl(const FixupArgs& a, const TierLists& tl, uint32_t lmin,
                              uint32_t lmax, hipStream_t s) {
    const size_t lds = sizeof(MediumLds<MAXL>);
    // set on every launch: cheap on the host, and right for whichever device is current
    hipError_t e = hipFuncSetAttribute((const void*)k_fix_medium<CODER, MAXL>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const uint32_t per_cu = (uint32_t)std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / lds));
    const uint32_t blocks = persistent_blocks() * per_cu;
    ProfScope ps(P_FIX_MEDIUM, s);
    hipLaunchKernelGGL((k_fix_medium<CODER, MAXL>), dim3(blocks), dim3(BLOCK), lds, s, tl.medium,
                       tl.medium_count, tl.medium_cap, (const uint8_t*)a.elems, a.offsets, a.n,
                       a.idx, a.key0, lmin, lmax);
    return hipGetLastError();
}

template <int CODER>
static hipError_t medium_classes(const FixupArgs& a, const TierLists& tl, uint32_t t_medium,
                                 hipStream_t s) {
    hipError_t e = medium_impl<CODER, 256>(a, tl, 0, std::min(t_medium, 256u), s);
    if (e != hipSuccess || t_medium <= 256) return e;
    e = medium_impl<CODER, 1024>(a, tl, 256, std::min(t_medium, 1024u), s);
    if (e != hipSuccess || t_medium <= 1024) return e;
    if (t_medium <= 2048) return medium_impl<CODER, 2048>(a, tl, 1024, t_medium, s);
    return medium_impl<CODER, 4096>(a, tl, 1024, t_medium, s);
}

hipError_t fixup_medium(const FixupArgs& a, const TierLists& tl, uint32_t t_medium,
                        hipStream_t s) {
    return a.coder == 0 ? medium_classes<0>(a, tl, t_medium, s) : medium_classes<1>(a, tl, t_medium, s);
}

hipError_t fixup_large_keys(const FixupArgs& a, const RunItem* items, const RadixScratch& seg,
                            const RadixConfig& cfg, uint32_t max_tiles, uint64_t* keys,
                            hipStream_t s) {
    if (!max_tiles) return hipSuccess;
    ProfScope ps(P_LARGE_KEYS, s);
#define HUSKY_LK(C, I)                                                                       \
    if (a.coder == C && cfg.items == I) {                                                    \
        hipLaunchKernelGGL((k_large_keys<C, I>), dim3(max_tiles), dim3(BLOCK), 0, s, items,  \
                           seg.segs, seg.counters, (const uint8_t*)a.elems, a.offsets, a.n,  \
                           a.idx, a.key0, keys);                                             \
        return hipGetLastError();                                                            \
    }
    HUSKY_LK(0, 16)
    HUSKY_LK(0, 12)
    HUSKY_LK(0, 8)
    HUSKY_LK(1, 16)
    HUSKY_LK(1, 12)
    HUSKY_LK(1, 8)
#undef HUSKY_LK
    return hipErrorInvalidValue;
}

}  // namespace husky
