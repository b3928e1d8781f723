// Step 3 of Huskysort on the GPU: re-sort every run of equal codes by the
// full comparator (the role the paper gives to the final Timsort pass,
// Sec. 3.1 Step 3; Sec. 3.3 expects few remaining inversions, so this pass is
// close to linear).
//
// Inside a run all codes are equal, so (given the coder's domain) every
// member agrees on its first min(len, m) elements (m = 9 bytes for ASCII7,
// 8 for the full-byte coder, 4 units for UTF16).  That count is the run's
// "origin" (any value up to 15 through husky_refine, 0 when equal keys imply
// nothing).  The run is ordered by "refinement keys": round r looks at the
// chunk of C elements starting at p = origin + C*r (C = 7 bytes / 3 units)
// and packs it into one 64-bit key
//     [63:60] min(len, origin) -- members shorter than the origin order by length
//     [59: 4] the chunk, big-endian, zero past the string end
//             (bytes: 7 bytes in [59:4]; UTF16: 3 units in [59:12])
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
//   LDS    (<= 8192)            one workgroup per run holding it in LDS for
//                               every round, each round a stable LSD radix
//                               sort of (group, key) over the digits that vary;
//   large                       device-wide: refinement keys for every member
//                               (k_large_keys), a segmented radix sort, and
//                               run detection on the keys for the next round.

#include <algorithm>

#include "common.h"
#include "internal.h"
#include "rank.h"

namespace husky {

template <int CODER>
__device__ __forceinline__ uint64_t chunk_key(const uint8_t* __restrict__ bytes, uint64_t total_bytes,
                                              uint64_t off, uint64_t len, uint32_t round,
                                              uint32_t origin) {
    if (CODER == 0) {
        const uint64_t p = (uint64_t)origin + (uint64_t)byte_chunk * round;
        const uint64_t top = len < (uint64_t)origin ? len : (uint64_t)origin;
        const uint64_t rem = len > p ? len - p : 0;
        const uint64_t clen = rem > (uint64_t)byte_chunk ? (uint64_t)byte_chunk + 1 : rem;
        const uint64_t nb = rem < (uint64_t)byte_chunk ? rem : (uint64_t)byte_chunk;
        uint64_t w = nb ? load8_unaligned(bytes, total_bytes, off + p) : 0ull;
        w &= nb ? ((1ull << (8 * nb)) - 1ull) : 0ull;
        const uint64_t chunk = bswap64(w) >> 8;  // byte p in bits 55..48
        return (top << 60) | (chunk << 4) | clen;
    } else {
        const uint64_t p = (uint64_t)origin + (uint64_t)utf16_chunk * round;
        const uint64_t top = len < (uint64_t)origin ? len : (uint64_t)origin;
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

// First refinement key of every string, in string order: round 0 from `origin`.
template <int CODER>
__global__ __launch_bounds__(BLOCK) void k_first_keys(const uint8_t* __restrict__ bytes,
                                                      const uint64_t* __restrict__ offsets,
                                                      uint32_t n, uint32_t origin,
                                                      uint64_t* __restrict__ key0) {
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        const uint64_t o = offsets[i];
        key0[i] = chunk_key<CODER>(bytes, total_bytes, o, offsets[i + 1] - o, 0u, origin);
    }
}

// ------------------------------------------------------------------ small tier
template <int CODER>
__global__ __launch_bounds__(BLOCK) void k_fix_small(const RunItem* __restrict__ items,
                                                     const uint32_t* __restrict__ count,
                                                     uint32_t cap, const uint8_t* __restrict__ bytes,
                                                     const uint64_t* __restrict__ offsets,
                                                     uint32_t n, uint32_t* __restrict__ idx,
                                                     const uint64_t* __restrict__ key0,
                                                     uint32_t origin, const uint32_t* __restrict__ from) {
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    const uint32_t n_items = min(*count, cap);
    const uint32_t it0 = from ? min(*from, n_items) : 0u;
    const uint32_t lane = lane_id();
    const uint32_t nw = gridDim.x * NWAVES;
    // Software pipelined over the wavefront's runs: the next run's item is
    // loaded while this run's first keys are gathered, and its members'
    // string indices while this run is ranked, so a run costs about one
    // dependent load instead of three.  Runs are disjoint, so reading the
    // next run's indices before this run's are written back is safe.
    uint32_t it = it0 + blockIdx.x * NWAVES + threadIdx.x / WAVE;
    RunItem r{0, 0, 0, 0};
    uint32_t member = 0;
    if (it < n_items) {
        r = items[it];
        if (lane < r.len) member = idx[r.start + lane];
    }
    while (it < n_items) {
        const uint32_t itn = it + nw;
        RunItem rn{0, 0, 0, 0};
        if (itn < n_items) rn = items[itn];
        const uint32_t L = r.len;  // 2..64
        const bool mine = lane < L;
        uint64_t off = 0, len = 0;
        bool have_ol = false;
        uint32_t g = 0, lt = 0;
        bool active = mine;
        uint32_t round = r.round;
        uint32_t member_next = 0;
        for (bool first = true;; first = false) {
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
                    key = chunk_key<CODER>(bytes, total_bytes, off, len, round, origin);
                }
            }
            if (first && lane < rn.len) member_next = idx[rn.start + lane];
            uint32_t first_pos = 0, eq = 0;
            lt = 0;
            for (uint32_t q = 0; q < L; ++q) {
                const uint32_t gq = readlane(g, (int)q);
                const uint64_t kq = readlane64(key, (int)q);
                const bool less = gq < g || (gq == g && kq < key);
                const bool same = gq == g && kq == key;
                first_pos += less ? 1u : 0u;
                eq += same ? 1u : 0u;
                lt += (less || (same && q < lane)) ? 1u : 0u;
            }
            const bool cont = active && key_continues<CODER>(key) && eq > 1;
            g = first_pos;
            active = cont;
            if (!ballot(cont)) break;
            ++round;
        }
        if (mine) idx[r.start + lt] = member;
        r = rn;
        member = member_next;
        it = itn;
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
                                                      uint32_t lmin, uint32_t lmax, uint32_t origin,
                                                      const uint32_t* __restrict__ from) {
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    extern __shared__ __align__(16) uint8_t lds_raw[];
    MediumLds<MAXL>& S = *reinterpret_cast<MediumLds<MAXL>*>(lds_raw);
    const uint32_t n_items = min(*count, cap);
    const uint32_t tid = threadIdx.x;
    for (uint32_t it = (from ? min(*from, n_items) : 0u) + blockIdx.x; it < n_items; it += gridDim.x) {
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
                    S.key[q] = S.act[q] ? chunk_key<CODER>(bytes, total_bytes, S.off[j], S.len[j], round, origin)
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

// ------------------------------------------------------------------ LDS tier
// One size class of the LDS tier (runs of at most NW * 64 * ITEMS), one
// workgroup per run.  Per member: its key and one word
//     sr = slot | group start << 16 | still tied << 31
// (slot: the member's place in the run when the kernel started; group start:
// the position of its group's first member).  Every round computes the keys
// of the tied members (the others carry 0), sorts them by (group start, key)
// with stable digit passes over the digits that vary, and splits groups where
// keys differ or stop continuing.  Members in singleton groups never move, so
// a round with at most one tied member per thread handles only the tied ones:
// they are compacted in position order (the tied positions are exactly the
// union of the tied groups, in group order), each finds its rank inside its
// group by counting, and moves to the tied position of that rank.  The order
// reached is the one the device-wide rounds reach.
template <int CODER, int ITEMS, int NW>
__global__ __launch_bounds__(NW * WAVE) void k_fix_lds(const RunItem* __restrict__ items,
                                                   const uint32_t* __restrict__ count, uint32_t cap,
                                                   const uint8_t* __restrict__ bytes,
                                                   const uint64_t* __restrict__ offsets, uint32_t n,
                                                   uint32_t* __restrict__ idx,
                                                   const uint64_t* __restrict__ key0,
                                                   uint32_t* __restrict__ queue, uint32_t origin,
                                                   const uint32_t* __restrict__ from) {
    constexpr uint32_t NT = NW * WAVE;
    constexpr uint32_t TILE = NT * ITEMS;
    static_assert(TILE <= 32768, "slots and group starts fit 15 bits");
    constexpr uint32_t TIED = 1u << 31;
    __shared__ uint64_t s_k[TILE];
    __shared__ uint32_t s_sr[TILE];
    __shared__ uint64_t s_ck[NT];   // sparse rounds: compacted keys
    __shared__ uint32_t s_csr[NT];  // ... their sr words
    __shared__ uint32_t s_cpos[NT]; // ... and the positions they came from
    __shared__ uint32_t s_whist[NW * 256];
    __shared__ uint32_t s_binstart[256];
    __shared__ uint32_t s_scan[NW];
    __shared__ uint64_t s_or[NW], s_and[NW];
    __shared__ uint32_t s_gor[NW], s_gand[NW], s_wt[NW];
    __shared__ uint32_t s_next;
    uint32_t* s_k32 = reinterpret_cast<uint32_t*>(s_k);  // scratch while keys sit in registers
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    const uint32_t n_items = min(*count, cap);
    const uint32_t it0 = from ? min(*from, n_items) : 0u;
    const uint32_t tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
    auto posof = [&](int i) { return w * WAVE * ITEMS + i * WAVE + lane; };
    auto key_of = [&](uint32_t m, uint32_t round) -> uint64_t {
        if (round == 0 && key0) return key0[m];
        const uint64_t o = offsets[m];
        return chunk_key<CODER>(bytes, total_bytes, o, offsets[m + 1] - o, round, origin);
    };
    // block-wide OR / AND of the keys and group starts each thread passes
    // (o = 0, a = ~0, g = 0, ga = ~0 for none); returns key bits and
    // group-start bits that differ among them
    auto varying = [&](uint64_t o, uint64_t a, uint32_t g, uint32_t ga, uint32_t* gvary,
                       uint64_t* kand) -> uint64_t {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            o |= (uint64_t)__shfl_xor((unsigned long long)o, d, WAVE);
            a &= (uint64_t)__shfl_xor((unsigned long long)a, d, WAVE);
            g |= __shfl_xor(g, d, WAVE);
            ga &= __shfl_xor(ga, d, WAVE);
        }
        if (lane == 0) {
            s_or[w] = o;
            s_and[w] = a;
            s_gor[w] = g;
            s_gand[w] = ga;
        }
        __syncthreads();
        uint64_t oo = 0, aa = ~0ull;
        uint32_t gg = 0, gga = ~0u;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            oo |= s_or[ww];
            aa &= s_and[ww];
            gg |= s_gor[ww];
            gga &= s_gand[ww];
        }
        __syncthreads();
        *gvary = gg ^ gga;
        *kand = aa;
        return oo ^ aa;
    };
    // workgroup b takes run b first, then runs past the grid one at a time
    // through a counter, so that workgroups finishing early take more of them
    for (bool first = true;; first = false) {
        uint32_t it = it0 + blockIdx.x;
        if (!first) {
            if (tid == 0) s_next = it0 + gridDim.x + atomicAdd(queue, 1u);
            __syncthreads();
            it = s_next;
            __syncthreads();
        }
        if (it >= n_items) break;
        const RunItem r = items[it];
        if (r.len < 2 || r.len > TILE) continue;  // never listed so; uniform per workgroup
        const uint32_t nvalid = r.len, start = r.start;
        uint64_t k[ITEMS];
        uint32_t sr[ITEMS], dig[ITEMS], pos[ITEMS], t[ITEMS];
        auto pass = [&]() {
            uint32_t bc;
            rank_digits<8, ITEMS, NW>(dig, nvalid, pos, s_whist, s_binstart, s_scan, &bc);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                s_k[pos[i]] = k[i];
                s_sr[pos[i]] = sr[i];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                k[i] = s_k[posof(i)];
                sr[i] = s_sr[posof(i)];
            }
            __syncthreads();
        };
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) sr[i] = posof(i) | (posof(i) < nvalid ? TIED : 0u);
        for (uint32_t round = r.round;; ++round) {
            // tied members in position order: ranks inside the wavefront,
            // then wavefront bases
            uint32_t crank[ITEMS], wtot = 0;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint64_t b = ballot((sr[i] & TIED) != 0);
                crank[i] = wtot + mbcnt(b);
                wtot += (uint32_t)__popcll(b);
            }
            if (lane == 0) s_wt[w] = wtot;
            __syncthreads();
            uint32_t wbase = 0, ntied = 0;
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t v = s_wt[ww];
                wbase += ww < (int)w ? v : 0u;
                ntied += v;
            }
            __syncthreads();
            if (ntied <= NT) {
                // sparse round: one tied member per thread
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    k[i] = 0;
                    if (sr[i] & TIED) {
                        s_csr[wbase + crank[i]] = sr[i];
                        s_cpos[wbase + crank[i]] = posof(i);
                    }
                }
                __syncthreads();
                // each tied member's place in its group: members with a
                // smaller key, or an equal key at an earlier position
                const bool mine = tid < ntied;
                const uint32_t csr = mine ? s_csr[tid] : 0u;
                const uint64_t ck = mine ? key_of(idx[start + (csr & 0xFFFFu)], round) : 0ull;
                if (mine) s_ck[tid] = ck;
                __syncthreads();
                if (mine) {
                    const uint32_t gs = csr & 0x7FFF0000u;
                    uint32_t g0 = tid;
                    while (g0 > 0 && (s_csr[g0 - 1] & 0x7FFF0000u) == gs) --g0;
                    uint32_t rank = g0;
                    for (uint32_t j = g0; j < ntied && (s_csr[j] & 0x7FFF0000u) == gs; ++j) {
                        const uint64_t kj = s_ck[j];
                        rank += (kj < ck || (kj == ck && j < tid)) ? 1u : 0u;
                    }
                    const uint32_t p = s_cpos[rank];
                    s_k[p] = ck;
                    s_sr[p] = csr;
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < ITEMS; ++i)
                    if (sr[i] & TIED) {
                        k[i] = s_k[posof(i)];
                        sr[i] = s_sr[posof(i)];
                    }
                __syncthreads();
            } else {
                // dense round: string indices first (every load issued before
                // any is used), then the keys
                uint32_t m[ITEMS];
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) m[i] = idx[start + ((sr[i] & TIED) ? (sr[i] & 0xFFFFu) : 0u)];
                if (round == 0 && key0) {
#pragma unroll
                    for (int i = 0; i < ITEMS; ++i) {
                        const uint64_t v = key0[m[i]];
                        k[i] = (sr[i] & TIED) ? v : 0ull;
                    }
                } else {
                    // keys from the string bytes, staged through LDS so that
                    // the loop is not unrolled ITEMS times
#pragma unroll
                    for (int i = 0; i < ITEMS; ++i) s_sr[posof(i)] = (sr[i] & TIED) ? m[i] : ~0u;
                    __syncthreads();
#pragma unroll 2
                    for (int i = 0; i < ITEMS; ++i) {
                        const uint32_t mm = s_sr[posof(i)];
                        s_k[posof(i)] = mm != ~0u ? key_of(mm, round) : 0ull;
                    }
                    __syncthreads();
#pragma unroll
                    for (int i = 0; i < ITEMS; ++i) k[i] = s_k[posof(i)];
                }
                uint64_t o = 0, a = ~0ull;
                uint32_t g = 0;
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    if (sr[i] & TIED) {
                        o |= k[i];
                        a &= k[i];
                    }
                    if (posof(i) < nvalid) g |= sr[i] & ~TIED;
                }
                // the first position's group start is 0: a group-start bit
                // varies where it is set anywhere
                uint32_t gv;
                uint64_t kand;
                const uint64_t vary = uniform64(varying(o, a, g, 0u, &gv, &kand));
                // the varying key bits with the varying group-start bits above
                // them in one word, when that takes fewer 8-bit passes than
                // the byte windows that hold a varying bit (in the 8-wave
                // classes: the 4-wave ones would lose an occupancy level to
                // the extra registers)
                // digits over the bits that vary, in the fewest passes: the
                // tied keys' varying bits, least significant first, then the
                // varying group-start bits above them (the order is by group
                // start, then key).  Each pass's 8-bit digit is read from the
                // unmodified key and group start as up to eight runs of
                // adjacent bits, so no packed copy of the keys is kept.
                const uint32_t gvary = (uint32_t)uniform64((gv >> 16) & 0x7FFFu);
                const int nb = __popcll(vary) + __popc(gvary);
                uint64_t km = vary;
                uint32_t gm = gvary;
                for (int p0 = 0; p0 < nb; p0 += 8) {
                    // this pass's runs: source shift | length << 8 | digit
                    // shift << 16 | from the group start << 24
                    uint32_t rw[8];
                    int nr = 0, dst = 0;
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        rw[r] = 0;
                        if (dst < 8 && (km | gm)) {
                            const bool g = km == 0;
                            const uint64_t m = g ? (uint64_t)gm : km;
                            const int sh = __builtin_ctzll(m);
                            const uint64_t rest = ~(m >> sh);
                            int len = rest ? __builtin_ctzll(rest) : 64 - sh;
                            len = min(len, 8 - dst);
                            const uint64_t bits = ((1ull << len) - 1ull) << sh;
                            if (g)
                                gm &= ~(uint32_t)bits;
                            else
                                km &= ~bits;
                            rw[r] = (uint32_t)sh | (uint32_t)len << 8 | (uint32_t)dst << 16 | (g ? 1u << 24 : 0u);
                            dst += len;
                            nr = r + 1;
                        }
                    }
#pragma unroll
                    for (int i = 0; i < ITEMS; ++i) {
                        const uint32_t gsv = (sr[i] >> 16) & 0x7FFFu;
                        uint32_t d = 0;
#pragma unroll
                        for (int r = 0; r < 8; ++r) {
                            if (r >= nr) break;
                            const uint32_t w = rw[r];
                            const uint32_t sh = w & 63u, len = (w >> 8) & 15u, dd = (w >> 16) & 7u;
                            const uint32_t src = (w >> 24) ? gsv >> sh : (uint32_t)(k[i] >> sh);
                            d |= (src & ((1u << len) - 1u)) << dd;
                        }
                        dig[i] = d;
                    }
                    pass();
                }
            }
            // groups: same group start, same key, and the key continues
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                s_k[posof(i)] = k[i];
                s_sr[posof(i)] = sr[i];
            }
            __syncthreads();
            uint32_t same = 0;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t p = posof(i);
                const bool sm = p > 0 && p < nvalid && (sr[i] & TIED) &&
                                ((s_sr[p - 1] ^ sr[i]) & 0x7FFF0000u) == 0 && s_k[p - 1] == k[i] &&
                                key_continues<CODER>(k[i]);
                same |= (sm ? 1u : 0u) << i;
                t[i] = sm ? 0u : p;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) s_k32[posof(i)] = (same >> i) & 1u;
            __syncthreads();
            bool any = false;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t p = posof(i);
                const bool tied = ((same >> i) & 1u) || (p + 1 < nvalid && s_k32[p + 1]);
                sr[i] = (sr[i] & 0xFFFFu) | (tied ? TIED : 0u);
                any = any || tied;
            }
            if (!__syncthreads_or(any)) break;
            tile_running_max<ITEMS, NW>(t, s_k32, s_scan);
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) sr[i] |= t[i] << 16;
        }
        // indices gathered by slot into LDS before any is overwritten
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (posof(i) < nvalid) s_k32[posof(i)] = idx[start + (sr[i] & 0xFFFFu)];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            if (posof(i) < nvalid) idx[start + posof(i)] = s_k32[posof(i)];
        __syncthreads();  // LDS is reused by the next run
    }
}

// ------------------------------------------------------------------ large tier common prefix
// Every member of a device-wide group is compared with the group's first
// member from the start of the round's chunk (from its length, for members
// shorter than that): the smallest position where a member differs from it
// -- a different element, or one of the two strings ending there -- goes to
// the item (atomic minimum), LCP_NONE staying when every member is the same
// string.  All members agree before that position, so the round's keys can
// start at the chunk holding it instead of walking the chunks they share one
// round at a time.  A comparison stops after LCP_SPAN elements and reports
// where it stopped, which is still a position all of them agree before.
constexpr uint32_t LCP_SPAN = 1024;

template <int CODER, int ITEMS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_large_lcp(RunItem* __restrict__ items,
                                                     const SegDesc* __restrict__ segs,
                                                     const uint32_t* __restrict__ counters,
                                                     const uint8_t* __restrict__ bytes,
                                                     const uint64_t* __restrict__ offsets, uint32_t n,
                                                     const uint32_t* __restrict__ idx,
                                                     const uint64_t* __restrict__ key0, uint32_t origin) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    constexpr uint32_t ES = CODER == 0 ? 1u : 2u;  // bytes per element
    constexpr uint32_t EPW = 8u / ES;              // elements per 8-byte word
    constexpr uint32_t C = CODER == 0 ? byte_chunk : utf16_chunk;
    __shared__ uint32_t s_min[NWAVES];
    const uint64_t total_bytes = offsets[n] * ES;
    HUSKY_UNITS_P(PS, t, counters[C_ALL_TILES]) {
    const uint32_t sidx = find_seg(segs, counters[C_NUM_SEGS], t);
    const SegDesc d = segs[sidx];
    const uint32_t lt = t - d.first_tile;
    const uint32_t base = d.start + lt * TILE;
    const uint32_t nvalid = min(TILE, d.len - lt * TILE);
    const uint32_t round = items[sidx].round;
    const uint64_t p = (uint64_t)origin + (uint64_t)C * round;
    const uint32_t ref = idx[d.start];
    uint32_t m[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t i = k * BLOCK + threadIdx.x;
        m[k] = i < nvalid ? idx[base + i] : ref;
    }
    // In the first round the first refinement keys settle most members with
    // one 8-byte gather: a different key puts the difference inside the
    // first chunk (no chunk to skip), an equal key that does not continue
    // makes the two the same string; only equal keys that continue are
    // compared further, from the end of that chunk.
    uint64_t q = LCP_NONE;
    bool scan[ITEMS];
    uint64_t from = p;
    if (round == 0 && key0) {
        const uint64_t kr = key0[ref];
        uint64_t kk[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) kk[k] = key0[m[k]];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            if (kk[k] != kr) q = p;
            scan[k] = kk[k] == kr && (kk[k] & 0xFull) == (uint64_t)C + 1;
        }
        from = p + C;
    } else {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) scan[k] = true;
    }
    bool any = false;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) any = any || scan[k];
    const uint64_t ro = offsets[ref], rl = offsets[ref + 1] - ro;
    uint64_t o[ITEMS], e[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        o[k] = scan[k] ? offsets[m[k]] : 0ull;
        e[k] = scan[k] ? offsets[m[k] + 1] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        if (!any || !scan[k]) continue;
        const uint64_t len = e[k] - o[k];
        const uint64_t L = len < rl ? len : rl;
        uint64_t pos = from < L ? from : L;
        const uint64_t stop = L - pos > LCP_SPAN ? pos + LCP_SPAN : L;
        uint64_t at = ~0ull;  // none: the same string
        while (pos < stop) {
            const uint64_t cnt = stop - pos < EPW ? stop - pos : EPW;
            uint64_t x = load8_unaligned(bytes, total_bytes, (o[k] + pos) * ES) ^
                         load8_unaligned(bytes, total_bytes, (ro + pos) * ES);
            if (cnt < EPW) x &= (1ull << (cnt * 8 * ES)) - 1ull;
            if (x) {
                at = pos + (uint64_t)__builtin_ctzll(x) / (8 * ES);
                break;
            }
            pos += cnt;
        }
        if (at == ~0ull && (stop < L || len != rl)) at = stop;  // stopped early, or one string ends
        // a position past 32 bits is lowered, which keeps it one all agree before
        if (at != ~0ull) q = min(q, min(at, (uint64_t)LCP_NONE - 1));
    }
    uint32_t qw = (uint32_t)q;
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) qw = min(qw, (uint32_t)__shfl_xor((int)qw, dd, WAVE));
    if (lane_id() == 0) s_min[threadIdx.x / WAVE] = qw;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tq = s_min[0];
        for (int w = 1; w < NWAVES; ++w) tq = min(tq, s_min[w]);
        if (tq != LCP_NONE) atomicMin(&items[sidx].lcp, tq);
    }
    if (PS) __syncthreads();
    }
}

// ------------------------------------------------------------------ large tier keys
// Every segment of a round is longer than one radix tile, so the key tiles
// here are the radix sort's tiles: each tile's OR and AND of its keys (the
// bits that vary, for the digit programs) go to korand[2t], korand[2t + 1].
template <int CODER, int ITEMS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_large_keys(const RunItem* __restrict__ items,
                                                      const SegDesc* __restrict__ segs,
                                                      const uint32_t* __restrict__ counters,
                                                      const uint8_t* __restrict__ bytes,
                                                      const uint64_t* __restrict__ offsets,
                                                      uint32_t n,
                                                      const uint32_t* __restrict__ idx,
                                                      const uint64_t* __restrict__ key0,
                                                      uint64_t* __restrict__ keys, uint32_t origin,
                                                      uint64_t* __restrict__ korand) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_o[NWAVES], s_a[NWAVES];
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    HUSKY_UNITS_P(PS, t, counters[C_ALL_TILES]) {
    const uint32_t sidx = find_seg(segs, counters[C_NUM_SEGS], t);
    const SegDesc d = segs[sidx];
    const RunItem ri = items[sidx];
    const uint32_t lt = t - d.first_tile;
    const uint32_t base = d.start + lt * TILE;
    const uint32_t nvalid = min(TILE, d.len - lt * TILE);
    uint64_t v[ITEMS];
    if (ri.lcp == LCP_NONE) {
        // every member is the same string: one key that does not continue
        // leaves them in index order
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) v[k] = 0;
    } else {
        const uint32_t round = keyed_round(ri, origin, CODER == 0 ? byte_chunk : utf16_chunk);
        // Each level of the gather (index, then first refinement key or
        // string offsets) is issued for all ITEMS members before any is
        // used, so a thread has ITEMS random loads in flight instead of one.
        // Padding slots gather string 0, which exists whenever a tile does.
        uint32_t m[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint32_t i = k * BLOCK + threadIdx.x;
            m[k] = i < nvalid ? idx[base + i] : 0u;
        }
        if (round == 0 && key0) {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) v[k] = key0[m[k]];
        } else {
            uint64_t o[ITEMS], e[ITEMS];
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                o[k] = offsets[m[k]];
                e[k] = offsets[m[k] + 1];
            }
#pragma unroll
            for (int k = 0; k < ITEMS; ++k)
                v[k] = chunk_key<CODER>(bytes, total_bytes, o[k], e[k] - o[k], round, origin);
        }
    }
    uint64_t vo = 0, va = ~0ull;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const uint32_t i = k * BLOCK + threadIdx.x;
        if (i < nvalid) {
            keys[base + i] = v[k];
            vo |= v[k];
            va &= v[k];
        }
    }
    if (korand) {
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1) {
            vo |= (uint64_t)__shfl_xor((unsigned long long)vo, dd, WAVE);
            va &= (uint64_t)__shfl_xor((unsigned long long)va, dd, WAVE);
        }
        if (lane_id() == 0) {
            s_o[threadIdx.x / WAVE] = vo;
            s_a[threadIdx.x / WAVE] = va;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < NWAVES; ++w) {
                vo |= s_o[w];
                va &= s_a[w];
            }
            korand[2 * (size_t)t] = vo;
            korand[2 * (size_t)t + 1] = va;
        }
        if (PS) __syncthreads();
    }
    }
}

// ------------------------------------------------------------------ tail
// Groups still tied after the device-wide rounds a call launched, too long
// for the LDS tier: one workgroup takes a group and runs every remaining
// round itself -- the LDS tier's algorithm with the group in global memory.
// Per round: the refinement keys of the members still tied; a stable LSD
// sort of the group's positions by (group start, key) over the 8-bit digits
// that vary; the new groups (a member starts one where the group start or
// the key changes) and which of them stay tied (two or more members whose key
// continues).  The round count is bounded by the longest member, and nothing
// here waits on another workgroup, so the kernel needs no host decision.
// Buffers over the group's positions [s, s + L): X = (idx, keyA, gsA) and
// Y = (idx_alt, keyB, gsB); gs holds the member's group start relative to s,
// bit 31 set while it is tied (groups of 2^31 members or more are left and
// counted in *unresolved).
constexpr uint32_t TAIL_ACTIVE = 1u << 31;
constexpr int TAIL_ITEMS = 8;
constexpr uint32_t TAIL_TILE = BLOCK * TAIL_ITEMS;

template <int CODER>
__global__ __launch_bounds__(BLOCK) void k_fix_tail(const RunItem* __restrict__ items,
                                                    const uint32_t* __restrict__ count, uint32_t cap,
                                                    const uint8_t* __restrict__ bytes,
                                                    const uint64_t* __restrict__ offsets, uint32_t n,
                                                    uint32_t* idx, uint32_t* idx_alt, uint64_t* keyA,
                                                    uint64_t* keyB, uint32_t* gsA, uint32_t* gsB,
                                                    uint32_t origin, uint32_t* __restrict__ unresolved) {
    __shared__ uint32_t s_whist[NWAVES * 256];
    __shared__ uint32_t s_binstart[256], s_run[256], s_cnt[256];
    __shared__ uint32_t s_scan[NWAVES];
    __shared__ uint32_t s_tmp[TAIL_TILE];
    __shared__ uint64_t s_or[NWAVES], s_and[NWAVES];
    __shared__ uint32_t s_gor[NWAVES], s_gand[NWAVES], s_act[NWAVES];
    __shared__ uint64_t s_prevk;
    __shared__ uint32_t s_prevg;
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    const uint32_t tid = threadIdx.x, w = tid / WAVE, lane = lane_id();
    auto posof = [&](int i) { return w * WAVE * TAIL_ITEMS + i * WAVE + lane; };
    const uint32_t ni = min(*count, cap);
    HUSKY_UNITS(it, ni) {
        const RunItem r = items[it];
        const uint32_t s0 = r.start, L = r.len;
        if (L >= TAIL_ACTIVE) {
            if (tid == 0) atomicAdd(unresolved, 1u);
            continue;
        }
        for (uint32_t p = tid; p < L; p += BLOCK) gsA[s0 + p] = TAIL_ACTIVE;
        __syncthreads();
        bool cur = false;  // false: the group is in X, true: in Y
        for (uint32_t round = r.round;; ++round) {
            uint32_t* ci = cur ? idx_alt : idx;
            uint64_t* ck = cur ? keyB : keyA;
            uint32_t* cg = cur ? gsB : gsA;
            // 1. keys of the tied members; bits of keys and group starts that vary
            uint64_t ko = 0, ka = ~0ull;
            uint32_t go = 0, ga = ~0u;
            for (uint32_t p = tid; p < L; p += BLOCK) {
                const uint32_t g = cg[s0 + p];
                uint64_t k = 0;
                if (g & TAIL_ACTIVE) {
                    const uint32_t m = ci[s0 + p];
                    const uint64_t o = offsets[m];
                    k = chunk_key<CODER>(bytes, total_bytes, o, offsets[m + 1] - o, round, origin);
                }
                ck[s0 + p] = k;
                ko |= k;
                ka &= k;
                go |= g & ~TAIL_ACTIVE;
                ga &= g & ~TAIL_ACTIVE;
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                ko |= (uint64_t)__shfl_xor((unsigned long long)ko, d, WAVE);
                ka &= (uint64_t)__shfl_xor((unsigned long long)ka, d, WAVE);
                go |= (uint32_t)__shfl_xor(go, d, WAVE);
                ga &= (uint32_t)__shfl_xor(ga, d, WAVE);
            }
            if (lane == 0) {
                s_or[w] = ko;
                s_and[w] = ka;
                s_gor[w] = go;
                s_gand[w] = ga;
            }
            __syncthreads();
            uint64_t kv = 0;
            uint32_t gv = 0;
            {
                uint64_t oo = 0, aa = ~0ull;
                uint32_t gg = 0, gn = ~0u;
#pragma unroll
                for (int q = 0; q < NWAVES; ++q) {
                    oo |= s_or[q];
                    aa &= s_and[q];
                    gg |= s_gor[q];
                    gn &= s_gand[q];
                }
                kv = oo ^ aa;
                gv = gg ^ gn;
            }
            __syncthreads();
            // 2. stable LSD passes by (group start, key): key digits first
            for (int dg = 0; dg < 12; ++dg) {
                const uint32_t sh = dg < 8 ? 8u * dg : 8u * (dg - 8);
                const bool on_key = dg < 8;
                if (!(on_key ? ((kv >> sh) & 0xFFull) : ((gv >> sh) & 0xFFu))) continue;
                uint32_t* si = cur ? idx_alt : idx;
                uint64_t* sk = cur ? keyB : keyA;
                uint32_t* sg = cur ? gsB : gsA;
                uint32_t* di = cur ? idx : idx_alt;
                uint64_t* dk = cur ? keyA : keyB;
                uint32_t* dgs = cur ? gsA : gsB;
                auto digit_of = [&](uint64_t k, uint32_t g) {
                    return on_key ? (uint32_t)(k >> sh) & 0xFFu : ((g & ~TAIL_ACTIVE) >> sh) & 0xFFu;
                };
                // digit counts of the whole group, then their starts
                if (tid < 256) s_cnt[tid] = 0;
                __syncthreads();
                for (uint32_t p = tid; p < L; p += BLOCK)
                    atomicAdd(&s_cnt[digit_of(sk[s0 + p], sg[s0 + p])], 1u);
                __syncthreads();
                {
                    uint32_t tot;
                    const uint32_t ex = block_exclusive_sum(tid < 256 ? s_cnt[tid] : 0u, s_scan, &tot);
                    if (tid < 256) s_run[tid] = ex;
                }
                __syncthreads();
                // tiles in order: rank stably inside the tile, place after the
                // digit's earlier tiles
                for (uint32_t t0 = 0; t0 < L; t0 += TAIL_TILE) {
                    const uint32_t nvalid = min(TAIL_TILE, L - t0);
                    uint64_t k[TAIL_ITEMS];
                    uint32_t g[TAIL_ITEMS], v[TAIL_ITEMS], dgt[TAIL_ITEMS], pos[TAIL_ITEMS];
#pragma unroll
                    for (int i = 0; i < TAIL_ITEMS; ++i) {
                        const uint32_t p = posof(i);
                        const bool ok = p < nvalid;
                        k[i] = ok ? sk[s0 + t0 + p] : 0ull;
                        g[i] = ok ? sg[s0 + t0 + p] : 0u;
                        v[i] = ok ? si[s0 + t0 + p] : 0u;
                        dgt[i] = digit_of(k[i], g[i]);
                    }
                    uint32_t bc = 0;
                    rank_digits<8, TAIL_ITEMS>(dgt, nvalid, pos, s_whist, s_binstart, s_scan, &bc);
#pragma unroll
                    for (int i = 0; i < TAIL_ITEMS; ++i) {
                        if (posof(i) < nvalid) {
                            const uint32_t d = dgt[i];
                            const uint32_t o = s0 + s_run[d] + (pos[i] - s_binstart[d]);
                            dk[o] = k[i];
                            dgs[o] = g[i];
                            di[o] = v[i];
                        }
                    }
                    __syncthreads();
                    if (tid < 256) s_run[tid] += bc;
                    __syncthreads();
                }
                cur = !cur;
            }
            // 3. new groups and which stay tied, tile by tile in order (the
            // old key and group start of the position before a tile are kept
            // in LDS; the position after it is still unwritten)
            ci = cur ? idx_alt : idx;
            ck = cur ? keyB : keyA;
            cg = cur ? gsB : gsA;
            uint32_t carry = 0, active = 0;
            for (uint32_t t0 = 0; t0 < L; t0 += TAIL_TILE) {
                const uint32_t nvalid = min(TAIL_TILE, L - t0);
                uint32_t hd[TAIL_ITEMS], nx[TAIL_ITEMS];
                uint64_t kk[TAIL_ITEMS];
#pragma unroll
                for (int i = 0; i < TAIL_ITEMS; ++i) {
                    const uint32_t p = t0 + posof(i);
                    hd[i] = nx[i] = 0;
                    kk[i] = 0;
                    if (posof(i) < nvalid) {
                        const uint64_t k = ck[s0 + p];
                        const uint32_t g = cg[s0 + p] & ~TAIL_ACTIVE;
                        kk[i] = k;
                        uint64_t pk;
                        uint32_t pg;
                        if (p == 0) {
                            pk = ~k;
                            pg = ~g;
                        } else if (posof(i) == 0) {
                            pk = s_prevk;
                            pg = s_prevg;
                        } else {
                            pk = ck[s0 + p - 1];
                            pg = cg[s0 + p - 1] & ~TAIL_ACTIVE;
                        }
                        hd[i] = (p == 0 || pk != k || pg != g) ? 1u : 0u;
                        // does the next position start a group?
                        if (p + 1 >= L) {
                            nx[i] = 1;
                        } else {
                            const uint64_t k2 = ck[s0 + p + 1];
                            const uint32_t g2 = cg[s0 + p + 1] & ~TAIL_ACTIVE;
                            nx[i] = (k2 != k || g2 != g) ? 1u : 0u;
                        }
                    }
                }
                __syncthreads();
                if (tid == 0) {
                    // old values of the tile's last position, for the next tile
                    s_prevk = ck[s0 + t0 + nvalid - 1];
                    s_prevg = cg[s0 + t0 + nvalid - 1] & ~TAIL_ACTIVE;
                }
                uint32_t st[TAIL_ITEMS];
#pragma unroll
                for (int i = 0; i < TAIL_ITEMS; ++i) st[i] = hd[i] ? t0 + posof(i) : 0u;
                tile_running_max<TAIL_ITEMS, NWAVES>(st, s_tmp, s_scan);
                uint32_t act = 0;
#pragma unroll
                for (int i = 0; i < TAIL_ITEMS; ++i) {
                    if (posof(i) < nvalid) {
                        const uint32_t start = max(st[i], carry);
                        const bool single = hd[i] && nx[i];
                        const bool tied = !single && key_continues<CODER>(kk[i]);
                        cg[s0 + t0 + posof(i)] = start | (tied ? TAIL_ACTIVE : 0u);
                        act += tied ? 1u : 0u;
                    }
                }
                // the carry: the group start of the tile's last position
#pragma unroll
                for (int i = 0; i < TAIL_ITEMS; ++i)
                    if (posof(i) == nvalid - 1) s_tmp[0] = max(st[i], carry);
                active += act;
                __syncthreads();
                carry = s_tmp[0];
                __syncthreads();
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) active += __shfl_xor(active, d, WAVE);
            if (lane == 0) s_act[w] = active;
            __syncthreads();
            uint32_t any = 0;
#pragma unroll
            for (int q = 0; q < NWAVES; ++q) any += s_act[q];
            __syncthreads();
            if (!any) break;
        }
        if (cur)
            for (uint32_t p = tid; p < L; p += BLOCK) idx[s0 + p] = idx_alt[s0 + p];
        __syncthreads();
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
                           tl.small_cap, (const uint8_t*)a.elems, a.offsets, a.n, a.idx, a.key0,
                           a.origin, tl.small_first);
    else
        hipLaunchKernelGGL(k_fix_small<1>, dim3(blocks), dim3(BLOCK), 0, s, tl.small, tl.small_count,
                           tl.small_cap, (const uint8_t*)a.elems, a.offsets, a.n, a.idx, a.key0,
                           a.origin, tl.small_first);
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
                       a.idx, a.key0, lmin, lmax, a.origin, tl.medium_first);
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

// The LDS list in four size classes, each a persistent launch walking the
// whole list: a smaller class needs fewer registers and less LDS, so more
// workgroups share a CU.
template <int CODER>
static hipError_t lds_classes(const FixupArgs& a, const TierLists& tl, uint32_t t_medium,
                              hipStream_t s, uint32_t spare_cus) {
    const uint32_t cus = persistent_blocks();
    ProfScope ps(P_FIX_LDS, s);
    hipError_t e = tl.lds_queue_zero ? hipSuccess : zero_u32(tl.lds_queue, 4, s);
    if (e != hipSuccess) return e;
#define HUSKY_FL(I, NW, PER_CU, C)                                                                 \
    static_assert(NW * WAVE * I == lds_class_max(C), "class tile");                                \
    hipLaunchKernelGGL((k_fix_lds<CODER, I, NW>), dim3(cus * PER_CU), dim3(NW * WAVE), 0, s,        \
                       tl.lds[C], tl.lds_count + C, tl.lds_cap[C], (const uint8_t*)a.elems, a.offsets, \
                       a.n, a.idx, a.key0, tl.lds_queue + C, a.origin,                             \
                       tl.lds_first ? tl.lds_first + C : nullptr)
    if (t_medium < lds_class_max(0)) HUSKY_FL(12, 4, 4, 0);
    if (t_medium < lds_class_max(1)) HUSKY_FL(16, 4, 3, 1);
    HUSKY_FL(12, 8, 2, 2);
    // the largest class takes a whole compute unit per workgroup: it leaves
    // `spare_cus` of them to work running beside it on other streams
    const uint32_t cus3 = cus > spare_cus + 8 ? cus - spare_cus : cus;
    hipLaunchKernelGGL((k_fix_lds<CODER, 16, 8>), dim3(cus3), dim3(8 * WAVE), 0, s, tl.lds[3],
                       tl.lds_count + 3, tl.lds_cap[3], (const uint8_t*)a.elems, a.offsets, a.n, a.idx,
                       a.key0, tl.lds_queue + 3, a.origin, tl.lds_first ? tl.lds_first + 3 : nullptr);
    static_assert(8 * WAVE * 16 == lds_class_max(3), "class tile");
#undef HUSKY_FL
    return hipGetLastError();
}

hipError_t fixup_lds(const FixupArgs& a, const TierLists& tl, uint32_t t_medium, hipStream_t s,
                     uint32_t spare_cus) {
    if (!tl.lds_max) return hipSuccess;
    return a.coder == 0 ? lds_classes<0>(a, tl, t_medium, s, spare_cus)
                        : lds_classes<1>(a, tl, t_medium, s, spare_cus);
}

hipError_t fixup_large_keys(const FixupArgs& a, const RunItem* items, const RadixScratch& seg,
                            const RadixConfig& cfg, uint32_t max_tiles, uint64_t* keys,
                            hipStream_t s, bool tile_orand) {
    uint64_t* korand = tile_orand ? seg.korand : nullptr;
    if (!max_tiles) return hipSuccess;
    ProfScope ps(P_LARGE_KEYS, s);
#define HUSKY_LK(C, I)                                                                       \
    if (a.coder == C && cfg.items == I) {                                                    \
        if (seg.grid_cap != ~0u)                                                             \
            hipLaunchKernelGGL((k_large_keys<C, I, true>), dim3(seg.grid(max_tiles)), dim3(BLOCK), 0, s, \
                               items, seg.segs, seg.counters, (const uint8_t*)a.elems, a.offsets,  \
                               a.n, a.idx, a.key0, keys, a.origin, korand);                        \
        else                                                                                 \
            hipLaunchKernelGGL((k_large_keys<C, I, false>), dim3(seg.grid(max_tiles)), dim3(BLOCK), 0, \
                               s, items, seg.segs, seg.counters, (const uint8_t*)a.elems, a.offsets, \
                               a.n, a.idx, a.key0, keys, a.origin, korand);                        \
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

hipError_t fixup_large_lcp(const FixupArgs& a, RunItem* items, const RadixScratch& seg,
                           const RadixConfig& cfg, uint32_t max_tiles, hipStream_t s) {
    if (!max_tiles) return hipSuccess;
    ProfScope ps(P_LARGE_KEYS, s);
#define HUSKY_LCP(C, I)                                                                      \
    if (a.coder == C && cfg.items == I) {                                                    \
        if (seg.grid_cap != ~0u)                                                             \
            hipLaunchKernelGGL((k_large_lcp<C, I, true>), dim3(seg.grid(max_tiles)), dim3(BLOCK), 0, s, \
                               items, seg.segs, seg.counters, (const uint8_t*)a.elems, a.offsets,  \
                               a.n, a.idx, a.key0, a.origin);                                      \
        else                                                                                 \
            hipLaunchKernelGGL((k_large_lcp<C, I, false>), dim3(seg.grid(max_tiles)), dim3(BLOCK), 0, \
                               s, items, seg.segs, seg.counters, (const uint8_t*)a.elems, a.offsets, \
                               a.n, a.idx, a.key0, a.origin);                                      \
        return hipGetLastError();                                                            \
    }
    HUSKY_LCP(0, 16)
    HUSKY_LCP(0, 12)
    HUSKY_LCP(0, 8)
    HUSKY_LCP(1, 16)
    HUSKY_LCP(1, 12)
    HUSKY_LCP(1, 8)
#undef HUSKY_LCP
    return hipErrorInvalidValue;
}

hipError_t fixup_tail(const FixupArgs& a, const RunItem* items, const uint32_t* count, uint32_t cap,
                      uint32_t* idx_alt, uint64_t* keyA, uint64_t* keyB, uint32_t* gs, uint32_t* unresolved,
                      hipStream_t s) {
    const uint32_t blocks = persistent_blocks() * 2;
    ProfScope ps(P_LARGE_KEYS, s);
    if (a.coder == 0)
        hipLaunchKernelGGL(k_fix_tail<0>, dim3(blocks), dim3(BLOCK), 0, s, items, count, cap,
                           (const uint8_t*)a.elems, a.offsets, a.n, a.idx, idx_alt, keyA, keyB, gs, gs + a.n,
                           a.origin, unresolved);
    else
        hipLaunchKernelGGL(k_fix_tail<1>, dim3(blocks), dim3(BLOCK), 0, s, items, count, cap,
                           (const uint8_t*)a.elems, a.offsets, a.n, a.idx, idx_alt, keyA, keyB, gs, gs + a.n,
                           a.origin, unresolved);
    return hipGetLastError();
}

hipError_t fixup_first_keys(const FixupArgs& a, uint64_t* key0, hipStream_t s) {
    if (!a.n) return hipSuccess;
    const uint32_t blocks = std::min<uint32_t>((a.n + BLOCK - 1) / BLOCK, 65536u);
    ProfScope ps(P_LARGE_KEYS, s);
    if (a.coder == 0)
        hipLaunchKernelGGL(k_first_keys<0>, dim3(blocks), dim3(BLOCK), 0, s, (const uint8_t*)a.elems,
                           a.offsets, a.n, a.origin, key0);
    else
        hipLaunchKernelGGL(k_first_keys<1>, dim3(blocks), dim3(BLOCK), 0, s, (const uint8_t*)a.elems,
                           a.offsets, a.n, a.origin, key0);
    return hipGetLastError();
}

}  // namespace husky
