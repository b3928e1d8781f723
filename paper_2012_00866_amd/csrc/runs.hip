// Runs of equal keys after a sort: the only places where inversions can
// remain when the coder is monotone (Sec. 3.2: x > y never yields a smaller
// code, so after sorting by code every inversion sits among equal codes).
// The paper checks for this globally (its "perfect" flag, Algorithm 3, and
// Sec. 3.4) and then re-sorts everything; here every run of two or more equal
// keys becomes a work item, and only those are re-sorted -- except, for ASCII
// codes carrying the per-string perfect bit (encode.hip), runs whose bit is
// clear: their strings are identical and already in index order.
//
// A run is a maximal range of equal keys inside a segment (runs never cross
// segment boundaries).  Three passes over the tile space of the segments:
//   k_runs_count  -- per tile, the number of run heads (first member of a
//                    run of length >= 2);
//   k_runs_scan   -- exclusive scan of the per-tile counts;
//   k_runs_write  -- ordered compaction: the k-th head and the k-th tail of
//                    the whole array belong to the same run;
// then k_runs_classify turns (head, tail) pairs into work items for the
// wavefront, workgroup or device-wide tier by run length.

#include "common.h"
#include "internal.h"
#include "rank.h"

namespace husky {

template <int CODER>
__device__ __forceinline__ bool continues(uint64_t key) {
    return (key & 0xFull) == (CODER == 0 ? 8ull : 4ull);
}

// Loads one tile's keys (wave-striped: item k of lane l of wave w is tile
// position w*64*ITEMS + k*64 + l; positions >= nvalid are not read) and
// stages them in LDS as s_k[1 + p], with the key before the tile at s_k[0]
// when the segment [s0, s1) has one and the key after it at s_k[nvalid + 1]
// likewise, so that every key is read from HBM once and its neighbours come
// from LDS.  s_k: TILE + 2 words.
template <int ITEMS>
__device__ __forceinline__ void stage_keys(const uint64_t* __restrict__ keys, uint32_t base,
                                           uint32_t nvalid, uint32_t s0, uint32_t s1,
                                           uint64_t* s_k, uint64_t (&k)[ITEMS]) {
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    const bool want_prev = threadIdx.x == 0 && base > s0;
    const bool want_next = threadIdx.x == 1 && base + nvalid < s1;
    uint64_t halo = 0;
    if (want_prev) halo = keys[base - 1];
    if (want_next) halo = keys[base + nvalid];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        k[i] = p < nvalid ? keys[base + p] : 0ull;
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        if (p < nvalid) s_k[1 + p] = k[i];
    }
    if (want_prev) s_k[0] = halo;
    if (want_next) s_k[nvalid + 1] = halo;
    __syncthreads();
}

// How keys are compared: codes with the perfect bit (`perfect`, encode.hip)
// are compared whole and a run is kept only if bit 0 is set (else its strings
// are identical) -- unless the sort left bit 0 out of its digits, when keys
// are compared without it (shift 1) and every run is kept; refinement keys
// are kept if they continue.
struct RunCmp {
    uint32_t shift;
    bool use_bit;
    __device__ static RunCmp make(bool perfect, const uint32_t* __restrict__ counters) {
        const bool off = perfect && counters[C_PERFECT_OFF] != 0;
        return RunCmp{off ? 1u : 0u, perfect && !off};
    }
};

template <int CODER, bool REFINE>
__device__ __forceinline__ bool keep_run(uint64_t kc, RunCmp rc) {
    return REFINE ? continues<CODER>(kc) : (!rc.use_bit || (kc & 1ull));
}

// Flags of tile position p (absolute position base + p inside segment
// [s0, s1), key kc) from the staged keys: multi-run head / tail.
// Also `inner`: kept and equal to the key before it (a run continues
// through p; what the write kernel needs at a tile's first position).
template <int CODER, bool REFINE>
__device__ __forceinline__ void run_flags(const uint64_t* s_k, uint64_t kc, uint32_t p,
                                          uint32_t base, uint32_t s0, uint32_t s1, RunCmp rc,
                                          bool& head, bool& tail, bool& inner) {
    // both neighbours read whatever the position (s_k[p + 2] is in bounds for
    // any p < TILE; a word never staged is masked off), so that the reads of
    // all of a thread's positions go out together
    const uint64_t kp = s_k[p], kn = s_k[p + 2];
    const bool has_prev = base + p > s0, has_next = base + p + 1 < s1;
    const bool eq_prev = has_prev & ((kp >> rc.shift) == (kc >> rc.shift));
    const bool eq_next = has_next & ((kn >> rc.shift) == (kc >> rc.shift));
    const bool keep = keep_run<CODER, REFINE>(kc, rc);
    head = keep && !eq_prev && eq_next;
    tail = keep && eq_prev && !eq_next;
    inner = keep && eq_prev;
}
constexpr uint8_t F_HEAD = 1, F_TAIL = 2, F_INNER = 4;

template <int CODER, bool REFINE, int ITEMS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_runs_count(const uint64_t* __restrict__ keys,
                                                      const SegDesc* __restrict__ segs,
                                                      const uint32_t* __restrict__ counters,
                                                      uint32_t* __restrict__ tile_counts,
                                                      bool perfect, uint8_t* __restrict__ flags) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_k[TILE + 2];
    __shared__ uint32_t s_cnt[NWAVES];
    HUSKY_UNITS_P(PS, t, counters[C_ALL_TILES]) {
    const SegDesc d = segs[find_seg(segs, counters[C_NUM_SEGS], t)];
    const RunCmp rc = RunCmp::make(perfect, counters);
    const uint32_t lt = t - d.first_tile;
    const uint32_t base = d.start + lt * TILE;
    const uint32_t nvalid = min(TILE, d.len - lt * TILE);
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    uint64_t k[ITEMS];
    stage_keys<ITEMS>(keys, base, nvalid, d.start, d.start + d.len, s_k, k);
    uint32_t heads = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        bool h, tl, in;
        run_flags<CODER, REFINE>(s_k, k[i], p, base, d.start, d.start + d.len, rc, h, tl, in);
        h = h && p < nvalid;
        if (flags && p < nvalid) flags[base + p] = (h ? F_HEAD : 0) | (tl ? F_TAIL : 0) | (in ? F_INNER : 0);
        heads += (uint32_t)__popcll(ballot(h));
    }
    if (lane == 0) s_cnt[w] = heads;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int i = 0; i < NWAVES; ++i) tot += s_cnt[i];
        tile_counts[t] = tot;
    }
    if (PS) __syncthreads();
    }
}

// Exclusive scan of tile_counts[0, total) in place (one workgroup); the grand
// total goes to *num_runs.
__global__ __launch_bounds__(BLOCK) void k_runs_scan(uint32_t* __restrict__ tile_counts,
                                                     const uint32_t* __restrict__ counters,
                                                     uint32_t* __restrict__ num_runs) {
    // each thread takes RS consecutive counts per sweep (all loads in
    // flight together), so 2^24 keys (4,098 tiles) need one block scan
    constexpr uint32_t RS = 16;
    __shared__ uint32_t scratch[NWAVES];
    const uint32_t total = counters[C_ALL_TILES];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < total; b += BLOCK * RS) {
        const uint32_t i0 = b + threadIdx.x * RS;
        uint32_t v[RS], sum = 0;
#pragma unroll
        for (uint32_t j = 0; j < RS; ++j) {
            v[j] = i0 + j < total ? tile_counts[i0 + j] : 0u;
            sum += v[j];
        }
        uint32_t tot;
        uint32_t run = carry + block_exclusive_sum(sum, scratch, &tot);
#pragma unroll
        for (uint32_t j = 0; j < RS; ++j) {
            if (i0 + j < total) tile_counts[i0 + j] = run;
            run += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *num_runs = carry;
}

template <int CODER, bool REFINE, int ITEMS, bool PS>
__global__ __launch_bounds__(BLOCK) void k_runs_write(const uint64_t* __restrict__ keys,
                                                      const SegDesc* __restrict__ segs,
                                                      const uint32_t* __restrict__ counters,
                                                      const uint32_t* __restrict__ tile_counts,
                                                      uint32_t* __restrict__ run_start,
                                                      uint32_t* __restrict__ run_end,
                                                      uint32_t* __restrict__ run_seg,
                                                      bool perfect, const uint8_t* __restrict__ flags) {
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint64_t s_k[TILE + 2];
    __shared__ uint32_t s_h[NWAVES], s_t[NWAVES];
    HUSKY_UNITS_P(PS, t, counters[C_ALL_TILES]) {
    const uint32_t sidx = find_seg(segs, counters[C_NUM_SEGS], t);
    const SegDesc d = segs[sidx];
    const RunCmp rc = RunCmp::make(perfect, counters);
    const uint32_t lt = t - d.first_tile;
    const uint32_t base = d.start + lt * TILE;
    const uint32_t nvalid = min(TILE, d.len - lt * TILE);
    const uint32_t w = threadIdx.x / WAVE, lane = lane_id();
    bool hf[ITEMS], tf[ITEMS];
    uint32_t nh = 0, nt = 0;
    bool open = false;  // a run open at the tile start had its head in an earlier tile
    if (flags) {
        // the count kernel's flags: one byte per key instead of the keys
        uint8_t f[ITEMS];
        load_tile<ITEMS>(flags + base, nvalid, f);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            hf[i] = (f[i] & F_HEAD) != 0;
            tf[i] = (f[i] & F_TAIL) != 0;
            nh += (uint32_t)__popcll(ballot(hf[i]));
            nt += (uint32_t)__popcll(ballot(tf[i]));
        }
        open = base > d.start && (flags[base] & F_INNER) != 0;
    } else {
        uint64_t k[ITEMS];
        stage_keys<ITEMS>(keys, base, nvalid, d.start, d.start + d.len, s_k, k);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
            hf[i] = tf[i] = false;
            bool in = false;
            if (p < nvalid)
                run_flags<CODER, REFINE>(s_k, k[i], p, base, d.start, d.start + d.len, rc, hf[i], tf[i], in);
            nh += (uint32_t)__popcll(ballot(hf[i]));
            nt += (uint32_t)__popcll(ballot(tf[i]));
        }
        if (base > d.start) {
            const uint64_t kc = s_k[1];
            open = (s_k[0] >> rc.shift) == (kc >> rc.shift) && keep_run<CODER, REFINE>(kc, rc);
        }
    }
    if (lane == 0) {
        s_h[w] = nh;
        s_t[w] = nt;
    }
    __syncthreads();
    uint32_t hb = tile_counts[t], tb = hb - (open ? 1u : 0u);
    for (uint32_t i = 0; i < w; ++i) {
        hb += s_h[i];
        tb += s_t[i];
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint64_t bh = ballot(hf[i]), bt = ballot(tf[i]);
        const uint32_t p = w * WAVE * ITEMS + i * WAVE + lane;
        if (hf[i]) {
            const uint32_t o = hb + mbcnt(bh);
            run_start[o] = base + p;
            run_seg[o] = sidx;
        }
        if (tf[i]) run_end[tb + mbcnt(bt)] = base + p;
        hb += (uint32_t)__popcll(bh);
        tb += (uint32_t)__popcll(bt);
    }
    if (PS) __syncthreads();
    }
}

// Work items for the three tiers.  Each workgroup takes a contiguous share
// of the run table, counts its items per tier (one LDS atomic per wavefront
// and tier), reserves its slots with one device atomic per tier, and writes
// them; the order inside a list does not matter.  For the device-wide list it
// also adds up what the host needs to size that tier's launches: the number
// of items longer than one radix tile and the tiles they span.
// List of a run: 0 wavefront, 1 workgroup, 2 device-wide, 3 + c LDS tier
// size class c.
__device__ __forceinline__ int list_of(uint32_t len, uint32_t t_small, uint32_t t_medium,
                                       uint32_t lds_max) {
    return len <= t_small ? 0 : (len <= t_medium ? 1 : (len <= lds_max ? 3 + lds_class_of(len) : 2));
}

__global__ __launch_bounds__(BLOCK) void k_runs_classify(
    const uint32_t* __restrict__ run_start, const uint32_t* __restrict__ run_end,
    const uint32_t* __restrict__ run_seg, const uint32_t* __restrict__ num_runs,
    const RunItem* __restrict__ items, TierLists tl, uint32_t t_small, uint32_t t_medium,
    uint32_t tile, uint32_t origin, uint32_t chunk, uint32_t* __restrict__ runs_seen) {
    constexpr int NL = 7;  // lists
    // s_n: items per list, then the device-wide list's items longer than one
    // tile, their tiles and the tiles of all its items
    __shared__ uint32_t s_n[NL + 3], s_base[NL], s_fill[NL];
    const uint32_t nr = *num_runs;
    const uint32_t per = ((nr + gridDim.x - 1) / gridDim.x + BLOCK - 1) / BLOCK * BLOCK;
    const uint32_t r0 = blockIdx.x * per, r1 = min(nr, r0 + per);
    if (threadIdx.x < NL + 3) s_n[threadIdx.x] = 0;
    if (threadIdx.x < NL) s_fill[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t lane = lane_id();
    // pass 1: counts
    for (uint32_t r = r0 + threadIdx.x; r < r0 + per; r += BLOCK) {
        const bool ok = r < r1;
        uint32_t len = 0;
        if (ok) len = run_end[r] - run_start[r] + 1;
        const int li = ok ? list_of(len, t_small, t_medium, tl.lds_max) : -1;
        const uint32_t big = (li == 2 && len > tile) ? 1u : 0u;
        uint32_t bt = big ? (len + tile - 1) / tile : 0u;
        uint32_t at = li == 2 ? (len + tile - 1) / tile : 0u;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            bt += __shfl_xor(bt, d, WAVE);
            at += __shfl_xor(at, d, WAVE);
        }
        if (lane == 0) {
            if (bt) atomicAdd(&s_n[NL + 1], bt);
            if (at) atomicAdd(&s_n[NL + 2], at);
        }
        const uint32_t nbig = (uint32_t)__popcll(ballot(big != 0));
        if (lane == 0 && nbig) atomicAdd(&s_n[NL], nbig);
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const uint32_t c = (uint32_t)__popcll(ballot(li == q));
            if (lane == 0 && c) atomicAdd(&s_n[q], c);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_base[0] = s_n[0] ? atomicAdd(tl.small_count, s_n[0]) : 0u;
        s_base[1] = s_n[1] ? atomicAdd(tl.medium_count, s_n[1]) : 0u;
        s_base[2] = s_n[2] ? atomicAdd(tl.large_count, s_n[2]) : 0u;
        if (s_n[NL]) atomicAdd(tl.large_count + 1, s_n[NL]);
        if (s_n[NL + 1]) atomicAdd(tl.large_count + 2, s_n[NL + 1]);
        if (s_n[NL + 2]) atomicAdd(tl.large_count + 3, s_n[NL + 2]);
        for (int c = 0; c < 4; ++c) s_base[3 + c] = s_n[3 + c] ? atomicAdd(tl.lds_count + c, s_n[3 + c]) : 0u;
    }
    __syncthreads();
    // pass 2: items
    for (uint32_t r = r0 + threadIdx.x; r < r0 + per; r += BLOCK) {
        const bool ok = r < r1;
        RunItem it{0, 0, 0, LCP_NONE};
        int li = -1;
        if (ok) {
            it.start = run_start[r];
            it.len = run_end[r] - it.start + 1;
            it.round = items ? keyed_round(items[run_seg[r]], origin, chunk) + 1 : 0;
            li = list_of(it.len, t_small, t_medium, tl.lds_max);
        }
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const uint64_t m = ballot(li == q);
            if (!m) continue;
            const uint32_t leader = (uint32_t)__ffsll((unsigned long long)m) - 1u;
            uint32_t o = 0;
            if (lane == leader) o = atomicAdd(&s_fill[q], (uint32_t)__popcll(m));
            o = readlane(o, (int)leader) + mbcnt(m) + s_base[q];
            if (li == q) {
                RunItem* list = q == 0 ? tl.small : (q == 1 ? tl.medium : (q == 2 ? tl.large : tl.lds[q - 3]));
                const uint32_t cap =
                    q == 0 ? tl.small_cap : (q == 1 ? tl.medium_cap : (q == 2 ? tl.large_cap : tl.lds_cap[q - 3]));
                if (o < cap) list[o] = it;
            }
        }
    }
    if (runs_seen && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(runs_seen, nr);
}

template <int CODER, bool REFINE, int ITEMS, bool PS>
static hipError_t find_runs_impl(const uint64_t* keys, const RadixScratch& seg,
                                 uint32_t max_tiles, const RunItem* items, const RunScratch& rs,
                                 const TierLists& tl, uint32_t t_small, uint32_t t_medium,
                                 uint32_t origin, hipStream_t s, bool perfect) {
    if (max_tiles == 0) return hipSuccess;
    uint32_t* num_runs = rs.counters + 0;
    ProfScope ps(P_RUNS, s);
    hipLaunchKernelGGL((k_runs_count<CODER, REFINE, ITEMS, PS>), dim3(seg.grid(max_tiles)), dim3(BLOCK), 0, s,
                       keys, seg.segs, seg.counters, rs.tile_counts, perfect, rs.flags);
    hipLaunchKernelGGL(k_runs_scan, dim3(1), dim3(BLOCK), 0, s, rs.tile_counts, seg.counters,
                       num_runs);
    hipLaunchKernelGGL((k_runs_write<CODER, REFINE, ITEMS, PS>), dim3(seg.grid(max_tiles)), dim3(BLOCK), 0, s,
                       keys, seg.segs, seg.counters, rs.tile_counts, rs.run_start, rs.run_end,
                       rs.run_start + rs.run_cap, perfect, (const uint8_t*)rs.flags);
    const uint32_t blocks = 96;
    hipLaunchKernelGGL(k_runs_classify, dim3(blocks), dim3(BLOCK), 0, s, rs.run_start, rs.run_end,
                       rs.run_start + rs.run_cap, num_runs, items, tl,
                       t_small, t_medium, (uint32_t)(BLOCK * ITEMS), origin,
                       CODER == 0 ? byte_chunk : utf16_chunk, REFINE ? nullptr : rs.runs_seen);
    return hipGetLastError();
}

hipError_t find_runs(const uint64_t* keys, const RadixScratch& seg, const RadixConfig& cfg,
                     uint32_t max_tiles, int coder, bool refinement, const RunItem* items,
                     const RunScratch& rs, const TierLists& tl, uint32_t t_small,
                     uint32_t t_medium, uint32_t origin, hipStream_t s, bool perfect_codes) {
#define HUSKY_RUNS_CASE(C, R, I)                                                               \
    if (coder == C && refinement == R && cfg.items == I)                                       \
        return seg.grid_cap != ~0u                                                               \
                   ? find_runs_impl<C, R, I, true>(keys, seg, max_tiles, items, rs, tl, t_small,      \
                                                   t_medium, origin, s, perfect_codes && !R)                  \
                   : find_runs_impl<C, R, I, false>(keys, seg, max_tiles, items, rs, tl, t_small,     \
                                                    t_medium, origin, s, perfect_codes && !R);
    HUSKY_RUNS_CASE(0, false, 16)
    HUSKY_RUNS_CASE(0, true, 16)
    HUSKY_RUNS_CASE(1, false, 16)
    HUSKY_RUNS_CASE(1, true, 16)
    HUSKY_RUNS_CASE(0, false, 12)
    HUSKY_RUNS_CASE(0, true, 12)
    HUSKY_RUNS_CASE(1, false, 12)
    HUSKY_RUNS_CASE(1, true, 12)
    HUSKY_RUNS_CASE(0, false, 8)
    HUSKY_RUNS_CASE(0, true, 8)
    HUSKY_RUNS_CASE(1, false, 8)
    HUSKY_RUNS_CASE(1, true, 8)
#undef HUSKY_RUNS_CASE
    return hipErrorInvalidValue;
}

}  // namespace husky
