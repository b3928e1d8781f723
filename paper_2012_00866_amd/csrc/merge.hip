// Step 3 as the paper writes it: a full stable pass over the whole array
// (Sec. 3.1 Step 3, the final Timsort), needed when the coder may invert two
// objects -- a lossy coder (Sec. 3.2: x > y with code(x) <= code(y) with
// probability p) or the Appendix's deliberate mis-coding.  Run-local fix-up
// cannot repair an inversion between different codes; this pass can, and it
// costs little when the array is nearly sorted.
//
// It is a natural merge sort, the idea Timsort is built on: the array is cut
// into its maximal ascending runs (positions where an element is smaller
// than the one before start a run), then runs are merged in pairs, level by
// level, until one is left -- ceil(log2 R) levels for R runs.  A merge places
// every element directly: an element at offset i of run A goes to A's start
// + i + (elements of its partner run B smaller than it), found by binary
// search, and likewise for B -- no element waits for another.
//
// Elements are compared by (string, original index), a total order, so the
// result is the unique stable sorting permutation whatever order the pass
// receives.  Each element carries its first 8 bytes (4 UTF-16 units) as a
// big-endian prefix key, which decides most comparisons without reading the
// strings; equal prefixes continue in the strings, 8 bytes (4 units) at a
// time.
//
// The number of levels is fixed from n on the host; the run count and the
// buffer holding the current order live on the device, and a level with a
// single run left does nothing, so the pass never synchronizes.

#include <algorithm>

#include "common.h"
#include "internal.h"

namespace husky {

namespace {

// Elements of `len` from element `p` of a string at element offset `off`, at
// most one chunk (8 bytes or 4 units), as a big-endian word with the first
// element highest and zeros past the chunk's end.
template <int EK>
__device__ __forceinline__ uint64_t be_chunk(const uint8_t* __restrict__ bytes, uint64_t total_bytes,
                                             uint64_t off, uint64_t p, uint64_t m) {
    if (EK == 0) {
        if (!m) return 0ull;
        uint64_t w = load8_unaligned(bytes, total_bytes, off + p);
        w &= m >= 8 ? ~0ull : ((1ull << (8 * m)) - 1ull);
        return bswap64(w);
    } else {
        if (!m) return 0ull;
        uint64_t w = load8_unaligned(bytes, total_bytes, (off + p) * 2);
        w &= m >= 4 ? ~0ull : ((1ull << (16 * m)) - 1ull);
        return ((w & 0xFFFFull) << 48) | (((w >> 16) & 0xFFFFull) << 32) | (((w >> 32) & 0xFFFFull) << 16) |
               (w >> 48);
    }
}

template <int EK>
constexpr uint64_t chunk_elems() { return EK == 0 ? 8 : 4; }

// string a (prefix key ka) before string b (prefix key kb) in the order
// (string, index)
template <int EK>
__device__ __forceinline__ bool before(const uint8_t* __restrict__ bytes, uint64_t total_bytes,
                                       const uint64_t* __restrict__ offsets, uint32_t a, uint64_t ka,
                                       uint32_t b, uint64_t kb) {
    if (ka != kb) return ka < kb;
    const uint64_t oa = offsets[a], la = offsets[a + 1] - oa;
    const uint64_t ob = offsets[b], lb = offsets[b + 1] - ob;
    const uint64_t lmin = la < lb ? la : lb;
    constexpr uint64_t C = chunk_elems<EK>();
    for (uint64_t p = C; p < lmin; p += C) {
        const uint64_t m = lmin - p < C ? lmin - p : C;
        const uint64_t wa = be_chunk<EK>(bytes, total_bytes, oa, p, m);
        const uint64_t wb = be_chunk<EK>(bytes, total_bytes, ob, p, m);
        if (wa != wb) return wa < wb;
    }
    if (la != lb) return la < lb;
    return a < b;
}

struct MergeState {
    uint32_t runs;  // runs in the current order
    uint32_t cur;   // 0: the order is in (idx, key A), 1: in (idx B, key B)
};

// Prefix key of every position; an index outside [0, n) (not a permutation:
// the result is then unspecified) is clamped so that no string read leaves
// the buffers.
template <int EK>
__global__ __launch_bounds__(BLOCK) void k_prefix_keys(const uint8_t* __restrict__ bytes,
                                                       const uint64_t* __restrict__ offsets, uint32_t n,
                                                       uint32_t* __restrict__ idx,
                                                       uint64_t* __restrict__ key) {
    const uint64_t total_bytes = offsets[n] * (EK == 0 ? 1u : 2u);
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < n; k += gridDim.x * BLOCK) {
        uint32_t i = idx[k];
        if (i >= n) {
            i = n - 1;
            idx[k] = i;
        }
        const uint64_t o = offsets[i], L = offsets[i + 1] - o;
        const uint64_t C = chunk_elems<EK>();
        key[k] = be_chunk<EK>(bytes, total_bytes, o, 0, L < C ? L : C);
    }
}

// flag[k] = 1 where a run starts: k = 0, or element k before element k - 1
template <int EK>
__global__ __launch_bounds__(BLOCK) void k_run_heads(const uint8_t* __restrict__ bytes,
                                                     const uint64_t* __restrict__ offsets, uint32_t n,
                                                     const uint32_t* __restrict__ idx,
                                                     const uint64_t* __restrict__ key,
                                                     uint32_t* __restrict__ flag) {
    const uint64_t total_bytes = offsets[n] * (EK == 0 ? 1u : 2u);
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < n; k += gridDim.x * BLOCK)
        flag[k] = k == 0 ? 1u
                         : (before<EK>(bytes, total_bytes, offsets, idx[k], key[k], idx[k - 1], key[k - 1]) ? 1u
                                                                                                         : 0u);
}

// ---- ordered compaction of the run heads: tile counts, their scan, placement
constexpr uint32_t CT_ITEMS = 8;
constexpr uint32_t CT_TILE = BLOCK * CT_ITEMS;

__global__ __launch_bounds__(BLOCK) void k_head_tiles(const uint32_t* __restrict__ flag, uint32_t n,
                                                      uint32_t* __restrict__ tile_cnt) {
    __shared__ uint32_t s_w[NWAVES];
    const uint32_t base = blockIdx.x * CT_TILE + threadIdx.x * CT_ITEMS;
    uint32_t c = 0;
#pragma unroll
    for (uint32_t q = 0; q < CT_ITEMS; ++q) c += base + q < n ? flag[base + q] : 0u;
    uint32_t total;
    block_exclusive_sum(c, s_w, &total);
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = total;
}

__global__ __launch_bounds__(BLOCK) void k_head_scan(uint32_t* __restrict__ tile_cnt, uint32_t tiles,
                                                     MergeState* __restrict__ st) {
    __shared__ uint32_t s_w[NWAVES];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < tiles; b += BLOCK) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t v = i < tiles ? tile_cnt[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_sum(v, s_w, &total);
        if (i < tiles) tile_cnt[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) {
        st->runs = carry;
        st->cur = 0;
    }
}

__global__ __launch_bounds__(BLOCK) void k_head_place(const uint32_t* __restrict__ flag, uint32_t n,
                                                      const uint32_t* __restrict__ tile_off,
                                                      uint32_t* __restrict__ runs) {
    __shared__ uint32_t s_w[NWAVES];
    const uint32_t base = blockIdx.x * CT_TILE + threadIdx.x * CT_ITEMS;
    uint32_t f[CT_ITEMS], c = 0;
#pragma unroll
    for (uint32_t q = 0; q < CT_ITEMS; ++q) {
        f[q] = base + q < n ? flag[base + q] : 0u;
        c += f[q];
    }
    uint32_t total;
    uint32_t pos = tile_off[blockIdx.x] + block_exclusive_sum(c, s_w, &total);
#pragma unroll
    for (uint32_t q = 0; q < CT_ITEMS; ++q)
        if (f[q]) runs[pos++] = base + q;
}

// ---- one merge level
// Number of elements of X[lo, hi) that come before element (e, ke).
template <int EK>
__device__ __forceinline__ uint32_t rank_in(const uint8_t* __restrict__ bytes, uint64_t total_bytes,
                                            const uint64_t* __restrict__ offsets,
                                            const uint32_t* __restrict__ xi, const uint64_t* __restrict__ xk,
                                            uint32_t lo, uint32_t hi, uint32_t e, uint64_t ke) {
    uint32_t a = lo, z = hi;  // first position whose element is not before e
    while (a < z) {
        const uint32_t mid = a + ((z - a) >> 1);
        if (before<EK>(bytes, total_bytes, offsets, xi[mid], xk[mid], e, ke))
            a = mid + 1;
        else
            z = mid;
    }
    return a - lo;
}

template <int EK>
__global__ __launch_bounds__(BLOCK) void k_merge_level(const uint8_t* __restrict__ bytes,
                                                       const uint64_t* __restrict__ offsets, uint32_t n,
                                                       const MergeState* __restrict__ st,
                                                       uint32_t* idxA, uint64_t* keyA, uint32_t* idxB,
                                                       uint64_t* keyB, const uint32_t* runsA,
                                                       const uint32_t* runsB) {
    const uint32_t R = st->runs;
    if (R <= 1) return;
    const uint32_t cur = st->cur;
    const uint32_t* __restrict__ si = cur ? idxB : idxA;
    const uint64_t* __restrict__ sk = cur ? keyB : keyA;
    uint32_t* __restrict__ di = cur ? idxA : idxB;
    uint64_t* __restrict__ dk = cur ? keyA : keyB;
    const uint32_t* __restrict__ runs = cur ? runsB : runsA;
    const uint64_t total_bytes = offsets[n] * (EK == 0 ? 1u : 2u);
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < n; k += gridDim.x * BLOCK) {
        // run r holding position k: the last run start <= k
        uint32_t a = 0, z = R;
        while (z - a > 1) {
            const uint32_t mid = (a + z) >> 1;
            if (runs[mid] <= k) a = mid; else z = mid;
        }
        const uint32_t r = a;
        const uint32_t s0 = runs[r];
        const uint32_t e = si[k];
        const uint64_t ke = sk[k];
        uint32_t out;
        if ((r & 1u) == 0) {
            if (r + 1 >= R) {
                out = k;  // the last run has no partner at this level
            } else {
                const uint32_t b0 = runs[r + 1], b1 = r + 2 < R ? runs[r + 2] : n;
                out = k + rank_in<EK>(bytes, total_bytes, offsets, si, sk, b0, b1, e, ke);
            }
        } else {
            const uint32_t a0 = runs[r - 1];
            out = a0 + (k - s0) + rank_in<EK>(bytes, total_bytes, offsets, si, sk, a0, s0, e, ke);
        }
        di[out] = e;
        dk[out] = ke;
    }
}

// run table of the next level: every other run start
__global__ __launch_bounds__(BLOCK) void k_merge_runs(const MergeState* __restrict__ st,
                                                      const uint32_t* runsA, const uint32_t* runsB,
                                                      uint32_t* runsA_out, uint32_t* runsB_out) {
    const uint32_t R = st->runs;
    if (R <= 1) return;
    const uint32_t* src = st->cur ? runsB : runsA;
    uint32_t* dst = st->cur ? runsA_out : runsB_out;
    for (uint32_t j = blockIdx.x * BLOCK + threadIdx.x; 2 * j < R; j += gridDim.x * BLOCK) dst[j] = src[2 * j];
}

__global__ void k_merge_state(MergeState* st) {
    if (st->runs <= 1) return;
    st->runs = (st->runs + 1) / 2;
    st->cur ^= 1u;
}

__global__ __launch_bounds__(BLOCK) void k_merge_finish(const MergeState* __restrict__ st, uint32_t n,
                                                        uint32_t* __restrict__ idxA,
                                                        const uint32_t* __restrict__ idxB) {
    if (!st->cur) return;
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < n; k += gridDim.x * BLOCK) idxA[k] = idxB[k];
}

uint32_t grid_for_n(uint64_t n) { return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + BLOCK - 1) / BLOCK, 65536)); }

}  // namespace

size_t merge_workspace_bytes(uint64_t n) {
    const uint64_t tiles = (n + CT_TILE - 1) / CT_TILE + 1;
    auto al = [](uint64_t b) { return (b + 255) / 256 * 256; };
    return al(sizeof(MergeState)) + al(4 * n) + 2 * al(8 * n) + al(4 * n) + 2 * al(4 * (n + 1)) + al(4 * tiles);
}

hipError_t merge_fixup(int ek, const void* elems, const uint64_t* offsets, uint32_t n, uint32_t* idx, void* ws,
                       hipStream_t s) {
    if (n < 2) return hipSuccess;
    auto al = [](uint64_t b) { return (b + 255) / 256 * 256; };
    uint8_t* p = (uint8_t*)ws;
    MergeState* st = (MergeState*)p;
    p += al(sizeof(MergeState));
    uint32_t* idxB = (uint32_t*)p;
    p += al(4ull * n);
    uint64_t* keyA = (uint64_t*)p;
    p += al(8ull * n);
    uint64_t* keyB = (uint64_t*)p;
    p += al(8ull * n);
    uint32_t* flag = (uint32_t*)p;
    p += al(4ull * n);
    uint32_t* runsA = (uint32_t*)p;
    p += al(4ull * (n + 1));
    uint32_t* runsB = (uint32_t*)p;
    p += al(4ull * (n + 1));
    uint32_t* tile = (uint32_t*)p;
    const uint8_t* bytes = (const uint8_t*)elems;
    const uint32_t g = grid_for_n(n);
    const uint32_t tiles = (n + CT_TILE - 1) / CT_TILE;
    ProfScope ps(P_MERGE, s);
    if (ek == 0) {
        hipLaunchKernelGGL(k_prefix_keys<0>, dim3(g), dim3(BLOCK), 0, s, bytes, offsets, n, idx, keyA);
        hipLaunchKernelGGL(k_run_heads<0>, dim3(g), dim3(BLOCK), 0, s, bytes, offsets, n, (const uint32_t*)idx,
                           (const uint64_t*)keyA, flag);
    } else {
        hipLaunchKernelGGL(k_prefix_keys<1>, dim3(g), dim3(BLOCK), 0, s, bytes, offsets, n, idx, keyA);
        hipLaunchKernelGGL(k_run_heads<1>, dim3(g), dim3(BLOCK), 0, s, bytes, offsets, n, (const uint32_t*)idx,
                           (const uint64_t*)keyA, flag);
    }
    hipLaunchKernelGGL(k_head_tiles, dim3(tiles), dim3(BLOCK), 0, s, (const uint32_t*)flag, n, tile);
    hipLaunchKernelGGL(k_head_scan, dim3(1), dim3(BLOCK), 0, s, tile, tiles, st);
    hipLaunchKernelGGL(k_head_place, dim3(tiles), dim3(BLOCK), 0, s, (const uint32_t*)flag, n,
                       (const uint32_t*)tile, runsA);
    // enough levels for n runs; levels after the last merge do nothing
    uint32_t levels = 0;
    while ((1ull << levels) < n) ++levels;
    for (uint32_t l = 0; l < levels; ++l) {
        if (ek == 0)
            hipLaunchKernelGGL(k_merge_level<0>, dim3(g), dim3(BLOCK), 0, s, bytes, offsets, n,
                               (const MergeState*)st, idx, keyA, idxB, keyB, (const uint32_t*)runsA,
                               (const uint32_t*)runsB);
        else
            hipLaunchKernelGGL(k_merge_level<1>, dim3(g), dim3(BLOCK), 0, s, bytes, offsets, n,
                               (const MergeState*)st, idx, keyA, idxB, keyB, (const uint32_t*)runsA,
                               (const uint32_t*)runsB);
        hipLaunchKernelGGL(k_merge_runs, dim3(grid_for_n(n / 2 + 1)), dim3(BLOCK), 0, s, (const MergeState*)st,
                           (const uint32_t*)runsA, (const uint32_t*)runsB, runsA, runsB);
        hipLaunchKernelGGL(k_merge_state, dim3(1), dim3(1), 0, s, st);
    }
    hipLaunchKernelGGL(k_merge_finish, dim3(g), dim3(BLOCK), 0, s, (const MergeState*)st, n, idx,
                       (const uint32_t*)idxB);
    return hipGetLastError();
}

}  // namespace husky
