// Exactness check on the device: a permutation is THE stable sorting
// permutation iff (1) it is a permutation of every instance's index range and
// (2) every adjacent pair is ordered by the full comparator, equal strings in
// ascending index.  Both properties are checked for every position, so the
// check holds at any size without a second sort.

#include <algorithm>

#include "../../include/husky.h"
#include "common.h"
#include "internal.h"

namespace husky {

// Compare strings a and b (lexicographic over unsigned elements, a proper
// prefix first): -1, 0 or 1.  Reads 8 bytes at a time.
template <int CODER>
__device__ int compare_strings(const uint8_t* __restrict__ bytes, uint64_t total_bytes, uint64_t oa,
                               uint64_t la, uint64_t ob, uint64_t lb) {
    const uint64_t es = CODER == 0 ? 1 : 2;
    const uint64_t n = la < lb ? la : lb;  // common length in elements
    const uint64_t per = 8 / es;
    for (uint64_t i = 0; i < n; i += per) {
        const uint64_t take = n - i < per ? n - i : per;
        const uint64_t mask = take * es >= 8 ? ~0ull : ((1ull << (8 * take * es)) - 1ull);
        uint64_t wa = load8_unaligned(bytes, total_bytes, (oa + i) * es) & mask;
        uint64_t wb = load8_unaligned(bytes, total_bytes, (ob + i) * es) & mask;
        if (wa != wb) {
            if (CODER == 0) {
                wa = bswap64(wa);
                wb = bswap64(wb);
            } else {  // big-endian order of 16-bit units
                wa = ((wa & 0xFFFFull) << 48) | (((wa >> 16) & 0xFFFFull) << 32) |
                     (((wa >> 32) & 0xFFFFull) << 16) | (wa >> 48);
                wb = ((wb & 0xFFFFull) << 48) | (((wb >> 16) & 0xFFFFull) << 32) |
                     (((wb >> 32) & 0xFFFFull) << 16) | (wb >> 48);
            }
            return wa < wb ? -1 : 1;
        }
    }
    return la < lb ? -1 : (la > lb ? 1 : 0);
}

// Instance of position k (binary search over seg_offsets), or 0 without
// instances.
__device__ __forceinline__ uint64_t seg_of(const uint64_t* seg, uint64_t nseg, uint64_t k) {
    if (!seg) return 0;
    uint64_t lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) >> 1;
        if (seg[mid] <= k)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(BLOCK) void k_check_perm_range(const uint32_t* __restrict__ perm,
                                                            uint32_t n, const uint64_t* seg,
                                                            uint64_t nseg, uint32_t* __restrict__ seen,
                                                            uint32_t* __restrict__ bad) {
    uint32_t local = 0;
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k < n; k += gridDim.x * BLOCK) {
        const uint32_t p = perm[k];
        bool ok = p < n;
        if (ok && seg) {
            const uint64_t s = seg_of(seg, nseg, k);
            ok = p >= seg[s] && p < seg[s + 1];
        }
        if (ok) {
            const uint32_t bit = 1u << (p & 31);
            ok = !(atomicOr(&seen[p >> 5], bit) & bit);
        }
        local += ok ? 0u : 1u;
    }
    if (local) atomicAdd(bad, local);
}

template <int CODER>
__global__ __launch_bounds__(BLOCK) void k_check_order(const uint8_t* __restrict__ bytes,
                                                       const uint64_t* __restrict__ offsets,
                                                       const uint32_t* __restrict__ perm, uint32_t n,
                                                       const uint64_t* seg, uint64_t nseg,
                                                       uint32_t* __restrict__ bad) {
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    uint32_t local = 0;
    for (uint32_t k = blockIdx.x * BLOCK + threadIdx.x; k + 1 < n; k += gridDim.x * BLOCK) {
        if (seg) {
            const uint64_t s = seg_of(seg, nseg, k);
            if ((uint64_t)k + 1 >= seg[s + 1]) continue;  // pair straddles instances
        }
        const uint32_t a = perm[k], b = perm[k + 1];
        if (a >= n || b >= n) continue;  // reported by the range check
        const uint64_t oa = offsets[a], ob = offsets[b];
        const int c = compare_strings<CODER>(bytes, total_bytes, oa, offsets[a + 1] - oa, ob,
                                             offsets[b + 1] - ob);
        local += (c < 0 || (c == 0 && a < b)) ? 0u : 1u;
    }
    if (local) atomicAdd(bad, local);
}

}  // namespace husky

using namespace husky;

extern "C" husky_status husky_check_perm(husky_coder coder, const void* elems,
                                         const uint64_t* offsets, uint64_t n,
                                         const uint64_t* seg_offsets_or_null, uint64_t n_segs,
                                         const uint32_t* perm, void* ws, size_t ws_bytes,
                                         uint32_t* violations, void* stream) {
    if (coder != HUSKY_CODER_ASCII7 && coder != HUSKY_CODER_UTF16 && coder != HUSKY_CODER_BYTES8)
        return HUSKY_ERR_ARG;
    if (n >= (1ull << 32) || !violations) return HUSKY_ERR_ARG;
    if (n > 0 && (!elems || !offsets || !perm)) return HUSKY_ERR_ARG;
    if (seg_offsets_or_null && n_segs == 0) return HUSKY_ERR_ARG;
    const size_t need = ((n + 31) / 32) * 4;
    if (!ws || ws_bytes < need) return HUSKY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    if (zero_u32((uint32_t*)ws, (n + 31) / 32, s) != hipSuccess) return HUSKY_ERR_HIP;
    if (zero_u32(violations, 1, s) != hipSuccess) return HUSKY_ERR_HIP;
    if (n == 0) return HUSKY_OK;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n + BLOCK - 1) / BLOCK, 8192);
    hipLaunchKernelGGL(k_check_perm_range, dim3(blocks), dim3(BLOCK), 0, s, perm, (uint32_t)n,
                       seg_offsets_or_null, n_segs, (uint32_t*)ws, violations);
    // byte strings (ASCII and full-byte coders) or UTF-16 units
    if (coder != HUSKY_CODER_UTF16)
        hipLaunchKernelGGL(k_check_order<0>, dim3(blocks), dim3(BLOCK), 0, s, (const uint8_t*)elems,
                           offsets, perm, (uint32_t)n, seg_offsets_or_null, n_segs, violations);
    else
        hipLaunchKernelGGL(k_check_order<1>, dim3(blocks), dim3(BLOCK), 0, s, (const uint8_t*)elems,
                           offsets, perm, (uint32_t)n, seg_offsets_or_null, n_segs, violations);
    return hipGetLastError() == hipSuccess ? HUSKY_OK : HUSKY_ERR_HIP;
}
