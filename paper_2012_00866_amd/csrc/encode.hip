// Step 1 of Huskysort: the husky code of every string (Algorithm 4,
// stringToLong, with the coder constants of Sec. 4.3), one string per lane.
//
// Strings are packed back to back, so the lanes of a wavefront read
// neighbouring bytes: each lane fetches the aligned 16-byte window holding its
// first nine bytes (two 8-byte loads) and the wavefront's loads coalesce into
// a few cache lines.  The code is assembled in registers:
//   ASCII7: sum over j < min(len, 9) of (b_j & 0x7F) << 7 * (8 - j)
//   UTF16 : sum over j < min(len, 4) of u_j << 16 * (3 - j)
// which is stringToLong's "shift in each character, then shift in the
// padding" written as fixed bit positions.

#include "common.h"
#include "internal.h"

namespace husky {

template <int CODER>
__global__ __launch_bounds__(BLOCK) void k_encode(const uint8_t* __restrict__ bytes,
                                                  const uint64_t* __restrict__ offsets,
                                                  uint32_t n,
                                                  uint64_t* __restrict__ codes,
                                                  uint32_t* __restrict__ idx,
                                                  uint32_t* __restrict__ status) {
    // bytes in the element buffer (uniform scalar load): the two-word window
    // below is used only where it stays inside the buffer.
    const uint64_t total_bytes = offsets[n] * (CODER == 0 ? 1u : 2u);
    uint32_t bad_here = 0;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        const uint64_t o0 = offsets[i], o1 = offsets[i + 1];
        const uint64_t len = o1 - o0;
        uint64_t code;
        if (CODER == 0) {
            const uint32_t L = len < 9 ? (uint32_t)len : 9u;
            const uint64_t base = o0 & ~7ull;
            const uint32_t sh = (uint32_t)(o0 & 7ull) * 8u;
            uint64_t lo, b8;
            if (base + 16 <= total_bytes) {
                const uint64_t* w = (const uint64_t*)(bytes + base);
                const uint64_t w0 = w[0], w1 = w[1];
                lo = sh ? ((w0 >> sh) | (w1 << (64 - sh))) : w0;
                b8 = (w1 >> sh) & 0xFFull;
            } else {
                lo = 0;
                for (uint32_t k = 0; k < 8; ++k)
                    if (k < L) lo |= (uint64_t)bytes[o0 + k] << (8 * k);
                b8 = L == 9 ? bytes[o0 + 8] : 0;
            }
            uint64_t c = b8 & 0x7Full;
#pragma unroll
            for (int j = 0; j < 8; ++j) c |= ((lo >> (8 * j)) & 0x7Full) << (7 * (8 - j));
            code = L == 0 ? 0ull : (c & (~0ull << (7 * (9 - L))));
            const uint64_t keep = L >= 8 ? ~0ull : ((1ull << (8 * L)) - 1ull);
            const bool bad = ((lo & 0x8080808080808080ull) & keep) != 0 || (L == 9 && (b8 & 0x80));
            bad_here += bad ? 1u : 0u;
        } else {
            const uint32_t L = len < 4 ? (uint32_t)len : 4u;
            uint64_t lo;
            const uint64_t addr = o0 * 2;
            const uint64_t base = addr & ~7ull;
            if (base + 16 <= total_bytes) {
                const uint32_t sh = (uint32_t)(addr & 7ull) * 8u;
                const uint64_t* w = (const uint64_t*)(bytes + base);
                const uint64_t w0 = w[0], w1 = w[1];
                lo = sh ? ((w0 >> sh) | (w1 << (64 - sh))) : w0;
            } else {
                lo = 0;
                const uint16_t* u = (const uint16_t*)bytes;
                for (uint32_t k = 0; k < 4; ++k)
                    if (k < L) lo |= (uint64_t)u[o0 + k] << (16 * k);
            }
            const uint64_t c = ((lo & 0xFFFFull) << 48) | (((lo >> 16) & 0xFFFFull) << 32) |
                               (((lo >> 32) & 0xFFFFull) << 16) | (lo >> 48);
            code = L == 0 ? 0ull : (c & (~0ull << (16 * (4 - L))));
        }
        codes[i] = code;
        if (idx) idx[i] = i;
    }
    if (CODER == 0 && status) {
        // one atomic per wavefront that saw a violation
        const uint64_t any = ballot(bad_here != 0);
        if (any) {
            uint32_t tot = bad_here;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, WAVE);
            if (lane_id() == 0) atomicAdd(status, tot);
        }
    }
}

hipError_t launch_encode(int coder, const void* elems, const uint64_t* offsets, uint32_t n,
                         uint64_t* codes, uint32_t* idx, uint32_t* status, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const uint32_t blocks = (n + BLOCK - 1) / BLOCK;
    ProfScope ps(P_ENCODE, s);
    if (coder == 0)
        hipLaunchKernelGGL(k_encode<0>, dim3(blocks), dim3(BLOCK), 0, s, (const uint8_t*)elems,
                           offsets, n, codes, idx, status);
    else
        hipLaunchKernelGGL(k_encode<1>, dim3(blocks), dim3(BLOCK), 0, s, (const uint8_t*)elems,
                           offsets, n, codes, idx, status);
    return hipGetLastError();
}

}  // namespace husky
