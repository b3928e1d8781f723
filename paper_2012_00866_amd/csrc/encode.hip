// Step 1 of Huskysort: the husky code of every string (Algorithm 4,
// stringToLong, with the coder constants of Sec. 4.3), one string per lane.
//
// Strings are packed back to back, so the lanes of a wavefront read
// neighbouring bytes: each lane fetches the aligned 16-byte window holding its
// first nine bytes (two 8-byte loads) and the wavefront's loads coalesce into
// a few cache lines.  The code is assembled in registers:
//   ASCII7: sum over j < min(len, 9) of (b_j & 0x7F) << 7 * (8 - j)
//   UTF16 : sum over j < min(len, 4) of u_j << 16 * (3 - j)
//   BYTES8: sum over j < min(len, 8) of b_j << 8 * (7 - j)
// which is stringToLong's "shift in each character, then shift in the
// padding" written as fixed bit positions.  The full-byte coder is the 8-bit
// member of the alphabet-dependent coders of Sec. 3.2: every byte value keeps
// its order, at the cost of one character fewer than the 7-bit coder.

#include "bucket.h"
#include "common.h"
#include "internal.h"

namespace husky {

// Optionally also the first refinement key of every string (key0): the
// chunk the fix-up compares first inside a run of equal codes (see
// fixup.hip for its layout).  Computing it here, while the string's bytes are
// streamed in order, spares the fix-up a random gather per run member.
// With LEARNED, each code's bucket under a fitted learned-CDF model is
// computed here as well, while the code is still in a register.
// With `perfect` (ASCII only) the code is written as code << 1 | f, where
// f = 0 exactly when the string is at most nine bytes long and none of them
// is NUL -- the string is then determined by its code alone, the per-string
// form of the paper's "perfect" coding (Algorithm 3).  The shifted code is
// still monotone: if s < t and code(s) = code(t) with f(t) = 0, t's bytes
// are s's first bytes padded by the code's zeros, so s >= t -- a
// contradiction; hence f(s) <= f(t).  Equal shifted codes with f = 0 are
// identical strings, which need no fix-up.  (Bit 63 of the ASCII code is
// always 0, so nothing is lost.)
template <int CODER, bool LEARNED>
__global__ __launch_bounds__(BLOCK) void k_encode(const uint8_t* __restrict__ bytes,
                                                  const uint64_t* __restrict__ offsets,
                                                  uint32_t n,
                                                  uint64_t* __restrict__ codes,
                                                  uint32_t* __restrict__ idx,
                                                  uint64_t* __restrict__ key0,
                                                  uint32_t* __restrict__ status,
                                                  const uint32_t* __restrict__ sel,
                                                  uint32_t n_out, BucketArgs bucket, bool perfect,
                                                  uint64_t* __restrict__ korand, uint32_t tile,
                                                  bool tag_low8) {
    // bytes in the element buffer (uniform scalar load): the three-word
    // window below is used only where it stays inside the buffer.
    constexpr uint32_t ES = CODER == 1 ? 2u : 1u;  // bytes per element
    const uint64_t total_bytes = offsets[n] * ES;
    uint32_t bad_here = 0;
    const uint32_t count = sel ? n_out : n;
    uint64_t m_lo = 0, m_hi = 0;
    uint32_t m_cp = 0;
    if (LEARNED) {
        m_lo = bucket.hdr->lo;
        m_hi = bucket.hdr->hi;
        m_cp = bucket.hdr->cp;
    }
    // Step 1 for entry t: writes its code (and index, first refinement key)
    // and returns the code
    auto encode_one = [&](uint32_t t) -> uint64_t {
        const uint32_t i = sel ? sel[t] : t;
        const uint64_t o0 = offsets[i], o1 = offsets[i + 1];
        const uint64_t len = o1 - o0;
        // string bytes 0..7 (lo) and 8..15 (mid), little-endian; bytes past
        // the string are masked off below
        const uint64_t addr = o0 * ES;
        const uint64_t base = addr & ~7ull;
        const uint32_t sh = (uint32_t)(addr & 7ull) * 8u;
        const uint64_t need = (CODER == 0 ? 9u : 8u) + (key0 ? 7u : 0u);  // bytes used from addr
        const uint64_t slen = len * ES;
        uint64_t lo = 0, mid = 0;
        if (base + 24 <= total_bytes) {
            const uint64_t* w = (const uint64_t*)(bytes + base);
            const uint64_t w0 = w[0], w1 = w[1];
            const uint64_t w2 = (sh + 8 * need > 128) ? w[2] : 0ull;
            lo = sh ? ((w0 >> sh) | (w1 << (64 - sh))) : w0;
            mid = sh ? ((w1 >> sh) | (w2 << (64 - sh))) : w1;
        } else {
            const uint64_t m = slen < need ? slen : need;
            for (uint32_t k = 0; k < 16; ++k)
                if (k < m) {
                    const uint64_t b = bytes[addr + k];
                    if (k < 8) lo |= b << (8 * k);
                    else mid |= b << (8 * (k - 8));
                }
        }
        uint64_t code, k0 = 0;
        if (CODER == 0) {
            const uint32_t L = len < 9 ? (uint32_t)len : 9u;
            const uint64_t b8 = mid & 0xFFull;
            uint64_t c = b8 & 0x7Full;
#pragma unroll
            for (int j = 0; j < 8; ++j) c |= ((lo >> (8 * j)) & 0x7Full) << (7 * (8 - j));
            code = L == 0 ? 0ull : (c & (~0ull << (7 * (9 - L))));
            const uint64_t keep = L >= 8 ? ~0ull : ((1ull << (8 * L)) - 1ull);
            const bool bad = ((lo & 0x8080808080808080ull) & keep) != 0 || (L == 9 && (b8 & 0x80));
            bad_here += bad ? 1u : 0u;
            if (perfect) {
                bool nul = L == 9 && b8 == 0;
#pragma unroll
                for (uint32_t j = 0; j < 8; ++j) nul = nul || (j < L && ((lo >> (8 * j)) & 0xFFull) == 0);
                code = (code << 1) | ((len > 9 || nul) ? 1ull : 0ull);
            }
            if (key0) {
                const uint64_t rem = len > 9 ? len - 9 : 0;
                const uint64_t nb = rem < 7 ? rem : 7;
                const uint64_t clen = rem > 7 ? 8 : rem;
                const uint64_t w = (mid >> 8) & (nb ? ((1ull << (8 * nb)) - 1ull) : 0ull);
                k0 = ((uint64_t)L << 60) | ((__builtin_bswap64(w) >> 8) << 4) | clen;
            }
        } else if (CODER == 2) {
            const uint32_t L = len < 8 ? (uint32_t)len : 8u;
            code = L == 0 ? 0ull : (__builtin_bswap64(lo) & (~0ull << (8 * (8 - L))));
            if (key0) {
                const uint64_t rem = len > 8 ? len - 8 : 0;
                const uint64_t nb = rem < 7 ? rem : 7;
                const uint64_t clen = rem > 7 ? 8 : rem;
                const uint64_t w = mid & (nb ? ((1ull << (8 * nb)) - 1ull) : 0ull);
                k0 = ((uint64_t)L << 60) | ((__builtin_bswap64(w) >> 8) << 4) | clen;
            }
        } else {
            const uint32_t L = len < 4 ? (uint32_t)len : 4u;
            const uint64_t c = ((lo & 0xFFFFull) << 48) | (((lo >> 16) & 0xFFFFull) << 32) |
                               (((lo >> 32) & 0xFFFFull) << 16) | (lo >> 48);
            code = L == 0 ? 0ull : (c & (~0ull << (16 * (4 - L))));
            if (key0) {
                const uint64_t rem = len > 4 ? len - 4 : 0;
                const uint64_t nu = rem < 3 ? rem : 3;
                const uint64_t clen = rem > 3 ? 4 : rem;
                const uint64_t w = mid & (nu ? ((1ull << (16 * nu)) - 1ull) : 0ull);
                const uint64_t ch = ((w & 0xFFFFull) << 32) | (((w >> 16) & 0xFFFFull) << 16) |
                                    ((w >> 32) & 0xFFFFull);
                k0 = ((uint64_t)L << 60) | (ch << 12) | clen;
            }
        }
        if (codes) codes[t] = code;
        // tag_low8: the code's low byte rides in the index's top byte (indices
        // below 2^24), as the first digit pass's count input
        if (idx) idx[t] = tag_low8 ? i | ((uint32_t)code & 0xFFu) << 24 : i;
        if (key0) key0[t] = k0;
        return code;
    };
    if (!LEARNED && korand) {
        // workgroup b encodes radix tile b and reduces its codes' OR / AND
        __shared__ uint64_t s_o[NWAVES], s_a[NWAVES];
        const uint32_t t0 = blockIdx.x * tile, t1 = min(count, t0 + tile);
        uint64_t o = 0, a = ~0ull;
        for (uint32_t t = t0 + threadIdx.x; t < t1; t += BLOCK) {
            const uint64_t c = encode_one(t);
            o |= c;
            a &= c;
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            o |= (uint64_t)__shfl_xor((unsigned long long)o, d, WAVE);
            a &= (uint64_t)__shfl_xor((unsigned long long)a, d, WAVE);
        }
        if (lane_id() == 0) {
            s_o[threadIdx.x / WAVE] = o;
            s_a[threadIdx.x / WAVE] = a;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < NWAVES; ++w) {
                o |= s_o[w];
                a &= s_a[w];
            }
            korand[2 * (size_t)blockIdx.x] = o;
            korand[2 * (size_t)blockIdx.x + 1] = a;
        }
    } else if (!LEARNED) {
        for (uint32_t t = blockIdx.x * BLOCK + threadIdx.x; t < count; t += gridDim.x * BLOCK)
            encode_one(t);
    } else {
        // LEARNED_K entries per thread (BLOCK apart, so stores stay coalesced),
        // their bucket lookups in flight together (bucket.h)
        for (uint32_t t0 = blockIdx.x * BLOCK * LEARNED_K + threadIdx.x; t0 < count;
             t0 += gridDim.x * BLOCK * LEARNED_K) {
            uint64_t cd[LEARNED_K];
            bool ok[LEARNED_K];
#pragma unroll
            for (int j = 0; j < LEARNED_K; ++j) {
                const uint32_t t = t0 + j * BLOCK;
                ok[j] = t < count;
                cd[j] = ok[j] ? encode_one(t) : 0ull;
            }
            uint32_t b[LEARNED_K];
            bucket_of<LEARNED_K>(bucket, cd, ok, m_lo, m_hi, m_cp, b);
#pragma unroll
            for (int j = 0; j < LEARNED_K; ++j)
                if (ok[j]) bucket.bid[t0 + j * BLOCK] = (uint16_t)b[j];
        }
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
                         uint64_t* codes, uint32_t* idx, uint64_t* key0, uint32_t* status,
                         hipStream_t s, const uint32_t* sel, uint32_t n_out,
                         const BucketArgs* bucket, bool perfect, uint64_t* korand, uint32_t tile,
                         bool tag_low8) {
    const uint32_t count = sel ? n_out : n;
    if (count == 0) return hipSuccess;
    if (bucket || !tile) korand = nullptr;
    const uint32_t per_block = korand ? tile : (bucket ? BLOCK * LEARNED_K : BLOCK);
    const uint32_t blocks = (count + per_block - 1) / per_block;
    ProfScope ps(P_ENCODE, s);
    const BucketArgs b = bucket ? *bucket : BucketArgs{};
    const uint8_t* e = (const uint8_t*)elems;
#define HUSKY_ENC(C, L)                                                                           \
    hipLaunchKernelGGL((k_encode<C, L>), dim3(blocks), dim3(BLOCK), 0, s, e, offsets, n, codes, idx, \
                       key0, status, sel, n_out, b, perfect && coder == 0, korand, tile,        \
                       tag_low8 && !sel && n <= (1u << 24))
    if (coder == CODER_ASCII7) {
        if (bucket) HUSKY_ENC(0, true); else HUSKY_ENC(0, false);
    } else if (coder == CODER_BYTES8) {
        if (bucket) HUSKY_ENC(2, true); else HUSKY_ENC(2, false);
    } else {
        if (bucket) HUSKY_ENC(1, true); else HUSKY_ENC(1, false);
    }
#undef HUSKY_ENC
    return hipGetLastError();
}

}  // namespace husky
