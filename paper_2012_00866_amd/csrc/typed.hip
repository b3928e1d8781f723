// Husky codes of the other object types the paper names as costly to compare
// (Sec. 3.2: date-times, with a perfect coder for nanosecond resolution over
// 128 years; Sec. 6: Integer, Long, Double, BigInteger, BigDecimal and
// tuples), and the order-preserving byte keys through which Step 3 compares
// the types whose code is not perfect.
//
// Codes (never decreasing in the type's order):
//   int32     (x + 2^31) << 32                                   perfect
//   int64     x + 2^63                                           perfect
//   float64   IEEE bits, sign flipped for positives, all bits     perfect
//             flipped for negatives, NaN made canonical first
//             (Java's Double.compare order: -0.0 < 0.0, NaN last)
//   datetime  1 + fields packed into 63 bits inside the window    perfect in
//             [base, base + 128) years (year 7 bits, month 4,     the window
//             day 5, hour 5, minute 6, second 6, nano 30);
//             0 below it, 2^63 + 1 above it
//   bigint, decimal, tuple: the first eight bytes of the key, big-endian.
// Keys (unsigned byte order = the type's order, equal exactly for equal values):
//   bigint    2-byte head (0x8000 + L for values >= 0, 0x7FFF - L below 0,
//             L = bytes of the shortest two's-complement form) + that form
//   decimal   class (00 negative, 01 zero, 02 positive), then for non-zero
//             values the decimal exponent E (value = 0.d x 10^E) + 32768 as
//             2 bytes and the significant digits d two per byte (digit + 1 per
//             nibble, a 0 nibble after an odd count); for negatives these
//             bytes are complemented and FF appended
//   tuple     the string with each 00 written 00 FF, then 00 00, then the
//             integer + 2^63 big-endian (string first, then the integer)
//   datetime  year + 2^31 (4 bytes), month, day, hour, minute, second, nano
//             (4 bytes), all big-endian: 13 bytes.

#include <algorithm>

#include "../../include/husky.h"
#include "common.h"
#include "internal.h"

namespace husky {

namespace {

__device__ __forceinline__ uint32_t ld_le32(const uint8_t* p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}
__device__ __forceinline__ uint64_t ld_le64(const uint8_t* p) {
    return (uint64_t)ld_le32(p) | ((uint64_t)ld_le32(p + 4) << 32);
}

// ---------------------------------------------------------------- fixed-width codes
template <int T>
__device__ __forceinline__ uint64_t fixed_code(const uint8_t* __restrict__ rec, int32_t base_year,
                                               bool* bad) {
    if (T == HUSKY_TYPE_INT32) {
        const uint32_t x = ld_le32(rec);
        return (uint64_t)(x ^ 0x80000000u) << 32;
    } else if (T == HUSKY_TYPE_INT64) {
        return ld_le64(rec) ^ 0x8000000000000000ull;
    } else if (T == HUSKY_TYPE_FLOAT64) {
        uint64_t b = ld_le64(rec);
        if (((b >> 52) & 0x7FF) == 0x7FF && (b & 0xFFFFFFFFFFFFFull)) b = 0x7FF8000000000000ull;
        return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
    } else {  // date-time
        const int32_t year = (int32_t)ld_le32(rec);
        const uint32_t month = rec[4], day = rec[5], hour = rec[6], minute = rec[7], second = rec[8];
        const uint32_t nano = ld_le32(rec + 12);
        *bad = !(month >= 1 && month <= 12 && day >= 1 && day <= 31 && hour <= 23 && minute <= 59 &&
                 second <= 59 && nano < 1000000000u);
        const int64_t dy = (int64_t)year - (int64_t)base_year;
        if (dy < 0) return 0ull;
        if (dy >= 128) return 0x8000000000000001ull;
        const uint64_t packed = ((uint64_t)dy << 56) | ((uint64_t)(month & 15) << 52) |
                                ((uint64_t)(day & 31) << 47) | ((uint64_t)(hour & 31) << 42) |
                                ((uint64_t)(minute & 63) << 36) | ((uint64_t)(second & 63) << 30) |
                                (uint64_t)(nano & 0x3FFFFFFFu);
        return 1ull + packed;
    }
}

template <int T>
__global__ __launch_bounds__(BLOCK) void k_fixed_codes(const uint8_t* __restrict__ recs, uint32_t n,
                                                       int32_t base_year, uint64_t* __restrict__ codes,
                                                       uint32_t* __restrict__ idx,
                                                       uint32_t* __restrict__ status) {
    constexpr uint32_t W = T == HUSKY_TYPE_INT32 ? 4 : (T == HUSKY_TYPE_DATETIME ? 16 : 8);
    uint32_t bad_here = 0;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        bool bad = false;
        codes[i] = fixed_code<T>(recs + (size_t)i * W, base_year, &bad);
        if (idx) idx[i] = i;
        bad_here += bad ? 1u : 0u;
    }
    if (status && ballot(bad_here != 0)) {
        uint32_t tot = bad_here;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, WAVE);
        if (lane_id() == 0) atomicAdd(status, tot);
    }
}

// ---------------------------------------------------------------- order keys
// A key is produced byte by byte into a sink: one that counts, one that
// stores, one that keeps the first eight bytes (the code).
struct CountSink {
    uint64_t n = 0;
    __device__ void put(uint32_t) { ++n; }
};
struct StoreSink {
    uint8_t* p;
    __device__ void put(uint32_t b) { *p++ = (uint8_t)b; }
};
struct CodeSink {
    uint64_t code = 0;
    uint32_t k = 0;
    __device__ void put(uint32_t b) {
        if (k < 8) code |= (uint64_t)(b & 0xFF) << (8 * (7 - k));
        ++k;
    }
};

// Shortest two's-complement form of the big-endian bytes r[0 .. L): its first
// byte (returned in *start) and its length; L == 0 reads as one zero byte.
__device__ __forceinline__ uint32_t shortest_twos(const uint8_t* r, uint32_t L, uint32_t* start) {
    uint32_t k = 0;
    if (L == 0) {
        *start = 0;
        return 0;
    }
    const bool neg = r[0] >= 0x80;
    while (k + 1 < L && r[k] == (neg ? 0xFF : 0x00) && ((r[k + 1] >= 0x80) == neg)) ++k;
    *start = k;
    return L - k;
}

template <class Sink>
__device__ void bigint_key(const uint8_t* r, uint32_t L, Sink& s, bool* bad) {
    *bad = L > 32767u;
    if (*bad) L = 0;
    uint32_t k = 0;
    const uint32_t m = shortest_twos(r, L, &k);
    const bool neg = m > 0 && r[k] >= 0x80;
    const uint32_t len = m ? m : 1u;
    const uint32_t head = neg ? 0x7FFFu - len : 0x8000u + len;
    s.put(head >> 8);
    s.put(head & 0xFF);
    if (!m) {
        s.put(0);
        return;
    }
    for (uint32_t j = 0; j < m; ++j) s.put(r[k + j]);
}

template <class Sink>
__device__ void decimal_key(const uint8_t* r, uint32_t L, Sink& s, bool* bad) {
    const int32_t scale = L >= 4 ? (int32_t)ld_le32(r) : 0;
    *bad = L < 4 || L - 4 > 16u || scale > 16000 || scale < -16000;
    if (*bad) {
        s.put(1);  // read as zero
        return;
    }
    const uint8_t* u = r + 4;
    const uint32_t ul = L - 4;
    // the unscaled value as a sign and a 128-bit magnitude in four 32-bit limbs
    const bool neg = ul > 0 && u[0] >= 0x80;
    uint32_t limb[4] = {0, 0, 0, 0};  // little-endian limbs of the two's complement value
    for (uint32_t j = 0; j < 16; ++j) {
        const uint32_t b = j < ul ? u[ul - 1 - j] : (neg ? 0xFFu : 0u);
        limb[j / 4] |= b << (8 * (j % 4));
    }
    if (neg) {  // magnitude = -value
        uint64_t c = 1;
        for (int q = 0; q < 4; ++q) {
            const uint64_t v = (uint64_t)(~limb[q]) + c;
            limb[q] = (uint32_t)v;
            c = v >> 32;
        }
    }
    if ((limb[0] | limb[1] | limb[2] | limb[3]) == 0) {
        s.put(1);
        return;
    }
    // decimal digits, least significant first (at most 39)
    uint8_t dig[40];
    uint32_t nd = 0;
    while (limb[0] | limb[1] | limb[2] | limb[3]) {
        uint64_t rem = 0;
        for (int q = 3; q >= 0; --q) {
            const uint64_t cur = (rem << 32) | limb[q];
            limb[q] = (uint32_t)(cur / 10u);
            rem = cur % 10u;
        }
        dig[nd++] = (uint8_t)rem;
    }
    uint32_t t = 0;  // trailing zeros (value = d x 10^t x 10^-scale)
    while (dig[t] == 0) ++t;
    const int32_t E = (int32_t)nd - scale;  // value = 0.d x 10^E
    const uint32_t flip = neg ? 0xFFu : 0u;
    s.put(neg ? 0x00u : 0x02u);
    const uint32_t e = (uint32_t)(E + 32768);
    s.put(((e >> 8) & 0xFF) ^ flip);
    s.put((e & 0xFF) ^ flip);
    // significant digits, most significant first: dig[nd - 1] .. dig[t]
    for (int32_t j = (int32_t)nd - 1; j >= (int32_t)t; j -= 2) {
        const uint32_t hi = dig[j] + 1u;
        const uint32_t lo = j - 1 >= (int32_t)t ? dig[j - 1] + 1u : 0u;
        s.put(((hi << 4) | lo) ^ flip);
    }
    if (neg) s.put(0xFF);
}

template <class Sink>
__device__ void tuple_key(const uint8_t* r, uint32_t L, Sink& s, bool* bad) {
    *bad = L < 8;
    const uint64_t v = *bad ? 0ull : ld_le64(r);
    for (uint32_t j = 8; j < L; ++j) {
        s.put(r[j]);
        if (r[j] == 0) s.put(0xFF);
    }
    s.put(0);
    s.put(0);
    const uint64_t b = v ^ 0x8000000000000000ull;
    for (int k = 7; k >= 0; --k) s.put((uint32_t)(b >> (8 * k)) & 0xFF);
}

template <class Sink>
__device__ void datetime_key(const uint8_t* r, Sink& s) {
    const uint32_t y = ld_le32(r) ^ 0x80000000u;
    for (int k = 3; k >= 0; --k) s.put((y >> (8 * k)) & 0xFF);
    for (int k = 4; k < 9; ++k) s.put(r[k]);
    const uint32_t ns = ld_le32(r + 12);
    for (int k = 3; k >= 0; --k) s.put((ns >> (8 * k)) & 0xFF);
}

template <int T, class Sink>
__device__ __forceinline__ void record_key(const uint8_t* r, uint32_t L, Sink& s, bool* bad) {
    if (T == HUSKY_TYPE_BIGINT) bigint_key(r, L, s, bad);
    else if (T == HUSKY_TYPE_DECIMAL) decimal_key(r, L, s, bad);
    else if (T == HUSKY_TYPE_TUPLE) tuple_key(r, L, s, bad);
    else { datetime_key(r, s); *bad = false; }
}

__device__ __forceinline__ void count_bad(uint32_t bad_here, uint32_t* status) {
    if (status && ballot(bad_here != 0)) {
        uint32_t tot = bad_here;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, WAVE);
        if (lane_id() == 0) atomicAdd(status, tot);
    }
}

// Variable-length records: key lengths (and the out-of-domain count).
template <int T>
__global__ __launch_bounds__(BLOCK) void k_key_lengths(const uint8_t* __restrict__ recs,
                                                       const uint64_t* __restrict__ offsets, uint32_t n,
                                                       uint64_t* __restrict__ lens,
                                                       uint32_t* __restrict__ status) {
    uint32_t bad_here = 0;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        const uint64_t o = offsets[i];
        CountSink c;
        bool bad = false;
        record_key<T>(recs + o, (uint32_t)min<uint64_t>(offsets[i + 1] - o, 0xFFFFFFFFull), c, &bad);
        lens[i] = c.n;
        bad_here += bad ? 1u : 0u;
    }
    count_bad(bad_here, status);
}

template <int T>
__global__ __launch_bounds__(BLOCK) void k_key_write(const uint8_t* __restrict__ recs,
                                                     const uint64_t* __restrict__ offsets, uint32_t n,
                                                     uint32_t fixed_width,
                                                     const uint64_t* __restrict__ key_offsets,
                                                     uint8_t* __restrict__ keys) {
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        const uint64_t o = offsets ? offsets[i] : (uint64_t)i * fixed_width;
        const uint64_t L = offsets ? offsets[i + 1] - o : fixed_width;
        StoreSink st{keys + key_offsets[i]};
        bool bad = false;
        record_key<T>(recs + o, (uint32_t)min<uint64_t>(L, 0xFFFFFFFFull), st, &bad);
    }
}

template <int T>
__global__ __launch_bounds__(BLOCK) void k_key_codes(const uint8_t* __restrict__ recs,
                                                     const uint64_t* __restrict__ offsets, uint32_t n,
                                                     uint64_t* __restrict__ codes,
                                                     uint32_t* __restrict__ status) {
    uint32_t bad_here = 0;
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        const uint64_t o = offsets[i];
        CodeSink c;
        bool bad = false;
        record_key<T>(recs + o, (uint32_t)min<uint64_t>(offsets[i + 1] - o, 0xFFFFFFFFull), c, &bad);
        codes[i] = c.code;
        bad_here += bad ? 1u : 0u;
    }
    count_bad(bad_here, status);
}

__global__ __launch_bounds__(BLOCK) void k_fixed_offsets(uint64_t* __restrict__ off, uint32_t n,
                                                         uint32_t width) {
    for (uint32_t i = blockIdx.x * BLOCK + threadIdx.x; i <= n; i += gridDim.x * BLOCK)
        off[i] = (uint64_t)i * width;
}

// ---------------------------------------------------------------- exclusive scan of u64
// out[0 .. n] = exclusive prefix sums of in[0 .. n) (out[n] = total): tile
// sums, one workgroup scanning the tile sums, then each tile its own prefix.
constexpr uint32_t SCAN_ITEMS = 8;
constexpr uint32_t SCAN_TILE = BLOCK * SCAN_ITEMS;

__device__ __forceinline__ uint64_t wave_incl_u64(uint64_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const uint64_t t = __shfl_up(v, d, WAVE);
        if (lane >= (uint32_t)d) v += t;
    }
    return v;
}

// Exclusive prefix of v over the workgroup; *total gets the sum.
__device__ __forceinline__ uint64_t block_excl_u64(uint64_t v, uint64_t* s_w, uint64_t* total) {
    const uint32_t w = threadIdx.x / WAVE;
    const uint64_t inc = wave_incl_u64(v);
    if (lane_id() == WAVE - 1) s_w[w] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < NWAVES; ++q) {
        before += q < (int)w ? s_w[q] : 0ull;
        all += s_w[q];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(BLOCK) void k_scan_tiles(const uint64_t* __restrict__ in, uint32_t n,
                                                      uint64_t* __restrict__ tile_sum) {
    __shared__ uint64_t s_w[NWAVES];
    const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_ITEMS; ++k) s += base + k < n ? in[base + k] : 0ull;
    uint64_t total;
    block_excl_u64(s, s_w, &total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(BLOCK) void k_scan_sums(uint64_t* __restrict__ tile_sum, uint32_t tiles) {
    __shared__ uint64_t s_w[NWAVES];
    uint64_t carry = 0;
    for (uint32_t b = 0; b < tiles; b += BLOCK) {
        const uint32_t i = b + threadIdx.x;
        const uint64_t v = i < tiles ? tile_sum[i] : 0ull;
        uint64_t total;
        const uint64_t ex = block_excl_u64(v, s_w, &total);
        if (i < tiles) tile_sum[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) tile_sum[tiles] = carry;
}

__global__ __launch_bounds__(BLOCK) void k_scan_apply(const uint64_t* __restrict__ in, uint32_t n,
                                                      const uint64_t* __restrict__ tile_prefix,
                                                      uint32_t tiles, uint64_t* __restrict__ out) {
    __shared__ uint64_t s_w[NWAVES];
    const uint32_t base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    uint64_t v[SCAN_ITEMS], s = 0;
#pragma unroll
    for (uint32_t k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = base + k < n ? in[base + k] : 0ull;
        s += v[k];
    }
    uint64_t total;
    uint64_t run = tile_prefix[blockIdx.x] + block_excl_u64(s, s_w, &total);
#pragma unroll
    for (uint32_t k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tile_prefix[tiles];
}

uint32_t grid_of(uint64_t n) { return (uint32_t)std::min<uint64_t>((n + BLOCK - 1) / BLOCK, 65536); }

}  // namespace

uint32_t typed_scan_tiles(uint32_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t typed_fixed_codes(int type, const void* recs, uint32_t n, int32_t base_year, uint64_t* codes,
                             uint32_t* idx, uint32_t* status, hipStream_t s) {
    if (!n) return hipSuccess;
    ProfScope ps(P_ENCODE, s);
    const uint8_t* r = (const uint8_t*)recs;
#define HUSKY_FC(T)                                                                           \
    case T:                                                                                  \
        hipLaunchKernelGGL(k_fixed_codes<T>, dim3(grid_of(n)), dim3(BLOCK), 0, s, r, n, base_year, \
                           codes, idx, status);                                              \
        break;
    switch (type) {
        HUSKY_FC(HUSKY_TYPE_INT32)
        HUSKY_FC(HUSKY_TYPE_INT64)
        HUSKY_FC(HUSKY_TYPE_FLOAT64)
        HUSKY_FC(HUSKY_TYPE_DATETIME)
        default: return hipErrorInvalidValue;
    }
#undef HUSKY_FC
    return hipGetLastError();
}

hipError_t typed_key_codes(int type, const void* recs, const uint64_t* offsets, uint32_t n,
                           uint64_t* codes, uint32_t* status, hipStream_t s) {
    if (!n) return hipSuccess;
    ProfScope ps(P_ENCODE, s);
    const uint8_t* r = (const uint8_t*)recs;
#define HUSKY_KC(T)                                                                             \
    case T:                                                                                    \
        hipLaunchKernelGGL(k_key_codes<T>, dim3(grid_of(n)), dim3(BLOCK), 0, s, r, offsets, n, codes, \
                           status);                                                            \
        break;
    switch (type) {
        HUSKY_KC(HUSKY_TYPE_BIGINT)
        HUSKY_KC(HUSKY_TYPE_DECIMAL)
        HUSKY_KC(HUSKY_TYPE_TUPLE)
        default: return hipErrorInvalidValue;
    }
#undef HUSKY_KC
    return hipGetLastError();
}

hipError_t typed_keys(int type, const void* recs, const uint64_t* offsets, uint32_t n, uint64_t* lens,
                      uint64_t* tile_tmp, uint64_t* key_offsets, uint8_t* keys, uint32_t* status,
                      hipStream_t s) {
    const uint8_t* r = (const uint8_t*)recs;
    if (type == HUSKY_TYPE_DATETIME) {  // 13-byte keys of fixed 16-byte records
        hipLaunchKernelGGL(k_fixed_offsets, dim3(grid_of((uint64_t)n + 1)), dim3(BLOCK), 0, s, key_offsets,
                           n, 13u);
        if (n)
            hipLaunchKernelGGL(k_key_write<HUSKY_TYPE_DATETIME>, dim3(grid_of(n)), dim3(BLOCK), 0, s, r,
                               (const uint64_t*)nullptr, n, 16u, (const uint64_t*)key_offsets, keys);
        return hipGetLastError();
    }
    if (n) {
#define HUSKY_KL(T)                                                                                 \
    case T:                                                                                        \
        hipLaunchKernelGGL(k_key_lengths<T>, dim3(grid_of(n)), dim3(BLOCK), 0, s, r, offsets, n, lens, \
                           status);                                                                \
        break;
        switch (type) {
            HUSKY_KL(HUSKY_TYPE_BIGINT)
            HUSKY_KL(HUSKY_TYPE_DECIMAL)
            HUSKY_KL(HUSKY_TYPE_TUPLE)
            default: return hipErrorInvalidValue;
        }
#undef HUSKY_KL
    }
    const uint32_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles) hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(BLOCK), 0, s, (const uint64_t*)lens, n, tile_tmp);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(BLOCK), 0, s, tile_tmp, tiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(std::max(tiles, 1u)), dim3(BLOCK), 0, s, (const uint64_t*)lens, n,
                       (const uint64_t*)tile_tmp, tiles, key_offsets);
    if (n) {
#define HUSKY_KW(T)                                                                                \
    case T:                                                                                       \
        hipLaunchKernelGGL(k_key_write<T>, dim3(grid_of(n)), dim3(BLOCK), 0, s, r, offsets, n, 0u,   \
                           (const uint64_t*)key_offsets, keys);                                   \
        break;
        switch (type) {
            HUSKY_KW(HUSKY_TYPE_BIGINT)
            HUSKY_KW(HUSKY_TYPE_DECIMAL)
            HUSKY_KW(HUSKY_TYPE_TUPLE)
            default: return hipErrorInvalidValue;
        }
#undef HUSKY_KW
    }
    return hipGetLastError();
}

}  // namespace husky
