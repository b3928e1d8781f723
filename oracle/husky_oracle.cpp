// Huskysort CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, single-threaded reference for what the GPU path computes.  Only
// the test-suite, the smoke check and the benchmark's CPU-baseline leg may load
// it; the product library never does.  It shares no code, header or table with
// the HIP path.
//
// It follows the paper's three steps (Sec. 3.1 "Overview", Algorithm 1):
//   1. code every string with stringToLong (Algorithm 4) and the coder
//      constants of Sec. 4.3 ("Constants": BITS_LONG = 64, 7-bit ASCII with 9
//      characters and mask 0x7F, 16-bit UTF-16 with 4 units);
//   2. sort the (code, index) pairs by code, keeping equal codes in index
//      order (the role of the quicksort-with-object-swap phase; a stable
//      library sort is used so that the result is unique);
//   3. re-sort every run of equal codes with the full string comparison (the
//      role of the final Timsort pass), again stably.
// Because both sorts are stable and the coder is monotone, the result is the
// stable sorting permutation of the strings under the full comparator:
// byte-lexicographic order for ASCII, UTF-16 code-unit order for UTF-16, a
// proper prefix sorting first, equal strings in ascending index.
//
// Build: g++ -O2 -shared -fPIC husky_oracle.cpp -o liboracle.so

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <utility>
#include <vector>

namespace {

// Coder constants, Sec. 4.3 "Constants".
const int BITS_LONG = 64;
const int BIT_WIDTH_ASCII = 7;
const int MAX_LENGTH_ASCII = BITS_LONG / BIT_WIDTH_ASCII;  // 9
const uint64_t MASK_ASCII = 0x7F;
const int BIT_WIDTH_UNICODE = 16;
const int MAX_LENGTH_UNICODE = BITS_LONG / BIT_WIDTH_UNICODE;  // 4
const uint64_t MASK_UNICODE = 0xFFFF;

// Algorithm 4, stringToLong: take at most maxLength characters, append each
// one (masked) in the low bitWidth bits, then shift the missing characters'
// width in as zero padding.  Elem is uint8_t (ASCII) or uint16_t (UTF-16).
template <typename Elem>
uint64_t string_to_long(const Elem* str, uint64_t str_length, int max_length, int bit_width,
                        uint64_t mask) {
    uint64_t length = std::min<uint64_t>(str_length, (uint64_t)max_length);
    uint64_t padding = (uint64_t)max_length - length;
    uint64_t result = 0;
    if (mask == 0) {
        for (uint64_t i = 0; i < length; ++i) result = (result << bit_width) | (uint64_t)str[i];
    } else {
        for (uint64_t i = 0; i < length; ++i)
            result = (result << bit_width) | ((uint64_t)str[i] & mask);
    }
    // A shift by the full 64 bits only happens for an empty string, whose
    // result is zero anyway; spell that out instead of shifting by 64.
    uint64_t shift = (uint64_t)bit_width * padding;
    result = shift >= 64 ? 0 : (result << shift);
    return result;
}

// Full comparator (the order Timsort uses in Step 3): lexicographic over the
// unsigned elements, a proper prefix sorting first.
template <typename Elem>
bool string_less(const Elem* elems, const uint64_t* offsets, uint32_t a, uint32_t b) {
    const Elem* pa = elems + offsets[a];
    const Elem* pb = elems + offsets[b];
    uint64_t la = offsets[a + 1] - offsets[a];
    uint64_t lb = offsets[b + 1] - offsets[b];
    return std::lexicographical_compare(pa, pa + la, pb, pb + lb);
}

template <typename Elem>
void fixup_runs(const Elem* elems, const uint64_t* offsets, uint64_t n, const uint64_t* codes,
                uint32_t* idx) {
    // Step 3 restricted to runs of equal codes: with a monotone coder every
    // inversion left after Step 2 lies inside such a run.
    uint64_t start = 0;
    while (start < n) {
        uint64_t end = start + 1;
        while (end < n && codes[end] == codes[start]) ++end;
        if (end - start >= 2) {
            std::stable_sort(idx + start, idx + end, [&](uint32_t a, uint32_t b) {
                return string_less(elems, offsets, a, b);
            });
        }
        start = end;
    }
}

void sort_pairs(uint64_t* codes, uint32_t* idx, uint64_t n) {
    std::vector<std::pair<uint64_t, uint32_t>> v(n);
    for (uint64_t i = 0; i < n; ++i) v[i] = {codes[i], idx[i]};
    std::stable_sort(v.begin(), v.end(), [](const std::pair<uint64_t, uint32_t>& x,
                                            const std::pair<uint64_t, uint32_t>& y) {
        return x.first < y.first;
    });
    for (uint64_t i = 0; i < n; ++i) {
        codes[i] = v[i].first;
        idx[i] = v[i].second;
    }
}

}  // namespace

extern "C" {

// coder: 0 = ASCII 7-bit (9 chars), 1 = UTF-16 16-bit (4 units, unsigned code),
//        2 = UTF-16 as printed in the paper's unicodeToLong (the same code
//            shifted right by one bit), 3 = null coder (every code 0).

// Step 1 (Algorithm 2 / Algorithm 3 loop over Algorithm 4).  Returns the number
// of ASCII strings holding a byte >= 0x80 among their first 9 bytes: masking
// such a byte breaks monotonicity, so those inputs are outside the domain.
uint64_t oracle_encode(int coder, const void* elems, const uint64_t* offsets, uint64_t n,
                       uint64_t* codes) {
    uint64_t violations = 0;
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t len = offsets[i + 1] - offsets[i];
        if (coder == 0) {
            const uint8_t* s = (const uint8_t*)elems + offsets[i];
            codes[i] = string_to_long(s, len, MAX_LENGTH_ASCII, BIT_WIDTH_ASCII, MASK_ASCII);
            for (uint64_t j = 0; j < len && j < (uint64_t)MAX_LENGTH_ASCII; ++j)
                if (s[j] >= 0x80) {
                    ++violations;
                    break;
                }
        } else if (coder == 1 || coder == 2) {
            const uint16_t* s = (const uint16_t*)elems + offsets[i];
            uint64_t c = string_to_long(s, len, MAX_LENGTH_UNICODE, BIT_WIDTH_UNICODE, MASK_UNICODE);
            codes[i] = coder == 2 ? (c >> 1) : c;
        } else {
            codes[i] = 0;
        }
    }
    return violations;
}

// Step 2: stable sort of the (code, index) pairs by code.
void oracle_sort_pairs(uint64_t* codes, uint32_t* idx, uint64_t n) { sort_pairs(codes, idx, n); }

// Step 3: re-sort every run of equal codes with the full comparator.
// elem_bytes: 1 (ASCII) or 2 (UTF-16).
void oracle_fixup(int elem_bytes, const void* elems, const uint64_t* offsets, uint64_t n,
                  const uint64_t* sorted_codes, uint32_t* idx) {
    if (elem_bytes == 1)
        fixup_runs((const uint8_t*)elems, offsets, n, sorted_codes, idx);
    else
        fixup_runs((const uint16_t*)elems, offsets, n, sorted_codes, idx);
}

// Algorithm 1 end to end: perm receives the stable sorting permutation.
// elem_bytes is 1 for byte strings and 2 for UTF-16 strings (the null coder
// works on either).  Returns the domain-violation count of Step 1.
uint64_t oracle_sort(int coder, int elem_bytes, const void* elems, const uint64_t* offsets,
                     uint64_t n, uint32_t* perm) {
    std::vector<uint64_t> codes(n);
    uint64_t bad = oracle_encode(coder, elems, offsets, n, codes.data());
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    sort_pairs(codes.data(), perm, n);
    oracle_fixup(elem_bytes, elems, offsets, n, codes.data(), perm);
    return bad;
}

// Independent sort instances (batched form): instance k holds strings
// seg_offsets[k] .. seg_offsets[k+1]-1 and is sorted on its own; perm holds
// global string indices, each instance's slice a permutation of its range.
uint64_t oracle_sort_batched(int coder, int elem_bytes, const void* elems,
                             const uint64_t* offsets, const uint64_t* seg_offsets,
                             uint64_t n_segs, uint32_t* perm) {
    uint64_t bad = 0;
    for (uint64_t k = 0; k < n_segs; ++k) {
        uint64_t lo = seg_offsets[k], hi = seg_offsets[k + 1];
        bad += oracle_sort(coder, elem_bytes, elems, offsets + lo, hi - lo, perm + lo);
        for (uint64_t i = lo; i < hi; ++i) perm[i] += (uint32_t)lo;
    }
    return bad;
}

// Checker for outputs too large to re-sort: counts adjacent pairs of perm that
// are out of order under the full comparator with ascending index for equal
// strings, and entries that break the permutation property.  A perm with a
// zero count is the (unique) stable sorting permutation.
uint64_t oracle_check_perm(int elem_bytes, const void* elems, const uint64_t* offsets, uint64_t n,
                           const uint32_t* perm, uint64_t* first_bad) {
    uint64_t bad = 0;
    *first_bad = n;
    std::vector<uint8_t> seen(n, 0);
    for (uint64_t k = 0; k < n; ++k) {
        uint32_t p = perm[k];
        if (p >= n || seen[p]) {
            if (bad == 0) *first_bad = k;
            ++bad;
            continue;
        }
        seen[p] = 1;
    }
    if (bad) return bad;
    for (uint64_t k = 0; k + 1 < n; ++k) {
        uint32_t a = perm[k], b = perm[k + 1];
        bool lt_ba = elem_bytes == 1 ? string_less((const uint8_t*)elems, offsets, b, a)
                                     : string_less((const uint16_t*)elems, offsets, b, a);
        bool lt_ab = elem_bytes == 1 ? string_less((const uint8_t*)elems, offsets, a, b)
                                     : string_less((const uint16_t*)elems, offsets, a, b);
        bool ok = lt_ab || (!lt_ba && a < b);
        if (!ok) {
            if (bad == 0) *first_bad = k;
            ++bad;
        }
    }
    return bad;
}

// The same check for the batched form: every instance's slice of perm must
// be a permutation of its own index range, ordered as above.
uint64_t oracle_check_perm_batched(int elem_bytes, const void* elems, const uint64_t* offsets,
                                   const uint64_t* seg_offsets, uint64_t n_segs,
                                   const uint32_t* perm, uint64_t* first_bad) {
    uint64_t bad = 0;
    uint64_t n = seg_offsets[n_segs];
    *first_bad = n;
    std::vector<uint8_t> seen(n, 0);
    for (uint64_t s = 0; s < n_segs; ++s) {
        uint64_t lo = seg_offsets[s], hi = seg_offsets[s + 1];
        for (uint64_t k = lo; k < hi; ++k) {
            uint32_t p = perm[k];
            bool ok = p >= lo && p < hi && !seen[p];
            if (ok) seen[p] = 1;
            if (ok && k + 1 < hi) {
                uint32_t q = perm[k + 1];
                if (q >= lo && q < hi) {
                    bool lt_qp = elem_bytes == 1 ? string_less((const uint8_t*)elems, offsets, q, p)
                                                 : string_less((const uint16_t*)elems, offsets, q, p);
                    bool lt_pq = elem_bytes == 1 ? string_less((const uint8_t*)elems, offsets, p, q)
                                                 : string_less((const uint16_t*)elems, offsets, p, q);
                    ok = lt_pq || (!lt_qp && p < q);
                }
            }
            if (!ok) {
                if (bad == 0) *first_bad = k;
                ++bad;
            }
        }
    }
    return bad;
}

}  // extern "C"
