// Huskysort CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, single-threaded reference for what the GPU path computes.  Only
// the test-suite, the smoke check and the benchmark's CPU-baseline leg may load
// it; the product library never does.  It shares no code, header or table with
// the HIP path.
//
// It follows the paper's three steps (Sec. 3.1 "Overview", Algorithm 1):
//   1. code every string (Algorithm 4 with the coder parameters of Sec. 4.3:
//      a 64-bit code, nine 7-bit ASCII characters masked with 0x7F, or four
//      16-bit UTF-16 units);
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

// The husky code of one string (Algorithm 4 with the coder parameters of
// Sec. 4.3), written from its definition as fixed bit positions: the first
// m elements each own a w-bit field, the first one most significant, and a
// missing element's field is zero:
//     code = sum over j < min(len, m) of (e_j & mask) << w * (m - 1 - j).
// ASCII: m = 9 fields of w = 7 bits (bits 62..0), mask 0x7F.  UTF-16: m = 4
// fields of w = 16 bits (all 64 bits), every bit of a unit kept.  Full bytes
// (the 8-bit member of the family of alphabet-dependent coders that Sec. 3.2
// discusses -- the wider the alphabet, the fewer characters fit): m = 8
// fields of w = 8 bits, every bit kept, so the code is the first eight bytes
// read as a big-endian number and is monotone for every byte value.
struct Coder {
    int m;          // elements coded
    int w;          // bits per element
    uint64_t mask;  // bits of an element that are kept
};
const Coder ASCII7 = {9, 7, 0x7F};
const Coder UTF16 = {4, 16, 0xFFFF};
const Coder BYTES8 = {8, 8, 0xFF};

template <typename Elem>
uint64_t husky_code(const Elem* s, uint64_t len, const Coder& c) {
    uint64_t code = 0;
    for (uint64_t j = 0; j < len && j < (uint64_t)c.m; ++j)
        code |= ((uint64_t)s[j] & c.mask) << (c.w * (c.m - 1 - (int)j));
    return code;
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
//            shifted right by one bit), 3 = null coder (every code 0),
//        4 = full bytes (8 chars x 8 bits, byte strings of any values).

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
            codes[i] = husky_code(s, len, ASCII7);
            for (uint64_t j = 0; j < len && j < (uint64_t)ASCII7.m; ++j)
                if (s[j] >= 0x80) {
                    ++violations;
                    break;
                }
        } else if (coder == 4) {
            codes[i] = husky_code((const uint8_t*)elems + offsets[i], len, BYTES8);
        } else if (coder == 1 || coder == 2) {
            const uint16_t* s = (const uint16_t*)elems + offsets[i];
            uint64_t c = husky_code(s, len, UTF16);
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

// Step 3 as the paper writes it (Sec. 3.1 Step 3, the final Timsort over the
// whole array, needed when the coder may invert two objects -- the lossy
// and deliberately mis-coded coders of Sec. 3.2 and the Appendix): idx holds
// any order of the strings (typically the result of sorting by such codes)
// and becomes the stable sorting permutation.  Written as its definition: a
// sort by (string, original index), which is a total order, so the result is
// unique whatever order idx arrived in.
void oracle_fixup_global(int elem_bytes, const void* elems, const uint64_t* offsets, uint64_t n,
                         uint32_t* idx) {
    auto by_string_then_index = [&](uint32_t a, uint32_t b) {
        bool lt = elem_bytes == 1 ? string_less((const uint8_t*)elems, offsets, a, b)
                                  : string_less((const uint16_t*)elems, offsets, a, b);
        bool gt = elem_bytes == 1 ? string_less((const uint8_t*)elems, offsets, b, a)
                                  : string_less((const uint16_t*)elems, offsets, b, a);
        return lt || (!gt && a < b);
    };
    std::sort(idx, idx + n, by_string_then_index);
}

// Algorithm 1 with caller-given codes of any quality (a lossy or non-monotone
// coder): Step 2 is the stable sort of (codes[i], i) by code, Step 3 the
// global pass above.
void oracle_sort_lossy(int elem_bytes, const void* elems, const uint64_t* offsets, uint64_t n,
                       const uint64_t* codes, uint32_t* perm) {
    std::vector<uint64_t> c(codes, codes + n);
    for (uint64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
    sort_pairs(c.data(), perm, n);
    oracle_fixup_global(elem_bytes, elems, offsets, n, perm);
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
