/*
 * husky.h -- C ABI of the MI355X (gfx950) Huskysort library, libhusky.so.
 *
 * Huskysort (Hillyard, Liaozheng, K R; Sec. 3.1 "Overview", Algorithm 1)
 * sorts objects that are expensive to compare in three steps:
 *   1. code every object into a 64-bit "husky code" that never inverts the
 *      order of two objects (Sec. 3.2; for strings, stringToLong,
 *      Algorithm 4, with the constants of Sec. 4.3);
 *   2. sort the (code, index) pairs with cheap integer comparisons while the
 *      indices travel with the codes (the "object swap", Sec. 3.1 Step 2);
 *   3. remove the inversions that remain, which can only sit among equal
 *      codes (the role of the final Timsort pass, Sec. 3.1 Step 3).
 * This library runs all three steps on the GPU: a coalesced encode kernel,
 * a stable LSD radix sort of (u64 code, u32 index) pairs, and a fix-up that
 * finds runs of equal codes and sorts each run by the full comparator at
 * wave, workgroup or device level depending on its length.
 *
 * Result.  Every sort returns the STABLE sorting permutation `perm`:
 * s[perm[k]] <= s[perm[k+1]] under the full comparator, and equal strings
 * appear in ascending index, so the answer is unique.  Comparators:
 *   HUSKY_CODER_ASCII7 -- strings of bytes, unsigned byte-lexicographic
 *     order, a proper prefix first.  The 7-bit code masks each of the first
 *     nine bytes with 0x7F (Algorithm 4), which preserves order only for
 *     bytes < 0x80 there; bytes >= 0x80 are allowed from the tenth byte on.
 *   HUSKY_CODER_UTF16 -- strings of 16-bit code units, code-unit
 *     lexicographic order (the order of Java's String.compareTo, which the
 *     paper's final pass uses), a proper prefix first.  The code keeps all
 *     64 bits of the first four units and is compared unsigned.
 *   HUSKY_CODER_BYTES8 -- strings of bytes of ANY value (binary keys, UTF-8
 *     text, whose byte order is code point order), unsigned
 *     byte-lexicographic order, a proper prefix first.  The code is the first
 *     eight bytes read big-endian: the 8-bit member of the alphabet-dependent
 *     coders of Sec. 3.2, monotone for every byte value, one character
 *     shorter than the 7-bit coder.
 *
 * Layout.  `elems` holds all strings back to back: uint8 elements for
 * ASCII7 and BYTES8, uint16 for UTF16.  `offsets` is uint64[n + 1] in ELEMENTS with
 * offsets[0] = 0, non-decreasing; string i is elems[offsets[i] ..
 * offsets[i+1]).  Empty strings and NUL elements are allowed.  n < 2^32.
 *
 * Memory.  Every pointer argument is a DEVICE pointer owned by the caller,
 * unless marked "host".  The library allocates no device memory: scratch
 * space comes from the caller's workspace `ws`, at least
 * husky_workspace_bytes(n, n_segs) bytes, 256-byte aligned.  The first 24
 * bytes of the workspace are the device status block (husky_device_status
 * below), written by every call that takes `ws`.
 *
 * Streams and errors.  Calls are enqueued on `stream` (a hipStream_t; NULL
 * is the default stream) and return after enqueueing.  Argument errors are
 * detected on the host and returned synchronously; nothing is enqueued then.
 * Conditions that only the device can see (an ASCII7 byte >= 0x80 among the
 * first nine bytes) are recorded in the device status block; read it after
 * synchronizing the stream.  With such a violation `perm` is unspecified.
 * No call synchronizes `stream` with the host, except husky_learned_fit
 * (once, to size its training loop) and the sorts when a caller asks for
 * adaptive refinement rounds (husky_tuning.max_rounds).
 * Side streams.  For 2^21 strings or more, parts of Step 3 (the run-local
 * tiers and, beside them, the device-wide round; and parts of the learned
 * form's bucket sort) that touch disjoint data run on two streams
 * the library creates once per device (default priority, kept until the
 * process ends), forked from and joined back into `stream` through events,
 * so the call still behaves as work enqueued on `stream` alone.  They are
 * created on the first such call that is not being captured into a graph;
 * a captured call before that keeps everything on `stream`.  Calls on one
 * device share them: calls from several host threads stay correct but
 * serialize there, and a graph capture must not overlap another call.
 */
#ifndef HUSKY_H
#define HUSKY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HUSKY_OK = 0,
    HUSKY_ERR_ARG = 1,         /* bad argument: null pointer, n >= 2^32, bad coder or bits */
    HUSKY_ERR_DOMAIN = 2,      /* (device status only) ASCII7 byte >= 0x80 in the first nine */
    HUSKY_ERR_WORKSPACE = 3,   /* workspace missing, too small or misaligned */
    HUSKY_ERR_HIP = 4,         /* a HIP runtime call failed */
    HUSKY_ERR_UNSUPPORTED = 5, /* tuning value outside the compiled variants */
    HUSKY_ERR_UNRESOLVED = 6,  /* (device status only) groups still tied after
                                * tuning.max_rounds fixed rounds: perm not final */
    HUSKY_ERR_TOO_LARGE = 7    /* husky_sort_noalloc: n above HUSKY_NOALLOC_MAX_STRINGS */
} husky_status;

typedef enum {
    HUSKY_CODER_ASCII7 = 0, /* uint8 elements, 9 chars x 7 bits, bits 62..0 */
    HUSKY_CODER_UTF16 = 1,  /* uint16 elements, 4 units x 16 bits, bits 63..0 */
    HUSKY_CODER_BYTES8 = 2  /* uint8 elements of any value, 8 x 8 bits, bits 63..0 */
} husky_coder;

/* Device status block at the start of the workspace (device memory). */
typedef struct {
    uint32_t domain_violations; /* ASCII7 strings with a byte >= 0x80 among the first nine */
    uint32_t large_rounds;      /* device-wide refinement rounds the last fix-up ran */
    uint32_t runs_fixed;        /* equal-key runs (length >= 2) the last fix-up visited */
    uint32_t unresolved;        /* groups left tied after max_rounds fixed rounds (else 0) */
    uint32_t overflow_buckets;  /* learned form: buckets above the LDS sort's 8,192 keys */
    uint32_t overflow_keys;     /* learned form: strings in those buckets */
} husky_device_status;

/* Launch tuning.  Zero in a field selects the library default.  The values
 * the autotuner picks are stored per (device, coder, size band).
 *   radix_bits -- digit width of every LSD pass: 6, 7 or 8;
 *   tile_items -- keys per thread in a radix tile (256 threads): 8, 12 or 16;
 *   t_small    -- equal-code runs of at most this many strings are sorted by
 *                 one wavefront (2..64);
 *   t_medium   -- runs of at most this many by one workgroup in LDS
 *                 (t_small < t_medium <= 4096, default 1024) with a bitonic
 *                 sort per round; runs of up to 8,192 by one workgroup that
 *                 keeps the run in LDS for all its rounds (a radix sort per
 *                 round); longer runs device-wide (a group of at most one
 *                 radix tile is then sorted in LDS by the segmented radix
 *                 sort);
 *   max_rounds -- device-wide refinement rounds (for runs of equal codes
 *                 longer than the LDS tier's 8,192 strings).  A round first
 *                 finds the position where the members of each group first
 *                 differ and keys the group on the chunk of C elements that
 *                 holds it (chunks start at m + C*j: ASCII 9 + 7j bytes,
 *                 UTF-16 4 + 3j units), so no round is spent on chunks all
 *                 members share, and a group of identical strings is done
 *                 in the round that meets it.
 *                 0 (default): one round launched without any host
 *                 synchronisation, then every group still tied is finished by
 *                 one workgroup per group running its remaining rounds in
 *                 global memory: the call never synchronizes, can be
 *                 captured into a HIP graph, and perm is always final.
 *                 k in 1..4096: exactly k rounds, no host synchronisation;
 *                 groups still tied after them are counted in
 *                 husky_device_status.unresolved and then perm is not final.
 *                 HUSKY_ROUNDS_ADAPTIVE: the host reads the work counts once
 *                 per round (synchronizing the stream) and runs rounds until
 *                 nothing is tied -- for inputs whose long runs still hold
 *                 long groups after a round (groups that split in few,
 *                 large parts at one position after another). */
#define HUSKY_ROUNDS_ADAPTIVE 0xFFFFFFFFu
typedef struct {
    int32_t radix_bits;
    int32_t tile_items;
    uint32_t t_small;
    uint32_t t_medium;
    uint32_t max_rounds;
} husky_tuning;

/* Workspace bytes that every call below needs for n strings in n_segs
 * instances (n_segs = 1 for a single sort). */
size_t husky_workspace_bytes(uint64_t n, uint64_t n_segs);

/* Step 1 -- Algorithm 4 (stringToLong) over every string, Algorithm 2/3.
 * codes[i] = sum over j < min(len_i, m) of (e_ij & mask) << w*(m-1-j):
 * ASCII7 m = 9, w = 7, mask 0x7F; UTF16 m = 4, w = 16, no mask; BYTES8 m = 8,
 * w = 8, no mask.
 * idx_or_null: if not NULL receives idx[i] = i (the index array that
 *   travels with the codes through Step 2).
 * status: device uint32 that is INCREMENTED by the number of ASCII7 strings
 *   holding a byte >= 0x80 among their first nine bytes (may be NULL; the
 *   caller zeroes it).
 * Errors: HUSKY_ERR_ARG for null elems/offsets/codes with n > 0. */
husky_status husky_encode(husky_coder coder, const void* elems, const uint64_t* offsets,
                          uint64_t n, uint64_t* codes, uint32_t* idx_or_null,
                          uint32_t* status, void* stream);

/* Step 2 -- stable sort of the pairs (codes[i], idx[i]) by codes[i], in place,
 * comparing only bits [begin_bit, end_bit) of each code (0 <= begin_bit <
 * end_bit <= 64); equal keys keep their input order.  LSD radix with
 * tuning->radix_bits per pass; passes whose digit is the same in every key are
 * skipped.  tuning may be NULL.  Errors: HUSKY_ERR_ARG, HUSKY_ERR_WORKSPACE,
 * HUSKY_ERR_UNSUPPORTED. */
husky_status husky_sort_pairs(uint64_t* codes, uint32_t* idx, uint64_t n, int begin_bit,
                              int end_bit, void* ws, size_t ws_bytes,
                              const husky_tuning* tuning, void* stream);

/* Step 3 -- given codes sorted ascending with idx carried along (the output
 * of Step 2), re-sort every run of equal codes by the full comparator so that
 * idx becomes the stable sorting permutation.  Runs never cross instance
 * boundaries: seg_offsets_or_null is uint64[n_segs + 1] string offsets of
 * independent instances (NULL with n_segs = 1 for one instance).  A run whose
 * members all have the same length <= m (9 ASCII, 8 BYTES8, 4 UTF-16) holds
 * identical strings already in index order and is left as it is.  idx is updated in
 * place; sorted_codes is read only.  Errors: HUSKY_ERR_ARG,
 * HUSKY_ERR_WORKSPACE, HUSKY_ERR_UNSUPPORTED, HUSKY_ERR_HIP. */
husky_status husky_fixup(husky_coder coder, const void* elems, const uint64_t* offsets,
                         uint64_t n, const uint64_t* sorted_codes, uint32_t* idx,
                         const uint64_t* seg_offsets_or_null, uint64_t n_segs, void* ws,
                         size_t ws_bytes, const husky_tuning* tuning, void* stream);

/* Step 3 as a general refinement step (recursive in-run Huskysort): given any
 * keys sorted ascending with idx carried along, re-sort every run of equal
 * keys by the full comparator, in place on idx.  The caller states what a run
 * is known to share: every member of a run agrees with the others on its
 * first min(len, shared_elems) elements (0 <= shared_elems <= 15; 0 assumes
 * nothing, so any keys work -- e.g. the result of a coarser sort; husky
 * codes of `coder` satisfy it with shared_elems = m, which is husky_fixup).
 * Each round then codes the next 7 bytes (3 UTF-16 units) of every member of
 * a still-tied group, from element shared_elems on, as a new key and sorts the
 * group by it -- the method applied again inside the run -- until no group
 * is tied.  Runs, instances, workspace, tuning and errors as husky_fixup
 * (plus HUSKY_ERR_ARG for shared_elems > 15).  If a run breaks the stated
 * sharing, idx is unspecified. */
husky_status husky_refine(husky_coder coder, const void* elems, const uint64_t* offsets,
                          uint64_t n, const uint64_t* sorted_keys, uint32_t* idx,
                          const uint64_t* seg_offsets_or_null, uint64_t n_segs,
                          uint32_t shared_elems, void* ws, size_t ws_bytes,
                          const husky_tuning* tuning, void* stream);

/* Algorithm 1 end to end on the GPU: encode, stable pair sort, fix-up.
 * perm receives uint32[n], the stable sorting permutation.  The device status
 * block in ws reports domain violations.  tuning may be NULL.
 * For ASCII7 the pair sort's key is code << 1 | f, f = 0 exactly when the
 * string has at most nine bytes and none is NUL (a per-string form of the
 * perfect coding of Algorithm 3 and Sec. 3.4; still monotone): runs of keys
 * with f = 0 hold identical strings and are not visited, so runs_fixed counts
 * only the others.  When f would cost a radix pass it is left out of the
 * digits and every run is visited.  The permutation is the same either way.
 * Errors: as husky_fixup. */
husky_status husky_sort(husky_coder coder, const void* elems, const uint64_t* offsets,
                        uint64_t n, uint32_t* perm, void* ws, size_t ws_bytes,
                        const husky_tuning* tuning, void* stream);

/* husky_sort without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The scratch space
 * is a fixed array of HUSKY_NOALLOC_SCRATCH_BYTES (64 MiB) in the library's
 * device memory, one copy per device, held until the process ends; it
 * covers up to HUSKY_NOALLOC_MAX_STRINGS strings (n above that:
 * HUSKY_ERR_TOO_LARGE, nothing enqueued).  Same arguments, result, errors
 * and stream behaviour as husky_sort otherwise; the device status block is
 * the first 24 bytes of that array, read with husky_noalloc_status.
 * Every call on one device uses the same array and leaves its contents
 * there: calls that overlap in time on one device (other streams or host
 * threads) race and give unspecified results -- order them. */
#define HUSKY_NOALLOC_SCRATCH_BYTES (64u << 20)
#define HUSKY_NOALLOC_MAX_STRINGS (1u << 20)
husky_status husky_sort_noalloc(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, uint32_t* perm, const husky_tuning* tuning,
                                void* stream);
/* Copies the status block of the current device's no-allocation scratch to
 * *out (host), after synchronizing stream (on which the sort ran).
 * Errors: HUSKY_ERR_ARG, HUSKY_ERR_HIP. */
husky_status husky_noalloc_status(husky_device_status* out, void* stream);

/* Batched form: n_segs independent instances sorted in the same launches.
 * n is the total number of strings; seg_offsets is uint64[n_segs + 1]
 * (device) string offsets, seg_offsets[0] = 0, non-decreasing,
 * seg_offsets[n_segs] = n.  perm[k] for k in instance j's range is a
 * GLOBAL string index inside that range: instance j's slice of perm is the
 * stable sorting permutation of its own strings.  Radix tiles never cross an
 * instance boundary and neither do runs.  Errors: as husky_fixup. */
husky_status husky_sort_batched(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, const uint64_t* seg_offsets, uint64_t n_segs,
                                uint32_t* perm, void* ws, size_t ws_bytes,
                                const husky_tuning* tuning, void* stream);

/* Exactness check on the device.  perm (uint32[n]) is the stable sorting
 * permutation -- of every instance's range when seg_offsets_or_null (uint64
 * [n_segs + 1]) is given -- iff the check finds no violation: every entry a
 * distinct index of its own instance, every adjacent pair inside an instance
 * ordered by the full comparator with equal strings in ascending index
 * (Sec. 3.2: the final pass must leave no inversion).  *violations (device
 * uint32) receives the number of failing positions.  ws needs (n + 31) / 32 *
 * 4 bytes (a bitmap).  Asynchronous on stream.  Errors: HUSKY_ERR_ARG,
 * HUSKY_ERR_WORKSPACE, HUSKY_ERR_HIP. */
husky_status husky_check_perm(husky_coder coder, const void* elems, const uint64_t* offsets,
                              uint64_t n, const uint64_t* seg_offsets_or_null, uint64_t n_segs,
                              const uint32_t* perm, void* ws, size_t ws_bytes,
                              uint32_t* violations, void* stream);

/* Kernel timing (diagnostics).  husky_profile_begin() starts bracketing
 * every launch of the library with a pair of HIP events recorded on that
 * launch's stream; husky_profile_end() waits for them and writes, for each
 * kernel class c < n_classes, the summed milliseconds ms[c] and the launch
 * count launches[c] (host arrays), then stops profiling.  Classes:
 * 0 encode, 1 radix varying-bit reduction and pass masks, 2 radix digit
 * counts and their scans (of the sort of the codes; class 16 for the
 * device-wide fix-up's), 3 radix scatter pass, 4 radix copy-back,
 * 5 single-tile LDS sort, 6 run detection, 7 wavefront fix-up, 8 workgroup
 * fix-up, 9 device-wide refinement keys, 10 segment setup, 11 radix scatter
 * pass of the device-wide fix-up (class 3 counts only the sort of the
 * codes), 12 learned bucket scatter pass, 13 learned bucket bounds (the
 * learned form's bucket ids are computed by the encode kernel, class 0),
 * 14 LDS-resident fix-up of runs longer than t_medium and at most 8,192,
 * 15 the full stable pass of the lossy-coder sort (husky_fixup_global),
 * 16 radix digit counts and scans of the device-wide fix-up.
 * Not for use during graph capture.
 * Returns HUSKY_OK or HUSKY_ERR_HIP. */
void husky_profile_begin(void);
int husky_profile_end(double* ms, uint32_t* launches, int n_classes);
/* Bracket only the classes whose bit is set in class_mask (default: all), so
 * that timing one kernel class barely perturbs the others. */
void husky_profile_select(uint32_t class_mask);

/* ---------------------------------------------------------------------
 * Lossy coders.  Sec. 3.2 allows a coder that inverts two objects with some
 * probability p (x > y but code(x) <= code(y)), and the Appendix sorts with
 * deliberately mis-coded objects; Step 3 is then the paper's full stable pass
 * over the whole array (Sec. 3.1 Step 3), which run-local fix-up cannot
 * replace.  Here that pass is a natural merge sort: the array's maximal
 * ascending runs are merged in pairs, level by level, every element placed
 * by binary search in its partner run, comparing (string, original index) --
 * a total order, so the result is the unique stable sorting permutation for
 * ANY input order.  Its cost grows with the log of the number of runs, so a
 * nearly sorted array is cheap.  It never synchronizes with the host. */

/* Workspace bytes of husky_fixup_global for n strings. */
size_t husky_global_workspace_bytes(uint64_t n);
/* The full stable pass: idx (device uint32[n]) holds the strings in any order
 * (e.g. sorted by lossy codes) and becomes the stable sorting permutation.
 * Errors: HUSKY_ERR_ARG, HUSKY_ERR_WORKSPACE, HUSKY_ERR_HIP. */
husky_status husky_fixup_global(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, uint32_t* idx, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes of husky_sort_lossy for n strings. */
size_t husky_lossy_workspace_bytes(uint64_t n);
/* Algorithm 1 with the caller's codes (device uint64[n], from any coder, even
 * one that inverts strings): Step 2 sorts (codes[i], i) stably, Step 3
 * re-sorts every run of equal codes by the full comparator from the first
 * element (the codes promise no shared prefix) and then runs the full stable
 * pass.  perm receives the stable sorting permutation whatever the codes.
 * `coder` only selects the element type and comparator (ASCII7 and BYTES8:
 * bytes, UTF16: units).  Errors: as husky_sort. */
husky_status husky_sort_lossy(husky_coder coder, const void* elems, const uint64_t* offsets,
                              uint64_t n, const uint64_t* codes, uint32_t* perm, void* ws,
                              size_t ws_bytes, const husky_tuning* tuning, void* stream);

/* ---------------------------------------------------------------------
 * Other object types.  The paper names more types that are costly to
 * compare and that a husky code speeds up: date-times (a perfect coder for
 * nanosecond resolution over 128 years, Sec. 3.2), Integer, Long, Double,
 * BigInteger and BigDecimal, and tuples (Sec. 6).  Records (device bytes):
 *   INT32, INT64, FLOAT64 -- little-endian values, 4 / 8 / 8 bytes each;
 *   DATETIME -- 16 bytes: int32 year, uint8 month, day, hour, minute,
 *     second, 3 pad bytes, uint32 nano (little-endian); compared field by
 *     field; valid fields: month 1..12, day 1..31, hour <= 23, minute <= 59,
 *     second <= 59, nano < 10^9 (others are domain violations);
 *   BIGINT -- two's-complement big-endian bytes of any length up to 32,767
 *     (an empty record is 0), compared by value;
 *   DECIMAL -- int32 scale (little-endian) then the unscaled value as
 *     two's-complement big-endian bytes (at most 16; none = 0): value =
 *     unscaled x 10^-scale, |scale| <= 16,000; compared by value, so 1.5 and
 *     1.50 are equal (Java's BigDecimal.compareTo);
 *   TUPLE -- int64 (little-endian) then a byte string; compared by the
 *     string (unsigned bytes, a proper prefix first), then the integer.
 * Variable-length types take offsets (uint64[n + 1], bytes) like strings.
 * FLOAT64 follows Java's Double.compare: -inf < ... < -0.0 < 0.0 < ... <
 * inf < NaN, every NaN equal.  Ties keep index order (stable).
 * Codes (husky_encode_typed): INT32 (x + 2^31) << 32; INT64 x + 2^63;
 * FLOAT64 the IEEE bits with the sign flipped for positives and every bit
 * flipped for negatives (NaN made canonical) -- perfect codes, so the sort is
 * Steps 1 and 2 only; DATETIME 1 + (year - base_year) << 56 | month << 52 |
 * day << 47 | hour << 42 | minute << 36 | second << 30 | nano for years in
 * [base_year, base_year + 128) (perfect there), 0 below, 2^63 + 1 above;
 * BIGINT, DECIMAL, TUPLE the first eight bytes (big-endian) of an
 * order-preserving byte key (bigint: a 2-byte sign-and-length head and the
 * shortest two's-complement bytes; decimal: sign class, decimal exponent,
 * significant digits two per byte; tuple: the string with each 00 written
 * 00 FF, 00 00, the integer + 2^63 big-endian).  Step 3 compares those keys
 * (13-byte field keys for date-times) with the full-byte fix-up. */
typedef enum {
    HUSKY_TYPE_INT32 = 0,
    HUSKY_TYPE_INT64 = 1,
    HUSKY_TYPE_FLOAT64 = 2,
    HUSKY_TYPE_DATETIME = 3,
    HUSKY_TYPE_BIGINT = 4,
    HUSKY_TYPE_DECIMAL = 5,
    HUSKY_TYPE_TUPLE = 6
} husky_type;

/* Workspace bytes of husky_sort_typed for n records of record_bytes bytes in
 * all (the size of the records buffer). */
size_t husky_typed_workspace_bytes(husky_type type, uint64_t n, uint64_t record_bytes);

/* Step 1 for typed records: codes[i] (device uint64[n]) = the husky code of
 * record i.  offsets_or_null: uint64[n + 1] byte offsets for BIGINT, DECIMAL
 * and TUPLE, NULL for the fixed-width types.  status (device, may be NULL) is
 * INCREMENTED by the number of out-of-domain records.  Errors: HUSKY_ERR_ARG. */
husky_status husky_encode_typed(husky_type type, const void* records, const uint64_t* offsets_or_null,
                                uint64_t n, int32_t base_year, uint64_t* codes, uint32_t* status,
                                void* stream);

/* Huskysort of typed records: perm receives the stable sorting permutation
 * under the type's comparator.  record_bytes is the size of the records
 * buffer (it bounds the keys' workspace).  base_year: the date-time window's
 * first year (ignored by the other types).  The device status block reports
 * out-of-domain records (perm is then unspecified).  Errors: HUSKY_ERR_ARG,
 * HUSKY_ERR_WORKSPACE, HUSKY_ERR_UNSUPPORTED, HUSKY_ERR_HIP. */
husky_status husky_sort_typed(husky_type type, const void* records, const uint64_t* offsets_or_null,
                              uint64_t n, uint64_t record_bytes, int32_t base_year, uint32_t* perm,
                              void* ws, size_t ws_bytes, const husky_tuning* tuning, void* stream);

/* ---------------------------------------------------------------------
 * Learned-CDF form (an extension of the method, not part of the paper).
 *
 * A model maps every code to one of HUSKY_LEARNED_BUCKETS buckets by a
 * function that never decreases as the code grows, so sorting the pairs
 * becomes: bucket ids, a stable scatter of (code, index) into bucket order,
 * and independent sorts of the buckets -- in LDS for buckets of at most 8,192
 * keys (by code, then by the first refinement key inside runs of equal codes,
 * so most of Step 3 happens there too), by the multi-tile radix passes for
 * larger ("overflow") buckets.  Step 3 then runs on what is still tied.  Since equal codes always
 * share a bucket and buckets are in code order, the permutation is exactly
 * husky_sort's whatever the model's quality; a poor model only costs time.
 *
 * The bucket function, for a model fitted on a sample of codes:
 *   - clamp the code to [lo, hi], the sample's extremes; W = its 24 bits
 *     right below the common prefix of lo and hi (a "cell"), x = W / 2^24;
 *   - cells holding at least two buckets' worth of the sample and at least
 *     16 sample keys ("dense cells", unless HUSKY_LEARNED_NO_DENSE) take their sample share of the
 *     buckets exactly; the network models the cumulative distribution of the
 *     remaining sample keys over x:  F(W) = (dense sample keys in cells
 *     below W + (other sample keys) * net(x)) / sample size;
 *   - LUT[W] = F(W) in 0.32 fixed point for all 2^24 + 1 cell starts, made
 *     non-decreasing by a running maximum (whatever the network computes),
 *     LUT[0] = 0, LUT[2^24] = 2^32 - 1; cell W owns the buckets
 *     [LUT[W] * B >> 32, LUT[W + 1] * B >> 32);
 *   - a cell owning k >= 2 buckets splits its codes by k - 1 equal-depth
 *     splitters taken from the cell's sorted sample codes; a table over the
 *     bits right below the splitters' common prefix ("sub-cells") narrows
 *     each key's search to the splitters of its sub-cell.
 * The network: 1 -> 64 -> 64 -> 1, ReLU after both hidden layers, every
 * weight softplus(raw parameter) > 0 (so it never decreases in x), output
 * clamped to [0, 1]; trained in FP32 by mean squared error against the
 * targets (rank + 0.5) / count with Adam, on the GPU.
 */
#define HUSKY_LEARNED_BUCKETS 65536u
#define HUSKY_LEARNED_HIDDEN 64
#define HUSKY_LEARNED_NPARAM 4353 /* v1[64] b1[64] v2[64][64] b2[64] v3[64] b3 */
#define HUSKY_LEARNED_CELLS (1u << 24)
#define HUSKY_LEARNED_NO_DENSE 1u /* husky_learned_params.flags: the network alone */

typedef enum {
    HUSKY_LEARNED_MONOTONE = 0,      /* the trained monotone network (default) */
    HUSKY_LEARNED_UNCONSTRAINED = 1, /* raw weights, trained: not monotone (tests) */
    HUSKY_LEARNED_EQUAL_WIDTH = 2,   /* no network: net(x) = x (equal-width cells) */
    HUSKY_LEARNED_UNTRAINED = 3,     /* the monotone network at its initialisation */
    HUSKY_LEARNED_CONSTANT = 4       /* no network: net(x) = 0 (tests) */
} husky_learned_mode;

/* Fit parameters; a zero field selects the default. */
typedef struct {
    double sample_frac; /* fraction of the strings sampled, (0, 1]; default 0.01 */
    uint64_t seed;      /* sample and initialisation seed; default 1 */
    uint32_t epochs;    /* default (0): enough for at least 150 Adam steps, at most 200 */
    uint32_t batch;     /* samples per Adam step; default 65536 */
    float lr;           /* Adam step size; default 0.02 */
    uint32_t mode;      /* husky_learned_mode */
    uint32_t flags;     /* HUSKY_LEARNED_NO_DENSE */
    uint32_t reserved;
} husky_learned_params;

/* First bytes of the model buffer (device memory). */
typedef struct {
    uint64_t lo, hi;     /* sample extremes */
    uint32_t cp;         /* common-prefix bits of lo and hi (64 if equal) */
    uint32_t buckets;    /* B */
    uint32_t mode;       /* husky_learned_mode */
    uint32_t sample;     /* sample size S */
    uint32_t steps;      /* Adam steps taken */
    float last_loss;     /* mean loss of the last epoch */
    uint32_t heavy;      /* cells owning two or more buckets */
    uint32_t dense;      /* dense cells */
    uint32_t dense_keys; /* sample keys in dense cells */
    uint32_t trained;    /* sample keys the network was trained on */
    uint32_t flags;
    uint32_t pad[5];
} husky_learned_header;

/* Parts of the model buffer, for husky_learned_offset. */
typedef enum {
    HUSKY_LM_HEADER = 0,    /* husky_learned_header */
    HUSKY_LM_PARAMS = 1,    /* float[NPARAM], raw parameters */
    HUSKY_LM_ADAM_M = 2,    /* float[NPARAM] */
    HUSKY_LM_ADAM_V = 3,    /* float[NPARAM] */
    HUSKY_LM_LUT = 4,       /* uint32[2^24 + 1] */
    HUSKY_LM_SPLITTERS = 5, /* uint64[B] */
    HUSKY_LM_DENSE = 6,     /* uint32[B / 2] dense cells, ascending */
    HUSKY_LM_DENSE_CUM = 7, /* uint32[B / 2 + 1] dense sample keys before each */
    HUSKY_LM_SUBTAB = 8,    /* uint16[16 B]: per heavy cell at 16 * first bucket: header {u16 P,
                             * u16 s, u32 0, u64 prefix}, then 2^s splitter counts, one per
                             * sub-cell (the s bits below the splitters' P-bit common prefix) */
    HUSKY_LM_CELLINFO = 9   /* uint64[2^24]: per cell, first bucket | end bucket << 16, and for
                             * a heavy cell P << 32 | s << 39 | the prefix bits below the cell
                             * << 44 (bit 63: read P, s and prefix from its subtab header) */
} husky_learned_part;

/* Size of the model buffer, and the byte offset of each part in it (SIZE_MAX
 * for an unknown part). */
size_t husky_learned_model_bytes(void);
size_t husky_learned_offset(int part);

/* Workspace bytes of husky_learned_fit and husky_sort_learned for n strings. */
size_t husky_learned_workspace_bytes(uint64_t n);

/* Fit the model: draw S = ceil(sample_frac * n) string indices by a seeded
 * counter-based hash (with replacement), code them with Step 1, sort the
 * sample codes (Step 2), find the dense cells, train the network on the
 * other sample keys, then build the LUT and the splitters.  `model` (device,
 * husky_learned_model_bytes(), 256-aligned) is overwritten.  Synchronizes
 * `stream` once (to size the training loop).  params may be NULL.  Domain
 * violations among the sampled strings are counted in the status block.
 * Errors: HUSKY_ERR_ARG (n == 0, bad params), HUSKY_ERR_WORKSPACE,
 * HUSKY_ERR_HIP. */
husky_status husky_learned_fit(husky_coder coder, const void* elems, const uint64_t* offsets,
                               uint64_t n, const husky_learned_params* params, void* model,
                               size_t model_bytes, void* ws, size_t ws_bytes, void* stream);

/* Sort with a fitted model.  perm receives the stable sorting permutation,
 * identical to husky_sort's.  The status block reports domain violations and
 * overflow_buckets / overflow_keys.  With tuning->max_rounds == 0 the call
 * synchronizes like husky_sort when long equal-code runs exist.
 * Errors: as husky_sort. */
husky_status husky_sort_learned(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, const void* model, uint32_t* perm, void* ws,
                                size_t ws_bytes, const husky_tuning* tuning, void* stream);

/* The bucket function alone: bucket[i] (uint16, device) = the bucket of
 * string i's code under the fitted model (the ids husky_sort_learned sorts
 * by; also the unit a sort would be range-partitioned by across devices).
 * status as in husky_encode (may be NULL).  Errors: HUSKY_ERR_ARG, HUSKY_ERR_HIP. */
husky_status husky_learned_buckets(husky_coder coder, const void* elems, const uint64_t* offsets,
                                   uint64_t n, const void* model, uint16_t* bucket,
                                   uint32_t* status, void* stream);

/* The training kernel alone, for checking it: grad (float[NPARAM + 1]) gets
 * the gradient of the mean squared error of the network (monotone != 0:
 * softplus weights; 0: raw weights) over the `count` samples (x[i], y[i])
 * with respect to the raw parameters, and grad[NPARAM] the sum of squared
 * errors.  ws needs husky_mlp_grad_workspace_bytes(count).
 * Errors: HUSKY_ERR_ARG, HUSKY_ERR_WORKSPACE, HUSKY_ERR_HIP. */
size_t husky_mlp_grad_workspace_bytes(uint32_t count);
husky_status husky_mlp_grad(const float* params, const float* x, const float* y, uint32_t count,
                            int monotone, float* grad, void* ws, size_t ws_bytes, void* stream);

/* The inference kernel alone, for checking it: lut (device uint32[2^24 + 1])
 * receives the table the fit builds -- F(W) of the network with raw
 * parameters `params` (device float[NPARAM], layout as HUSKY_LM_PARAMS) over
 * the header and dense cells of the fitted `model` (read only), in 0.32
 * fixed point, made non-decreasing by a running maximum.  mode: a
 * husky_learned_mode; MONOTONE and UNTRAINED evaluate the softplus-weight
 * network, UNCONSTRAINED the raw-weight one, EQUAL_WIDTH and CONSTANT ignore
 * params.  ws (device) needs husky_learned_lut_workspace_bytes() bytes.
 * Asynchronous on stream.  Errors: HUSKY_ERR_ARG, HUSKY_ERR_WORKSPACE,
 * HUSKY_ERR_HIP. */
size_t husky_learned_lut_workspace_bytes(void);
husky_status husky_learned_eval_lut(const float* params, int mode, const void* model, uint32_t* lut,
                                    void* ws, size_t ws_bytes, void* stream);

/* Static text for a status code (host). */
const char* husky_status_string(husky_status s);

#ifdef __cplusplus
}
#endif

#endif /* HUSKY_H */
