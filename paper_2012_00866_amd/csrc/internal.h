// Host-side interfaces between the kernel files and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.h"

namespace husky {

// ---- profile.hip: per-launch HIP-event timing, off unless husky_profile_begin ran
enum ProfClass {
    P_ENCODE = 0, P_VARY = 1, P_COUNT_SCAN = 2, P_SCATTER = 3, P_COPY_BACK = 4, P_TILE_SORT = 5,
    P_RUNS = 6, P_FIX_SMALL = 7, P_FIX_MEDIUM = 8, P_LARGE_KEYS = 9, P_SETUP = 10,
    P_SCATTER_FIX = 11, P_BUCKET = 12, P_BUCKET_BOUNDS = 13, P_FIX_LDS = 14, P_MERGE = 15,
    P_COUNT_SCAN_FIX = 16, P_NUM = 17
};
bool prof_on();
class ProfScope {
  public:
    ProfScope(int cls, hipStream_t s);
    // For one launch made with hipExtLaunchKernelGGL: *start / *stop receive
    // the scope's events (null when the class is not timed), for the launch
    // to record with its dispatch, which times the kernel itself rather than
    // the host's enqueueing around it.
    ProfScope(int cls, hipStream_t s, hipEvent_t* start, hipEvent_t* stop);
    ~ProfScope();
  private:
    int cls_;
    hipStream_t s_;
    int idx_;
    bool deferred_ = false;
};

// ---- encode.hip
// codes, idx and key0 (the first refinement key of every string) may each be
// null.  With sel, entry i codes string sel[i] (i < n_out) instead of string i.
// With bucket, every code's learned bucket id is written too (bucket.h).
// With perfect (ASCII only), codes are written as code << 1 | f, f = 0 iff
// the string is at most nine bytes with no NUL (encode.hip).
struct BucketArgs;
// With korand (one sort over all n strings): each workgroup encodes one
// radix tile of `tile` strings and writes its OR and AND of the codes to
// korand[2t], korand[2t + 1], in place of radix_reduce_tiles.
hipError_t launch_encode(int coder, const void* elems, const uint64_t* offsets, uint32_t n,
                         uint64_t* codes, uint32_t* idx, uint64_t* key0, uint32_t* status,
                         hipStream_t s, const uint32_t* sel = nullptr, uint32_t n_out = 0,
                         const BucketArgs* bucket = nullptr, bool perfect = false,
                         uint64_t* korand = nullptr, uint32_t tile = 0, bool tag_low8 = false);

// ---- radix.hip
struct RadixConfig {
    int bits;        // digit width: 6, 7 or 8
    int items;       // keys per thread: 8, 12 or 16 (tile = 256 * items)
    int tile() const { return BLOCK * items; }
};

// Device scratch used by one segmented sort; carved from the workspace.
struct RadixScratch {
    SegDesc* segs;         // [seg_cap] every segment
    BigDesc* bigs;         // [big_cap] segments longer than one tile
    uint64_t* korand;      // [2 * big_tile_cap] OR and AND of the keys of each big tile
    uint32_t* binstart;    // [big_cap][256] digit starts of the current pass
    uint32_t* cnt;         // [big_tile_cap][256] tile digit counts / offsets
    uint32_t* gtot;        // [group_cap][256] group totals / offsets
    uint32_t* counters;    // [64]: tile and segment totals (see common.h)
    uint64_t* segvary;     // [big_cap] bits that vary inside each big segment
    uint32_t* prog;        // [MAX_PASSES * PROG_WORDS] digit programs (common.h)
    // [n] per key position, the digit the key there takes in its segment's
    // next pass, written by the scatter that moved it there; the count
    // kernel of every pass but a segment's first reads these bytes instead
    // of the 8-byte keys (nullptr: it always reads the keys)
    uint8_t* dig = nullptr;
    // Set by callers whose values (string indices) and positions are below
    // 2^24: the next digit then rides in each value's top byte instead of in
    // dig, which spares the scatter a third store per key.
    bool dig_in_vals = false;
    // Set (with dig_in_vals) by a caller whose encode kernel put each key's
    // low byte in the top byte of its value: a first pass whose digit is
    // bits 0..7 counts those bytes instead of the keys, and the values of a
    // segment that runs no pass are cleaned by the copy-back kernel.
    bool vals_low8 = false;
    uint32_t seg_cap, big_cap, big_tile_cap, group_cap;
    // Largest grid of a launch sized from a host bound (a multiple of 8;
    // ~0u: none): the kernels walk their work units (HUSKY_UNITS), so a
    // capped grid only lengthens each workgroup's walk.
    uint32_t grid_cap = ~0u;
    uint32_t grid(uint32_t bound) const { return bound < grid_cap ? bound : grid_cap; }
};

// Largest n whose values and positions leave a value's top byte free.
constexpr uint64_t DIG_IN_VALS_MAX = 1ull << 24;

// Build segment descriptors from uint64 string offsets (n_segs + 1 entries).
// (z0[0..nz0) and z1[0..nz1) are cleared by the same launch.)
hipError_t radix_segments_from_offsets(const uint64_t* seg_offsets, uint32_t n_segs,
                                       const RadixScratch& sc, const RadixConfig& cfg,
                                       hipStream_t s, uint32_t* z0 = nullptr, uint32_t nz0 = 0,
                                       uint32_t* z1 = nullptr, uint32_t nz1 = 0);
// Build segment descriptors for a single segment [0, n).
hipError_t radix_segments_single(uint32_t n, const RadixScratch& sc, const RadixConfig& cfg,
                                 hipStream_t s, uint32_t* z0 = nullptr, uint32_t nz0 = 0,
                                 uint32_t* z1 = nullptr, uint32_t nz1 = 0);
// Build segment descriptors from a fix-up work list (count in device memory).
hipError_t radix_segments_from_items(const RunItem* items, const uint32_t* count,
                                     uint32_t max_items, const RadixScratch& sc,
                                     const RadixConfig& cfg, hipStream_t s);

// Bits that vary inside every big segment: per-tile OR / AND of the keys
// (skipped by callers whose key kernel already wrote them), then the digit
// programs over the bits that vary in any big segment, each big segment's
// mask of digit passes and their union (counters[C_EXEC_UNION]).
hipError_t radix_reduce_tiles(const uint64_t* keys, uint32_t max_tiles, const RadixScratch& sc,
                              const RadixConfig& cfg, hipStream_t s);
// With perfect_lsb (ASCII codes with the perfect bit), bit 0 is left out of
// the digits when that saves a pass (counters[C_PERFECT_OFF] = 1).
hipError_t radix_exec_masks(int begin_bit, int end_bit, uint32_t max_segs, uint32_t max_tiles,
                            const RadixScratch& sc, const RadixConfig& cfg, hipStream_t s,
                            bool perfect_lsb = false);

// Stable sort of (keys, vals) by bits [begin_bit, end_bit) inside every
// segment described in sc (built by one of the functions above, with the
// pass masks from radix_exec_masks); keys_alt / vals_alt are ping-pong
// buffers of the same size.  The result ends in keys / vals.  max_tiles /
// max_segs bound the grid sizes; passes outside pass_union (a host mask,
// ~0u when unknown) are not launched.
// tile_segments false: single-tile segments are left to the caller.
hipError_t radix_sort_segments(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt,
                               uint32_t* vals_alt, int begin_bit, int end_bit,
                               uint32_t max_segs, uint32_t max_tiles, uint32_t pass_union,
                               const RadixScratch& sc, const RadixConfig& cfg, int pclass,
                               hipStream_t s, bool tile_segments = true);

// ---- runs.hip
struct RunScratch {
    uint32_t* tile_counts;  // [tile_cap + 1]
    uint32_t* run_start;    // [2 * run_cap]: run heads, then each run's segment
    uint32_t* run_end;      // [run_cap]
    uint32_t* counters;     // [16]
    uint32_t* runs_seen;    // device counter of runs found by the first detection (or null)
    // [positions] one byte per key, written by the count kernel (run head,
    // run tail, inside a run after its head) and read by the write kernel in
    // place of the keys (null: the write kernel reads the keys again)
    uint8_t* flags = nullptr;
    uint32_t tile_cap, run_cap;
};

// Fix-up work lists, one per tier (device lists, device counts).
// The LDS tier (runs of t_medium < len <= 8192) in four size classes by
// length: up to 3072, 4096, 6144 and 8192.
__host__ __device__ constexpr uint32_t lds_class_max(int c) {
    return c == 0 ? 3072u : (c == 1 ? 4096u : (c == 2 ? 6144u : 8192u));
}
__host__ __device__ constexpr int lds_class_of(uint32_t len) {
    return len > 6144u ? 3 : (len > 4096u ? 2 : (len > 3072u ? 1 : 0));
}

struct TierLists {
    RunItem* small;
    RunItem* medium;
    RunItem* large;
    RunItem* lds[4];  // LDS tier, one list per size class
    uint32_t* small_count;
    uint32_t* medium_count;
    uint32_t* large_count;  // [4]: items, items longer than one tile, their tiles, all their tiles
    uint32_t* lds_count;    // [4]
    uint32_t* lds_queue;    // [4] work counters of the LDS tier's kernels
    uint32_t small_cap, medium_cap, large_cap;
    uint32_t lds_cap[4];
    uint32_t lds_max;  // 0: no LDS tier (those runs go device-wide)
    // First list entry a tier launch takes (device words; null: 0): a launch
    // after the device-wide round takes only the runs that round appended.
    const uint32_t* small_first = nullptr;
    const uint32_t* medium_first = nullptr;
    const uint32_t* lds_first = nullptr;  // [4]
    bool lds_queue_zero = false;  // the caller cleared lds_queue already
};

// Find runs (length >= 2) of equal keys inside every segment of sc; when
// `require_cont` is set a run is kept only if its keys carry the
// "continues" marker (refinement keys).  Appends each kept run to the tier
// list chosen by its length, with refinement round 0 (or, when `items` is
// given, the segment item's round + 1).
// `max_tiles` bounds the tile count over every segment (grid size).
// With `perfect_codes` (codes written with the perfect bit, encode.hip) a run
// of codes whose bit 0 is clear holds identical strings and is not listed --
// unless the sort left bit 0 out (counters[C_PERFECT_OFF]): then keys are
// compared without it and every run is listed.
hipError_t find_runs(const uint64_t* keys, const RadixScratch& seg, const RadixConfig& cfg,
                     uint32_t max_tiles, int coder, bool refinement, const RunItem* items,
                     const RunScratch& rs, const TierLists& tl, uint32_t t_small,
                     uint32_t t_medium, uint32_t origin, hipStream_t s, bool perfect_codes = false);

// Zero-fill kernels (graph-capture friendly).
hipError_t zero_u64(uint64_t* p, size_t n, hipStream_t s);
hipError_t zero_u32(uint32_t* p, size_t n, hipStream_t s);

// ---- fixup.hip
struct FixupArgs {
    int coder;                // element kind: 0 bytes, 1 UTF-16 units (elem_kind)
    const void* elems;
    const uint64_t* offsets;  // [n + 1]; offsets[n] is the element total
    uint32_t n;
    uint32_t* idx;            // permutation being fixed, in place
    const uint64_t* key0;     // [n] first refinement key of every string
    uint32_t origin;          // elements every member of a run shares (up to
                              // its length): refinement round r compares from
                              // origin + C*r; at most 15
};

hipError_t fixup_small(const FixupArgs& a, const TierLists& tl, uint32_t t_small, hipStream_t s);
hipError_t fixup_medium(const FixupArgs& a, const TierLists& tl, uint32_t t_medium,
                        hipStream_t s);
// Runs of t_medium < len <= LDS_RUN_MAX, every round inside one workgroup.
constexpr uint32_t LDS_RUN_MAX = 8192;
// spare_cus: compute units the largest size class leaves to concurrent work.
hipError_t fixup_lds(const FixupArgs& a, const TierLists& tl, uint32_t t_medium, hipStream_t s,
                     uint32_t spare_cus = 0);
// Device-wide tier, before the keys of a round: the position every group's
// members first differ at (RunItem::lcp), so that the keys skip the chunks
// all of them share.
hipError_t fixup_large_lcp(const FixupArgs& a, RunItem* items, const RadixScratch& seg,
                           const RadixConfig& cfg, uint32_t max_tiles, hipStream_t s);
// Refinement keys for every position of the large-tier segments; with
// tile_orand (every segment longer than one radix tile) also each tile's OR
// and AND of its keys, in place of radix_reduce_tiles.
hipError_t fixup_large_keys(const FixupArgs& a, const RunItem* items, const RadixScratch& seg,
                            const RadixConfig& cfg, uint32_t max_tiles, uint64_t* keys,
                            hipStream_t s, bool tile_orand);
// Groups left tied after the device-wide rounds (items, device count): one
// workgroup runs every remaining round of a group in global memory.
// Scratch: idx_alt u32[n], keyA / keyB u64[n], gs u32[2n].
hipError_t fixup_tail(const FixupArgs& a, const RunItem* items, const uint32_t* count, uint32_t cap,
                      uint32_t* idx_alt, uint64_t* keyA, uint64_t* keyB, uint32_t* gs, uint32_t* unresolved,
                      hipStream_t s);
// key0[i] = string i's first refinement key (round 0 from a.origin).
hipError_t fixup_first_keys(const FixupArgs& a, uint64_t* key0, hipStream_t s);

// ---- typed.hip (the other object types: numbers, date-times, big numbers, tuples)
// codes of fixed-width records (int32, int64, float64, date-time) and the
// index iota; status (may be null) counts date-times outside the field ranges
hipError_t typed_fixed_codes(int type, const void* recs, uint32_t n, int32_t base_year, uint64_t* codes,
                             uint32_t* idx, uint32_t* status, hipStream_t s);
// codes of variable-length records (big integers, decimals, tuples): the first
// eight bytes of their order keys
hipError_t typed_key_codes(int type, const void* recs, const uint64_t* offsets, uint32_t n,
                           uint64_t* codes, uint32_t* status, hipStream_t s);
// order keys of every record into keys, key_offsets[0 .. n] (lens: n words,
// tile_tmp: typed_scan_tiles(n) words of scratch); date-times: 13 bytes each
hipError_t typed_keys(int type, const void* recs, const uint64_t* offsets, uint32_t n, uint64_t* lens,
                      uint64_t* tile_tmp, uint64_t* key_offsets, uint8_t* keys, uint32_t* status,
                      hipStream_t s);
uint32_t typed_scan_tiles(uint32_t n);

// ---- merge.hip: Step 3 as a full stable pass (natural merge sort by
// (string, index)); idx in place; ek: element kind
size_t merge_workspace_bytes(uint64_t n);
hipError_t merge_fixup(int ek, const void* elems, const uint64_t* offsets, uint32_t n, uint32_t* idx,
                       void* ws, hipStream_t s);

// ---- learned.hip
constexpr uint32_t LEARNED_BUCKETS = 65536;
constexpr uint32_t LEARNED_LDS_CAP = 8192;  // largest bucket sorted in LDS
size_t learned_model_bytes();
size_t learned_model_offset(int part);
uint32_t learned_nparam();
uint32_t learned_lut_tiles();
size_t learned_partial_bytes(uint32_t max_blocks);
uint32_t learned_pass_tiles(uint32_t n);
const uint32_t* learned_dense_keys_ptr(void* model);
hipError_t learned_sample(uint32_t* sel, uint32_t S, uint32_t n, uint64_t seed, hipStream_t s);
hipError_t learned_prepare(void* model, const uint64_t* sorted_sample, uint32_t S, uint32_t mode,
                           uint32_t flags, uint8_t* fl, uint2* tsum, float* x, float* y,
                           hipStream_t s);
hipError_t learned_init(void* model, uint64_t seed, bool raw, hipStream_t s);
hipError_t learned_grad(const float* params, const float* x, const float* y, uint32_t count,
                        bool mono, float* partial, uint32_t max_blocks, float* grad, hipStream_t s);
hipError_t learned_train(void* model, const float* x, const float* y, uint32_t count,
                         uint32_t epochs, uint32_t batch, float lr, bool mono, float* partial,
                         uint32_t max_blocks, float* grad, float* loss_acc, hipStream_t s);
hipError_t learned_build_lut(void* model, uint32_t mode, uint32_t* tmax, hipStream_t s);
// The LUT of `params` (mode as husky_learned_mode) over the header and dense
// cells of `model`, written to lut (uint32[2^24 + 1]), running maximum included.
hipError_t learned_eval_lut(const float* params, const void* model, uint32_t mode, uint32_t* lut,
                            uint32_t* tmax, hipStream_t s);
hipError_t learned_splitters(void* model, const uint64_t* sorted_sample, uint32_t S, hipStream_t s);
BucketArgs learned_bucket_args(const void* model, uint16_t* bid);
hipError_t learned_bucket_pass(int pass, const uint64_t* ks, const uint32_t* vs, const uint16_t* bs,
                               const uint64_t* k0s, uint64_t* kd, uint32_t* vd, uint16_t* bd,
                               uint64_t* k0d, uint32_t n, uint32_t* cnt, uint32_t* gtot,
                               uint32_t* binstart, hipStream_t s);
// fallback[c] (LEARNED_BUCKETS entries, count zeroed by the caller) receives
// class c's buckets whose varying (code, key) bits exceed one word.
// Size classes [c_begin, c_end) only.
hipError_t learned_bucket_refine(int coder, uint64_t* codes, uint32_t* perm, const uint64_t* k0,
                                 RunItem* const lists[4], const uint32_t* counts,
                                 RunItem* const fallback[4], uint32_t* fallback_counts,
                                 RunItem* scan_list, uint32_t* scan_count, int c_begin, int c_end,
                                 hipStream_t s);
hipError_t learned_bucket_bounds(const uint16_t* bid, uint32_t n, uint64_t* seg, uint32_t* overflow,
                                 RunItem* big_list, uint32_t* big_count, RunItem* scan_list,
                                 uint32_t* scan_count, RunItem* const lists[4],
                                 uint32_t* class_count, hipStream_t s);

// Coders (husky_coder) and the geometry of their refinement keys: the code
// covers the first m elements; a refinement round covers the next chunk of
// 7 bytes or 3 UTF-16 units.
constexpr int ascii_m = 9, bytes8_m = 8, utf16_m = 4;
constexpr int byte_chunk = 7, utf16_chunk = 3;
constexpr int CODER_ASCII7 = 0, CODER_UTF16 = 1, CODER_BYTES8 = 2;
// Element kind of a coder (0: bytes, 1: 16-bit units): what the run
// detection, fix-up and device check depend on.
__host__ __device__ constexpr int elem_kind(int coder) { return coder == CODER_UTF16 ? 1 : 0; }
// Elements a husky code covers.
__host__ __device__ constexpr uint32_t coder_m(int coder) {
    return coder == CODER_ASCII7 ? ascii_m : (coder == CODER_UTF16 ? utf16_m : bytes8_m);
}

// A refinement key whose length field says the string goes on past its chunk:
// two such equal keys are still tied.
template <int CODER>
__device__ __forceinline__ bool key_continues(uint64_t key) {
    return (key & 0xFull) == (CODER == 0 ? (uint64_t)byte_chunk + 1 : (uint64_t)utf16_chunk + 1);
}

}  // namespace husky
