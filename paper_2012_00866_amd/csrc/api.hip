// C ABI of libhusky.so: argument checks, workspace layout and the order of
// the kernel launches for every entry point declared in include/husky.h.
// Each step's kernels live in encode.hip (Step 1), radix.hip (Step 2),
// runs.hip and fixup.hip (Step 3).

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "../../include/husky.h"
#include "bucket.h"
#include "common.h"
#include "internal.h"

namespace husky {
namespace {

constexpr size_t ALIGN = 256;
constexpr uint32_t MIN_TILE = BLOCK * 8;  // smallest compiled tile
constexpr uint32_t MIN_T_MEDIUM = 64;
constexpr uint32_t MAX_T_MEDIUM = 4096;
constexpr uint32_t MAX_T_SMALL = 64;
// Device-wide refinement rounds a call launches without reading anything back
// (groups still tied after them go to the in-workgroup tail), and the largest
// grid of their launches (a multiple of 8: the kernels walk their work units).
constexpr uint32_t DEFAULT_ROUNDS = 1;
constexpr uint32_t ROUND_GRID_CAP = 2048;
// Compute units the LDS tier's largest size class leaves to the device-wide
// round running beside it (four per XCD).
constexpr uint32_t ROUND_SPARE_CUS = 32;

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Learned form: training workgroups at most, and the per-workgroup
// gradient partials they need.
constexpr uint32_t LEARN_MAX_BLOCKS = 256;

// Byte offsets of every region inside the caller's workspace.  The learned
// form adds the bucket ids (two u16 arrays), the bucket bounds and the
// training scratch; its fit borrows the sort's regions for the sample (see
// husky_learned_fit).
struct Layout {
    size_t status, counters, codes_a, codes_b, idx_b, key0, segs, bigs, korand, segvary, prog, dig, binstart,
        cnt, gtot,
        tile_counts, run_start, run_end, small, medium, large_a, large_b, lds, bid, bseg, k0a, k0b, scan,
        biglist, classes, fallback, lpartial, lgrad, ltmax, total;
    uint32_t seg_cap, big_cap, tile_cap, big_tile_cap, group_cap, run_cap, small_cap, medium_cap,
        large_cap, lds_cap[4];
};

Layout make_layout(uint64_t n, uint64_t n_segs, bool learned = false) {
    Layout L{};
    if (learned) n_segs = std::max<uint64_t>(n_segs, LEARNED_BUCKETS);
    const uint64_t S = n_segs ? n_segs : 1;
    L.large_cap = (uint32_t)(n / (MIN_T_MEDIUM + 1) + 2);
    L.seg_cap = (uint32_t)std::max<uint64_t>(S, L.large_cap);
    // tiles over any set of segments used by one sort: instances or
    // device-wide fix-up groups
    L.tile_cap = (uint32_t)(n / MIN_TILE + L.seg_cap + 2);
    // multi-tile segments hold more than one tile (>= MIN_TILE positions) each
    L.big_cap = (uint32_t)(n / MIN_TILE + 2);
    L.big_tile_cap = 2 * L.big_cap;
    L.group_cap = L.big_tile_cap / GROUP_TILES + L.big_cap + 2;
    L.run_cap = (uint32_t)(n / 2 + 1);
    L.small_cap = L.run_cap;
    L.medium_cap = (uint32_t)(n / 3 + 1);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.status = take(sizeof(husky_device_status));
    L.counters = take(128 * sizeof(uint32_t));
    L.codes_a = take(n * 8);
    L.codes_b = take(n * 8);
    L.idx_b = take(n * 4);
    L.key0 = take(n * 8);
    L.segs = take((size_t)L.seg_cap * sizeof(SegDesc));
    L.bigs = take((size_t)L.big_cap * sizeof(BigDesc));
    L.korand = take((size_t)L.big_tile_cap * 16);
    L.segvary = take((size_t)L.big_cap * 8);
    L.prog = take((size_t)MAX_PASSES * PROG_WORDS * 4);
    L.dig = take(n);
    L.binstart = take((size_t)L.big_cap * 256 * 4);
    L.cnt = take((size_t)L.big_tile_cap * 256 * 4);
    L.gtot = take((size_t)L.group_cap * 256 * 4);
    L.tile_counts = take((size_t)(L.tile_cap + 1) * 4);
    L.run_start = take((size_t)L.run_cap * 2 * 4);
    L.run_end = take((size_t)L.run_cap * 4);
    L.small = take((size_t)L.small_cap * sizeof(RunItem));
    L.medium = take((size_t)L.medium_cap * sizeof(RunItem));
    L.large_a = take((size_t)L.large_cap * sizeof(RunItem));
    L.large_b = take((size_t)L.large_cap * sizeof(RunItem));
    // LDS-tier runs are disjoint and longer than t_medium >= MIN_T_MEDIUM and
    // than the class below's largest
    size_t lds_items = 0;
    for (int k = 0; k < 4; ++k) {
        const uint64_t shorter = k == 0 ? MIN_T_MEDIUM : lds_class_max(k - 1);
        L.lds_cap[k] = (uint32_t)(n / (shorter + 1) + 2);
        lds_items += L.lds_cap[k];
    }
    L.lds = take(lds_items * sizeof(RunItem));
    if (learned) {
        L.bid = take(n * 4);
        L.bseg = take(((size_t)LEARNED_BUCKETS + 1) * 8);
        L.k0a = take(n * 8);  // first refinement keys in bucket order (ping-pong)
        L.k0b = take(n * 8);
        L.scan = take((size_t)LEARNED_BUCKETS * sizeof(RunItem));     // buckets Step 3 scans
        L.biglist = take((size_t)LEARNED_BUCKETS * sizeof(RunItem));  // buckets the radix passes sort
        L.classes = take((size_t)4 * LEARNED_BUCKETS * sizeof(RunItem));  // LDS size classes
        L.fallback = take((size_t)4 * LEARNED_BUCKETS * sizeof(RunItem)); // ... not on the packed path
        L.lpartial = take(learned_partial_bytes(LEARN_MAX_BLOCKS));
        L.lgrad = take(((size_t)learned_nparam() + 1) * 4 + 256);
        L.ltmax = take((size_t)learned_lut_tiles() * 4);
    }
    L.total = o;
    return L;
}

// counters region: [0, 64) radix counters; [64, 80) run counters;
// [80] small count, [81] medium count; [84, 88) and
// [88, 92) the two device-wide lists: item count, items longer than one
// tile, their tiles, tiles of all items; [92, 96) LDS-tier class counts;
// [96, 102) learned-form lists; [104, 108) work counters of the LDS tier;
// [108, 112) learned-form buckets per size class off the packed path;
// [112, 118) the small, medium and four LDS-class counts as run detection
// left them before the device-wide round; [120, 124) work counters of the
// LDS tier's launch after that round
constexpr int CNT_RUNS = 64, CNT_SMALL = 80, CNT_MEDIUM = 81, CNT_LARGE_A = 84, CNT_LARGE_B = 88,
              CNT_LDS = 92,
              CNT_SCAN = 96,  // learned form: buckets on the run-detection list
              CNT_BIG = 97,   // learned form: buckets for the multi-tile radix passes
              CNT_CLASS = 98, // learned form: buckets per LDS size class (four)
              CNT_LDS_QUEUE = 104,  // LDS fix-up tier: work counters of its size classes (four)
              CNT_FALLBACK = 108,   // learned form: buckets per class off the packed path (four)
              CNT_SNAP = 112,       // tier counts before the device-wide round (six)
              CNT_LDS_QUEUE2 = 120; // LDS tier after the round: work counters (four)
static_assert(CNT_LDS == CNT_SMALL + 12 && CNT_MEDIUM == CNT_SMALL + 1, "tier count slots");

struct Ctx {
    Layout L;
    uint8_t* ws;
    RadixScratch rad;
    RunScratch runs;
    TierLists tiers;
    husky_device_status* status;
    uint32_t* counters;
    template <typename T>
    T* at(size_t off) const {
        return reinterpret_cast<T*>(ws + off);
    }
};

Ctx make_ctx(void* ws, uint64_t n, uint64_t n_segs, bool learned = false) {
    Ctx c;
    c.L = make_layout(n, n_segs, learned);
    c.ws = (uint8_t*)ws;
    c.status = c.at<husky_device_status>(c.L.status);
    c.counters = c.at<uint32_t>(c.L.counters);
    c.rad.segs = c.at<SegDesc>(c.L.segs);
    c.rad.bigs = c.at<BigDesc>(c.L.bigs);
    c.rad.korand = c.at<uint64_t>(c.L.korand);
    c.rad.segvary = c.at<uint64_t>(c.L.segvary);
    c.rad.prog = c.at<uint32_t>(c.L.prog);
    c.rad.dig = c.at<uint8_t>(c.L.dig);
    c.rad.binstart = c.at<uint32_t>(c.L.binstart);
    c.rad.cnt = c.at<uint32_t>(c.L.cnt);
    c.rad.gtot = c.at<uint32_t>(c.L.gtot);
    c.rad.counters = c.counters;
    c.rad.seg_cap = c.L.seg_cap;
    c.rad.big_cap = c.L.big_cap;
    c.rad.big_tile_cap = c.L.big_tile_cap;
    c.rad.group_cap = c.L.group_cap;
    c.runs.tile_counts = c.at<uint32_t>(c.L.tile_counts);
    c.runs.run_start = c.at<uint32_t>(c.L.run_start);
    c.runs.run_end = c.at<uint32_t>(c.L.run_end);
    c.runs.counters = c.counters + CNT_RUNS;
    c.runs.runs_seen = &c.status->runs_fixed;
    c.runs.flags = c.at<uint8_t>(c.L.dig);  // free whenever runs are detected
    c.runs.tile_cap = c.L.tile_cap;
    c.runs.run_cap = c.L.run_cap;
    c.tiers.small = c.at<RunItem>(c.L.small);
    c.tiers.medium = c.at<RunItem>(c.L.medium);
    c.tiers.large = c.at<RunItem>(c.L.large_a);
    {
        RunItem* l = c.at<RunItem>(c.L.lds);
        for (int k = 0; k < 4; ++k) {
            c.tiers.lds[k] = l;
            c.tiers.lds_cap[k] = c.L.lds_cap[k];
            l += c.L.lds_cap[k];
        }
    }
    c.tiers.small_count = c.counters + CNT_SMALL;
    c.tiers.medium_count = c.counters + CNT_MEDIUM;
    c.tiers.large_count = c.counters + CNT_LARGE_A;
    c.tiers.lds_count = c.counters + CNT_LDS;
    c.tiers.lds_queue = c.counters + CNT_LDS_QUEUE;
    c.tiers.small_cap = c.L.small_cap;
    c.tiers.medium_cap = c.L.medium_cap;
    c.tiers.large_cap = c.L.large_cap;
    c.tiers.lds_max = 0;
    return c;
}

struct Tune {
    RadixConfig rc;
    uint32_t t_small, t_medium, max_rounds;
};

husky_status resolve_tuning(const husky_tuning* t, Tune* out) {
    Tune r{{8, 16}, 64, 1024, 0};
    if (t) {
        if (t->radix_bits) r.rc.bits = t->radix_bits;
        if (t->tile_items) r.rc.items = t->tile_items;
        if (t->t_small) r.t_small = t->t_small;
        if (t->t_medium) r.t_medium = t->t_medium;
        r.max_rounds = t->max_rounds;
    }
    if (r.max_rounds > 4096 && r.max_rounds != HUSKY_ROUNDS_ADAPTIVE) return HUSKY_ERR_UNSUPPORTED;
    if (r.rc.bits < 6 || r.rc.bits > 8) return HUSKY_ERR_UNSUPPORTED;
    if (r.rc.items != 8 && r.rc.items != 12 && r.rc.items != 16) return HUSKY_ERR_UNSUPPORTED;
    if (r.t_small < 2 || r.t_small > MAX_T_SMALL) return HUSKY_ERR_UNSUPPORTED;
    if (r.t_medium < MIN_T_MEDIUM || r.t_medium > MAX_T_MEDIUM || r.t_medium <= r.t_small)
        return HUSKY_ERR_UNSUPPORTED;
    *out = r;
    return HUSKY_OK;
}

husky_status check_ws(void* ws, size_t ws_bytes, uint64_t n, uint64_t n_segs,
                      bool learned = false) {
    if (!ws) return HUSKY_ERR_WORKSPACE;
    if (((uintptr_t)ws) % ALIGN) return HUSKY_ERR_WORKSPACE;
    if (ws_bytes < make_layout(n, n_segs, learned).total) return HUSKY_ERR_WORKSPACE;
    return HUSKY_OK;
}

constexpr size_t STATUS_WORDS = sizeof(husky_device_status) / sizeof(uint32_t);

__global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }
__global__ void k_copy_u32(uint32_t* dst, const uint32_t* src) { *dst = *src; }
// snap[0..6) = the small, medium and four LDS-class tier counts
__global__ void k_snap_tiers(uint32_t* __restrict__ snap, const uint32_t* __restrict__ small_count,
                             const uint32_t* __restrict__ medium_count,
                             const uint32_t* __restrict__ lds_count) {
    snap[0] = *small_count;
    snap[1] = *medium_count;
    for (int k = 0; k < 4; ++k) snap[2 + k] = lds_count[k];
}

husky_status hip_status(hipError_t e) { return e == hipSuccess ? HUSKY_OK : HUSKY_ERR_HIP; }

#define HUSKY_TRY(expr)                              \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return HUSKY_ERR_HIP;  \
    } while (0)

hipError_t read_u32(const uint32_t* dev, uint32_t* host, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(host, dev, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

uint32_t tiles_bound(uint64_t n, uint64_t segs, const RadixConfig& rc) {
    return (uint32_t)((n + rc.tile() - 1) / rc.tile() + segs + 1);
}

// Two streams per device (default priority) that the wavefront and workgroup
// tiers of Step 3 run on, beside the LDS tier on the caller's stream: the
// tiers touch disjoint runs, and the LDS tier's largest class holds one
// workgroup per CU, so the others can use the rest of each CU.  Created on
// the first call on a device that is not being captured into a graph; until
// then the tiers run one after the other.  Calls on one device share them,
// and the fork and join events are recorded and waited on under a lock, so
// concurrent calls from several host threads stay ordered.
struct SideStreams {
    hipStream_t st[2];
    hipEvent_t fork, join[2];
};
static std::mutex g_side_mutex;
static std::map<int, SideStreams> g_side;

static const SideStreams* side_streams(bool create) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto it = g_side.find(dev);
    if (it != g_side.end()) return &it->second;
    if (!create) return nullptr;
    SideStreams ss{};
    bool ok = true;
    for (int i = 0; i < 2 && ok; ++i) ok = hipStreamCreateWithFlags(&ss.st[i], hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < 2 && ok; ++i)
        ok = hipEventCreateWithFlags(&ss.join[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) return nullptr;  // the tiers then share the caller's stream
    return &(g_side[dev] = ss);
}

// Below this many strings the fork and join (about 50 µs per call) cost more
// than running the tiers side by side saves.
constexpr uint64_t SIDE_MIN_N = 1ull << 21;

// Work enqueued on s so far must finish before anything enqueued on the side
// streams from now on; *out is null when there are no side streams or n is
// small (then everything stays on s).
static hipError_t side_fork(hipStream_t s, uint64_t n, const SideStreams** out) {
    *out = nullptr;
    if (n < SIDE_MIN_N) return hipSuccess;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_side_mutex);
    const SideStreams* ss = side_streams(cap == hipStreamCaptureStatusNone);
    if (!ss) return hipSuccess;
    e = hipEventRecord(ss->fork, s);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipStreamWaitEvent(ss->st[i], ss->fork, 0);
    if (e == hipSuccess) *out = ss;
    return e;
}

// Work enqueued on s from now on waits for everything enqueued on the side
// streams so far.
static hipError_t side_join(hipStream_t s, const SideStreams* ss) {
    if (!ss) return hipSuccess;
    std::lock_guard<std::mutex> lock(g_side_mutex);
    hipError_t e = hipSuccess;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipEventRecord(ss->join[i], ss->st[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, ss->join[i], 0);
    }
    return e;
}

// Step 3 over the segments currently described in c.rad (the instances the
// codes were sorted in).  `codes` are the sorted codes; `keys`/`keys_alt`
// are scratch key buffers (may alias `codes` once the runs are found).
husky_status run_fixup(Ctx& c, const Tune& tn, int coder, uint32_t origin, const void* elems,
                       const uint64_t* offsets, uint64_t n, uint64_t n_segs,
                       const uint64_t* codes, uint64_t* keys, uint64_t* keys_alt, uint32_t* idx,
                       hipStream_t s, bool perfect_codes = false, bool tier_counts_zero = false) {
    // tier counts [80, 96); with tier_counts_zero the caller cleared all of
    // [80, 128) (the LDS tier's work counters too)
    if (!tier_counts_zero) HUSKY_TRY(zero_u32(c.counters + CNT_SMALL, 16, s));
    c.tiers.lds_queue_zero = tier_counts_zero;
    c.tiers.lds_max = tn.t_medium < LDS_RUN_MAX ? LDS_RUN_MAX : 0u;
    const uint32_t tb = tiles_bound(n, n_segs, tn.rc);
    const int ek = elem_kind(coder);
    HUSKY_TRY(find_runs(codes, c.rad, tn.rc, tb, ek, false, nullptr, c.runs, c.tiers,
                        tn.t_small, tn.t_medium, origin, s, perfect_codes));
    FixupArgs fa{ek, elems, offsets, (uint32_t)n, idx, c.at<uint64_t>(c.L.key0), origin};
    uint32_t rounds = 0;
    RunItem* cur = c.at<RunItem>(c.L.large_a);
    RunItem* nxt = c.at<RunItem>(c.L.large_b);
    uint32_t* cur_cnt = c.counters + CNT_LARGE_A;
    uint32_t* nxt_cnt = c.counters + CNT_LARGE_B;
    // Rounds: adaptive (host reads the work counts once per round and stops
    // when nothing is left), or a fixed number launched without host reads
    // -- tuning.max_rounds, or the default DEFAULT_ROUNDS followed by the
    // in-workgroup tail for whatever is still tied.
    const bool adaptive = tn.max_rounds == HUSKY_ROUNDS_ADAPTIVE;
    const bool bounded = !adaptive && tn.max_rounds > 0;
    const uint32_t big_min0 = c.tiers.lds_max ? c.tiers.lds_max : tn.t_medium;
    // no run can reach the device-wide tier when n is within the run-local ones
    const uint32_t fixed_rounds = bounded ? tn.max_rounds : (n > big_min0 ? DEFAULT_ROUNDS : 0u);
    // host bounds for the rounds launched without host reads: every
    // device-wide item is longer than the LDS tier's (or, without it, the
    // workgroup tier's) limit, and their tiles number at most n / tile + items
    const uint32_t big_min = c.tiers.lds_max ? c.tiers.lds_max : tn.t_medium;
    const uint32_t nl_bound = std::min<uint32_t>(c.L.large_cap, (uint32_t)(n / (big_min + 1) + 1));
    const uint32_t tiles_bound_l = (uint32_t)(n / tn.rc.tile()) + nl_bound + 1;
    // Default rounds with side streams: the run-local tiers start on the runs
    // run detection listed (counts snapshotted first) beside the device-wide
    // round, which runs on a side stream; the runs the round splits off are
    // appended past the snapshot and taken by a second launch of each tier
    // after it.  The two touch disjoint positions and buffers (the round: its
    // groups' indices, the code buffers, the radix and run-detection scratch;
    // the tiers: their runs' indices; both only read the first keys).
    const SideStreams* ss = nullptr;
    hipStream_t rs = s;  // the rounds' stream
    uint32_t* snap = c.counters + CNT_SNAP;
    TierLists after = c.tiers;  // the tiers' launch after an overlapped round
    if (!adaptive && !bounded && fixed_rounds > 0 && n >= SIDE_MIN_N) {
        hipLaunchKernelGGL(k_snap_tiers, dim3(1), dim3(1), 0, s, snap, c.tiers.small_count,
                           c.tiers.medium_count, c.tiers.lds_count);
        HUSKY_TRY(hipGetLastError());
        HUSKY_TRY(side_fork(s, n, &ss));
        if (ss) {
            TierLists before = c.tiers;
            before.small_count = snap;
            before.medium_count = snap + 1;
            before.lds_count = snap + 2;
            after.small_first = snap;
            after.medium_first = snap + 1;
            after.lds_first = snap + 2;
            after.lds_queue = c.counters + CNT_LDS_QUEUE2;
            HUSKY_TRY(fixup_medium(fa, before, tn.t_medium, ss->st[0]));
            HUSKY_TRY(fixup_small(fa, before, tn.t_small, ss->st[1]));
            // the round's launches would otherwise wait for the largest class,
            // whose workgroups each hold a compute unit
            HUSKY_TRY(fixup_lds(fa, before, tn.t_medium, s, ROUND_SPARE_CUS));
            rs = ss->st[1];
        }
    }
    if (!adaptive) c.rad.grid_cap = ROUND_GRID_CAP;
    for (;;) {
        uint32_t nl, all_tiles, big_tiles;
        if (!adaptive) {
            if (rounds == fixed_rounds) break;
            nl = nl_bound;
            all_tiles = big_tiles = tiles_bound_l;
        } else {
            // items, items longer than one tile, their tiles, all their tiles
            uint32_t st[4];
            HUSKY_TRY(hipMemcpyAsync(st, cur_cnt, sizeof(st), hipMemcpyDeviceToHost, s));
            HUSKY_TRY(hipStreamSynchronize(s));
            nl = std::min(st[0], c.L.large_cap);
            if (nl == 0) break;
            all_tiles = st[3] + 1;
            big_tiles = st[1] ? st[2] + 1 : 0;
        }
        HUSKY_TRY(radix_segments_from_items(cur, cur_cnt, c.L.large_cap, c.rad, tn.rc, rs));
        HUSKY_TRY(fixup_large_lcp(fa, cur, c.rad, tn.rc, all_tiles, rs));
        // every item is longer than the LDS tier's limit, so longer than a
        // radix tile: the key tiles are the sort's tiles, and the key kernel
        // writes their OR / AND itself
        const bool tile_orand = big_min >= (uint32_t)tn.rc.tile();
        HUSKY_TRY(fixup_large_keys(fa, cur, c.rad, tn.rc, all_tiles, keys, rs, tile_orand));
        uint32_t pass_union = ~0u;
        if (big_tiles) {
            if (!tile_orand) HUSKY_TRY(radix_reduce_tiles(keys, big_tiles, c.rad, tn.rc, rs));
            HUSKY_TRY(radix_exec_masks(0, 64, nl, big_tiles, c.rad, tn.rc, rs));
            // the digit passes any group needs: refinement keys hold long
            // constant stretches, so passes nobody runs are not launched
            if (adaptive) HUSKY_TRY(read_u32(c.counters + C_EXEC_UNION, &pass_union, rs));
        }
        // every device-wide item spans several tiles: no single-tile segments
        HUSKY_TRY(radix_sort_segments(keys, idx, keys_alt, c.at<uint32_t>(c.L.idx_b), 0, 64, nl,
                                      big_tiles, pass_union, c.rad, tn.rc, P_SCATTER_FIX, rs,
                                      big_min < (uint32_t)tn.rc.tile()));
        TierLists t2 = c.tiers;
        t2.large = nxt;
        t2.large_count = nxt_cnt;
        HUSKY_TRY(zero_u32(nxt_cnt, 4, rs));
        HUSKY_TRY(find_runs(keys, c.rad, tn.rc, all_tiles, ek, true, cur, c.runs, t2,
                            tn.t_small, tn.t_medium, origin, rs));
        std::swap(cur, nxt);
        std::swap(cur_cnt, nxt_cnt);
        ++rounds;
    }
    c.rad.grid_cap = ~0u;
    if (bounded) {
        hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, s, &c.status->unresolved, cur_cnt);
        HUSKY_TRY(hipGetLastError());
    }
    if (ss) {
        // the runs the round split off, after it on its stream
        HUSKY_TRY(fixup_medium(fa, after, tn.t_medium, rs));
        HUSKY_TRY(fixup_small(fa, after, tn.t_small, rs));
        HUSKY_TRY(fixup_lds(fa, after, tn.t_medium, rs));
        HUSKY_TRY(side_join(s, ss));
    } else {
        // the three run-local tiers: workgroup and wavefront tiers on the
        // side streams (when there are any), the LDS tier on the caller's
        // stream
        HUSKY_TRY(side_fork(s, n, &ss));
        HUSKY_TRY(fixup_medium(fa, c.tiers, tn.t_medium, ss ? ss->st[0] : s));
        HUSKY_TRY(fixup_small(fa, c.tiers, tn.t_small, ss ? ss->st[1] : s));
        HUSKY_TRY(fixup_lds(fa, c.tiers, tn.t_medium, s));
        HUSKY_TRY(side_join(s, ss));
    }
    if (!adaptive && !bounded) {
        // groups still tied after the default rounds: every remaining round
        // in one workgroup per group (after the run-local tiers, whose first
        // refinement keys share the scratch it uses)
        HUSKY_TRY(fixup_tail(fa, cur, cur_cnt, c.L.large_cap, c.at<uint32_t>(c.L.idx_b), keys, keys_alt,
                             c.at<uint32_t>(c.L.key0), &c.status->unresolved, s));
    }
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, &c.status->large_rounds, rounds);
    HUSKY_TRY(hipGetLastError());
    return HUSKY_OK;
}

__global__ void k_copy_codes_iota(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                                  uint32_t* __restrict__ idx, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        dst[i] = src[i];
        idx[i] = i;
    }
}

hipError_t copy_codes_iota(const uint64_t* src, uint64_t* dst, uint32_t* idx, uint32_t n, hipStream_t s) {
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_copy_codes_iota, dim3(blocks), dim3(256), 0, s, src, dst, idx, n);
    return hipGetLastError();
}

husky_status check_common(int coder, const void* elems, const uint64_t* offsets, uint64_t n) {
    if (coder != HUSKY_CODER_ASCII7 && coder != HUSKY_CODER_UTF16 && coder != HUSKY_CODER_BYTES8)
        return HUSKY_ERR_ARG;
    if (n >= (1ull << 32)) return HUSKY_ERR_ARG;
    if (n > 0 && (!elems || !offsets)) return HUSKY_ERR_ARG;
    return HUSKY_OK;
}

}  // namespace
}  // namespace husky

using namespace husky;

extern "C" {

size_t husky_workspace_bytes(uint64_t n, uint64_t n_segs) { return make_layout(n, n_segs).total; }

husky_status husky_encode(husky_coder coder, const void* elems, const uint64_t* offsets,
                          uint64_t n, uint64_t* codes, uint32_t* idx_or_null, uint32_t* status,
                          void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n > 0 && !codes) return HUSKY_ERR_ARG;
    return hip_status(launch_encode(coder, elems, offsets, (uint32_t)n, codes, idx_or_null, nullptr, status,
                                    (hipStream_t)stream));
}

husky_status husky_sort_pairs(uint64_t* codes, uint32_t* idx, uint64_t n, int begin_bit,
                              int end_bit, void* ws, size_t ws_bytes, const husky_tuning* tuning,
                              void* stream) {
    if (n >= (1ull << 32)) return HUSKY_ERR_ARG;
    if (n > 0 && (!codes || !idx)) return HUSKY_ERR_ARG;
    if (begin_bit < 0 || end_bit > 64 || begin_bit >= end_bit) return HUSKY_ERR_ARG;
    Tune tn;
    husky_status st = resolve_tuning(tuning, &tn);
    if (st != HUSKY_OK) return st;
    st = check_ws(ws, ws_bytes, n, 1);
    if (st != HUSKY_OK) return st;
    if (n < 2) return HUSKY_OK;
    hipStream_t s = (hipStream_t)stream;
    Ctx c = make_ctx(ws, n, 1);
    HUSKY_TRY(radix_segments_single((uint32_t)n, c.rad, tn.rc, s));
    const uint32_t tb = tiles_bound(n, 1, tn.rc);
    HUSKY_TRY(radix_reduce_tiles(codes, tb, c.rad, tn.rc, s));
    HUSKY_TRY(radix_exec_masks(begin_bit, end_bit, 1, tb, c.rad, tn.rc, s));
    HUSKY_TRY(radix_sort_segments(codes, idx, c.at<uint64_t>(c.L.codes_b), c.at<uint32_t>(c.L.idx_b),
                                  begin_bit, end_bit, 1, tb, ~0u, c.rad, tn.rc, P_SCATTER, s));
    return HUSKY_OK;
}

// Step 3 over runs of equal keys: husky_fixup (keys are husky codes; the
// first refinement keys come from the encode kernel) and husky_refine (any
// sorted keys whose runs share `origin` elements; first keys from the fix-up's
// own key kernel).
static husky_status refine_common(husky_coder coder, const void* elems, const uint64_t* offsets,
                                  uint64_t n, const uint64_t* sorted_keys, uint32_t* idx,
                                  const uint64_t* seg_offsets_or_null, uint64_t n_segs,
                                  uint32_t origin, bool codes_are_husky, void* ws, size_t ws_bytes,
                                  const husky_tuning* tuning, void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n > 0 && (!sorted_keys || !idx)) return HUSKY_ERR_ARG;
    if (seg_offsets_or_null && (n_segs == 0 || n_segs >= (1ull << 32))) return HUSKY_ERR_ARG;
    if (origin > 15) return HUSKY_ERR_ARG;
    if (!seg_offsets_or_null) n_segs = 1;
    Tune tn;
    st = resolve_tuning(tuning, &tn);
    if (st != HUSKY_OK) return st;
    st = check_ws(ws, ws_bytes, n, n_segs);
    if (st != HUSKY_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Ctx c = make_ctx(ws, n, n_segs);
    HUSKY_TRY(zero_u32((uint32_t*)c.status, STATUS_WORDS, s));
    if (n < 2) return HUSKY_OK;
    if (seg_offsets_or_null)
        HUSKY_TRY(radix_segments_from_offsets(seg_offsets_or_null, (uint32_t)n_segs, c.rad, tn.rc, s));
    else
        HUSKY_TRY(radix_segments_single((uint32_t)n, c.rad, tn.rc, s));
    // first refinement key of every string, read in string order
    uint64_t* key0 = c.at<uint64_t>(c.L.key0);
    if (codes_are_husky) {
        HUSKY_TRY(launch_encode(coder, elems, offsets, (uint32_t)n, nullptr, nullptr, key0, nullptr, s));
    } else {
        const FixupArgs fa{elem_kind(coder), elems, offsets, (uint32_t)n, idx, nullptr, origin};
        HUSKY_TRY(fixup_first_keys(fa, key0, s));
    }
    return run_fixup(c, tn, coder, origin, elems, offsets, n, n_segs, sorted_keys,
                     c.at<uint64_t>(c.L.codes_a), c.at<uint64_t>(c.L.codes_b), idx, s);
}

husky_status husky_fixup(husky_coder coder, const void* elems, const uint64_t* offsets, uint64_t n,
                         const uint64_t* sorted_codes, uint32_t* idx,
                         const uint64_t* seg_offsets_or_null, uint64_t n_segs, void* ws,
                         size_t ws_bytes, const husky_tuning* tuning, void* stream) {
    return refine_common(coder, elems, offsets, n, sorted_codes, idx, seg_offsets_or_null, n_segs,
                         coder_m(coder), true, ws, ws_bytes, tuning, stream);
}

husky_status husky_refine(husky_coder coder, const void* elems, const uint64_t* offsets, uint64_t n,
                          const uint64_t* sorted_keys, uint32_t* idx,
                          const uint64_t* seg_offsets_or_null, uint64_t n_segs,
                          uint32_t shared_elems, void* ws, size_t ws_bytes,
                          const husky_tuning* tuning, void* stream) {
    return refine_common(coder, elems, offsets, n, sorted_keys, idx, seg_offsets_or_null, n_segs,
                         shared_elems, false, ws, ws_bytes, tuning, stream);
}

static husky_status sort_common(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, const uint64_t* seg_offsets, uint64_t n_segs,
                                uint32_t* perm, void* ws, size_t ws_bytes,
                                const husky_tuning* tuning, void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n > 0 && !perm) return HUSKY_ERR_ARG;
    Tune tn;
    st = resolve_tuning(tuning, &tn);
    if (st != HUSKY_OK) return st;
    st = check_ws(ws, ws_bytes, n, n_segs);
    if (st != HUSKY_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Ctx c = make_ctx(ws, n, n_segs);
    if (n == 0) return hip_status(zero_u32((uint32_t*)c.status, STATUS_WORDS, s));
    // the segment descriptors (they depend on the sizes alone); the same
    // launch clears the status and Step 3's counters [80, 128) (tier counts,
    // LDS work counters: untouched until run detection)
    uint32_t* z0 = (uint32_t*)c.status;
    uint32_t* z1 = c.counters + CNT_SMALL;
    if (seg_offsets)
        HUSKY_TRY(radix_segments_from_offsets(seg_offsets, (uint32_t)n_segs, c.rad, tn.rc, s, z0,
                                              (uint32_t)STATUS_WORDS, z1, 48));
    else
        HUSKY_TRY(radix_segments_single((uint32_t)n, c.rad, tn.rc, s, z0, (uint32_t)STATUS_WORDS, z1, 48));
    uint64_t* codes = c.at<uint64_t>(c.L.codes_a);
    uint64_t* codes_b = c.at<uint64_t>(c.L.codes_b);
    // ASCII codes carry the perfect bit (encode.hip): all 64 bits are key
    // bits, and runs of identical short strings are never listed
    const bool perfect = coder == HUSKY_CODER_ASCII7;
    // one instance: its radix tiles are the string order's, so the encode
    // kernel reduces each tile's OR / AND as it writes the codes
    const bool enc_orand = !seg_offsets;
    // ... and, for one instance longer than a tile, puts each code's low
    // byte in its index's top byte for the first digit pass's count
    const bool low8 = enc_orand && n <= DIG_IN_VALS_MAX && n > (uint64_t)tn.rc.tile();
    HUSKY_TRY(launch_encode(coder, elems, offsets, (uint32_t)n, codes, perm, c.at<uint64_t>(c.L.key0),
                            &c.status->domain_violations, s, nullptr, 0, nullptr, perfect,
                            enc_orand ? c.rad.korand : nullptr, (uint32_t)tn.rc.tile(), low8));
    const int end_bit = 64;
    const uint32_t tb = tiles_bound(n, n_segs, tn.rc);
    if (!enc_orand) HUSKY_TRY(radix_reduce_tiles(codes, tb, c.rad, tn.rc, s));
    HUSKY_TRY(radix_exec_masks(0, end_bit, (uint32_t)n_segs, tb, c.rad, tn.rc, s, perfect));
    // every pass is launched (no host synchronisation); passes no instance
    // needs end at once.  The values are string indices (as in the
    // device-wide fix-up's sorts after it).
    c.rad.dig_in_vals = n <= DIG_IN_VALS_MAX;
    // one instance longer than a tile has no single-tile segment to sort
    const bool tile_segs = !(n_segs == 1 && n > (uint64_t)tn.rc.tile());
    c.rad.vals_low8 = low8;
    HUSKY_TRY(radix_sort_segments(codes, perm, codes_b, c.at<uint32_t>(c.L.idx_b), 0, end_bit,
                                  (uint32_t)n_segs, tb, ~0u, c.rad, tn.rc, P_SCATTER, s, tile_segs));
    c.rad.vals_low8 = false;  // the fix-up's sorts start from clean values
    // the sorted codes are not needed once the runs are listed, so the
    // device-wide fix-up reuses both code buffers for its keys
    return run_fixup(c, tn, coder, coder_m(coder), elems, offsets, n, n_segs, codes, codes, codes_b, perm,
                     s, perfect, true);
}

husky_status husky_sort(husky_coder coder, const void* elems, const uint64_t* offsets, uint64_t n,
                        uint32_t* perm, void* ws, size_t ws_bytes, const husky_tuning* tuning,
                        void* stream) {
    return sort_common(coder, elems, offsets, n, nullptr, 1, perm, ws, ws_bytes, tuning, stream);
}

// ------------------------------------------------- sort without allocation
// Scratch of husky_sort_noalloc: one copy per device, held until the process
// ends.  Host code never passes `scratch` itself to a kernel or copy (on the
// host it names a stand-in, not device memory): it uses the address
// hipGetSymbolAddress gives for the current device, looked up once per
// device and kept in g_scratch.
static __device__ __align__(256) uint8_t scratch[HUSKY_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch[MAX_DEVICES];
}  // namespace

// Device address of this device's scratch array (null on failure).
static void* device_scratch() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

husky_status husky_sort_noalloc(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, uint32_t* perm, const husky_tuning* tuning,
                                void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n > HUSKY_NOALLOC_MAX_STRINGS) return HUSKY_ERR_TOO_LARGE;
    const size_t need = make_layout(n, 1).total;
    if (need > (size_t)HUSKY_NOALLOC_SCRATCH_BYTES) return HUSKY_ERR_TOO_LARGE;
    void* ws = device_scratch();
    if (!ws) return HUSKY_ERR_HIP;
    return sort_common(coder, elems, offsets, n, nullptr, 1, perm, ws, need, tuning, stream);
}

husky_status husky_noalloc_status(husky_device_status* out, void* stream) {
    if (!out) return HUSKY_ERR_ARG;
    void* ws = device_scratch();
    if (!ws) return HUSKY_ERR_HIP;
    hipStream_t s = (hipStream_t)stream;
    HUSKY_TRY(hipMemcpyAsync(out, ws, sizeof(husky_device_status), hipMemcpyDeviceToHost, s));
    HUSKY_TRY(hipStreamSynchronize(s));
    return HUSKY_OK;
}

husky_status husky_sort_batched(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, const uint64_t* seg_offsets, uint64_t n_segs,
                                uint32_t* perm, void* ws, size_t ws_bytes,
                                const husky_tuning* tuning, void* stream) {
    if (!seg_offsets || n_segs == 0 || n_segs >= (1ull << 32)) return HUSKY_ERR_ARG;
    return sort_common(coder, elems, offsets, n, seg_offsets, n_segs, perm, ws, ws_bytes, tuning,
                       stream);
}

// ---------------------------------------------------------------- lossy coders
size_t husky_global_workspace_bytes(uint64_t n) { return merge_workspace_bytes(n); }

husky_status husky_fixup_global(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, uint32_t* idx, void* ws, size_t ws_bytes, void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n > 0 && !idx) return HUSKY_ERR_ARG;
    if (!ws || ((uintptr_t)ws) % ALIGN || ws_bytes < merge_workspace_bytes(n)) return HUSKY_ERR_WORKSPACE;
    return hip_status(merge_fixup(elem_kind(coder), elems, offsets, (uint32_t)n, idx, ws, (hipStream_t)stream));
}

size_t husky_lossy_workspace_bytes(uint64_t n) {
    return align_up(make_layout(n, 1).total) + merge_workspace_bytes(n);
}

husky_status husky_sort_lossy(husky_coder coder, const void* elems, const uint64_t* offsets, uint64_t n,
                              const uint64_t* codes, uint32_t* perm, void* ws, size_t ws_bytes,
                              const husky_tuning* tuning, void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n > 0 && (!codes || !perm)) return HUSKY_ERR_ARG;
    Tune tn;
    if ((st = resolve_tuning(tuning, &tn)) != HUSKY_OK) return st;
    const size_t sort_bytes = align_up(make_layout(n, 1).total);
    if (!ws || ((uintptr_t)ws) % ALIGN || ws_bytes < sort_bytes + merge_workspace_bytes(n))
        return HUSKY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    Ctx c = make_ctx(ws, n, 1);
    HUSKY_TRY(zero_u32((uint32_t*)c.status, STATUS_WORDS, s));
    if (n == 0) return HUSKY_OK;
    const uint32_t nn = (uint32_t)n;
    uint64_t* k = c.at<uint64_t>(c.L.codes_a);
    uint64_t* kb = c.at<uint64_t>(c.L.codes_b);
    // Step 2 on the caller's codes (copied, with the index iota)
    HUSKY_TRY(copy_codes_iota(codes, k, perm, nn, s));
    HUSKY_TRY(radix_segments_single(nn, c.rad, tn.rc, s));
    const uint32_t tb = tiles_bound(n, 1, tn.rc);
    HUSKY_TRY(radix_reduce_tiles(k, tb, c.rad, tn.rc, s));
    HUSKY_TRY(radix_exec_masks(0, 64, 1, tb, c.rad, tn.rc, s));
    HUSKY_TRY(radix_sort_segments(k, perm, kb, c.at<uint32_t>(c.L.idx_b), 0, 64, 1, tb, ~0u, c.rad, tn.rc,
                                  P_SCATTER, s));
    // runs of equal codes by the full comparator, from the first element (the
    // codes promise nothing), then the full stable pass for what lies across
    // codes
    const FixupArgs fa{elem_kind(coder), elems, offsets, nn, perm, nullptr, 0u};
    HUSKY_TRY(fixup_first_keys(fa, c.at<uint64_t>(c.L.key0), s));
    st = run_fixup(c, tn, coder, 0u, elems, offsets, n, 1, k, k, kb, perm, s);
    if (st != HUSKY_OK) return st;
    return hip_status(merge_fixup(elem_kind(coder), elems, offsets, nn, perm, (uint8_t*)ws + sort_bytes, s));
}

// ---------------------------------------------------------------- typed records
namespace {
bool typed_fixed(int t) { return t >= HUSKY_TYPE_INT32 && t <= HUSKY_TYPE_DATETIME; }
uint32_t typed_width(int t) { return t == HUSKY_TYPE_INT32 ? 4u : (t == HUSKY_TYPE_DATETIME ? 16u : 8u); }

// Key bytes that n records of record_bytes bytes can need at most.
uint64_t typed_key_bound(int t, uint64_t n, uint64_t record_bytes) {
    switch (t) {
        case HUSKY_TYPE_DATETIME: return 13 * n;
        case HUSKY_TYPE_BIGINT: return record_bytes + 3 * n;      // head + shortest form (empty: 00)
        case HUSKY_TYPE_DECIMAL: return 24 * n;                    // 1 + 2 + 20 digit bytes + FF
        case HUSKY_TYPE_TUPLE: return 2 * record_bytes + 10 * n;  // escaped string + 00 00 + 8
        default: return 0;
    }
}

struct TypedLayout {
    size_t sort, key_off, lens, tiles, bad, keys, total;
};

TypedLayout typed_layout(int t, uint64_t n, uint64_t record_bytes) {
    TypedLayout T{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    T.sort = take(make_layout(n, 1).total);
    if (t == HUSKY_TYPE_DATETIME || !typed_fixed(t)) {
        T.key_off = take((n + 1) * 8);
        T.lens = take(n * 8);
        T.tiles = take((size_t)typed_scan_tiles((uint32_t)n) * 8 + 8);
        T.bad = take(4);
        T.keys = take(typed_key_bound(t, n, record_bytes) + 16);
    }
    T.total = o;
    return T;
}

__global__ void k_add_u32(uint32_t* dst, const uint32_t* src) { *dst += *src; }
}  // namespace

size_t husky_typed_workspace_bytes(husky_type type, uint64_t n, uint64_t record_bytes) {
    if (type < HUSKY_TYPE_INT32 || type > HUSKY_TYPE_TUPLE) return 0;
    return typed_layout(type, n, record_bytes).total;
}

husky_status husky_encode_typed(husky_type type, const void* records, const uint64_t* offsets_or_null,
                                uint64_t n, int32_t base_year, uint64_t* codes, uint32_t* status,
                                void* stream) {
    if (type < HUSKY_TYPE_INT32 || type > HUSKY_TYPE_TUPLE || n >= (1ull << 32)) return HUSKY_ERR_ARG;
    if (n > 0 && (!records || !codes)) return HUSKY_ERR_ARG;
    if (!typed_fixed(type) && n > 0 && !offsets_or_null) return HUSKY_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (typed_fixed(type))
        return hip_status(typed_fixed_codes(type, records, (uint32_t)n, base_year, codes, nullptr, status, s));
    return hip_status(typed_key_codes(type, records, offsets_or_null, (uint32_t)n, codes, status, s));
}

husky_status husky_sort_typed(husky_type type, const void* records, const uint64_t* offsets_or_null,
                              uint64_t n, uint64_t record_bytes, int32_t base_year, uint32_t* perm,
                              void* ws, size_t ws_bytes, const husky_tuning* tuning, void* stream) {
    if (type < HUSKY_TYPE_INT32 || type > HUSKY_TYPE_TUPLE || n >= (1ull << 32)) return HUSKY_ERR_ARG;
    if (n > 0 && (!records || !perm)) return HUSKY_ERR_ARG;
    if (!typed_fixed(type) && n > 0 && !offsets_or_null) return HUSKY_ERR_ARG;
    Tune tn;
    husky_status st = resolve_tuning(tuning, &tn);
    if (st != HUSKY_OK) return st;
    const TypedLayout T = typed_layout(type, n, record_bytes);
    if (!ws || ((uintptr_t)ws) % ALIGN || ws_bytes < T.total) return HUSKY_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    uint8_t* base = (uint8_t*)ws;
    const uint32_t nn = (uint32_t)n;
    if (!typed_fixed(type)) {
        // Step 0: order keys of the records; then Huskysort of the keys with
        // the full-byte coder (its code is the record's husky code)
        uint32_t* bad = (uint32_t*)(base + T.bad);
        uint64_t* key_off = (uint64_t*)(base + T.key_off);
        uint8_t* keys = base + T.keys;
        HUSKY_TRY(zero_u32(bad, 1, s));
        HUSKY_TRY(typed_keys(type, records, offsets_or_null, nn, (uint64_t*)(base + T.lens),
                             (uint64_t*)(base + T.tiles), key_off, keys, bad, s));
        st = sort_common(HUSKY_CODER_BYTES8, keys, key_off, n, nullptr, 1, perm, base + T.sort,
                         make_layout(n, 1).total, tuning, stream);
        if (st != HUSKY_OK) return st;
        hipLaunchKernelGGL(k_add_u32, dim3(1), dim3(1), 0, s, (uint32_t*)(base + T.sort), (const uint32_t*)bad);
        return hip_status(hipGetLastError());
    }
    Ctx c = make_ctx(base + T.sort, n, 1);
    HUSKY_TRY(zero_u32((uint32_t*)c.status, STATUS_WORDS, s));
    if (n == 0) return HUSKY_OK;
    uint64_t* codes = c.at<uint64_t>(c.L.codes_a);
    uint64_t* codes_b = c.at<uint64_t>(c.L.codes_b);
    HUSKY_TRY(typed_fixed_codes(type, records, nn, base_year, codes, perm, &c.status->domain_violations, s));
    HUSKY_TRY(radix_segments_single(nn, c.rad, tn.rc, s));
    const uint32_t tb = tiles_bound(n, 1, tn.rc);
    HUSKY_TRY(radix_reduce_tiles(codes, tb, c.rad, tn.rc, s));
    HUSKY_TRY(radix_exec_masks(0, 64, 1, tb, c.rad, tn.rc, s));
    HUSKY_TRY(radix_sort_segments(codes, perm, codes_b, c.at<uint32_t>(c.L.idx_b), 0, 64, 1, tb, ~0u, c.rad,
                                  tn.rc, P_SCATTER, s));
    if (type != HUSKY_TYPE_DATETIME) return HUSKY_OK;  // perfect codes: nothing left to fix
    // date-times outside the window share codes: Step 3 on their 13-byte
    // field keys, compared from the first byte
    uint64_t* key_off = (uint64_t*)(base + T.key_off);
    uint8_t* keys = base + T.keys;
    HUSKY_TRY(typed_keys(type, records, nullptr, nn, nullptr, nullptr, key_off, keys, nullptr, s));
    const FixupArgs fa{0, keys, key_off, nn, perm, nullptr, 0u};
    HUSKY_TRY(fixup_first_keys(fa, c.at<uint64_t>(c.L.key0), s));
    return run_fixup(c, tn, HUSKY_CODER_BYTES8, 0u, keys, key_off, n, 1, codes, codes, codes_b, perm, s);
}

// ---------------------------------------------------------------- learned form

size_t husky_learned_model_bytes(void) { return learned_model_bytes(); }
size_t husky_learned_offset(int part) { return learned_model_offset(part); }
size_t husky_learned_workspace_bytes(uint64_t n) { return make_layout(n, 1, true).total; }

static husky_status check_model(const void* model, size_t model_bytes) {
    if (!model || ((uintptr_t)model) % ALIGN) return HUSKY_ERR_ARG;
    if (model_bytes < learned_model_bytes()) return HUSKY_ERR_ARG;
    return HUSKY_OK;
}

husky_status husky_learned_fit(husky_coder coder, const void* elems, const uint64_t* offsets,
                               uint64_t n, const husky_learned_params* params, void* model,
                               size_t model_bytes, void* ws, size_t ws_bytes, void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n == 0) return HUSKY_ERR_ARG;
    if ((st = check_model(model, model_bytes)) != HUSKY_OK) return st;
    husky_learned_params p{0.01, 1, 0, 65536, 0.02f, HUSKY_LEARNED_MONOTONE, 0, 0};
    if (params) {
        if (params->sample_frac != 0.0) p.sample_frac = params->sample_frac;
        if (params->seed) p.seed = params->seed;
        if (params->epochs) p.epochs = params->epochs;
        if (params->batch) p.batch = params->batch;
        if (params->lr != 0.f) p.lr = params->lr;
        p.mode = params->mode;
        p.flags = params->flags;
    }
    if (!(p.sample_frac > 0.0 && p.sample_frac <= 1.0)) return HUSKY_ERR_ARG;
    if (p.mode > HUSKY_LEARNED_CONSTANT || (p.flags & ~HUSKY_LEARNED_NO_DENSE)) return HUSKY_ERR_ARG;
    if (p.epochs > 10000 || !(p.lr > 0.f)) return HUSKY_ERR_ARG;
    if ((st = check_ws(ws, ws_bytes, n, 1, true)) != HUSKY_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Ctx c = make_ctx(ws, n, 1, true);
    const Layout& L = c.L;
    const uint32_t S = (uint32_t)std::min<uint64_t>(
        n, std::max<uint64_t>(1, (uint64_t)std::ceil(p.sample_frac * (double)n)));
    // sample regions, borrowed from the sort's (S <= n): indices in the bucket
    // id region, codes in the two code buffers, the indices the sort carries
    // in run_start / idx_b, training pairs in key0, flags in run_end, tile
    // sums in the small-run list
    uint32_t* sel = c.at<uint32_t>(L.bid);
    uint64_t* sc = c.at<uint64_t>(L.codes_a);
    uint32_t* sv = c.at<uint32_t>(L.run_start);
    float* x = c.at<float>(L.key0);
    float* y = x + S;
    uint8_t* fl = c.at<uint8_t>(L.run_end);
    uint2* tsum = c.at<uint2>(L.small);
    float* grad = c.at<float>(L.lgrad);
    float* loss_acc = grad + learned_nparam() + 1;
    HUSKY_TRY(zero_u32((uint32_t*)c.status, STATUS_WORDS, s));
    HUSKY_TRY(learned_sample(sel, S, (uint32_t)n, p.seed, s));
    HUSKY_TRY(launch_encode(coder, elems, offsets, (uint32_t)n, sc, sv, nullptr,
                            &c.status->domain_violations, s, sel, S));
    Tune tn;
    (void)resolve_tuning(nullptr, &tn);  // library defaults
    const int end_bit = coder == HUSKY_CODER_ASCII7 ? 63 : 64;
    if (S > 1) {
        HUSKY_TRY(radix_segments_single(S, c.rad, tn.rc, s));
        const uint32_t tb = tiles_bound(S, 1, tn.rc);
        HUSKY_TRY(radix_reduce_tiles(sc, tb, c.rad, tn.rc, s));
        HUSKY_TRY(radix_exec_masks(0, end_bit, 1, tb, c.rad, tn.rc, s));
        HUSKY_TRY(radix_sort_segments(sc, sv, c.at<uint64_t>(L.codes_b), c.at<uint32_t>(L.idx_b), 0,
                                      end_bit, 1, tb, ~0u, c.rad, tn.rc, P_SCATTER, s));
    }
    HUSKY_TRY(learned_prepare(model, sc, S, p.mode, p.flags, fl, tsum, x, y, s));
    uint32_t dense_keys = 0;
    HUSKY_TRY(read_u32(learned_dense_keys_ptr(model), &dense_keys, s));
    const uint32_t count = S - std::min(dense_keys, S);
    HUSKY_TRY(learned_init(model, p.seed, p.mode == HUSKY_LEARNED_UNCONSTRAINED, s));
    const bool train = p.mode == HUSKY_LEARNED_MONOTONE || p.mode == HUSKY_LEARNED_UNCONSTRAINED;
    // epochs 0: as many as give at least MIN_STEPS Adam steps (at most 200)
    uint32_t epochs = p.epochs;
    if (!epochs) {
        constexpr uint32_t MIN_STEPS = 150;
        const uint32_t per_epoch = std::max(1u, (count + p.batch - 1) / p.batch);
        epochs = std::min(200u, std::max(1u, (MIN_STEPS + per_epoch - 1) / per_epoch));
    }
    HUSKY_TRY(learned_train(model, x, y, train ? count : 0u, epochs, p.batch, p.lr,
                            p.mode != HUSKY_LEARNED_UNCONSTRAINED, c.at<float>(L.lpartial),
                            LEARN_MAX_BLOCKS, grad, loss_acc, s));
    HUSKY_TRY(learned_build_lut(model, p.mode, c.at<uint32_t>(L.ltmax), s));
    HUSKY_TRY(learned_splitters(model, sc, S, s));
    return HUSKY_OK;
}

husky_status husky_sort_learned(husky_coder coder, const void* elems, const uint64_t* offsets,
                                uint64_t n, const void* model, uint32_t* perm, void* ws,
                                size_t ws_bytes, const husky_tuning* tuning, void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n > 0 && !perm) return HUSKY_ERR_ARG;
    if ((st = check_model(model, learned_model_bytes())) != HUSKY_OK) return st;
    Tune tn;
    if ((st = resolve_tuning(tuning, &tn)) != HUSKY_OK) return st;
    if ((st = check_ws(ws, ws_bytes, n, 1, true)) != HUSKY_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Ctx c = make_ctx(ws, n, 1, true);
    const Layout& L = c.L;
    HUSKY_TRY(zero_u32((uint32_t*)c.status, STATUS_WORDS, s));
    if (n == 0) return HUSKY_OK;
    uint64_t* codes = c.at<uint64_t>(L.codes_a);
    uint64_t* codes_b = c.at<uint64_t>(L.codes_b);
    uint32_t* idx_b = c.at<uint32_t>(L.idx_b);
    uint16_t* bid_a = c.at<uint16_t>(L.bid);
    uint16_t* bid_b = bid_a + n;
    uint64_t* bseg = c.at<uint64_t>(L.bseg);
    const uint32_t nn = (uint32_t)n;
    // codes, first refinement keys and bucket ids in one pass over the strings,
    // then two stable 8-bit passes over the ids (low byte, high byte) that
    // carry (code, index, id, first refinement key); the first pass takes the
    // indices from the input order
    uint64_t* key0 = c.at<uint64_t>(L.key0);
    uint64_t* k0a = c.at<uint64_t>(L.k0a);
    uint64_t* k0b = c.at<uint64_t>(L.k0b);
    const BucketArgs ba = learned_bucket_args(model, bid_a);
    HUSKY_TRY(launch_encode(coder, elems, offsets, nn, codes, nullptr, key0,
                            &c.status->domain_violations, s, nullptr, 0, &ba));
    HUSKY_TRY(learned_bucket_pass(0, codes, nullptr, bid_a, key0, codes_b, idx_b, bid_b, k0b, nn,
                                  c.rad.cnt, c.rad.gtot, c.rad.binstart, s));
    HUSKY_TRY(learned_bucket_pass(1, codes_b, idx_b, bid_b, k0b, codes, perm, bid_a, k0a, nn,
                                  c.rad.cnt, c.rad.gtot, c.rad.binstart, s));
    RunItem* scan = c.at<RunItem>(L.scan);
    RunItem* biglist = c.at<RunItem>(L.biglist);
    uint32_t* scan_count = c.counters + CNT_SCAN;
    uint32_t* big_count = c.counters + CNT_BIG;
    uint32_t* class_count = c.counters + CNT_CLASS;
    RunItem* const classes[4] = {c.at<RunItem>(L.classes), c.at<RunItem>(L.classes) + LEARNED_BUCKETS,
                                 c.at<RunItem>(L.classes) + 2 * LEARNED_BUCKETS,
                                 c.at<RunItem>(L.classes) + 3 * LEARNED_BUCKETS};
    HUSKY_TRY(zero_u32(scan_count, 6, s));  // scan, big, four classes
    HUSKY_TRY(learned_bucket_bounds(bid_a, nn, bseg, &c.status->overflow_buckets, biglist, big_count,
                                    scan, scan_count, classes, class_count, s));
    // buckets of at most LEARNED_LDS_CAP keys, in LDS: by code, then by the
    // first refinement key inside runs of equal codes; their codes become tie
    // keys, and those with a group still tied join the scan list
    const uint32_t B = LEARNED_BUCKETS;
    RunItem* const fallback[4] = {c.at<RunItem>(L.fallback), c.at<RunItem>(L.fallback) + LEARNED_BUCKETS,
                                  c.at<RunItem>(L.fallback) + 2 * LEARNED_BUCKETS,
                                  c.at<RunItem>(L.fallback) + 3 * LEARNED_BUCKETS};
    HUSKY_TRY(zero_u32(c.counters + CNT_FALLBACK, 4, s));
    // the size classes of the LDS sort (two on each side stream) and the
    // radix passes of the larger buckets (on s) touch disjoint buckets and run
    // side by side
    const SideStreams* ss = nullptr;
    HUSKY_TRY(side_fork(s, n, &ss));
    HUSKY_TRY(learned_bucket_refine(coder, codes, perm, k0a, classes, class_count, fallback,
                                    c.counters + CNT_FALLBACK, scan, scan_count, 0, 2,
                                    ss ? ss->st[0] : s));
    HUSKY_TRY(learned_bucket_refine(coder, codes, perm, k0a, classes, class_count, fallback,
                                    c.counters + CNT_FALLBACK, scan, scan_count, 2, 4,
                                    ss ? ss->st[1] : s));
    // larger buckets: the multi-tile radix passes on the code
    HUSKY_TRY(radix_segments_from_items(biglist, big_count, B, c.rad, tn.rc, s));
    const int end_bit = coder == HUSKY_CODER_ASCII7 ? 63 : 64;
    const uint32_t tb = tiles_bound(n, B, tn.rc);
    HUSKY_TRY(radix_reduce_tiles(codes, tb, c.rad, tn.rc, s));
    HUSKY_TRY(radix_exec_masks(0, end_bit, B, tb, c.rad, tn.rc, s));
    c.rad.dig_in_vals = n <= DIG_IN_VALS_MAX;  // the values are string indices
    HUSKY_TRY(radix_sort_segments(codes, perm, codes_b, idx_b, 0, end_bit, B, tb, ~0u, c.rad, tn.rc,
                                  P_SCATTER, s, false));
    HUSKY_TRY(side_join(s, ss));
    // Step 3 scans only the listed buckets: the larger ones and those with a
    // group still tied (equal codes share a bucket, so no run crosses one)
    HUSKY_TRY(radix_segments_from_items(scan, scan_count, B, c.rad, tn.rc, s));
    return run_fixup(c, tn, coder, coder_m(coder), elems, offsets, n, B, codes, codes, codes_b, perm, s);
}

husky_status husky_learned_buckets(husky_coder coder, const void* elems, const uint64_t* offsets,
                                   uint64_t n, const void* model, uint16_t* bucket,
                                   uint32_t* status, void* stream) {
    husky_status st = check_common(coder, elems, offsets, n);
    if (st != HUSKY_OK) return st;
    if (n > 0 && !bucket) return HUSKY_ERR_ARG;
    if ((st = check_model(model, learned_model_bytes())) != HUSKY_OK) return st;
    const BucketArgs ba = learned_bucket_args(model, bucket);
    return hip_status(launch_encode(coder, elems, offsets, (uint32_t)n, nullptr, nullptr, nullptr,
                                    status, (hipStream_t)stream, nullptr, 0, &ba));
}

size_t husky_mlp_grad_workspace_bytes(uint32_t count) {
    const uint32_t blocks = std::max(1u, std::min(LEARN_MAX_BLOCKS, (count + 255) / 256));
    return learned_partial_bytes(blocks);
}

husky_status husky_mlp_grad(const float* params, const float* x, const float* y, uint32_t count,
                            int monotone, float* grad, void* ws, size_t ws_bytes, void* stream) {
    if (!params || !grad) return HUSKY_ERR_ARG;
    if (count > 0 && (!x || !y)) return HUSKY_ERR_ARG;
    if (!ws || ws_bytes < husky_mlp_grad_workspace_bytes(count)) return HUSKY_ERR_WORKSPACE;
    return hip_status(learned_grad(params, x, y, count, monotone != 0, (float*)ws, LEARN_MAX_BLOCKS,
                                   grad, (hipStream_t)stream));
}

size_t husky_learned_lut_workspace_bytes(void) { return (size_t)learned_lut_tiles() * 4; }

husky_status husky_learned_eval_lut(const float* params, int mode, const void* model, uint32_t* lut,
                                    void* ws, size_t ws_bytes, void* stream) {
    if (!lut || (!params && (mode == HUSKY_LEARNED_MONOTONE || mode == HUSKY_LEARNED_UNCONSTRAINED ||
                             mode == HUSKY_LEARNED_UNTRAINED)))
        return HUSKY_ERR_ARG;
    if (mode < 0 || mode > HUSKY_LEARNED_CONSTANT) return HUSKY_ERR_ARG;
    husky_status st = check_model(model, learned_model_bytes());
    if (st != HUSKY_OK) return st;
    if (!ws || ws_bytes < husky_learned_lut_workspace_bytes()) return HUSKY_ERR_WORKSPACE;
    return hip_status(learned_eval_lut(params, model, (uint32_t)mode, lut, (uint32_t*)ws,
                                       (hipStream_t)stream));
}

const char* husky_status_string(husky_status s) {
    switch (s) {
        case HUSKY_OK: return "ok";
        case HUSKY_ERR_ARG: return "invalid argument";
        case HUSKY_ERR_DOMAIN: return "ASCII7 byte >= 0x80 among the first nine bytes";
        case HUSKY_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
        case HUSKY_ERR_HIP: return "HIP runtime error";
        case HUSKY_ERR_UNSUPPORTED: return "tuning value not supported";
        case HUSKY_ERR_UNRESOLVED: return "groups still tied after the fixed refinement rounds";
        case HUSKY_ERR_TOO_LARGE: return "more strings than the no-allocation scratch holds";
    }
    return "unknown status";
}

}  // extern "C"
