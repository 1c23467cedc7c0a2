// Internal declarations shared by the HIP sources of libturboreg (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/turboreg.h"

namespace tr {

constexpr int kSc2Tile = 256;     // output tile edge of the FP4 MFMA SC2 kernel; npad is a multiple
constexpr int kHistGroups = 8;    // SC2 tiles add their weight histograms into this many copies per pair
constexpr int kCompatTile = 64;   // tile edge of the compatibility kernel
// Row pitch of C in bytes: npad / 2 packed entries, plus 64 bytes where npad / 2 is a multiple
// of 512, so that the rows an SC2 stage reads (one 64-byte chunk of each of 256 rows) are not all
// at one offset modulo 512 bytes. At N = 5000 (npad / 2 = 2560) the padding made the SC2 kernel
// 1.2-1.9 us faster; padding every pitch made the uneven 256-pair batch 1 % slower.
constexpr int kCRowPad = 64;
__host__ __device__ inline int64_t c_pitch(int32_t npad)
{
    return npad / 2 + ((npad & 1023) == 0 ? kCRowPad : 0);
}
constexpr int kRowsPerItem = 4;   // rows per work item of the pivot scans (one per wave)
constexpr int kPrepRows = 256;    // rows per work item of the prep / feature kernels
constexpr int kRankSortMax = 4096; // candidate lists up to this size are ordered by a rank sort
constexpr int kScoreHyp = 64;     // hypotheses per scoring work item (four per thread)
constexpr int kScorePts = 256;    // points per scoring work item (staged in LDS)
// Counters that many workgroups update with device-scope atomics are spread out: same-address
// device atomics are served one after another, so one shared counter serialises the stage.
constexpr int kCollectRegions = 8; // pivot collection: one pool region and counter per XCD
constexpr int kHypGroup = 16;     // clique-search items per first-level ticket
constexpr int kTickLine = 32;     // int32 per counter: one counter per 128-byte line
constexpr int kTickHyp0 = kCollectRegions;      // first clique-search group ticket
constexpr int kFusedPool = 512;   // learned pools up to this size are reordered inside the hypothesis kernel

// Work-list stages whose per-pair item counts depend on N_b; each has a
// prefix array of B+1 entries in Work::pre, over the pairs in cost order.
enum Stage { kPrep = 0, kCompat, kSc2, kRowBlk, kScore, kNumPrefix };
// Rows of Work::pre after the stage prefixes: the cost order (slot -> pair), its inverse.
constexpr int kOrderRow = kNumPrefix, kSlotRow = kNumPrefix + 1, kPreRows = kNumPrefix + 2;

struct PairDesc {
    int32_t n;        // matches in this pair (0 when the pair is invalid)
    int32_t npad;     // n rounded up to kSc2Tile
    int32_t pt_off;   // first match of this pair in src/dst
    int32_t kpiv;     // pivots to select: min(k1 or pool, n(n-1)/2)
    int64_t c_off;    // entry offset of this pair in the npad x npad arenas (the bit rows of C: c_off / 8 bytes)
    int64_t g_off;    // element offset of this pair's G in the G arena (npad x npad uint16)
    int64_t cb_off;   // byte offset of this pair's C (E2M1 nibbles, npad rows of c_pitch(npad) bytes)
};

// Per-pair scalars written by the kernels.
struct PairState {
    int32_t status;     // tr_status
    int32_t nonfinite;  // 1 if any coordinate is NaN/Inf (summed from the compatibility tiles)
    int32_t n_boundary;
    int32_t n_edges;
    int32_t alpha;      // weight of the last pivot (the K-th largest, Eq. 4)
    int32_t c_gt;       // edges heavier than alpha (all selected)
    int32_t m_eq;       // edges of weight alpha to take, in lexicographic order
    int32_t fallback;   // learned scores were not finite
    int32_t fast;       // every pair of weight >= alpha fits the pivot pool: collected unordered, then sorted
    int32_t ncand;      // keys the sort ranks (fast: c_gt + all ties; else K)
    int32_t done;       // ticket groups of the clique-search stage that have finished this pair
};

struct Plan {
    int32_t B;
    int32_t total[kNumPrefix];
    int32_t sc2_split[9];   // SC2 items [sc2_split[x], sc2_split[x+1]) go to XCD x: equal modelled cost
};

// Device views passed to every kernel.
struct Work {
    const float *src, *dst;
    const PairDesc *pairs;
    PairState *state;
    const Plan *plan;
    const int32_t *pre;       // kPreRows x (max_batch + 1): per stage, the first item of the pair in
                              // each slot of the cost order (largest pairs first); then the order
                              // (slot -> pair) and its inverse (pair -> slot)
    int32_t pre_stride;       // max_batch + 1
    int32_t n1;               // N of a single-pair call (its plan is computed in registers), 0 for a batch
    int32_t max_n;            // per-pair row stride of the per-row arenas
    int32_t k1, k2, pool;     // pool = plain pivots selected (k1, or pool_factor*k1 in learned mode)
    int32_t H;                // k1 * k2 hypotheses per pair
    int32_t graph;
    int32_t sc2_super;        // SC2 tile walk: super-tile side in output tiles (launch configuration)
    int32_t sc2_sparse_cap;   // SC2 tiles with at most this many edges take the bit-count path; 0: none
                              // does, and Cbits is not written (launch configuration)
    float tau, theta;
    uint8_t *C;               // C arena (E2M1 nibbles, the MFMA operands)
    uint8_t *Cbits;           // C arena as bits: per pair npad x npad bits in blocks of 128 columns,
                              // [column / 128][row][16 bytes] (bit c % 8 of byte (c % 128) / 8); offset c_off / 8
    uint16_t *G;              // G arena
    int32_t *ghist;           // max_batch x kHistGroups x hist_stride weight histograms (filled by the SC2 epilogue)
    int32_t hist_stride;      // max_n rounded up to 8 (16-byte aligned copies)
    int32_t *rowmax;          // max_batch x max_n: max_{j>i} G_ij (filled by the SC2 epilogue)
    int32_t *cnt_part;        // per compatibility work item: (boundary pairs, edges, non-finite input)
    int32_t *rowcnt;          // max_batch x max_n: pairs of weight alpha per row (ordered path)
    uint64_t *rowseg;         // max_batch x max_n: bit s set if the row's s-th 512-column segment (counted
                              // from its first column j > i) holds a pair of weight alpha (ordered path)
    int32_t *blkcnt;          // max_batch x nblk: pairs of weight alpha per block of kRowsPerItem rows
    int32_t nblk_stride;      // blocks of kRowsPerItem rows per pair (for max_n)
    uint64_t *cand;           // max_batch x kCollectRegions x pool_cap selection candidates (sort keys); the
                              // ordered path writes region 0 only
    int32_t *tick;            // max_batch x tick_stride counters, kTickLine apart: kCollectRegions collection
                              // counters, then one ticket per group of kHypGroup clique-search items
    int32_t tick_stride;
    uint64_t *hyp_rec;        // max_batch x rec_stride: per clique-search item, its best key and valid count
    int32_t rec_stride;       // 2 x the most clique-search items of a pair (k1_cap / 4, rounded up)
    int32_t pool_cap;
    int32_t *pivots_plain;    // max_batch x pool_cap x 3
    int32_t *pivots;          // pivots the clique search uses: max_batch x piv_stride x 3
    int32_t piv_stride;       // pool_cap in plain mode (pivots == pivots_plain), k1_cap in learned mode
    int32_t *cliques;         // max_batch x h_cap x 3
    float *poses;             // max_batch x h_cap x 12
    int32_t *inl;             // max_batch x h_cap
    float *gscore;            // max_batch x h_cap error-based scores (metric != 0)
    int32_t metric;           // hypothesis ranking: 0 inlier number, 1 MAE form, 2 MSE form
    int32_t h_cap;
    int32_t *rowstat;         // max_batch x max_n x 20 feature accumulators (learned mode)
    int32_t *mark;            // max_batch x max_n: row claimed by a candidate-feature workgroup
    int32_t feat_all;         // learned features for every match (training) instead of the pool's
    uint16_t *feat;           // max_batch x max_n x 19 bfloat16 features
    float *scores;            // max_batch x max_n learned scores
    tr_result *out;
    uint8_t *masks;           // nullable; pair b's mask starts at pairs[b].pt_off
    int32_t learned;          // learned pivot mode / feature accumulation on
    int32_t rank_in_hyp;      // learned pool of at most kFusedPool entries: the hypothesis kernel orders it
    // Profiled calls only (null otherwise): the hypothesis kernel's phase durations in ticks of
    // the 100 MHz real-time clock, per work item (max_batch x rec_stride / 2 x 4: clique search,
    // rigid fits, scoring, records), and their sums over calls (kProfSlots counters).
    uint32_t *hyp_prof;
    unsigned long long *prof_acc;
};

// Sums of the hypothesis kernel's phases over profiled calls (prof_acc slots).
enum { kProfSearch = 0, kProfFit, kProfScore, kProfRecords, kProfSelect, kProfItems, kProfPairs, kProfSlots };


// Largest b in [0, B) with pre[b] <= item (pre is non-decreasing, pre[0] = 0).
// Length of a difference vector in float32: first square rounded, the other
// two fused, then the correctly rounded square root (the order is part of the
// bit-exact contract of C).
__device__ __forceinline__ float length32(float ax, float ay, float az)
{
    float s = ax * ax;
    s = __builtin_fmaf(ay, ay, s);
    s = __builtin_fmaf(az, az, s);
    return __builtin_sqrtf(s);
}

// Learned reorder key of plain pool entry r (smaller = earlier): e = s_i + s_j descending, then
// the plain rank r; keys are distinct. fb: the pair's scores are not all finite, keep plain order.
__device__ __forceinline__ uint64_t reorder_key(const int32_t *pl, const float *sc, int r, bool fb)
{
    uint32_t hi = 0;
    if (!fb) {
        const float e = (sc[pl[3 * r]] + sc[pl[3 * r + 1]]) + 0.0f;   // +0.0f folds -0 into +0
        const uint32_t u = __float_as_uint(e);
        const uint32_t ord = (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // ascending float order
        hi = ~ord;                                                            // descending
    }
    return ((uint64_t)hi << 32) | (uint32_t)r;
}

// Number of the keys in [q0, q1) (LDS, padded with ~0 to a multiple of 16) smaller than `mine`,
// eight 16-byte broadcast reads in flight; q0, q1 multiples of 16.
__device__ __forceinline__ int count_smaller(const uint64_t *keys, int q0, int q1, uint64_t mine)
{
    int rk = 0;
    for (int q = q0; q < q1; q += 16) {
        uint4 a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = *reinterpret_cast<const uint4 *>(&keys[q + 2 * u]);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            rk += (((uint64_t)a[u].y << 32) | a[u].x) < mine;
            rk += (((uint64_t)a[u].w << 32) | a[u].z) < mine;
        }
    }
    return rk;
}

__device__ __forceinline__ int find_pair(const int32_t *pre, int B, int item)
{
    int lo = 0, hi = B - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Per-pair sizes of a valid pair (3 <= n <= max_n): the descriptor and the
// work items of every stage. The device planner and single-pair calls (which
// compute their plan in registers) use the same formulas.
__host__ __device__ inline PairDesc pair_desc_of(int32_t n, int32_t pt_off, int64_t arena_off, int64_t c_bytes_off,
                                                 int32_t pool)
{
    PairDesc d;
    d.n = n;
    d.npad = (n + kSc2Tile - 1) / kSc2Tile * kSc2Tile;
    d.pt_off = pt_off;
    const int64_t pairs_all = (int64_t)n * (n - 1) / 2;
    d.kpiv = (int32_t)(pairs_all < pool ? pairs_all : pool);
    d.c_off = arena_off;
    d.g_off = arena_off;
    d.cb_off = c_bytes_off;
    return d;
}

__host__ __device__ inline int64_t stage_items(int stage, int32_t n, int32_t H)
{
    const int64_t npad = (n + kSc2Tile - 1) / kSc2Tile * kSc2Tile;
    const int64_t nb64 = npad / kCompatTile, nbs = npad / kSc2Tile;
    switch (stage) {
    case kPrep: return (n + kPrepRows - 1) / kPrepRows;
    case kCompat: return nb64 * (nb64 + 1) / 2;
    case kSc2: return nbs * (nbs + 1) / 2;
    case kRowBlk: return (n + kRowsPerItem - 1) / kRowsPerItem;
    default: return (int64_t)((H + kScoreHyp - 1) / kScoreHyp) * ((n + kScorePts - 1) / kScorePts);
    }
}

// Work lists: all items of a stage, pair after pair, in the plan's slot order: for batches of
// 16 pairs or more, the pairs sorted by decreasing size (npad; pairs of one size in index order) and dealt to the eight XCDs, each
// XCD's pairs in size order, so that eight SC2 ranges of equal cost hold like mixes of sizes and
// a workgroup striding through a list takes costly items first. A single-pair call (n1 > 0)
// derives everything from n1; a batch reads the device plan.
__device__ __forceinline__ int stage_total(const Work &w, int stage)
{
    return w.n1 ? (int)stage_items(stage, w.n1, w.H) : w.plan->total[stage];
}

// The pair in slot k of the cost order (kernels with one workgroup, or a fixed number, per
// pair take their pairs in this order too).
__device__ __forceinline__ int batch_pair(const Work &w, int k)
{
    return w.n1 ? k : w.pre[kOrderRow * w.pre_stride + k];
}

// The pair an item belongs to, and the item's index inside that pair.
__device__ __forceinline__ int stage_pair(const Work &w, int stage, int item, int &local)
{
    if (w.n1) {
        local = item;
        return 0;
    }
    const int32_t *pre = w.pre + stage * w.pre_stride;
    const int k = find_pair(pre, w.plan->B, item);
    local = item - pre[k];
    return w.pre[kOrderRow * w.pre_stride + k];
}

// The same lookup from a copy in LDS of a stage's prefix sums and the slot order, for kernels
// with many short items (the binary search then takes no device-memory round trips). Batches of
// at most kSlotCacheMax pairs; the copy is made by slot_cache_fill, followed by a barrier.
constexpr int kSlotCacheMax = 1024;
struct SlotCache {
    int32_t pre[kSlotCacheMax + 1];
    int32_t order[kSlotCacheMax];
};

__device__ __forceinline__ bool slot_cache_fill(const Work &w, int stage, SlotCache &c)
{
    if (w.n1 || w.plan->B > kSlotCacheMax) return false;
    const int B = w.plan->B;
    for (int k = threadIdx.x; k <= B; k += blockDim.x) {
        c.pre[k] = w.pre[stage * w.pre_stride + k];
        if (k < B) c.order[k] = w.pre[kOrderRow * w.pre_stride + k];
    }
    return true;
}

__device__ __forceinline__ int stage_pair_cached(const Work &w, int stage, const SlotCache &c, bool cached, int item,
                                                 int &local)
{
    if (!cached) return stage_pair(w, stage, item, local);
    const int k = find_pair(c.pre, w.plan->B, item);
    local = item - c.pre[k];
    return c.order[k];
}

// First item of pair b in a stage's list, and its item count.
__device__ __forceinline__ int stage_first(const Work &w, int stage, int b)
{
    return w.n1 ? 0 : w.pre[stage * w.pre_stride + w.pre[kSlotRow * w.pre_stride + b]];
}

__device__ __forceinline__ int stage_count(const Work &w, int stage, int b)
{
    if (w.n1) return (int)stage_items(stage, w.n1, w.H);
    const int k = w.pre[kSlotRow * w.pre_stride + b];
    return w.pre[stage * w.pre_stride + k + 1] - w.pre[stage * w.pre_stride + k];
}

__device__ __forceinline__ PairDesc pair_desc(const Work &w, int b)
{
    return w.n1 ? pair_desc_of(w.n1, 0, 0, 0, w.pool) : w.pairs[b];
}

// Ascending bitonic sort of P keys in LDS by one workgroup (P a power of two,
// P >= 64). Stages with stride >= 64 exchange through LDS; the stages with
// stride < 64 of each merge run on 64-key blocks held one key per lane and
// exchanged with wave shuffles, so a merge costs one barrier per LDS stage
// plus one.
__device__ inline void bitonic_sort_lds(uint64_t *keys, int P)
{
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nthr >> 6;
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride >= 64; stride >>= 1) {
            for (int t = tid; t < P / 2; t += nthr) {
                const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = keys[lo], c = keys[hi];
                if ((a > c) == up) { keys[lo] = c; keys[hi] = a; }
            }
            __syncthreads();
        }
        for (int blk = wv; blk < P / 64; blk += nw) {
            const int p = blk * 64 + lane;
            const bool up = (p & size) == 0;
            uint64_t key = keys[p];
            for (int stride = (size >> 1) < 32 ? (size >> 1) : 32; stride >= 1; stride >>= 1) {
                const uint64_t other = __shfl_xor(key, stride, 64);
                const bool keep_min = ((lane & stride) == 0) == up;
                key = keep_min ? (key < other ? key : other) : (key > other ? key : other);
            }
            keys[p] = key;
        }
        __syncthreads();
    }
}

// ---- launchers (one per kernel family); each returns the launch's hipError_t ----
hipError_t launch_plan(const Work &w, const int32_t *offsets, int32_t n_single, int32_t B,
                       int32_t max_n, PairDesc *pairs, PairState *state, Plan *plan, int32_t *pre,
                       hipStream_t s);
hipError_t launch_compat(const Work &w, int grid, hipStream_t s);
hipError_t launch_sc2(const Work &w, int grid, hipStream_t s);
hipError_t launch_pivots(const Work &w, int B, int grid_rows, hipStream_t s);
hipError_t launch_prep_learned(const Work &w, int grid, hipStream_t s);
hipError_t launch_hyp(const Work &w, int B, int ppw, int grid, hipStream_t s);
hipError_t launch_fit_triplets(const float *src, const float *dst, int n, const int32_t *tri, int T, float *poses,
                               int32_t *ok, int grid, hipStream_t s);
hipError_t launch_score_poses(const float *src, const float *dst, int n, const float *poses, int P, float theta,
                              int metric, int32_t *in_out, float *score_out, int grid, hipStream_t s);
hipError_t setup_hyp_kernels();

// Once per process and device, before any launch (and so outside stream capture):
// raise the dynamic-LDS limits of the kernels that need more than 64 KiB.
hipError_t setup_graph_kernels();
hipError_t setup_pivot_kernels();

}  // namespace tr
