// libturboreg host side: handle and workspace, the launch sequence of the
// registration path, hipGraph capture for batches, and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <type_traits>
#include <vector>

#include "common.h"
#include "mlp.h"

using namespace tr;

namespace {

struct GraphKey {
    const void *src, *dst, *offsets, *out, *masks;
    void *stream;
    int32_t B, max_n;
    tr_params p;
    tr_tuning cfg;
    bool operator<(const GraphKey &o) const
    {
        return std::memcmp(this, &o, sizeof(GraphKey)) < 0;
    }
};

}  // namespace

struct tr_handle {
    int device = 0;
    int num_cus = 256;
    char arch[64] = "unknown";   // gcnArchName of the device (tuning files are per architecture and CU count)
    int32_t max_n = 0, max_batch = 0, max_k1 = 0, max_k2 = 0;
    int32_t npad_max = 0, pool_cap = 0, k1_cap = 0, h_cap = 0, nblk_stride = 0, pre_stride = 0;
    // workspace
    PairDesc *pairs = nullptr;
    PairState *state = nullptr;
    Plan *plan = nullptr;
    int32_t *pre = nullptr;
    uint8_t *C = nullptr, *Cbits = nullptr;
    uint16_t *G = nullptr;
    int32_t *ghist = nullptr, *rowmax = nullptr, *cnt_part = nullptr, *rowcnt = nullptr, *blkcnt = nullptr;
    uint64_t *cand = nullptr, *rowseg = nullptr, *hyp_rec = nullptr;
    int32_t *tick = nullptr;
    int32_t tick_stride = 0, rec_stride = 0;
    int32_t *pivots_plain = nullptr, *pivots = nullptr, *cliques = nullptr, *inl = nullptr;
    float *poses = nullptr, *gscore = nullptr;
    int32_t *rowstat = nullptr, *mark = nullptr;
    uint16_t *feat = nullptr;
    float *scores = nullptr;
    tr_result *scratch_out = nullptr;   // results of feature-only passes
    uint32_t *hyp_prof = nullptr;       // profiled calls: per-item phase durations of the hypothesis kernel
    unsigned long long *prof_acc = nullptr;   // and their sums (kProfSlots)
    // learned scorer
    MlpState mlp;
    bool has_scorer = false;
    // last call, for inspection
    Work last{};
    int32_t last_B = 0;
    hipStream_t last_stream = nullptr;
    bool last_valid = false;
    // profiling: a ring of event sets, one set per profiled call, read without
    // stalling the stream; per-stage sums over the calls since the last read
    static constexpr int kRing = 256;
    std::vector<hipEvent_t> ring;          // kRing x (TR_NUM_STAGES + 1)
    std::vector<char> ring_pending;        // 0 free, 1 all stages recorded, 2 only the SC2 stage
    std::vector<uint32_t> ring_mask;       // bit k: event k of the set was recorded (a stage with a kernel)
    int64_t ring_next = 0;
    double stage_sum[TR_NUM_STAGES] = {};
    int64_t stage_calls[TR_NUM_STAGES] = {};
    // captured batches, at most kMaxGraphs, the least recently launched evicted first
    struct Captured {
        hipGraph_t g;
        hipGraphExec_t ge;
        uint64_t last_use;
    };
    static constexpr size_t kMaxGraphs = 8;
    std::map<GraphKey, Captured> graphs;
    uint64_t graph_clock = 0;
    // launch configurations by (256-row tiles of the largest pair, batch size)
    std::map<std::pair<int32_t, int32_t>, tr_tuning> tuning;
    std::vector<void *> allocs;
};

namespace {

template <typename T>
hipError_t alloc(tr_handle *h, T **p, size_t count)
{
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    h->allocs.push_back(q);
    *p = static_cast<T *>(q);
    return hipSuccess;
}

void release(tr_handle *h)
{
    for (auto &g : h->graphs) {
        hipGraphExecDestroy(g.second.ge);
        hipGraphDestroy(g.second.g);
    }
    h->graphs.clear();
    for (auto &e : h->ring)
        if (e) hipEventDestroy(e);
    h->ring.clear();
    mlp_release(&h->mlp);
    for (void *p : h->allocs) hipFree(p);
    h->allocs.clear();
}

// Strides and capacities of a workspace for up to max_batch pairs of up to max_n matches,
// K1 <= max_k1 and K2 <= max_k2.
void size_handle(tr_handle *h, int32_t max_n, int32_t max_batch, int32_t max_k1, int32_t max_k2)
{
    h->max_n = max_n;
    h->max_batch = max_batch;
    h->max_k1 = max_k1;
    h->max_k2 = max_k2;
    h->npad_max = (max_n + kSc2Tile - 1) / kSc2Tile * kSc2Tile;
    h->pool_cap = std::min(TR_MAX_POOL, 8 * max_k1);
    h->k1_cap = max_k1;
    h->h_cap = max_k1 * max_k2;
    h->nblk_stride = (max_n + kRowsPerItem - 1) / kRowsPerItem;
    const int items = (max_k1 + 3) / 4;   // clique-search work items of a pair (at least 4 pivots each)
    h->rec_stride = 2 * items;
    h->tick_stride = (kTickHyp0 + (items + kHypGroup - 1) / kHypGroup) * kTickLine;
    h->pre_stride = max_batch + 1;
}

// The workspace buffers of a sized handle, in order: get(pointer member, element count) places
// each one (device allocations for a handle, a carve of the static scratch for the entry point
// that allocates nothing).
template <class Get>
void workspace_layout(tr_handle *h, Get &&get)
{
    const size_t B = h->max_batch, nn = (size_t)h->npad_max * h->npad_max, max_n = h->max_n;
    get(h->pairs, B);
    get(h->state, B);
    get(h->plan, 1);
    get(h->pre, (size_t)kPreRows * h->pre_stride);
    get(h->C, B * (nn / 2 + (size_t)h->npad_max * kCRowPad));   // packed E2M1, two entries per byte, padded rows
    get(h->Cbits, B * nn / 8);   // the same matrix as bits
    get(h->G, B * nn);
    get(h->ghist, B * kHistGroups * (size_t)((max_n + 7) & ~(size_t)7));
    get(h->rowmax, B * max_n);
    const size_t nb64 = h->npad_max / kCompatTile;
    get(h->cnt_part, B * nb64 * (nb64 + 1) / 2 * 3);   // boundary pairs, edges, non-finite flag
    get(h->rowcnt, B * max_n);
    get(h->blkcnt, B * h->nblk_stride);
    get(h->cand, B * kCollectRegions * h->pool_cap);
    get(h->tick, B * h->tick_stride);
    get(h->hyp_rec, B * h->rec_stride);
    get(h->rowseg, B * max_n);
    get(h->pivots_plain, B * h->pool_cap * 3);
    get(h->pivots, B * h->k1_cap * 3);
    get(h->cliques, B * h->h_cap * 3);
    get(h->poses, B * h->h_cap * 12);
    get(h->inl, B * h->h_cap);
    get(h->gscore, B * h->h_cap);
    get(h->rowstat, B * max_n * 20);
    get(h->mark, B * max_n);
    get(h->feat, B * max_n * 19);
    get(h->scores, B * max_n);
    get(h->scratch_out, B);
    get(h->hyp_prof, B * (size_t)h->rec_stride * 2);
    get(h->prof_acc, (size_t)kProfSlots);
}

std::pair<int32_t, int32_t> tuning_key(int32_t max_n, int32_t B)
{
    return {(max_n + kSc2Tile - 1) / kSc2Tile, B};
}

tr_tuning tuning_for(const tr_handle *h, int32_t max_n, int32_t B)
{
    auto it = h->tuning.find(tuning_key(max_n, B));
    if (it != h->tuning.end()) return it->second;
    tr_tuning t;
    t.sc2_super = 5;
    t.compat_per_cu = 8;   // twice the workgroups a CU holds: late ones fill the slots that free first
    t.hyp_ppw = B == 1 ? 4 : 16;   // batches: more pivots per workgroup, fewer passes over each pair's matches
    t.hyp_per_cu = 4;
    t.sc2_sparse_cap = 0;
    return t;
}

bool tuning_valid(const tr_tuning &t)
{
    return t.sc2_super >= 1 && t.sc2_super <= 16 && t.compat_per_cu >= 1 && t.compat_per_cu <= 16 &&
           t.hyp_ppw >= 4 && t.hyp_ppw <= 16 && t.hyp_ppw % 4 == 0 && t.hyp_per_cu >= 1 && t.hyp_per_cu <= 16 &&
           t.sc2_sparse_cap >= 0 && t.sc2_sparse_cap <= TR_SC2_SPARSE_CAP_MAX;
}

int grid_cap(tr_handle *h, int64_t items, int per_cu)
{
    int64_t cap = (int64_t)h->num_cus * per_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>(items, cap));
}

Work make_work(tr_handle *h, const float *src, const float *dst, const tr_params &p, tr_result *out,
               uint8_t *masks, bool learned, int32_t B, int32_t max_n)
{
    Work w{};
    w.src = src;
    w.dst = dst;
    w.pairs = h->pairs;
    w.state = h->state;
    w.plan = h->plan;
    w.pre = h->pre;
    w.pre_stride = h->pre_stride;
    w.n1 = 0;
    w.max_n = h->max_n;
    w.k1 = p.k1;
    w.k2 = p.k2;
    w.pool = learned ? p.k1 * p.pool_factor : p.k1;
    w.H = p.k1 * p.k2;
    w.graph = p.graph;
    w.sc2_super = 5;
    w.sc2_sparse_cap = 0;
    w.tau = p.tau;
    w.theta = p.inlier_thresh;
    w.C = h->C;
    w.Cbits = h->Cbits;
    w.G = h->G;
    w.ghist = h->ghist;
    w.hist_stride = (h->max_n + 7) & ~7;
    w.rowmax = h->rowmax;
    w.cnt_part = h->cnt_part;
    w.rowcnt = h->rowcnt;
    w.blkcnt = h->blkcnt;
    w.nblk_stride = h->nblk_stride;
    w.cand = h->cand;
    w.tick = h->tick;
    w.tick_stride = h->tick_stride;
    w.hyp_rec = h->hyp_rec;
    w.rec_stride = h->rec_stride;
    w.rowseg = h->rowseg;
    w.pool_cap = h->pool_cap;
    w.pivots_plain = h->pivots_plain;
    if (learned) { w.pivots = h->pivots; w.piv_stride = h->k1_cap; }
    else { w.pivots = h->pivots_plain; w.piv_stride = h->pool_cap; }
    w.cliques = h->cliques;
    w.poses = h->poses;
    w.inl = h->inl;
    w.gscore = h->gscore;
    w.metric = (p.flags & TR_FLAG_RANK_MAE) ? 1 : (p.flags & TR_FLAG_RANK_MSE) ? 2 : 0;
    w.h_cap = h->h_cap;
    w.rowstat = h->rowstat;
    w.mark = h->mark;
    w.feat_all = 0;
    w.feat = h->feat;
    w.scores = h->scores;
    w.out = out;
    w.masks = masks;
    w.learned = learned ? 1 : 0;
    w.rank_in_hyp = learned && w.pool <= kFusedPool ? 1 : 0;
    return w;
}

tr_status check_params(tr_handle *h, const tr_params *p)
{
    if (!p) return TR_ERR_INVALID_ARG;
    if (!(p->tau >= 0.0f) || !std::isfinite(p->tau)) return TR_ERR_INVALID_ARG;
    if (!(p->inlier_thresh >= 0.0f) || !std::isfinite(p->inlier_thresh)) return TR_ERR_INVALID_ARG;
    if ((p->flags & TR_FLAG_RANK_MAE) && (p->flags & TR_FLAG_RANK_MSE)) return TR_ERR_INVALID_ARG;
    // the error-based scores divide by theta
    if ((p->flags & (TR_FLAG_RANK_MAE | TR_FLAG_RANK_MSE)) && !(p->inlier_thresh > 0.0f)) return TR_ERR_INVALID_ARG;
    if (p->k1 < 1 || p->k2 < 1 || p->k2 > TR_MAX_K2) return TR_ERR_INVALID_ARG;
    if (p->graph != TR_GRAPH_O2 && p->graph != TR_GRAPH_SC2) return TR_ERR_INVALID_ARG;
    if (p->pivot_mode != TR_PIVOTS_PLAIN && p->pivot_mode != TR_PIVOTS_LEARNED) return TR_ERR_INVALID_ARG;
    if (p->k1 > h->max_k1 || p->k2 > h->max_k2) return TR_ERR_WORKSPACE;
    if (p->pivot_mode == TR_PIVOTS_LEARNED) {
        if (p->pool_factor < 1) return TR_ERR_INVALID_ARG;
        if ((int64_t)p->pool_factor * p->k1 > h->pool_cap) return TR_ERR_WORKSPACE;
        if (!h->has_scorer) return TR_ERR_NO_SCORER;
    }
    return TR_OK;
}

// The launch sequence for B pairs (offsets on the device) or one pair (n_single).
// features_only stops after the learned features.
tr_status enqueue(tr_handle *h, const Work &w_in, const int32_t *offsets, int32_t n_single, int32_t B,
                  int32_t max_n, hipEvent_t *ev, int ev_mode, bool features_only, hipStream_t s,
                  const tr_tuning &cfg, uint32_t *ev_mask = nullptr)
{
    uint32_t ev_mask_unused = 0;
    if (!ev_mask) ev_mask = &ev_mask_unused;
    Work w = w_in;
    w.sc2_super = cfg.sc2_super;
    w.sc2_sparse_cap = cfg.sc2_sparse_cap;
    const bool profile = ev != nullptr;
    const int64_t npad = (max_n + kSc2Tile - 1) / kSc2Tile * kSc2Tile;
    const int64_t nb64 = npad / kCompatTile, nbs = npad / kSc2Tile;
    const int64_t rows_items = (int64_t)B * ((max_n + kRowsPerItem - 1) / kRowsPerItem);
    // an event opens each stage that launches a kernel (and one closes the last); a stage without
    // a kernel records nothing, so no interval is an empty pair of events
    auto mark = [&](int stage) {
        if (profile && (ev_mode == 1 || stage == TR_STAGE_SC2 || stage == TR_STAGE_SC2 + 1)) {
            hipEventRecord(ev[stage], s);
            *ev_mask |= 1u << stage;
        }
    };
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (x != hipSuccess && e == hipSuccess) e = x;
    };
    if (profile && ev_mode == 1) {   // the hypothesis kernel adds its phase durations to the handle's sums
        w.hyp_prof = h->hyp_prof;
        w.prof_acc = h->prof_acc;
    }
    if (!w.n1 || (w.learned && w.feat_all)) mark(TR_STAGE_PLAN);
    if (!w.n1) chk(launch_plan(w, offsets, n_single, B, max_n, h->pairs, h->state, h->plan, h->pre, s));
    if (w.learned && w.feat_all)
        chk(launch_prep_learned(w, grid_cap(h, (int64_t)B * ((max_n + kPrepRows - 1) / kPrepRows), 8), s));
    mark(TR_STAGE_COMPAT);
    chk(launch_compat(w, grid_cap(h, (int64_t)B * nb64 * (nb64 + 1) / 2, cfg.compat_per_cu), s));
    mark(TR_STAGE_SC2);
    {
        // one workgroup per CU; the kernel splits its items into 8 ranges, one per XCD
        // (workgroup g runs on XCD g mod 8), of equal counts for one pair and of equal modelled
        // cost for a batch, so the grid is a multiple of 8 with as many workgroups per XCD as an
        // even range would hold items, up to the XCD's CUs
        const int64_t items = (int64_t)B * nbs * (nbs + 1) / 2;
        const int64_t per_xcd = std::min<int64_t>((items + 7) / 8, std::max(1, h->num_cus / 8));
        chk(launch_sc2(w, (int)(8 * per_xcd), s));
    }
    if (features_only) return e == hipSuccess ? TR_OK : TR_ERR_HIP;
    mark(TR_STAGE_PIVOTS);
    chk(launch_pivots(w, B, grid_cap(h, rows_items, 8), s));
    if (w.learned) mark(TR_STAGE_LEARNED);
    if (w.learned) {
        // features and scores of the pool's endpoints, then the reorder of the pool
        chk(launch_learned_order(w, h->mlp, B, h->num_cus, s));
    }
    mark(TR_STAGE_CLIQUES);
    // cliques, their poses, their inlier counts and (last workgroup per pair) the selection
    chk(launch_hyp(w, B, cfg.hyp_ppw, h->num_cus * cfg.hyp_per_cu, s));
    mark(TR_NUM_STAGES);
    if (e != hipSuccess) {
        std::fprintf(stderr, "turboreg: launch failed: %s\n", hipGetErrorString(e));
        return TR_ERR_HIP;
    }
    return TR_OK;
}

void remember(tr_handle *h, const Work &w, int32_t B, hipStream_t s)
{
    h->last = w;
    h->last_B = B;
    h->last_stream = s;
    h->last_valid = true;
}

// Fold the timings of one completed event set into the per-stage sums.
hipError_t ring_collect(tr_handle *h, int slot)
{
    hipEvent_t *ev = &h->ring[(size_t)slot * (TR_NUM_STAGES + 1)];
    const bool all = h->ring_pending[slot] == 1;
    hipError_t e = hipEventSynchronize(ev[all ? TR_NUM_STAGES : TR_STAGE_SC2 + 1]);
    if (e != hipSuccess) return e;
    // a recorded event opens its stage, which ends at the next recorded event; the cliques
    // interval is the whole hypothesis kernel (split into its phases in tr_stage_times)
    const uint32_t m = h->ring_mask[slot];
    for (int k = 0; k < TR_NUM_STAGES; ++k) {
        if (!(m & (1u << k)) || (!all && k != TR_STAGE_SC2)) continue;
        int nx = k + 1;
        while (nx < TR_NUM_STAGES && !(m & (1u << nx))) ++nx;
        float t = 0;
        e = hipEventElapsedTime(&t, ev[k], ev[nx]);
        if (e != hipSuccess) return e;
        h->stage_sum[k] += t;
        h->stage_calls[k] += 1;
    }
    h->ring_pending[slot] = 0;
    return hipSuccess;
}

int profile_mode(uint32_t flags)
{
    return (flags & TR_FLAG_PROFILE) ? 1 : ((flags & TR_FLAG_PROFILE_SC2) ? 2 : 0);
}

// Event set for the next profiled call (created on first use); mode 1: every
// stage, 2: the SC2 stage only.
hipEvent_t *ring_slot(tr_handle *h, int mode, uint32_t **mask)
{
    if (h->ring.empty()) {
        h->ring.assign((size_t)tr_handle::kRing * (TR_NUM_STAGES + 1), nullptr);
        h->ring_pending.assign(tr_handle::kRing, 0);
        h->ring_mask.assign(tr_handle::kRing, 0);
        for (auto &e : h->ring)
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
    }
    const int slot = (int)(h->ring_next % tr_handle::kRing);
    if (h->ring_pending[slot] && ring_collect(h, slot) != hipSuccess) return nullptr;
    h->ring_pending[slot] = (char)mode;
    h->ring_mask[slot] = 0;
    *mask = &h->ring_mask[slot];
    h->ring_next += 1;
    return &h->ring[(size_t)slot * (TR_NUM_STAGES + 1)];
}

}  // namespace

extern "C" {

const char *tr_status_string(int32_t s)
{
    switch (s) {
    case TR_OK: return "ok";
    case TR_ERR_INVALID_ARG: return "invalid argument";
    case TR_ERR_NONFINITE: return "non-finite input coordinates";
    case TR_ERR_NO_HYPOTHESIS: return "no valid TurboClique";
    case TR_ERR_WORKSPACE: return "request exceeds the handle's workspace";
    case TR_ERR_HIP: return "HIP error";
    case TR_WARN_SCORER_FALLBACK: return "learned scores not finite; plain pivots used";
    case TR_ERR_NO_SCORER: return "no learned scorer loaded";
    case TR_ERR_BAD_BLOB: return "bad scorer weights blob";
    default: return "unknown status";
    }
}

tr_status tr_create(tr_handle **out, int32_t max_n, int32_t max_batch, int32_t max_k1, int32_t max_k2,
                    int32_t device)
{
    if (!out) return TR_ERR_INVALID_ARG;
    *out = nullptr;
    if (max_n < 3 || max_n > 32767 || max_batch < 1 || max_k1 < 1 || max_k2 < 1 || max_k2 > TR_MAX_K2 ||
        max_k1 > TR_MAX_POOL)
        return TR_ERR_INVALID_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return TR_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return TR_ERR_HIP;
    tr_handle *h = new (std::nothrow) tr_handle();
    if (!h) return TR_ERR_HIP;
    h->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        h->num_cus = prop.multiProcessorCount;
        std::snprintf(h->arch, sizeof(h->arch), "%s", prop.gcnArchName);
        for (char *c = h->arch; *c; ++c)
            if (*c == ' ') *c = '_';
    }
    size_handle(h, max_n, max_batch, max_k1, max_k2);
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    workspace_layout(h, [&](auto *&p, size_t count) { A(alloc(h, &p, count)); });
    if (e == hipSuccess) A(hipMemset(h->prof_acc, 0, kProfSlots * sizeof(unsigned long long)));
    if (e == hipSuccess) A(mlp_create(&h->mlp));
    A(setup_graph_kernels());
    A(setup_pivot_kernels());
    A(setup_mlp_kernels());
    A(setup_hyp_kernels());
    if (e != hipSuccess) {
        std::fprintf(stderr, "turboreg: tr_create failed: %s\n", hipGetErrorString(e));
        release(h);
        delete h;
        return TR_ERR_HIP;
    }
    if (const char *cache = std::getenv("TURBOREG_TUNING_CACHE")) tr_tuning_load(h, cache);   // refused: ignored
    *out = h;
    return TR_OK;
}

tr_status tr_destroy(tr_handle *h)
{
    if (!h) return TR_ERR_INVALID_ARG;
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    release(h);
    delete h;
    return TR_OK;
}

tr_status tr_register(tr_handle *h, const float *src, const float *dst, int32_t n, const tr_params *p,
                      tr_result *out_dev, uint8_t *mask_dev, void *stream)
{
    if (!h || !src || !dst || !out_dev || n < 3) return TR_ERR_INVALID_ARG;
    if (n > h->max_n) return TR_ERR_WORKSPACE;
    tr_status st = check_params(h, p);
    if (st != TR_OK) return st;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    const bool learned = p->pivot_mode == TR_PIVOTS_LEARNED;
    const int pmode = profile_mode(p->flags);
    Work w = make_work(h, src, dst, *p, out_dev, mask_dev, learned, 1, n);
    w.n1 = n;   // the kernels derive this pair's plan from n (no planner launch)
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t *ev = nullptr;
    uint32_t *ev_mask = nullptr;
    if (pmode && !(ev = ring_slot(h, pmode, &ev_mask))) return TR_ERR_HIP;
    st = enqueue(h, w, nullptr, n, 1, n, ev, pmode, false, s, tuning_for(h, n, 1), ev_mask);
    if (st == TR_OK) remember(h, w, 1, s);
    return st;
}

// ---------------------------------------------------------------- entry point without allocation

// The workspace of tr_register_noalloc: one static array per device, carved by the same layout
// as a handle's allocations. Host code uses the address hipGetSymbolAddress returns on each
// device, never this name (which on the host is only a stand-in).
static __device__ __align__(256) uint8_t scratch[TR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kNoAllocDevices = 64;

struct NoAllocDevice {
    bool ready = false;
    tr_status status = TR_OK;   // of the set-up on this device
    tr_handle h;                // sizes and the carved workspace (no allocations of its own)
};

std::mutex g_noalloc_mutex;
NoAllocDevice g_noalloc[kNoAllocDevices];

// Once per device, with that device current: the array's address there, the workspace carved
// from it, and the kernel attributes tr_create would set.
tr_status noalloc_setup(int device, tr_handle &h)
{
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TR_ERR_HIP;
    h.device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        h.num_cus = cus;
    size_handle(&h, TR_NOALLOC_MAX_N, 1, TR_NOALLOC_MAX_K1, TR_MAX_K2);
    size_t off = 0;
    bool fits = true;
    workspace_layout(&h, [&](auto *&q, size_t count) {
        using T = std::remove_reference_t<decltype(*q)>;
        off = (off + 255) & ~(size_t)255;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (off + bytes > TR_NOALLOC_SCRATCH_BYTES) {
            fits = false;
            q = nullptr;
            return;
        }
        q = reinterpret_cast<T *>(static_cast<uint8_t *>(ptr) + off);
        off += bytes;
    });
    if (!fits) return TR_ERR_WORKSPACE;
    hipError_t e = setup_graph_kernels();
    if (e == hipSuccess) e = setup_pivot_kernels();
    if (e == hipSuccess) e = setup_hyp_kernels();
    return e == hipSuccess ? TR_OK : TR_ERR_HIP;
}

}  // namespace

tr_status tr_register_noalloc(const float *src, const float *dst, int32_t n, const tr_params *p,
                              tr_result *out_dev, uint8_t *mask_dev, void *stream)
{
    if (!src || !dst || !out_dev || !p || n < 3) return TR_ERR_INVALID_ARG;
    if (p->pivot_mode != TR_PIVOTS_PLAIN || (p->flags & (TR_FLAG_PROFILE | TR_FLAG_PROFILE_SC2)))
        return TR_ERR_INVALID_ARG;
    if (n > TR_NOALLOC_MAX_N || p->k1 > TR_NOALLOC_MAX_K1) return TR_ERR_WORKSPACE;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kNoAllocDevices) return TR_ERR_HIP;
    NoAllocDevice &d = g_noalloc[device];
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mutex);
        if (!d.ready) {
            d.status = noalloc_setup(device, d.h);
            d.ready = true;
        }
    }
    if (d.status != TR_OK) return d.status;
    tr_status st = check_params(&d.h, p);
    if (st != TR_OK) return st;
    Work w = make_work(&d.h, src, dst, *p, out_dev, mask_dev, false, 1, n);
    w.n1 = n;
    return enqueue(&d.h, w, nullptr, n, 1, n, nullptr, 0, false, static_cast<hipStream_t>(stream),
                   tuning_for(&d.h, n, 1));
}

tr_status tr_register_batch(tr_handle *h, const float *src, const float *dst, const int32_t *offsets_dev, int32_t B,
                            int32_t max_n, const tr_params *p, tr_result *out_dev, uint8_t *masks_dev, void *stream)
{
    if (!h || !src || !dst || !offsets_dev || !out_dev || B < 1 || max_n < 3) return TR_ERR_INVALID_ARG;
    if (B > h->max_batch || max_n > h->max_n) return TR_ERR_WORKSPACE;
    tr_status st = check_params(h, p);
    if (st != TR_OK) return st;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    const bool learned = p->pivot_mode == TR_PIVOTS_LEARNED;
    const int pmode = profile_mode(p->flags);
    Work w = make_work(h, src, dst, *p, out_dev, masks_dev, learned, B, max_n);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const tr_tuning cfg = tuning_for(h, max_n, B);
    if (pmode || s == nullptr) {
        // events (and the legacy default stream) stay out of captured graphs: run eagerly
        hipEvent_t *ev = nullptr;
        uint32_t *ev_mask = nullptr;
        if (pmode && !(ev = ring_slot(h, pmode, &ev_mask))) return TR_ERR_HIP;
        st = enqueue(h, w, offsets_dev, 0, B, max_n, ev, pmode, false, s, cfg, ev_mask);
        if (st == TR_OK) remember(h, w, B, s);
        return st;
    }
    GraphKey key;
    std::memset(&key, 0, sizeof(key));
    key.src = src;
    key.dst = dst;
    key.offsets = offsets_dev;
    key.out = out_dev;
    key.masks = masks_dev;
    key.stream = stream;
    key.B = B;
    key.max_n = max_n;
    key.p = *p;
    key.cfg = cfg;
    auto it = h->graphs.find(key);
    if (it == h->graphs.end()) {
        if (h->graphs.size() >= tr_handle::kMaxGraphs) {
            // a launch of the evicted graph may still run (on any stream): wait for the device
            // before destroying it; only callers that cycle through more buffer sets pay this
            auto lru = h->graphs.begin();
            for (auto jt = h->graphs.begin(); jt != h->graphs.end(); ++jt)
                if (jt->second.last_use < lru->second.last_use) lru = jt;
            if (hipDeviceSynchronize() != hipSuccess) return TR_ERR_HIP;
            hipGraphExecDestroy(lru->second.ge);
            hipGraphDestroy(lru->second.g);
            h->graphs.erase(lru);
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return TR_ERR_HIP;
        st = enqueue(h, w, offsets_dev, 0, B, max_n, nullptr, 0, false, s, cfg);
        hipError_t ec = hipStreamEndCapture(s, &g);
        if (st != TR_OK || ec != hipSuccess) {
            if (g) hipGraphDestroy(g);
            return st != TR_OK ? st : TR_ERR_HIP;
        }
        if (hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(g);
            return TR_ERR_HIP;
        }
        it = h->graphs.emplace(key, tr_handle::Captured{g, ge, 0}).first;
    }
    it->second.last_use = ++h->graph_clock;
    if (hipGraphLaunch(it->second.ge, s) != hipSuccess) return TR_ERR_HIP;
    remember(h, w, B, s);
    return TR_OK;
}

tr_status tr_fit_triplets(tr_handle *h, const float *src, const float *dst, int32_t n, const int32_t *triplets_dev,
                          int32_t T, float *poses_dev, int32_t *ok_dev, void *stream)
{
    if (!h || !src || !dst || !triplets_dev || !poses_dev || !ok_dev || n < 3 || T < 0) return TR_ERR_INVALID_ARG;
    if (T == 0) return TR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    const hipError_t e = launch_fit_triplets(src, dst, n, triplets_dev, T, poses_dev, ok_dev, h->num_cus * 4,
                                             static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TR_OK : TR_ERR_HIP;
}

tr_status tr_score_poses(tr_handle *h, const float *src, const float *dst, int32_t n, const float *poses_dev,
                         int32_t P, float theta, int32_t metric, int32_t *in_dev, float *score_dev, void *stream)
{
    if (!h || !src || !dst || !poses_dev || !in_dev || n < 1 || P < 0) return TR_ERR_INVALID_ARG;
    if (!(theta >= 0.0f) || !std::isfinite(theta) || metric < 0 || metric > 2 || (metric && !score_dev))
        return TR_ERR_INVALID_ARG;
    if (metric && !(theta > 0.0f)) return TR_ERR_INVALID_ARG;   // the error-based scores divide by theta
    if (P == 0) return TR_OK;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    const hipError_t e = launch_score_poses(src, dst, n, poses_dev, P, theta, metric, in_dev, score_dev,
                                            h->num_cus * 4, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? TR_OK : TR_ERR_HIP;
}

tr_status tr_tuning_get(tr_handle *h, int32_t max_n, int32_t B, tr_tuning *out)
{
    if (!h || !out || max_n < 3 || B < 1) return TR_ERR_INVALID_ARG;
    *out = tuning_for(h, max_n, B);
    return TR_OK;
}

tr_status tr_tuning_set(tr_handle *h, int32_t max_n, int32_t B, const tr_tuning *t)
{
    if (!h || !t || max_n < 3 || B < 1 || !tuning_valid(*t)) return TR_ERR_INVALID_ARG;
    h->tuning[tuning_key(max_n, B)] = *t;
    return TR_OK;
}

namespace {
constexpr int kTuningFileVersion = 1;
}

tr_status tr_tuning_save(tr_handle *h, const char *path)
{
    if (!h || !path) return TR_ERR_INVALID_ARG;
    std::FILE *f = std::fopen(path, "w");
    if (!f) return TR_ERR_INVALID_ARG;
    bool ok = std::fprintf(f, "turboreg-tuning %d %s %d\n", kTuningFileVersion, h->arch, h->num_cus) > 0;
    for (const auto &g : h->tuning) {
        const tr_tuning &t = g.second;
        ok = ok && std::fprintf(f, "%d %d %d %d %d %d %d\n", g.first.first, g.first.second, t.sc2_super,
                                t.compat_per_cu, t.hyp_ppw, t.hyp_per_cu, t.sc2_sparse_cap) > 0;
    }
    ok = std::fclose(f) == 0 && ok;
    return ok ? TR_OK : TR_ERR_INVALID_ARG;
}

tr_status tr_tuning_load(tr_handle *h, const char *path)
{
    if (!h || !path) return TR_ERR_INVALID_ARG;
    std::FILE *f = std::fopen(path, "r");
    if (!f) return TR_ERR_INVALID_ARG;
    char arch[64] = {0};
    int version = 0, cus = 0;
    bool ok = std::fscanf(f, "turboreg-tuning %d %63s %d", &version, arch, &cus) == 3 &&
              version == kTuningFileVersion && std::strcmp(arch, h->arch) == 0 && cus == h->num_cus;
    std::map<std::pair<int32_t, int32_t>, tr_tuning> read;
    while (ok) {
        int tiles = 0, B = 0;
        tr_tuning t{};
        const int k = std::fscanf(f, "%d %d %d %d %d %d %d", &tiles, &B, &t.sc2_super, &t.compat_per_cu, &t.hyp_ppw,
                                  &t.hyp_per_cu, &t.sc2_sparse_cap);
        if (k == EOF) break;
        ok = k == 7 && tiles >= 1 && B >= 1 && tuning_valid(t);
        if (ok) read[{tiles, B}] = t;
    }
    std::fclose(f);
    if (!ok) return TR_ERR_INVALID_ARG;
    for (const auto &g : read) h->tuning[g.first] = g.second;
    return TR_OK;
}

tr_status tr_autotune(tr_handle *h, const float *src, const float *dst, const int32_t *offsets_dev, int32_t B,
                      int32_t max_n, const tr_params *p, tr_result *out_dev, uint8_t *masks_dev, void *stream,
                      tr_tuning *best, float *best_ms)
{
    if (!h || !src || !dst || !out_dev || B < 1 || max_n < 3) return TR_ERR_INVALID_ARG;
    if (!offsets_dev && B != 1) return TR_ERR_INVALID_ARG;
    if (B > h->max_batch || max_n > h->max_n) return TR_ERR_WORKSPACE;
    tr_status st = check_params(h, p);
    if (st != TR_OK) return st;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    const bool learned = p->pivot_mode == TR_PIVOTS_LEARNED;
    Work w = make_work(h, src, dst, *p, out_dev, masks_dev, learned, B, max_n);
    const int32_t n_single = offsets_dev ? 0 : max_n;
    if (!offsets_dev) w.n1 = max_n;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return TR_ERR_HIP;
    }
    constexpr int kRuns = 8, kBatches = 3;
    // milliseconds of one call under configuration c: after one untimed warm-up, the fastest of
    // three batches of eight back-to-back calls (the minimum is robust to interference)
    auto time_cfg = [&](const tr_tuning &c, float &ms) -> tr_status {
        tr_status q = enqueue(h, w, offsets_dev, n_single, B, max_n, nullptr, 0, false, s, c);
        if (q != TR_OK) return q;
        ms = 0.0f;
        for (int bt = 0; bt < kBatches; ++bt) {
            if (hipEventRecord(e0, s) != hipSuccess) return TR_ERR_HIP;
            for (int r = 0; r < kRuns; ++r) {
                q = enqueue(h, w, offsets_dev, n_single, B, max_n, nullptr, 0, false, s, c);
                if (q != TR_OK) return q;
            }
            float t = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return TR_ERR_HIP;
            if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) return TR_ERR_HIP;
            t /= kRuns;
            if (bt == 0 || t < ms) ms = t;
        }
        return TR_OK;
    };
    tr_tuning cur = tuning_for(h, max_n, B);
    float cur_ms = 0.0f;
    st = time_cfg(cur, cur_ms);
    static const int kPpw[] = {4, 8, 16}, kPerCu[] = {2, 4, 8}, kSuper[] = {3, 4, 5, 6, 8}, kCompat[] = {4, 8, 16},
                     kSparse[] = {0, 1024, 2048, 4096, TR_SC2_SPARSE_CAP_MAX};
    struct Field {
        int32_t tr_tuning::*f;
        const int *v;
        int n;
    };
    const Field fields[] = {{&tr_tuning::hyp_ppw, kPpw, 3},
                            {&tr_tuning::hyp_per_cu, kPerCu, 3},
                            {&tr_tuning::sc2_super, kSuper, 5},
                            {&tr_tuning::compat_per_cu, kCompat, 3},
                            {&tr_tuning::sc2_sparse_cap, kSparse, 5}};
    for (const Field &fd : fields) {
        const int32_t start = cur.*fd.f;
        for (int k = 0; k < fd.n && st == TR_OK; ++k) {
            if (fd.v[k] == start) continue;
            tr_tuning c = cur;
            c.*fd.f = fd.v[k];
            float ms = 0.0f, again = 0.0f;
            st = time_cfg(c, ms);
            // the incumbent is timed again beside each candidate (drift); a candidate must be at
            // least 2% faster
            if (st == TR_OK) st = time_cfg(cur, again);
            if (st == TR_OK) cur_ms = std::min(cur_ms, again);
            if (st == TR_OK && ms < 0.98f * cur_ms) {
                cur = c;
                cur_ms = ms;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != TR_OK) return st;
    h->tuning[tuning_key(max_n, B)] = cur;
    remember(h, w, B, s);
    if (best) *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return TR_OK;
}

tr_status tr_features_batch(tr_handle *h, const float *src, const float *dst, const int32_t *offsets_dev, int32_t B,
                            int32_t max_n, const tr_params *p, uint16_t *feat_dev, void *stream)
{
    if (!h || !src || !dst || !offsets_dev || !feat_dev || !p || B < 1 || max_n < 3) return TR_ERR_INVALID_ARG;
    if (B > h->max_batch || max_n > h->max_n) return TR_ERR_WORKSPACE;
    if (!(p->tau >= 0.0f) || !std::isfinite(p->tau)) return TR_ERR_INVALID_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    tr_params q = *p;
    q.k1 = 1;
    q.k2 = 1;
    q.pool_factor = 1;
    Work w = make_work(h, src, dst, q, h->scratch_out, nullptr, true, B, max_n);
    w.feat_all = 1;   // every match's features (training data)
    hipStream_t s = static_cast<hipStream_t>(stream);
    tr_status st = enqueue(h, w, offsets_dev, 0, B, max_n, nullptr, 0, true, s, tuning_for(h, max_n, B));
    if (st != TR_OK) return st;
    if (launch_features(w, feat_dev, grid_cap(h, (int64_t)B * ((max_n + kPrepRows - 1) / kPrepRows), 8), s) !=
        hipSuccess)
        return TR_ERR_HIP;
    remember(h, w, B, s);
    return TR_OK;
}

tr_status tr_debug_copy(tr_handle *h, int32_t tap, int32_t pair, void *host_dst, size_t bytes, size_t *needed)
{
    if (!h || !h->last_valid || pair < 0 || pair >= h->last_B) return TR_ERR_INVALID_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    if (hipStreamSynchronize(h->last_stream) != hipSuccess) return TR_ERR_HIP;
    const Work &w = h->last;
    PairDesc d;
    if (w.n1) d = pair_desc_of(w.n1, 0, 0, 0, w.pool);   // single-pair calls keep no device descriptor
    else if (hipMemcpy(&d, h->pairs + pair, sizeof(d), hipMemcpyDeviceToHost) != hipSuccess) return TR_ERR_HIP;
    const size_t n = d.n;
    size_t need = 0;
    const void *srcp = nullptr;
    size_t pitch = 0, width = 0, rows = 0;
    switch (tap) {
    case TR_TAP_C: {   // stored as E2M1 nibbles (0x2 = 1): unpacked to one byte per entry here
        need = n * n;
        if (needed) *needed = need;
        if (!host_dst) return TR_OK;
        if (bytes < need) return TR_ERR_INVALID_ARG;
        const size_t rb = (n + 1) / 2;
        std::vector<uint8_t> packed(rb * n);
        if (n && hipMemcpy2D(packed.data(), rb, h->C + d.cb_off, (size_t)c_pitch(d.npad), rb, n,
                             hipMemcpyDeviceToHost) != hipSuccess)
            return TR_ERR_HIP;
        uint8_t *o = static_cast<uint8_t *>(host_dst);
        for (size_t i = 0; i < n; ++i)
            for (size_t j = 0; j < n; ++j) {
                const int nib = (packed[i * rb + j / 2] >> (4 * (j & 1))) & 0xF;
                o[i * n + j] = nib == 0x2 ? 1 : (nib == 0 ? 0 : 0xFF);   // 0xFF: not a valid entry
            }
        return TR_OK;
    }
    case TR_TAP_G:
        need = n * n * 2; srcp = h->G + d.g_off; pitch = (size_t)d.npad * 2; width = n * 2; rows = n; break;
    case TR_TAP_PIVOTS:
        if (w.learned) { need = (size_t)w.k1 * 12; srcp = h->pivots + (size_t)pair * h->k1_cap * 3; }
        else { need = (size_t)w.k1 * 12; srcp = h->pivots_plain + (size_t)pair * h->pool_cap * 3; }
        break;
    case TR_TAP_PLAIN_PIVOTS:
        need = (size_t)w.pool * 12; srcp = h->pivots_plain + (size_t)pair * h->pool_cap * 3; break;
    case TR_TAP_CLIQUES:
        need = (size_t)w.H * 12; srcp = h->cliques + (size_t)pair * h->h_cap * 3; break;
    case TR_TAP_POSES:
        need = (size_t)w.H * 48; srcp = h->poses + (size_t)pair * h->h_cap * 12; break;
    case TR_TAP_IN:
        need = (size_t)w.H * 4; srcp = h->inl + (size_t)pair * h->h_cap; break;
    case TR_TAP_RANK_SCORES:
        need = (size_t)w.H * 4; srcp = h->gscore + (size_t)pair * h->h_cap; break;
    case TR_TAP_FEATURES:
        need = n * 19 * 2; srcp = h->feat + (size_t)pair * h->max_n * 19; break;
    case TR_TAP_SCORES:
        need = n * 4; srcp = h->scores + (size_t)pair * h->max_n; break;
    default: return TR_ERR_INVALID_ARG;
    }
    if (needed) *needed = need;
    if (!host_dst) return TR_OK;
    if (bytes < need) return TR_ERR_INVALID_ARG;
    hipError_t e;
    if (rows) e = hipMemcpy2D(host_dst, width, srcp, pitch, width, rows, hipMemcpyDeviceToHost);
    else e = hipMemcpy(host_dst, srcp, need, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return TR_ERR_HIP;
    if (tap == TR_TAP_G) {   // the device holds only i < j; the tap is the O2Graph, zero elsewhere
        uint16_t *g = static_cast<uint16_t *>(host_dst);
        for (size_t i = 0; i < n; ++i)
            for (size_t j = 0; j <= i; ++j) g[i * n + j] = 0;
    }
    return TR_OK;
}

tr_status tr_stage_times(tr_handle *h, float *ms, int32_t count)
{
    if (!h || !ms || count < 0 || count > TR_NUM_STAGES) return TR_ERR_INVALID_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    for (int slot = 0; slot < (int)h->ring_pending.size(); ++slot)
        if (h->ring_pending[slot] && ring_collect(h, slot) != hipSuccess) return TR_ERR_HIP;
    int64_t calls = 0;
    for (int k = 0; k < TR_NUM_STAGES; ++k) calls += h->stage_calls[k];
    if (calls == 0) return TR_ERR_INVALID_ARG;
    double avg[TR_NUM_STAGES];
    for (int k = 0; k < TR_NUM_STAGES; ++k)
        avg[k] = h->stage_calls[k] ? h->stage_sum[k] / (double)h->stage_calls[k] : 0.0;
    // the hypothesis kernel's interval, split by the shares of its workgroups' time in each phase
    // (in-kernel clock stamps summed over the profiled calls)
    unsigned long long acc[kProfSlots];
    if (hipMemcpy(acc, h->prof_acc, sizeof(acc), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemset(h->prof_acc, 0, sizeof(acc)) != hipSuccess)
        return TR_ERR_HIP;
    const double work = (double)acc[kProfSearch] + acc[kProfFit] + acc[kProfScore] + acc[kProfRecords] +
                        acc[kProfSelect];
    if (work > 0) {
        const double hyp = avg[TR_STAGE_CLIQUES];
        avg[TR_STAGE_CLIQUES] = hyp * acc[kProfSearch] / work;
        avg[TR_STAGE_KABSCH] = hyp * acc[kProfFit] / work;
        avg[TR_STAGE_SCORE] = hyp * (acc[kProfScore] + acc[kProfRecords]) / work;
        avg[TR_STAGE_SELECT] = hyp * acc[kProfSelect] / work;
    }
    for (int k = 0; k < count; ++k) ms[k] = (float)avg[k];
    for (int k = 0; k < TR_NUM_STAGES; ++k) {
        h->stage_sum[k] = 0;
        h->stage_calls[k] = 0;
    }
    return TR_OK;
}

// ---- learned scorer ----

tr_status tr_scorer_set(tr_handle *h, const float *params_host)
{
    if (!h || !params_host) return TR_ERR_INVALID_ARG;
    for (int k = 0; k < TR_MLP_NPARAM; ++k)
        if (!std::isfinite(params_host[k])) return TR_ERR_INVALID_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    if (mlp_set(&h->mlp, params_host) != hipSuccess) return TR_ERR_HIP;
    h->has_scorer = true;
    return TR_OK;
}

tr_status tr_scorer_get(tr_handle *h, float *params_host)
{
    if (!h || !params_host) return TR_ERR_INVALID_ARG;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    return mlp_get(&h->mlp, params_host) == hipSuccess ? TR_OK : TR_ERR_HIP;
}

static uint64_t fnv1a(const void *p, size_t n)
{
    const uint8_t *b = static_cast<const uint8_t *>(p);
    uint64_t x = 1469598103934665603ull;
    for (size_t k = 0; k < n; ++k) { x ^= b[k]; x *= 1099511628211ull; }
    return x;
}

static const char kMagic[8] = {'T', 'R', 'M', 'L', 'P', '0', '0', '1'};
static const size_t kBlobBytes = 8 + TR_MLP_NPARAM * 4 + 8;

tr_status tr_scorer_save(tr_handle *h, void *blob, size_t capacity, size_t *written)
{
    if (!h) return TR_ERR_INVALID_ARG;
    if (written) *written = kBlobBytes;
    if (!blob) return written ? TR_OK : TR_ERR_INVALID_ARG;   // size query
    if (capacity < kBlobBytes) return TR_ERR_INVALID_ARG;
    std::vector<float> w(TR_MLP_NPARAM);
    tr_status st = tr_scorer_get(h, w.data());
    if (st != TR_OK) return st;
    uint8_t *b = static_cast<uint8_t *>(blob);
    std::memcpy(b, kMagic, 8);
    std::memcpy(b + 8, w.data(), TR_MLP_NPARAM * 4);
    const uint64_t c = fnv1a(b + 8, TR_MLP_NPARAM * 4);
    std::memcpy(b + 8 + TR_MLP_NPARAM * 4, &c, 8);
    return TR_OK;
}

tr_status tr_scorer_load(tr_handle *h, const void *blob, size_t bytes)
{
    if (!h || !blob) return TR_ERR_INVALID_ARG;
    if (bytes != kBlobBytes) return TR_ERR_BAD_BLOB;
    const uint8_t *b = static_cast<const uint8_t *>(blob);
    if (std::memcmp(b, kMagic, 8) != 0) return TR_ERR_BAD_BLOB;
    uint64_t c;
    std::memcpy(&c, b + 8 + TR_MLP_NPARAM * 4, 8);
    if (c != fnv1a(b + 8, TR_MLP_NPARAM * 4)) return TR_ERR_BAD_BLOB;
    std::vector<float> w(TR_MLP_NPARAM);
    std::memcpy(w.data(), b + 8, TR_MLP_NPARAM * 4);
    tr_status st = tr_scorer_set(h, w.data());
    return st == TR_ERR_INVALID_ARG ? TR_ERR_BAD_BLOB : st;
}

tr_status tr_mlp_forward(tr_handle *h, const uint16_t *feat_dev, int64_t m, float *scores_dev, void *stream)
{
    if (!h || !feat_dev || !scores_dev || m < 0) return TR_ERR_INVALID_ARG;
    if (!h->has_scorer) return TR_ERR_NO_SCORER;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    return mlp_forward(&h->mlp, feat_dev, m, scores_dev, static_cast<hipStream_t>(stream)) == hipSuccess ? TR_OK
                                                                                                          : TR_ERR_HIP;
}

tr_status tr_mlp_grads(tr_handle *h, const uint16_t *feat_dev, const uint8_t *labels_dev, int64_t m,
                       float *grads_dev, float *loss_dev, void *stream)
{
    if (!h || !feat_dev || !labels_dev || !grads_dev || m < 1) return TR_ERR_INVALID_ARG;
    if (!h->has_scorer) return TR_ERR_NO_SCORER;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    return mlp_grads(&h->mlp, feat_dev, labels_dev, m, grads_dev, loss_dev, static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? TR_OK
               : TR_ERR_HIP;
}

tr_status tr_train_step(tr_handle *h, const uint16_t *feat_dev, const uint8_t *labels_dev, int64_t m, float lr,
                        float *loss_dev, void *stream)
{
    if (!h || !feat_dev || !labels_dev || m < 1 || !(lr >= 0.0f)) return TR_ERR_INVALID_ARG;
    if (!h->has_scorer) return TR_ERR_NO_SCORER;
    if (hipSetDevice(h->device) != hipSuccess) return TR_ERR_HIP;
    return mlp_train_step(&h->mlp, feat_dev, labels_dev, m, lr, loss_dev, static_cast<hipStream_t>(stream)) ==
                   hipSuccess
               ? TR_OK
               : TR_ERR_HIP;
}

}  // extern "C"
