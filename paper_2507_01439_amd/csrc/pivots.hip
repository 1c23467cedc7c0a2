// Pivot selection (Eq. 4) on gfx950.
//
// The pivots are the first K pairs i < j of the O2Graph ordered by
// (weight desc, i asc, j asc), K = min(K1, N(N-1)/2). Weights are integers
// below N, so the K-th largest weight alpha comes from an exact histogram.
// Every pair heavier than alpha is a pivot, and the first m pairs of weight
// alpha in row-major order fill the remaining slots.
//
//   (the SC2 epilogue leaves kHistGroups weight histograms per pair and the
//   per-row maximum of the upper triangle)
//   k_thresh   sums the histograms; finds alpha, the pairs heavier than it
//              (c_gt) and the ties to take (m); sums the compatibility
//              kernel's per-tile counts (boundary pairs, edges, non-finite)
//   k_rowscan  collects every pair of weight >= alpha when they fit the pool
//              (fast path), else the pairs heavier than alpha and, per row and
//              per row block, the count of pairs of weight alpha (ordered path)
//   k_sort     ranks the collected keys by (w desc, i asc, j asc) and keeps
//              the first K; on the ordered path it places the first m ties in
//              row-major order after the c_gt heavier pairs
// The key set is exact on both paths and every position is decided by a rank
// or a row-major tie index, so the pivot list does not depend on the order
// atomics were served in.
#include "common.h"

namespace tr {
namespace {

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_excl_scan(int v, int lane)
{
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x - v;
}

// Inclusive prefix sum over the 64 lanes: shifts by 1, 2, 4, 8 inside each
// 16-lane row, then the last lane of row 0 is added to row 1 and of row 2 to
// row 3, then lane 31 to rows 2 and 3 (DPP row_shr / row_bcast, no LDS).
__device__ __forceinline__ int wave_incl_scan(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return x;
}

template <typename T>
__device__ T block_exclusive_scan(T v, T *lds, T &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    T x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T acc = 0;
        for (int k = 0; k < nw; ++k) { T t = lds[k]; lds[k] = acc; acc += t; }
        lds[nw] = acc;
    }
    __syncthreads();
    T res = lds[wid] + x - v;
    total = lds[nw];
    __syncthreads();
    return res;
}

// Sort key: smaller key = earlier pivot.
__device__ __forceinline__ uint64_t pivot_key(uint32_t w, uint32_t i, uint32_t j)
{
    return ((uint64_t)(0xFFFFu - w) << 40) | ((uint64_t)i << 20) | (uint64_t)j;
}

// Eight consecutive weights G[i][8c .. 8c+7] (rows are 256-byte aligned).
__device__ __forceinline__ void load8(const uint16_t *row, int c, int (&v)[8])
{
    const uint4 q = *reinterpret_cast<const uint4 *>(row + 8 * c);
    const uint32_t u[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = (int)(u[k] & 0xFFFFu);
        v[2 * k + 1] = (int)(u[k] >> 16);
    }
}

// alpha = the K-th largest weight over all N(N-1)/2 pairs (zeros included).
__global__ void __launch_bounds__(1024) k_thresh(Work w)
{
    extern __shared__ int32_t hs[];
    __shared__ int32_t res[3], wtot[16];
    __shared__ int32_t tally[16][3];
    const int b = batch_pair(w, blockIdx.x);
    const PairDesc d = pair_desc(w, b);
    const int64_t K = d.kpiv;
    // this call's counters of the pair (collection regions, clique-search tickets) start at zero;
    // the later kernels of the call update them
    for (int k = threadIdx.x; k < w.tick_stride / kTickLine; k += 1024) w.tick[(int64_t)b * w.tick_stride + k * kTickLine] = 0;
    if (K <= 0) return;
    // boundary pairs, edges and non-finite input of the pair, summed over its compatibility tiles;
    // the first eight tiles per thread are loaded together with the histogram
    constexpr int kTiles = 8;
    const int t0 = stage_first(w, kCompat, b), t1 = t0 + stage_count(w, kCompat, b);
    int cc[3] = {0, 0, 0};
    int tv[kTiles][3];
    auto load_tiles = [&](int tb) {
#pragma unroll
        for (int u = 0; u < kTiles; ++u) {
            const int t = tb + 1024 * u;
#pragma unroll
            for (int f = 0; f < 3; ++f) tv[u][f] = t < t1 ? w.cnt_part[3 * (int64_t)t + f] : 0;
        }
    };
    load_tiles(t0 + (int)threadIdx.x);
    const int32_t *gh = w.ghist + (int64_t)b * kHistGroups * w.hist_stride;
    // eight consecutive bins per thread: two 16-byte loads from each copy, all issued before any is
    // summed (the pass is latency-bound: one round up to N = 8192); bins at or past n are never
    // written and are not summed (the copies are padded to a multiple of 8)
    for (int v0 = 8 * threadIdx.x; v0 < d.n; v0 += 8 * 1024) {
        int4 c[kHistGroups][2];
#pragma unroll
        for (int g = 0; g < kHistGroups; ++g) {
            c[g][0] = *reinterpret_cast<const int4 *>(gh + (int64_t)g * w.hist_stride + v0);
            c[g][1] = *reinterpret_cast<const int4 *>(gh + (int64_t)g * w.hist_stride + v0 + 4);
        }
        int32_t sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int g = 0; g < kHistGroups; ++g) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                sum[4 * h] += c[g][h].x;
                sum[4 * h + 1] += c[g][h].y;
                sum[4 * h + 2] += c[g][h].z;
                sum[4 * h + 3] += c[g][h].w;
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (v0 + u < d.n) hs[v0 + u] = sum[u];
    }
    for (int tb = t0 + (int)threadIdx.x;;) {
#pragma unroll
        for (int u = 0; u < kTiles; ++u)
#pragma unroll
            for (int f = 0; f < 3; ++f) cc[f] += tv[u][f];
        tb += 1024 * kTiles;
        if (tb >= t1) break;
        load_tiles(tb);
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cc[f] += __shfl_xor(cc[f], o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        tally[threadIdx.x >> 6][0] = cc[0];
        tally[threadIdx.x >> 6][1] = cc[1];
        tally[threadIdx.x >> 6][2] = cc[2];
    }
    __syncthreads();
    // bins w = 1 .. n-1 walked from the top: thread t sums the contiguous positions u0 .. u1-1
    // (u = n-1-w); an in-wave scan and the sixteen wave totals give each thread the count above
    // its range, and the thread whose range holds the K-th largest weight walks it (counts stay
    // below n(n-1)/2 < 2^31)
    const int nb = d.n - 1;
    const int cs = (nb + 1023) / 1024;
    const int u0 = min(nb, (int)threadIdx.x * cs), u1 = min(nb, u0 + cs);
    int local = 0;
    for (int u = u0; u < u1; ++u) local += hs[d.n - 1 - u];
    const int incl = wave_incl_scan(local);
    if ((threadIdx.x & 63) == 63) wtot[threadIdx.x >> 6] = incl;
    __syncthreads();
    int64_t tot = 0, before = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int t = wtot[v];
        before += v < (int)(threadIdx.x >> 6) ? t : 0;
        tot += t;
    }
    const int64_t excl = before + incl - local;
    if (threadIdx.x == 0 && K > tot) { res[0] = 0; res[1] = (int32_t)tot; res[2] = (int32_t)(K - tot); }
    if (K <= tot && excl < K && K <= excl + local) {
        int64_t cum = excl;
        for (int u = u0; u < u1; ++u) {
            const int wt = d.n - 1 - u;
            const int64_t c = hs[wt];
            if (cum + c >= K) { res[0] = wt; res[1] = (int32_t)cum; res[2] = (int32_t)(K - cum); break; }
            cum += c;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int alpha = res[0], c_gt = res[1];
        // pairs of weight alpha: the histogram bin, or every pair of weight 0
        const int64_t ties = alpha > 0 ? hs[alpha] : (int64_t)d.n * (d.n - 1) / 2 - tot;
        const bool fast = c_gt + ties <= w.pool_cap;
        w.state[b].alpha = alpha;
        w.state[b].c_gt = c_gt;
        w.state[b].m_eq = res[2];
        w.state[b].fast = fast ? 1 : 0;
        w.state[b].ncand = fast ? (int32_t)(c_gt + ties) : (int32_t)K;
        int tb = 0, te = 0, tn = 0;
        for (int v = 0; v < 16; ++v) {
            tb += tally[v][0];
            te += tally[v][1];
            tn |= tally[v][2];
        }
        w.state[b].n_boundary = tb;
        w.state[b].n_edges = te;
        w.state[b].nonfinite = tn != 0;
    }
}

// ---------------------------------------------------------------- row scan

constexpr int kCollectCap = 2048;   // keys a workgroup stages in LDS before its one global reservation

// One row (i, j > i) of the O2Graph per wave, all of its 16-byte chunks of
// weights loaded before any is used (the pass is latency-bound); rows whose
// maximum is below alpha are not read. Each chunk gives two 8-bit masks: the
// pairs (inside i < j < n) heavier than alpha and those equal to it.
//
// Collected keys: on the fast path (every pair of weight >= alpha fits the
// pool) the pairs of weight >= alpha, on the ordered path the pairs heavier
// than alpha (there are c_gt < K of them); either way they are appended to the
// workgroup's XCD region of the pool in no particular order and the rank sort
// fixes the order. A workgroup stages its keys in LDS, reserves its range with
// one atomic and copies them out; if its rows hold more than kCollectCap keys
// it reserves the count first and writes straight to the pool on a second
// read of those rows.
//
// Ordered path, besides: per row, the pairs of weight alpha and a mask of the
// 512-column segments holding any; per row block, their sum. The sort kernel
// locates the first m ties in row-major order from these.
__global__ void __launch_bounds__(256) k_rowscan(Work w)
{
    __shared__ uint64_t buf[kCollectCap];
    __shared__ int32_t nbuf, base;
    __shared__ int32_t part[4];
    __shared__ SlotCache slots;
    // batches of up to kInfoMax pairs: each slot's threshold, path and sizes in LDS as well, so an
    // item (four rows) starts with no device-memory round trip but its rows' maxima
    constexpr int kInfoMax = 256;
    struct SlotInfo {
        int32_t alpha, fast, kpiv, n, npad, pad;
        int64_t g_off;
    };
    __shared__ SlotInfo info[kInfoMax];
    const bool cached = slot_cache_fill(w, kRowBlk, slots);
    const bool with_info = cached && w.plan->B <= kInfoMax;
    __syncthreads();
    if (with_info)
        for (int k = threadIdx.x; k < w.plan->B; k += blockDim.x) {
            const int b = slots.order[k];
            const PairState st = w.state[b];
            const PairDesc d = w.pairs[b];
            info[k] = SlotInfo{st.alpha, st.fast, d.kpiv, d.n, d.npad, 0, d.g_off};
        }
    __syncthreads();
    const int total = stage_total(w, kRowBlk);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        int blk, b, alpha, fast;
        PairDesc d;
        if (with_info) {
            const int k = find_pair(slots.pre, w.plan->B, item);
            blk = item - slots.pre[k];
            b = slots.order[k];
            const SlotInfo &f = info[k];
            alpha = f.alpha;
            fast = f.fast;
            d.kpiv = f.kpiv;
            d.n = f.n;
            d.npad = f.npad;
            d.g_off = f.g_off;
        } else {
            b = stage_pair_cached(w, kRowBlk, slots, cached, item, blk);
            const PairState st = w.state[b];
            d = pair_desc(w, b);
            alpha = st.alpha;
            fast = st.fast;
        }
        if (d.kpiv <= 0) continue;   // same for the whole workgroup
        const bool ordered = !fast;
        const int c1 = (d.n + 7) >> 3;
        const int i = blk * kRowsPerItem + wv;
        const int rm = i < d.n ? w.rowmax[(int64_t)b * w.max_n + i] : 0;
        const bool live = i < d.n && !(alpha > 0 && rm < alpha);
        const uint16_t *row = w.G + d.g_off + (int64_t)i * d.npad;
        const int c_lo = (i + 1) >> 3;
        // the pool region and counter of this workgroup's XCD (workgroup g runs on XCD g mod 8)
        const int rgn = blockIdx.x & (kCollectRegions - 1);
        uint64_t *cand = w.cand + ((int64_t)b * kCollectRegions + rgn) * w.pool_cap;
        // direct = false: stage the keys into buf; true: write cand[base + ...]. ties / segs: the
        // lane's pairs of weight alpha and the segments holding any (ordered path)
        auto scan = [&](bool direct, int &ties, uint64_t &segs) {
            ties = 0;
            segs = 0;
            for (int c0 = c_lo; c0 < c1; c0 += 1024) {
                uint4 q[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int c = c0 + 64 * u + lane;
                    q[u] = c < c1 ? *reinterpret_cast<const uint4 *>(row + 8 * c) : make_uint4(0, 0, 0, 0);
                }
                const int steps = min(16, (c1 - c0 + 63) >> 6);   // the same on every lane
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    if (u >= steps) continue;   // uniform: the loop stays unrolled
                    const int c = c0 + 64 * u + lane;
                    // bit e: pair (i, 8c + e) lies in i < j < n and weighs more than / exactly alpha
                    const int lo = min(max(i + 1 - 8 * c, 0), 8), hi = min(max(d.n - 8 * c, 0), 8);
                    const uint32_t range = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
                    const uint32_t uw[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
                    uint32_t hge = 0, heq = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        hge |= ((uint32_t)((int)(uw[k] & 0xFFFFu) >= alpha) << (2 * k)) |
                               ((uint32_t)((int)(uw[k] >> 16) >= alpha) << (2 * k + 1));
                    hge &= range;
                    if (ordered) {   // the same on the whole workgroup
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            heq |= ((uint32_t)((int)(uw[k] & 0xFFFFu) == alpha) << (2 * k)) |
                                   ((uint32_t)((int)(uw[k] >> 16) == alpha) << (2 * k + 1));
                        heq &= range;
                        if (!direct) {
                            ties += __builtin_popcount(heq);
                            if (__any(heq != 0)) segs |= 1ull << ((c0 - c_lo) / 64 + u);   // at most 64 segments (N < 32768)
                        }
                    }
                    const uint32_t hits = hge & ~heq;   // fast path: heq is 0
                    if (!__any(hits != 0)) continue;   // most chunks hold no key
                    const int m = __builtin_popcount(hits);
                    const int incl = wave_incl_scan(m);
                    const int tot = __builtin_amdgcn_readlane(incl, 63);
                    int off = 0;
                    if (lane == 63) off = atomicAdd(&nbuf, tot);
                    off = __builtin_amdgcn_readlane(off, 63) + incl - m;
                    if (hits) {
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            if ((hits >> e) & 1u) {
                                const uint32_t v = (uw[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
                                const uint64_t key = pivot_key(v, i, 8 * c + e);
                                if (direct) {
                                    if (base + off < w.pool_cap) cand[base + off] = key;
                                } else if (off < kCollectCap) {
                                    buf[off] = key;
                                }
                                ++off;
                            }
                        }
                    }
                }
            }
        };
        int ties = 0, unused = 0;
        uint64_t segs = 0, unused_segs = 0;
        if (tid == 0) nbuf = 0;
        __syncthreads();
        if (live) scan(false, ties, segs);
        __syncthreads();
        const int n_wg = nbuf;
        __syncthreads();   // every thread has read nbuf before it is reset
        if (n_wg > 0) {
            if (tid == 0) base = atomicAdd(&w.tick[(int64_t)b * w.tick_stride + rgn * kTickLine], n_wg);
            __syncthreads();
            if (n_wg <= kCollectCap) {
                for (int k = tid; k < n_wg; k += 256)
                    if (base + k < w.pool_cap) cand[base + k] = buf[k];
            } else {
                if (tid == 0) nbuf = 0;
                __syncthreads();
                if (live) scan(true, unused, unused_segs);
            }
        }
        if (ordered) {
            ties = __builtin_amdgcn_readlane(wave_incl_scan(ties), 63);
            if (lane == 0) {
                if (i < d.n) {
                    w.rowcnt[(int64_t)b * w.max_n + i] = ties;
                    w.rowseg[(int64_t)b * w.max_n + i] = segs;
                }
                part[wv] = ties;
            }
            __syncthreads();
            if (tid == 0) w.blkcnt[(int64_t)b * w.nblk_stride + blk] = part[0] + part[1] + part[2] + part[3];
        }
        __syncthreads();   // buf, nbuf, base and part are the next item's
    }
}

// ---------------------------------------------------------------- ordering

// Order the K pivots of one pair by (w desc, i asc, j asc) and write (i, j, w).
// Keys are distinct, so a key's rank is the number of smaller keys. Each
// workgroup of kSortWaves waves copies the pair's collected keys into its LDS
// and ranks 64 of them: wave v counts the smaller keys in its slice of the
// list with eight 16-byte broadcast reads in flight, and the partial counts
// are summed. The work of one pair is spread over ceil(K/64) CUs.
//
// Ordered path: the collected keys are the c_gt pairs heavier than alpha and
// fill slots 0 .. c_gt-1; slot c_gt + t holds the t-th pair of weight alpha in
// row-major order. A workgroup whose 64 slots reach past c_gt finds its ties
// from the row scan's counts: an exclusive scan of the per-block tie counts
// names the (at most 64) blocks that hold them, and one wave per block walks
// its rows' segments, counting ties in order, and writes those in its range.
constexpr int kSortWaves = 16;
constexpr int kSortThreads = 64 * kSortWaves;

__global__ void __launch_bounds__(kSortThreads) k_sort(Work w, int blocks_per_pair)
{
    extern __shared__ uint64_t keys[];
    __shared__ int32_t part[kSortWaves][64];
    __shared__ int64_t lds[17];
    __shared__ int32_t nrel, rel_blk[64], rel_pre[64];
    const int slot = blockIdx.x / blocks_per_pair, b = batch_pair(w, slot), g = blockIdx.x - slot * blocks_per_pair;
    const PairDesc d = pair_desc(w, b);
    const int K = d.kpiv, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // the collection counters are read together with the state (they are zeroed for every pair)
    int c[kCollectRegions];
#pragma unroll
    for (int r = 0; r < kCollectRegions; ++r) c[r] = w.tick[(int64_t)b * w.tick_stride + r * kTickLine];
    const PairState st = w.state[b];
    // the keys sit in the kCollectRegions regions of the pool, as many in each as its counter says
    int rb[kCollectRegions + 1];
    rb[0] = 0;
#pragma unroll
    for (int r = 0; r < kCollectRegions; ++r) rb[r + 1] = rb[r] + min(max(c[r], 0), w.pool_cap);
    // keys ranked (the first K are kept): fast path c_gt + all ties, ordered path c_gt
    const int want = K > 0 ? (st.fast ? st.ncand : st.c_gt) : 0;
    const int NC = min(min(want, rb[kCollectRegions]), w.pool_cap);
    int32_t *out = w.pivots_plain + (int64_t)b * w.pool_cap * 3;
    if (g * 64 >= max(NC, w.pool)) return;
    const uint64_t *cand = w.cand + (int64_t)b * kCollectRegions * w.pool_cap;
    const int K16 = (NC + 15) & ~15;   // padded with keys larger than any real one
    for (int k0 = tid; k0 < K16; k0 += kSortThreads * 8) {   // eight keys per thread loaded before any is stored
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + kSortThreads * u;
            int r = 0, o = 0;   // the region holding key k and its first key (rb is non-decreasing)
#pragma unroll
            for (int q = 1; q < kCollectRegions; ++q)
                if (k >= rb[q]) { r = q; o = rb[q]; }
            v[u] = k < NC ? cand[(int64_t)r * w.pool_cap + (k - o)] : ~0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (k0 + kSortThreads * u < K16) keys[k0 + kSortThreads * u] = v[u];
    }
    __syncthreads();
    const int p = g * 64 + lane;
    const uint64_t mine = p < NC ? keys[p] : 0;
    if (g * 64 < NC) {   // the same on the whole workgroup
        const int per = ((K16 / 16 + kSortWaves - 1) / kSortWaves) * 16;   // a slice of whole 16-key groups
        const int q0 = min(K16, wv * per), q1 = min(K16, q0 + per);
        int r = 0;
        for (int q = q0; q < q1; q += 16) {
            uint4 a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = *reinterpret_cast<const uint4 *>(&keys[q + 2 * u]);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                r += (((uint64_t)a[u].y << 32) | a[u].x) < mine;
                r += (((uint64_t)a[u].w << 32) | a[u].z) < mine;
            }
        }
        part[wv][lane] = r;
        __syncthreads();
        if (wv == 0) {
            int rk = 0;
#pragma unroll
            for (int v = 0; v < kSortWaves; ++v) rk += part[v][lane];
            if (p < NC && rk < K) {
                out[3 * rk] = (int32_t)((mine >> 20) & 0xFFFFF);
                out[3 * rk + 1] = (int32_t)(mine & 0xFFFFF);
                out[3 * rk + 2] = (int32_t)(0xFFFFu - (uint32_t)(mine >> 40));
            }
        }
    }
    if (wv == 0 && p >= K && p < w.pool) {   // slots past the pair's pivots
        out[3 * p] = -1;
        out[3 * p + 1] = -1;
        out[3 * p + 2] = 0;
    }
    if (K <= 0 || st.fast) return;
    // ordered path: ties t0 .. t1-1 of this workgroup's slots
    const int cgt = st.c_gt, alpha = st.alpha;
    const int t0 = max(g * 64, cgt) - cgt, t1 = min(g * 64 + 64, K) - cgt;
    if (t1 <= t0) return;
    const int nblk = (d.n + kRowsPerItem - 1) / kRowsPerItem;
    const int32_t *bc = w.blkcnt + (int64_t)b * w.nblk_stride;
    int bcnt[8];
    int64_t local = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {   // blocks 8t .. 8t+7 per thread (nblk <= 8192)
        const int k = 8 * tid + u;
        bcnt[u] = k < nblk ? bc[k] : 0;
        local += bcnt[u];
    }
    if (tid == 0) nrel = 0;
    int64_t total;
    int64_t run = block_exclusive_scan<int64_t>(local, lds, total);   // its barriers order nrel's reset
#pragma unroll
    for (int u = 0; u < 8; ++u) {
        if (bcnt[u] > 0 && run < t1 && run + bcnt[u] > t0) {   // the block holds a tie of the range
            const int slot = atomicAdd(&nrel, 1);
            if (slot < 64) {
                rel_blk[slot] = 8 * tid + u;
                rel_pre[slot] = (int32_t)run;
            }
        }
        run += bcnt[u];
    }
    __syncthreads();
    const int nr = min(nrel, 64);
    const uint16_t *G = w.G + d.g_off;
    const int c1 = (d.n + 7) >> 3;
    for (int x = wv; x < nr; x += kSortWaves) {
        int pre = rel_pre[x];
        const int blk = rel_blk[x];
        for (int rr = 0; rr < kRowsPerItem; ++rr) {
            const int i = blk * kRowsPerItem + rr;
            if (i >= d.n || pre >= t1) break;
            const int ne = w.rowcnt[(int64_t)b * w.max_n + i];
            if (ne > 0 && pre + ne > t0) {
                // the row's ties in order, eight segments (512 columns each) loaded at a time
                const uint16_t *row = G + (int64_t)i * d.npad;
                const int c_lo = (i + 1) >> 3;
                uint64_t todo = w.rowseg[(int64_t)b * w.max_n + i];
                int idx0 = pre;   // tie index of the row's next tie
                while (todo && idx0 < t1) {
                    uint4 q[8];
                    int cs[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        int cc = -1;
                        if (todo) {
                            cc = c_lo + 64 * __builtin_ctzll(todo) + lane;
                            todo &= todo - 1;
                        }
                        cs[u] = cc;
                        q[u] = (cc >= 0 && cc < c1) ? *reinterpret_cast<const uint4 *>(row + 8 * cc)
                                                    : make_uint4(0, 0, 0, 0);
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int cc = cs[u];
                        if (__builtin_amdgcn_readfirstlane(cc) < 0) break;   // no segment left (the same on every lane)
                        const int lo = min(max(i + 1 - 8 * cc, 0), 8), hi = min(max(d.n - 8 * cc, 0), 8);
                        const uint32_t uw[4] = {q[u].x, q[u].y, q[u].z, q[u].w};
                        uint32_t heq = 0;
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            heq |= ((uint32_t)((int)(uw[k] & 0xFFFFu) == alpha) << (2 * k)) |
                                   ((uint32_t)((int)(uw[k] >> 16) == alpha) << (2 * k + 1));
                        heq &= ((1u << hi) - 1u) & ~((1u << lo) - 1u);
                        const int m = __builtin_popcount(heq);
                        const int incl = wave_incl_scan(m);
                        int idx = idx0 + incl - m;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            if ((heq >> e) & 1u) {
                                if (idx >= t0 && idx < t1) {
                                    const int slot = cgt + idx;   // < K <= pool_cap
                                    out[3 * slot] = i;
                                    out[3 * slot + 1] = 8 * cc + e;
                                    out[3 * slot + 2] = alpha;
                                }
                                ++idx;
                            }
                        }
                        idx0 += __builtin_amdgcn_readlane(incl, 63);
                    }
                }
            }
            pre += ne;
        }
    }
}

}  // namespace

// grid_rows: workgroups of the row scan
hipError_t launch_pivots(const Work &w, int B, int grid_rows, hipStream_t s)
{
    hipLaunchKernelGGL(k_thresh, dim3(B), dim3(1024), (size_t)w.max_n * sizeof(int32_t), s, w);
    hipLaunchKernelGGL(k_rowscan, dim3(grid_rows), dim3(256), 0, s, w);
    const int bpp = (w.pool_cap + 63) / 64;   // the fast path may rank up to pool_cap keys
    hipLaunchKernelGGL(k_sort, dim3(B * bpp), dim3(kSortThreads), (size_t)((w.pool_cap + 15) & ~15) * sizeof(uint64_t),
                       s, w, bpp);
    return hipGetLastError();
}

hipError_t setup_pivot_kernels()
{
    // up to TR_MAX_POOL keys (128 KiB) / 32767 histogram bins in LDS
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_sort),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, TR_MAX_POOL * (int)sizeof(uint64_t));
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_thresh), hipFuncAttributeMaxDynamicSharedMemorySize,
                                32768 * (int)sizeof(int32_t));
    return e;
}

}  // namespace tr
