// Graph construction on gfx950: work planning, the pairwise-length
// compatibility matrix (Eq. 1) and the SC2 weights of the O2Graph
// (Eq. 2 restricted to i < j, Definition 2) on FP4 MFMA with exact float32 accumulation.
#include "common.h"

namespace tr {
namespace {

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Upper-triangular tile index t (row-major over bi <= bj < nb) -> (bi, bj).
__device__ __forceinline__ void tri_decode(int t, int nb, int &bi, int &bj)
{
    // start(r) = r*(2nb - r + 1)/2 tiles precede row r
    float a = (float)(2 * nb + 1);
    int r = (int)((a - sqrtf(a * a - 8.0f * (float)t)) * 0.5f);
    r = r < 0 ? 0 : (r >= nb ? nb - 1 : r);
    while (r > 0 && r * (2 * nb - r + 1) / 2 > t) --r;
    while (r + 1 < nb && (r + 1) * (2 * nb - r) / 2 <= t) ++r;
    bi = r;
    bj = r + (t - r * (2 * nb - r + 1) / 2);
}

// SC2 tile order: the upper triangle of nb x nb tiles is walked in super-tiles
// of sup x sup (super-rows I <= J, row-major), tiles row-major inside.
// Consecutive items then share few row blocks of C, so the tiles one XCD runs
// at the same time reuse each other's operand rows in its L2. sup >= 1 is a
// launch parameter (the autotuner's); the order does not change any result.
__device__ __forceinline__ void super_decode(int t, int nb, int sup, int &bi, int &bj)
{
    const int ns = (nb + sup - 1) / sup;
    for (int I = 0; I < ns; ++I) {
        const int r0 = I * sup, r1 = min(nb, r0 + sup);
        for (int J = I; J < ns; ++J) {
            const int c0 = J * sup, c1 = min(nb, c0 + sup);
            int cnt;
            if (I == J) { const int s = r1 - r0; cnt = s * (s + 1) / 2; }
            else cnt = (r1 - r0) * (c1 - c0);
            if (t < cnt) {
                if (I == J) {
                    // triangle of side s: row r holds s - r tiles
                    int r = 0, s = r1 - r0;
                    while (t >= s - r) { t -= s - r; ++r; }
                    bi = r0 + r;
                    bj = bi + t;
                } else {
                    bi = r0 + t / (c1 - c0);
                    bj = c0 + t % (c1 - c0);
                }
                return;
            }
            t -= cnt;
        }
    }
    bi = bj = 0;   // not reached for t < nb (nb + 1) / 2
}

// ---------------------------------------------------------------- planning

// Exclusive scan of NV values per thread across the workgroup (one pass).
template <int NV>
__device__ void block_scan_multi(const int64_t (&v)[NV], int64_t (&excl)[NV], int64_t (&total)[NV],
                                 int64_t (*lds)[NV])
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t x[NV];
#pragma unroll
    for (int s = 0; s < NV; ++s) {
        x[s] = v[s];
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x[s], o, 64);
            if (lane >= o) x[s] += y;
        }
        if (lane == 63) lds[wid][s] = x[s];
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        int64_t acc = 0;
        for (int k = 0; k < nw; ++k) { const int64_t t = lds[k][threadIdx.x]; lds[k][threadIdx.x] = acc; acc += t; }
        lds[nw][threadIdx.x] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NV; ++s) {
        excl[s] = lds[wid][s] + x[s] - v[s];
        total[s] = lds[nw][s];
    }
    __syncthreads();
}

constexpr int kCostKeys = 32767 / kSc2Tile + 2;   // npad / kSc2Tile of a valid pair (max_n <= 32767), 0 if invalid
constexpr int kOrderMinB = 16;   // smaller batches keep their pairs in index order

// Slot of the pair at position p of the size order (largest first) among B pairs: the order is
// dealt to the eight XCDs in a snake (positions 0-7 to XCDs 0-7, 8-15 to XCDs 7-0, ...), and the
// slots hold XCD 0's pairs, then XCD 1's, ..., each XCD's pairs in size order. Cut into eight
// ranges of equal cost, the SC2 list then gives each XCD a like mix of sizes, costly items first.
__device__ __forceinline__ int xcd_pairs(int x, int B)
{
    const int R = B >> 3, rem = B & 7;
    return R + (rem && ((R & 1) ? x >= 8 - rem : x < rem));
}

__device__ __forceinline__ int xcd_first_slot(int x, int B)
{
    int first = 0;
    for (int y = 0; y < x; ++y) first += xcd_pairs(y, B);
    return first;
}

__device__ __forceinline__ int snake_slot(int p, int B)
{
    const int r = p >> 3, c = p & 7;
    return xcd_first_slot((r & 1) ? 7 - c : c, B) + r;
}

// One workgroup: per-pair sizes, arena offsets (pair order) and zeroed per-pair state; the
// order of the pairs (from 16 pairs on: by decreasing npad, pairs of one size in index order,
// dealt to the XCDs; else index order);
// the work-item counts of every stage and their prefix sums over that order; the XCD ranges of
// the SC2 list, equal in modelled cost.
__global__ void __launch_bounds__(1024) k_plan(const int32_t *offsets, int32_t n_single, int32_t B,
                                               int32_t max_n, int32_t pool, int32_t H,
                                               PairDesc *pairs, PairState *state, Plan *plan,
                                               int32_t *pre, int32_t pre_stride)
{
    constexpr int NV = kNumPrefix + 1;   // the work-list stages, then the SC2 cost
    __shared__ int64_t lds[17][NV];
    __shared__ int64_t lds1[17][3];
    __shared__ int32_t kfirst[kCostKeys];        // pairs per size key, then the key's next free position
    __shared__ int32_t wfirst[16][kCostKeys];    // per wave of a chunk: pairs per key, then first position
    __shared__ int32_t nl[1024], ol[1024];       // B <= 1024: n of each valid pair (0 if invalid); the order
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
    int32_t *order = pre + kOrderRow * pre_stride, *slot_of = pre + kSlotRow * pre_stride;
    auto size_of = [&](int b, int32_t &n, int32_t &pt) {   // n and first match of pair b; valid?
        n = pt = 0;
        if (b >= B) return false;
        if (offsets) { pt = offsets[b]; n = offsets[b + 1] - pt; }
        else n = n_single;
        return n >= 3 && n <= max_n;
    };
    const bool small = B <= 1024;
    auto valid_n = [&](int b) {   // n of pair b if it is valid, else 0 (passes 2 and 3)
        if (b >= B) return 0;
        if (small) return nl[b];
        int32_t n, pt;
        return size_of(b, n, pt) ? n : 0;
    };
    // modelled cost of one SC2 item in K columns of its main loop: npad columns, plus the
    // epilogue (scan, histogram, stores), which takes about as long as 2048 columns
    auto sc2_unit = [](int32_t npad) { return (int64_t)npad + 2048; };
    for (int k = tid; k < kCostKeys; k += blockDim.x) kfirst[k] = 0;
    __syncthreads();
    // pass 1, pair order: descriptors, state, arena offsets, size-key counts, total SC2 cost
    int64_t acarry = 0, ccarry = 0, sc2_cost = 0;
    for (int base = 0; base < B; base += blockDim.x) {
        const int b = base + tid;
        int32_t n, pt;
        const bool ok = size_of(b, n, pt);
        const int32_t npad = ok ? (n + kSc2Tile - 1) / kSc2Tile * kSc2Tile : 0;
        int64_t v[3] = {(int64_t)npad * npad, ok ? stage_items(kSc2, n, H) * sc2_unit(npad) : 0,
                        ok ? npad * c_pitch(npad) : 0}, excl[3], tot[3];
        block_scan_multi<3>(v, excl, tot, lds1);
        if (b < B) {
            PairDesc d = pair_desc_of(n, pt, excl[0] + acarry, excl[2] + ccarry, pool);
            if (!ok) d.n = d.npad = d.kpiv = 0;
            pairs[b] = d;
            PairState st = {};
            st.status = ok ? TR_OK : TR_ERR_INVALID_ARG;
            state[b] = st;
            atomicAdd(&kfirst[npad / kSc2Tile], 1);
            if (small) nl[b] = ok ? n : 0;
        }
        acarry += tot[0];
        sc2_cost += tot[1];
        ccarry += tot[2];
    }
    __syncthreads();
    if (B < kOrderMinB) {   // a few pairs: slots in pair order
        for (int b = tid; b < B; b += blockDim.x) {
            order[b] = slot_of[b] = b;
            if (small) ol[b] = b;
        }
    } else {
        {   // first position of each key, the largest key first
            int64_t v[3] = {tid < kCostKeys ? kfirst[kCostKeys - 1 - tid] : 0, 0, 0}, excl[3], tot[3];
            block_scan_multi<3>(v, excl, tot, lds1);
            if (tid < kCostKeys) kfirst[kCostKeys - 1 - tid] = (int32_t)excl[0];
            __syncthreads();
        }
        // pass 2, pair order: positions (pairs of one key in index order: rank in the wave by
        // ballots, then the waves of the chunk in order), and slots
        for (int base = 0; base < B; base += blockDim.x) {
            const int b = base + tid;
            const int key = (valid_n(b) + kSc2Tile - 1) / kSc2Tile;
            const int nwa = min(nw, (B - base + 63) >> 6);   // waves of the chunk that hold pairs
            for (int k = tid; k < nwa * kCostKeys; k += blockDim.x) (&wfirst[0][0])[k] = 0;
            __syncthreads();
            bool pending = b < B;
            int rank = 0;
            uint64_t todo = __ballot(pending);
            while (todo) {
                const int lk = __builtin_amdgcn_readlane(key, __builtin_ctzll(todo));
                const bool mine = pending && key == lk;
                const uint64_t m = __ballot(mine);
                if (mine) {
                    rank = __builtin_popcountll(m & ((1ull << lane) - 1));
                    pending = false;
                }
                if (lane == 0) wfirst[wid][lk] = __builtin_popcountll(m);
                todo &= ~m;
            }
            __syncthreads();
            for (int k = tid; k < kCostKeys; k += blockDim.x) {
                int32_t acc = kfirst[k];
                for (int v = 0; v < nwa; ++v) {
                    const int32_t c = wfirst[v][k];
                    wfirst[v][k] = acc;
                    acc += c;
                }
                kfirst[k] = acc;
            }
            __syncthreads();
            if (b < B) {
                const int slot = snake_slot(wfirst[wid][key] + rank, B);
                order[slot] = b;
                slot_of[b] = slot;
                if (small) ol[slot] = b;
            }
            __syncthreads();   // wfirst is cleared next chunk
        }
    }
    __syncthreads();   // order[] is read by other threads below
    // pass 3, slot order: stage prefixes; SC2 range boundaries at x / 8 of the cost
    if (tid == 0) {
        plan->B = B;
        plan->sc2_split[0] = 0;
        for (int x = 1; x < 8; ++x)
            if (sc2_cost * x / 8 == 0) plan->sc2_split[x] = 0;
    }
    int64_t carry[NV] = {};
    for (int base = 0; base < B; base += blockDim.x) {
        const int slot = base + tid;
        const int b = slot >= B ? B : small ? ol[slot] : order[slot];
        const int32_t n = valid_n(b);
        const bool ok = n > 0;
        int64_t cnt[NV], excl[NV], tot[NV];
        for (int s = 0; s < kNumPrefix; ++s) cnt[s] = ok ? stage_items(s, n, H) : 0;
        cnt[kScore] = ok ? cnt[kScore] : (b < B);   // an invalid pair's one (empty) scoring item writes its record
        const int32_t npad = ok ? (n + kSc2Tile - 1) / kSc2Tile * kSc2Tile : 0;
        cnt[kNumPrefix] = ok ? cnt[kSc2] * sc2_unit(npad) : 0;
        block_scan_multi<NV>(cnt, excl, tot, lds);
        if (slot < B) {
            for (int s = 0; s < kNumPrefix; ++s) pre[s * pre_stride + slot] = (int32_t)(excl[s] + carry[s]);
            // a target in (c0, c1] falls in this pair's items: the first item whose cost prefix reaches it
            const int64_t c0 = excl[kNumPrefix] + carry[kNumPrefix], c1 = c0 + cnt[kNumPrefix];
            for (int x = 1; x < 8; ++x) {
                const int64_t tgt = sc2_cost * x / 8;
                if (tgt > c0 && tgt <= c1) {
                    const int64_t u = sc2_unit(npad);
                    plan->sc2_split[x] = (int32_t)(excl[kSc2] + carry[kSc2] + (tgt - c0 + u - 1) / u);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NV; ++s) carry[s] += tot[s];
    }
    if (tid == 0) {
        for (int s = 0; s < kNumPrefix; ++s) {
            pre[s * pre_stride + B] = (int32_t)carry[s];
            plan->total[s] = (int32_t)carry[s];
        }
        plan->sc2_split[8] = (int32_t)carry[kSc2];
    }
}

// Learned mode: zero the per-row feature accumulators.
__global__ void __launch_bounds__(256) k_prep_learned(Work w)
{
    const int total = stage_total(w, kPrep);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        int local;
        const int b = stage_pair(w, kPrep, item, local);
        const int i = local * kPrepRows + threadIdx.x;
        if (i < pair_desc(w, b).n) {
            int32_t *rs = w.rowstat + ((int64_t)b * w.max_n + i) * 20;
            for (int f = 0; f < 20; ++f) rs[f] = 0;
        }
    }
}

// ---------------------------------------------------------------- Eq. 1


constexpr int kNibStride = 32;    // LDS row stride of a packed 64-column tile (two entries per byte)

// Four 0/1 bytes -> four E2M1 nibbles (1.0 = 0x2, 0.0 = 0x0), byte k -> bits 4k..4k+3.
__device__ __forceinline__ uint32_t pack_e2m1(uint32_t x)
{
    return ((x << 1) & 0x2u) | ((x >> 3) & 0x20u) | ((x >> 7) & 0x200u) | ((x >> 11) & 0x2000u);
}

// Eight E2M1 entries (0x2 = 1, 0x0 = 0) of a packed word -> eight bits, entry k -> bit k.
__device__ __forceinline__ uint32_t nibbles_to_bits(uint32_t x)
{
    x = (x >> 1) & 0x11111111u;          // entry k at bit 4k
    x = (x | (x >> 3)) & 0x03030303u;    // entries 2m, 2m+1 at bits 8m, 8m+1
    x = (x | (x >> 6)) & 0x000F000Fu;    // at bits 16m .. 16m+3
    return (x | (x >> 12)) & 0xFFu;
}

// Guard band of the fast compatibility test: v_sqrt_f32 is within a few ulps,
// so |delta_fast - delta_exact| <= 2^-21 (|x| + |y|); a pair whose fast delta
// lies within 2^-19 (|x| + |y|) + 2e-6 of tau is re-evaluated exactly, which
// also covers every pair the boundary report counts (|delta - tau| < 1e-6).
__device__ __forceinline__ bool near_tau(float la, float lb, float dl, float tau)
{
    return __builtin_fabsf(dl - tau) <= __builtin_fmaf(la + lb, 0x1p-19f, 2e-6f) || !(dl == dl);
}

// One 64 x 64 tile (bi <= bj) of C per work item. Each thread evaluates a
// 4 x 4 block of pairs once: the plain path with the hardware square root and
// a guard band around tau (any lane with a pair inside it redoes its 16 pairs
// with the correctly rounded square root, so decisions are identical to the
// exact evaluation); learned mode always evaluates exactly, because its delta
// histogram needs the exact value. The tile and its transpose are staged in
// LDS and written to both triangles with 16-byte stores. The next item's
// points are loaded while the current one is computed. Per-tile counts
// (boundary pairs, edges) go to a per-item slot, so no atomics are needed;
// non-finite inputs are counted by the diagonal tiles (third slot), which also clear the
// pair's weight histograms and row maxima for their rows.
template <bool LEARNED, bool BITS>
__global__ void __launch_bounds__(256, 2) k_compat(Work w)
{
    __shared__ float px[2][64][3], py[2][64][3];
    __shared__ __attribute__((aligned(16))) uint8_t tile[2][64 * kNibStride];
    __shared__ int32_t hrow[LEARNED ? 64 : 1][17], hcol[LEARNED ? 64 : 1][17];
    __shared__ int32_t red[4][3];
    __shared__ SlotCache slots;
    const bool cached = slot_cache_fill(w, kCompat, slots);
    __syncthreads();
    const int total = stage_total(w, kCompat);
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15, lane = tid & 63, wv = tid >> 6;
    const float tau = w.tau, q = tau * 0.25f;
    // prefetch registers: thread t < 128 holds point (t & 63) of side t >> 6
    float nx[3] = {0, 0, 0}, ny[3] = {0, 0, 0};
    auto fetch = [&](int item) {
        if (tid < 128 && item < total) {
            int local;
            const int b = stage_pair_cached(w, kCompat, slots, cached, item, local);
            const PairDesc d = pair_desc(w, b);
            int bi, bj;
            tri_decode(local, d.npad / kCompatTile, bi, bj);
            const int i = ((tid >> 6) ? bj : bi) * kCompatTile + (tid & 63);
            for (int k = 0; k < 3; ++k) {
                nx[k] = i < d.n ? w.src[3 * (int64_t)(d.pt_off + i) + k] : 0.0f;
                ny[k] = i < d.n ? w.dst[3 * (int64_t)(d.pt_off + i) + k] : 0.0f;
            }
        }
    };
    if (w.n1 && blockIdx.x == 0 && tid == 0) {   // a single-pair call has no planner: reset its state here
        PairState st = {};
        st.status = TR_OK;
        w.state[0] = st;
    }
    fetch(blockIdx.x);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        int local;
        const int b = stage_pair_cached(w, kCompat, slots, cached, item, local);
        const PairDesc d = pair_desc(w, b);
        int bi, bj;
        tri_decode(local, d.npad / kCompatTile, bi, bj);
        const bool diag = bi == bj;
        bool bad = false;
        if (tid < 128) {
            const int side = tid >> 6, r = tid & 63;
            for (int k = 0; k < 3; ++k) {
                px[side][r][k] = nx[k];
                py[side][r][k] = ny[k];
                bad |= diag && side == 0 && !(isfinite(nx[k]) && isfinite(ny[k]));
            }
        }
        if (diag) {   // the diagonal tiles clear this pair's histogram copies and row maxima for their 64 rows
            for (int k = tid; k < kHistGroups * 64; k += 256) {
                const int i = bi * kCompatTile + (k & 63);
                if (i < d.n) w.ghist[((int64_t)b * kHistGroups + (k >> 6)) * w.hist_stride + i] = 0;
            }
            if (tid < 64 && bi * kCompatTile + tid < d.n) {
                const int64_t ri = (int64_t)b * w.max_n + bi * kCompatTile + tid;
                w.rowmax[ri] = 0;
                if (!LEARNED && w.learned) {   // pool-feature mode: the SC2 row statistics and the row marks
                    w.rowstat[ri * 20 + 1] = 0;
                    w.rowstat[ri * 20 + 2] = 0;
                    w.mark[ri] = 0;
                }
            }
        }
        if (LEARNED) {
            for (int k = tid; k < 64 * 17; k += 256) { hrow[k / 17][k % 17] = 0; hcol[k / 17][k % 17] = 0; }
        }
        const bool any_bad = __any(bad);
        __syncthreads();
        fetch(item + gridDim.x);
        float dl[4][4];
        bool need_exact = LEARNED;
        if (!LEARNED) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int r = ty * 4 + a;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = tx * 4 + e;
                    float s1 = (px[0][r][0] - px[1][c][0]) * (px[0][r][0] - px[1][c][0]);
                    s1 = __builtin_fmaf(px[0][r][1] - px[1][c][1], px[0][r][1] - px[1][c][1], s1);
                    s1 = __builtin_fmaf(px[0][r][2] - px[1][c][2], px[0][r][2] - px[1][c][2], s1);
                    float s2 = (py[0][r][0] - py[1][c][0]) * (py[0][r][0] - py[1][c][0]);
                    s2 = __builtin_fmaf(py[0][r][1] - py[1][c][1], py[0][r][1] - py[1][c][1], s2);
                    s2 = __builtin_fmaf(py[0][r][2] - py[1][c][2], py[0][r][2] - py[1][c][2], s2);
                    const float la = __builtin_amdgcn_sqrtf(s1), lb = __builtin_amdgcn_sqrtf(s2);
                    dl[a][e] = __builtin_fabsf(la - lb);
                    need_exact |= near_tau(la, lb, dl[a][e], tau);
                }
            }
        }
        if (__any(need_exact)) {
            if (need_exact) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int r = ty * 4 + a;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = tx * 4 + e;
                        const float lx = length32(px[0][r][0] - px[1][c][0], px[0][r][1] - px[1][c][1],
                                                  px[0][r][2] - px[1][c][2]);
                        const float ly = length32(py[0][r][0] - py[1][c][0], py[0][r][1] - py[1][c][1],
                                                  py[0][r][2] - py[1][c][2]);
                        dl[a][e] = __builtin_fabsf(lx - ly);
                    }
                }
            }
        }
        uint32_t rowbits[4] = {0, 0, 0, 0}, colbits[4] = {0, 0, 0, 0};
        int nbnd = 0, nedge = 0;
        // every pair of an interior tile (bi < bj, both blocks below n) is live with i < j: the
        // edges are the bits set, and a boundary pair (|delta - tau| < 1e-6) can only occur in a
        // lane that took the exact path (the guard band is wider)
        const bool interior = !LEARNED && bi < bj && (bj + 1) * kCompatTile <= d.n;
        if (interior) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t bit = dl[a][e] <= tau ? 1u : 0u;
                    rowbits[a] |= bit << (8 * e);
                    colbits[e] |= bit << (8 * a);
                }
            nedge = __builtin_popcount(rowbits[0]) + __builtin_popcount(rowbits[1]) + __builtin_popcount(rowbits[2]) +
                    __builtin_popcount(rowbits[3]);
            if (need_exact) {
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int e = 0; e < 4; ++e) nbnd += __builtin_fabsf(dl[a][e] - tau) < 1e-6f;
            }
        } else {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int r = ty * 4 + a, i = bi * kCompatTile + r;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = tx * 4 + e, j = bj * kCompatTile + c;
                    const bool live = i != j && i < d.n && j < d.n;
                    const uint32_t bit = (live && dl[a][e] <= tau) ? 1u : 0u;
                    rowbits[a] |= bit << (8 * e);
                    colbits[e] |= bit << (8 * a);
                    if (live && i < j) {
                        nbnd += __builtin_fabsf(dl[a][e] - tau) < 1e-6f;
                        nedge += (int)bit;
                    }
                    if (LEARNED && live) {
                        int bin = 0;
#pragma unroll
                        for (int k = 1; k < 16; ++k) bin += dl[a][e] >= (float)k * q;
                        atomicAdd(&hrow[r][bin], 1);
                        atomicAdd(&hrow[r][16], (int)bit);
                        if (!diag) {
                            atomicAdd(&hcol[c][bin], 1);
                            atomicAdd(&hcol[c][16], (int)bit);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
            *reinterpret_cast<uint16_t *>(&tile[0][(ty * 4 + a) * kNibStride + tx * 2]) = (uint16_t)pack_e2m1(rowbits[a]);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            *reinterpret_cast<uint16_t *>(&tile[1][(tx * 4 + e) * kNibStride + ty * 2]) = (uint16_t)pack_e2m1(colbits[e]);
        nbnd = wave_sum(nbnd);
        nedge = wave_sum(nedge);
        if (lane == 0) { red[wv][0] = nbnd; red[wv][1] = nedge; red[wv][2] = any_bad; }
        __syncthreads();
        uint8_t *Cb = w.C + d.cb_off;
        const int64_t rs = c_pitch(d.npad);
        const int r = tid >> 2, c8 = (tid & 3) * 8;
        *reinterpret_cast<uint2 *>(Cb + ((int64_t)bi * kCompatTile + r) * rs + bj * (kCompatTile / 2) + c8) =
            *reinterpret_cast<const uint2 *>(&tile[0][r * kNibStride + c8]);
        if (!diag)
            *reinterpret_cast<uint2 *>(Cb + ((int64_t)bj * kCompatTile + r) * rs + bi * (kCompatTile / 2) + c8) =
                *reinterpret_cast<const uint2 *>(&tile[1][r * kNibStride + c8]);
        if (BITS && tid < (diag ? 64 : 128)) {
            // the same rows as bits (read only by the SC2 bit-count path) (threads 0-63: the tile's rows, 64-127: its transpose), 8 bytes per
            // row into the 16-byte piece of the row's 128-column block
            const int side = tid >> 6, rr = tid & 63;
            const uint4 *src = reinterpret_cast<const uint4 *>(&tile[side][rr * kNibStride]);
            const uint4 lo = src[0], hi = src[1];
            const uint32_t nib[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
            uint32_t word[2] = {0, 0};
#pragma unroll
            for (int k = 0; k < 8; ++k) word[k >> 2] |= nibbles_to_bits(nib[k]) << (8 * (k & 3));
            const int rb = side ? bj : bi, cb = side ? bi : bj;
            uint8_t *dst = w.Cbits + d.c_off / 8 +
                           ((int64_t)(cb >> 1) * d.npad + (int64_t)rb * kCompatTile + rr) * 16 + (cb & 1) * 8;
            *reinterpret_cast<uint2 *>(dst) = make_uint2(word[0], word[1]);
        }
        if (tid < 3) w.cnt_part[3 * (int64_t)item + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
        if (LEARNED) {
            for (int k = tid; k < 64 * 17; k += 256) {
                const int rr = k / 17, f = k % 17;
                // feature slots: 0 degree, 3..18 histogram
                const int slot = f == 16 ? 0 : 3 + f;
                const int i = bi * kCompatTile + rr, j = bj * kCompatTile + rr;
                if (i < d.n && hrow[rr][f]) atomicAdd(&w.rowstat[((int64_t)b * w.max_n + i) * 20 + slot], hrow[rr][f]);
                if (!diag && j < d.n && hcol[rr][f]) atomicAdd(&w.rowstat[((int64_t)b * w.max_n + j) * 20 + slot], hcol[rr][f]);
            }
        }
    }
}

// ---------------------------------------------------------------- Eq. 2 on FP4 MFMA

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v8i __attribute__((ext_vector_type(8)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) void gvoid;
typedef __attribute__((address_space(3))) void lvoid;

constexpr int kBK = 64;                        // bytes of a packed row per pipeline stage (128 k)
constexpr int kStages = 4;                     // LDS ring depth (three stages in flight)
constexpr int kMatBytes = kSc2Tile * kBK;      // one operand's stage: 256 rows x 64 bytes
constexpr int kStageBytes = 2 * kMatBytes;
constexpr int kRingBytes = kStages * kStageBytes;   // 128 KiB
constexpr int kTileBytes = kSc2Tile * kSc2Tile * 2;  // the finished tile as uint16 (128 KiB), over the ring
constexpr int kHistLdsBins = 8192;             // weights below this are histogrammed in LDS first
constexpr int kSc2Lds = kRingBytes + kHistLdsBins * 4;   // 160 KiB: ring (then tile), histogram
static_assert(kTileBytes <= kRingBytes, "the finished tile must fit the ring");
constexpr float kAccBias = 8388608.0f;         // 2^23: a count v < 2^16 is then the low 16 bits of 2^23 + v
// Bit-count path (tiles with few edges): Eq. 2 is needed only where C_ij = 1, so a tile holding at
// most kSddmmCap edges counts popcount(row_i AND row_j) for each of its edges instead of forming
// the dense product (the threshold is a launch parameter up to kSddmmCap; 0 turns the path and the
// compatibility kernel's bit rows off). Rows arrive in chunks of kChunkKb 128-column blocks (bits),
// kChunkBufs - 1 chunks in flight; each thread keeps its edges and their counts in registers.
// LDS layout: the chunk buffers (I rows then J rows, [block][row][16 bytes] each); the edge list
// lies in the last buffer, which receives no chunk before every thread has its edges.
constexpr int kSddmmCap = 8192;                       // 32 edges per thread
constexpr int kEdgesPerThread = kSddmmCap / 256;
static_assert(kSddmmCap == TR_SC2_SPARSE_CAP_MAX, "the launch parameter's range is the path's capacity");
constexpr int kChunkKb = 4;                           // 512 columns of C per chunk
constexpr int kChunkSide = kChunkKb * kSc2Tile * 16;  // 16 KiB: one side's 256 rows of a chunk
constexpr int kChunkBytes = 2 * kChunkSide;
constexpr int kChunkBufs = 4;
constexpr int kEdgeOff = (kChunkBufs - 1) * kChunkBytes;   // edge list: uint16 (i_local << 8 | j_local)
constexpr int kScanOff = kEdgeOff + 2 * kSddmmCap;    // four wave totals of the edge-count scan
static_assert(kChunkBufs * kChunkBytes <= kRingBytes && kScanOff + 64 <= kRingBytes,
              "the bit-count path stays below the histogram");

// Wait until at most N vector-memory loads of this wave are outstanding, then
// meet the other waves. The memory clobber keeps LDS reads of the new stage
// after it; unlike __syncthreads it does not drain the later stages in flight.
#define SC2_WAIT_BARRIER(N) asm volatile("s_waitcnt vmcnt(" #N ")\n\ts_barrier" ::: "memory")

// Maximum / sum over each half of the wave (lanes 0-31, 32-63), left in lanes 31 and 63: prefix
// steps inside each 16-lane DPP row, then the last lane of rows 0 and 2 joins rows 1 and 3.
// Inputs are >= 0, so lanes that receive no value (they read 0) do not change a maximum.
__device__ __forceinline__ int half_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));   // row_bcast:15 into rows 1, 3
    return v;
}

__device__ __forceinline__ int half_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    return v;
}

// G[i][j] = C_ij * sum_k C_ik C_jk for i < j < n over 256 x 256 output tiles
// with bi <= bj. C is symmetric, so the product is C C^T and both MFMA
// operands are rows of C read along k.
//
// C is stored as E2M1 (FP4) nibbles, 1.0 = 0x2: every product is 0 or 1 and
// every partial sum is an integer below 2^24, so the float32 accumulation of
// v_mfma_scale_f32_32x32x64_f8f6f4 (unit scales) is exact, and FP4 halves the
// operand bytes of an int8 product. Accumulators start at 2^23, so a finished
// count is read from the low 16 bits of the float without a conversion.
//
// Four waves in a 2 x 2 layout each own a 128 x 128 sub-tile as 4 x 4 blocks
// of 32 x 32 (accumulators in AGPRs). Stages of 64 bytes (128 k) arrive by
// direct global->LDS 16-byte loads into a four-deep ring, three stages in
// flight (a fifth stage in flight measured slower); a row's four 16-byte chunks are stored XOR-swizzled by (row/4) mod 4
// for the fragment reads (ds_read_b128). Work items are split into 8
// contiguous ranges, one per XCD, so tiles that share rows of C share an L2.
//
// Epilogue: the tile is restaged in LDS as uint16 (weights are below 2^16),
// then read row-major: masked by C_ij and i < j < n, stored with 16-byte
// writes (whole chunks: outside i < j < n they hold zeros, which nothing reads), counted into a weight histogram (LDS, added into one of
// kHistGroups copies per pair) and reduced into the per-row maximum of the
// upper triangle. In learned mode it also adds row and column sums / maxima
// of the symmetric SC2 matrix for the per-match features.
template <bool LEARNED, bool SPARSE>
__global__ void __launch_bounds__(256, 1) k_sc2(Work w)
{
    extern __shared__ __attribute__((aligned(16))) uint8_t smem[];
    int32_t *hist = reinterpret_cast<int32_t *>(smem + kRingBytes);   // zero outside the epilogue
    uint16_t *T = reinterpret_cast<uint16_t *>(smem);
    const int total = stage_total(w, kSc2);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
    const int xcd = blockIdx.x & 7, nx = (gridDim.x - xcd + 7) >> 3, lb = blockIdx.x >> 3;
    // XCD x takes a contiguous range of the list (neighbouring tiles share rows of C in its L2):
    // equal counts for one pair, equal shares of the modelled cost for a batch
    const int chunk = (total + 7) >> 3;
    const int start = w.n1 ? xcd * chunk : w.plan->sc2_split[xcd];
    const int end = w.n1 ? min(total, (xcd + 1) * chunk) : w.plan->sc2_split[xcd + 1];
    // fragment read offsets inside a stage: row (lane & 31) of a 32-row block, chunk (ks*2 + lane/32)
    const int frow = lane & 31, fsw = (frow >> 2) & 3;
    const int foff0 = frow * kBK + 16 * ((lane >> 5) ^ fsw), foff1 = frow * kBK + 16 * ((2 + (lane >> 5)) ^ fsw);
    for (int k = tid; k < kHistLdsBins; k += 256) hist[k] = 0;
    __syncthreads();
    for (int item = start + lb; item < end; item += nx) {
        int local;
        const int b = stage_pair(w, kSc2, item, local);
        const PairDesc d = pair_desc(w, b);
        int bi, bj;
        super_decode(local, d.npad / kSc2Tile, w.sc2_super, bi, bj);
        const uint8_t *Cb = w.C + d.cb_off;
        const int64_t rs = c_pitch(d.npad);          // row pitch
        const int nk = (int)(d.npad / 2 / kBK);      // stages over the packed row
        // ---- the tile's edges: thread t holds row t of the I block over the tile's 256 columns
        const uint8_t *Cbit = w.Cbits + d.c_off / 8;
        const int64_t kbs = (int64_t)d.npad * 16;   // bytes of one 128-column block over all rows
        const bool diag = bi == bj;
        uint32_t mw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (SPARSE) {
            const int64_t ro = ((int64_t)bi * kSc2Tile + tid) * 16;
            const uint4 m0 = *reinterpret_cast<const uint4 *>(Cbit + (2 * bj) * kbs + ro);
            const uint4 m1 = *reinterpret_cast<const uint4 *>(Cbit + (2 * bj + 1) * kbs + ro);
            mw[0] = m0.x; mw[1] = m0.y; mw[2] = m0.z; mw[3] = m0.w;
            mw[4] = m1.x; mw[5] = m1.y; mw[6] = m1.z; mw[7] = m1.w;
        }
        int ecount = 0, eprefix = 0, etotal = 0;
        bool sparse = false;
        if (SPARSE) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (diag) {   // i < j only: columns above the thread's row
                    const int lo = tid + 1 - 32 * k;
                    mw[k] &= lo <= 0 ? 0xFFFFFFFFu : (lo >= 32 ? 0u : (0xFFFFFFFFu << lo));
                }
                ecount += __builtin_popcount(mw[k]);
            }
            int32_t *scanL = reinterpret_cast<int32_t *>(smem + kScanOff);
            eprefix = ecount;   // inclusive scan inside the wave, then the waves before
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(eprefix, o, 64);
                if (lane >= o) eprefix += y;
            }
            if (lane == 63) scanL[wv] = eprefix;
            __syncthreads();
            etotal = scanL[0] + scanL[1] + scanL[2] + scanL[3];
            for (int v = 0; v < wv; ++v) eprefix += scanL[v];
            eprefix -= ecount;   // exclusive
            sparse = etotal <= w.sc2_sparse_cap;
        }
        if (sparse) {
            uint16_t *edgeL = reinterpret_cast<uint16_t *>(smem + kEdgeOff);
            {
                int pos = eprefix;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    uint32_t x = mw[k];
                    while (x) {
                        const int c = __builtin_ctz(x);
                        x &= x - 1;
                        edgeL[pos] = (uint16_t)((tid << 8) | (32 * k + c));
                        ++pos;
                    }
                }
            }
            __syncthreads();   // the edge list is complete
            // thread t counts edges [e0, e1): about etotal / 256 consecutive edges (few rows each),
            // held in registers with their counts
            const int q = (etotal + 255) >> 8, e0 = min(etotal, tid * q), e1 = min(etotal, e0 + q), ne = e1 - e0;
            uint32_t myv[kEdgesPerThread];
            int myc[kEdgesPerThread];
#pragma unroll
            for (int k = 0; k < kEdgesPerThread; ++k) {
                myv[k] = k < ne ? edgeL[e0 + k] : 0u;
                myc[k] = 0;
            }
            __syncthreads();   // the edge list's buffer may now receive a chunk
            const int nkb = d.npad / 128, nch = (nkb + kChunkKb - 1) / kChunkKb;
            // chunk c: blocks kChunkKb c .. of the I rows (and J rows off the diagonal) by direct
            // global->LDS 16-byte loads; wave v loads rows 64v .. 64v+63 of each block
            auto issue_chunk = [&](int c) {
                uint8_t *dst = smem + (c % kChunkBufs) * kChunkBytes + wv * 1024;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    if (side && diag) break;
                    const int64_t ro = ((int64_t)(side ? bj : bi) * kSc2Tile + wv * 64 + lane) * 16;
#pragma unroll
                    for (int kb = 0; kb < kChunkKb; ++kb)   // past the last block: a copy of it, not counted
                        __builtin_amdgcn_global_load_lds((gvoid *)(Cbit + (int64_t)min(c * kChunkKb + kb, nkb - 1) * kbs + ro),
                                                         (lvoid *)(dst + side * kChunkSide + kb * 4096), 16, 0, 0);
                }
            };
            const int lpc = (diag ? 1 : 2) * kChunkKb;   // loads per chunk and lane
            const int nrun = etotal > 0 ? nch : 0;
            for (int c = 0; c < min(nrun, kChunkBufs - 1); ++c) issue_chunk(c);
            for (int c = 0; c < nrun; ++c) {
                // chunk c has landed once at most (chunks issued after it) x lpc loads are outstanding;
                // the barrier also tells every wave that chunk c - 1's buffer is free
                const int outstanding = min(kChunkBufs - 2, nrun - 1 - c) * lpc;
                switch (outstanding) {
                case 16: SC2_WAIT_BARRIER(16); break;
                case 12: SC2_WAIT_BARRIER(12); break;
                case 8: SC2_WAIT_BARRIER(8); break;
                case 6: SC2_WAIT_BARRIER(6); break;
                case 4: SC2_WAIT_BARRIER(4); break;
                case 2: SC2_WAIT_BARRIER(2); break;
                default: SC2_WAIT_BARRIER(0); break;
                }
                if (c + kChunkBufs - 1 < nrun) issue_chunk(c + kChunkBufs - 1);
                const uint8_t *Ib = smem + (c % kChunkBufs) * kChunkBytes, *Jb = diag ? Ib : Ib + kChunkSide;
                const int kbn = min(kChunkKb, nkb - c * kChunkKb);
                int cur = -1;
                uint4 ri[kChunkKb];
                constexpr int kU = 2;   // edges whose J rows are read together
#pragma unroll
                for (int k0 = 0; k0 < kEdgesPerThread; k0 += kU) {
                    if (k0 >= ne) continue;   // (not break: the loop must unroll, the arrays stay in registers)
                    uint4 rj[kU][kChunkKb];
#pragma unroll
                    for (int u = 0; u < kU; ++u)
#pragma unroll
                        for (int kb = 0; kb < kChunkKb; ++kb)
                            rj[u][kb] = k0 + u < ne && kb < kbn
                                            ? *reinterpret_cast<const uint4 *>(Jb + kb * 4096 + (myv[k0 + u] & 255) * 16)
                                            : make_uint4(0, 0, 0, 0);
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const int li = (int)(myv[k0 + u] >> 8);
                        if (k0 + u < ne && li != cur) {
                            cur = li;
#pragma unroll
                            for (int kb = 0; kb < kChunkKb; ++kb) ri[kb] = *reinterpret_cast<const uint4 *>(Ib + kb * 4096 + li * 16);
                        }
                        int sum = 0;
#pragma unroll
                        for (int kb = 0; kb < kChunkKb; ++kb)
                            sum += __builtin_popcount(ri[kb].x & rj[u][kb].x) + __builtin_popcount(ri[kb].y & rj[u][kb].y) +
                                   __builtin_popcount(ri[kb].z & rj[u][kb].z) + __builtin_popcount(ri[kb].w & rj[u][kb].w);
                        myc[k0 + u] += k0 + u < ne ? sum : 0;
                    }
                }
            }
            // the LDS becomes the tile T (zero, then the counts scattered in; weights below 2^16)
            __syncthreads();
            for (int k = tid; k < kTileBytes / 16; k += 256) reinterpret_cast<uint4 *>(smem)[k] = make_uint4(0, 0, 0, 0);
            __syncthreads();
            int32_t *ghs = w.ghist + ((int64_t)b * kHistGroups + local % kHistGroups) * w.hist_stride;
            const bool small_hist = d.n <= kHistLdsBins;
#pragma unroll
            for (int k = 0; k < kEdgesPerThread; ++k) {
                if (k < ne) {
                    T[(myv[k] >> 8) * kSc2Tile + (myv[k] & 255)] = (uint16_t)myc[k];
                    const int c = myc[k];
                    if (c > 0) {   // the weight histogram counts nonzero weights
                        if (small_hist || c < kHistLdsBins) atomicAdd(&hist[c], 1);
                        else atomicAdd(&ghs[c], 1);
                    }
                }
            }
            __syncthreads();
        } else {
        // load s of a stage: row r = (s&3)*64 + wv*16 + lane/4 of operand s/4 into LDS chunk lane&3,
        // which holds the row's global chunk (lane&3) ^ ((r/4)&3)
        uint32_t goff[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int r = (s & 3) * 64 + wv * 16 + (lane >> 2);
            const int64_t row = (int64_t)((s >> 2) ? bj : bi) * kSc2Tile + r;
            goff[s] = (uint32_t)(row * rs + 16 * ((lane & 3) ^ ((r >> 2) & 3)));
        }
        auto issue = [&](int kt) {
            uint8_t *dst = smem + (kt % kStages) * kStageBytes + wv * 1024;
            const uint8_t *src = Cb + (int64_t)kt * kBK;
#pragma unroll
            for (int s = 0; s < 8; ++s)
                __builtin_amdgcn_global_load_lds((gvoid *)(src + goff[s]),
                                                 (lvoid *)(dst + (s >> 2) * kMatBytes + (s & 3) * 4096), 16, 0, 0);
        };
        v16f acc[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[x][y][r] = kAccBias;
#pragma unroll
        for (int kt = 0; kt < kStages - 1; ++kt)
            if (kt < nk) issue(kt);
        for (int kt = 0; kt < nk; ++kt) {
            // stage kt has landed once at most (stages issued after it) x 8 loads are outstanding
            const int later = min(kStages - 2, nk - 1 - kt);
            if (later >= 2) SC2_WAIT_BARRIER(16);
            else if (later == 1) SC2_WAIT_BARRIER(8);
            else SC2_WAIT_BARRIER(0);
            if (kt + kStages - 1 < nk) issue(kt + kStages - 1);
            const uint8_t *As = smem + (kt % kStages) * kStageBytes, *Bs = As + kMatBytes;
            // fragment reads run ahead of the MFMAs that use them: the eight of the first half and
            // the four A fragments of the second are issued before the first MFMA, the four B
            // fragments of the second half after the first row of four MFMAs (at most twelve LDS
            // reads outstanding, below the counter's limit); the scheduling barriers keep this order
            v4i fa[2][4], fb[2][4];
            auto mfma_row = [&](int ks, int x) {
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    // 32 FP4 values of k per lane: 16 bytes, the upper half of the operand is unused
                    const v8i a8 = {fa[ks][x][0], fa[ks][x][1], fa[ks][x][2], fa[ks][x][3], 0, 0, 0, 0};
                    const v8i b8 = {fb[ks][y][0], fb[ks][y][1], fb[ks][y][2], fb[ks][y][3], 0, 0, 0, 0};
                    acc[x][y] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc[x][y], 4, 4, 0, 127, 0,
                                                                                 127);
                }
            };
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                fa[0][x] = *reinterpret_cast<const v4i *>(As + (wm * 128 + x * 32) * kBK + foff0);
                fb[0][x] = *reinterpret_cast<const v4i *>(Bs + (wn * 128 + x * 32) * kBK + foff0);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int x = 0; x < 4; ++x) fa[1][x] = *reinterpret_cast<const v4i *>(As + (wm * 128 + x * 32) * kBK + foff1);
            __builtin_amdgcn_sched_barrier(0);
            mfma_row(0, 0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int y = 0; y < 4; ++y) fb[1][y] = *reinterpret_cast<const v4i *>(Bs + (wn * 128 + y * 32) * kBK + foff1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int x = 1; x < 4; ++x) mfma_row(0, x);
#pragma unroll
            for (int x = 0; x < 4; ++x) mfma_row(1, x);
        }
        __syncthreads();   // no stage is read any more: the ring becomes the tile T[256][256] (uint16)
        // lane holds column (lane & 31) and rows 8*(r/4) + 4*(lane/32) + r%4 of each 32 x 32 block;
        // the whole vector is reinterpreted before the low halves are taken
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const v16i ai = __builtin_bit_cast(v16i, acc[x][y]);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int lr = wm * 128 + x * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int lc = wn * 128 + y * 32 + (lane & 31);
                    T[lr * kSc2Tile + lc] = (uint16_t)ai[r];
                }
            }
        __syncthreads();
        }   // dense (MFMA) path
        int32_t *gh = w.ghist + ((int64_t)b * kHistGroups + local % kHistGroups) * w.hist_stride;
        int32_t *rowmax = w.rowmax + (int64_t)b * w.max_n;
        int32_t *rstat = w.rowstat + (int64_t)b * w.max_n * 20;
        uint16_t *Gb = w.G + d.g_off;
        // every pair of the tile is in the strict upper triangle and below n: no per-entry test
        const bool interior = bi < bj && (bj + 1) * kSc2Tile <= d.n;
        const bool small_n = d.n <= kHistLdsBins;
        // thread t: column chunk cc = t % 32 (8 columns) of rows lr = 8k + t / 32, k = 0..31, in four
        // batches of eight rows; the packed C_ij of the next batch are in flight while one is processed.
        // Lanes 0-31 of a wave hold one row, lanes 32-63 the next.
        const int cc = tid & 31;
        const int j0 = bj * kSc2Tile + cc * 8;
        const uint8_t *crow = Cb + ((int64_t)bi * kSc2Tile + (tid >> 5)) * rs + j0 / 2;
        // (the bit-count path's T holds only its edges' weights: no C_ij or range masking)
        uint32_t cur[8], nxt[8];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            cur[q] = sparse ? 0x22222222u : *reinterpret_cast<const uint32_t *>(crow + (int64_t)(q * 8) * rs);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            if (kb < 3) {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    nxt[q] = sparse ? 0x22222222u
                                    : *reinterpret_cast<const uint32_t *>(crow + (int64_t)(((kb + 1) * 8 + q) * 8) * rs);
            }
            uint4 tv[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                tv[q] = *reinterpret_cast<const uint4 *>(&T[((kb * 8 + q) * 8 + (tid >> 5)) * kSc2Tile + cc * 8]);
            int rmax[8], rsum[8];
            uint32_t ow[8][4], nzq[8];
            // masking, stores and row maxima of the eight rows first (straight-line code), the
            // histogram of their nonzero weights after
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int lr = (kb * 8 + q) * 8 + (tid >> 5);
                const int i = bi * kSc2Tile + lr;
                const uint32_t tw[4] = {tv[q].x, tv[q].y, tv[q].z, tv[q].w};
                // entries e of the chunk with i < j0 + e < n (all eight except at the diagonal and the edge)
                const int e_lo = min(8, max(0, i + 1 - j0)), e_hi = min(8, max(0, d.n - j0));
                const uint32_t vm = (interior || sparse) ? 0xFFu : (((1u << e_hi) - 1u) & ~((1u << e_lo) - 1u));
                const uint32_t cb = cur[q] >> 1;   // C of column e at bit 4e
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const uint32_t lo = ((cb >> (8 * k)) & 1u) & (vm >> (2 * k));
                    const uint32_t hi = ((cb >> (8 * k + 4)) & 1u) & (vm >> (2 * k + 1));
                    ow[q][k] = tw[k] & ((lo * 0xFFFFu) | (hi * 0xFFFF0000u));
                }
                const u16x2 m2 = __builtin_elementwise_max(
                    __builtin_elementwise_max(__builtin_bit_cast(u16x2, ow[q][0]), __builtin_bit_cast(u16x2, ow[q][1])),
                    __builtin_elementwise_max(__builtin_bit_cast(u16x2, ow[q][2]), __builtin_bit_cast(u16x2, ow[q][3])));
                rmax[q] = max((int)m2.x, (int)m2.y);
                rsum[q] = 0;
                if (LEARNED) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) rsum[q] += (int)((ow[q][e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
                    // the masked tile, for the column pass
                    *reinterpret_cast<uint4 *>(&T[lr * kSc2Tile + cc * 8]) =
                        make_uint4(ow[q][0], ow[q][1], ow[q][2], ow[q][3]);
                }
                // every chunk is stored whole: entries with j <= i or j >= n are zero and no reader looks at them
                *reinterpret_cast<uint4 *>(Gb + (int64_t)i * d.npad + j0) =
                    make_uint4(ow[q][0], ow[q][1], ow[q][2], ow[q][3]);
                uint32_t nz = 0;
#pragma unroll
                for (int e = 0; e < 8; ++e) nz |= (uint32_t)(((ow[q][e >> 1] >> (16 * (e & 1))) & 0xFFFFu) != 0) << e;
                nzq[q] = nz;
            }
            // weight histogram: one LDS atomic per nonzero weight, round by round (a lane's next
            // nonzero each round) over four rows at a time, as many rounds as the lane with the
            // most nonzero weights in them needs. Entry e of the 32: row e / 8, 16 bits at
            // 16 (e mod 4) of that row's low or high 64-bit half, selected arithmetically (a
            // lane-varying switch would become branches).
#pragma unroll
            for (int g4 = 0; g4 < 2; ++g4) {
                if (sparse) break;   // the bit-count path histogrammed its edges already
                uint32_t nz = 0;
                uint64_t h64[8];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = g4 * 4 + u;
                    nz |= nzq[q] << (8 * u);
                    h64[2 * u] = (uint64_t)ow[q][0] | ((uint64_t)ow[q][1] << 32);
                    h64[2 * u + 1] = (uint64_t)ow[q][2] | ((uint64_t)ow[q][3] << 32);
                }
                auto next_weight = [&]() -> int {
                    const int e = __builtin_ctz(nz);
                    nz &= nz - 1;
                    const int hsel = e >> 2;   // half index 0..7
                    const uint64_t a0 = (hsel & 1) ? h64[1] : h64[0], a1 = (hsel & 1) ? h64[3] : h64[2];
                    const uint64_t a2 = (hsel & 1) ? h64[5] : h64[4], a3 = (hsel & 1) ? h64[7] : h64[6];
                    const uint64_t b0 = (hsel & 2) ? a1 : a0, b1 = (hsel & 2) ? a3 : a2;
                    const uint64_t half = (hsel & 4) ? b1 : b0;
                    return (int)((half >> (16 * (e & 3))) & 0xFFFFu);
                };
                if (small_n) {   // every weight is below n <= kHistLdsBins
                    while (__any(nz))
                        if (nz) atomicAdd(&hist[next_weight()], 1);
                } else {
                    while (__any(nz)) {
                        if (nz) {
                            const int v = next_weight();
                            if (v < kHistLdsBins) atomicAdd(&hist[v], 1);
                            else atomicAdd(&gh[v], 1);
                        }
                    }
                }
            }
            // row maxima (and sums) over the 32 lanes of each row, eight rows interleaved (DPP, no LDS)
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                rmax[q] = half_max(rmax[q]);
                if (LEARNED) rsum[q] = half_sum(rsum[q]);
            }
            if ((lane & 31) == 31) {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = bi * kSc2Tile + (kb * 8 + q) * 8 + (tid >> 5);
                    if (rmax[q] > 0) {
                        atomicMax(&rowmax[i], rmax[q]);
                        if (LEARNED) {
                            atomicAdd(&rstat[i * 20 + 1], rsum[q]);
                            atomicMax(&rstat[i * 20 + 2], rmax[q]);
                        }
                    }
                }
            }
            if (kb < 3) {
#pragma unroll
                for (int q = 0; q < 8; ++q) cur[q] = nxt[q];
            }
        }
        if (LEARNED) {
            // column j of the upper tile is row j of the lower one (Ghat is symmetric): thread t sums
            // and maximises columns 2c, 2c+1 (c = t mod 128) of the masked tile over rows of parity
            // t / 128, sixteen 4-byte reads in flight; the two parities meet in LDS
            __syncthreads();
            const int cp = tid & 127, par = tid >> 7;
            const uint32_t *Tw = reinterpret_cast<const uint32_t *>(T);
            int s0 = 0, s1 = 0;
            u16x2 mx = {0, 0};
            for (int m0 = 0; m0 < kSc2Tile / 2; m0 += 16) {
                uint32_t v[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) v[u] = Tw[(2 * (m0 + u) + par) * (kSc2Tile / 2) + cp];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    s0 += (int)(v[u] & 0xFFFFu);
                    s1 += (int)(v[u] >> 16);
                    mx = __builtin_elementwise_max(mx, __builtin_bit_cast(u16x2, v[u]));
                }
            }
            __syncthreads();   // the tile is read
            int32_t *xl = reinterpret_cast<int32_t *>(smem);
            if (par) {
                xl[3 * cp] = s0;
                xl[3 * cp + 1] = s1;
                xl[3 * cp + 2] = (int32_t)__builtin_bit_cast(uint32_t, mx);
            }
            __syncthreads();
            if (!par) {
                const u16x2 m2 = __builtin_elementwise_max(mx, __builtin_bit_cast(u16x2, (uint32_t)xl[3 * cp + 2]));
                const int cs[2] = {s0 + xl[3 * cp], s1 + xl[3 * cp + 1]}, cm[2] = {(int)m2.x, (int)m2.y};
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int j = bj * kSc2Tile + 2 * cp + e;
                    if (cm[e] > 0) {
                        atomicAdd(&rstat[j * 20 + 1], cs[e]);
                        atomicMax(&rstat[j * 20 + 2], cm[e]);
                    }
                }
            }
        }
        __syncthreads();
        const int hl = min(d.n, kHistLdsBins);
        for (int k = tid; k < hl; k += 256) {
            const int c = hist[k];
            if (c) {
                atomicAdd(&gh[k], c);
                hist[k] = 0;
            }
        }
        __syncthreads();   // T is the next item's ring
    }
}

}  // namespace

hipError_t launch_plan(const Work &w, const int32_t *offsets, int32_t n_single, int32_t B, int32_t max_n,
                       PairDesc *pairs, PairState *state, Plan *plan, int32_t *pre, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, offsets, n_single, B, max_n, w.pool, w.H, pairs,
                       state, plan, pre, w.pre_stride);
    return hipGetLastError();
}

hipError_t launch_prep_learned(const Work &w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_prep_learned, dim3(grid), dim3(256), 0, s, w);
    return hipGetLastError();
}

hipError_t launch_compat(const Work &w, int grid, hipStream_t s)
{
    // the bit rows are written only for an SC2 launch that may take the bit-count path
    const bool learned = w.learned && w.feat_all, bits = w.sc2_sparse_cap > 0;
    if (learned && bits) hipLaunchKernelGGL((k_compat<true, true>), dim3(grid), dim3(256), 0, s, w);
    else if (learned) hipLaunchKernelGGL((k_compat<true, false>), dim3(grid), dim3(256), 0, s, w);
    else if (bits) hipLaunchKernelGGL((k_compat<false, true>), dim3(grid), dim3(256), 0, s, w);
    else hipLaunchKernelGGL((k_compat<false, false>), dim3(grid), dim3(256), 0, s, w);
    return hipGetLastError();
}

hipError_t launch_sc2(const Work &w, int grid, hipStream_t s)
{
    // separate instances: the dense-only kernel carries none of the bit-count path's registers
    const bool sparse = w.sc2_sparse_cap > 0;
    if (w.learned && sparse) hipLaunchKernelGGL((k_sc2<true, true>), dim3(grid), dim3(256), kSc2Lds, s, w);
    else if (w.learned) hipLaunchKernelGGL((k_sc2<true, false>), dim3(grid), dim3(256), kSc2Lds, s, w);
    else if (sparse) hipLaunchKernelGGL((k_sc2<false, true>), dim3(grid), dim3(256), kSc2Lds, s, w);
    else hipLaunchKernelGGL((k_sc2<false, false>), dim3(grid), dim3(256), kSc2Lds, s, w);
    return hipGetLastError();
}

hipError_t setup_graph_kernels()
{
    const void *fns[4] = {reinterpret_cast<const void *>(k_sc2<false, false>),
                          reinterpret_cast<const void *>(k_sc2<false, true>),
                          reinterpret_cast<const void *>(k_sc2<true, false>),
                          reinterpret_cast<const void *>(k_sc2<true, true>)};
    hipError_t e = hipSuccess;
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
        e = hipFuncSetAttribute(fns[k], hipFuncAttributeMaxDynamicSharedMemorySize, kSc2Lds);
    return e;
}

}  // namespace tr
