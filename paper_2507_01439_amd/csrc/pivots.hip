// Pivot selection (Eq. 4) on gfx950.
//
// The pivots are the first K pairs i < j of the O2Graph ordered by
// (weight desc, i asc, j asc), K = min(K1, N(N-1)/2). Weights are integers
// below N, so the K-th largest weight alpha comes from an exact histogram; every
// pair heavier than alpha is a pivot and the first m pairs of weight alpha in
// row-major order fill the remaining slots. Per-row counts give each row its
// output position, so the emission is deterministic without atomics on the
// output, and a single-workgroup bitonic sort orders the K keys.
#include "common.h"

namespace tr {
namespace {

constexpr int kHistLds = 8192;   // weights below this are histogrammed in LDS first

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
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

// Histogram of the nonzero O2Graph weights of every pair.
__global__ void __launch_bounds__(256) k_hist(Work w)
{
    __shared__ int32_t h[kHistLds];
    const int total = w.plan->total[kRowBlk], B = w.plan->B;
    const int32_t *pre = w.pre + kRowBlk * w.pre_stride;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = find_pair(pre, B, item);
        const PairDesc d = w.pairs[b];
        const int lim = min(d.n, kHistLds);
        for (int k = threadIdx.x; k < lim; k += 256) h[k] = 0;
        __syncthreads();
        int32_t *gh = w.hist + (int64_t)b * w.max_n;
        const int r0 = (item - pre[b]) * kRowsPerItem, r1 = min(r0 + kRowsPerItem, d.n);
        for (int i = r0; i < r1; ++i) {
            const uint16_t *row = w.G + d.g_off + (int64_t)i * d.npad;
            for (int j = i + 1 + threadIdx.x; j < d.n; j += 256) {
                const int v = row[j];
                if (v > 0) {
                    if (v < kHistLds) atomicAdd(&h[v], 1);
                    else atomicAdd(&gh[v], 1);
                }
            }
        }
        __syncthreads();
        for (int k = 1 + threadIdx.x; k < lim; k += 256)
            if (h[k]) atomicAdd(&gh[k], h[k]);
        __syncthreads();
    }
}

// alpha = the K-th largest weight over all N(N-1)/2 pairs (zeros included).
__global__ void __launch_bounds__(1024) k_thresh(Work w)
{
    __shared__ int64_t lds[17];
    __shared__ int32_t res[3];
    const int b = blockIdx.x;
    const PairDesc d = w.pairs[b];
    const int64_t K = d.kpiv;
    if (K <= 0) return;
    const int32_t *gh = w.hist + (int64_t)b * w.max_n;
    const int nb = d.n - 1;                     // bins w = 1 .. n-1, walked from the top
    const int cs = (nb + 1023) / 1024;
    const int u0 = min(nb, (int)threadIdx.x * cs), u1 = min(nb, u0 + cs);
    int64_t local = 0;
    for (int u = u0; u < u1; ++u) local += gh[d.n - 1 - u];
    int64_t tot;
    const int64_t excl = block_exclusive_scan<int64_t>(local, lds, tot);
    if (threadIdx.x == 0 && K > tot) { res[0] = 0; res[1] = (int32_t)tot; res[2] = (int32_t)(K - tot); }
    if (K <= tot && excl < K && K <= excl + local) {
        int64_t cum = excl;
        for (int u = u0; u < u1; ++u) {
            const int wt = d.n - 1 - u;
            const int64_t c = gh[wt];
            if (cum + c >= K) { res[0] = wt; res[1] = (int32_t)cum; res[2] = (int32_t)(K - cum); break; }
            cum += c;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        w.state[b].alpha = res[0];
        w.state[b].c_gt = res[1];
        w.state[b].m_eq = res[2];
    }
}

// Per row: pairs heavier than alpha and pairs equal to alpha; per block: their sums.
__global__ void __launch_bounds__(256) k_rowcount(Work w)
{
    __shared__ int32_t part[4][2];
    const int total = w.plan->total[kRowBlk], B = w.plan->B;
    const int32_t *pre = w.pre + kRowBlk * w.pre_stride;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = find_pair(pre, B, item);
        const PairDesc d = w.pairs[b];
        const int alpha = w.state[b].alpha;
        const int blk = item - pre[b];
        int sg = 0, se = 0;
        for (int rr = 0; rr < kRowsPerItem / 4; ++rr) {
            const int i = blk * kRowsPerItem + wv * (kRowsPerItem / 4) + rr;
            if (i >= d.n) break;
            const uint16_t *row = w.G + d.g_off + (int64_t)i * d.npad;
            int cg = 0, ce = 0;
            for (int j = i + 1 + lane; j < d.n; j += 64) {
                const int v = row[j];
                cg += v > alpha;
                ce += v == alpha;
            }
            cg = wave_sum(cg);
            ce = wave_sum(ce);
            if (lane == 0) {
                w.rowcnt[((int64_t)b * w.max_n + i) * 2] = cg;
                w.rowcnt[((int64_t)b * w.max_n + i) * 2 + 1] = ce;
            }
            sg += cg;
            se += ce;
        }
        if (lane == 0) { part[wv][0] = sg; part[wv][1] = se; }
        __syncthreads();
        if (threadIdx.x < 2) {
            int s = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] + part[3][threadIdx.x];
            w.blkcnt[((int64_t)b * w.nblk_stride + blk) * 2 + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

// Write every pivot's key at its final rank among (> alpha) or (== alpha) pairs.
__global__ void __launch_bounds__(256) k_emit(Work w)
{
    __shared__ int64_t lds[17];
    __shared__ int32_t rowpre[kRowsPerItem][2];
    const int total = w.plan->total[kRowBlk], B = w.plan->B;
    const int32_t *pre = w.pre + kRowBlk * w.pre_stride;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = find_pair(pre, B, item);
        const PairDesc d = w.pairs[b];
        const PairState st = w.state[b];
        const int blk = item - pre[b];
        // counts of all earlier blocks of this pair
        int64_t pg = 0, pe = 0;
        for (int k = threadIdx.x; k < blk; k += 256) {
            pg += w.blkcnt[((int64_t)b * w.nblk_stride + k) * 2];
            pe += w.blkcnt[((int64_t)b * w.nblk_stride + k) * 2 + 1];
        }
        int64_t tg, te;
        block_exclusive_scan<int64_t>(pg, lds, tg);
        block_exclusive_scan<int64_t>(pe, lds, te);
        if (threadIdx.x == 0) {
            int32_t g = (int32_t)tg, e = (int32_t)te;
            for (int rr = 0; rr < kRowsPerItem; ++rr) {
                const int i = blk * kRowsPerItem + rr;
                rowpre[rr][0] = g;
                rowpre[rr][1] = e;
                if (i < d.n) {
                    g += w.rowcnt[((int64_t)b * w.max_n + i) * 2];
                    e += w.rowcnt[((int64_t)b * w.max_n + i) * 2 + 1];
                }
            }
        }
        __syncthreads();
        uint64_t *cand = w.cand + (int64_t)b * w.pool_cap;
        for (int rr = 0; rr < kRowsPerItem / 4; ++rr) {
            const int lr = wv * (kRowsPerItem / 4) + rr, i = blk * kRowsPerItem + lr;
            if (i >= d.n) break;
            const int ng = w.rowcnt[((int64_t)b * w.max_n + i) * 2];
            const int ne = w.rowcnt[((int64_t)b * w.max_n + i) * 2 + 1];
            int rg = rowpre[lr][0], re = rowpre[lr][1];
            const int gend = rg + ng;
            const int eend = min(re + ne, st.m_eq);
            if (rg >= gend && re >= eend) continue;
            const uint16_t *row = w.G + d.g_off + (int64_t)i * d.npad;
            for (int j0 = i + 1; j0 < d.n && (rg < gend || re < eend); j0 += 64) {
                const int j = j0 + lane;
                const int v = j < d.n ? (int)row[j] : -1;
                const bool isg = v > st.alpha, ise = v == st.alpha;
                const uint64_t mg = __ballot(isg), me = __ballot(ise);
                const uint64_t below = (lane == 0) ? 0 : (~0ull >> (64 - lane));
                if (isg) cand[rg + __popcll(mg & below)] = pivot_key(v, i, j);
                if (ise) {
                    const int r = re + __popcll(me & below);
                    if (r < st.m_eq) cand[st.c_gt + r] = pivot_key(v, i, j);
                }
                rg += __popcll(mg);
                re += __popcll(me);
            }
        }
        __syncthreads();
    }
}

// Bitonic sort of the K selected keys of one pair in LDS; write (i, j, w).
__global__ void __launch_bounds__(1024) k_sort(Work w)
{
    extern __shared__ uint64_t keys[];
    const int b = blockIdx.x;
    const PairDesc d = w.pairs[b];
    const int K = d.kpiv;
    int P = 1;
    while (P < K) P <<= 1;
    const uint64_t *cand = w.cand + (int64_t)b * w.pool_cap;
    for (int k = threadIdx.x; k < P; k += 1024) keys[k] = k < K ? cand[k] : ~0ull;
    __syncthreads();
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < P / 2; t += 1024) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = keys[lo], c = keys[hi];
                if ((a > c) == up) { keys[lo] = c; keys[hi] = a; }
            }
            __syncthreads();
        }
    }
    int32_t *out = w.pivots_plain + (int64_t)b * w.pool_cap * 3;
    for (int p = threadIdx.x; p < w.pool; p += 1024) {
        if (p < K) {
            const uint64_t k = keys[p];
            out[3 * p] = (int32_t)((k >> 20) & 0xFFFFF);
            out[3 * p + 1] = (int32_t)(k & 0xFFFFF);
            out[3 * p + 2] = (int32_t)(0xFFFFu - (uint32_t)(k >> 40));
        } else {
            out[3 * p] = -1;
            out[3 * p + 1] = -1;
            out[3 * p + 2] = 0;
        }
    }
}

}  // namespace

hipError_t launch_pivots(const Work &w, int B, int grid_rows, hipStream_t s)
{
    hipLaunchKernelGGL(k_hist, dim3(grid_rows), dim3(256), 0, s, w);
    hipLaunchKernelGGL(k_thresh, dim3(B), dim3(1024), 0, s, w);
    hipLaunchKernelGGL(k_rowcount, dim3(grid_rows), dim3(256), 0, s, w);
    hipLaunchKernelGGL(k_emit, dim3(grid_rows), dim3(256), 0, s, w);
    int P = 1;
    while (P < w.pool) P <<= 1;
    static bool lds_raised = false;   // keys of up to TR_MAX_POOL pivots: 128 KiB of the 160 KiB LDS
    if (!lds_raised) {
        hipFuncSetAttribute(reinterpret_cast<const void *>(k_sort), hipFuncAttributeMaxDynamicSharedMemorySize,
                            TR_MAX_POOL * (int)sizeof(uint64_t));
        lds_raised = true;
    }
    hipLaunchKernelGGL(k_sort, dim3(B), dim3(1024), (size_t)P * sizeof(uint64_t), s, w);
    return hipGetLastError();
}

}  // namespace tr
