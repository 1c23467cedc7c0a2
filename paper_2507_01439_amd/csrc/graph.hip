// Graph construction on gfx950: work planning, the pairwise-length
// compatibility matrix (Eq. 1) and the SC2 weights of the O2Graph
// (Eq. 2 restricted to i < j, Definition 2) on int8 MFMA.
#include "common.h"

namespace tr {
namespace {

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

// ---------------------------------------------------------------- planning

__global__ void __launch_bounds__(1024) k_plan(const int32_t *offsets, int32_t n_single, int32_t B,
                                               int32_t max_n, int32_t pool, int32_t H,
                                               PairDesc *pairs, PairState *state, Plan *plan,
                                               int32_t *pre, int32_t pre_stride)
{
    __shared__ int64_t lds[17];
    int64_t carry[kNumPrefix + 1] = {0, 0, 0, 0, 0, 0};
    for (int base = 0; base < B; base += blockDim.x) {
        const int b = base + threadIdx.x;
        int32_t n = 0, pt = 0;
        bool ok = false;
        if (b < B) {
            if (offsets) { pt = offsets[b]; n = offsets[b + 1] - pt; }
            else n = n_single;
            ok = n >= 3 && n <= max_n;
        }
        const int32_t nn = ok ? n : 0;
        const int32_t npad = ok ? (n + kSc2Tile - 1) / kSc2Tile * kSc2Tile : 0;
        const int64_t nb64 = npad / kCompatTile, nb128 = npad / kSc2Tile;
        int64_t cnt[kNumPrefix + 1];
        cnt[kPrep] = (nn + kPrepRows - 1) / kPrepRows;
        cnt[kCompat] = nb64 * (nb64 + 1) / 2;
        cnt[kSc2] = nb128 * (nb128 + 1) / 2;
        cnt[kRowBlk] = (nn + kRowsPerItem - 1) / kRowsPerItem;
        cnt[kScore] = ok ? (int64_t)((H + kScoreHyp - 1) / kScoreHyp) * ((nn + kScorePts - 1) / kScorePts) : 0;
        cnt[kNumPrefix] = (int64_t)npad * npad;   // arena bytes
        int64_t excl[kNumPrefix + 1];
        for (int s = 0; s <= kNumPrefix; ++s) {
            int64_t tot;
            excl[s] = block_exclusive_scan<int64_t>(cnt[s], lds, tot) + carry[s];
            carry[s] += tot;
        }
        if (b < B) {
            for (int s = 0; s < kNumPrefix; ++s) pre[s * pre_stride + b] = (int32_t)excl[s];
            PairDesc d;
            d.n = nn;
            d.npad = npad;
            d.pt_off = pt;
            const int64_t pairs_all = (int64_t)nn * (nn - 1) / 2;
            d.kpiv = (int32_t)(pairs_all < pool ? pairs_all : pool);
            d.c_off = excl[kNumPrefix];
            d.g_off = excl[kNumPrefix];
            pairs[b] = d;
            PairState st = {};
            st.status = (b < B && !ok) ? TR_ERR_INVALID_ARG : TR_OK;
            state[b] = st;
        }
    }
    if (threadIdx.x == 0) {
        plan->B = B;
        for (int s = 0; s < kNumPrefix; ++s) {
            pre[s * pre_stride + B] = (int32_t)carry[s];
            plan->total[s] = (int32_t)carry[s];
        }
    }
}

// Zero the per-row accumulators of every pair and flag non-finite input.
__global__ void __launch_bounds__(256) k_prep(Work w)
{
    const int total = w.plan->total[kPrep], B = w.plan->B;
    const int32_t *pre = w.pre + kPrep * w.pre_stride;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = find_pair(pre, B, item);
        const PairDesc d = w.pairs[b];
        const int i = (item - pre[b]) * kPrepRows + threadIdx.x;
        bool bad = false;
        if (i < d.n) {
            w.hist[(int64_t)b * w.max_n + i] = 0;
            if (w.learned) {
                int32_t *rs = w.rowstat + ((int64_t)b * w.max_n + i) * 20;
                for (int f = 0; f < 20; ++f) rs[f] = 0;
            }
            const float *x = w.src + 3 * (int64_t)(d.pt_off + i), *y = w.dst + 3 * (int64_t)(d.pt_off + i);
            for (int k = 0; k < 3; ++k) bad |= !isfinite(x[k]) || !isfinite(y[k]);
        }
        if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(&w.state[b].nonfinite, 1);
    }
}

// ---------------------------------------------------------------- Eq. 1

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

// One 64 x 64 tile (bi <= bj) of C per work item: each thread evaluates a
// 4 x 4 block of pairs once and writes it to both triangles with 4-byte
// stores (16 lanes cover one 64-byte row segment).
__global__ void __launch_bounds__(256) k_compat(Work w)
{
    __shared__ float px[2][64][3], py[2][64][3];
    __shared__ int32_t hrow[64][17], hcol[64][17];   // learned mode: delta histogram and degree per row / col
    const int total = w.plan->total[kCompat], B = w.plan->B;
    const int32_t *pre = w.pre + kCompat * w.pre_stride;
    const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
    const float tau = w.tau, q = tau * 0.25f;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int b = find_pair(pre, B, item);
        const PairDesc d = w.pairs[b];
        int bi, bj;
        tri_decode(item - pre[b], d.npad / kCompatTile, bi, bj);
        if (tid < 128) {
            const int side = tid >> 6, r = tid & 63;
            const int i = (side ? bj : bi) * kCompatTile + r;
            for (int k = 0; k < 3; ++k) {
                px[side][r][k] = i < d.n ? w.src[3 * (int64_t)(d.pt_off + i) + k] : 0.0f;
                py[side][r][k] = i < d.n ? w.dst[3 * (int64_t)(d.pt_off + i) + k] : 0.0f;
            }
        }
        if (w.learned) {
            for (int k = tid; k < 64 * 17; k += 256) { hrow[k / 17][k % 17] = 0; hcol[k / 17][k % 17] = 0; }
        }
        __syncthreads();
        uint32_t rowbits[4] = {0, 0, 0, 0}, colbits[4] = {0, 0, 0, 0};
        int nbnd = 0, nedge = 0;
        const bool diag = bi == bj;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int r = ty * 4 + a, i = bi * kCompatTile + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int c = tx * 4 + e, j = bj * kCompatTile + c;
                const float lx = length32(px[0][r][0] - px[1][c][0], px[0][r][1] - px[1][c][1],
                                          px[0][r][2] - px[1][c][2]);
                const float ly = length32(py[0][r][0] - py[1][c][0], py[0][r][1] - py[1][c][1],
                                          py[0][r][2] - py[1][c][2]);
                const float dl = __builtin_fabsf(lx - ly);
                const bool live = i != j && i < d.n && j < d.n;
                const uint32_t bit = (live && dl <= tau) ? 1u : 0u;
                rowbits[a] |= bit << (8 * e);
                colbits[e] |= bit << (8 * a);
                if (live && i < j) {
                    nbnd += __builtin_fabsf(dl - tau) < 1e-6f;
                    nedge += (int)bit;
                }
                if (w.learned && live) {
                    int bin = 0;
#pragma unroll
                    for (int k = 1; k < 16; ++k) bin += dl >= (float)k * q;
                    atomicAdd(&hrow[r][bin], 1);
                    atomicAdd(&hrow[r][16], (int)bit);
                    if (!diag) {
                        atomicAdd(&hcol[c][bin], 1);
                        atomicAdd(&hcol[c][16], (int)bit);
                    }
                }
            }
        }
        uint8_t *Cb = w.C + d.c_off;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int64_t i = bi * kCompatTile + ty * 4 + a;
            *reinterpret_cast<uint32_t *>(Cb + i * d.npad + bj * kCompatTile + tx * 4) = rowbits[a];
        }
        if (!diag) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t j = bj * kCompatTile + tx * 4 + e;
                *reinterpret_cast<uint32_t *>(Cb + j * d.npad + bi * kCompatTile + ty * 4) = colbits[e];
            }
        }
        nbnd = wave_sum(nbnd);
        nedge = wave_sum(nedge);
        if ((tid & 63) == 0 && (nbnd | nedge)) {
            atomicAdd(&w.state[b].n_boundary, nbnd);
            atomicAdd(&w.state[b].n_edges, nedge);
        }
        if (w.learned) {
            __syncthreads();
            for (int k = tid; k < 64 * 17; k += 256) {
                const int r = k / 17, f = k % 17;
                // feature slots: 0 degree, 3..18 histogram
                const int slot = f == 16 ? 0 : 3 + f;
                const int i = bi * kCompatTile + r, j = bj * kCompatTile + r;
                if (i < d.n && hrow[r][f]) atomicAdd(&w.rowstat[((int64_t)b * w.max_n + i) * 20 + slot], hrow[r][f]);
                if (!diag && j < d.n && hcol[r][f]) atomicAdd(&w.rowstat[((int64_t)b * w.max_n + j) * 20 + slot], hcol[r][f]);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- Eq. 2 on int8 MFMA

typedef int32_t v4i __attribute__((ext_vector_type(4)));
typedef int32_t v16i __attribute__((ext_vector_type(16)));

constexpr int kKT = 128;          // K bytes per pipeline stage
constexpr int kLdsStride = 144;   // padded LDS row stride: 16 lanes of a ds_read_b128 hit distinct banks
constexpr int kLdsMat = kSc2Tile * kLdsStride;

// G[i][j] = C_ij * sum_k C_ik C_jk for i < j < n, over 128 x 128 output tiles
// with bi <= bj. C is symmetric, so the product is C C^T and both MFMA
// operands are rows of C read along k. 4 waves in a 2 x 2 layout each own a
// 64 x 64 sub-tile as 2 x 2 blocks of v_mfma_i32_32x32x32_i8 (int32 sums are
// exact: at most N - 2). Global -> LDS staging is double-buffered; work items
// are split into 8 contiguous ranges, one per XCD, so that tiles sharing rows
// of C share an L2.
__global__ void __launch_bounds__(256, 2) k_sc2(Work w)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[2][2][kLdsMat];
    const int total = w.plan->total[kSc2], B = w.plan->B;
    const int32_t *pre = w.pre + kSc2 * w.pre_stride;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, wm = wv >> 1, wn = wv & 1;
    const int xcd = blockIdx.x & 7, nx = (gridDim.x - xcd + 7) >> 3, lb = blockIdx.x >> 3;
    const int chunk = (total + 7) >> 3;
    const int end = min(total, (xcd + 1) * chunk);
    for (int item = xcd * chunk + lb; item < end; item += nx) {
        const int b = find_pair(pre, B, item);
        const PairDesc d = w.pairs[b];
        int bi, bj;
        tri_decode(item - pre[b], d.npad / kSc2Tile, bi, bj);
        const uint8_t *Cb = w.C + d.c_off;
        const int64_t npad = d.npad;
        const int nk = d.npad / kKT;
        // global load slots: 8 x 16 B per thread, A rows then B rows, 8 lanes per 128-byte row
        const uint8_t *gsrc[8];
        int ldsoff[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int idx = q * 256 + tid, mat = idx >> 10, r = (idx >> 3) & 127, ch = idx & 7;
            const int64_t row = (int64_t)(mat ? bj : bi) * kSc2Tile + r;
            gsrc[q] = Cb + row * npad + ch * 16;
            ldsoff[q] = mat * kLdsMat + r * kLdsStride + ch * 16;
        }
        v4i stage[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) stage[q] = *reinterpret_cast<const v4i *>(gsrc[q]);
#pragma unroll
        for (int q = 0; q < 8; ++q) *reinterpret_cast<v4i *>(&lds[0][0][0] + ldsoff[q]) = stage[q];
        __syncthreads();
        v16i acc[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[x][y] = (v16i){};
        const int arow = wm * 64 + (lane & 31), brow = wn * 64 + (lane & 31), koff = (lane >> 5) * 16;
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    stage[q] = *reinterpret_cast<const v4i *>(gsrc[q] + (int64_t)(kt + 1) * kKT);
            }
            const uint8_t *la = &lds[cur][0][0], *lbm = &lds[cur][1][0];
#pragma unroll
            for (int ks = 0; ks < kKT / 32; ++ks) {
                v4i fa[2], fb[2];
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    fa[x] = *reinterpret_cast<const v4i *>(la + (arow + 32 * x) * kLdsStride + ks * 32 + koff);
                    fb[x] = *reinterpret_cast<const v4i *>(lbm + (brow + 32 * x) * kLdsStride + ks * 32 + koff);
                }
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[x], fb[y], acc[x][y], 0, 0, 0);
            }
            if (kt + 1 < nk) {
#pragma unroll
                for (int q = 0; q < 8; ++q) *reinterpret_cast<v4i *>(&lds[cur ^ 1][0][0] + ldsoff[q]) = stage[q];
            }
            __syncthreads();
        }
        // epilogue: lane holds column (lane & 31) and rows 8*(r/4) + 4*(lane/32) + r%4 of each 32 x 32 block
        uint16_t *Gb = w.G + d.g_off;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t i = (int64_t)bi * kSc2Tile + wm * 64 + x * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int64_t j = (int64_t)bj * kSc2Tile + wn * 64 + y * 32 + (lane & 31);
                    if (i < j && j < d.n) {
                        const int32_t v = Cb[i * npad + j] ? acc[x][y][r] : 0;
                        Gb[i * npad + j] = (uint16_t)v;
                        if (w.learned && v > 0) {
                            int32_t *ri = w.rowstat + ((int64_t)b * w.max_n + i) * 20;
                            int32_t *rj = w.rowstat + ((int64_t)b * w.max_n + j) * 20;
                            atomicAdd(ri + 1, v);
                            atomicAdd(rj + 1, v);
                            atomicMax(ri + 2, v);
                            atomicMax(rj + 2, v);
                        }
                    }
                }
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

hipError_t launch_prep(const Work &w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_prep, dim3(grid), dim3(256), 0, s, w);
    return hipGetLastError();
}

hipError_t launch_compat(const Work &w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_compat, dim3(grid), dim3(256), 0, s, w);
    return hipGetLastError();
}

hipError_t launch_sc2(const Work &w, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_sc2, dim3(grid), dim3(256), 0, s, w);
    return hipGetLastError();
}

}  // namespace tr
