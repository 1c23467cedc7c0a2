// Learned pivot scorer on gfx950: per-match features, a 19 -> 64 -> 64 -> 1
// GELU MLP with bfloat16 weights and activations and float32 accumulation,
// the learned pivot reorder with plain SC2 order as fallback, and the
// training kernels (forward/backward, weight-gradient reduction, Adam).
#include <vector>

#include "mlp.h"

namespace tr {
namespace {

constexpr float kGeluC = 0.7978845608028654f;   // sqrt(2/pi)

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);   // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bfround(float f) { return bf2f(f2bf(f)); }

// tanh-form GELU (Hendrycks & Gimpel 2016) and its derivative.
__device__ __forceinline__ float gelu(float x)
{
    return 0.5f * x * (1.0f + tanhf(kGeluC * (x + 0.044715f * x * x * x)));
}

__device__ __forceinline__ float gelu_grad(float x)
{
    const float th = tanhf(kGeluC * (x + 0.044715f * x * x * x));
    return 0.5f * (1.0f + th) + 0.5f * x * (1.0f - th * th) * kGeluC * (1.0f + 3.0f * 0.044715f * x * x);
}

// Parameters in LDS as float32: the weights are the bfloat16 copies, the biases the master values.
struct MlpLds {
    float p[TR_MLP_NPARAM];
};

__device__ void load_params(MlpLds &L, const uint16_t *wbf16, const float *w32)
{
    for (int k = threadIdx.x; k < TR_MLP_NPARAM; k += blockDim.x) {
        const bool bias = (k >= kB1 && k < kW2) || (k >= kB2 && k < kW3) || k == kB3;
        L.p[k] = bias ? w32[k] : bf2f(wbf16[k]);
    }
}

// Forward pass of one sample (inference): float32 accumulation, bfloat16
// activations. Layer 1 is fully unrolled so a1 stays in registers.
__device__ float forward(const MlpLds &L, const float (&x)[19])
{
    float a1[64];
#pragma unroll
    for (int o = 0; o < 64; ++o) {
        float acc = L.p[kB1 + o];
#pragma unroll
        for (int k = 0; k < 19; ++k) acc = __builtin_fmaf(L.p[kW1 + 19 * o + k], x[k], acc);
        a1[o] = bfround(gelu(acc));
    }
    float s = L.p[kB3];
#pragma unroll 2
    for (int o = 0; o < 64; ++o) {
        float acc = L.p[kB2 + o];
#pragma unroll
        for (int k = 0; k < 64; ++k) acc = __builtin_fmaf(L.p[kW2 + 64 * o + k], a1[k], acc);
        s = __builtin_fmaf(L.p[kW3 + o], bfround(gelu(acc)), s);
    }
    return s;
}

// ---------------------------------------------------------------- features

// 19 values per match from the integer accumulators (degree, SC2 row sum and
// max, 16-bin delta histogram): ratios formed in float64, rounded to float32,
// then to bfloat16.
__global__ void __launch_bounds__(256) k_features(Work w, uint16_t *packed)
{
    const int total = stage_total(w, kPrep);
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        int local;
        const int b = stage_pair(w, kPrep, item, local);
        const PairDesc d = pair_desc(w, b);
        const int i = local * kPrepRows + threadIdx.x;
        if (i >= d.n) continue;
        const int32_t *rs = w.rowstat + ((int64_t)b * w.max_n + i) * 20;
        const double n1 = (double)(d.n - 1), n = (double)d.n;
        uint16_t *f = packed ? packed + (int64_t)(d.pt_off + i) * 19 : w.feat + ((int64_t)b * w.max_n + i) * 19;
        f[0] = f2bf((float)((double)rs[0] / n1));
        f[1] = f2bf((float)((double)rs[1] / (n1 * n)));
        f[2] = f2bf((float)((double)rs[2] / n));
#pragma unroll
        for (int k = 0; k < 16; ++k) f[3 + k] = f2bf((float)((double)rs[3 + k] / n1));
    }
}

// ---------------------------------------------------------------- inference + reorder

__device__ __forceinline__ float lane_f(float v, int k)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}

// Sum over the 64 lanes (DPP), valid in every lane.
__device__ __forceinline__ int wave_total(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return __builtin_amdgcn_readlane(v, 63);
}

// The scorer's weights in LDS, unit-minor so that lane o of a wave reads
// unit o's weight for input k from consecutive words (no bank conflicts); rows
// padded to 65 words so that the staging writes, which follow the parameters'
// global (unit-major) order, fall in distinct banks too.
struct MlpWave {
    static constexpr int kPad = 65;
    float w1[19][kPad], w2[64][kPad], b1[64], b2[64], w3[64], b3;
    // Thread tid's share of the weights (coalesced loads of the parameter
    // vector), fetched into registers early and written to LDS later (put), so
    // that the global reads overlap other work.
    struct Share {
        float a[5], c[16], e[3], f;
    };
    __device__ static Share fetch(const uint16_t *wbf16, const float *w32, int tid)
    {
        Share r;
#pragma unroll
        for (int u = 0; u < 5; ++u) r.a[u] = tid + 256 * u < 19 * 64 ? bf2f(wbf16[kW1 + tid + 256 * u]) : 0.0f;
#pragma unroll
        for (int u = 0; u < 16; ++u) r.c[u] = bf2f(wbf16[kW2 + tid + 256 * u]);
        const int t = tid & 63;
        r.e[0] = w32[kB1 + t];
        r.e[1] = w32[kB2 + t];
        r.e[2] = bf2f(wbf16[kW3 + t]);
        r.f = w32[kB3];
        return r;
    }
    // By a whole 256-thread workgroup; the caller synchronises after.
    __device__ void put(const Share &r, int tid)
    {
#pragma unroll
        for (int u = 0; u < 5; ++u) {
            const int t = tid + 256 * u;   // W1[o][k], o = t / 19, k = t % 19
            if (t < 19 * 64) w1[t % 19][t / 19] = r.a[u];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int t = tid + 256 * u;   // W2[o][k], o = t / 64, k = t % 64
            w2[t & 63][t >> 6] = r.c[u];
        }
        if (tid < 64) {
            b1[tid] = r.e[0];
            b2[tid] = r.e[1];
            w3[tid] = r.e[2];
        }
        if (tid == 0) b3 = r.f;
    }
    // Score of one match by a whole wave: lane o computes hidden unit o, each
    // layer one multiply-add chain per lane over inputs broadcast from the
    // wave's LDS row x (64 floats), in the same order as the one-thread forward
    // pass. fb: lane k < 19 holds feature k (bfloat16 bits).
    __device__ float score(uint16_t fb, int lane, float *x) const
    {
        auto publish = [&](float v) {   // every lane's value to x, visible to the whole wave
            x[lane] = v;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };
        publish(lane < 19 ? bf2f(fb) : 0.0f);
        float acc = b1[lane];
#pragma unroll
        for (int k = 0; k < 19; ++k) acc = __builtin_fmaf(w1[k][lane], x[k], acc);
        const float a1 = bfround(gelu(acc));
        __builtin_amdgcn_wave_barrier();   // every lane has read the features
        publish(a1);
        acc = b2[lane];
#pragma unroll
        for (int k = 0; k < 64; ++k) acc = __builtin_fmaf(w2[k][lane], x[k], acc);
        const float a2 = bfround(gelu(acc));
        __builtin_amdgcn_wave_barrier();
        publish(a2);
        float s = b3;
#pragma unroll
        for (int o = 0; o < 64; ++o) s = __builtin_fmaf(w3[o], x[o], s);
        __builtin_amdgcn_wave_barrier();   // x is free for the wave's next row
        return s;
    }
};

// Feature k of a match from its integer accumulator v, as k_features.
__device__ __forceinline__ uint16_t feature_bits(int32_t v, int k, int n)
{
    const double n1 = (double)(n - 1), nn = (double)n;
    return f2bf((float)((double)v / (k == 0 ? n1 : k == 1 ? n1 * nn : k == 2 ? nn : n1)));
}

constexpr int kCandRows = 4;   // rows evaluated together against each loaded point

// Pool entry r moves to slot rk (kept if rk < K1); slots past the pair's K pivots are empty.
__device__ __forceinline__ void place_pivot(const Work &w, int b, int K, int p, uint64_t mine, int rk)
{
    const int32_t *pl = w.pivots_plain + (int64_t)b * w.pool_cap * 3;
    int32_t *out = w.pivots + (int64_t)b * w.piv_stride * 3;
    if (p < K && rk < w.k1) {
        const int r = (int)(uint32_t)mine;
        out[3 * rk] = pl[3 * r];
        out[3 * rk + 1] = pl[3 * r + 1];
        out[3 * rk + 2] = pl[3 * r + 2];
    }
    if (p >= K && p < w.k1) {
        out[3 * p] = -1;
        out[3 * p + 1] = -1;
        out[3 * p + 2] = 0;
    }
}

// Features and score of every match the reorder needs: the endpoints of the
// pair's plain pivot pool. The endpoints are cut into chunks of R (at most
// kCandRows); wave 0 claims each distinct row of its chunk by compare-and-swap
// on the row's mark, so every row is evaluated once. The workgroup then reads
// each of the pair's points once and evaluates delta_ij against all claimed
// rows, exactly as the compatibility kernel does (same operation order,
// correctly rounded square roots), counting the degree and the 16-bin delta
// histogram; the SC2 row sum and maximum come from the SC2 epilogue (loaded at
// the claim, in flight during the point loop). Each wave then scores the rows
// of its slot. Matches outside the pool get no features and no score.
//
__global__ void __launch_bounds__(256) k_cand_rows(Work w, int B, int R, const uint16_t *wbf16, const float *w32)
{
    __shared__ float crd[kCandRows][6];
    __shared__ int32_t row_l[kCandRows], rsv_l[kCandRows][2];
    __shared__ int32_t cnt_l;
    __shared__ int32_t red[4][kCandRows][9];
    __shared__ MlpWave mlp;
    __shared__ float act_l[4][64];   // per-wave broadcast row of the scorer
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    {   // the weights go to LDS while the first chunk's loads are in flight (first barrier below)
        const MlpWave::Share share = MlpWave::fetch(wbf16, w32, tid);
        mlp.put(share, tid);
    }
    const float tau = w.tau, q = tau * 0.25f;
    float edge[16];
#pragma unroll
    for (int k = 1; k < 16; ++k) edge[k] = (float)k * q;   // bin edges as the compatibility kernel forms them
    // Fast bin decision: t = delta / q in float32 is within 2^-22 t of the quotient and v_sqrt_f32
    // moves delta by at most 2^-21 (|x| + |y|); away from every edge by the guard band
    // 2^-19 (|x| + |y|) + 2e-6 + 2^-17 q, floor(t) is the bin and delta <= tau is decided.
    const float inv_q = 1.0f / q, guard0 = __builtin_fmaf(q, 0x1p-17f, 2e-6f);
    const int cpp = (2 * w.pool + R - 1) / R, total = B * cpp;
    for (int c = blockIdx.x; c < total; c += gridDim.x) {
        const int slot = c / cpp, b = batch_pair(w, slot), e0 = (c - slot * cpp) * R;
        const PairDesc d = pair_desc(w, b);
        if (e0 < 2 * d.kpiv) {   // the same for the whole workgroup
            // Two batches of kU points per thread are in flight before the rows are claimed
            // (N <= 4096 takes one round trip); later batches are fetched into the buffer
            // just consumed while the other one is evaluated.
            constexpr int kU = 8;
            float pa[kU][6], pb[kU][6];
            auto fetch_points = [&](float (&p)[kU][6], int j0) {
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int64_t gj = d.pt_off + min(j0 + 256 * u, d.n - 1);
                    const float3 a = *reinterpret_cast<const float3 *>(w.src + 3 * gj);   // one 12-byte load
                    const float3 cc = *reinterpret_cast<const float3 *>(w.dst + 3 * gj);
                    p[u][0] = a.x; p[u][1] = a.y; p[u][2] = a.z;
                    p[u][3] = cc.x; p[u][4] = cc.y; p[u][5] = cc.z;
                }
            };
            fetch_points(pa, tid);
            if (256 * kU < d.n) fetch_points(pb, tid + 256 * kU);
            int rsum = 0, rmax = 0, pos = -1;   // wave 0: the SC2 row statistics of its claimed row
            if (wv == 0) {
                const int e = e0 + lane;
                int i = -1;
                if (lane < R && e < 2 * d.kpiv) {
                    i = w.pivots_plain[((int64_t)b * w.pool_cap + (e >> 1)) * 3 + (e & 1)];
                    if (i < 0 || i >= d.n || atomicCAS(&w.mark[(int64_t)b * w.max_n + i], 0, 1) != 0) i = -1;
                }
                const uint64_t m = __ballot(i >= 0);
                if (i >= 0) {
                    pos = __popcll(m & ((1ull << lane) - 1ull));
                    const int64_t gi = d.pt_off + i;
                    const int32_t *rs = w.rowstat + ((int64_t)b * w.max_n + i) * 20;
                    rsum = rs[1];
                    rmax = rs[2];
                    row_l[pos] = i;
                    crd[pos][0] = w.src[3 * gi]; crd[pos][1] = w.src[3 * gi + 1]; crd[pos][2] = w.src[3 * gi + 2];
                    crd[pos][3] = w.dst[3 * gi]; crd[pos][4] = w.dst[3 * gi + 1]; crd[pos][5] = w.dst[3 * gi + 2];
                }
                if (lane == 0) cnt_l = __popcll(m);
            }
            __syncthreads();
            const int cnt = cnt_l;
            if (cnt > 0) {   // the same for the whole workgroup
                uint32_t cw[kCandRows][4];   // 16 bins, 8 bits each (at most ceil(32767/256) per thread)
                int deg[kCandRows];
#pragma unroll
                for (int r = 0; r < kCandRows; ++r) {
                    deg[r] = 0;
                    cw[r][0] = cw[r][1] = cw[r][2] = cw[r][3] = 0;
                }
                auto eval_points = [&](float (&p)[kU][6], int j0) {
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const int j = j0 + 256 * u;
#pragma unroll
                        for (int r = 0; r < kCandRows; ++r) {
                            if (r >= cnt) break;
                            // hardware square roots first; a pair whose delta lies within the guard
                            // band of a bin edge k q (tau = 4 q is edge 4) is evaluated again with
                            // the correctly rounded ones, so every decision is the exact one
                            const float ax = crd[r][0] - p[u][0], ay = crd[r][1] - p[u][1], az = crd[r][2] - p[u][2];
                            const float bx = crd[r][3] - p[u][3], by = crd[r][4] - p[u][4], bz = crd[r][5] - p[u][5];
                            float s1 = ax * ax, s2 = bx * bx;
                            s1 = __builtin_fmaf(ay, ay, s1);
                            s2 = __builtin_fmaf(by, by, s2);
                            s1 = __builtin_fmaf(az, az, s1);
                            s2 = __builtin_fmaf(bz, bz, s2);
                            const float la = __builtin_amdgcn_sqrtf(s1), lb = __builtin_amdgcn_sqrtf(s2);
                            float dl = __builtin_fabsf(la - lb);
                            const float t = dl * inv_q;
                            const float kn = __builtin_fminf(__builtin_fmaxf(__builtin_rintf(t), 1.0f), 15.0f);
                            const float guard = __builtin_fmaf(la + lb, 0x1p-19f, guard0);
                            int bin;
                            if (__builtin_fabsf(dl - kn * q) <= guard || !(dl == dl)) {
                                const float lx = length32(ax, ay, az), ly = length32(bx, by, bz);
                                dl = __builtin_fabsf(lx - ly);
                                bin = 0;
#pragma unroll
                                for (int k = 1; k < 16; ++k) bin += dl >= edge[k];
                            } else {
                                bin = (int)__builtin_fminf(t, 15.0f);   // t >= 0, at least the guard from an integer
                            }
                            const bool in = j < d.n && j != row_l[r];
                            deg[r] += in && dl <= tau;
                            const uint32_t inc = in ? 1u << (8 * (bin & 3)) : 0u;
                            cw[r][0] += (bin >> 2) == 0 ? inc : 0u;
                            cw[r][1] += (bin >> 2) == 1 ? inc : 0u;
                            cw[r][2] += (bin >> 2) == 2 ? inc : 0u;
                            cw[r][3] += (bin >> 2) == 3 ? inc : 0u;
                        }
                    }
                };
                for (int j0 = tid; j0 < d.n; j0 += 2 * 256 * kU) {
                    eval_points(pa, j0);
                    if (j0 + 2 * 256 * kU < d.n) fetch_points(pa, j0 + 2 * 256 * kU);
                    if (j0 + 256 * kU < d.n) eval_points(pb, j0 + 256 * kU);
                    if (j0 + 3 * 256 * kU < d.n) fetch_points(pb, j0 + 3 * 256 * kU);
                }
                // Per row: bytes 0,2 and 1,3 of each counter word widen to 16-bit
                // fields (a workgroup's count of one bin is below 2^15).
#pragma unroll
                for (int r = 0; r < kCandRows; ++r) {
                    if (r >= cnt) break;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int te = wave_total((int)(cw[r][m] & 0x00FF00FFu));
                        const int to = wave_total((int)((cw[r][m] >> 8) & 0x00FF00FFu));
                        if (lane == 0) {
                            red[wv][r][2 * m] = te;
                            red[wv][r][2 * m + 1] = to;
                        }
                    }
                    const int td = wave_total(deg[r]);
                    if (lane == 0) red[wv][r][8] = td;
                }
                if (pos >= 0) {
                    rsv_l[pos][0] = rsum;
                    rsv_l[pos][1] = rmax;
                }
                __syncthreads();
#pragma unroll 1
                for (int r = wv; r < cnt; r += 4) {
                    const int i = row_l[r];
                    int32_t *rs = w.rowstat + ((int64_t)b * w.max_n + i) * 20;
                    int32_t v = 0;
                    if (lane == 0) {
                        v = red[0][r][8] + red[1][r][8] + red[2][r][8] + red[3][r][8];
                    } else if (lane < 3) {
                        v = rsv_l[r][lane - 1];   // SC2 row sum / maximum
                    } else if (lane < 19) {
                        const int bin = lane - 3, idx = 2 * (bin >> 2) + (bin & 1), sh = 16 * ((bin >> 1) & 1);
#pragma unroll
                        for (int g = 0; g < 4; ++g) v += (red[g][r][idx] >> sh) & 0xFFFF;
                    }
                    uint16_t fb = 0;
                    if (lane < 19) {
                        if (lane == 0 || lane >= 3) rs[lane] = v;
                        fb = feature_bits(v, lane, d.n);
                        w.feat[((int64_t)b * w.max_n + i) * 19 + lane] = fb;
                    }
                    const float sc = mlp.score(fb, lane, act_l[wv]);
                    if (lane == 0) {
                        w.scores[(int64_t)b * w.max_n + i] = sc;
                        if (!isfinite(sc)) atomicOr(&w.state[b].fallback, 1);
                    }
                }
            }
        }
        __syncthreads();   // row_l, crd, red, rsv_l and cnt_l are the next chunk's
    }
}

// Order the pool of plain pivots by e = s_i + s_j (desc), ties by plain rank,
// keep the first K1. Non-finite scores anywhere in the pair: keep plain order.
// Keys are distinct (the plain rank is part of each), so a key's new position
// is the number of smaller keys: each 256-thread workgroup rebuilds the
// pair's K keys in LDS and ranks 64 of them, a quarter of the list per wave,
// eight 16-byte broadcast reads in flight. (Pools larger than kFusedPool; the hypothesis
// kernel orders smaller ones.)
__global__ void __launch_bounds__(256) k_reorder(Work w, int blocks_per_pair)
{
    extern __shared__ uint64_t keys[];
    __shared__ int32_t part[4][64];
    const int slot = blockIdx.x / blocks_per_pair, b = batch_pair(w, slot), g = blockIdx.x - slot * blocks_per_pair;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const PairDesc d = pair_desc(w, b);
    const int K = d.kpiv;
    if (g * 64 >= max(K, w.k1)) return;
    const bool fb = w.state[b].fallback != 0;
    const int32_t *pl = w.pivots_plain + (int64_t)b * w.pool_cap * 3;
    const float *sc = w.scores + (int64_t)b * w.max_n;
    const int K16 = (K + 15) & ~15;
    for (int r = tid; r < K16; r += 256) keys[r] = r < K ? reorder_key(pl, sc, r, fb) : ~0ull;
    __syncthreads();
    const int p = g * 64 + lane;
    const uint64_t mine = p < K ? keys[p] : 0;
    const int per = ((K16 / 16 + 3) / 4) * 16;
    const int q0 = min(K16, wv * per), q1 = min(K16, q0 + per);
    part[wv][lane] = count_smaller(keys, q0, q1, mine);
    __syncthreads();
    if (wv != 0) return;
    const int rk = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
    place_pivot(w, b, K, p, mine, rk);
}

// ---------------------------------------------------------------- standalone forward

__global__ void __launch_bounds__(256) k_mlp_forward(const uint16_t *feat, int64_t m, float *scores,
                                                     const uint16_t *wbf16, const float *w32)
{
    __shared__ MlpLds L;
    load_params(L, wbf16, w32);
    __syncthreads();
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < m; n += (int64_t)gridDim.x * 256) {
        float x[19];
#pragma unroll
        for (int k = 0; k < 19; ++k) x[k] = bf2f(feat[n * 19 + k]);
        scores[n] = forward(L, x);
    }
}

// ---------------------------------------------------------------- training

// Scratch of a training step, for m samples rounded up to whole tiles (mp): A1, A2, D1, D2
// (64 floats per sample each, tile-major as Scratch::at places them), then DS[mp] and LS[mp].
constexpr int kTile = 256;   // samples per weight-gradient work item
constexpr int kSub = 32;     // samples staged in LDS at a time
constexpr int kSubPad = kSub + 1;   // LDS row stride: the rows a wave reads at one sample fall in distinct banks

// Per-sample rows of the backward pass, tile-major: the 64 entries of sample n in one of the four
// arrays are at at(f, n), f < 64, so the kTile samples of a weight-gradient work item occupy one
// contiguous block of 64 x kTile floats per array (consecutive samples stay consecutive).
struct Scratch {
    float *a1, *a2, *d1, *d2, *ds, *ls;
    __device__ __forceinline__ int64_t at(int f, int64_t n) const
    {
        return (n / kTile) * (64 * kTile) + f * kTile + n % kTile;
    }
};

// Samples the scratch holds for m: whole tiles.
__host__ __device__ __forceinline__ int64_t scratch_samples(int64_t m) { return (m + kTile - 1) / kTile * kTile; }

__device__ __forceinline__ Scratch scratch_view(float *base, int64_t m)
{
    const int64_t mp = scratch_samples(m);
    Scratch s;
    s.a1 = base;
    s.a2 = base + 64 * mp;
    s.d1 = base + 128 * mp;
    s.d2 = base + 192 * mp;
    s.ds = base + 256 * mp;
    s.ls = base + 257 * mp;
    return s;
}

// Per sample: forward (bfloat16 activations), BCE-with-logits loss and the
// deltas of the backward pass. ds is already divided by m (mean loss).
__global__ void __launch_bounds__(256) k_mlp_fwdbwd(const uint16_t *feat, const uint8_t *labels, int64_t m,
                                                    float *scratch, const uint16_t *wbf16, const float *w32)
{
    __shared__ MlpLds L;
    load_params(L, wbf16, w32);
    __syncthreads();
    const Scratch S = scratch_view(scratch, m);
    const float inv_m = 1.0f / (float)m;
    for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < m; n += (int64_t)gridDim.x * 256) {
        float x[19];
#pragma unroll
        for (int k = 0; k < 19; ++k) x[k] = bf2f(feat[n * 19 + k]);
        // forward; gelu'(z1) and gelu'(z2) are parked in the D1 / D2 slots
        float a1[64];
#pragma unroll
        for (int o = 0; o < 64; ++o) {
            float acc = L.p[kB1 + o];
#pragma unroll
            for (int k = 0; k < 19; ++k) acc = __builtin_fmaf(L.p[kW1 + 19 * o + k], x[k], acc);
            a1[o] = bfround(gelu(acc));
            S.d1[S.at(o, n)] = gelu_grad(acc);
        }
        float s = L.p[kB3];
#pragma unroll 2
        for (int o = 0; o < 64; ++o) {
            float acc = L.p[kB2 + o];
#pragma unroll
            for (int k = 0; k < 64; ++k) acc = __builtin_fmaf(L.p[kW2 + 64 * o + k], a1[k], acc);
            const float a = bfround(gelu(acc));
            S.a2[S.at(o, n)] = a;
            S.d2[S.at(o, n)] = gelu_grad(acc);
            s = __builtin_fmaf(L.p[kW3 + o], a, s);
        }
#pragma unroll
        for (int o = 0; o < 64; ++o) S.a1[S.at(o, n)] = a1[o];
        // loss and backward
        const float y = labels[n] ? 1.0f : 0.0f;
        const float loss = fmaxf(s, 0.0f) - s * y + log1pf(expf(-fabsf(s)));
        const float ds = (1.0f / (1.0f + expf(-s)) - y) * inv_m;
        float d2[64];
#pragma unroll
        for (int o = 0; o < 64; ++o) {
            d2[o] = ds * L.p[kW3 + o] * S.d2[S.at(o, n)];
            S.d2[S.at(o, n)] = d2[o];
        }
#pragma unroll 2
        for (int k = 0; k < 64; ++k) {
            float acc = 0.0f;
#pragma unroll
            for (int o = 0; o < 64; ++o) acc = __builtin_fmaf(L.p[kW2 + 64 * o + k], d2[o], acc);
            S.d1[S.at(k, n)] = acc * S.d1[S.at(k, n)];
        }
        S.ds[n] = ds;
        S.ls[n] = loss * inv_m;
    }
}

typedef float v16f __attribute__((ext_vector_type(16)));

// Partial sums over one tile of samples of every gradient (and the loss).
// The weight gradients are contractions over the samples: dW2 = D2^T A1 and
// dW1 = D1^T X on float32 MFMA (32 x 32 x 2, float32 products and sums): wave
// w owns the 32 x 32 block (w / 2, w % 2) of dW2, waves 0 and 1 also the rows
// 32 w .. 32 w + 31 of dW1 (19 of 32 columns used). Thread t also sums one of
// the vectors (db1, db2, dW3, db3, loss) in sample order.
__global__ void __launch_bounds__(256) k_mlp_wgrad(const uint16_t *feat, int64_t m, const float *scratch,
                                                   float *partial)
{
    __shared__ float sa1[64][kSubPad], sa2[64][kSubPad], sd1[64][kSubPad], sd2[64][kSubPad], sx[19][kSubPad], sds[kSub],
        sls[kSub];
    const Scratch S = scratch_view(const_cast<float *>(scratch), m);
    const int t = threadIdx.x, w = t >> 6, li = t & 31, lk = (t >> 5) & 1;
    const int ob = w >> 1, kb = w & 1;   // this wave's dW2 block: rows 32 ob.., columns 32 kb..
    const int64_t n0 = (int64_t)blockIdx.x * kTile;
    v16f acc2 = {}, acc1 = {};
    float gv = 0.0f;
    // staging: thread t moves entries idx = t + 256 u (u < kStageIt) of each kSub-sample block,
    // row f = idx / kSub, sample c = idx % kSub; a block's loads are all issued into registers
    // before any is used, and the next block's while the current one is summed
    constexpr int kStageIt = 64 * kSub / 256;
    float va1[kStageIt], va2[kStageIt], vd1[kStageIt], vd2[kStageIt], vx[kStageIt], vq = 0.0f;
    auto fetch = [&](int sub) {
#pragma unroll
        for (int u = 0; u < kStageIt; ++u) {
            const int idx = t + 256 * u, f = idx / kSub, c = idx % kSub;
            const int64_t n = n0 + sub + c;
            const bool ok = n < m;
            va1[u] = ok ? S.a1[S.at(f, n)] : 0.0f;
            va2[u] = ok ? S.a2[S.at(f, n)] : 0.0f;
            vd1[u] = ok ? S.d1[S.at(f, n)] : 0.0f;
            vd2[u] = ok ? S.d2[S.at(f, n)] : 0.0f;
            vx[u] = ok && f < 19 ? bf2f(feat[n * 19 + f]) : 0.0f;
            if (f == 19) vq = ok ? S.ds[n] : 0.0f;   // rows 19 and 20 (delta, loss) fall to different threads
            if (f == 20) vq = ok ? S.ls[n] : 0.0f;
        }
    };
    fetch(0);
    for (int sub = 0; sub < kTile; sub += kSub) {
#pragma unroll
        for (int u = 0; u < kStageIt; ++u) {
            const int idx = t + 256 * u, f = idx / kSub, c = idx % kSub;
            sa1[f][c] = va1[u];
            sa2[f][c] = va2[u];
            sd1[f][c] = vd1[u];
            sd2[f][c] = vd2[u];
            if (f < 19) sx[f][c] = vx[u];
            if (f == 19) sds[c] = vq;
            if (f == 20) sls[c] = vq;
        }
        __syncthreads();
        if (sub + kSub < kTile) fetch(sub + kSub);
        // two samples per MFMA: lane (li, lk) supplies row li of the A block and column li of the
        // B block at sample c0 + lk
#pragma unroll
        for (int c0 = 0; c0 < kSub; c0 += 2) {
            acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(sd2[32 * ob + li][c0 + lk], sa1[32 * kb + li][c0 + lk], acc2, 0,
                                                        0, 0);
            if (w < 2)
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(sd1[32 * w + li][c0 + lk], li < 19 ? sx[li][c0 + lk] : 0.0f,
                                                            acc1, 0, 0, 0);
        }
        // the vector sums, one per thread, over the block's samples in order (the branch is taken
        // once per block, so each thread's reads are issued together)
        if (t < 64) {
#pragma unroll
            for (int c = 0; c < kSub; ++c) gv += sd1[t][c];
        } else if (t < 128) {
#pragma unroll
            for (int c = 0; c < kSub; ++c) gv += sd2[t - 64][c];
        } else if (t < 192) {
#pragma unroll
            for (int c = 0; c < kSub; ++c) gv = __builtin_fmaf(sds[c], sa2[t - 128][c], gv);
        } else if (t == 192) {
#pragma unroll
            for (int c = 0; c < kSub; ++c) gv += sds[c];
        } else if (t == 193) {
#pragma unroll
            for (int c = 0; c < kSub; ++c) gv += sls[c];
        }
        __syncthreads();
    }
    float *out = partial + (int64_t)blockIdx.x * kGradSlots;
    // block entry (i, j) of register r in lane (li, lk): i = 8 (r / 4) + 4 lk + r % 4, j = li
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int i = 8 * (r >> 2) + 4 * lk + (r & 3);
        out[kW2 + 64 * (32 * ob + i) + 32 * kb + li] = acc2[r];
        if (w < 2 && li < 19) out[kW1 + 19 * (32 * w + i) + li] = acc1[r];
    }
    if (t < 64) out[kB1 + t] = gv;
    else if (t < 128) out[kB2 + t - 64] = gv;
    else if (t < 192) out[kW3 + t - 128] = gv;
    else if (t == 192) out[kB3] = gv;
    else if (t == 193) out[TR_MLP_NPARAM] = gv;
}

// Sum the tiles' partials in tile order (deterministic); the loads of kReduceBatch tiles are
// issued together, then added one after another.
constexpr int kReduceBatch = 32;
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *partial, int64_t tiles, float *grads, float *loss)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kGradSlots) return;
    float acc = 0.0f;
    for (int64_t t0 = 0; t0 < tiles; t0 += kReduceBatch) {
        float v[kReduceBatch];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) v[u] = t0 + u < tiles ? partial[(t0 + u) * kGradSlots + p] : 0.0f;
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u)
            if (t0 + u < tiles) acc += v[u];
    }
    if (p < TR_MLP_NPARAM) grads[p] = acc;
    else if (loss) *loss = acc;
}

__global__ void __launch_bounds__(256) k_adam(float *w, float *mo, float *ve, uint16_t *wbf16, const float *g,
                                              float lr, float c1, float c2)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= TR_MLP_NPARAM) return;
    const float gp = g[p];
    const float m = 0.9f * mo[p] + 0.1f * gp;
    const float v = 0.999f * ve[p] + 0.001f * gp * gp;
    mo[p] = m;
    ve[p] = v;
    const float nw = w[p] - lr * (m / c1) / (sqrtf(v / c2) + 1e-8f);
    w[p] = nw;
    wbf16[p] = f2bf(nw);
}

__global__ void k_to_bf16(const float *w, uint16_t *wbf16, int n)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < n) wbf16[p] = f2bf(w[p]);
}

int grid_for(int64_t m)
{
    const int64_t g = (m + 255) / 256;
    return (int)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}

hipError_t ensure_scratch(MlpState *s, int64_t m)
{
    if (s->scratch_m < m) {
        if (s->scratch) hipFree(s->scratch);
        s->scratch = nullptr;
        s->scratch_m = 0;
        hipError_t e = hipMalloc(&s->scratch, sizeof(float) * 258 * (size_t)scratch_samples(m));
        if (e != hipSuccess) return e;
        s->scratch_m = m;
    }
    const int64_t tiles = (m + kTile - 1) / kTile;
    if (s->partial_tiles < tiles) {
        if (s->partial) hipFree(s->partial);
        s->partial = nullptr;
        s->partial_tiles = 0;
        hipError_t e = hipMalloc(&s->partial, sizeof(float) * kGradSlots * (size_t)tiles);
        if (e != hipSuccess) return e;
        s->partial_tiles = tiles;
    }
    return hipSuccess;
}

}  // namespace

hipError_t setup_mlp_kernels()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(k_reorder), hipFuncAttributeMaxDynamicSharedMemorySize,
                               TR_MAX_POOL * (int)sizeof(uint64_t));
}

hipError_t mlp_create(MlpState *s)
{
    hipError_t e = hipMalloc(&s->w32, sizeof(float) * TR_MLP_NPARAM);
    if (e == hipSuccess) e = hipMalloc(&s->m, sizeof(float) * TR_MLP_NPARAM);
    if (e == hipSuccess) e = hipMalloc(&s->v, sizeof(float) * TR_MLP_NPARAM);
    if (e == hipSuccess) e = hipMalloc(&s->wbf16, sizeof(uint16_t) * TR_MLP_NPARAM);
    if (e == hipSuccess) e = hipMalloc(&s->grads, sizeof(float) * kGradSlots);
    return e;
}

void mlp_release(MlpState *s)
{
    for (void *p : {(void *)s->w32, (void *)s->m, (void *)s->v, (void *)s->wbf16, (void *)s->grads,
                    (void *)s->scratch, (void *)s->partial})
        if (p) hipFree(p);
    *s = MlpState();
}

hipError_t mlp_set(MlpState *s, const float *host)
{
    std::vector<float> zero(TR_MLP_NPARAM, 0.0f);
    hipError_t e = hipMemcpy(s->w32, host, sizeof(float) * TR_MLP_NPARAM, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->m, zero.data(), sizeof(float) * TR_MLP_NPARAM, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->v, zero.data(), sizeof(float) * TR_MLP_NPARAM, hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_to_bf16, dim3((TR_MLP_NPARAM + 255) / 256), dim3(256), 0, 0, s->w32, s->wbf16, TR_MLP_NPARAM);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    s->step = 0;
    return e;
}

hipError_t mlp_get(MlpState *s, float *host)
{
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    return hipMemcpy(host, s->w32, sizeof(float) * TR_MLP_NPARAM, hipMemcpyDeviceToHost);
}

hipError_t mlp_forward(MlpState *s, const uint16_t *feat, int64_t m, float *scores, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid_for(m)), dim3(256), 0, st, feat, m, scores, s->wbf16, s->w32);
    return hipGetLastError();
}

hipError_t mlp_grads(MlpState *s, const uint16_t *feat, const uint8_t *labels, int64_t m, float *grads, float *loss,
                     hipStream_t st)
{
    hipError_t e = ensure_scratch(s, m);
    if (e != hipSuccess) return e;
    const int64_t tiles = (m + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3(grid_for(m)), dim3(256), 0, st, feat, labels, m, s->scratch, s->wbf16,
                       s->w32);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)tiles), dim3(256), 0, st, feat, m, s->scratch, s->partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kGradSlots + 255) / 256), dim3(256), 0, st, s->partial, tiles, grads, loss);
    return hipGetLastError();
}

hipError_t mlp_train_step(MlpState *s, const uint16_t *feat, const uint8_t *labels, int64_t m, float lr, float *loss,
                          hipStream_t st)
{
    hipError_t e = mlp_grads(s, feat, labels, m, s->grads, loss, st);
    if (e != hipSuccess) return e;
    s->step += 1;
    // bias corrections 1 - beta^t in float64: in float32, 1 - 0.999^t loses ~3e-5 relative to
    // cancellation at small t, which would move every early step by as much
    const float c1 = (float)(1.0 - pow(0.9, (double)s->step)), c2 = (float)(1.0 - pow(0.999, (double)s->step));
    hipLaunchKernelGGL(k_adam, dim3((TR_MLP_NPARAM + 255) / 256), dim3(256), 0, st, s->w32, s->m, s->v, s->wbf16,
                       s->grads, lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_features(const Work &w, uint16_t *packed, int grid, hipStream_t st)
{
    hipLaunchKernelGGL(k_features, dim3(grid), dim3(256), 0, st, w, packed);
    return hipGetLastError();
}

hipError_t launch_learned_order(const Work &w, const MlpState &mlp, int B, int grid, hipStream_t st)
{
    // Rows per chunk: few enough chunks that all run at once (two workgroups
    // per CU fit), at most kCandRows rows each.
    const int cand = B * 2 * w.pool;
    const int R = max(1, min(kCandRows, (cand + 2 * grid - 1) / (2 * grid)));
    const int chunks = B * ((2 * w.pool + R - 1) / R);
    hipLaunchKernelGGL(k_cand_rows, dim3(min(chunks, grid * 2)), dim3(256), 0, st, w, B, R, mlp.wbf16, mlp.w32);
    if (!w.rank_in_hyp) {   // small pools are ordered by the hypothesis kernel itself
        const int bpp = (max(w.pool, w.k1) + 63) / 64;
        hipLaunchKernelGGL(k_reorder, dim3(B * bpp), dim3(256), (size_t)((w.pool + 15) & ~15) * sizeof(uint64_t), st,
                           w, bpp);
    }
    return hipGetLastError();
}

}  // namespace tr
