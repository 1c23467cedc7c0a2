// Hypothesis generation and scoring on gfx950: TurboClique search with
// top-K2 selection (Eqs. 5-8, Algorithms 1-2), one rigid fit per clique
// (Section 3.5), inlier numbers (Eq. 9) and the final argmax.
#include "common.h"

namespace tr {
namespace {

// ---------------------------------------------------------------- Section 3.5

// One Jacobi rotation of the symmetric 4x4 A (and the eigenvector matrix V)
// that zeroes A[p][q].
template <int p, int q>
__device__ __forceinline__ void jacobi_rot(double (&A)[4][4], double (&V)[4][4])
{
    const double apq = A[p][q];
    if (apq == 0.0) return;
    const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
    const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
    }
}

// 3x3 determinant of the 4x4 A with row R and column C removed.
template <int R, int C>
__device__ __forceinline__ double minor3(const double (&A)[4][4])
{
    constexpr int r0 = R == 0 ? 1 : 0, r1 = R <= 1 ? 2 : 1, r2 = R <= 2 ? 3 : 2;
    constexpr int c0 = C == 0 ? 1 : 0, c1 = C <= 1 ? 2 : 1, c2 = C <= 2 ? 3 : 2;
    return A[r0][c0] * (A[r1][c1] * A[r2][c2] - A[r1][c2] * A[r2][c1]) -
           A[r0][c1] * (A[r1][c0] * A[r2][c2] - A[r1][c2] * A[r2][c0]) +
           A[r0][c2] * (A[r1][c0] * A[r2][c1] - A[r1][c1] * A[r2][c0]);
}

// Column `col` of adj(A): entry r is (-1)^(r+col) times the minor of A without row col and column r.
template <int col>
__device__ __forceinline__ void adj_col(const double (&A)[4][4], double (&v)[4])
{
    v[0] = ((0 + col) & 1 ? -1.0 : 1.0) * minor3<col, 0>(A);
    v[1] = ((1 + col) & 1 ? -1.0 : 1.0) * minor3<col, 1>(A);
    v[2] = ((2 + col) & 1 ? -1.0 : 1.0) * minor3<col, 2>(A);
    v[3] = ((3 + col) & 1 ? -1.0 : 1.0) * minor3<col, 3>(A);
}

// Least-squares rotation of three matches by Horn's unit-quaternion method
// (J. Opt. Soc. Am. A 4(4), 1987): the rotation maximising sum (R p_a).q_a on
// centred points is the unit eigenvector of the largest eigenvalue of a
// traceless symmetric 4x4 matrix K built from M = sum p_a q_a^T.
//
// The eigenvalue is found as in the QCP method (Theobald, Acta Cryst. A 61,
// 2005; Liu, Agrafiotis & Theobald, J. Comput. Chem. 31, 2010): Newton's
// iteration on the characteristic polynomial
//   det(lambda I - K) = lambda^4 - tr(K^2)/2 lambda^2 - tr(K^3)/3 lambda + det K
// from E0 = (sum |p_a|^2 + sum |q_a|^2)/2, an upper bound of the root, until
// the step falls below 1e-15 relative or stops being positive. The
// eigenvector is the largest column of adj(K - lambda I). When the top
// eigenvalue is repeated or nearly so (collinear, nearly collinear or
// coincident points), where that column loses its accuracy, the cyclic Jacobi
// method on K decides instead. float64 throughout, then R and t
// are rounded to float32. An empty clique (z < 0) gives the identity and false.
__device__ bool fit_pose(const Work &w, const PairDesc &d, int ia, int ib, int ic, float (&pose)[12])
{
    {
        if (d.n == 0 || ic < 0) {
#pragma unroll
            for (int k = 0; k < 12; ++k) pose[k] = (k < 9 && k % 4 == 0) ? 1.0f : 0.0f;
            return false;
        }
        const int idx[3] = {ia, ib, ic};
        double P[3][3], Q[3][3], pb[3] = {0, 0, 0}, qb[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                P[a][k] = w.src[3 * (int64_t)(d.pt_off + idx[a]) + k];
                Q[a][k] = w.dst[3 * (int64_t)(d.pt_off + idx[a]) + k];
                pb[k] += P[a][k];
                qb[k] += Q[a][k];
            }
#pragma unroll
        for (int k = 0; k < 3; ++k) { pb[k] /= 3.0; qb[k] /= 3.0; }
        double M[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, E0 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                const double pr = P[a][r] - pb[r], qr = Q[a][r] - qb[r];
                E0 += 0.5 * (pr * pr + qr * qr);
#pragma unroll
                for (int s = 0; s < 3; ++s) M[r][s] += pr * (Q[a][s] - qb[s]);
            }
        const double Sxx = M[0][0], Sxy = M[0][1], Sxz = M[0][2], Syx = M[1][0], Syy = M[1][1], Syz = M[1][2],
                     Szx = M[2][0], Szy = M[2][1], Szz = M[2][2];
        double K[4][4] = {{Sxx + Syy + Szz, Syz - Szy, Szx - Sxz, Sxy - Syx},
                          {Syz - Szy, Sxx - Syy - Szz, Sxy + Syx, Szx + Sxz},
                          {Szx - Sxz, Sxy + Syx, -Sxx + Syy - Szz, Syz + Szy},
                          {Sxy - Syx, Szx + Sxz, Syz + Szy, -Sxx - Syy + Szz}};
        // characteristic polynomial: lambda^4 + c2 lambda^2 + c1 lambda + c0
        double K2[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                K2[r][s] = K[r][0] * K[0][s] + K[r][1] * K[1][s] + K[r][2] * K[2][s] + K[r][3] * K[3][s];
        double tr2 = 0, tr3 = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            tr2 += K2[r][r];
#pragma unroll
            for (int s = 0; s < 4; ++s) tr3 += K2[r][s] * K[s][r];
        }
        const double detK = K[0][0] * minor3<0, 0>(K) - K[0][1] * minor3<0, 1>(K) + K[0][2] * minor3<0, 2>(K) -
                            K[0][3] * minor3<0, 3>(K);
        const double c2 = -0.5 * tr2, c1 = -tr3 / 3.0, c0 = detK;
        double lam = E0;
        for (int it = 0; it < 60; ++it) {
            const double l2 = lam * lam;
            const double f = (l2 + c2) * l2 + c1 * lam + c0;
            const double fp = 2.0 * lam * (2.0 * l2 + c2) + c1;
            if (!(fp > 0.0)) break;
            const double step = f / fp;
            // from above the largest root the exact steps are positive and shrink: a step that is
            // not positive is rounding noise at the root (it would only oscillate there)
            if (!(step > 0.0)) break;
            lam -= step;
            if (step <= 1e-15 * fabs(lam)) break;
        }
        // eigenvector: the largest column of adj(K - lambda I)
        double A[4][4];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int s = 0; s < 4; ++s) A[r][s] = K[r][s] - (r == s ? lam : 0.0);
        double qv[4], best, cand[4], nn;
        adj_col<0>(A, qv);
        best = qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3];
        auto take = [&]() {
            nn = cand[0] * cand[0] + cand[1] * cand[1] + cand[2] * cand[2] + cand[3] * cand[3];
            if (nn > best) {
                best = nn;
#pragma unroll
                for (int r = 0; r < 4; ++r) qv[r] = cand[r];
            }
        };
        adj_col<1>(A, cand);
        take();
        adj_col<2>(A, cand);
        take();
        adj_col<3>(A, cand);
        take();
        // The adjugate column has norm between P/2 and P, P = prod_{k>1} (lambda_1 - lambda_k). K's
        // spectrum for three matches is +-(s1 + s2), +-(s1 - s2) (s1 >= s2 the singular values of
        // M), so P ~ 4 lambda^3 g with g the relative gap to the second eigenvalue. Near a double
        // root the Newton root carries an error ~ eps lambda / g and the adjugate vector one of
        // ~ eps / g^2 (3.6e-4 rad at g = 6e-7 on nearly collinear outdoor cliques); below
        // g ~ 1e-4 the Jacobi method decides, whose error is ~ eps / g.
        const double scale3 = E0 * E0 * E0, lam3 = lam * lam * lam;
        if (!(best > 1e-24 * scale3 * scale3) || !(best < 1e300) || !(best > 1.6e-7 * lam3 * lam3)) {
            // repeated or nearly repeated top eigenvalue (nearly collinear or coincident points,
            // or no spread at all): cyclic Jacobi on K
            double V[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
            double fro = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int s = 0; s < 4; ++s) fro += K[r][s] * K[r][s];
            for (int sweep = 0; sweep < 16; ++sweep) {
                const double off = K[0][1] * K[0][1] + K[0][2] * K[0][2] + K[0][3] * K[0][3] + K[1][2] * K[1][2] +
                                   K[1][3] * K[1][3] + K[2][3] * K[2][3];
                if (off <= 1e-30 * fro) break;
                jacobi_rot<0, 1>(K, V);
                jacobi_rot<0, 2>(K, V);
                jacobi_rot<0, 3>(K, V);
                jacobi_rot<1, 2>(K, V);
                jacobi_rot<1, 3>(K, V);
                jacobi_rot<2, 3>(K, V);
            }
            int bi = 0;
            double bv = K[0][0];
#pragma unroll
            for (int k = 1; k < 4; ++k)
                if (K[k][k] > bv) { bv = K[k][k]; bi = k; }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (bi == k) { qv[0] = V[0][k]; qv[1] = V[1][k]; qv[2] = V[2][k]; qv[3] = V[3][k]; }
        }
        const double nq = 1.0 / sqrt(qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2] + qv[3] * qv[3]);
        const double q0 = qv[0] * nq, qx = qv[1] * nq, qy = qv[2] * nq, qz = qv[3] * nq;
        const double R[9] = {q0 * q0 + qx * qx - qy * qy - qz * qz, 2 * (qx * qy - q0 * qz), 2 * (qx * qz + q0 * qy),
                             2 * (qy * qx + q0 * qz), q0 * q0 - qx * qx + qy * qy - qz * qz, 2 * (qy * qz - q0 * qx),
                             2 * (qz * qx - q0 * qy), 2 * (qz * qy + q0 * qx), q0 * q0 - qx * qx - qy * qy + qz * qz};
#pragma unroll
        for (int k = 0; k < 9; ++k) pose[k] = (float)R[k];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            pose[9 + r] = (float)(qb[r] - (R[3 * r] * pb[0] + R[3 * r + 1] * pb[1] + R[3 * r + 2] * pb[2]));
        return true;
    }
}

// ---------------------------------------------------------------- Eqs. 5-8

// Candidate key of a third vertex z: larger T = G(i,z) + G(j,z) first, then smaller z. The
// clique weight S = G(i,j) + T (Eq. 7) differs from T by the same G(i,j) for every z of a pivot,
// so T orders the candidates like S. Weights are below N <= 32767, so T < 2^16 and z < 2^15:
// key = T * 2^15 + (32767 - z) fits 31 bits, and 0 means "empty" (a candidate has T >= 2).
__device__ __forceinline__ uint32_t clique_key(uint32_t T, uint32_t z)
{
    return (T << 15) + (32767u - z);
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    return v;
}

template <int KMAX>
__device__ __forceinline__ void top_insert(uint32_t (&top)[KMAX], uint32_t k)
{
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        const uint32_t t = top[s];
        top[s] = max(t, k);
        k = min(t, k);
    }
}

// One wavefront per pivot (p of pair b). On the O2Graph each lane reads eight consecutive
// weights of rows i and j with one 16-byte load each (the wave covers 512
// third vertices per step, z > j only, and only the steps the row holds); on
// the undirected graph lanes stride over z and read the lower triangle through
// the transpose. Each lane keeps its KMAX best keys sorted in registers
// (max / min insertion, no dynamic register indexing); K2 rounds of a
// wave-wide max then pick the pivot's cliques in (S desc, z asc) order and
// write them (slot-major); lane s < K2 returns the third vertex of clique s
// (-1: none), pi / pj the pivot (-1 for an empty slot).
template <int KMAX>
__device__ int clique_search(const Work &w, const PairDesc &d, int b, int p, const int32_t *pv, int lane, int &pi,
                             int &pj)
{
    {
        int i = d.n > 0 ? pv[0] : -1, j = d.n > 0 ? pv[1] : -1;
        if (i < 0 || j < 0 || i >= d.n || j >= d.n || i == j) i = j = -1;   // an empty slot (or a bad index) finds no clique
        int32_t *cl = w.cliques + (int64_t)b * w.h_cap * 3;
        uint32_t top[KMAX];
#pragma unroll
        for (int s = 0; s < KMAX; ++s) top[s] = 0;
        if (i >= 0) {
            const uint16_t *G = w.G + d.g_off;
            const int64_t npad = d.npad;
            const int wij = i < j ? G[i * npad + j] : G[(int64_t)j * npad + i];
            if (w.graph == TR_GRAPH_O2) {
                const uint16_t *ri = G + i * npad, *rj = G + (int64_t)j * npad;
                const int c1 = (d.n + 7) >> 3;
                // sixteen chunks of each row per lane in flight (every z of a row up to N = 8192 at
                // once), issued together with w_ij
                for (int c0 = ((j + 1) >> 3); c0 < c1; c0 += 1024) {
                    uint4 qi[16], qj[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int c = c0 + 64 * u + lane;
                        qi[u] = c < c1 ? *reinterpret_cast<const uint4 *>(ri + 8 * c) : make_uint4(0, 0, 0, 0);
                        qj[u] = c < c1 ? *reinterpret_cast<const uint4 *>(rj + 8 * c) : make_uint4(0, 0, 0, 0);
                    }
                    if (wij == 0) continue;   // not an edge: no clique (Eq. 8)
                    const int steps = min(16, (c1 - c0 + 63) >> 6);   // the same on every lane
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        if (u >= steps) continue;   // uniform: the loop stays unrolled
                        const int c = c0 + 64 * u + lane;
                        // elements e of the chunk with j < 8c + e < n (none when c >= c1)
                        const int lo = min(max(j + 1 - 8 * c, 0), 8), hi = min(max(d.n - 8 * c, 0), 8);
                        const uint32_t vm = ((1u << hi) - 1u) & ~((1u << lo) - 1u);
                        const uint32_t zb = 32767u - 8u * (uint32_t)c;
                        const uint32_t ui[4] = {qi[u].x, qi[u].y, qi[u].z, qi[u].w};
                        const uint32_t uj[4] = {qj[u].x, qj[u].y, qj[u].z, qj[u].w};
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            // two weights per word; G(i,z) of elements outside the range masked to 0
                            const uint32_t mw = (((vm >> (2 * k)) & 1u) ? 0xFFFFu : 0u) |
                                                (((vm >> (2 * k + 1)) & 1u) ? 0xFFFF0000u : 0u);
                            const uint32_t a = ui[k] & mw, bj = uj[k];
                            const uint32_t t0 = (a & 0xFFFFu) + (bj & 0xFFFFu), t1 = (a >> 16) + (bj >> 16);
                            const bool e0 = (a & 0xFFFFu) != 0 && (bj & 0xFFFFu) != 0;
                            const bool e1 = (a >> 16) != 0 && (bj >> 16) != 0;
                            top_insert<KMAX>(top, e0 ? (t0 << 15) + (zb - 2 * k) : 0u);
                            top_insert<KMAX>(top, e1 ? (t1 << 15) + (zb - 2 * k - 1) : 0u);
                        }
                    }
                }
            } else if (wij > 0) {
                for (int z = lane; z < d.n; z += 64) {
                    if (z == i || z == j) continue;
                    const int giz = i < z ? G[i * npad + z] : G[(int64_t)z * npad + i];
                    const int gjz = j < z ? G[(int64_t)j * npad + z] : G[(int64_t)z * npad + j];
                    if (giz > 0 && gjz > 0) top_insert<KMAX>(top, clique_key((uint32_t)(giz + gjz), (uint32_t)z));
                }
            }
        }
        int zmine = -1;   // lane s < K2 keeps the third vertex of clique s
        for (int s = 0; s < w.k2; ++s) {
            const uint32_t best = wave_max_u32(top[0]);
            if (best != 0 && top[0] == best) {          // keys are unique per z: one owner
#pragma unroll
                for (int q = 0; q + 1 < KMAX; ++q) top[q] = top[q + 1];
                top[KMAX - 1] = 0;
            }
            const int z = best ? (int32_t)(32767u - (best & 0x7FFFu)) : -1;
            if (lane == s) zmine = z;
            if (lane == 0) {
                const int64_t h = (int64_t)s * w.k1 + p;
                cl[3 * h] = i;
                cl[3 * h + 1] = j;
                cl[3 * h + 2] = z;
            }
        }
        pi = i;
        pj = j;
        return zmine;
    }
}

// ---------------------------------------------------------------- Eq. 9

// Residual |R x + t - y|^2 in float32 with the pinned operation order: each
// component starts at t and adds the three products by fused multiply-adds;
// the squared norm rounds the first square and fuses the other two.
__device__ __forceinline__ float residual2(const float (&ps)[12], float x0, float x1, float x2, float y0, float y1,
                                           float y2)
{
    float u = ps[9];
    u = __builtin_fmaf(ps[0], x0, u);
    u = __builtin_fmaf(ps[1], x1, u);
    u = __builtin_fmaf(ps[2], x2, u);
    const float rx = u - y0;
    float v = ps[10];
    v = __builtin_fmaf(ps[3], x0, v);
    v = __builtin_fmaf(ps[4], x1, v);
    v = __builtin_fmaf(ps[5], x2, v);
    const float ry = v - y1;
    float z = ps[11];
    z = __builtin_fmaf(ps[6], x0, z);
    z = __builtin_fmaf(ps[7], x1, z);
    z = __builtin_fmaf(ps[8], x2, z);
    const float rz = z - y2;
    float s = rx * rx;
    s = __builtin_fmaf(ry, ry, s);
    s = __builtin_fmaf(rz, rz, s);
    return s;
}

// Inclusive prefix sum inside each 16-lane DPP row: the last lane of a row (16r + 15) holds its total.
__device__ __forceinline__ int row16_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    return v;
}

// Sum over the 64 lanes (DPP), returned to every lane.
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

// The pair's result once every hypothesis is scored: argmax of IN (lowest h
// on ties), the compatibility counts summed over the pair's tiles, the result
// record and the inlier mask under the selected pose. Run by one workgroup of
// NW waves (every thread calls it).
template <int NW>
__device__ void select_pair(const Work &w, int b, int ipp)
{
    constexpr int NT = 64 * NW;
    __shared__ uint64_t red_k[NW];
    __shared__ int32_t red_n[NW];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const uint64_t t_sel0 = w.hyp_prof ? __builtin_amdgcn_s_memrealtime() : 0;
    const PairDesc d = pair_desc(w, b);
    // the mask's first matches (kM per thread) do not depend on the selection: their loads are
    // issued before the records are read
    constexpr int kM = 12;
    const bool want_mask = w.masks && d.n > 0;
    float x[kM][3], y[kM][3];
    auto load_pts = [&](int k0) {
#pragma unroll
        for (int m = 0; m < kM; ++m) {
            const int64_t g = d.pt_off + min(k0 + NT * m, d.n - 1);
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                x[m][f] = w.src[3 * g + f];
                y[m][f] = w.dst[3 * g + f];
            }
        }
    };
    if (want_mask) load_pts(tid);
    const PairState st = w.state[b];
    // every work item of the pair left its best key and valid count in its record (device scope,
    // written by other workgroups of this launch); four records per thread are loaded at once
    const uint64_t *rec = w.hyp_rec + (int64_t)b * w.rec_stride;
    uint64_t best = 0;
    int nvalid = 0;
    for (int k0 = tid; k0 < ipp; k0 += 4 * NT) {
        uint64_t rk[4], rn[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + NT * u;
            rk[u] = k < ipp ? __hip_atomic_load(rec + 2 * k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
            rn[u] = k < ipp ? __hip_atomic_load(rec + 2 * k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            best = rk[u] > best ? rk[u] : best;
            nvalid += (int)rn[u];
        }
    }
    best = wave_max_u64(best);
    nvalid = wave_total(nvalid);
    if (lane == 0) {
        red_k[wv] = best;
        red_n[wv] = nvalid;
    }
    __syncthreads();
    best = red_k[0];
    nvalid = red_n[0];
#pragma unroll
    for (int k = 1; k < NW; ++k) {
        best = red_k[k] > best ? red_k[k] : best;
        nvalid += red_n[k];
    }
    const int nbnd = st.n_boundary, nedge = st.n_edges, nbad = st.nonfinite;
    const int hbest = best ? (int)(0xFFFFFFFFu - (uint32_t)best) : -1;
    float ps[12];
    if (hbest >= 0) {
        const uint32_t *pose = reinterpret_cast<const uint32_t *>(w.poses + ((int64_t)b * w.h_cap + hbest) * 12);
#pragma unroll
        for (int k = 0; k < 12; ++k)   // written by other workgroups of this launch
            ps[k] = __uint_as_float(__hip_atomic_load(pose + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    } else {
#pragma unroll
        for (int k = 0; k < 12; ++k) ps[k] = (k < 9 && k % 4 == 0) ? 1.0f : 0.0f;
    }
    if (tid == 0) {
        tr_result r;
        for (int k = 0; k < 9; ++k) r.R[k] = ps[k];
        for (int k = 0; k < 3; ++k) r.t[k] = ps[9 + k];
        r.best_inliers = hbest < 0 ? 0
                         : w.metric ? __hip_atomic_load(&w.inl[(int64_t)b * w.h_cap + hbest], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT)
                                    : (int32_t)(best >> 32) - 1;
        r.best_hyp = hbest;
        r.n_valid_hyp = nvalid;
        int status = TR_OK;
        if (st.status == TR_ERR_INVALID_ARG) status = TR_ERR_INVALID_ARG;
        else if (nbad) status = TR_ERR_NONFINITE;
        else if (hbest < 0) status = TR_ERR_NO_HYPOTHESIS;
        else if (st.fallback) status = TR_WARN_SCORER_FALLBACK;
        r.status = status;
        r.n_boundary_pairs = nbnd;
        r.n_pivots = d.n > 0 ? min(w.k1, d.kpiv) : 0;
        r.n_edges = nedge;
        r.reserved = 0;
        w.out[b] = r;
    }
    if (want_mask) {
        // kM matches per thread per step, their loads all issued before any residual is formed
        const float th2 = w.theta * w.theta;
        for (int k0 = tid; k0 < d.n; k0 += NT * kM) {
            if (k0 != tid) load_pts(k0);
#pragma unroll
            for (int m = 0; m < kM; ++m) {
                const int k = k0 + NT * m;
                if (k < d.n) {
                    const bool in = hbest >= 0 &&
                                    residual2(ps, x[m][0], x[m][1], x[m][2], y[m][0], y[m][1], y[m][2]) <= th2;
                    w.masks[d.pt_off + k] = in ? 1 : 0;
                }
            }
        }
    }
    if (w.hyp_prof) {
        // profiled call: this pair's phase durations, summed over its items (written before their
        // tickets), and the selection's own duration, added to the per-handle sums
        __syncthreads();
        const uint32_t *ip = w.hyp_prof + (int64_t)b * w.rec_stride * 2;
        unsigned long long sum[4] = {0, 0, 0, 0};
        for (int k = tid; k < ipp; k += NT)
#pragma unroll
            for (int f = 0; f < 4; ++f)
                sum[f] += __hip_atomic_load(ip + 4 * k + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            sum[f] = (unsigned long long)wave_total((int)sum[f]);
            if (lane == 0) red_k[wv] = sum[f];
            __syncthreads();
            if (tid == 0) {
                unsigned long long t = 0;
                for (int v = 0; v < NW; ++v) t += red_k[v];
                atomicAdd(&w.prof_acc[kProfSearch + f], t);
            }
            __syncthreads();
        }
        if (tid == 0) {
            atomicAdd(&w.prof_acc[kProfSelect], (unsigned long long)(__builtin_amdgcn_s_memrealtime() - t_sel0));
            atomicAdd(&w.prof_acc[kProfItems], (unsigned long long)ipp);
            atomicAdd(&w.prof_acc[kProfPairs], 1ull);
        }
    }
}

// One DPP move of a float (the control word is a template constant).
template <int CTRL, int RMASK>
__device__ __forceinline__ float dpp_f(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, RMASK, 0xf, false));
}

// Sum over the 64 lanes (DPP, a fixed order), valid in every lane.
__device__ __forceinline__ float wave_total_f(float v)
{
    v += dpp_f<0x111, 0xf>(v);   // row_shr:1
    v += dpp_f<0x112, 0xf>(v);   // row_shr:2
    v += dpp_f<0x114, 0xf>(v);   // row_shr:4
    v += dpp_f<0x118, 0xf>(v);   // row_shr:8
    v += dpp_f<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
    v += dpp_f<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ void store_agent(float *p, float v)
{
    __hip_atomic_store(reinterpret_cast<uint32_t *>(p), __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Hypotheses of ppw pivots per work item (item = pair b, pivots g*ppw ..), one
// workgroup of NW waves: wave v finds the cliques of pivots v, v+NW, ...
// (Eqs. 5-8) and lanes 0..K2-1 fit their poses (Section 3.5) into LDS; then
// the whole workgroup scores the item's ppw*K2 hypotheses against all N
// matches of the pair (Eq. 9), each thread reading four matches per step from
// L2 (the next step's loads in flight) and evaluating eight poses held in
// registers per pass; wave sums
// (DPP) are added into per-hypothesis LDS totals, so IN needs no global
// atomics. IN and the poses are stored at device scope, each item stores its
// best (IN, h) and valid count in its own record, and the workgroup that
// finishes a pair's last item (two levels of atomic tickets, no waiting)
// selects the result.
template <int KMAX, int METRIC, int NW>
__global__ void __launch_bounds__(64 * NW) k_hyp(Work w, int B, int ppw)
{
    constexpr int NT = 64 * NW;
    static_assert(METRIC == 0 || NW == 4, "error-score sums keep the four-wave order of k_score_poses");
    __shared__ float pose_l[16 * TR_MAX_K2][12];
    __shared__ int32_t valid_l[16 * TR_MAX_K2], tot_l[16 * TR_MAX_K2];
    __shared__ float sc_l[4][16 * TR_MAX_K2];   // per-wave error-score sums (METRIC only)
    __shared__ uint64_t key_l[NW];
    __shared__ int32_t nv_l[NW], last;
    __shared__ __attribute__((aligned(16))) uint64_t rkeys[kFusedPool];   // learned pool ordered here
    __shared__ int32_t piv_l[16][3];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int ipp = (w.k1 + ppw - 1) / ppw, total = B * ipp;
    const float th2 = w.theta * w.theta;
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int slot = item / ipp, b = batch_pair(w, slot), g = item - slot * ipp;
        const PairDesc d = pair_desc(w, b);
        const int nloc = ppw * w.k2;   // local hypothesis hl = (pivot lp) * K2 + slot
        // profiled calls: phase stamps of thread 0 (clique search of wave 0's pivots, fits up to
        // the workgroup barrier, scoring, records), 100 MHz real-time clock
        uint64_t ts0 = 0, ts1 = 0, ts2 = 0, ts3 = 0;
        if (w.hyp_prof) ts0 = ts1 = __builtin_amdgcn_s_memrealtime();
        if (tid < 16 * TR_MAX_K2) tot_l[tid] = 0;
        if (w.rank_in_hyp) {
            // learned pivots (pool of K <= kFusedPool plain pivots): the item's ppw positions of the
            // pool ordered by the learned key, each key ranked against all of the pair's keys
            const int K = d.kpiv, K16 = (K + 15) & ~15;
            const bool fb = w.state[b].fallback != 0;
            const int32_t *pl = w.pivots_plain + (int64_t)b * w.pool_cap * 3;
            const float *sc = w.scores + (int64_t)b * w.max_n;
            for (int r = tid; r < K16; r += NT) rkeys[r] = r < K ? reorder_key(pl, sc, r, fb) : ~0ull;
            if (tid < 3 * ppw) piv_l[tid / 3][tid % 3] = tid % 3 == 2 ? 0 : -1;   // positions past K stay empty
            __syncthreads();
            for (int r = tid; r < K; r += NT) {
                const int rk = count_smaller(rkeys, 0, K16, rkeys[r]), lp = rk - g * ppw;
                if (lp >= 0 && lp < ppw && rk < w.k1) {
                    piv_l[lp][0] = pl[3 * r];
                    piv_l[lp][1] = pl[3 * r + 1];
                    piv_l[lp][2] = pl[3 * r + 2];
                }
            }
            __syncthreads();
            if (tid < ppw && g * ppw + tid < w.k1) {   // the ordered list, for inspection
                int32_t *o = w.pivots + ((int64_t)b * w.piv_stride + g * ppw + tid) * 3;
                o[0] = piv_l[tid][0];
                o[1] = piv_l[tid][1];
                o[2] = piv_l[tid][2];
            }
        }
        for (int r = 0; r < (ppw + NW - 1) / NW; ++r) {
            const int lp = r * NW + wv, p = g * ppw + lp;
            if (lp >= ppw) break;   // the same on the whole wave
            int pi = -1, pj = -1, z = -1;
            const int32_t *pv = w.rank_in_hyp ? &piv_l[lp][0] : w.pivots + ((int64_t)b * w.piv_stride + p) * 3;
            if (p < w.k1) z = clique_search<KMAX>(w, d, b, p, pv, lane, pi, pj);
            if (w.hyp_prof && tid == 0) ts1 = __builtin_amdgcn_s_memrealtime();
            if (lane < w.k2) {
                float pose[12];
                const bool ok = p < w.k1 && fit_pose(w, d, pi, pj, z, pose);
                const int hl = lp * w.k2 + lane;
#pragma unroll
                for (int k = 0; k < 12; ++k) pose_l[hl][k] = pose[k];
                valid_l[hl] = ok;
            }
        }
        __syncthreads();
        if (w.hyp_prof) ts2 = __builtin_amdgcn_s_memrealtime();
        for (int h0 = 0; h0 < nloc; h0 += 8) {
            float ps[8][12];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int hl = min(h0 + u, nloc - 1);
#pragma unroll
                for (int k = 0; k < 12; ++k) ps[u][k] = pose_l[hl][k];
            }
            int cu[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            float su[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // error-based scores (METRIC only)
            // four matches per thread per step; the next step's loads are issued before this
            // step's residuals are formed
            float x[4][3], y[4][3];
            auto load4 = [&](int k0) {
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int64_t gi = d.pt_off + min(k0 + NT * m, d.n - 1);
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        x[m][f] = w.src[3 * gi + f];
                        y[m][f] = w.dst[3 * gi + f];
                    }
                }
            };
            load4(tid);
            for (int k0 = tid; k0 < d.n; k0 += 4 * NT) {
                float cx[4][3], cy[4][3];
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int f = 0; f < 3; ++f) {
                        cx[m][f] = x[m][f];
                        cy[m][f] = y[m][f];
                    }
                if (k0 + 4 * NT < d.n) load4(k0 + 4 * NT);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const bool in = k0 + NT * m < d.n;
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const float r2 = residual2(ps[u], cx[m][0], cx[m][1], cx[m][2], cy[m][0], cy[m][1], cy[m][2]);
                        const bool hit = in && r2 <= th2;
                        cu[u] += hit;
                        if (METRIC) {
                            const float c = fmaxf((w.theta - __builtin_sqrtf(r2)) / w.theta, 0.0f);
                            su[u] += hit ? (METRIC == 1 ? c : c * c) : 0.0f;
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int t = wave_total(cu[u]);
                if (lane == 0 && t && h0 + u < nloc) atomicAdd(&tot_l[h0 + u], t);
                if (METRIC) {   // per-wave sums, added in wave order below (deterministic)
                    const float f = wave_total_f(su[u]);
                    if (lane == 0 && h0 + u < nloc) sc_l[wv][h0 + u] = f;
                }
            }
        }
        __syncthreads();
        if (w.hyp_prof) ts3 = __builtin_amdgcn_s_memrealtime();
        uint64_t key = 0;
        int nv = 0;
        if (tid < nloc) {
            const int lp = tid / w.k2, s2 = tid - lp * w.k2, p = g * ppw + lp;
            if (p < w.k1) {
                const int64_t h = (int64_t)s2 * w.k1 + p, slot = (int64_t)b * w.h_cap + h;
                __hip_atomic_store(&w.inl[slot], valid_l[tid] ? tot_l[tid] : -1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                for (int k = 0; k < 12; ++k) store_agent(w.poses + slot * 12 + k, pose_l[tid][k]);
                uint32_t primary = (uint32_t)(tot_l[tid] + 1);
                if (METRIC) {
                    const float sc = ((sc_l[0][tid] + sc_l[1][tid]) + sc_l[2][tid]) + sc_l[3][tid];
                    store_agent(w.gscore + slot, valid_l[tid] ? sc : -1.0f);
                    primary = __float_as_uint(sc) + 1u;   // sc >= 0: the bits order like the values
                }
                if (valid_l[tid]) {
                    key = ((uint64_t)primary << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)h);
                    nv = 1;
                }
            }
        }
        // this item's best hypothesis (lowest h on ties) and valid count, stored in its own record
        key = wave_max_u64(key);
        nv = wave_total(nv);
        if (lane == 0) {
            key_l[wv] = key;
            nv_l[wv] = nv;
        }
        __syncthreads();
        if (tid == 0) {
            uint64_t k = key_l[0];
            int n = nv_l[0];
#pragma unroll
            for (int v = 1; v < NW; ++v) {
                k = key_l[v] > k ? key_l[v] : k;
                n += nv_l[v];
            }
            uint64_t *rec = w.hyp_rec + (int64_t)b * w.rec_stride + 2 * g;
            __hip_atomic_store(rec, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(rec + 1, (uint64_t)n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (w.hyp_prof) {
                const uint64_t ts4 = __builtin_amdgcn_s_memrealtime();
                uint32_t *ip = w.hyp_prof + ((int64_t)b * w.rec_stride / 2 + g) * 4;
                const uint32_t dur[4] = {(uint32_t)(ts1 - ts0), (uint32_t)(ts2 - ts1), (uint32_t)(ts3 - ts2),
                                         (uint32_t)(ts4 - ts3)};
#pragma unroll
                for (int f = 0; f < 4; ++f) __hip_atomic_store(ip + f, dur[f], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // Two levels of tickets: the last item of a group of kHypGroup takes a ticket of the pair,
        // and the workgroup that takes the pair's last ticket reads the records and the best pose
        // (no counter is shared by more than kHypGroup items or ceil(ipp / kHypGroup) groups).
        // The workgroup's stores are ordered before its ticket by the barrier and the ticket's
        // release at device scope; the last taker's acquire orders its reads after every ticket.
        __syncthreads();
        if (tid == 0) {
            const int grp = g / kHypGroup, ngrp = (ipp + kHypGroup - 1) / kHypGroup;
            const int gsz = min(kHypGroup, ipp - grp * kHypGroup);
            int32_t *gt = w.tick + (int64_t)b * w.tick_stride + (kTickHyp0 + grp) * kTickLine;
            bool l = __hip_atomic_fetch_add(gt, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == gsz - 1;
            if (l)
                l = __hip_atomic_fetch_add(&w.state[b].done, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) ==
                    ngrp - 1;
            last = l;
        }
        __syncthreads();
        if (last) select_pair<NW>(w, b, ipp);
        __syncthreads();   // LDS is the next item's
    }
}

// Inlier numbers (Eq. 9) and, for metric 1 / 2, the error-based scores of
// caller-given poses against one pair's matches: eight poses per workgroup,
// the matches strided over the 256 threads and every sum formed in the same
// order as in k_hyp, so a pose scores the same bits here as there.
__global__ void __launch_bounds__(256) k_score_poses(const float *src, const float *dst, int n, const float *poses,
                                                     int P, float theta, int metric, int32_t *in_out,
                                                     float *score_out)
{
    __shared__ int32_t cnt_l[4][8];
    __shared__ float sum_l[4][8];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const float th2 = theta * theta;
    for (int p0 = blockIdx.x * 8; p0 < P; p0 += gridDim.x * 8) {
        float ps[8][12];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int k = 0; k < 12; ++k) ps[u][k] = poses[(int64_t)min(p0 + u, P - 1) * 12 + k];
        int cu[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        float su[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int k0 = tid; k0 < n; k0 += 1024) {
            float x[4][3], y[4][3];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int64_t gi = min(k0 + 256 * m, n - 1);
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    x[m][f] = src[3 * gi + f];
                    y[m][f] = dst[3 * gi + f];
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const bool in = k0 + 256 * m < n;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const float r2 = residual2(ps[u], x[m][0], x[m][1], x[m][2], y[m][0], y[m][1], y[m][2]);
                    const bool hit = in && r2 <= th2;
                    cu[u] += hit;
                    if (metric) {
                        const float c = fmaxf((theta - __builtin_sqrtf(r2)) / theta, 0.0f);
                        su[u] += hit ? (metric == 1 ? c : c * c) : 0.0f;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int t = wave_total(cu[u]);
            const float f = wave_total_f(su[u]);
            if (lane == 0) {
                cnt_l[wv][u] = t;
                sum_l[wv][u] = f;
            }
        }
        __syncthreads();
        if (tid < 8 && p0 + tid < P) {
            in_out[p0 + tid] = cnt_l[0][tid] + cnt_l[1][tid] + cnt_l[2][tid] + cnt_l[3][tid];
            if (metric && score_out)
                score_out[p0 + tid] = ((sum_l[0][tid] + sum_l[1][tid]) + sum_l[2][tid]) + sum_l[3][tid];
        }
        __syncthreads();   // the LDS totals are the next group's
    }
}

// One rigid fit (Section 3.5, the registration's fit_pose) per caller-given
// triplet of match indices; a triplet with an index outside [0, n) or a
// negative one gets the identity pose and ok = 0.
__global__ void __launch_bounds__(256) k_fit_triplets(Work w, PairDesc d, const int32_t *tri, int T, float *poses,
                                                      int32_t *ok)
{
    for (int t = blockIdx.x * 256 + threadIdx.x; t < T; t += gridDim.x * 256) {
        const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        float pose[12];
        const bool in = a >= 0 && a < d.n && b >= 0 && b < d.n && c >= 0 && c < d.n;
        const bool fit = fit_pose(w, d, in ? a : 0, in ? b : 0, in ? c : -1, pose);
#pragma unroll
        for (int k = 0; k < 12; ++k) poses[(int64_t)t * 12 + k] = pose[k];
        ok[t] = in && fit;
    }
}

}  // namespace

hipError_t launch_fit_triplets(const float *src, const float *dst, int n, const int32_t *tri, int T, float *poses,
                               int32_t *ok, int grid, hipStream_t s)
{
    Work w{};
    w.src = src;
    w.dst = dst;
    PairDesc d{};
    d.n = n;
    d.pt_off = 0;
    grid = max(1, min(grid, (T + 255) / 256));
    hipLaunchKernelGGL(k_fit_triplets, dim3(grid), dim3(256), 0, s, w, d, tri, T, poses, ok);
    return hipGetLastError();
}

hipError_t launch_score_poses(const float *src, const float *dst, int n, const float *poses, int P, float theta,
                              int metric, int32_t *in_out, float *score_out, int grid, hipStream_t s)
{
    grid = max(1, min(grid, (P + 7) / 8));
    hipLaunchKernelGGL(k_score_poses, dim3(grid), dim3(256), 0, s, src, dst, n, poses, P, theta, metric, in_out,
                       score_out);
    return hipGetLastError();
}

hipError_t setup_hyp_kernels()
{
    return hipSuccess;
}

// ppw: pivots per work item, a multiple of 4 up to 16 (the LDS pose slots);
// grid: workgroups to launch (capped at the number of items).
hipError_t launch_hyp(const Work &w, int B, int ppw, int grid, hipStream_t s)
{
    if (ppw < 4 || ppw > 16 || ppw % 4) return hipErrorInvalidValue;
    const int total = B * ((w.k1 + ppw - 1) / ppw);
    grid = max(1, min(total, grid));
    const bool small = w.k2 <= 2;
    // inlier-number ranking: eight waves per workgroup (two per SIMD) share the scoring; the
    // error-based rankings keep four, the summation order tr_score_poses reproduces
    if (w.metric == 1) {
        if (small) hipLaunchKernelGGL((k_hyp<2, 1, 4>), dim3(grid), dim3(256), 0, s, w, B, ppw);
        else hipLaunchKernelGGL((k_hyp<TR_MAX_K2, 1, 4>), dim3(grid), dim3(256), 0, s, w, B, ppw);
    } else if (w.metric == 2) {
        if (small) hipLaunchKernelGGL((k_hyp<2, 2, 4>), dim3(grid), dim3(256), 0, s, w, B, ppw);
        else hipLaunchKernelGGL((k_hyp<TR_MAX_K2, 2, 4>), dim3(grid), dim3(256), 0, s, w, B, ppw);
    } else {
        if (small) hipLaunchKernelGGL((k_hyp<2, 0, 8>), dim3(grid), dim3(512), 0, s, w, B, ppw);
        else hipLaunchKernelGGL((k_hyp<TR_MAX_K2, 0, 8>), dim3(grid), dim3(512), 0, s, w, B, ppw);
    }
    return hipGetLastError();
}

}  // namespace tr
