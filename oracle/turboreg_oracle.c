/*
 * TurboReg CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow host implementation of what the TurboReg path computes, written
 * from the paper (Yan et al., ICCV 2025, arXiv 2507.01439). Each function cites
 * the passage it follows. It exists to check the HIP library against: only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it, and
 * it shares no code, header or table with the HIP path.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math -lm.
 * Floating-point contraction is off so that every a*b and a+b below is one
 * IEEE-rounded operation; fused multiply-adds appear only as explicit fmaf().
 * A second build adds -fopenmp: the pragmas below split loops whose iterations
 * write disjoint outputs (integer sums are reduced exactly), so both builds
 * compute the same bits; without -fopenmp the pragmas are ignored.
 *
 * Every function is pinned by tests that do not reuse this code: brute-force
 * triangle enumeration, closed forms, hand-counted graphs, LAPACK/numpy
 * routines, finite differences.
 */
#include "turboreg_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Eq. 1 -- pairwise length compatibility                              */
/* ------------------------------------------------------------------ */

/* Length of (ax, ay, az) in float32: the square of the first component is
 * rounded, the other two are added by fused multiply-adds, then the correctly
 * rounded square root. This order is the decision arithmetic both the oracle
 * and the HIP kernel follow, so that C is reproducible bit for bit. */
static float length32(float ax, float ay, float az)
{
    float s = ax * ax;
    s = fmaf(ay, ay, s);
    s = fmaf(az, az, s);
    return sqrtf(s);
}

/* delta_ij of Eq. 1 in float32: | |x_i - x_j| - |y_i - y_j| |. */
static float delta32(const float *X, const float *Y, int32_t i, int32_t j)
{
    float lx = length32(X[3 * i] - X[3 * j], X[3 * i + 1] - X[3 * j + 1], X[3 * i + 2] - X[3 * j + 2]);
    float ly = length32(Y[3 * i] - Y[3 * j], Y[3 * i + 1] - Y[3 * j + 1], Y[3 * i + 2] - Y[3 * j + 2]);
    return fabsf(lx - ly);
}

/* The same quantity in float64 from the float32 inputs, for boundary reports. */
static double delta64(const float *X, const float *Y, int32_t i, int32_t j)
{
    double ax = (double)X[3 * i] - X[3 * j], ay = (double)X[3 * i + 1] - X[3 * j + 1],
           az = (double)X[3 * i + 2] - X[3 * j + 2];
    double bx = (double)Y[3 * i] - Y[3 * j], by = (double)Y[3 * i + 1] - Y[3 * j + 1],
           bz = (double)Y[3 * i + 2] - Y[3 * j + 2];
    return fabs(sqrt(ax * ax + ay * ay + az * az) - sqrt(bx * bx + by * by + bz * bz));
}

int tro_compat(const float *X, const float *Y, int32_t n, float tau, uint8_t *C,
               int64_t *n_boundary32, int64_t *n_boundary64, int64_t *n_flip)
{
    if (!X || !Y || !C || n < 0) return -1;
    int64_t nb32 = 0, nb64 = 0, nf = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : nb32, nb64, nf)
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < n; ++j) {
            if (i == j) { C[(int64_t)i * n + j] = 0; continue; }   /* no self loops (reading) */
            float d = delta32(X, Y, i, j);
            C[(int64_t)i * n + j] = (uint8_t)(d <= tau);            /* Eq. 1 uses "<=" */
            if (i < j) {
                if (fabsf(d - tau) < 1e-6f) ++nb32;
                double d64 = delta64(X, Y, i, j);
                if (fabs(d64 - (double)tau) < 1e-6) ++nb64;
                if ((d64 <= (double)tau) != (d <= tau)) ++nf;
            }
        }
    }
    /* IEEE subtraction is sign-symmetric, so the matrix must come out symmetric. */
    int asym = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : asym)
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j)
            asym |= C[(int64_t)i * n + j] != C[(int64_t)j * n + i];
    if (asym) return -2;
    if (n_boundary32) *n_boundary32 = nb32;
    if (n_boundary64) *n_boundary64 = nb64;
    if (n_flip) *n_flip = nf;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. 2 -- second-order compatibility                                 */
/* ------------------------------------------------------------------ */

/* Ghat_ij = C_ij * sum_k C_ik C_jk. The inner sum over k is the number of set
 * bits of (row_i AND row_j) with each row of C held as a bit set; it is the
 * definition evaluated exactly in integers. */
int tro_sc2(const uint8_t *C, int32_t n, int32_t *Ghat)
{
    if (!C || !Ghat || n < 0) return -1;
    int64_t words = ((int64_t)n + 63) / 64;
    uint64_t *bits = (uint64_t *)calloc((size_t)(words * (n > 0 ? n : 1)), sizeof(uint64_t));
    if (!bits) return -3;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = 0; k < n; ++k)
            if (C[(int64_t)i * n + k]) bits[i * words + k / 64] |= (uint64_t)1 << (k % 64);
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t i = 0; i < n; ++i) {
        for (int32_t j = 0; j < n; ++j) {
            int32_t v = 0;
            if (C[(int64_t)i * n + j]) {
                const uint64_t *ri = bits + i * words, *rj = bits + j * words;
                for (int64_t w = 0; w < words; ++w) v += __builtin_popcountll(ri[w] & rj[w]);
            }
            Ghat[(int64_t)i * n + j] = v;
        }
    }
    free(bits);
    return 0;
}

/* Definition 2: keep only edges oriented from the lower to the higher index. */
int tro_o2graph(const int32_t *Ghat, int32_t n, int32_t *Gt)
{
    if (!Ghat || !Gt || n < 0) return -1;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < n; ++j)
            Gt[(int64_t)i * n + j] = (i < j) ? Ghat[(int64_t)i * n + j] : 0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. 4 -- pivot selection                                            */
/* ------------------------------------------------------------------ */

typedef struct { int32_t w, i, j; } edge_t;

/* Weight descending; among equal weights the lexicographically smaller pair
 * first (the paper only says tied edges are taken until K1 are chosen). */
static int edge_cmp(const void *a, const void *b)
{
    const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
    if (x->w != y->w) return x->w > y->w ? -1 : 1;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return 0;
}

/* All pairs i<j ordered by edge_cmp, first K1 kept. Weights are counts (never
 * negative), so every zero-weight pair sorts after every positive one and the
 * zero-weight pairs among themselves in (i, j) order: only the positive pairs
 * are sorted, and the zero-weight pairs are appended by a row-major scan. The
 * result equals a sort of all N(N-1)/2 pairs. */
int64_t tro_pivots(const int32_t *Gbar, int32_t n, int32_t k1, int32_t *P)
{
    if (!Gbar || !P || n < 0 || k1 < 0) return -1;
    int64_t m = (int64_t)n * (n - 1) / 2, pos = 0;
    int negative = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : pos) reduction(| : negative)
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j) {
            negative |= Gbar[(int64_t)i * n + j] < 0;
            pos += Gbar[(int64_t)i * n + j] > 0;
        }
    if (negative) return -1;
    edge_t *e = (edge_t *)malloc((size_t)(pos > 0 ? pos : 1) * sizeof(edge_t));
    if (!e) return -3;
    int64_t c = 0;
    for (int32_t i = 0; i < n; ++i)
        for (int32_t j = i + 1; j < n; ++j)
            if (Gbar[(int64_t)i * n + j] > 0) {
                e[c].w = Gbar[(int64_t)i * n + j];
                e[c].i = i;
                e[c].j = j;
                ++c;
            }
    qsort(e, (size_t)pos, sizeof(edge_t), edge_cmp);
    int64_t np = m < k1 ? m : k1, p = 0;
    for (; p < np && p < pos; ++p) { P[3 * p] = e[p].i; P[3 * p + 1] = e[p].j; P[3 * p + 2] = e[p].w; }
    for (int32_t i = 0; i < n && p < np; ++i)
        for (int32_t j = i + 1; j < n && p < np; ++j)
            if (Gbar[(int64_t)i * n + j] == 0) { P[3 * p] = i; P[3 * p + 1] = j; P[3 * p + 2] = 0; ++p; }
    for (; p < k1; ++p) { P[3 * p] = -1; P[3 * p + 1] = -1; P[3 * p + 2] = 0; }
    free(e);
    return np;
}

/* ------------------------------------------------------------------ */
/* Eqs. 5-8, Algorithm 1 -- TurboClique search and top-K2 selection     */
/* ------------------------------------------------------------------ */

int tro_cliques(const int32_t *Gbar, int32_t n, const int32_t *P, int32_t n_pivots,
                int32_t k1, int32_t k2, int32_t *cliques)
{
    if (!Gbar || !P || !cliques || n < 0 || k1 < 0 || k2 < 1 || n_pivots > k1) return -1;
    int failed = 0;
#pragma omp parallel reduction(| : failed)
    {
        /* the pivot's K2 best (S, z) so far, one list per thread */
        int32_t *bs = (int32_t *)malloc(sizeof(int32_t) * (size_t)k2);
        int32_t *bz = (int32_t *)malloc(sizeof(int32_t) * (size_t)k2);
        failed |= !bs || !bz;
#pragma omp for schedule(dynamic, 4)
        for (int32_t p = 0; p < k1; ++p) {
            if (!bs || !bz) continue;
            for (int32_t s = 0; s < k2; ++s) { bs[s] = -1; bz[s] = -1; }
            int32_t i = -1, j = -1;
            if (p < n_pivots) {
                i = P[3 * p];
                j = P[3 * p + 1];
                int32_t gij = Gbar[(int64_t)i * n + j];
                for (int32_t z = 0; z < n; ++z) {
                    if (z == i || z == j) continue;
                    int32_t giz = Gbar[(int64_t)i * n + z], gjz = Gbar[(int64_t)j * n + z];
                    /* verification condition (Eq. 8): all three weights positive */
                    if (!(gij > 0 && giz > 0 && gjz > 0)) continue;
                    int32_t S = gij + giz + gjz;                     /* Eq. 6 */
                    /* keep the k2 best by (S desc, z asc); z grows, so a tie never displaces */
                    int32_t pos = k2;
                    for (int32_t q = 0; q < k2; ++q)
                        if (bz[q] < 0 || S > bs[q]) { pos = q; break; }
                    if (pos == k2) continue;
                    for (int32_t q = k2 - 1; q > pos; --q) { bs[q] = bs[q - 1]; bz[q] = bz[q - 1]; }
                    bs[pos] = S;
                    bz[pos] = z;
                }
            }
            for (int32_t s = 0; s < k2; ++s) {
                int64_t h = (int64_t)s * k1 + p;                      /* Algorithm 2 layout */
                cliques[3 * h] = i;
                cliques[3 * h + 1] = j;
                cliques[3 * h + 2] = bz[s];
            }
        }
        free(bs);
        free(bz);
    }
    return failed ? -3 : 0;
}

/* ------------------------------------------------------------------ */
/* Section 3.5 -- Kabsch fit of each clique (float64)                  */
/* ------------------------------------------------------------------ */

/* Singular value decomposition of a 3x3 matrix by one-sided (Hestenes) Jacobi:
 * plane rotations applied on the right orthogonalise the columns of A = H;
 * then A V = U diag(S). Columns are sorted so that S[0] >= S[1] >= S[2].
 * On return U holds the scaled columns (not yet normalised). */
static void jacobi_svd3(const double Hm[9], double A[9], double V[9], double S[3])
{
    memcpy(A, Hm, 9 * sizeof(double));
    for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
    static const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int sweep = 0; sweep < 64; ++sweep) {
        int rotated = 0;
        for (int pp = 0; pp < 3; ++pp) {
            int p = pairs[pp][0], q = pairs[pp][1];
            double alpha = 0, beta = 0, gamma = 0;
            for (int r = 0; r < 3; ++r) {
                alpha += A[3 * r + p] * A[3 * r + p];
                beta += A[3 * r + q] * A[3 * r + q];
                gamma += A[3 * r + p] * A[3 * r + q];
            }
            if (gamma == 0.0 || fabs(gamma) <= 1e-15 * sqrt(alpha * beta)) continue;
            rotated = 1;
            double zeta = (beta - alpha) / (2.0 * gamma);
            double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
            for (int r = 0; r < 3; ++r) {
                double ap = A[3 * r + p], aq = A[3 * r + q];
                A[3 * r + p] = c * ap - s * aq;
                A[3 * r + q] = s * ap + c * aq;
                double vp = V[3 * r + p], vq = V[3 * r + q];
                V[3 * r + p] = c * vp - s * vq;
                V[3 * r + q] = s * vp + c * vq;
            }
        }
        if (!rotated) break;
    }
    for (int k = 0; k < 3; ++k)
        S[k] = sqrt(A[k] * A[k] + A[3 + k] * A[3 + k] + A[6 + k] * A[6 + k]);
    for (int a = 0; a < 2; ++a)          /* selection sort, columns of A and V together */
        for (int b = a + 1; b < 3; ++b)
            if (S[b] > S[a]) {
                double tmp = S[a]; S[a] = S[b]; S[b] = tmp;
                for (int r = 0; r < 3; ++r) {
                    tmp = A[3 * r + a]; A[3 * r + a] = A[3 * r + b]; A[3 * r + b] = tmp;
                    tmp = V[3 * r + a]; V[3 * r + a] = V[3 * r + b]; V[3 * r + b] = tmp;
                }
            }
}

static double det3(const double M[9])
{
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) +
           M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/* Least-squares rotation and translation mapping points p_a onto q_a
 * (Kabsch 1976): H = sum_a (p_a - pbar)(q_a - qbar)^T = U S V^T,
 * R = V diag(1, 1, d) U^T with d = sign det(V U^T), t = qbar - R pbar.
 * Returns 1, or 2 when sigma_2 <= 1e-9 sigma_1. */
static int kabsch3(const double p[3][3], const double q[3][3], double R[9], double t[3])
{
    double pb[3] = {0, 0, 0}, qb[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) { pb[c] += p[a][c] / 3.0; qb[c] += q[a][c] / 3.0; }
    double Hm[9] = {0};
    for (int a = 0; a < 3; ++a)
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Hm[3 * r + c] += (p[a][r] - pb[r]) * (q[a][c] - qb[c]);
    double A[9], V[9], S[3], U[9];
    jacobi_svd3(Hm, A, V, S);
    int flag = 1;
    /* u1 */
    if (S[0] > 0) { for (int r = 0; r < 3; ++r) U[3 * r] = A[3 * r] / S[0]; }
    else { U[0] = 1; U[3] = 0; U[6] = 0; flag = 2; }
    /* u2: from A when sigma_2 is well separated from zero, else any unit vector orthogonal to u1 */
    if (S[1] > 1e-9 * S[0] && S[0] > 0) {
        for (int r = 0; r < 3; ++r) U[3 * r + 1] = A[3 * r + 1] / S[1];
    } else {
        flag = 2;
        double e[3] = {0, 0, 0};
        int m = 0;   /* axis least aligned with u1 */
        for (int r = 1; r < 3; ++r) if (fabs(U[3 * r]) < fabs(U[3 * m])) m = r;
        e[m] = 1.0;
        double d = e[0] * U[0] + e[1] * U[3] + e[2] * U[6], nn = 0;
        for (int r = 0; r < 3; ++r) { U[3 * r + 1] = e[r] - d * U[3 * r]; nn += U[3 * r + 1] * U[3 * r + 1]; }
        nn = sqrt(nn);
        for (int r = 0; r < 3; ++r) U[3 * r + 1] /= nn;
    }
    /* u3 = u1 x u2: three centred points span at most a plane, so sigma_3 = 0 */
    U[2] = U[3] * U[7] - U[6] * U[4];
    U[5] = U[6] * U[1] - U[0] * U[7];
    U[8] = U[0] * U[4] - U[3] * U[1];
    double d = (det3(V) * det3(U) < 0) ? -1.0 : 1.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            R[3 * r + c] = V[3 * r] * U[3 * c] + V[3 * r + 1] * U[3 * c + 1] + d * V[3 * r + 2] * U[3 * c + 2];
    for (int r = 0; r < 3; ++r) t[r] = qb[r] - (R[3 * r] * pb[0] + R[3 * r + 1] * pb[1] + R[3 * r + 2] * pb[2]);
    return flag;
}

int tro_kabsch(const float *X, const float *Y, const int32_t *cliques, int32_t H,
               double *R, double *t, int32_t *flags)
{
    if (!X || !Y || !cliques || !R || !t || !flags || H < 0) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t h = 0; h < H; ++h) {
        const int32_t *c = cliques + 3 * (int64_t)h;
        double *Rh = R + 9 * (int64_t)h, *th = t + 3 * (int64_t)h;
        if (c[0] < 0 || c[1] < 0 || c[2] < 0) {
            for (int k = 0; k < 9; ++k) Rh[k] = (k % 4 == 0) ? 1.0 : 0.0;
            th[0] = th[1] = th[2] = 0.0;
            flags[h] = 0;
            continue;
        }
        double p[3][3], q[3][3];
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 3; ++k) { p[a][k] = X[3 * c[a] + k]; q[a][k] = Y[3 * c[a] + k]; }
        flags[h] = kabsch3(p, q, Rh, th);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. 9 -- hypothesis scoring by inlier number, and selection         */
/* ------------------------------------------------------------------ */

/* Residual |R x + t - y|^2 in float32: each component starts at t and adds
 * R_r0 x, R_r1 y, R_r2 z by fused multiply-adds; the squared norm rounds the
 * first square and fuses the other two. */
static float residual2(const float *pose, const float *x, const float *y)
{
    float r[3];
    for (int a = 0; a < 3; ++a) {
        float u = pose[9 + a];
        u = fmaf(pose[3 * a], x[0], u);
        u = fmaf(pose[3 * a + 1], x[1], u);
        u = fmaf(pose[3 * a + 2], x[2], u);
        r[a] = u - y[a];
    }
    float s = r[0] * r[0];
    s = fmaf(r[1], r[1], s);
    s = fmaf(r[2], r[2], s);
    return s;
}

int tro_score(const float *X, const float *Y, int32_t n, const float *poses,
              const int32_t *valid, int32_t H, float theta, int32_t *IN)
{
    if (!X || !Y || !poses || !valid || !IN || n < 0 || H < 0) return -1;
    float th2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t h = 0; h < H; ++h) {
        if (!valid[h]) { IN[h] = -1; continue; }
        int32_t c = 0;
        for (int32_t k = 0; k < n; ++k)
            c += residual2(poses + 12 * (int64_t)h, X + 3 * (int64_t)k, Y + 3 * (int64_t)k) <= th2;
        IN[h] = c;
    }
    return 0;
}

int tro_mask(const float *X, const float *Y, int32_t n, const float *pose, float theta,
             uint8_t *mask)
{
    if (!X || !Y || !pose || !mask || n < 0) return -1;
    float th2 = theta * theta;
    for (int32_t k = 0; k < n; ++k)
        mask[k] = residual2(pose, X + 3 * (int64_t)k, Y + 3 * (int64_t)k) <= th2;
    return 0;
}

int32_t tro_select(const int32_t *IN, int32_t H)
{
    int32_t best = -1;
    for (int32_t h = 0; h < H; ++h)
        if (IN[h] >= 0 && (best < 0 || IN[h] > IN[best])) best = h;
    return best;
}

/* Error-based hypothesis scores (the ranking study of the supplementary
 * material, Table 6: hypotheses ranked by mean absolute / mean squared error
 * instead of the inlier number). Reading: over the inliers of Eq. 9 (the same
 * float32 test r^2 <= theta^2), with e = sqrt(r^2) (float32, correctly rounded)
 * and u = max(0, (theta - e) / theta) in float32, the MAE score is the sum of u and the
 * MSE score the sum of u * u (float32 products), summed in float64 and rounded
 * to float32. Larger is better: more inliers, and closer ones. An invalid
 * hypothesis scores -1. metric: 1 = MAE, 2 = MSE. */
int tro_score_metric(const float *X, const float *Y, int32_t n, const float *poses,
                     const int32_t *valid, int32_t H, float theta, int32_t metric, float *S)
{
    /* theta = 0 leaves u = 0/0 undefined: the error-based rankings need theta > 0 */
    if (!X || !Y || !poses || !valid || !S || n < 0 || H < 0 || (metric != 1 && metric != 2) || !(theta > 0.0f))
        return -1;
    const float th2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 4)
    for (int32_t h = 0; h < H; ++h) {
        if (!valid[h]) { S[h] = -1.0f; continue; }
        double acc = 0.0;
        for (int32_t k = 0; k < n; ++k) {
            const float r2 = residual2(poses + 12 * (int64_t)h, X + 3 * (int64_t)k, Y + 3 * (int64_t)k);
            if (!(r2 <= th2)) continue;
            float u = (theta - sqrtf(r2)) / theta;
            /* e <= theta whenever theta^2 is a normal float32 (a correctly rounded square root of
             * a correctly rounded square returns the operand); a subnormal theta^2 has lost bits,
             * and e can then exceed theta: the truncation keeps u at 0 */
            if (u < 0.0f) u = 0.0f;
            acc += metric == 1 ? (double)u : (double)(u * u);
        }
        S[h] = (float)acc;
    }
    return 0;
}

/* The largest score (lowest h among equal ones); -1 when every score is negative. */
int32_t tro_select_score(const float *S, int32_t H)
{
    int32_t best = -1;
    for (int32_t h = 0; h < H; ++h)
        if (S[h] >= 0.0f && (best < 0 || S[h] > S[best])) best = h;
    return best;
}

/* ------------------------------------------------------------------ */
/* Whole path                                                          */
/* ------------------------------------------------------------------ */

int tro_register(const float *X, const float *Y, int32_t n, const tro_params *p,
                 tro_result *out, uint8_t *mask)
{
    return tro_register_ex(X, Y, n, p, 0, NULL, NULL, out, mask, NULL, NULL, NULL, NULL, NULL, NULL);
}

/* The whole path in the paper's order, optionally with the learned reorder of the pivot pool by
 * given scores, optionally scoring given float32 poses instead of the fit's own rounding (the
 * inlier numbers are defined on identical float32 poses), and optionally returning every
 * hypothesis's clique, float64 fit and inlier number. */
int tro_register_ex(const float *X, const float *Y, int32_t n, const tro_params *p, int32_t pool_factor,
                    const float *scores, const float *poses_in, tro_result *out, uint8_t *mask,
                    int32_t *cliques_out, double *R_out, double *t_out, int32_t *flags_out,
                    int32_t *IN_out, int32_t *pivots_out)
{
    if (!X || !Y || !p || !out || n < 3 || p->k1 < 1 || p->k2 < 1) return -1;
    if (scores && pool_factor < 1) return -1;
    memset(out, 0, sizeof(*out));
    int64_t nn = (int64_t)n * n;
    int64_t H = (int64_t)p->k1 * p->k2;
    const int32_t pool = scores ? p->k1 * pool_factor : p->k1;
    uint8_t *C = (uint8_t *)malloc((size_t)nn);
    int32_t *G = (int32_t *)malloc((size_t)nn * sizeof(int32_t));
    int32_t *Pp = (int32_t *)malloc((size_t)pool * 3 * sizeof(int32_t));
    int32_t *P = (int32_t *)malloc((size_t)p->k1 * 3 * sizeof(int32_t));
    int32_t *cl = (int32_t *)malloc((size_t)H * 3 * sizeof(int32_t));
    double *R = (double *)malloc((size_t)H * 9 * sizeof(double));
    double *t = (double *)malloc((size_t)H * 3 * sizeof(double));
    int32_t *flags = (int32_t *)malloc((size_t)H * sizeof(int32_t));
    float *poses = (float *)malloc((size_t)H * 12 * sizeof(float));
    int32_t *IN = (int32_t *)malloc((size_t)H * sizeof(int32_t));
    int rc = -3;
    if (!C || !G || !Pp || !P || !cl || !R || !t || !flags || !poses || !IN) goto done;
    rc = tro_compat(X, Y, n, p->tau, C, &out->n_boundary32, &out->n_boundary64, &out->n_flip);
    if (rc) goto done;
    rc = tro_sc2(C, n, G);
    if (rc) goto done;
    if (p->graph == 0) tro_o2graph(G, n, G);
    {
        int64_t np = tro_pivots(G, n, pool, Pp);
        if (np < 0) { rc = (int)np; goto done; }
        out->n_pivots = np < p->k1 ? np : p->k1;
    }
    if (scores) {
        rc = tro_pivots_learned(Pp, pool, scores, p->k1, P);
        if (rc < 0) goto done;
    } else {
        memcpy(P, Pp, (size_t)p->k1 * 3 * sizeof(int32_t));
    }
    if (pivots_out) memcpy(pivots_out, P, (size_t)p->k1 * 3 * sizeof(int32_t));
    rc = tro_cliques(G, n, P, (int32_t)out->n_pivots, p->k1, p->k2, cl);
    if (rc) goto done;
    rc = tro_kabsch(X, Y, cl, (int32_t)H, R, t, flags);
    if (rc) goto done;
    for (int64_t h = 0; h < H; ++h) {
        for (int k = 0; k < 9; ++k) poses[12 * h + k] = (float)R[9 * h + k];
        for (int k = 0; k < 3; ++k) poses[12 * h + 9 + k] = (float)t[3 * h + k];
        out->n_valid_hyp += flags[h] != 0;
    }
    if (poses_in) memcpy(poses, poses_in, (size_t)H * 12 * sizeof(float));
    rc = tro_score(X, Y, n, poses, flags, (int32_t)H, p->theta, IN);
    if (rc) goto done;
    int32_t hb = tro_select(IN, (int32_t)H);
    out->best_hyp = hb;
    if (hb < 0) {
        out->status = 3;
        out->best_inliers = 0;
        for (int k = 0; k < 9; ++k) { out->R[k] = (k % 4 == 0); out->R32[k] = (float)(k % 4 == 0); }
        if (mask) memset(mask, 0, (size_t)n);
    } else {
        out->status = 0;
        out->best_inliers = IN[hb];
        memcpy(out->R, R + 9 * (int64_t)hb, 9 * sizeof(double));
        memcpy(out->t, t + 3 * (int64_t)hb, 3 * sizeof(double));
        memcpy(out->R32, poses + 12 * (int64_t)hb, 9 * sizeof(float));
        memcpy(out->t32, poses + 12 * (int64_t)hb + 9, 3 * sizeof(float));
        if (mask) tro_mask(X, Y, n, poses + 12 * (int64_t)hb, p->theta, mask);
    }
    if (cliques_out) memcpy(cliques_out, cl, (size_t)H * 3 * sizeof(int32_t));
    if (R_out) memcpy(R_out, R, (size_t)H * 9 * sizeof(double));
    if (t_out) memcpy(t_out, t, (size_t)H * 3 * sizeof(double));
    if (flags_out) memcpy(flags_out, flags, (size_t)H * sizeof(int32_t));
    if (IN_out) memcpy(IN_out, IN, (size_t)H * sizeof(int32_t));
    rc = 0;
done:
    free(C); free(G); free(Pp); free(P); free(cl); free(R); free(t); free(flags); free(poses); free(IN);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Learned pivot scorer                                                */
/* ------------------------------------------------------------------ */

float tro_bf16_round(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return x;   /* NaN */
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

static double bf(double x, int on) { return on ? (double)tro_bf16_round((float)x) : x; }

int tro_features(const float *X, const float *Y, int32_t n, float tau,
                 const uint8_t *C, const int32_t *Ghat, double *F)
{
    if (!X || !Y || !C || !Ghat || !F || n < 2) return -1;
    float q = tau * 0.25f, edge[16];
    for (int k = 0; k < 16; ++k) edge[k] = (float)k * q;
#pragma omp parallel for schedule(dynamic, 16)
    for (int32_t a = 0; a < n; ++a) {
        int64_t deg = 0, sum = 0, hist[16] = {0};
        int32_t mx = 0;
        for (int32_t b = 0; b < n; ++b) {
            if (b == a) continue;
            deg += C[(int64_t)a * n + b];
            int32_t g = Ghat[(int64_t)a * n + b];
            sum += g;
            if (g > mx) mx = g;
            float d = delta32(X, Y, a, b);
            int k = 15;
            while (k > 0 && !(d >= edge[k])) --k;
            hist[k]++;
        }
        double *f = F + 19 * (int64_t)a;
        f[0] = (double)deg / (double)(n - 1);
        f[1] = (double)sum / ((double)(n - 1) * (double)n);
        f[2] = (double)mx / (double)n;
        for (int k = 0; k < 16; ++k) f[3 + k] = (double)hist[k] / (double)(n - 1);
    }
    return 0;
}

/* tanh-form GELU (Hendrycks & Gimpel 2016) and its derivative. */
static double gelu(double x)
{
    const double c = 0.7978845608028654;   /* sqrt(2/pi) */
    return 0.5 * x * (1.0 + tanh(c * (x + 0.044715 * x * x * x)));
}

static double gelu_grad(double x)
{
    const double c = 0.7978845608028654;
    double u = c * (x + 0.044715 * x * x * x), th = tanh(u);
    return 0.5 * (1.0 + th) + 0.5 * x * (1.0 - th * th) * c * (1.0 + 3.0 * 0.044715 * x * x);
}

/* Forward pass of one sample; keeps pre-activations for the backward pass. */
static double mlp_one(const double *f, const double *W1, const double *b1, const double *W2,
                      const double *b2, const double *W3, const double *b3, int rnd,
                      double x[19], double z1[64], double a1[64], double z2[64], double a2[64])
{
    for (int k = 0; k < 19; ++k) x[k] = bf(f[k], rnd);
    for (int o = 0; o < 64; ++o) {
        double acc = b1[o];
        for (int k = 0; k < 19; ++k) acc += W1[19 * o + k] * x[k];
        z1[o] = acc;
        a1[o] = bf(gelu(acc), rnd);
    }
    for (int o = 0; o < 64; ++o) {
        double acc = b2[o];
        for (int k = 0; k < 64; ++k) acc += W2[64 * o + k] * a1[k];
        z2[o] = acc;
        a2[o] = bf(gelu(acc), rnd);
    }
    double s = b3[0];
    for (int k = 0; k < 64; ++k) s += W3[k] * a2[k];
    return s;
}

int tro_mlp_fwd(const double *F, int32_t n, const double *W1, const double *b1,
                const double *W2, const double *b2, const double *W3, const double *b3,
                double *s)
{
    if (!F || !W1 || !b1 || !W2 || !b2 || !W3 || !b3 || !s || n < 0) return -1;
    double x[19], z1[64], a1[64], z2[64], a2[64];
    for (int32_t r = 0; r < n; ++r)
        s[r] = mlp_one(F + 19 * (int64_t)r, W1, b1, W2, b2, W3, b3, 1, x, z1, a1, z2, a2);
    return 0;
}

/* Backward of the mean BCE-with-logits loss. rnd = 1 rounds stored values to
 * bfloat16 as the GPU does (rounding treated as identity in the backward);
 * rnd = 0 gives the exact float64 function for finite-difference checks. */
static int mlp_bwd_impl(const double *F, const uint8_t *labels, int32_t n,
                        const double *W1, const double *b1, const double *W2, const double *b2,
                        const double *W3, const double *b3,
                        double *gW1, double *gb1, double *gW2, double *gb2, double *gW3, double *gb3,
                        double *loss, int rnd)
{
    if (!F || !labels || n < 1) return -1;
    memset(gW1, 0, 64 * 19 * sizeof(double)); memset(gb1, 0, 64 * sizeof(double));
    memset(gW2, 0, 64 * 64 * sizeof(double)); memset(gb2, 0, 64 * sizeof(double));
    memset(gW3, 0, 64 * sizeof(double)); gb3[0] = 0;
    double L = 0;
    double x[19], z1[64], a1[64], z2[64], a2[64], dz2[64], dz1[64];
    for (int32_t r = 0; r < n; ++r) {
        double s = mlp_one(F + 19 * (int64_t)r, W1, b1, W2, b2, W3, b3, rnd, x, z1, a1, z2, a2);
        double y = labels[r] ? 1.0 : 0.0;
        L += (s > 0 ? s : 0.0) - s * y + log1p(exp(-fabs(s)));
        double ds = (1.0 / (1.0 + exp(-s)) - y) / (double)n;
        gb3[0] += ds;
        for (int k = 0; k < 64; ++k) { gW3[k] += ds * a2[k]; dz2[k] = ds * W3[k] * gelu_grad(z2[k]); }
        for (int o = 0; o < 64; ++o) {
            gb2[o] += dz2[o];
            for (int k = 0; k < 64; ++k) gW2[64 * o + k] += dz2[o] * a1[k];
        }
        for (int k = 0; k < 64; ++k) {
            double acc = 0;
            for (int o = 0; o < 64; ++o) acc += W2[64 * o + k] * dz2[o];
            dz1[k] = acc * gelu_grad(z1[k]);
        }
        for (int o = 0; o < 64; ++o) {
            gb1[o] += dz1[o];
            for (int k = 0; k < 19; ++k) gW1[19 * o + k] += dz1[o] * x[k];
        }
    }
    *loss = L / (double)n;
    return 0;
}

int tro_mlp_bwd(const double *F, const uint8_t *labels, int32_t n,
                const double *W1, const double *b1, const double *W2, const double *b2,
                const double *W3, const double *b3,
                double *gW1, double *gb1, double *gW2, double *gb2, double *gW3, double *gb3,
                double *loss)
{
    return mlp_bwd_impl(F, labels, n, W1, b1, W2, b2, W3, b3, gW1, gb1, gW2, gb2, gW3, gb3, loss, 1);
}

/* Same without bfloat16 rounding: the smooth function finite differences can check. */
int tro_mlp_bwd_exact(const double *F, const uint8_t *labels, int32_t n,
                      const double *W1, const double *b1, const double *W2, const double *b2,
                      const double *W3, const double *b3,
                      double *gW1, double *gb1, double *gW2, double *gb2, double *gW3, double *gb3,
                      double *loss)
{
    return mlp_bwd_impl(F, labels, n, W1, b1, W2, b2, W3, b3, gW1, gb1, gW2, gb2, gW3, gb3, loss, 0);
}

int tro_adam(double *w, const double *g, double *m, double *v, int64_t count, int32_t t,
             double lr, double beta1, double beta2, double eps)
{
    if (!w || !g || !m || !v || count < 0 || t < 1) return -1;
    double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t k = 0; k < count; ++k) {
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k];
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k];
        w[k] -= lr * (m[k] / c1) / (sqrt(v[k] / c2) + eps);
    }
    return 0;
}

typedef struct { float e; int32_t r; } lkey_t;

static int lkey_cmp(const void *a, const void *b)
{
    const lkey_t *x = (const lkey_t *)a, *y = (const lkey_t *)b;
    if (x->e != y->e) return x->e > y->e ? -1 : 1;
    return x->r < y->r ? -1 : (x->r > y->r);
}

/* Learned reorder of the plain pool: key e = s_i + s_j in float32, descending, ties by plain
 * rank; a non-finite score at either end of any valid pool pivot keeps the plain order and
 * reports the fallback (the scorer's output cannot be trusted for that pair). */
int tro_pivots_learned(const int32_t *P_plain, int32_t pool, const float *s, int32_t k1,
                       int32_t *P)
{
    if (!P_plain || !s || !P || pool < 0 || k1 < 0) return -1;
    int32_t valid = 0;
    while (valid < pool && P_plain[3 * valid] >= 0) ++valid;
    lkey_t *k = (lkey_t *)malloc(sizeof(lkey_t) * (size_t)(valid > 0 ? valid : 1));
    if (!k) return -3;
    int fallback = 0;
    for (int32_t r = 0; r < valid; ++r) {
        k[r].e = s[P_plain[3 * r]] + s[P_plain[3 * r + 1]];
        k[r].r = r;
        if (!isfinite(s[P_plain[3 * r]]) || !isfinite(s[P_plain[3 * r + 1]])) fallback = 1;
    }
    if (!fallback) qsort(k, (size_t)valid, sizeof(lkey_t), lkey_cmp);
    for (int32_t p = 0; p < k1; ++p) {
        if (p < valid) {
            int32_t r = fallback ? p : k[p].r;
            P[3 * p] = P_plain[3 * r]; P[3 * p + 1] = P_plain[3 * r + 1]; P[3 * p + 2] = P_plain[3 * r + 2];
        } else { P[3 * p] = -1; P[3 * p + 1] = -1; P[3 * p + 2] = 0; }
    }
    free(k);
    return fallback;
}

/* Threads the OpenMP loops above use (1 in the build without OpenMP). */
int tro_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
