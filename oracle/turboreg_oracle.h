/*
 * TurboReg CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct host implementation of the TurboReg
 * robust-estimation path (Yan et al., "TurboReg: TurboClique for Robust and
 * Efficient Point Cloud Registration", ICCV 2025). Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it. The product
 * path (the HIP library) never links, loads or calls it, and it shares no code
 * with that path.
 *
 * Conventions: indices are 0-based (the paper's are 1-based); points are N x 3
 * float32 row-major; matrices are N x N row-major; every buffer is owned by the
 * caller. Functions return 0 on success and a negative value on bad arguments.
 */
#ifndef TURBOREG_ORACLE_H
#define TURBOREG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Eq. 1: C_ij = [ | |x_i-x_j| - |y_i-y_j| | <= tau ], C_ii = 0, decided in
 * float32 with a fixed operation order (see the source). Also reports
 *   n_boundary32 = #{i<j : |delta32 - tau| < 1e-6}  (float32 arithmetic)
 *   n_boundary64 = #{i<j : |delta64 - tau| < 1e-6}  (float64 shadow)
 *   n_flip       = #{i<j : float64 decision != float32 decision}
 * Any of the three count pointers may be NULL. */
int tro_compat(const float *X, const float *Y, int32_t n, float tau, uint8_t *C,
               int64_t *n_boundary32, int64_t *n_boundary64, int64_t *n_flip);

/* Eq. 2: Ghat_ij = C_ij * sum_k C_ik C_jk (symmetric, int32, N x N). */
int tro_sc2(const uint8_t *C, int32_t n, int32_t *Ghat);

/* Definition 2: Gt_ij = Ghat_ij if i < j else 0. In-place allowed. */
int tro_o2graph(const int32_t *Ghat, int32_t n, int32_t *Gt);

/* Eq. 4: pivots = the first min(k1, N(N-1)/2) pairs i<j ordered by
 * (Gbar_ij desc, i asc, j asc). P is k1 x 3 (i, j, w); rows past the returned
 * count are set to (-1, -1, 0). Returns the number of pivots. */
int64_t tro_pivots(const int32_t *Gbar, int32_t n, int32_t k1, int32_t *P);

/* Eqs. 5-8 / Algorithm 1: for each pivot p = (i, j) the third vertices z not in
 * {i, j} with Gbar_ij * Gbar_iz * Gbar_jz > 0, scored S = Gbar_ij + Gbar_iz +
 * Gbar_jz; keep the first k2 by (S desc, z asc). Output slot-major (Algorithm 2
 * layout): row h = s * k1 + p of `cliques` (k1*k2 x 3 int32) holds (i, j, z);
 * an empty slot has z = -1 (and i = j = -1 when pivot p does not exist). */
int tro_cliques(const int32_t *Gbar, int32_t n, const int32_t *P, int32_t n_pivots,
                int32_t k1, int32_t k2, int32_t *cliques);

/* Section 3.5: least-squares rigid fit (Kabsch) to the three matches of every
 * valid clique, in float64. R is H x 9 (row-major), t is H x 3. flags[h] is
 * 0 for an invalid clique (R = I, t = 0), 1 for a well-conditioned fit, 2 when
 * sigma_2 <= 1e-9 sigma_1 (collinear or coincident points: R not unique). */
int tro_kabsch(const float *X, const float *Y, const int32_t *cliques, int32_t H,
               double *R, double *t, int32_t *flags);

/* Eq. 9, g = inlier number: IN_h = #{n : |R_h x_n + t_h - y_n|^2 <= theta^2}
 * evaluated in float32 with a fixed operation order on float32 poses
 * (H x 12: R row-major then t). IN_h = -1 where valid[h] == 0. */
int tro_score(const float *X, const float *Y, int32_t n, const float *poses,
              const int32_t *valid, int32_t H, float theta, int32_t *IN);

/* Inlier mask of one float32 pose under the same arithmetic as tro_score. */
int tro_mask(const float *X, const float *Y, int32_t n, const float *pose, float theta,
             uint8_t *mask);

/* argmax_h IN_h, lowest h among ties; -1 if no IN_h >= 0. */
int32_t tro_select(const int32_t *IN, int32_t H);
/* Error-based scores of valid hypotheses (metric 1 = MAE, 2 = MSE; larger is better, -1 if
 * invalid) and their argmax (lowest h on ties, -1 if none is valid). */
int tro_score_metric(const float *X, const float *Y, int32_t n, const float *poses,
                     const int32_t *valid, int32_t H, float theta, int32_t metric, float *S);
int32_t tro_select_score(const float *S, int32_t H);

typedef struct {
    float tau, theta;
    int32_t k1, k2;
    int32_t graph;   /* 0 = O2Graph (Definition 2), 1 = undirected SC2 graph */
} tro_params;

typedef struct {
    double R[9], t[3];          /* float64 fit of the selected clique */
    float R32[9], t32[3];       /* the float32 pose that was scored */
    int32_t best_inliers, best_hyp, n_valid_hyp, status;
    int64_t n_boundary32, n_boundary64, n_flip;
    int64_t n_pivots;
} tro_result;

/* Whole path: compat -> SC2 -> O2Graph -> pivots -> cliques -> Kabsch (float64)
 * -> round poses to float32 -> score -> select -> mask. status 0 = ok,
 * 3 = no valid hypothesis (R = I, t = 0). mask may be NULL. */
int tro_register(const float *X, const float *Y, int32_t n, const tro_params *p,
                 tro_result *out, uint8_t *mask);
/* The same path with three options. scores (nullable, N float32): select the first
 * pool_factor*k1 plain pivots and reorder them by the learned keys (tro_pivots_learned) before
 * the cliques. poses_in (nullable, H x 12 float32): score and select on these poses instead of
 * the float32 rounding of the path's own fits (inlier numbers are defined on identical float32
 * poses). The nullable outputs receive every hypothesis's clique (H x 3), float64 fit
 * (H x 9, H x 3), fit flag (H), inlier number (H) and the pivots used (k1 x 3). */
int tro_register_ex(const float *X, const float *Y, int32_t n, const tro_params *p, int32_t pool_factor,
                    const float *scores, const float *poses_in, tro_result *out, uint8_t *mask,
                    int32_t *cliques_out, double *R_out, double *t_out, int32_t *flags_out,
                    int32_t *IN_out, int32_t *pivots_out);

/* ---- learned pivot scorer (float64 reference) ---- */

/* 19 features per correspondence n: deg_n/(N-1); mean_{j!=n} Ghat_nj / N;
 * max_j Ghat_nj / N; 16-bin histogram of delta_nj (j != n) with float32 bin
 * edges e_k = k * (tau/4), bin = max{k : delta >= e_k}, each count / (N-1).
 * delta is the float32 value of Eq. 1. F is N x 19 float64. */
int tro_features(const float *X, const float *Y, int32_t n, float tau,
                 const uint8_t *C, const int32_t *Ghat, double *F);

/* MLP 19 -> 64 -> 64 -> 1 with tanh-form GELU. Inputs, weights and hidden
 * activations are rounded to bfloat16 (round to nearest even) where the GPU
 * stores them; arithmetic in float64. W1 64x19, W2 64x64, W3 1x64 row-major
 * (out x in); b1 64, b2 64, b3 1. */
int tro_mlp_fwd(const double *F, int32_t n, const double *W1, const double *b1,
                const double *W2, const double *b2, const double *W3, const double *b3,
                double *s);

/* Mean binary cross-entropy with logits over n samples and its gradients
 * (same shapes as the weights). Returns the loss through *loss. */
int tro_mlp_bwd(const double *F, const uint8_t *labels, int32_t n,
                const double *W1, const double *b1, const double *W2, const double *b2,
                const double *W3, const double *b3,
                double *gW1, double *gb1, double *gW2, double *gb2, double *gW3, double *gb3,
                double *loss);

/* As tro_mlp_bwd with no bfloat16 rounding anywhere: the smooth float64
 * function that central finite differences can check. */
int tro_mlp_bwd_exact(const double *F, const uint8_t *labels, int32_t n,
                      const double *W1, const double *b1, const double *W2, const double *b2,
                      const double *W3, const double *b3,
                      double *gW1, double *gb1, double *gW2, double *gb2, double *gW3, double *gb3,
                      double *loss);

/* One Adam step (Kingma & Ba 2015) on `count` parameters, step number t >= 1. */
int tro_adam(double *w, const double *g, double *m, double *v, int64_t count, int32_t t,
             double lr, double beta1, double beta2, double eps);

/* Learned pivot order: from the first `pool` plain pivots (k x 3), order by
 * e = fl32(s_i + s_j) desc, ties by plain rank, and keep the first k1. */
int tro_pivots_learned(const int32_t *P_plain, int32_t pool, const float *s, int32_t k1,
                       int32_t *P);

/* float -> bfloat16 -> float, round to nearest even (NaN kept NaN). */
float tro_bf16_round(float x);

/* Threads the parallel loops use: omp_get_max_threads() in the OpenMP build, else 1. */
int tro_threads(void);

#ifdef __cplusplus
}
#endif
#endif
