/*
 * turboreg.h -- C ABI of the MI355X (gfx950) TurboReg robust-estimation library.
 *
 * TurboReg (Yan et al., ICCV 2025, arXiv 2507.01439) estimates a rigid pose
 * T = (R, t) from N putative point matches m_i = (x_i, y_i) (Section 3.1):
 *   1. compatibility graph C_ij = [ | |x_i-x_j| - |y_i-y_j| | <= tau ]   (Eq. 1)
 *   2. SC2 weights Ghat = C o (C C); O2Graph keeps i < j                  (Eq. 2, Def. 2)
 *   3. the K1 heaviest edges are the pivots                                (Eq. 4)
 *   4. per pivot, the K2 best third vertices form TurboCliques             (Eqs. 5-8, Alg. 1-2)
 *   5. one Kabsch pose per clique; the pose with most inliers wins         (Section 3.5, Eq. 9)
 *
 * Conventions for every entry point:
 *   - Points are N x 3 float32, row-major (x, y, z per match), in DEVICE memory.
 *   - All device buffers are caller-owned; the library never frees them.
 *   - Work is enqueued on the caller's HIP stream and is asynchronous. The
 *     return value reports only errors the host can see synchronously (bad
 *     arguments, sizes beyond the handle's limits, HIP launch failures).
 *     Data-dependent outcomes are written to tr_result.status on the device.
 *   - A handle owns a workspace sized at tr_create; it is not thread-safe and
 *     calls on one handle must be ordered (one stream, or synchronised).
 */
#ifndef TURBOREG_H
#define TURBOREG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TR_MAX_K2 8          /* largest supported K2 (cliques per pivot)              */
#define TR_SC2_SPARSE_CAP_MAX 8192   /* largest tr_tuning.sc2_sparse_cap               */
#define TR_NOALLOC_MAX_N 2048        /* largest n of tr_register_noalloc                */
#define TR_NOALLOC_MAX_K1 1024       /* largest k1 of tr_register_noalloc               */
#define TR_NOALLOC_SCRATCH_BYTES (13u << 20)   /* its static workspace per device       */
#define TR_MAX_POOL 16384    /* largest pivot list one workgroup sorts (K1 or pool)  */
#define TR_MLP_IN 19         /* learned scorer: features per correspondence           */
#define TR_MLP_HID 64        /* learned scorer: hidden width                          */
#define TR_MLP_NPARAM (64 * 19 + 64 + 64 * 64 + 64 + 64 + 1)   /* 5505 float32 parameters */

typedef enum {
    TR_OK = 0,
    TR_ERR_INVALID_ARG = 1,     /* bad argument (host) or pair with N < 3 / N > max_n (device) */
    TR_ERR_NONFINITE = 2,       /* device: some input coordinate is NaN/Inf (those matches get no edge) */
    TR_ERR_NO_HYPOTHESIS = 3,   /* device: no valid TurboClique; R = I, t = 0, mask all zero */
    TR_ERR_WORKSPACE = 4,       /* host: request exceeds the handle's limits; create a larger handle */
    TR_ERR_HIP = 5,             /* host: a HIP call failed */
    TR_WARN_SCORER_FALLBACK = 6,/* device: learned scores not finite; plain SC2 pivots were used */
    TR_ERR_NO_SCORER = 7,       /* host: learned pivots requested but no weights are loaded */
    TR_ERR_BAD_BLOB = 8         /* host: scorer weights blob has a wrong size, magic or checksum */
} tr_status;

enum { TR_GRAPH_O2 = 0, TR_GRAPH_SC2 = 1 };          /* Definition 2 / undirected SC2 graph */
enum { TR_PIVOTS_PLAIN = 0, TR_PIVOTS_LEARNED = 1 };
enum {
    TR_FLAG_PROFILE = 1u,       /* record per-stage HIP events; read with tr_stage_times          */
    TR_FLAG_PROFILE_SC2 = 2u,   /* record only the two events around the SC2 kernel (its launch  */
                                /* duration, least perturbation); ignored with TR_FLAG_PROFILE   */
    /* Selection by an error-based score instead of the inlier number (the ranking study of the
     * paper's supplementary Table 6). Over the inliers of Eq. 9 (r^2 <= theta^2), with
     * e = sqrt(r^2) and u = max(0, (theta - e) / theta) in float32, the score is the sum of u (MAE form)
     * or of u*u (MSE form), summed in float32; the largest score wins (lowest h on ties).
     * best_inliers is still the selected hypothesis's inlier number. At most one of the two;
     * either needs theta > 0 (TR_ERR_INVALID_ARG otherwise). */
    TR_FLAG_RANK_MAE = 4u,
    TR_FLAG_RANK_MSE = 8u
};

typedef struct {
    float tau;            /* compatibility threshold, metres; Eq. 1 uses "<="                    */
    float inlier_thresh;  /* theta: a match is an inlier of T when |R x + t - y| <= theta (Eq. 9) */
    int32_t k1;           /* pivots (Eq. 4), >= 1                                                  */
    int32_t k2;           /* TurboCliques per pivot (Eq. 7), 1..TR_MAX_K2                          */
    int32_t graph;        /* TR_GRAPH_O2 (default) or TR_GRAPH_SC2                                 */
    int32_t pivot_mode;   /* TR_PIVOTS_PLAIN or TR_PIVOTS_LEARNED                                  */
    int32_t pool_factor;  /* learned mode: reorder the first pool_factor*k1 plain pivots (>= 1)    */
    uint32_t flags;       /* TR_FLAG_*                                                             */
} tr_params;

/* Per-pair result, written on the device (80 bytes). */
typedef struct {
    float R[9];                /* row-major rotation of the selected hypothesis                   */
    float t[3];
    int32_t best_inliers;      /* inlier number of the selected hypothesis (Eq. 9)                */
    int32_t best_hyp;          /* its index h = s*K1 + p (Algorithm 2 layout), -1 if none          */
    int32_t n_valid_hyp;       /* hypotheses from valid cliques                                   */
    int32_t status;            /* tr_status                                                       */
    int32_t n_boundary_pairs;  /* pairs i<j with |delta_ij - tau| < 1e-6 m (float32), reported only */
    int32_t n_pivots;          /* pivots selected: min(K1, N(N-1)/2)                               */
    int32_t n_edges;           /* compatible pairs i<j                                             */
    int32_t reserved;
} tr_result;

typedef struct tr_handle tr_handle;

/* Create a handle on `device` whose workspace holds up to `max_batch` pairs of
 * up to `max_n` matches, K1 <= max_k1 and K2 <= max_k2. Learned mode needs
 * pool_factor*K1 <= min(8*max_k1, TR_MAX_POOL). Allocates device memory
 * (about 2.5 * max_batch * round_up(max_n,256)^2 bytes for C and the SC2 weights, plus about
 * max_batch * (80 * min(8*max_k1, TR_MAX_POOL) + 70 * max_k1 * max_k2) bytes for the pivot pool,
 * the hypotheses and their counters); max_n <= 32767. *out is NULL on error. */
tr_status tr_create(tr_handle **out, int32_t max_n, int32_t max_batch, int32_t max_k1,
                    int32_t max_k2, int32_t device);
tr_status tr_destroy(tr_handle *h);

/* Register one pair: src, dst are N x 3 float32 device arrays; out_dev is one
 * tr_result in device memory; mask_dev (nullable) receives N uint8 inlier flags
 * under the selected pose. `stream` is a hipStream_t (NULL = default stream). */
tr_status tr_register(tr_handle *h, const float *src, const float *dst, int32_t n,
                      const tr_params *p, tr_result *out_dev, uint8_t *mask_dev, void *stream);

/* Register one pair with no allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid it): the same
 * launch sequence as tr_register with its default launch configuration, on the calling
 * thread's current device, but its workspace is a fixed static device array of
 * TR_NOALLOC_SCRATCH_BYTES per device (held until the process ends), so no handle is needed.
 * Limits: 3 <= n <= TR_NOALLOC_MAX_N, k1 <= TR_NOALLOC_MAX_K1, k2 <= TR_MAX_K2 (larger ->
 * TR_ERR_WORKSPACE); plain pivots only and no TR_FLAG_PROFILE* flags (TR_ERR_INVALID_ARG).
 * The first call on a device resolves the array's address there and may return TR_ERR_HIP.
 * Every call on one device shares that device's array: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller. The kernels clear every
 * counter they use at the start of each call, so no state carries over between calls.
 * Arguments as tr_register; outputs are bit-identical to tr_register's on the same inputs. */
tr_status tr_register_noalloc(const float *src, const float *dst, int32_t n, const tr_params *p,
                              tr_result *out_dev, uint8_t *mask_dev, void *stream);

/* Register B pairs of uneven size in one pass. Pair b owns matches
 * [offsets[b], offsets[b+1]) of src/dst; offsets_dev is B+1 int32 in device
 * memory, non-decreasing, every N_b <= max_n (host-side bound, <= the handle's).
 * A pair with N_b < 3 or N_b > max_n gets status TR_ERR_INVALID_ARG. out_dev is
 * B results; masks_dev (nullable) is offsets[B] uint8. On a stream other than the
 * legacy default one, the launch sequence is captured once into a hipGraph per
 * (pointers, stream, B, max_n, params) and replayed; a handle keeps the 8 most recently
 * launched graphs, and a call that must evict one first waits for the whole device. */
tr_status tr_register_batch(tr_handle *h, const float *src, const float *dst,
                            const int32_t *offsets_dev, int32_t B, int32_t max_n,
                            const tr_params *p, tr_result *out_dev, uint8_t *masks_dev,
                            void *stream);

/* Rigid fits of caller-given triplets of match indices (T x 3 int32 device array) of one pair
 * (N x 3 src, dst device arrays), by the registration's own 3-point fit (Section 3.5: Horn's
 * quaternion form in float64, rounded to float32): poses_dev receives T x 12 float32 (R
 * row-major, then t), ok_dev T int32 (1 = a well-posed fit; 0 = degenerate triplet or an
 * index outside [0, n), with the identity pose). For studies of the fits themselves, such as
 * 3-point against larger-clique estimates. TR_ERR_INVALID_ARG for n < 3 or T < 0. */
tr_status tr_fit_triplets(tr_handle *h, const float *src, const float *dst, int32_t n, const int32_t *triplets_dev,
                          int32_t T, float *poses_dev, int32_t *ok_dev, void *stream);

/* Score caller-given poses against one pair (N x 3 src, dst device arrays): for each of the P
 * poses (P x 12 float32 device array, R row-major then t) its inlier number (Eq. 9, the same
 * float32 test as the registration) into in_dev (P int32), and for metric 1 (MAE form) or 2
 * (MSE form) its error-based score into score_dev (P float32; may be NULL for metric 0), both
 * computed in the same arithmetic and order as the registration's hypothesis scoring, so a
 * hypothesis pose scores the same bits. For evaluating external poses (a ground-truth
 * transformation, poses from another method). TR_ERR_INVALID_ARG for n < 1, P < 0, a negative
 * or non-finite theta, theta = 0 with metric 1 or 2, metric outside 0..2 or a missing score
 * buffer. */
tr_status tr_score_poses(tr_handle *h, const float *src, const float *dst, int32_t n, const float *poses_dev,
                         int32_t P, float theta, int32_t metric, int32_t *in_dev, float *score_dev, void *stream);

/* ---- launch configuration and autotuner ----
 * Calls are grouped by shape: the number of 256-row tiles of their largest
 * pair, round_up(max_n, 256) / 256, and the batch size B (1 for tr_register).
 * Each group has a launch configuration; a group never tuned or set uses the
 * defaults (5, 8, 4 for one pair or 16 for a batch, 4, 0). No configuration
 * changes any result: C, weights, pivots, cliques, poses, inlier numbers and
 * the selection are the same under every valid configuration. */
typedef struct {
    int32_t sc2_super;      /* SC2 tile walk: side of the super-tiles (in 256 x 256
                               output tiles) whose tiles run close together, 1..16  */
    int32_t compat_per_cu;  /* compatibility work items launched per CU, 1..16     */
    int32_t hyp_ppw;        /* pivots per hypothesis work item: 4, 8, 12 or 16     */
    int32_t hyp_per_cu;     /* hypothesis workgroups launched per CU, 1..16        */
    int32_t sc2_sparse_cap; /* SC2 output tiles (256 x 256) with at most this many
                               edges count common neighbours per edge from bit rows
                               instead of the dense product; 0 = every tile takes
                               the product. 0..TR_SC2_SPARSE_CAP_MAX             */
} tr_tuning;

/* Configuration of the group of (max_n, B). TR_ERR_INVALID_ARG for max_n < 3, B < 1. */
tr_status tr_tuning_get(tr_handle *h, int32_t max_n, int32_t B, tr_tuning *out);
/* Set the configuration of the group of (max_n, B); TR_ERR_INVALID_ARG if a
 * field is outside its range. Later calls of that group use it (batches on a
 * stream capture a new hipGraph for it). */
tr_status tr_tuning_set(tr_handle *h, int32_t max_n, int32_t B, const tr_tuning *t);
/* Persist the launch configurations of a handle: tr_tuning_save writes every
 * group the handle holds (tuned or set) to a text file: a header line
 * "turboreg-tuning <version> <gcn arch name> <CU count>", then one line per group
 * "<256-row tiles> <B> <sc2_super> <compat_per_cu> <hyp_ppw> <hyp_per_cu>
 * <sc2_sparse_cap>". tr_tuning_load reads such a file into the handle, replacing
 * the groups it names; a file of another version, architecture or CU count, or
 * with a malformed or out-of-range line, is refused (TR_ERR_INVALID_ARG) and
 * changes nothing. I/O failures are TR_ERR_INVALID_ARG too. tr_create loads the
 * file named by the environment variable TURBOREG_TUNING_CACHE when it is set
 * and readable (a refused file is ignored there). */
tr_status tr_tuning_save(tr_handle *h, const char *path);
tr_status tr_tuning_load(tr_handle *h, const char *path);

/* Autotuner: runs the registration of the given inputs (one pair of N = max_n
 * if offsets_dev is NULL and B == 1, else the batch as tr_register_batch) under
 * candidate configurations, one field at a time starting from the group's
 * current one (hyp_ppw, hyp_per_cu, sc2_super, compat_per_cu, sc2_sparse_cap), each candidate
 * timed by HIP events on `stream` as the fastest of three batches of eight runs after one
 * warm-up, with the incumbent timed again beside it, keeps a candidate only if it is at
 * least 2% faster, stores the result for the group
 * and writes it to *best (nullable) with its time per registration call in
 * *best_ms (nullable). Runs eagerly and synchronises the stream; out_dev and
 * masks_dev receive the results of the last run. Same argument errors as the
 * registration calls. */
tr_status tr_autotune(tr_handle *h, const float *src, const float *dst, const int32_t *offsets_dev,
                      int32_t B, int32_t max_n, const tr_params *p, tr_result *out_dev,
                      uint8_t *masks_dev, void *stream, tr_tuning *best, float *best_ms);

/* ---- learned pivot scorer (MLP 19 -> 64 -> 64 -> 1, GELU, bfloat16) ---- */

/* Load weights from a host blob written by tr_scorer_save: "TRMLP001", then
 * TR_MLP_NPARAM float32 (W1 64x19, b1, W2 64x64, b2, W3 1x64, b3; row-major,
 * out x in), then an FNV-1a 64-bit checksum of those bytes. */
tr_status tr_scorer_load(tr_handle *h, const void *blob, size_t bytes);
/* Write the current float32 master weights in that format; *written = the
 * blob size. blob == NULL with written != NULL is a size query (TR_OK);
 * capacity below the blob size is TR_ERR_INVALID_ARG. */
tr_status tr_scorer_save(tr_handle *h, void *blob, size_t capacity, size_t *written);
/* Set weights from TR_MLP_NPARAM host float32 values (same order) and reset Adam state. */
tr_status tr_scorer_set(tr_handle *h, const float *params_host);
/* Copy the float32 master weights to the host. */
tr_status tr_scorer_get(tr_handle *h, float *params_host);

/* Per-correspondence features of the learned pivot scorer: for
 * each pair of a batch, N_b x 19 bfloat16 values (uint16 bit patterns) into
 * feat_dev at row offsets[b]. Runs compatibility and SC2 on the way. */
tr_status tr_features_batch(tr_handle *h, const float *src, const float *dst,
                            const int32_t *offsets_dev, int32_t B, int32_t max_n,
                            const tr_params *p, uint16_t *feat_dev, void *stream);

/* MLP forward: M x 19 bfloat16 features -> M float32 logits. */
tr_status tr_mlp_forward(tr_handle *h, const uint16_t *feat_dev, int64_t m, float *scores_dev,
                         void *stream);

/* Gradients of the mean BCE-with-logits loss over M samples (labels uint8 0/1)
 * at the current weights: grads_dev receives TR_MLP_NPARAM float32 in weight
 * order, loss_dev (nullable) one float32. */
tr_status tr_mlp_grads(tr_handle *h, const uint16_t *feat_dev, const uint8_t *labels_dev,
                       int64_t m, float *grads_dev, float *loss_dev, void *stream);

/* One training step: gradients as tr_mlp_grads, then Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8) on the float32 master weights and a bfloat16 refresh. */
tr_status tr_train_step(tr_handle *h, const uint16_t *feat_dev, const uint8_t *labels_dev,
                        int64_t m, float lr, float *loss_dev, void *stream);

/* ---- inspection ---- */

enum {
    TR_TAP_C = 0,         /* N x N uint8 compatibility matrix                          */
    TR_TAP_G = 1,         /* N x N uint16 O2Graph weights (i < j; the tap zeroes j <= i) */
    TR_TAP_PIVOTS = 2,    /* k1 x 3 int32 (i, j, w): the pivots the cliques used (learned
                             pivots in learned mode), (-1, -1, 0) past the last     */
    TR_TAP_CLIQUES = 3,   /* H x 3 int32 (i, j, z), H = k1*k2, slot-major, z = -1 empty  */
    TR_TAP_POSES = 4,     /* H x 12 float32 (R row-major, t)                           */
    TR_TAP_IN = 5,        /* H int32 inlier numbers, -1 for an invalid hypothesis      */
    TR_TAP_FEATURES = 6,  /* N x 19 uint16 bfloat16 features (learned mode; only rows that
                             are endpoints of the plain pool's pivots are written, the
                             others keep older values)                                 */
    TR_TAP_SCORES = 7,    /* N float32 learned scores (learned mode; same rows as above)  */
    TR_TAP_PLAIN_PIVOTS = 8, /* pool x 3 int32 plain pivots before the learned reorder */
    TR_TAP_RANK_SCORES = 9  /* H float32 error-based scores (TR_FLAG_RANK_* calls only), -1
                               for an invalid hypothesis                                 */
};

/* Synchronise the handle's last stream and copy intermediate `tap` of pair
 * `pair` of the last call into host memory (dense layout above). Returns
 * TR_ERR_INVALID_ARG if `bytes` is too small; *needed (nullable) = size. */
tr_status tr_debug_copy(tr_handle *h, int32_t tap, int32_t pair, void *host_dst, size_t bytes,
                        size_t *needed);

enum { TR_STAGE_PLAN = 0, TR_STAGE_COMPAT, TR_STAGE_SC2, TR_STAGE_PIVOTS, TR_STAGE_LEARNED,
       TR_STAGE_CLIQUES, TR_STAGE_KABSCH, TR_STAGE_SCORE, TR_STAGE_SELECT, TR_NUM_STAGES };

/* Average milliseconds per stage over the calls made with TR_FLAG_PROFILE
 * (every stage) or TR_FLAG_PROFILE_SC2 (the SC2 stage only; 0 elsewhere unless
 * other calls recorded them) since the previous read (HIP events recorded on each call's stream, kept in
 * a ring so profiled calls never wait on the host). Synchronises those events
 * and resets the averages. TR_ERR_INVALID_ARG if no profiled call was made.
 * count <= TR_NUM_STAGES. Events open only stages that launch a kernel: PLAN is
 * 0 for single-pair calls (no planner) and LEARNED is 0 with plain pivots.
 * Clique search, rigid fits, scoring and selection run in one kernel: its event
 * interval is split into CLIQUES (clique search), KABSCH (fits), SCORE (inlier
 * numbers and per-item records) and SELECT (argmax, result and mask) by the
 * shares of its workgroups' time in each phase, from in-kernel clock stamps of
 * the profiled calls. */
tr_status tr_stage_times(tr_handle *h, float *ms, int32_t count);

const char *tr_status_string(int32_t status);

#ifdef __cplusplus
}
#endif
#endif
