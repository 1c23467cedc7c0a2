/* Host AddressSanitizer / UndefinedBehaviorSanitizer run of the CPU oracle:
 * every entry point on small inputs (ragged sizes, degenerate cliques, all
 * outliers, learned reorder, MLP forward/backward, Adam), with buffers sized
 * exactly as the header states, so any read or write outside them aborts.
 * Built and run by tests/test_asan_host.py; prints "ok" on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/turboreg_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double uniform(void)   /* splitmix64, top 53 bits */
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static void *xmalloc(size_t bytes)
{
    void *p = malloc(bytes ? bytes : 1);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
    return p;
}

/* n matches: the first n_in a rotation about z plus a shift, the rest uniform outliers */
static void make_pair(int n, int n_in, float *X, float *Y)
{
    const double c = cos(0.3), s = sin(0.3);
    for (int i = 0; i < n; ++i) {
        double x[3] = {3 * uniform() - 1.5, 3 * uniform() - 1.5, 3 * uniform() - 1.5};
        for (int k = 0; k < 3; ++k) X[3 * i + k] = (float)x[k];
        if (i < n_in) {
            Y[3 * i] = (float)(c * x[0] - s * x[1] + 0.2);
            Y[3 * i + 1] = (float)(s * x[0] + c * x[1] - 0.1);
            Y[3 * i + 2] = (float)(x[2] + 0.05);
        } else {
            for (int k = 0; k < 3; ++k) Y[3 * i + k] = (float)(3 * uniform() - 1.5);
        }
    }
}

static int check(int rc, const char *what)
{
    if (rc < 0) { fprintf(stderr, "%s failed (%d)\n", what, rc); exit(1); }
    return rc;
}

static void whole_path(int n, int n_in, int k1, int k2, int graph)
{
    float *X = xmalloc(sizeof(float) * 3 * n), *Y = xmalloc(sizeof(float) * 3 * n);
    make_pair(n, n_in, X, Y);
    tro_params p = {0.1f, 0.1f, k1, k2, graph};
    tro_result r;
    uint8_t *mask = xmalloc(n);
    check(tro_register(X, Y, n, &p, &r, mask), "tro_register");
    const int H = k1 * k2;
    int32_t *cl = xmalloc(sizeof(int32_t) * 3 * H), *fl = xmalloc(sizeof(int32_t) * H), *IN = xmalloc(sizeof(int32_t) * H);
    int32_t *piv = xmalloc(sizeof(int32_t) * 3 * k1);
    double *R = xmalloc(sizeof(double) * 9 * H), *t = xmalloc(sizeof(double) * 3 * H);
    float *sc = xmalloc(sizeof(float) * n);
    for (int i = 0; i < n; ++i) sc[i] = (float)uniform();
    check(tro_register_ex(X, Y, n, &p, 4, sc, NULL, &r, mask, cl, R, t, fl, IN, piv), "tro_register_ex");
    float *poses = xmalloc(sizeof(float) * 12 * H);
    for (int h = 0; h < H; ++h) {
        for (int k = 0; k < 9; ++k) poses[12 * h + k] = (float)R[9 * h + k];
        for (int k = 0; k < 3; ++k) poses[12 * h + 9 + k] = (float)t[3 * h + k];
    }
    check(tro_register_ex(X, Y, n, &p, 0, NULL, poses, &r, NULL, NULL, NULL, NULL, NULL, NULL, NULL), "poses_in");
    float *S = xmalloc(sizeof(float) * H);
    check(tro_score_metric(X, Y, n, poses, fl, H, 0.1f, 1, S), "tro_score_metric");
    (void)tro_select_score(S, H);
    /* per-step entry points, including features */
    uint8_t *C = xmalloc((size_t)n * n);
    int32_t *G = xmalloc(sizeof(int32_t) * n * n), *Gt = xmalloc(sizeof(int32_t) * n * n);
    int64_t b32, b64, flip;
    check(tro_compat(X, Y, n, 0.1f, C, &b32, &b64, &flip), "tro_compat");
    check(tro_sc2(C, n, G), "tro_sc2");
    check(tro_o2graph(G, n, Gt), "tro_o2graph");
    const int64_t np = check((int)tro_pivots(Gt, n, k1, piv), "tro_pivots");
    check(tro_cliques(Gt, n, piv, (int32_t)np, k1, k2, cl), "tro_cliques");
    double *F = xmalloc(sizeof(double) * 19 * n);
    check(tro_features(X, Y, n, 0.1f, C, G, F), "tro_features");
    free(X); free(Y); free(mask); free(cl); free(fl); free(IN); free(piv); free(R); free(t); free(sc);
    free(poses); free(S); free(C); free(G); free(Gt); free(F);
}

static void mlp(int n)
{
    double *F = xmalloc(sizeof(double) * 19 * n), *s = xmalloc(sizeof(double) * n);
    uint8_t *lab = xmalloc(n);
    const int np = 64 * 19 + 64 + 64 * 64 + 64 + 64 + 1;
    double *w = xmalloc(sizeof(double) * np), *g = xmalloc(sizeof(double) * np);
    double *m = calloc(np, sizeof(double)), *v = calloc(np, sizeof(double)), loss = 0;
    for (int i = 0; i < 19 * n; ++i) F[i] = uniform();
    for (int i = 0; i < n; ++i) lab[i] = uniform() < 0.3;
    for (int i = 0; i < np; ++i) w[i] = 0.2 * (uniform() - 0.5);
    double *W1 = w, *b1 = W1 + 64 * 19, *W2 = b1 + 64, *b2 = W2 + 64 * 64, *W3 = b2 + 64, *b3 = W3 + 64;
    double *gW1 = g, *gb1 = gW1 + 64 * 19, *gW2 = gb1 + 64, *gb2 = gW2 + 64 * 64, *gW3 = gb2 + 64, *gb3 = gW3 + 64;
    check(tro_mlp_fwd(F, n, W1, b1, W2, b2, W3, b3, s), "tro_mlp_fwd");
    check(tro_mlp_bwd(F, lab, n, W1, b1, W2, b2, W3, b3, gW1, gb1, gW2, gb2, gW3, gb3, &loss), "tro_mlp_bwd");
    check(tro_mlp_bwd_exact(F, lab, n, W1, b1, W2, b2, W3, b3, gW1, gb1, gW2, gb2, gW3, gb3, &loss), "bwd_exact");
    for (int t = 1; t <= 3; ++t) check(tro_adam(w, g, m, v, np, t, 1e-3, 0.9, 0.999, 1e-8), "tro_adam");
    int32_t P[30], Pl[30];
    float sc[8];
    for (int k = 0; k < 10; ++k) { P[3 * k] = k % 8; P[3 * k + 1] = (k + 3) % 8; P[3 * k + 2] = 10 - k; }
    for (int k = 0; k < 8; ++k) sc[k] = (float)uniform();
    check(tro_pivots_learned(P, 10, sc, 10, Pl), "tro_pivots_learned");
    free(F); free(s); free(lab); free(w); free(g); free(m); free(v);
}

int main(void)
{
    const int sizes[] = {3, 4, 5, 17, 64, 65, 130};
    for (unsigned k = 0; k < sizeof(sizes) / sizeof(sizes[0]); ++k) {
        const int n = sizes[k];
        whole_path(n, n / 2, 40, 2, 0);
        whole_path(n, n, 7, 3, 1);
        whole_path(n, 0, 5, 1, 0);   /* all outliers */
    }
    float Xc[9] = {0, 0, 0, 1, 1, 1, 2, 2, 2}, Yc[9] = {0, 1, 0, 2, 0, 1, 1, 1, 1};
    int32_t cl[6] = {0, 1, 2, 0, 1, -1}, fl[2];
    double R[18], t[6];
    check(tro_kabsch(Xc, Yc, cl, 2, R, t, fl), "tro_kabsch degenerate");
    mlp(37);
    printf("ok\n");
    return 0;
}
