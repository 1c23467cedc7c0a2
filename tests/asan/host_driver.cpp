// Host AddressSanitizer run of the library's host code (the HIP kernels are
// not instrumented): argument checking without a device, then, when a GPU is
// present, every entry point once on a small synthetic pair, so a host-side
// read or write outside a buffer, a use after free or a leak of host memory
// in the library aborts the run. Built by the package's build step
// (_build_asan/host_driver) and run by tests/test_asan_host.py; prints "ok".
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/turboreg.h"

namespace {

int failures = 0;

void expect(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

void expect_status(tr_status got, tr_status want, const char *what)
{
    if (got != want) {
        std::fprintf(stderr, "FAILED: %s: status %d (%s), expected %d\n", what, (int)got, tr_status_string(got),
                     (int)want);
        ++failures;
    }
}

// n matches, the first n_in a rigid motion of their sources, the rest uniform outliers (LCG draws)
void make_pair(int n, int n_in, std::vector<float> &X, std::vector<float> &Y, uint64_t seed)
{
    uint64_t s = seed;
    auto u = [&]() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(s >> 11) * (1.0 / 9007199254740992.0);
    };
    X.resize(3 * n);
    Y.resize(3 * n);
    const double c = std::cos(0.4), sn = std::sin(0.4);
    for (int i = 0; i < n; ++i) {
        const double x[3] = {3 * u() - 1.5, 3 * u() - 1.5, 3 * u() - 1.5};
        for (int k = 0; k < 3; ++k) X[3 * i + k] = (float)x[k];
        if (i < n_in) {
            Y[3 * i] = (float)(c * x[0] - sn * x[1] + 0.3);
            Y[3 * i + 1] = (float)(sn * x[0] + c * x[1]);
            Y[3 * i + 2] = (float)(x[2] - 0.2);
        } else {
            for (int k = 0; k < 3; ++k) Y[3 * i + k] = (float)(3 * u() - 1.5);
        }
    }
}

template <typename T>
T *dev_copy(const std::vector<T> &v)
{
    T *p = nullptr;
    if (hipMalloc(&p, v.size() * sizeof(T)) != hipSuccess) std::abort();
    if (hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) std::abort();
    return p;
}

void without_device()
{
    tr_params p{0.1f, 0.1f, 10, 2, TR_GRAPH_O2, TR_PIVOTS_PLAIN, 4, 0};
    float x[9] = {0};
    tr_handle *h = nullptr;
    expect_status(tr_create(nullptr, 100, 1, 10, 2, 0), TR_ERR_INVALID_ARG, "tr_create(null)");
    expect_status(tr_create(&h, 2, 1, 10, 2, 0), TR_ERR_INVALID_ARG, "tr_create(max_n 2)");
    expect_status(tr_create(&h, 100, 0, 10, 2, 0), TR_ERR_INVALID_ARG, "tr_create(max_batch 0)");
    expect_status(tr_create(&h, 100, 1, 10, TR_MAX_K2 + 1, 0), TR_ERR_INVALID_ARG, "tr_create(k2)");
    expect(h == nullptr, "no handle after failed creates");
    expect_status(tr_destroy(nullptr), TR_ERR_INVALID_ARG, "tr_destroy(null)");
    expect_status(tr_register(nullptr, x, x, 3, &p, nullptr, nullptr, nullptr), TR_ERR_INVALID_ARG, "register(null)");
    expect_status(tr_register_noalloc(x, x, 2, &p, nullptr, nullptr, nullptr), TR_ERR_INVALID_ARG, "noalloc(n 2)");
    tr_params big = p;
    big.k1 = TR_NOALLOC_MAX_K1 + 1;
    expect_status(tr_register_noalloc(x, x, 10, &big, (tr_result *)x, nullptr, nullptr), TR_ERR_WORKSPACE,
                  "noalloc(k1)");
    expect_status(tr_scorer_load(nullptr, x, sizeof(x)), TR_ERR_INVALID_ARG, "scorer_load(null)");
    expect_status(tr_tuning_load(nullptr, "x"), TR_ERR_INVALID_ARG, "tuning_load(null)");
    expect_status(tr_tuning_save(nullptr, "x"), TR_ERR_INVALID_ARG, "tuning_save(null)");
    for (int s = -1; s < 12; ++s) expect(tr_status_string((tr_status)s) != nullptr, "status string");
}

void with_device()
{
    const int n = 700, B = 3;
    std::vector<float> X, Y;
    make_pair(n, 140, X, Y, 7);
    float *src = dev_copy(X), *dst = dev_copy(Y);
    tr_handle *h = nullptr;
    expect_status(tr_create(&h, 1000, B, 200, 3, 0), TR_OK, "tr_create");
    if (!h) return;
    tr_params p{0.1f, 0.1f, 150, 2, TR_GRAPH_O2, TR_PIVOTS_PLAIN, 4, TR_FLAG_PROFILE};
    tr_result *out = nullptr;
    uint8_t *mask = nullptr;
    hipMalloc(&out, B * sizeof(tr_result));
    hipMalloc(&mask, B * 1000);
    expect_status(tr_register(h, src, dst, n, &p, out, mask, nullptr), TR_OK, "tr_register");
    expect_status(tr_register(h, src, dst, 1001, &p, out, mask, nullptr), TR_ERR_WORKSPACE, "register(n > max_n)");
    tr_result r;
    hipMemcpy(&r, out, sizeof(r), hipMemcpyDeviceToHost);
    expect(r.status == TR_OK && r.best_inliers >= 100, "registration finds the inliers");
    float st[TR_NUM_STAGES];
    expect_status(tr_stage_times(h, st, TR_NUM_STAGES), TR_OK, "tr_stage_times");
    // every tap of the call, through a size query and a copy
    for (int tap = TR_TAP_C; tap <= TR_TAP_PLAIN_PIVOTS; ++tap) {
        size_t need = 0;
        tr_status q = tr_debug_copy(h, tap, 0, nullptr, 0, &need);
        if (q != TR_OK || need == 0) continue;
        std::vector<char> buf(need);
        expect_status(tr_debug_copy(h, tap, 0, buf.data(), need, &need), TR_OK, "tr_debug_copy");
        expect(tr_debug_copy(h, tap, 0, buf.data(), need - 1, &need) != TR_OK, "debug copy refuses a short buffer");
    }
    // a batch of three pairs (the middle one too small), captured on a stream and replayed
    std::vector<int32_t> offs = {0, n, n + 2, 2 * n + 2};
    std::vector<float> X3(X), Y3(Y);
    X3.insert(X3.end(), X.begin(), X.begin() + 6);
    Y3.insert(Y3.end(), Y.begin(), Y.begin() + 6);
    X3.insert(X3.end(), X.begin(), X.end());
    Y3.insert(Y3.end(), Y.begin(), Y.end());
    float *src3 = dev_copy(X3), *dst3 = dev_copy(Y3);
    int32_t *offs_d = dev_copy(offs);
    hipStream_t s;
    hipStreamCreate(&s);
    p.flags = 0;
    for (int k = 0; k < 3; ++k)
        expect_status(tr_register_batch(h, src3, dst3, offs_d, B, n, &p, out, mask, s), TR_OK, "tr_register_batch");
    hipStreamSynchronize(s);
    // launch configurations and the autotuner
    tr_tuning t;
    expect_status(tr_tuning_get(h, n, 1, &t), TR_OK, "tr_tuning_get");
    t.sc2_sparse_cap = TR_SC2_SPARSE_CAP_MAX;
    expect_status(tr_tuning_set(h, n, 1, &t), TR_OK, "tr_tuning_set");
    t.hyp_ppw = 5;
    expect_status(tr_tuning_set(h, n, 1, &t), TR_ERR_INVALID_ARG, "tuning_set(ppw 5)");
    float ms = 0;
    expect_status(tr_autotune(h, src, dst, nullptr, 1, n, &p, out, mask, nullptr, &t, &ms), TR_OK, "tr_autotune");
    const char *cache = "asan_tuning_cache.txt";
    expect_status(tr_tuning_save(h, cache), TR_OK, "tr_tuning_save");
    expect_status(tr_tuning_load(h, cache), TR_OK, "tr_tuning_load");
    expect_status(tr_tuning_load(h, "/nonexistent/tuning.txt"), TR_ERR_INVALID_ARG, "tuning_load(missing)");
    std::remove(cache);
    // the scorer: set, save, load (and a corrupted blob), learned registration
    std::vector<float> w(TR_MLP_NPARAM);
    for (int k = 0; k < TR_MLP_NPARAM; ++k) w[k] = 0.01f * (float)((k * 37) % 19 - 9);
    expect_status(tr_scorer_set(h, w.data()), TR_OK, "tr_scorer_set");
    size_t bytes = 0;
    expect_status(tr_scorer_save(h, nullptr, 0, &bytes), TR_OK, "scorer size query");
    std::vector<char> blob(bytes);
    expect_status(tr_scorer_save(h, blob.data(), blob.size(), &bytes), TR_OK, "tr_scorer_save");
    expect_status(tr_scorer_load(h, blob.data(), blob.size()), TR_OK, "tr_scorer_load");
    blob[20] ^= 1;
    expect(tr_scorer_load(h, blob.data(), blob.size()) != TR_OK, "corrupted blob refused");
    tr_params pl = p;
    pl.pivot_mode = TR_PIVOTS_LEARNED;
    expect_status(tr_register(h, src, dst, n, &pl, out, mask, nullptr), TR_OK, "learned tr_register");
    // poses, triplets, features, MLP
    std::vector<int32_t> tri = {0, 1, 2, 3, 4, 5, 0, 0, 1, -1, 2, 3};
    int32_t *tri_d = dev_copy(tri), *ok_d = nullptr, *in_d = nullptr;
    float *poses_d = nullptr, *sc_d = nullptr;
    hipMalloc(&poses_d, 4 * 12 * sizeof(float));
    hipMalloc(&ok_d, 4 * sizeof(int32_t));
    hipMalloc(&in_d, 4 * sizeof(int32_t));
    hipMalloc(&sc_d, 4 * sizeof(float));
    expect_status(tr_fit_triplets(h, src, dst, n, tri_d, 4, poses_d, ok_d, nullptr), TR_OK, "tr_fit_triplets");
    expect_status(tr_score_poses(h, src, dst, n, poses_d, 4, 0.1f, 1, in_d, sc_d, nullptr), TR_OK, "tr_score_poses");
    uint16_t *feat = nullptr;
    hipMalloc(&feat, (2 * n + 2) * 19 * sizeof(uint16_t));
    expect_status(tr_features_batch(h, src3, dst3, offs_d, B, n, &p, feat, nullptr), TR_OK, "tr_features_batch");
    std::vector<uint8_t> lab(2 * n + 2);
    for (size_t k = 0; k < lab.size(); ++k) lab[k] = k % 5 == 0;
    uint8_t *lab_d = dev_copy(lab);
    float *scores = nullptr, *grads = nullptr, *loss = nullptr;
    hipMalloc(&scores, lab.size() * sizeof(float));
    hipMalloc(&grads, TR_MLP_NPARAM * sizeof(float));
    hipMalloc(&loss, sizeof(float));
    expect_status(tr_mlp_forward(h, feat, (int64_t)lab.size(), scores, nullptr), TR_OK, "tr_mlp_forward");
    expect_status(tr_mlp_grads(h, feat, lab_d, (int64_t)lab.size(), grads, loss, nullptr), TR_OK, "tr_mlp_grads");
    expect_status(tr_train_step(h, feat, lab_d, (int64_t)lab.size(), 1e-3f, loss, nullptr), TR_OK, "tr_train_step");
    expect_status(tr_register_noalloc(src, dst, n, &p, out, mask, nullptr), TR_OK, "tr_register_noalloc");
    hipDeviceSynchronize();
    expect_status(tr_destroy(h), TR_OK, "tr_destroy");
    hipStreamDestroy(s);
    for (void *q : {(void *)src, (void *)dst, (void *)src3, (void *)dst3, (void *)offs_d, (void *)out, (void *)mask,
                    (void *)tri_d, (void *)ok_d, (void *)in_d, (void *)poses_d, (void *)sc_d, (void *)feat,
                    (void *)lab_d, (void *)scores, (void *)grads, (void *)loss})
        hipFree(q);
}

}  // namespace

int main()
{
    without_device();
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) with_device();
    else std::printf("no device: argument checks only\n");
    if (failures) return 1;
    std::printf("ok\n");
    return 0;
}
