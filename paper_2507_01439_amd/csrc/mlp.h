// Learned pivot scorer: state and launchers (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace tr {

// Parameter layout (float32, row-major out x in), TR_MLP_NPARAM values.
constexpr int kW1 = 0, kB1 = 64 * 19, kW2 = kB1 + 64, kB2 = kW2 + 64 * 64, kW3 = kB2 + 64, kB3 = kW3 + 64;
static_assert(kB3 + 1 == TR_MLP_NPARAM, "parameter layout");
constexpr int kGradSlots = TR_MLP_NPARAM + 1;   // gradients then the loss

struct MlpState {
    float *w32 = nullptr;        // master weights
    float *m = nullptr, *v = nullptr;   // Adam moments
    uint16_t *wbf16 = nullptr;   // bfloat16 copies of all parameters (biases are read in float32)
    int32_t step = 0;            // Adam step count
    float *scratch = nullptr;    // per-sample activations and deltas for the backward pass
    int64_t scratch_m = 0;       // samples the scratch holds
    float *partial = nullptr;    // per-tile gradient partial sums
    int64_t partial_tiles = 0;
    float *grads = nullptr;      // kGradSlots
};

hipError_t setup_mlp_kernels();
hipError_t mlp_create(MlpState *s);
void mlp_release(MlpState *s);
hipError_t mlp_set(MlpState *s, const float *host);
hipError_t mlp_get(MlpState *s, float *host);
hipError_t mlp_forward(MlpState *s, const uint16_t *feat, int64_t m, float *scores, hipStream_t st);
hipError_t mlp_grads(MlpState *s, const uint16_t *feat, const uint8_t *labels, int64_t m, float *grads,
                     float *loss, hipStream_t st);
hipError_t mlp_train_step(MlpState *s, const uint16_t *feat, const uint8_t *labels, int64_t m, float lr,
                          float *loss, hipStream_t st);

// Features of every pair from the accumulators filled by the compatibility and
// SC2 kernels; written to w.feat, or packed by match index into `packed`.
hipError_t launch_features(const Work &w, uint16_t *packed, int grid, hipStream_t st);
// Learned scores of every match, then the per-pair pivot reorder.
hipError_t launch_learned_order(const Work &w, const MlpState &mlp, int B, int grid, hipStream_t st);

}  // namespace tr
