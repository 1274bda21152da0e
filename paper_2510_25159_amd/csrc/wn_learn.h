// Learned depth predictor: constants and launchers (wn_learn.hip).
#pragma once

#include "wn_internal.h"

namespace wn {

constexpr int kMlpIn = 16;
constexpr int kMlpH = 64;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH;
constexpr int kMlpParams = kOffB3 + 1;  // 5313
// BF16 copy of W1 and W2 in the order of the matrix-core operand fragments
// (four layer-1 tiles, then eight layer-2 tile / K-step pairs; 64 lanes of
// eight values each); layer 1's K padding slots hold zero.
constexpr int kMlpFragSlots = 12 * 64 * 8;
constexpr int kBins = 32;               // depth bins of the near queue

// Analytic depth estimate (control for the learned predictor): the level at
// which the sub-ellipse axis B 2^-k falls below the distance from the query
// to the chord, ceil(log2(B / max(eps, d_chord))), d_chord recovered from the
// ellipse-frame features (f0, f1 in units of a = B/2, f2 = a, f14 = L/2).
__host__ __device__ inline float heuristic_depth(const float* f, float eps) {
    const float a = f[2];
    const float along = fmaxf(fabsf(f[0] * a) - f[14], 0.f), across = f[1] * a;
    const float d = fmaxf(sqrtf(along * along + across * across), eps);
    return a > 0.f ? fmaxf(ceilf(log2f(2.f * a / d)), 0.f) : 0.f;
}

struct TrainBufs {
    float *H1, *H2, *DH1, *DH2, *DY;  // [B][64] activations / gradients, [B] output gradient
    float* grad;                      // [kMlpParams]
    float* loss;                      // [1] summed loss (atomic)
};

hipError_t launch_pair_features(const Segs& sg, const Points& pts, const int32_t* pp, const int32_t* ps, int64_t n,
                                double eps, float* out, hipStream_t st);
hipError_t launch_queue_features(const Segs& sg, const Points& pts, NearQueue nq, const uint8_t* seg_per, double eps,
                                 uint64_t limit, float* out, int grid, hipStream_t st);
hipError_t launch_predict(const float* w, const float* X, int64_t n, float* out, hipStream_t st);
hipError_t launch_train_step(const float* w, const float* X, const float* Y, const int32_t* idx, int B, float delta,
                             TrainBufs tb, hipStream_t st);
hipError_t launch_adamw(float* master, float* m, float* v, const float* grad, float lr, float beta1, float beta2,
                        float eps, float wd, int step, float* wbf, uint16_t* w16, hipStream_t st);
hipError_t launch_round_params(const float* master, float* wbf, uint16_t* w16, hipStream_t st);
// Predictions on the matrix cores (BF16 inputs, weights and hidden activations,
// FP32 accumulation).
// X: [n][16], 16-byte aligned; cus: compute units (the persistent grid).
hipError_t launch_predict_mfma(const uint16_t* w16, const float* w, const float* X, int64_t n, float* out, int cus,
                               hipStream_t st);
// Bin counts, offsets and scatter of the near queue.  mode 0 (the MLP): on the
// matrix cores when w16 (the BF16 weights) is given, else the VALU version.
hipError_t launch_binning(const Segs& sg, const Points& pts, NearQueue nq, const uint8_t* seg_per, double eps,
                          int mode, const float* w, const uint16_t* w16, const float* norm, const uint8_t* measured,
                          uint8_t* bins, uint32_t* wg_hist, int G, uint2* qs_out, double2* sh_out, hipStream_t st);

}  // namespace wn
