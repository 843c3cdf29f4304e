// Shapes and launchers of the dispatcher's MLP (16 -> 64 -> 64 -> 4, FP32).
#pragma once
#include "bmlp_internal.h"

namespace bmlp {

constexpr int kIn = 16, kH1 = 64, kH2 = 64, kOut = 4;
constexpr int kParams = kH1 * kIn + kH1 + kH2 * kH1 + kH2 + kOut * kH2 + kOut;  // 5,508

// Y (rows x 4) = MLP(X); H1, H2 (rows x 64) may be null (inference)
hipError_t launch_mlp_forward(const float* P, const float* mu, const float* sd, const float* X, i64 rows, float* H1,
                              float* H2, float* Y, hipStream_t s);
// G = dL/dP for the masked MSE against T; *loss += L (loss must be zeroed)
hipError_t launch_mlp_backward(const float* P, const float* mu, const float* sd, const float* X, const float* H1,
                               const float* H2, const float* Y, const float* T, const float* Msk, i64 rows,
                               float inv_m, float* dY, float* dH2, float* dH1, float* G, float* loss, hipStream_t s);
// one sample: pred (4) = MLP(feat); *decision = argmin of pred over the outputs set in `allowed`
hipError_t launch_mlp_decide(const float* P, const float* mu, const float* sd, const float* feat, float* pred,
                             u32* decision, u32 allowed, hipStream_t s);
// The call-level features (features.h) of a request from device counts: gstats = (bits, largest row, nonempty
// rows) of the relation, *delta0 = the set bits of the query rows; one thread writes f[16].
hipError_t launch_call_features(const unsigned long long* gstats, const unsigned long long* delta0, i64 n, i64 k,
                                float context, int reflexive, float* f, hipStream_t s);
hipError_t launch_adam(float* P, const float* G, float* M1, float* M2, float lr, float beta1, float beta2, float eps,
                       int step, hipStream_t s);

}  // namespace bmlp
