// The dispatcher's multilayer perceptron: 16 features -> 64 -> 64 -> 4 outputs
// (ReLU hidden layers, linear outputs), FP32.  It predicts the log device time
// of the kernel arms a call can use; it never touches a result bit.
//
// Parameter vector layout (5,508 floats):
//   W1[64][16] b1[64] W2[64][64] b2[64] W3[4][64] b3[4]
// Inputs are standardised with per-feature mean / std stored beside the weights.
//
// Training: masked mean-squared error over the outputs a sample has a target
// for, L = sum_i sum_a m_ia (y_ia - t_ia)^2 / sum m, minimised with Adam.
// Kernels are deliberately plain: one thread per (sample, unit) in the forward
// and delta passes, one thread per parameter for the gradient reduction and
// the Adam step.
#include "bmlp_internal.h"
#include "bmlp_mlp.h"
#include "features.h"

namespace bmlp {

namespace {

__device__ __forceinline__ const float* W1(const float* p) { return p; }
__device__ __forceinline__ const float* B1(const float* p) { return p + kH1 * kIn; }
__device__ __forceinline__ const float* W2(const float* p) { return p + kH1 * kIn + kH1; }
__device__ __forceinline__ const float* B2(const float* p) { return p + kH1 * kIn + kH1 + kH2 * kH1; }
__device__ __forceinline__ const float* W3(const float* p) { return p + kH1 * kIn + kH1 + kH2 * kH1 + kH2; }
__device__ __forceinline__ const float* B3(const float* p) { return p + kH1 * kIn + kH1 + kH2 * kH1 + kH2 + kOut * kH2; }

// activations of sample i: h1 (64), h2 (64), y (4)
__global__ void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ mu, const float* __restrict__ sd,
                              const float* __restrict__ X, i64 rows, float* __restrict__ H1, float* __restrict__ H2,
                              float* __restrict__ Y) {
  __shared__ float xs[4][kIn];
  __shared__ float h1s[4][kH1];
  __shared__ float h2s[4][kH2];
  const int lane = threadIdx.x & 63;
  const int sub = threadIdx.x >> 6;  // 4 samples per workgroup, one wave each
  const i64 i = blockIdx.x * 4 + sub;
  const bool live = i < rows;
  if (live && lane < kIn) xs[sub][lane] = (X[i * kIn + lane] - mu[lane]) / sd[lane];
  __syncthreads();
  if (live) {
    float a = B1(P)[lane];
    for (int f = 0; f < kIn; ++f) a += W1(P)[lane * kIn + f] * xs[sub][f];
    a = a > 0.f ? a : 0.f;
    h1s[sub][lane] = a;
    if (H1) H1[i * kH1 + lane] = a;
  }
  __syncthreads();
  if (live) {
    float a = B2(P)[lane];
    for (int f = 0; f < kH1; ++f) a += W2(P)[lane * kH1 + f] * h1s[sub][f];
    a = a > 0.f ? a : 0.f;
    h2s[sub][lane] = a;
    if (H2) H2[i * kH2 + lane] = a;
  }
  __syncthreads();
  if (live && lane < kOut) {
    float a = B3(P)[lane];
    for (int f = 0; f < kH2; ++f) a += W3(P)[lane * kH2 + f] * h2s[sub][f];
    Y[i * kOut + lane] = a;
  }
}

// output deltas dY = 2 m (y - t) / M (M = sum of the mask), back-propagated to the
// hidden layers: dH2 = (W3^T dY) * [h2 > 0], dH1 = (W2^T dH2) * [h1 > 0]; also
// accumulates the loss
__global__ void k_mlp_deltas(const float* __restrict__ P, const float* __restrict__ H1, const float* __restrict__ H2,
                             const float* __restrict__ Y, const float* __restrict__ T, const float* __restrict__ Msk,
                             i64 rows, float inv_m, float* __restrict__ dY, float* __restrict__ dH2,
                             float* __restrict__ dH1, float* __restrict__ loss) {
  __shared__ float dys[4][kOut];
  __shared__ float dh2s[4][kH2];
  const int lane = threadIdx.x & 63;
  const int sub = threadIdx.x >> 6;
  const i64 i = blockIdx.x * 4 + sub;
  const bool live = i < rows;
  if (live && lane < kOut) {
    const float e = Y[i * kOut + lane] - T[i * kOut + lane];
    const float m = Msk[i * kOut + lane];
    const float d = 2.f * m * e * inv_m;
    dys[sub][lane] = d;
    dY[i * kOut + lane] = d;
    if (m != 0.f) atomicAdd(loss, m * e * e * inv_m);
  }
  __syncthreads();
  if (live) {
    float a = 0.f;
    for (int o = 0; o < kOut; ++o) a += W3(P)[o * kH2 + lane] * dys[sub][o];
    a = H2[i * kH2 + lane] > 0.f ? a : 0.f;
    dh2s[sub][lane] = a;
    dH2[i * kH2 + lane] = a;
  }
  __syncthreads();
  if (live) {
    float a = 0.f;
    for (int o = 0; o < kH2; ++o) a += W2(P)[o * kH1 + lane] * dh2s[sub][o];
    a = H1[i * kH1 + lane] > 0.f ? a : 0.f;
    dH1[i * kH1 + lane] = a;
  }
}

// gradient of every parameter: a sum over the samples of (delta x input)
__global__ void k_mlp_grad(const float* __restrict__ mu, const float* __restrict__ sd, const float* __restrict__ X,
                           const float* __restrict__ H1, const float* __restrict__ H2, const float* __restrict__ dY,
                           const float* __restrict__ dH2, const float* __restrict__ dH1, i64 rows,
                           float* __restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  float acc = 0.f;
  int q = p;
  if (q < kH1 * kIn) {  // W1[j][f]
    const int j = q / kIn, f = q % kIn;
    for (i64 i = 0; i < rows; ++i) acc += dH1[i * kH1 + j] * ((X[i * kIn + f] - mu[f]) / sd[f]);
  } else if ((q -= kH1 * kIn) < kH1) {  // b1[j]
    for (i64 i = 0; i < rows; ++i) acc += dH1[i * kH1 + q];
  } else if ((q -= kH1) < kH2 * kH1) {  // W2[j][f]
    const int j = q / kH1, f = q % kH1;
    for (i64 i = 0; i < rows; ++i) acc += dH2[i * kH2 + j] * H1[i * kH1 + f];
  } else if ((q -= kH2 * kH1) < kH2) {  // b2[j]
    for (i64 i = 0; i < rows; ++i) acc += dH2[i * kH2 + q];
  } else if ((q -= kH2) < kOut * kH2) {  // W3[o][f]
    const int o = q / kH2, f = q % kH2;
    for (i64 i = 0; i < rows; ++i) acc += dY[i * kOut + o] * H2[i * kH2 + f];
  } else {  // b3[o]
    q -= kOut * kH2;
    for (i64 i = 0; i < rows; ++i) acc += dY[i * kOut + q];
  }
  G[p] = acc;
}

// Device-side choice: forward pass on one feature vector (one wave, lane =
// hidden unit), then *decision = the index of the smallest predicted log time
// among the outputs allowed by `allowed` (bit o set = output o allowed).  For a
// semi-naive round the product and sparse kernels read *decision as their
// predicate.
__global__ void k_mlp_decide(const float* __restrict__ P, const float* __restrict__ mu, const float* __restrict__ sd,
                             const float* __restrict__ feat, float* __restrict__ pred, u32* __restrict__ decision,
                             u32 allowed) {
  __shared__ float xs[kIn];
  __shared__ float h1s[kH1];
  __shared__ float h2s[kH2];
  __shared__ float ys[kOut];
  const int lane = threadIdx.x;
  if (lane < kIn) xs[lane] = (feat[lane] - mu[lane]) / sd[lane];
  __syncthreads();
  float a = B1(P)[lane];
  for (int f = 0; f < kIn; ++f) a += W1(P)[lane * kIn + f] * xs[f];
  h1s[lane] = a > 0.f ? a : 0.f;
  __syncthreads();
  a = B2(P)[lane];
  for (int f = 0; f < kH1; ++f) a += W2(P)[lane * kH1 + f] * h1s[f];
  h2s[lane] = a > 0.f ? a : 0.f;
  __syncthreads();
  if (lane < kOut) {
    a = B3(P)[lane];
    for (int f = 0; f < kH2; ++f) a += W3(P)[lane * kH2 + f] * h2s[f];
    ys[lane] = a;
    pred[lane] = a;
  }
  __syncthreads();
  if (lane == 0) {
    int best = -1;
    for (int o = 0; o < kOut; ++o)
      if (((allowed >> o) & 1u) && (best < 0 || ys[o] < ys[best])) best = o;  // ties keep the lower index
    *decision = (u32)(best < 0 ? 0 : best);
  }
}

// Adam (Kingma and Ba, 2015), step t >= 1
__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M1,
                       float* __restrict__ M2, float lr, float beta1, float beta2, float eps, float bc1, float bc2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float g = G[p];
  const float m = beta1 * M1[p] + (1.f - beta1) * g;
  const float v = beta2 * M2[p] + (1.f - beta2) * g * g;
  M1[p] = m;
  M2[p] = v;
  P[p] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

__global__ void k_call_features(const unsigned long long* __restrict__ gstats,
                                const unsigned long long* __restrict__ delta0, i64 n, i64 k, float context,
                                int reflexive, float* __restrict__ f) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double d0 = (double)*delta0;
  make_features(f, (double)n, (double)gstats[0], (double)gstats[1], (double)gstats[2], (double)k, context, 1, 0, d0,
                d0, reflexive ? d0 : 0.0, reflexive);
}

}  // namespace

hipError_t launch_mlp_forward(const float* P, const float* mu, const float* sd, const float* X, i64 rows, float* H1,
                              float* H2, float* Y, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, P, mu, sd, X, rows, H1, H2, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* P, const float* mu, const float* sd, const float* X, const float* H1,
                               const float* H2, const float* Y, const float* T, const float* Msk, i64 rows,
                               float inv_m, float* dY, float* dH2, float* dH1, float* G, float* loss, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_deltas, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, P, H1, H2, Y, T, Msk, rows,
                     inv_m, dY, dH2, dH1, loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_grad, dim3((kParams + 255) / 256), dim3(256), 0, s, mu, sd, X, H1, H2, dY, dH2, dH1, rows,
                     G);
  return hipGetLastError();
}

hipError_t launch_mlp_decide(const float* P, const float* mu, const float* sd, const float* feat, float* pred,
                             u32* decision, u32 allowed, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_decide, dim3(1), dim3(64), 0, s, P, mu, sd, feat, pred, decision, allowed);
  return hipGetLastError();
}

hipError_t launch_call_features(const unsigned long long* gstats, const unsigned long long* delta0, i64 n, i64 k,
                                float context, int reflexive, float* f, hipStream_t s) {
  hipLaunchKernelGGL(k_call_features, dim3(1), dim3(64), 0, s, gstats, delta0, n, k, context, reflexive, f);
  return hipGetLastError();
}

hipError_t launch_adam(float* P, const float* G, float* M1, float* M2, float lr, float beta1, float beta2, float eps,
                       int step, hipStream_t s) {
  const float bc1 = 1.f - powf(beta1, (float)step);
  const float bc2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, P, G, M1, M2, lr, beta1, beta2, eps, bc1,
                     bc2);
  return hipGetLastError();
}

}  // namespace bmlp
