// The learned parameter choice: a small MLP (16 features -> 64 -> 64 -> 32,
// ReLU, fp32) mapping a graph's sampled degree/locality features to the
// predicted (normalised) log run time of each of the 32 kernel
// configurations; the plan takes the argmin.  Forward, backward and Adam
// update are plain FMA loops (the network is far too small for matrix
// cores); every reduction runs in a fixed order, so training is
// deterministic.
//
// Parameter layout (floats): W1[16][64], b1[64], W2[64][64], b2[64],
// W3[64][32], b3[32]  (row-major, y = x W + b).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gt.h"
#include "gt_mlp.h"

namespace gt {

namespace {
constexpr int F = kMlpIn, H = kMlpHidden, G = kMlpOut;
constexpr int oW1 = 0, ob1 = oW1 + F * H, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + H * G;
static_assert(ob3 + G == kMlpParams, "parameter layout");
}  // namespace

// Activations of one row per workgroup of H threads.  work: H1[B][H],
// H2[B][H] (pre-ReLU values are not kept: ReLU'(z) = (relu(z) > 0)).
__global__ __launch_bounds__(H) void k_mlp_fwd(const float *__restrict__ p, const float *__restrict__ x, int batch,
                                               float *__restrict__ y, float *__restrict__ h1o,
                                               float *__restrict__ h2o) {
  __shared__ float s_x[F], s_h1[H], s_h2[H];
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= batch) return;
  if (j < F) s_x[j] = x[(int64_t)b * F + j];
  __syncthreads();
  float a = p[ob1 + j];
  for (int k = 0; k < F; ++k) a = fmaf(s_x[k], p[oW1 + k * H + j], a);
  a = a > 0.f ? a : 0.f;
  s_h1[j] = a;
  if (h1o) h1o[(int64_t)b * H + j] = a;
  __syncthreads();
  a = p[ob2 + j];
  for (int k = 0; k < H; ++k) a = fmaf(s_h1[k], p[oW2 + k * H + j], a);
  a = a > 0.f ? a : 0.f;
  s_h2[j] = a;
  if (h2o) h2o[(int64_t)b * H + j] = a;
  __syncthreads();
  if (j < G) {
    a = p[ob3 + j];
    for (int k = 0; k < H; ++k) a = fmaf(s_h2[k], p[oW3 + k * G + j], a);
    y[(int64_t)b * G + j] = a;
  }
}

// Per row: dY = 2 (Y - T) / (B G), dH2 = (dY W3^T) * [H2 > 0],
// dH1 = (dH2 W2^T) * [H1 > 0].
__global__ __launch_bounds__(H) void k_mlp_bwd_rows(const float *__restrict__ p, const float *__restrict__ t,
                                                    int batch, const float *__restrict__ y,
                                                    const float *__restrict__ h1, const float *__restrict__ h2,
                                                    float *__restrict__ dy, float *__restrict__ dh2,
                                                    float *__restrict__ dh1) {
  __shared__ float s_dy[G], s_dh2[H];
  const int b = blockIdx.x, j = threadIdx.x;
  if (b >= batch) return;
  const float scale = 2.0f / ((float)batch * (float)G);
  if (j < G) {
    const float d = scale * (y[(int64_t)b * G + j] - t[(int64_t)b * G + j]);
    s_dy[j] = d;
    dy[(int64_t)b * G + j] = d;
  }
  __syncthreads();
  float a = 0.f;
  for (int k = 0; k < G; ++k) a = fmaf(s_dy[k], p[oW3 + j * G + k], a);
  a = h2[(int64_t)b * H + j] > 0.f ? a : 0.f;
  s_dh2[j] = a;
  dh2[(int64_t)b * H + j] = a;
  __syncthreads();
  a = 0.f;
  for (int k = 0; k < H; ++k) a = fmaf(s_dh2[k], p[oW2 + j * H + k], a);
  dh1[(int64_t)b * H + j] = h1[(int64_t)b * H + j] > 0.f ? a : 0.f;
}

// One thread per parameter: its gradient summed over the batch in row order.
__global__ void k_mlp_wgrad(const float *__restrict__ x, int batch, const float *__restrict__ h1,
                            const float *__restrict__ h2, const float *__restrict__ dy,
                            const float *__restrict__ dh2, const float *__restrict__ dh1, float *__restrict__ g) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kMlpParams) return;
  const float *in, *gr;
  int ni, no, k = 0, j;
  bool bias = false;
  if (q < ob1) { in = x; ni = F; gr = dh1; no = H; k = (q - oW1) / H; j = (q - oW1) % H; }
  else if (q < oW2) { in = x; ni = F; gr = dh1; no = H; j = q - ob1; bias = true; }
  else if (q < ob2) { in = h1; ni = H; gr = dh2; no = H; k = (q - oW2) / H; j = (q - oW2) % H; }
  else if (q < oW3) { in = h1; ni = H; gr = dh2; no = H; j = q - ob2; bias = true; }
  else if (q < ob3) { in = h2; ni = H; gr = dy; no = G; k = (q - oW3) / G; j = (q - oW3) % G; }
  else { in = h2; ni = H; gr = dy; no = G; j = q - ob3; bias = true; }
  float a = 0.f;
  for (int b = 0; b < batch; ++b) {
    const float u = gr[(int64_t)b * no + j];
    a = bias ? a + u : fmaf(in[(int64_t)b * ni + k], u, a);
  }
  g[q] = a;
}

// Mean squared error over the batch (one workgroup, fixed order).
__global__ __launch_bounds__(256) void k_mlp_loss(const float *__restrict__ y, const float *__restrict__ t,
                                                  int batch, float *loss) {
  __shared__ float s[256];
  const int j = threadIdx.x;
  float a = 0.f;
  for (int64_t i = j; i < (int64_t)batch * G; i += 256) {
    const float d = y[i] - t[i];
    a = fmaf(d, d, a);
  }
  s[j] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (j < w) s[j] += s[j + w];
    __syncthreads();
  }
  if (j == 0) *loss = s[0] / ((float)batch * (float)G);
}

// Adam (Kingma & Ba 2015) with bias correction; step counts from 1.
__global__ void k_mlp_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                           float *__restrict__ m2, int step, float lr, float beta1, float beta2, float eps) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= kMlpParams) return;
  const float gq = g[q];
  const float a = beta1 * m1[q] + (1.f - beta1) * gq;
  const float v = beta2 * m2[q] + (1.f - beta2) * gq * gq;
  m1[q] = a;
  m2[q] = v;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  p[q] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

size_t mlp_work_floats(int batch) { return (size_t)batch * (2 * H + G + 2 * H + G); }

hipError_t mlp_forward(const float *params, const float *x, int batch, float *y, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(batch), dim3(H), 0, st, params, x, batch, y, nullptr, nullptr);
  return hipGetLastError();
}

}  // namespace gt

using namespace gt;

extern "C" {

int32_t gt_mlp_num_params(void) { return kMlpParams; }

size_t gt_mlp_work_floats(int32_t batch) { return batch > 0 ? mlp_work_floats(batch) : 0; }

gt_status gt_mlp_forward(const float *params, const float *x, int32_t batch, float *y, void *stream) {
  if (params == nullptr || x == nullptr || y == nullptr || batch < 0) return GT_ERR_INVALID_ARGUMENT;
  return mlp_forward(params, x, batch, y, (hipStream_t)stream) == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status gt_mlp_gradient(const float *params, const float *x, const float *target, int32_t batch, float *y,
                          float *grad, float *loss, float *work, void *stream) {
  if (!params || !x || !target || !y || !grad || !loss || !work || batch <= 0) return GT_ERR_INVALID_ARGUMENT;
  hipStream_t st = (hipStream_t)stream;
  float *h1 = work, *h2 = h1 + (size_t)batch * H, *dy = h2 + (size_t)batch * H, *dh2 = dy + (size_t)batch * G,
        *dh1 = dh2 + (size_t)batch * H;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(batch), dim3(H), 0, st, params, x, batch, y, h1, h2);
  hipLaunchKernelGGL(k_mlp_bwd_rows, dim3(batch), dim3(H), 0, st, params, target, batch, y, h1, h2, dy, dh2, dh1);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, x, batch, h1, h2, dy, dh2, dh1,
                     grad);
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, y, target, batch, loss);
  return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status gt_mlp_adam(float *params, const float *grad, float *m1, float *m2, int32_t step, float lr, float beta1,
                      float beta2, float eps, void *stream) {
  if (!params || !grad || !m1 || !m2 || step < 1) return GT_ERR_INVALID_ARGUMENT;
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad, m1,
                     m2, step, lr, beta1, beta2, eps);
  return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

}  // extern "C"
