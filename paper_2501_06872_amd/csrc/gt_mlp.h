// The parameter-choice MLP (interface shared by the policies and the kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace gt {

constexpr int kMlpIn = 16;      // sampled features (gt_sample.h)
constexpr int kMlpHidden = 64;
constexpr int kMlpOut = 32;     // kernel configurations (gt_config)
constexpr int kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpHidden * kMlpOut + kMlpOut;

size_t mlp_work_floats(int batch);
hipError_t mlp_forward(const float *params, const float *x, int batch, float *y, hipStream_t st);

// Configuration c of the learned/autotuned choice:
// fine_bits = 6 + c / 8, variant = 1 + (c / 2) % 4, digit_bits = (c % 2) ? 10 : 8.
__host__ __device__ inline void config_params(int c, int *fine_bits, int *digit_bits, int *variant) {
  *fine_bits = 6 + c / 8;
  *variant = 1 + (c / 2) % 4;
  *digit_bits = (c % 2) ? 10 : 8;
}

}  // namespace gt
