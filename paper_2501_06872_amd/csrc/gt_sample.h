// Degree sampling and feature extraction (interface).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gt_internal.h"

namespace gt {

constexpr int kNumFeatures = 16;
constexpr int kSampleAcc = 72;  // 0..7 sums and counts, 8..39 keys per log2 bucket, 40..71 counts per bucket

struct SampleArgs {
  const int64_t *O;
  const int32_t *D;
  int64_t n, m, s;
  uint64_t seed;
  bool payload;
  uint32_t mask;     // table capacity - 1
  int32_t *keys;     // [capacity] sampled destinations, -1 = empty
  uint32_t *counts;  // [capacity]
  uint64_t *acc;     // [kSampleAcc]
  uint32_t *bins;    // [n/256 + 1] samples per 256-vertex bin
};

int64_t sample_count(int64_t n, int64_t m);
size_t sample_scratch_bytes(int64_t n, int64_t m);
// `table_out` (optional) receives the frequency table's location.
hipError_t enqueue_sampling(const int64_t *O, const int32_t *D, int64_t n, int64_t m, bool payload, uint64_t seed,
                            char *scratch, float **features_dev, hipStream_t st, SampleArgs *table_out = nullptr);

}  // namespace gt
