// Degree sampling and graph features (Section IV-C, Step 0: a sample of 1% of
// |V| positions of the edge array; Section V-G: coverage of the most frequent
// destinations).  The features feed the parameter policies; the sample never
// changes the transposition's output.
//
// Sample i (0 <= i < s) takes position lo + (r mod (hi - lo)) in the stratum
// [lo, hi) = [floor(i m / s), floor((i+1) m / s)) of the edge array, where r
// is the (i+1)-th output of splitmix64 seeded with `seed` (Steele, Lea, Flood
// 2014).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gt_device.hpp"
#include "gt_sample.h"

namespace gt {

__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}

__device__ void sample_one(SampleArgs a, int64_t i, unsigned long long *s_acc);

// One thread per sample: position, destination, source (binary search of
// the offsets), frequency count in an open-addressing table, locality sums,
// and the sample count of the destination's 256-vertex bin.  The three
// locality sums are reduced in LDS, one global atomic per block each.
__global__ __launch_bounds__(256) void k_sample(SampleArgs a) {
  __shared__ unsigned long long s_acc[3];
  if (threadIdx.x < 3) s_acc[threadIdx.x] = 0ull;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < a.s) sample_one(a, i, s_acc);
  __syncthreads();
  if (threadIdx.x < 3 && s_acc[threadIdx.x] != 0ull)
    atomicAdd((unsigned long long *)&a.acc[threadIdx.x], s_acc[threadIdx.x]);
}

__device__ void sample_one(SampleArgs a, int64_t i, unsigned long long *s_acc) {
  const uint64_t q = (uint64_t)a.m / (uint64_t)a.s, r = (uint64_t)a.m % (uint64_t)a.s;
  const uint64_t lo = (uint64_t)i * q + ((uint64_t)i * r) / (uint64_t)a.s;
  const uint64_t hi = (uint64_t)(i + 1) * q + ((uint64_t)(i + 1) * r) / (uint64_t)a.s;
  const uint64_t pos = lo + splitmix64_at(a.seed, (uint64_t)i) % (hi - lo);
  uint32_t dst = (uint32_t)a.D[pos];
  if (dst >= (uint32_t)a.n) dst = 0;  // invalid graphs are reported by the transposition itself
  int64_t l = 0, h = a.n;  // largest u with O[u] <= pos
  while (h - l > 1) {
    const int64_t mid = (l + h) >> 1;
    if (a.O[mid] <= (int64_t)pos) l = mid; else h = mid;
  }
  const uint32_t src = (uint32_t)l;
  // frequency table
  uint32_t slot = hash32(dst) & a.mask;
  while (true) {
    const int32_t prev = atomicCAS(&a.keys[slot], -1, (int32_t)dst);
    if (prev == -1 || prev == (int32_t)dst) { atomicAdd(&a.counts[slot], 1u); break; }
    slot = (slot + 1) & a.mask;
  }
  const uint32_t dist = dst > src ? dst - src : src - dst;
  atomicAdd(&s_acc[0], (unsigned long long)dist);
  if (dist < 256u) atomicAdd(&s_acc[1], 1ull);
  if (dist < 65536u) atomicAdd(&s_acc[2], 1ull);
  atomicAdd(&a.bins[dst >> 8], 1u);
}

// Over the table: per log2 bucket of the sample count, the number of
// destinations and their summed counts; number of distinct destinations.
// Reduced in LDS per block, then one global atomic per nonzero sum.
__global__ __launch_bounds__(256) void k_sample_table(SampleArgs a) {
  __shared__ unsigned long long s_keys[32], s_sum[32], s_distinct;
  if (threadIdx.x < 32) { s_keys[threadIdx.x] = 0ull; s_sum[threadIdx.x] = 0ull; }
  if (threadIdx.x == 0) s_distinct = 0ull;
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i <= (int64_t)a.mask && a.keys[i] != -1) {
    const uint32_t c = a.counts[i];
    const int j = 31 - __clz(c);
    atomicAdd(&s_keys[j], 1ull);
    atomicAdd(&s_sum[j], (unsigned long long)c);
    atomicAdd(&s_distinct, 1ull);
  }
  __syncthreads();
  if (threadIdx.x < 32) {
    const int j = threadIdx.x;
    if (s_keys[j]) {
      atomicAdd((unsigned long long *)&a.acc[8 + j], s_keys[j]);
      atomicAdd((unsigned long long *)&a.acc[40 + j], s_sum[j]);
    }
  }
  if (threadIdx.x == 0 && s_distinct) atomicAdd((unsigned long long *)&a.acc[3], s_distinct);
}

// Over the 256-vertex bins: samples falling in bins whose estimated edge
// count exceeds `big` edges.
__global__ void k_sample_bins(SampleArgs a, int64_t nbins256, double scale, double big) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nbins256) return;
  const uint32_t c = a.bins[i];
  if (c > 0 && (double)c * scale > big) atomicAdd((unsigned long long *)&a.acc[4], (unsigned long long)c);
}

// Feature vector (fp32) from the aggregates; one thread.
__global__ void k_features(SampleArgs a, float *out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double s = (double)a.s, n = (double)a.n, m = (double)a.m;
  const uint64_t *acc = a.acc;
  double f[kNumFeatures];
  f[0] = log2(n + 1.0) / 32.0;
  f[1] = log2(m + 1.0) / 40.0;
  f[2] = log2(m / (n > 0 ? n : 1.0) + 1.0) / 8.0;
  f[3] = a.payload ? 1.0 : 0.0;
  // fraction of sampled edges on destinations seen >= 2, 4, 16, 64 times
  const int thr[4] = {1, 2, 4, 6};
  for (int t = 0; t < 4; ++t) {
    double c = 0;
    for (int j = thr[t]; j < 32; ++j) c += (double)acc[40 + j];
    f[4 + t] = c / s;
  }
  // estimated coverage of the k most frequent destinations, k = 2^10, 2^14, 2^18
  const int lk[3] = {10, 14, 18};
  for (int t = 0; t < 3; ++t) {
    double need = (double)(1ull << lk[t]), cov = 0;
    for (int j = 31; j >= 0 && need > 0; --j) {
      const double keys = (double)acc[8 + j], sum = (double)acc[40 + j];
      if (keys <= 0) continue;
      if (keys <= need) { cov += sum; need -= keys; }
      else { cov += need * (sum / keys); need = 0; }
    }
    f[8 + t] = cov / s;
  }
  f[11] = (double)acc[0] / (s * (n > 0 ? n : 1.0));
  f[12] = (double)acc[1] / s;
  f[13] = (double)acc[2] / s;
  f[14] = (double)acc[4] / s;
  f[15] = (double)acc[3] / s;
  for (int k = 0; k < kNumFeatures; ++k) out[k] = (float)f[k];
}

}  // namespace gt

namespace gt {

int64_t sample_count(int64_t n, int64_t m) {
  int64_t s = (n + 99) / 100;  // 1% of |V|
  if (s < 4096) s = 4096;
  if (s > m) s = m;
  return s;
}

size_t sample_scratch_bytes(int64_t n, int64_t m) {
  const int64_t s = sample_count(n, m);
  uint64_t cap = 1;
  while (cap < (uint64_t)(2 * s + 1)) cap <<= 1;
  const size_t nb = (size_t)((n >> 8) + 1);
  return 8 * cap + 8 * kSampleAcc + 4 * nb + 4 * kNumFeatures + 4 * 256;
}

// Enqueue the sampling kernels of one graph into `scratch`; the features
// land in *features_dev (kNumFeatures floats inside the scratch region).
hipError_t enqueue_sampling(const int64_t *O, const int32_t *D, int64_t n, int64_t m, bool payload, uint64_t seed,
                            char *scratch, float **features_dev, hipStream_t st, SampleArgs *table_out) {
  SampleArgs a{};
  a.O = O; a.D = D; a.n = n; a.m = m; a.seed = seed; a.payload = payload;
  a.s = sample_count(n, m);
  uint64_t cap = 1;
  while (cap < (uint64_t)(2 * a.s + 1)) cap <<= 1;
  a.mask = (uint32_t)(cap - 1);
  size_t off = 0;
  a.keys = reinterpret_cast<int32_t *>(scratch + off); off += 4 * cap;
  a.counts = reinterpret_cast<uint32_t *>(scratch + off); off += 4 * cap;
  a.acc = reinterpret_cast<uint64_t *>(scratch + off); off += 8 * kSampleAcc;
  const int64_t nb = (n >> 8) + 1;
  a.bins = reinterpret_cast<uint32_t *>(scratch + off); off += 4 * (size_t)nb;
  float *feat = reinterpret_cast<float *>(scratch + off);
  *features_dev = feat;
  hipError_t e;
  if ((e = launch_fill(reinterpret_cast<uint32_t *>(a.keys), cap, 0xFFFFFFFFu, st)) != hipSuccess) return e;
  if ((e = launch_fill(a.counts, cap, 0u, st)) != hipSuccess) return e;
  if ((e = launch_fill(reinterpret_cast<uint32_t *>(a.acc), 2 * kSampleAcc, 0u, st)) != hipSuccess) return e;
  if ((e = launch_fill(a.bins, (uint64_t)nb, 0u, st)) != hipSuccess) return e;
  if (m > 0 && n > 0) {
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((a.s + 255) / 256)), dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_sample_table, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, st, a);
    const double scale = (double)m / (double)a.s;
    hipLaunchKernelGGL(k_sample_bins, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, st, a, nb, scale,
                       (double)final_tile_size());
  } else {
    a.s = 1;  // features of an empty graph: sizes only
  }
  hipLaunchKernelGGL(k_features, dim3(1), dim3(64), 0, st, a, feat);
  if (table_out) *table_out = a;
  return hipGetLastError();
}

}  // namespace gt
