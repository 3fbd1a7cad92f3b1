// Random-access microbenchmark: the GPU counterpart of the measurement behind
// Fig. 3 (Section III-B), which compares random reads, writes and atomic
// writes to arrays that fit a cache level with arrays far larger than it.
// Here the levels are a workgroup's LDS, the per-XCD L2, the Infinity Cache
// (MALL) and HBM, chosen by the array size; Eq. 2 and Eq. 3 (Section IV-B)
// take their per-access times from these rates.
//
// Every thread draws its indices from a counter-based generator: the 32-bit
// MurmurHash3 finalizer (Appleby) applied to a Weyl sequence with increment
// 0x9E3779B9 started at fmix32(seed ^ thread), i.e. the SplitMix construction
// (Steele, Lea, Flood 2014) in 32 bits.  Access j of thread t goes to
// index ((uint64)r * words) >> 32 with r = fmix32(start_t + (j + 1) * 0x9E3779B9),
// which lies in [0, words).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/gt.h"

namespace gt {
namespace {

constexpr int kMbThreads = 256;
constexpr uint32_t kWeyl = 0x9E3779B9u;
constexpr uint64_t kMbMaxLdsWords = 16384;  // 64 KB of LDS per workgroup
constexpr int64_t kMbMaxBlocks = 1 << 20;

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// One access of kind K to a[idx] by thread t; reads and index draws fold
// into `acc`, which the thread stores at the end so no access is dead code.
template <int K>
__device__ __forceinline__ void access(uint32_t *a, uint64_t idx, uint32_t t, uint32_t &acc) {
  if constexpr (K == GT_ACCESS_READ) acc ^= a[idx];
  else if constexpr (K == GT_ACCESS_WRITE) a[idx] = t;
  else if constexpr (K == GT_ACCESS_ATOMIC) atomicAdd(a + idx, 1u);
  else acc ^= (uint32_t)idx;
}

template <int K>
__global__ __launch_bounds__(kMbThreads) void k_random_global(uint32_t *buf, uint64_t words, uint32_t seed,
                                                             int64_t per_thread, uint32_t *sink) {
  const uint32_t t = blockIdx.x * kMbThreads + threadIdx.x;
  uint32_t ctr = fmix32(seed ^ t);
  uint32_t acc = 0;
#pragma unroll 4
  for (int64_t j = 0; j < per_thread; ++j) {
    ctr += kWeyl;
    const uint64_t idx = ((uint64_t)fmix32(ctr) * words) >> 32;
    access<K>(buf, idx, t, acc);
  }
  if (sink != nullptr) sink[t] = acc;
}

// LDS level: workgroup b loads buf[b * words, (b + 1) * words) into LDS, runs
// the same accesses there, and stores the image back.
template <int K>
__global__ __launch_bounds__(kMbThreads) void k_random_lds(uint32_t *buf, uint32_t words, uint32_t seed,
                                                          int64_t per_thread, uint32_t *sink) {
  extern __shared__ uint32_t s_img[];
  const uint32_t t = blockIdx.x * kMbThreads + threadIdx.x;
  uint32_t *img = buf + (uint64_t)blockIdx.x * words;
  for (uint32_t i = threadIdx.x; i < words; i += kMbThreads) s_img[i] = img[i];
  __syncthreads();
  uint32_t ctr = fmix32(seed ^ t);
  uint32_t acc = 0;
#pragma unroll 4
  for (int64_t j = 0; j < per_thread; ++j) {
    ctr += kWeyl;
    const uint64_t idx = ((uint64_t)fmix32(ctr) * words) >> 32;
    access<K>(s_img, idx, t, acc);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < words; i += kMbThreads) img[i] = s_img[i];
  if (sink != nullptr) sink[t] = acc;
}

template <int K>
hipError_t launch_random(uint32_t *buf, uint64_t words, int32_t memory, uint32_t seed, int64_t per_thread,
                         int32_t blocks, uint32_t *sink, hipStream_t st) {
  if (memory == GT_MEMORY_LDS)
    hipLaunchKernelGGL(k_random_lds<K>, dim3((unsigned)blocks), dim3(kMbThreads), (size_t)words * 4, st, buf,
                       (uint32_t)words, seed, per_thread, sink);
  else
    hipLaunchKernelGGL(k_random_global<K>, dim3((unsigned)blocks), dim3(kMbThreads), 0, st, buf, words, seed,
                       per_thread, sink);
  return hipGetLastError();
}

}  // namespace
}  // namespace gt

extern "C" gt_status gt_random_access(uint32_t *buf, uint64_t words, int32_t kind, int32_t memory, uint32_t seed,
                                      int64_t per_thread, int32_t blocks, uint32_t *sink, void *stream) {
  using namespace gt;
  if (buf == nullptr || words == 0 || per_thread < 0 || blocks < 1 || blocks > kMbMaxBlocks)
    return GT_ERR_INVALID_ARGUMENT;
  if (kind < GT_ACCESS_READ || kind > GT_ACCESS_INDEX || (memory != GT_MEMORY_GLOBAL && memory != GT_MEMORY_LDS))
    return GT_ERR_INVALID_ARGUMENT;
  if (words > (memory == GT_MEMORY_LDS ? kMbMaxLdsWords : (uint64_t)1 << 32)) return GT_ERR_UNSUPPORTED;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  switch (kind) {
    case GT_ACCESS_READ: e = launch_random<GT_ACCESS_READ>(buf, words, memory, seed, per_thread, blocks, sink, st); break;
    case GT_ACCESS_WRITE: e = launch_random<GT_ACCESS_WRITE>(buf, words, memory, seed, per_thread, blocks, sink, st); break;
    case GT_ACCESS_ATOMIC: e = launch_random<GT_ACCESS_ATOMIC>(buf, words, memory, seed, per_thread, blocks, sink, st); break;
    default: e = launch_random<GT_ACCESS_INDEX>(buf, words, memory, seed, per_thread, blocks, sink, st); break;
  }
  return e == hipSuccess ? GT_OK : GT_ERR_HIP;
}
