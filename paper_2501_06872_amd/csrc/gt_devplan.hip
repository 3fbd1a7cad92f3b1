// Planning on the device (GT_FLAG_DEVICE_PLAN).  The learned choice of every
// graph (Section IV-C: sampled features, the network's predicted times, the
// fastest configuration) is made by kernels and stays in the workspace; every
// gt_transpose_batched call then lays each graph out, builds its kernels'
// arguments and the persistent kernel's phase table in one planning kernel,
// with the same layout functions the host planner uses (gt_layout.hpp).  No
// step needs the host to see the choice, so a plan and its transpositions
// capture into one HIP graph.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gt_device.hpp"
#include "gt_layout.hpp"
#include "gt_mlp.h"

namespace gt {

// x[i][k] = feature k of graph i (each graph's features sit in its own
// sampling scratch).
__global__ void k_gather_features(const float *const *fdev, int32_t count, float *x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)count * kMlpIn) return;
  x[i] = fdev[i / kMlpIn][i % kMlpIn];
}

// The learned choice of every graph when its features lie in the training
// range (a margin of a tenth of the range), else the heuristic's; either
// adjusted to the persistent kernel's bodies (variant-1 tiles, digits of at
// most 9 bits).
__global__ void k_choose(const float *x, const float *y, const float *fmin, const float *fmax, int32_t count,
                         const DevChoice *heur, DevChoice *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  bool in = true;
  for (int k = 0; k < kMlpIn; ++k) {
    const float span = fmax[k] - fmin[k];
    const float margin = 0.1f * span + 0.01f;
    const float v = x[(int64_t)i * kMlpIn + k];
    if (!(v >= fmin[k] - margin && v <= fmax[k] + margin)) in = false;
  }
  DevChoice c = heur[i];
  if (in) {
    const float *yi = y + (int64_t)i * kMlpOut;
    int best = 0;
    for (int k = 1; k < kMlpOut; ++k)
      if (yi[k] < yi[best]) best = k;
    config_params(best, &c.fine_bits, &c.digit_bits, &c.variant);
    c.config = best;
  }
  c.variant = 1;
  if (c.digit_bits > 9) c.digit_bits = 9;
  out[i] = c;
}

// One workgroup: (1) every graph's layout in its region, the arguments of
// its kernels and its phases; (2) the queue, level by level (every graph's
// phase of one kind, the largest graph first), each phase waiting for its
// graph's previous one, the ticket of each phase from a scan of the tickets
// before it; (3) the ticket -> phase table and the queue's size.  The same
// order and the same counts as the host planner's.
constexpr int kPlanThreads = 1024;

__global__ __launch_bounds__(kPlanThreads) void k_persist_plan(DevPlanArgs a) {
  __shared__ uint64_t s_val[kDevPlanMaxGraphs];  // per order position: (tickets << 24) | 1, then its prefix
  __shared__ uint64_t s_w[kPlanThreads / kWave + 1];
  __shared__ uint32_t s_prev[kDevPlanMaxGraphs];  // per graph: its last phase in the queue
  __shared__ uint8_t s_cur[kDevPlanMaxGraphs];    // per graph: its next phase in its own list
  __shared__ uint8_t s_nph[kDevPlanMaxGraphs];    // per graph: its number of phases
  const int tid = threadIdx.x;
  const int count = a.count;
  for (int i = tid; i < count; i += kPlanThreads) {
    const DevGraph &G = a.graphs[i];
    const DevChoice c = a.choice[i];
    GraphPlan p{};
    p.n = G.n;
    p.m = G.m;
    p.pay = G.payload != nullptr;
    p.strategy = GT_STRATEGY_STABLE;
    p.fine_bits = c.fine_bits;
    p.digit_bits = c.digit_bits;
    p.variant = c.variant;
    p.config = c.config;
    finalize_stable(p, G.base);
    gt_csr_t g;
    g.n = G.n; g.m = G.m; g.offsets = G.offsets; g.indices = G.indices; g.payload = G.payload;
    gt_csc_t out;
    out.offsets = G.out_offsets; out.indices = G.out_indices; out.payload = G.out_payload;
    a.desc[i] = stable_launch(p, g, out, a.ws, a.validate);
    PersistPhase *ph = a.tmp + (int64_t)i * kPersistMaxPhases;
    const int k = persist_phases(p, &a.desc[i], &out, i, a.validate, ph);
    for (int j = 0; j < k; ++j) ph[j].chunk = persist_chunk(ph[j].kind, ph[j].nitems, a.grid);
    s_nph[i] = (uint8_t)k;
    s_cur[i] = 0;
    s_prev[i] = kNoDep;
  }
  __syncthreads();
  uint64_t tickets = 0;
  uint32_t phases = 0;
  for (uint32_t kind = 0; kind <= (uint32_t)kPhFinal; ++kind) {
    for (int o = tid; o < count; o += kPlanThreads) {
      const uint32_t g = a.order[o];
      const PersistPhase *ph = a.tmp + (int64_t)g * kPersistMaxPhases;
      uint64_t v = 0;
      if (s_cur[g] < s_nph[g] && ph[s_cur[g]].kind == kind) {
        const PersistPhase &q = ph[s_cur[g]];
        v = ((uint64_t)((q.nitems + q.chunk - 1) / q.chunk) << 24) | 1u;
      }
      s_val[o] = v;
    }
    __syncthreads();
    const uint64_t sum = block_excl_scan<kPlanThreads, uint64_t>(s_val, count, s_w);
    for (int o = tid; o < count; o += kPlanThreads) {
      const uint32_t g = a.order[o];
      const PersistPhase *ph = a.tmp + (int64_t)g * kPersistMaxPhases;
      if (s_cur[g] < s_nph[g] && ph[s_cur[g]].kind == kind) {
        PersistPhase q = ph[s_cur[g]];
        const uint32_t pos = phases + (uint32_t)(s_val[o] & 0xFFFFFFu);
        q.dep = s_prev[g];
        q.start = tickets + (s_val[o] >> 24);
        a.table[pos] = q;
        s_prev[g] = pos;
        s_cur[g] = s_cur[g] + 1;
      }
    }
    tickets += sum >> 24;
    phases += (uint32_t)(sum & 0xFFFFFFu);
    __syncthreads();
  }
  // every phase's tickets in the coarse table; past the end, the last phase
  for (uint32_t j = tid; j < phases; j += kPlanThreads) {
    const PersistPhase &q = a.table[j];
    const uint64_t end = q.start + (q.nitems + q.chunk - 1) / q.chunk;
    constexpr uint64_t step = uint64_t(1) << kPersistTabShift;
    for (uint64_t b = (q.start + step - 1) >> kPersistTabShift; (b << kPersistTabShift) < end; ++b) a.tab[b] = j;
  }
  const uint64_t ntab = (tickets >> kPersistTabShift) + 2;
  for (uint64_t b = ((tickets + (uint64_t(1) << kPersistTabShift) - 1) >> kPersistTabShift) + tid; b < ntab;
       b += kPlanThreads)
    a.tab[b] = phases - 1;
  if (tid == 0) {
    a.meta[0] = tickets;
    a.meta[1] = phases;
  }
}

hipError_t launch_gather_features(const float *const *fdev, int32_t count, float *x, hipStream_t st) {
  const int64_t n = (int64_t)count * kMlpIn;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_features, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, fdev, count, x);
  return hipGetLastError();
}

hipError_t launch_choose(const float *x, const float *y, const float *fmin, const float *fmax, int32_t count,
                         const DevChoice *heur, DevChoice *out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_choose, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, x, y, fmin, fmax, count,
                     heur, out);
  return hipGetLastError();
}

hipError_t launch_persist_plan(const DevPlanArgs &a, hipStream_t st) {
  if (a.count <= 0 || a.count > kDevPlanMaxGraphs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_persist_plan, dim3(1), dim3(kPlanThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace gt
