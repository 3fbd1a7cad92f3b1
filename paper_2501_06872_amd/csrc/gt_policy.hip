// Parameter policies of a plan: heuristic (sizes + sampled features),
// fixed, learned (MLP over sampled features), and the autotuner that times
// every configuration.  None of them can change the output: every
// configuration computes the same stable transposition.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "gt_internal.h"
#include "gt_layout.hpp"
#include "gt_mlp.h"
#include "gt_plan.h"
#include "gt_sample.h"

namespace gt {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Sampling scratch of every graph of a plan, laid out back to back, then the
// learned policy's parameters, inputs and outputs.
size_t plan_scratch_bytes(const gt_csr_t *graphs, int32_t count) {
  size_t total = 0;
  for (int32_t i = 0; i < count; ++i) total += align256(sample_scratch_bytes(graphs[i].n, graphs[i].m));
  total += align256(sizeof(float) * ((size_t)kMlpParams + (size_t)count * (kMlpIn + kMlpOut)));
  return total;
}

// Heuristic (sizes only): a k_final bin should hold about one 8K-edge tile,
// so fine_bits ~ log2(8192 / average in-degree); digits of up to 10 bits;
// the 8-wave x 16-edge tile.
static void heuristic(GraphPlan &p) {
  const double avg = p.n > 0 ? (double)p.m / (double)p.n : 1.0;
  int fb = (int)lround(log2(8192.0 / std::max(avg, 1.0)));
  p.fine_bits = std::min(std::max(fb, 4), kMaxFineBits);
  // 10-bit digits only for a single pass: with 19 or 20 coarse bits, three
  // passes of at most 7 bits beat a 10-bit pass (whose 1024 look-back words
  // per tile and 98 KB of LDS allow one workgroup per CU)
  int L = 1;
  while (L < 31 && (int64_t(1) << L) < std::max<int64_t>(p.n, 2)) ++L;
  p.digit_bits = (L - p.fine_bits > 18) ? 9 : 10;
  p.variant = 1;
}

// Scratch region at the end of the workspace.
static char *scratch_base(const gt_csr_t *graphs, int32_t count, void *workspace, size_t workspace_bytes) {
  const size_t need = plan_scratch_bytes(graphs, count);
  if (workspace == nullptr || workspace_bytes < need + 256) return nullptr;
  return static_cast<char *>(workspace) + ((workspace_bytes - need) & ~size_t(255));
}

// Sample every graph of the plan (one synchronisation for all of them) and
// copy the feature vectors to the host.
static gt_status sample_features(gt_plan_st *plan, const gt_csr_t *graphs, int32_t count, uint64_t seed,
                                 char *base, hipStream_t st) {
  std::vector<float *> fdev(count);
  size_t off = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (enqueue_sampling(graphs[i].offsets, graphs[i].indices, graphs[i].n, graphs[i].m,
                         graphs[i].payload != nullptr, seed, base + off, &fdev[i], st) != hipSuccess)
      return GT_ERR_HIP;
    off += align256(sample_scratch_bytes(graphs[i].n, graphs[i].m));
  }
  for (int32_t i = 0; i < count; ++i) {
    GraphPlan &p = plan->graphs[i];
    if (hipMemcpyAsync(p.features, fdev[i], sizeof(float) * kNumFeatures, hipMemcpyDeviceToHost, st) != hipSuccess)
      return GT_ERR_HIP;
    p.nfeatures = kNumFeatures;
  }
  if (hipStreamSynchronize(st) != hipSuccess) return GT_ERR_HIP;
  return GT_OK;
}

// Model file: "GTMLP1\0\0", int32 inputs, hidden, outputs, nparams, then
// float params[nparams], fmin[inputs], fmax[inputs] (the training range).
struct MlpModel {
  std::vector<float> params, fmin, fmax;
};

static bool load_model(const char *path, MlpModel &mdl) {
  if (path == nullptr) return false;
  FILE *f = fopen(path, "rb");
  if (!f) return false;
  char magic[8];
  int32_t hdr[4];
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "GTMLP1\0\0", 8) == 0 && fread(hdr, 4, 4, f) == 4 &&
            hdr[0] == kMlpIn && hdr[1] == kMlpHidden && hdr[2] == kMlpOut && hdr[3] == kMlpParams;
  if (ok) {
    mdl.params.resize(kMlpParams);
    mdl.fmin.resize(kMlpIn);
    mdl.fmax.resize(kMlpIn);
    ok = fread(mdl.params.data(), 4, kMlpParams, f) == (size_t)kMlpParams &&
         fread(mdl.fmin.data(), 4, kMlpIn, f) == (size_t)kMlpIn && fread(mdl.fmax.data(), 4, kMlpIn, f) == (size_t)kMlpIn;
  }
  fclose(f);
  return ok;
}

static bool in_training_range(const MlpModel &mdl, const float *x) {
  for (int k = 0; k < kMlpIn; ++k) {
    const float span = mdl.fmax[k] - mdl.fmin[k];
    const float margin = 0.1f * span + 0.01f;
    if (!(x[k] >= mdl.fmin[k] - margin && x[k] <= mdl.fmax[k] + margin)) return false;
  }
  return true;
}

// Learned choice for every graph: the MLP's forward pass on the device, the
// argmin over the predicted run times on the host.  Graphs whose features
// leave the training range keep the heuristic.
static gt_status mlp_choose(gt_plan_st *plan, int32_t count, const MlpModel &mdl, char *mbase, hipStream_t st) {
  float *dparams = reinterpret_cast<float *>(mbase);
  float *dx = dparams + kMlpParams;
  float *dy = dx + (size_t)count * kMlpIn;
  std::vector<float> x((size_t)count * kMlpIn), y((size_t)count * kMlpOut);
  for (int32_t i = 0; i < count; ++i)
    for (int k = 0; k < kMlpIn; ++k) x[(size_t)i * kMlpIn + k] = plan->graphs[i].features[k];
  if (hipMemcpyAsync(dparams, mdl.params.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dx, x.data(), sizeof(float) * x.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
      mlp_forward(dparams, dx, count, dy, st) != hipSuccess ||
      hipMemcpyAsync(y.data(), dy, sizeof(float) * y.size(), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return GT_ERR_HIP;
  for (int32_t i = 0; i < count; ++i) {
    GraphPlan &p = plan->graphs[i];
    if (!in_training_range(mdl, p.features)) continue;
    int best = 0;
    for (int c = 1; c < kMlpOut; ++c)
      if (y[(size_t)i * kMlpOut + c] < y[(size_t)i * kMlpOut + best]) best = c;
    config_params(best, &p.fine_bits, &p.digit_bits, &p.variant);
    p.learned = true;
    p.config = best;
  }
  return GT_OK;
}

gt_status device_plan_setup(gt_plan_st *plan, const gt_csr_t *graphs, const gt_options_t &opt, char *ws,
                            hipStream_t st) {
  const int32_t count = plan->count;
  const DevPlanStage d = dev_plan_stage(count);
  if (hipHostMalloc(&plan->dp_host, d.staged, hipHostMallocDefault) != hipSuccess) {
    plan->dp_host = nullptr;
    return GT_ERR_HIP;
  }
  plan->dp_bytes = d.staged;
  if (hipEventCreateWithFlags(&plan->dp_event, hipEventDisableTiming) != hipSuccess) {
    plan->dp_event = nullptr;
    return GT_ERR_HIP;
  }
  char *h = static_cast<char *>(plan->dp_host);
  char *dev = ws + plan->off_pdp;
  DevChoice *heur = reinterpret_cast<DevChoice *>(h + d.heur);
  for (int32_t i = 0; i < count; ++i) {
    const GraphPlan &p = plan->graphs[i];
    heur[i] = DevChoice{p.fine_bits, p.digit_bits, p.variant, -1};
  }
  // the queue order: graphs by edge count, the largest first (ties: index)
  plan->order.resize(count);
  for (int32_t i = 0; i < count; ++i) plan->order[i] = (uint32_t)i;
  std::stable_sort(plan->order.begin(), plan->order.end(),
                   [&](uint32_t a, uint32_t b) { return plan->graphs[a].m > plan->graphs[b].m; });
  DevChoice *choice = reinterpret_cast<DevChoice *>(ws + plan->off_pchoice);
  MlpModel mdl;
  if (!load_model(opt.model_path, mdl)) {  // no network: the heuristic's choices
    if (hipMemcpyAsync(dev + d.heur, h + d.heur, sizeof(DevChoice) * (size_t)count, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(choice, dev + d.heur, sizeof(DevChoice) * (size_t)count, hipMemcpyDeviceToDevice, st) !=
            hipSuccess ||
        hipEventRecord(plan->dp_event, st) != hipSuccess)
      return GT_ERR_HIP;
    return GT_OK;
  }
  memcpy(h + d.params, mdl.params.data(), sizeof(float) * kMlpParams);
  memcpy(h + d.fmin, mdl.fmin.data(), sizeof(float) * kMlpIn);
  memcpy(h + d.fmax, mdl.fmax.data(), sizeof(float) * kMlpIn);
  // Step 0 of every graph into its own sampling scratch
  float **fdev = reinterpret_cast<float **>(h + d.fdev);
  char *samp = ws + plan->off_psamp;
  for (int32_t i = 0; i < count; ++i) {
    if (enqueue_sampling(graphs[i].offsets, graphs[i].indices, graphs[i].n, graphs[i].m,
                         graphs[i].payload != nullptr, opt.seed ? opt.seed : 0x5eedull, samp, &fdev[i], st) !=
        hipSuccess)
      return GT_ERR_HIP;
    samp += align256(sample_scratch_bytes(graphs[i].n, graphs[i].m));
  }
  float *x = reinterpret_cast<float *>(dev + d.x);
  float *y = reinterpret_cast<float *>(dev + d.y);
  if (hipMemcpyAsync(dev, h, d.staged, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(plan->dp_event, st) != hipSuccess ||
      launch_gather_features(reinterpret_cast<const float *const *>(dev + d.fdev), count, x, st) != hipSuccess ||
      mlp_forward(reinterpret_cast<const float *>(dev + d.params), x, count, y, st) != hipSuccess ||
      launch_choose(x, y, reinterpret_cast<const float *>(dev + d.fmin), reinterpret_cast<const float *>(dev + d.fmax),
                    count, reinterpret_cast<const DevChoice *>(dev + d.heur), choice, st) != hipSuccess)
    return GT_ERR_HIP;
  return GT_OK;
}

gt_status choose_params(gt_plan_st *plan, const gt_csr_t *graphs, int32_t count, const gt_options_t &opt,
                        void *workspace, size_t workspace_bytes, hipStream_t st) {
  for (int32_t i = 0; i < count; ++i) {
    GraphPlan &p = plan->graphs[i];
    p = GraphPlan{};
    p.n = graphs[i].n;
    p.m = graphs[i].m;
    p.pay = graphs[i].payload != nullptr;
    p.force_wide = (opt.flags & GT_FLAG_WIDE_STATUS) != 0;
    p.step3 = (opt.flags & GT_FLAG_STEP3_STEAL) ? 2 : ((opt.flags & GT_FLAG_STEP3_STATIC) ? 1 : 0);
    p.step3_times = (opt.flags & GT_FLAG_STEP3_TIMES) != 0;
    p.config = -1;
    p.strategy = opt.strategy;
    p.hdv_max = opt.hdv_max;
    p.seed = opt.seed ? opt.seed : 0x5eedull;
    heuristic(p);
    if (opt.policy == GT_POLICY_FIXED) {
      if (opt.fine_bits) p.fine_bits = opt.fine_bits;
      if (opt.digit_bits) p.digit_bits = opt.digit_bits;
      if (opt.variant) p.variant = opt.variant;
    }
  }
  // HEURISTIC and FIXED choose from the sizes alone: no device work and no
  // synchronisation unless features were asked for.
  // a device plan samples and chooses on the device (device_plan_setup)
  if ((opt.policy == GT_POLICY_MLP || (opt.flags & GT_FLAG_FEATURES)) && !(opt.flags & GT_FLAG_DEVICE_PLAN)) {
    char *base = scratch_base(graphs, count, workspace, workspace_bytes);
    if (base == nullptr) return GT_ERR_WORKSPACE_TOO_SMALL;
    gt_status s = sample_features(plan, graphs, count, opt.seed ? opt.seed : 0x5eedull, base, st);
    if (s != GT_OK) return s;
    if (opt.policy == GT_POLICY_MLP) {
      MlpModel mdl;
      if (load_model(opt.model_path, mdl)) {
        size_t off = 0;
        for (int32_t i = 0; i < count; ++i) off += align256(sample_scratch_bytes(graphs[i].n, graphs[i].m));
        s = mlp_choose(plan, count, mdl, base + off, st);
        if (s != GT_OK) return s;
      }
    }
  }
  return GT_OK;
}

// Batched launch: graphs are spread over kLanes internal streams (largest
// first, each to the least loaded lane), forked from the caller's stream by
// one event and joined back by one event per lane, so the kernels of small
// graphs run concurrently.  Everything is enqueued without a host
// synchronisation, so the whole batch can be captured into one HIP graph.
constexpr int kLanes = 8;

static gt_status ensure_lanes(gt_plan_st *plan) {
  if (!plan->lanes.empty()) return GT_OK;
  const int nl = std::min<int>(kLanes, std::max<int32_t>(plan->count, 1));
  for (int i = 0; i < nl; ++i) {
    hipStream_t s;
    hipEvent_t e;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return GT_ERR_HIP;
    plan->lanes.push_back(s);
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return GT_ERR_HIP;
    plan->lane_events.push_back(e);
  }
  if (hipEventCreateWithFlags(&plan->fork_event, hipEventDisableTiming) != hipSuccess) return GT_ERR_HIP;
  // assignment: largest graphs first, each to the lane with the least edges
  std::vector<int> order(plan->count);
  for (int i = 0; i < plan->count; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return plan->graphs[a].m > plan->graphs[b].m; });
  std::vector<double> load(nl, 0.0);
  plan->lane_of.assign(plan->count, 0);
  for (int i : order) {
    int best = 0;
    for (int l = 1; l < nl; ++l) if (load[l] < load[best]) best = l;
    plan->lane_of[i] = best;
    load[best] += (double)plan->graphs[i].m + 1e5;  // per-graph fixed cost
  }
  return GT_OK;
}

// ---- Persistent batched launch.  The phase table: every graph's phases in
// pipeline order (PersistKind order), each waiting for the graph's previous
// phase; the queue holds them level by level (all graphs' phases of one kind,
// the largest graph first, before any phase of the next kind), so that the
// items of a level find their graph's previous level finished or nearly so.
// A device plan: the graphs' pointers and the queue order to the device,
// then the planning kernel (layout, kernel arguments, phase table, ticket
// table, queue size) and the persistent kernel.
static gt_status enqueue_device_planned(gt_plan_st *plan, const gt_csr_t *graphs, const gt_csc_t *outs, char *ws,
                                        hipStream_t st) {
  const int32_t count = plan->count;
  char *host = static_cast<char *>(plan->pk_host);
  DevGraph *dg = reinterpret_cast<DevGraph *>(host);
  uint32_t *order = reinterpret_cast<uint32_t *>(host + (plan->off_porder - plan->off_pgraph));
  for (int32_t i = 0; i < count; ++i) {
    DevGraph &g = dg[i];
    g.n = graphs[i].n;
    g.m = graphs[i].m;
    g.offsets = graphs[i].offsets;
    g.indices = graphs[i].indices;
    g.payload = graphs[i].payload;
    g.out_offsets = outs[i].offsets;
    g.out_indices = outs[i].indices;
    g.out_payload = outs[i].payload;
    g.base = plan->graph_base[i];
    order[i] = plan->order[i];
  }
  const size_t copy = plan->off_porder + sizeof(uint32_t) * (size_t)count - plan->off_pgraph;
  if (hipMemcpyAsync(ws + plan->off_pgraph, host, copy, hipMemcpyHostToDevice, st) != hipSuccess) return GT_ERR_HIP;
  if (hipEventRecord(plan->pk_event, st) != hipSuccess) return GT_ERR_HIP;
  plan->pk_pending = true;
  // status word, ticket and the done counters of every phase there can be
  if (launch_fill(reinterpret_cast<uint32_t *>(ws), persist_counters_end(count) / 4, 0u, st) != hipSuccess)
    return GT_ERR_HIP;
  DevPlanArgs d{};
  d.graphs = reinterpret_cast<const DevGraph *>(ws + plan->off_pgraph);
  d.order = reinterpret_cast<const uint32_t *>(ws + plan->off_porder);
  d.choice = reinterpret_cast<const DevChoice *>(ws + plan->off_pchoice);
  d.count = count;
  d.validate = plan->validate;
  d.grid = plan->pk_grid;
  d.ws = ws;
  d.desc = reinterpret_cast<StableLaunch *>(ws + plan->off_pdesc);
  d.tmp = reinterpret_cast<PersistPhase *>(ws + plan->off_ptmp);
  d.table = reinterpret_cast<PersistPhase *>(ws + plan->off_pphase);
  d.tab = reinterpret_cast<uint32_t *>(ws + plan->off_ptab);
  d.meta = reinterpret_cast<uint64_t *>(ws + plan->off_pmeta);
  if (launch_persist_plan(d, st) != hipSuccess) return GT_ERR_HIP;
  PersistArgs a{};
  a.graphs = d.desc;
  a.phases = d.table;
  a.meta = d.meta;
  a.tab = d.tab;
  a.ticket = reinterpret_cast<unsigned long long *>(ws + 8);
  a.done = reinterpret_cast<uint32_t *>(ws + kPersistDoneOff);
  a.err = reinterpret_cast<uint32_t *>(ws);
  if (launch_persistent(a, plan->pk_grid, st) != hipSuccess) return GT_ERR_HIP;
  return GT_OK;
}

static gt_status enqueue_persistent(gt_plan_st *plan, const gt_csr_t *graphs, const gt_csc_t *outs, char *ws,
                                    hipStream_t st) {
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return GT_ERR_HIP;
  // the previous call's copy may still read the staging buffer
  if (plan->pk_pending && cap == hipStreamCaptureStatusNone) {
    if (hipEventSynchronize(plan->pk_event) != hipSuccess) return GT_ERR_HIP;
    plan->pk_pending = false;
  }
  if (plan->device_plan) return enqueue_device_planned(plan, graphs, outs, ws, st);
  const int32_t count = plan->count;
  char *host = static_cast<char *>(plan->pk_host);
  StableLaunch *desc = reinterpret_cast<StableLaunch *>(host);
  PersistPhase *table = reinterpret_cast<PersistPhase *>(host + (plan->off_pphase - plan->off_pdesc));
  uint32_t *tab = reinterpret_cast<uint32_t *>(host + (plan->off_ptab - plan->off_pdesc));
  // every graph's phases, then the queue order
  std::vector<PersistPhase> all;
  all.reserve((size_t)count * kPersistMaxPhases);
  std::vector<int> first(count);
  PersistPhase buf[kPersistMaxPhases];
  for (int32_t i = 0; i < count; ++i) {
    const GraphPlan &p = plan->graphs[i];
    desc[i] = stable_launch(p, graphs[i], outs[i], ws, plan->validate);
    const int k = persist_phases(p, &desc[i], &outs[i], i, plan->validate, buf);
    first[i] = (int)all.size();
    all.insert(all.end(), buf, buf + k);
  }
  std::vector<int> order(all.size());
  for (size_t j = 0; j < order.size(); ++j) order[j] = (int)j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const PersistPhase &x = all[a], &y = all[b];
    if (x.kind != y.kind) return x.kind < y.kind;
    const int64_t mx = plan->graphs[x.graph].m, my = plan->graphs[y.graph].m;
    if (mx != my) return mx > my;
    return x.graph < y.graph;
  });
  std::vector<uint32_t> pos(all.size());
  for (size_t j = 0; j < order.size(); ++j) pos[order[j]] = (uint32_t)j;
  uint64_t total = 0;
  for (size_t j = 0; j < order.size(); ++j) {
    const int a = order[j];
    PersistPhase q = all[a];
    const int i = (int)q.graph;
    q.dep = a > first[i] ? pos[a - 1] : kNoDep;  // the graph's previous phase
    q.chunk = persist_chunk(q.kind, q.nitems, plan->pk_grid);
    q.start = total;
    total += (q.nitems + q.chunk - 1) / q.chunk;
    table[j] = q;
  }
  const int32_t nphases = (int32_t)order.size();
  if (total == 0) return GT_OK;
  // coarse ticket -> phase table
  const uint64_t ntab = (total >> kPersistTabShift) + 2;
  if (ntab > plan->ptab_entries) return GT_ERR_INVALID_ARGUMENT;
  for (uint64_t b = 0, j = 0; b < ntab; ++b) {
    const uint64_t t = std::min<uint64_t>(b << kPersistTabShift, total - 1);
    while (j + 1 < (uint64_t)nphases && table[j + 1].start <= t) ++j;
    tab[b] = (uint32_t)j;
  }
  uint64_t *meta = reinterpret_cast<uint64_t *>(host + (plan->off_pmeta - plan->off_pdesc));
  meta[0] = total;
  meta[1] = (uint64_t)nphases;
  const size_t copy = plan->off_pmeta + 2 * sizeof(uint64_t) - plan->off_pdesc;
  if (hipMemcpyAsync(ws + plan->off_pdesc, host, copy, hipMemcpyHostToDevice, st) != hipSuccess) return GT_ERR_HIP;
  if (hipEventRecord(plan->pk_event, st) != hipSuccess) return GT_ERR_HIP;
  plan->pk_pending = true;
  // status word, ticket and done counters
  if (launch_fill(reinterpret_cast<uint32_t *>(ws), (kPersistDoneOff + 4 * (size_t)nphases) / 4, 0u, st) !=
      hipSuccess)
    return GT_ERR_HIP;
  PersistArgs a{};
  a.graphs = reinterpret_cast<const StableLaunch *>(ws + plan->off_pdesc);
  a.phases = reinterpret_cast<const PersistPhase *>(ws + plan->off_pphase);
  a.meta = reinterpret_cast<const uint64_t *>(ws + plan->off_pmeta);
  a.tab = reinterpret_cast<const uint32_t *>(ws + plan->off_ptab);
  a.ticket = reinterpret_cast<unsigned long long *>(ws + 8);
  a.done = reinterpret_cast<uint32_t *>(ws + kPersistDoneOff);
  a.err = reinterpret_cast<uint32_t *>(ws);
  const int grid = (int)std::min<uint64_t>((uint64_t)plan->pk_grid, total);
  if (launch_persistent(a, grid, st) != hipSuccess) return GT_ERR_HIP;
  return GT_OK;
}

gt_status enqueue_batched(gt_plan_st *plan, const gt_csr_t *graphs, const gt_csc_t *outs, char *ws,
                          hipStream_t st) {
  if (plan->persistent) return enqueue_persistent(plan, graphs, outs, ws, st);
  gt_status s = ensure_lanes(plan);
  if (s != GT_OK) return s;
  if (launch_fill(reinterpret_cast<uint32_t *>(ws), 1, 0u, st) != hipSuccess) return GT_ERR_HIP;
  if (hipEventRecord(plan->fork_event, st) != hipSuccess) return GT_ERR_HIP;
  for (hipStream_t l : plan->lanes)
    if (hipStreamWaitEvent(l, plan->fork_event, 0) != hipSuccess) return GT_ERR_HIP;
  Profiler *prof = nullptr;  // per-kernel events are recorded for single-stream launches only
  for (int32_t i = 0; i < plan->count; ++i) {
    s = enqueue_graph(plan->graphs[i], graphs[i], outs[i], ws, plan->validate, false, prof,
                      plan->lanes[plan->lane_of[i]]);
    if (s != GT_OK) return s;
  }
  for (size_t l = 0; l < plan->lanes.size(); ++l) {
    if (hipEventRecord(plan->lane_events[l], plan->lanes[l]) != hipSuccess) return GT_ERR_HIP;
    if (hipStreamWaitEvent(st, plan->lane_events[l], 0) != hipSuccess) return GT_ERR_HIP;
  }
  return GT_OK;
}

}  // namespace gt

using namespace gt;

extern "C" {

int32_t gt_num_configs(void) { return kMlpOut; }

gt_status gt_config(int32_t idx, int32_t *fine_bits, int32_t *digit_bits, int32_t *variant) {
  if (idx < 0 || idx >= kMlpOut) return GT_ERR_INVALID_ARGUMENT;
  int fb, db, v;
  config_params(idx, &fb, &db, &v);
  if (fine_bits) *fine_bits = fb;
  if (digit_bits) *digit_bits = db;
  if (variant) *variant = v;
  return GT_OK;
}

gt_status gt_plan_features(gt_plan_t plan, int32_t i, float *out, int32_t nmax, int32_t *nout) {
  if (plan == nullptr || i < 0 || i >= plan->count || out == nullptr || nout == nullptr) return GT_ERR_INVALID_ARGUMENT;
  const GraphPlan &p = plan->graphs[i];
  const int32_t k = std::min<int32_t>(nmax, p.nfeatures);
  for (int32_t j = 0; j < k; ++j) out[j] = p.features[j];
  *nout = p.nfeatures;
  return GT_OK;
}

// Time every configuration on one graph (median of `reps` timed runs after
// one warm-up, HIP events on `stream`); ms_out[c] for c < gt_num_configs().
// The output buffers receive the (identical) transposition.  Synchronous.
gt_status gt_autotune(const gt_csr_t *g, gt_csc_t *out, void *workspace, size_t workspace_bytes, void *stream,
                      int32_t reps, float *ms_out) {
  if (g == nullptr || out == nullptr || workspace == nullptr || ms_out == nullptr || reps < 1)
    return GT_ERR_INVALID_ARGUMENT;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return GT_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return GT_ERR_HIP; }
  gt_status status = GT_OK;
  std::vector<float> t(reps);
  for (int c = 0; c < kMlpOut && status == GT_OK; ++c) {
    gt_options_t o{};
    o.policy = GT_POLICY_FIXED;
    config_params(c, &o.fine_bits, &o.digit_bits, &o.variant);
    gt_plan_t plan = nullptr;
    status = gt_plan(g, 1, &o, workspace, workspace_bytes, stream, &plan);
    if (status != GT_OK) break;
    status = gt_transpose(plan, g, out, workspace, workspace_bytes, stream);
    for (int r = 0; r < reps && status == GT_OK; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess) { status = GT_ERR_HIP; break; }
      status = gt_transpose(plan, g, out, workspace, workspace_bytes, stream);
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t[r], e0, e1) != hipSuccess)
        status = GT_ERR_HIP;
    }
    gt_plan_destroy(plan);
    if (status != GT_OK) break;
    std::vector<float> s(t);
    std::sort(s.begin(), s.end());
    ms_out[c] = s[reps / 2];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}

// Replace the parameters of graph i of a plan by configuration `config`
// (e.g. the autotuner's best); the plan's workspace size may grow.
gt_status gt_plan_set_config(gt_plan_t plan, int32_t i, int32_t config) {
  if (plan == nullptr || i < 0 || i >= plan->count || config < 0 || config >= kMlpOut) return GT_ERR_INVALID_ARGUMENT;
  if (plan->device_plan) return GT_ERR_UNSUPPORTED;  // the choice lives on the device
  GraphPlan &p = plan->graphs[i];
  const GraphPlan keep = p;
  config_params(config, &p.fine_bits, &p.digit_bits, &p.variant);
  p.config = config;
  if (plan->persistent) persist_coerce(p);
  layout_plan(plan);
  if (plan->persistent && !persist_eligible(p)) {
    p = keep;
    layout_plan(plan);
    return GT_ERR_UNSUPPORTED;
  }
  return plan->persistent ? persist_staging(plan) : GT_OK;
}

}  // extern "C"
