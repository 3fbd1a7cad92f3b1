// C ABI of the transposition library: planning, workspace layout, launch
// sequence.  See include/gt.h for the contract.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/gt.h"
#include "gt_internal.h"
#include "gt_layout.hpp"
#include "gt_mlp.h"
#include "gt_plan.h"
#include "gt_sample.h"
#include "gt_unordered.h"

using namespace gt;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int ceil_log2(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x) ++b;
  return b;
}

bool valid_csr_args(const gt_csr_t &g) {
  if (g.n < 0 || g.m < 0 || g.n > INT32_MAX) return false;
  if (g.offsets == nullptr) return false;
  if (g.m > 0 && g.indices == nullptr) return false;
  return true;
}

// Argument status of one graph: the descriptor itself, then the size limit
// (m <= 2^32 keeps every per-vertex chunk prefix of a big bin in 32 bits).
gt_status csr_args_status(const gt_csr_t &g) {
  if (!valid_csr_args(g)) return GT_ERR_INVALID_ARGUMENT;
  if (g.m > kMaxEdges) return GT_ERR_UNSUPPORTED;
  return GT_OK;
}

gt_status graphs_args_status(const gt_csr_t *graphs, int32_t count) {
  for (int32_t i = 0; i < count; ++i) {
    const gt_status s = csr_args_status(graphs[i]);
    if (s != GT_OK) return s;
  }
  return GT_OK;
}

// Scratch of gt_transpose_noalloc, for callers that cannot allocate device
// memory: one static array per GPU, held from the module's load on that GPU
// until the process ends.  In host code the array's name is not a device
// address; each device's copy is resolved once, with that device current,
// by hipGetSymbolAddress, and only that pointer is handed to kernels.
__device__ __align__(256) unsigned char scratch[GT_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices];

// The current device's copy of `scratch` (resolved on the first call there).
gt_status current_scratch(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return GT_ERR_HIP;
  if (dev < 0 || dev >= kMaxScratchDevices) return GT_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return GT_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GT_OK;
}

}  // namespace

namespace gt {

// Derive passes/shifts/bins from (n, m, fine_bits, digit_bits, variant) and
// lay out the workspace regions of one graph starting at byte `base`.
// Workspace of the unordered strategies: sampling scratch (HLH), frequency
// histogram and HDV list, in-degree counters, LDV cursors, per-chunk HDV
// counts, scan status words.
size_t unordered_workspace_end(GraphPlan &p, size_t base) {
  const bool hlh = p.strategy == GT_STRATEGY_HLH;
  p.kmax = hlh ? (p.hdv_max > 0 && p.hdv_max < kHlhMaxHdv ? p.hdv_max : kHlhMaxHdv) : 0;
  // chunks of at least 64K edges: up to 2048 (dispatched), or as many as
  // workgroups of the scatter fit on the device (static, two-phase)
  int64_t max_chunks = 2048;
  if (p.step3 != 0) {
    const int64_t resident = hlh_resident_workgroups();
    max_chunks = resident > 0 ? resident : 512;
  }
  p.nchunks = p.m > 0 ? std::min<int64_t>(std::max<int64_t>((p.m + 65535) / 65536, 1), max_chunks) : 0;
  p.chunk = p.nchunks > 0 ? (p.m + p.nchunks - 1) / p.nchunks : 0;
  // two-phase Step 3: a head of 80% of the chunk, then four tail parts
  p.nparts = p.step3 == 2 ? 5 : 1;
  p.head = p.step3 == 2 ? (p.chunk * 4) / 5 : p.chunk;
  size_t off = base;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const size_t nv = (size_t)std::max<int64_t>(p.n, 1);
  p.off_u_samp = hlh ? take(sample_scratch_bytes(p.n, p.m)) : 0;
  p.off_u_hist = take(4 * (size_t)kHdvHistBins);
  p.off_u_thr = take(4);
  p.off_u_hdv = take(4 * (size_t)std::max(p.kmax, 1));
  p.off_u_nhdv = take(4);
  p.off_u_cnt = take(4 * nv);
  p.off_u_cur = take(8 * nv);
  p.off_u_H = take(4 * (size_t)std::max<int64_t>(p.nchunks * p.nparts, 1) * (size_t)std::max(p.kmax, 1));
  p.off_u_steal = take(4);
  p.off_u_times = p.step3_times ? take(24 * (size_t)std::max<int64_t>(p.nchunks, 1)) : 0;
  p.off_u_sstatus = take(8 * (size_t)((p.n + offsets_scan_tile() - 1) / offsets_scan_tile() + 1));
  p.off_u_ticket = take(4);
  return off;
}

void finalize_params(GraphPlan &p, size_t base) {
  if (p.strategy != GT_STRATEGY_STABLE) {
    p.ws_end = unordered_workspace_end(p, base);
    return;
  }
  finalize_stable(p, base);
}

size_t persist_counters_end(int32_t count) {
  return kPersistDoneOff + 4 * (size_t)count * kPersistMaxPhases;
}

size_t persist_tables_bytes(int32_t count, uint64_t tab_entries) {
  return align_up(sizeof(StableLaunch) * (size_t)count) +
         align_up(sizeof(PersistPhase) * (size_t)count * kPersistMaxPhases) + align_up(4 * (size_t)tab_entries) +
         align_up(2 * sizeof(uint64_t));
}

DevPlanStage dev_plan_stage(int32_t count) {
  DevPlanStage d{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = (off + bytes + 15) & ~size_t(15); return o; };
  d.params = take(sizeof(float) * kMlpParams);
  d.fmin = take(sizeof(float) * kMlpIn);
  d.fmax = take(sizeof(float) * kMlpIn);
  d.heur = take(sizeof(DevChoice) * (size_t)count);
  d.fdev = take(sizeof(float *) * (size_t)count);
  d.staged = off;  // the parts above are copied from the host
  d.x = take(sizeof(float) * kMlpIn * (size_t)count);
  d.y = take(sizeof(float) * kMlpOut * (size_t)count);
  d.total = off;
  return d;
}

size_t device_plan_bytes(int32_t count) {
  return align_up(sizeof(PersistPhase) * (size_t)count * kPersistMaxPhases) +
         align_up(sizeof(DevChoice) * (size_t)count) + align_up(sizeof(DevGraph) * (size_t)count) +
         align_up(sizeof(uint32_t) * (size_t)count) + align_up(dev_plan_stage(count).total);
}

// A device plan's region for one graph: the most any choice the network or
// the heuristic can make needs; false if one of them does not fit the
// persistent kernel's bodies.
static bool device_region(const GraphPlan &heur, size_t *bytes) {
  size_t most = 0;
  bool ok = true;
  for (int c = -1; c < kMlpOut; ++c) {
    GraphPlan q = heur;
    if (c >= 0) config_params(c, &q.fine_bits, &q.digit_bits, &q.variant);
    persist_coerce(q);
    finalize_stable(q, 0);
    most = std::max(most, q.ws_end);
    ok = ok && persist_eligible(q);
  }
  *bytes = most;
  return ok;
}

uint64_t persist_item_bound(int64_t n, int64_t m) {
  // fixed-size phases, tiles of the passes and their scans, bins, work items
  return 8192 + 8 * ((uint64_t)m / 4096 + 1) + 4 * ((uint64_t)n + 1);
}

void layout_plan(gt_plan_st *plan) {
  size_t base = plan->persistent ? align_up(persist_counters_end(plan->count)) : kAlign;  // byte 0: status word
  if (plan->device_plan) plan->graph_base.assign(plan->count, 0);
  for (int32_t i = 0; i < plan->count; ++i) {
    GraphPlan &p = plan->graphs[i];
    finalize_params(p, base);
    if (plan->device_plan) {  // a region for any choice
      size_t most = 0;
      (void)device_region(p, &most);
      plan->graph_base[i] = base;
      base = align_up(base + std::max(most, p.ws_end - base));
    } else {
      base = align_up(p.ws_end);
    }
  }
  if (plan->persistent) {
    uint64_t items = 0;
    PersistPhase buf[kPersistMaxPhases];
    for (const GraphPlan &p : plan->graphs) {
      if (plan->device_plan) {  // any choice
        items += persist_item_bound(p.n, p.m);
        continue;
      }
      const int k = persist_phases(p, nullptr, nullptr, 0, plan->validate, buf);
      for (int j = 0; j < k; ++j) items += buf[j].nitems;
    }
    plan->ptab_entries = (items >> kPersistTabShift) + 2;  // tickets <= items
    plan->off_pdesc = base;
    plan->off_pphase = base + align_up(sizeof(StableLaunch) * (size_t)plan->count);
    plan->off_ptab = plan->off_pphase + align_up(sizeof(PersistPhase) * (size_t)plan->count * kPersistMaxPhases);
    plan->off_pmeta = plan->off_ptab + align_up(4 * (size_t)plan->ptab_entries);
    base += persist_tables_bytes(plan->count, plan->ptab_entries);
  }
  if (plan->device_plan) {
    const size_t n = (size_t)plan->count;
    plan->off_ptmp = base;
    plan->off_pchoice = plan->off_ptmp + align_up(sizeof(PersistPhase) * n * kPersistMaxPhases);
    plan->off_pgraph = plan->off_pchoice + align_up(sizeof(DevChoice) * n);
    plan->off_porder = plan->off_pgraph + align_up(sizeof(DevGraph) * n);
    plan->off_pdp = plan->off_porder + align_up(sizeof(uint32_t) * n);
    plan->off_psamp = plan->off_pdp + align_up(dev_plan_stage(plan->count).total);
    base = plan->off_psamp;
    for (const GraphPlan &p : plan->graphs) base += align_up(sample_scratch_bytes(p.n, p.m));
  }
  plan->ws_bytes = std::max<size_t>(base, 256);
}

// Largest workspace any policy can need for one graph.
size_t graph_workspace_bound(int64_t n, int64_t m, bool pay) {
  size_t best = 0;
  for (int fb = 0; fb <= kMaxFineBits; ++fb)
    for (int variant = 1; variant <= 4; ++variant)
      for (int db = 4; db <= 10; ++db) {
        GraphPlan p{};
        p.n = n; p.m = m; p.pay = pay; p.fine_bits = fb; p.digit_bits = db; p.variant = variant;
        p.force_wide = true;
        finalize_params(p, 0);
        best = std::max(best, p.ws_end);
      }
  for (int strategy : {GT_STRATEGY_HLH, GT_STRATEGY_ATOMIC})
    for (int step3 : {0, 2}) {  // the static mode needs less than the two-phase one
      GraphPlan p{};
      p.n = n; p.m = m; p.pay = pay; p.strategy = strategy;
      p.step3 = step3;
      p.step3_times = true;
      best = std::max(best, unordered_workspace_end(p, 0));
    }
  return best;
}

hipEvent_t Profiler::get() {
  if (used == pool.size()) {
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    pool.push_back(ev);
  }
  return pool[used++];
}

hipError_t Profiler::begin(const char *name, hipStream_t st) {
  if (!on) return hipSuccess;
  ProfRec r{name, get(), get()};
  if (!r.start || !r.stop) return hipErrorOutOfMemory;
  recs.push_back(r);
  return hipEventRecord(r.start, st);
}

hipError_t Profiler::end(hipStream_t st) {
  if (!on || recs.empty()) return hipSuccess;
  return hipEventRecord(recs.back().stop, st);
}

// Enqueue the whole transposition of one graph.
gt_status enqueue_graph(const GraphPlan &p, const gt_csr_t &g, const gt_csc_t &out, char *ws, bool validate,
                        bool reset_status, Profiler *prof, hipStream_t st) {
  hipError_t e = hipSuccess;
#define GT_CHK(x) do { e = (x); if (e != hipSuccess) return GT_ERR_HIP; } while (0)
#define GT_TIMED(name, x) do { if (prof) GT_CHK(prof->begin(name, st)); GT_CHK(x); if (prof) GT_CHK(prof->end(st)); } while (0)
  uint32_t *err = reinterpret_cast<uint32_t *>(ws);
  if (reset_status) GT_CHK(launch_fill(err, 1, 0u, st));
  if (p.n == 0 || p.m == 0) {
    // T = 0 everywhere
    GT_CHK(launch_fill(reinterpret_cast<uint32_t *>(out.offsets), 2 * (uint64_t)(p.n + 1), 0u, st));
    if (validate && p.n > 0) GT_CHK(launch_validate_offsets(g.offsets, p.n, p.m, err, st));
    return GT_OK;
  }
  if (validate) GT_CHK(launch_validate_offsets(g.offsets, p.n, p.m, err, st));
  if (p.strategy != GT_STRATEGY_STABLE) return enqueue_unordered(p, g, out, ws, prof, st);

  const StableLaunch L = stable_launch(p, g, out, ws, validate);
  // k_hist counts the first pass's digit only: every later pass counts its
  // own per tile (below), and its digit totals come from those counts
  HistArgs h0 = L.h;
  h0.passes = 1;
  GT_TIMED("k_hist", launch_hist(L.D, L.m, L.n, h0, L.tile, L.ntiles, L.hist_blocks, L.part, L.tcnt, L.err, st));
  GT_TIMED("k_tile_scan", launch_tile_scan(L.tcnt, L.ntiles, L.radix0, L.tbsum, L.dtot, L.toff, st));
  GT_TIMED("k_digit_scan", launch_digit_scan(L.part, L.hist_blocks, h0, L.dtot, L.digit, L.bins, L.nbins_total,
                                             L.m, L.err, st));
  GT_TIMED("k_tile_src", launch_tile_src(L.O, L.n, L.m, L.tile, L.ntiles, L.tsrc, st));
  for (int pass = 0; pass < L.passes; ++pass) {
    const bool first = pass == 0, last = pass == L.passes - 1;
    LsdArgs a = L.lsd[pass];
    if (!first) {
      // The first pass places its tiles with k_hist's tile counts.  A later
      // pass counts its digit per tile over its input (the previous pass's
      // keys) and places its tiles with their column prefix too, instead of
      // a look-back (the persistent kernel keeps the look-back).  The tile
      // buffers are the first pass's (a later digit is never wider).
      const int radix = 1 << p.bits[pass];
      const void *keys = L.pk[pass] ? static_cast<const void *>(a.in_key16) : static_cast<const void *>(a.in_key);
      GT_TIMED("k_tile_hist", launch_tile_hist(keys, L.pk[pass], L.m, a.shift, radix, L.tile, L.ntiles, L.tcnt, st));
      GT_TIMED("k_tile_scan", launch_tile_scan(L.tcnt, L.ntiles, radix, L.tbsum, L.dtot + pass * kMaxRadix, L.toff,
                                               st));
      GT_TIMED("k_digit_scan", launch_digit_scan_pass(L.dtot, L.h, pass, L.digit, L.bins, L.nbins_total, L.m, L.err,
                                                      st));
      a.tile_off = L.toff;
      a.placed = 1;
    }
    static const char *kLsdNames[kMaxPasses] = {"k_lsd_pass0", "k_lsd_pass1", "k_lsd_pass2"};
    GT_TIMED(kLsdNames[pass], launch_lsd(L.variant, p.bits[pass], a, first, L.pay, last, L.pk[pass], L.wide, st));
  }
  const FinalArgs &f = L.f;
  GT_TIMED("k_bin_items", launch_bin_items(f, st));
  GT_CHK(launch_fill(L.sstatus, (uint64_t)L.scan_tiles, 0u, st));
  GT_CHK(launch_fill(f.total_items + 1, 3, 0u, st));  // scan ticket, big- and huge-bin counts
  GT_TIMED("k_scan_u32", launch_scan_u32(f.nch, f.item_base, f.nbins, L.sstatus, f.total_items + 1, f.total_items,
                                         st));
  GT_TIMED("k_item_map", launch_item_map(f, st));
  GT_TIMED("k_big_count", launch_big_count(f, L.max_items, st));
  GT_TIMED("k_big_scan", launch_big_scan(f, L.max_big, L.max_huge, st));
  GT_TIMED("k_final", launch_final(f, L.max_items, L.pay, st));
#undef GT_TIMED
#undef GT_CHK
  return GT_OK;
}

// The unordered strategies (Atomic GT and HLH): count, aggregate, scatter.
static UnorderedArgs unordered_args(const GraphPlan &p, const gt_csr_t &g, const gt_csc_t *out, char *ws) {
  UnorderedArgs u{};
  u.O = g.offsets; u.D = g.indices; u.P = g.payload;
  u.n = p.n; u.m = p.m;
  u.chunk = p.chunk; u.nchunks = p.nchunks; u.span = p.chunk;
  u.nparts = p.nparts; u.head = p.head;
  u.steal_ticket = reinterpret_cast<uint32_t *>(ws + p.off_u_steal);
  u.times = p.step3_times ? reinterpret_cast<unsigned long long *>(ws + p.off_u_times) : nullptr;
  u.kmax = p.kmax;
  u.log2slots = kHlhLog2Slots;
  u.hdv = reinterpret_cast<const int32_t *>(ws + p.off_u_hdv);
  u.cnt = reinterpret_cast<uint32_t *>(ws + p.off_u_cnt);
  u.H = reinterpret_cast<uint32_t *>(ws + p.off_u_H);
  if (out) { u.T = out->offsets; u.S = out->indices; u.Q = out->payload; }
  u.cur = reinterpret_cast<unsigned long long *>(ws + p.off_u_cur);
  u.err = reinterpret_cast<uint32_t *>(ws);
  u.scan_status = reinterpret_cast<uint64_t *>(ws + p.off_u_sstatus);
  u.scan_ticket = reinterpret_cast<uint32_t *>(ws + p.off_u_ticket);
  return u;
}

// Step 0 of HLH: the degree sample and the HDV list (at most kmax vertices).
static hipError_t enqueue_hdv_list(const GraphPlan &p, const gt_csr_t &g, char *ws, Profiler *prof, hipStream_t st) {
  hipError_t e = hipSuccess;
  SampleArgs sa{};
  float *feat = nullptr;
  if (prof && (e = prof->begin("k_sample", st)) != hipSuccess) return e;
  if ((e = enqueue_sampling(g.offsets, g.indices, p.n, p.m, p.pay, p.seed, ws + p.off_u_samp, &feat, st, &sa)) !=
      hipSuccess)
    return e;
  if (prof && (e = prof->end(st)) != hipSuccess) return e;
  if (prof && (e = prof->begin("k_hdv_select", st)) != hipSuccess) return e;
  if ((e = launch_hdv_select(sa.keys, sa.counts, sa.mask, p.kmax, reinterpret_cast<uint32_t *>(ws + p.off_u_hist),
                             reinterpret_cast<uint32_t *>(ws + p.off_u_thr),
                             reinterpret_cast<int32_t *>(ws + p.off_u_hdv),
                             reinterpret_cast<uint32_t *>(ws + p.off_u_nhdv), st)) != hipSuccess)
    return e;
  if (prof && (e = prof->end(st)) != hipSuccess) return e;
  return hipSuccess;
}

// The probe of Section IV-C: Step 1 (the in-degree count) timed with the HDV
// table and without it (Atomic GT) on a sixteenth of the edges, the first
// sixteenth of every chunk, so that the sample spans the whole edge array and
// runs on the grid of a full launch; the plan keeps the faster.  Runs in `ws`
// (the layout of an HLH plan at offset kAlign) and synchronises `st`.
gt_status probe_strategy(GraphPlan &p, const gt_csr_t &g, char *ws, size_t ws_bytes, hipStream_t st) {
  if (p.n == 0 || p.m == 0) { p.strategy = GT_STRATEGY_ATOMIC; return GT_OK; }
  GraphPlan q = p;
  q.strategy = GT_STRATEGY_HLH;
  if (ws == nullptr || unordered_workspace_end(q, kAlign) > ws_bytes) return GT_ERR_WORKSPACE_TOO_SMALL;
  UnorderedArgs u = unordered_args(q, g, nullptr, ws);
  u.span = std::max<int64_t>(1, q.chunk / 16);
  u.nparts = 1;  // the first sixteenth of every chunk, one row per chunk
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  gt_status status = GT_OK;
  for (auto &x : ev)
    if (hipEventCreate(&x) != hipSuccess) status = GT_ERR_HIP;
  if (status == GT_OK && enqueue_hdv_list(q, g, ws, nullptr, st) != hipSuccess) status = GT_ERR_HIP;
  const uint32_t *nhdv = reinterpret_cast<const uint32_t *>(ws + q.off_u_nhdv);
  for (int rep = 0; rep < 2 && status == GT_OK; ++rep) {  // the second round is timed
    for (int way = 0; way < 2 && status == GT_OK; ++way) {
      u.nhdv = way == 0 ? nhdv : nullptr;
      if (launch_fill(u.cnt, (uint64_t)q.n, 0u, st) != hipSuccess || hipEventRecord(ev[2 * way], st) != hipSuccess ||
          launch_hlh_count(u, st) != hipSuccess || hipEventRecord(ev[2 * way + 1], st) != hipSuccess)
        status = GT_ERR_HIP;
    }
  }
  float t_hlh = 0.f, t_atomic = 0.f;
  if (status == GT_OK && (hipEventSynchronize(ev[3]) != hipSuccess || hipEventElapsedTime(&t_hlh, ev[0], ev[1]) !=
                          hipSuccess || hipEventElapsedTime(&t_atomic, ev[2], ev[3]) != hipSuccess))
    status = GT_ERR_HIP;
  for (auto &x : ev)
    if (x) (void)hipEventDestroy(x);
  if (status == GT_OK) p.strategy = t_hlh <= t_atomic ? GT_STRATEGY_HLH : GT_STRATEGY_ATOMIC;
  return status;
}

gt_status enqueue_unordered(const GraphPlan &p, const gt_csr_t &g, const gt_csc_t &out, char *ws, Profiler *prof,
                            hipStream_t st) {
  hipError_t e = hipSuccess;
#define GT_CHK(x) do { e = (x); if (e != hipSuccess) return GT_ERR_HIP; } while (0)
#define GT_TIMED(name, x) do { if (prof) GT_CHK(prof->begin(name, st)); GT_CHK(x); if (prof) GT_CHK(prof->end(st)); } while (0)
  UnorderedArgs u = unordered_args(p, g, &out, ws);
  GT_CHK(launch_fill(u.cnt, (uint64_t)p.n, 0u, st));
  if (p.strategy == GT_STRATEGY_HLH) {
    GT_CHK(enqueue_hdv_list(p, g, ws, prof, st));
    u.nhdv = reinterpret_cast<uint32_t *>(ws + p.off_u_nhdv);
  }
  GT_TIMED("k_hlh_count", launch_hlh_count(u, st));
  GT_TIMED("k_hdv_colscan", launch_hdv_colscan(u, st));
  const int64_t scan_tiles = (p.n + offsets_scan_tile() - 1) / offsets_scan_tile();
  GT_CHK(launch_fill(reinterpret_cast<uint32_t *>(u.scan_status), 2 * (uint64_t)scan_tiles, 0u, st));
  GT_CHK(launch_fill(u.scan_ticket, 1, 0u, st));
  GT_TIMED("k_scan_offsets", launch_scan_offsets(u, st));
  GT_CHK(launch_fill(u.steal_ticket, 1, 0u, st));
  GT_TIMED("k_hlh_scatter", launch_hlh_scatter(u, st));
#undef GT_TIMED
#undef GT_CHK
  return GT_OK;
}

}  // namespace gt

// Persistent plans: every graph must fit the persistent kernel's bodies;
// the pinned staging buffer, its event and the launch's grid.
gt_status gt::persist_staging(gt_plan_st *plan) {
  // host plans stage the tables; device plans the graphs' pointers and the
  // queue order (the planning kernel builds the tables)
  const size_t need = plan->device_plan ? plan->off_porder + sizeof(uint32_t) * (size_t)plan->count - plan->off_pgraph
                                        : persist_tables_bytes(plan->count, plan->ptab_entries);
  if (plan->pk_host != nullptr && plan->pk_bytes >= need) return GT_OK;
  if (plan->pk_host != nullptr) {
    if (plan->pk_event != nullptr && hipEventSynchronize(plan->pk_event) != hipSuccess) return GT_ERR_HIP;
    (void)hipHostFree(plan->pk_host);
    plan->pk_host = nullptr;
    plan->pk_bytes = 0;
    plan->pk_pending = false;
  }
  if (hipHostMalloc(&plan->pk_host, need, hipHostMallocDefault) != hipSuccess) {
    plan->pk_host = nullptr;
    return GT_ERR_HIP;
  }
  plan->pk_bytes = need;
  return GT_OK;
}

static gt_status persist_setup(gt_plan_st *plan) {
  for (const GraphPlan &p : plan->graphs)
    if (!persist_eligible(p)) return GT_ERR_UNSUPPORTED;
  const gt_status s = persist_staging(plan);
  if (s != GT_OK) return s;
  if (hipEventCreateWithFlags(&plan->pk_event, hipEventDisableTiming) != hipSuccess) {
    plan->pk_event = nullptr;
    return GT_ERR_HIP;
  }
  int dev = 0, cus = 0;
  const int per_cu = persistent_workgroups_per_cu();
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu <= 0 ||
      cus <= 0)
    return GT_ERR_HIP;
  plan->pk_grid = per_cu * cus;
  return GT_OK;
}

gt_plan_st::~gt_plan_st() {
  if (pk_event) (void)hipEventSynchronize(pk_event);  // no copy still reads the staging buffers
  if (dp_event) (void)hipEventSynchronize(dp_event);
  if (pk_event) (void)hipEventDestroy(pk_event);
  if (dp_event) (void)hipEventDestroy(dp_event);
  if (pk_host) (void)hipHostFree(pk_host);
  if (dp_host) (void)hipHostFree(dp_host);
  for (hipEvent_t e : prof.pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : lane_events) (void)hipEventDestroy(e);
  if (fork_event) (void)hipEventDestroy(fork_event);
  for (hipStream_t s : lanes) (void)hipStreamDestroy(s);
}

extern "C" {

const char *gt_status_string(gt_status s) {
  switch (s) {
    case GT_OK: return "ok";
    case GT_ERR_INVALID_ARGUMENT: return "invalid argument";
    case GT_ERR_INVALID_GRAPH: return "invalid graph";
    case GT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case GT_ERR_UNSUPPORTED: return "unsupported parameters";
    case GT_ERR_HIP: return "HIP runtime error";
    case GT_ERR_COUNTER_OVERFLOW: return "counter overflow";
    case GT_ERR_STALLED: return "persistent kernel stalled";
  }
  return "unknown status";
}

gt_status gt_workspace_size(const gt_csr_t *graphs, int32_t count, size_t *bytes_out) {
  if (graphs == nullptr || count <= 0 || bytes_out == nullptr) return GT_ERR_INVALID_ARGUMENT;
  const gt_status as = graphs_args_status(graphs, count);
  if (as != GT_OK) return as;
  size_t total = 0;
  for (int32_t i = 0; i < count; ++i)
    total += align_up(graph_workspace_bound(graphs[i].n, graphs[i].m, graphs[i].payload != nullptr));
  // status word, or a persistent plan's counters and tables
  uint64_t items = 0;
  for (int32_t i = 0; i < count; ++i) items += persist_item_bound(graphs[i].n, graphs[i].m);
  total += align_up(persist_counters_end(count)) + persist_tables_bytes(count, (items >> kPersistTabShift) + 2);
  total += device_plan_bytes(count);
  total += align_up(plan_scratch_bytes(graphs, count));
  *bytes_out = total;
  return GT_OK;
}

gt_status gt_plan_scratch_size(const gt_csr_t *graphs, int32_t count, size_t *bytes_out) {
  if (graphs == nullptr || count <= 0 || bytes_out == nullptr) return GT_ERR_INVALID_ARGUMENT;
  const gt_status as = graphs_args_status(graphs, count);
  if (as != GT_OK) return as;
  *bytes_out = align_up(plan_scratch_bytes(graphs, count)) + kAlign;
  return GT_OK;
}

gt_status gt_plan_workspace_size(gt_plan_t plan, size_t *bytes_out) {
  if (plan == nullptr || bytes_out == nullptr) return GT_ERR_INVALID_ARGUMENT;
  *bytes_out = plan->ws_bytes;
  return GT_OK;
}

gt_status gt_plan(const gt_csr_t *graphs, int32_t count, const gt_options_t *opt, void *workspace,
                  size_t workspace_bytes, void *stream, gt_plan_t *plan_out) {
  if (graphs == nullptr || count <= 0 || plan_out == nullptr) return GT_ERR_INVALID_ARGUMENT;
  const gt_status as = graphs_args_status(graphs, count);
  if (as != GT_OK) return as;
  gt_options_t o{};
  if (opt) o = *opt;
  if (o.policy < GT_POLICY_HEURISTIC || o.policy > GT_POLICY_MLP) return GT_ERR_INVALID_ARGUMENT;
  if (o.strategy < GT_STRATEGY_STABLE || o.strategy > GT_STRATEGY_PROBE || o.hdv_max < 0 || o.hdv_max > kHlhMaxHdv)
    return GT_ERR_UNSUPPORTED;
  if (o.policy == GT_POLICY_FIXED) {
    if ((o.fine_bits != 0 && (o.fine_bits < 1 || o.fine_bits > kMaxFineBits)) ||
        (o.digit_bits != 0 && (o.digit_bits < 4 || o.digit_bits > 10)) || o.variant < 0 || o.variant > 4)
      return GT_ERR_UNSUPPORTED;
  }
  const bool device_plan = (o.flags & GT_FLAG_DEVICE_PLAN) != 0;
  if (device_plan && (!(o.flags & GT_FLAG_PERSISTENT) || o.policy != GT_POLICY_MLP ||
                      o.strategy != GT_STRATEGY_STABLE || (o.flags & GT_FLAG_WIDE_STATUS) || count > kDevPlanMaxGraphs))
    return GT_ERR_UNSUPPORTED;
  gt_plan_st *plan = new (std::nothrow) gt_plan_st();
  if (!plan) return GT_ERR_INVALID_ARGUMENT;
  plan->count = count;
  plan->validate = o.validate != 0;
  plan->device_plan = device_plan;
  plan->graphs.resize(count);
  gt_status st = choose_params(plan, graphs, count, o, workspace, workspace_bytes, (hipStream_t)stream);
  if (st != GT_OK) { delete plan; return st; }
  for (int32_t i = 0; i < count && o.strategy == GT_STRATEGY_PROBE; ++i) {
    st = probe_strategy(plan->graphs[i], graphs[i], static_cast<char *>(workspace), workspace_bytes,
                        (hipStream_t)stream);
    if (st != GT_OK) { delete plan; return st; }
  }
  plan->persistent = (o.flags & GT_FLAG_PERSISTENT) != 0;
  if (plan->persistent)
    for (GraphPlan &p : plan->graphs) persist_coerce(p);
  layout_plan(plan);
  if (plan->persistent) {
    st = persist_setup(plan);
    if (st != GT_OK) { delete plan; return st; }
  }
  if (device_plan) {
    for (const GraphPlan &p : plan->graphs) {
      size_t most = 0;
      if (!device_region(p, &most)) { delete plan; return GT_ERR_UNSUPPORTED; }
    }
    if (workspace == nullptr || workspace_bytes < plan->ws_bytes) { delete plan; return GT_ERR_WORKSPACE_TOO_SMALL; }
    st = device_plan_setup(plan, graphs, o, static_cast<char *>(workspace), (hipStream_t)stream);
    if (st != GT_OK) { delete plan; return st; }
  }
  *plan_out = plan;
  return GT_OK;
}

static gt_status check_io(const GraphPlan &p, const gt_csr_t *g, const gt_csc_t *out) {
  if (g == nullptr || out == nullptr) return GT_ERR_INVALID_ARGUMENT;
  const gt_status as = csr_args_status(*g);
  if (as != GT_OK) return as;
  if (g->n != p.n || g->m != p.m || (g->payload != nullptr) != p.pay) return GT_ERR_INVALID_ARGUMENT;
  if (out->offsets == nullptr || (p.m > 0 && out->indices == nullptr)) return GT_ERR_INVALID_ARGUMENT;
  if ((out->payload != nullptr) != p.pay) return GT_ERR_INVALID_ARGUMENT;
  return GT_OK;
}

gt_status gt_transpose(gt_plan_t plan, const gt_csr_t *g, gt_csc_t *out, void *workspace, size_t workspace_bytes,
                       void *stream) {
  if (plan == nullptr || plan->count != 1 || workspace == nullptr) return GT_ERR_INVALID_ARGUMENT;
  if (plan->device_plan) return GT_ERR_UNSUPPORTED;  // its choice is on the device: gt_transpose_batched
  const GraphPlan &p = plan->graphs[0];
  gt_status s = check_io(p, g, out);
  if (s != GT_OK) return s;
  if (workspace_bytes < plan->ws_bytes) return GT_ERR_WORKSPACE_TOO_SMALL;
  return enqueue_graph(p, *g, *out, static_cast<char *>(workspace), plan->validate, true, &plan->prof,
                       (hipStream_t)stream);
}

gt_status gt_transpose_noalloc(gt_plan_t plan, const gt_csr_t *g, gt_csc_t *out, uint32_t *status_out,
                               void *stream) {
  if (plan == nullptr || plan->count != 1) return GT_ERR_INVALID_ARGUMENT;
  if (plan->device_plan) return GT_ERR_UNSUPPORTED;
  const GraphPlan &p = plan->graphs[0];
  gt_status s = check_io(p, g, out);
  if (s != GT_OK) return s;
  if (plan->ws_bytes > (size_t)GT_NOALLOC_SCRATCH_BYTES) return GT_ERR_WORKSPACE_TOO_SMALL;
  int cur = -1, sdev = -1;
  if (hipGetDevice(&cur) != hipSuccess || hipStreamGetDevice((hipStream_t)stream, &sdev) != hipSuccess)
    return GT_ERR_HIP;
  if (cur != sdev) return GT_ERR_INVALID_ARGUMENT;
  void *ws = nullptr;
  s = current_scratch(&ws);
  if (s != GT_OK) return s;
  // no profiler: recording its events could create some
  s = enqueue_graph(p, *g, *out, static_cast<char *>(ws), plan->validate, true, nullptr, (hipStream_t)stream);
  if (s != GT_OK) return s;
  if (status_out != nullptr &&
      launch_copy_u32(status_out, static_cast<const uint32_t *>(ws), 1, (hipStream_t)stream) != hipSuccess)
    return GT_ERR_HIP;
  return GT_OK;
}

gt_status gt_transpose_batched(gt_plan_t plan, int32_t count, const gt_csr_t *graphs, gt_csc_t *outs,
                               void *workspace, size_t workspace_bytes, void *stream) {
  if (plan == nullptr || graphs == nullptr || outs == nullptr || workspace == nullptr || count != plan->count)
    return GT_ERR_INVALID_ARGUMENT;
  for (int32_t i = 0; i < count; ++i) {
    gt_status s = check_io(plan->graphs[i], &graphs[i], &outs[i]);
    if (s != GT_OK) return s;
  }
  if (workspace_bytes < plan->ws_bytes) return GT_ERR_WORKSPACE_TOO_SMALL;
  return enqueue_batched(plan, graphs, outs, static_cast<char *>(workspace), (hipStream_t)stream);
}

gt_status gt_device_status(const void *workspace) {
  if (workspace == nullptr) return GT_ERR_INVALID_ARGUMENT;
  uint32_t err = 0;
  if (hipMemcpy(&err, workspace, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) return GT_ERR_HIP;
  if (err & (kErrBadIndex | kErrBadOffsets)) return GT_ERR_INVALID_GRAPH;
  if (err & kErrOverflow) return GT_ERR_COUNTER_OVERFLOW;
  if (err & kErrStall) return GT_ERR_STALLED;
  return GT_OK;
}

gt_status gt_plan_device_choice(gt_plan_t plan, const void *workspace, int32_t i, int32_t *fine_bits,
                                int32_t *digit_bits, int32_t *variant, int32_t *config) {
  if (plan == nullptr || workspace == nullptr || i < 0 || i >= plan->count) return GT_ERR_INVALID_ARGUMENT;
  if (!plan->device_plan) return GT_ERR_UNSUPPORTED;
  DevChoice c{};
  const char *src = static_cast<const char *>(workspace) + plan->off_pchoice + sizeof(DevChoice) * (size_t)i;
  if (hipMemcpy(&c, src, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return GT_ERR_HIP;
  if (fine_bits) *fine_bits = c.fine_bits;
  if (digit_bits) *digit_bits = c.digit_bits;
  if (variant) *variant = c.variant;
  if (config) *config = c.config;
  return GT_OK;
}

gt_status gt_plan_device_status(gt_plan_t plan, const void *workspace) {
  if (plan == nullptr) return GT_ERR_INVALID_ARGUMENT;
  return gt_device_status(workspace);
}

gt_status gt_plan_params(gt_plan_t plan, int32_t i, int32_t *fine_bits, int32_t *digit_bits, int32_t *passes,
                         int32_t *variant) {
  if (plan == nullptr || i < 0 || i >= plan->count) return GT_ERR_INVALID_ARGUMENT;
  const GraphPlan &p = plan->graphs[i];
  if (fine_bits) *fine_bits = p.fine_bits;
  if (digit_bits) *digit_bits = p.max_bits;
  if (passes) *passes = p.passes;
  if (variant) *variant = p.variant;
  return GT_OK;
}

gt_status gt_plan_packed(gt_plan_t plan, int32_t i, int32_t *packed) {
  if (plan == nullptr || i < 0 || i >= plan->count || packed == nullptr) return GT_ERR_INVALID_ARGUMENT;
  *packed = plan->graphs[i].packed ? 1 : 0;
  return GT_OK;
}

gt_status gt_plan_strategy(gt_plan_t plan, int32_t i, int32_t *strategy) {
  if (plan == nullptr || i < 0 || i >= plan->count || strategy == nullptr) return GT_ERR_INVALID_ARGUMENT;
  *strategy = plan->graphs[i].strategy;
  return GT_OK;
}

gt_status gt_plan_step3_times(gt_plan_t plan, int32_t i, const void *workspace, uint64_t *out,
                              int32_t max_chunks, int32_t *nchunks_out, double *clock_hz) {
  if (plan == nullptr || i < 0 || i >= plan->count || workspace == nullptr || nchunks_out == nullptr ||
      clock_hz == nullptr || (max_chunks > 0 && out == nullptr))
    return GT_ERR_INVALID_ARGUMENT;
  const GraphPlan &p = plan->graphs[i];
  if (p.strategy == GT_STRATEGY_STABLE || !p.step3_times) return GT_ERR_INVALID_ARGUMENT;
  *nchunks_out = (int32_t)p.nchunks;
  *clock_hz = hlh_clock_hz();
  const int64_t rows = std::min<int64_t>(p.nchunks, std::max(max_chunks, 0));
  if (rows > 0 && hipMemcpy(out, static_cast<const char *>(workspace) + p.off_u_times, 24 * (size_t)rows,
                            hipMemcpyDeviceToHost) != hipSuccess)
    return GT_ERR_HIP;
  return GT_OK;
}

gt_status gt_plan_destroy(gt_plan_t plan) {
  delete plan;
  return GT_OK;
}

gt_status gt_profile(gt_plan_t plan, int32_t enable) {
  if (plan == nullptr) return GT_ERR_INVALID_ARGUMENT;
  plan->prof.on = enable != 0;
  plan->prof.recs.clear();
  plan->prof.used = 0;
  return GT_OK;
}

gt_status gt_profile_read(gt_plan_t plan, int32_t max_kernels, char (*names)[32], double *total_ms,
                          int32_t *launches, int32_t *count_out) {
  if (plan == nullptr || count_out == nullptr || (max_kernels > 0 && (!names || !total_ms || !launches)))
    return GT_ERR_INVALID_ARGUMENT;
  int32_t count = 0;
  for (const ProfRec &r : plan->prof.recs) {
    if (hipEventSynchronize(r.stop) != hipSuccess) return GT_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) return GT_ERR_HIP;
    int32_t k = 0;
    while (k < count && strncmp(names[k], r.name, 31) != 0) ++k;
    if (k == count) {
      if (count >= max_kernels) continue;
      strncpy(names[k], r.name, 31);
      names[k][31] = 0;
      total_ms[k] = 0.0;
      launches[k] = 0;
      ++count;
    }
    total_ms[k] += ms;
    launches[k] += 1;
  }
  plan->prof.recs.clear();
  plan->prof.used = 0;
  *count_out = count;
  return GT_OK;
}

}  // extern "C"
