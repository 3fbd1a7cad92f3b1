// Plan structures shared by the C ABI, the parameter policies and the
// batched launcher.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/gt.h"
#include "gt_internal.h"

namespace gt {

struct GraphPlan {
  int64_t n, m;
  bool pay;
  // chosen parameters
  int fine_bits;   // log2 of the destination range of one k_final workgroup
  int digit_bits;  // maximum digit width per partition pass
  int variant;     // tile variant of k_lsd
  // derived
  int passes, bits[3], shift[3], max_bits, total_bits;
  int64_t nbins_total, nbins, tile, ntiles;
  bool wide_status;  // 64-bit look-back words (m >= 2^31)
  // two-pass plans whose key and source bits fit 48: the intermediate
  // between the passes is packed into 6 bytes per edge (16-bit key + source
  // word carrying the high fine bits); id_bits = bits of a vertex ID
  bool packed = false;
  int id_bits = 0;
  bool force_wide;
  // workspace byte offsets (relative to the workspace start)
  size_t off_err, off_ticket, off_part, off_digit, off_dtot, off_bin, off_status, off_tsrc;
  size_t off_tcnt, off_tbsum, off_toff;  // first pass: per-tile digit counts, block sums, tile offsets
  size_t off_a_src, off_a_key, off_a_pay, off_a2_src, off_a2_key, off_a2_pay;
  size_t off_b_src, off_b_key, off_b_pay;
  size_t off_nch, off_ibase, off_ibin, off_itotal, off_sstatus, off_cntab, off_big, off_huge;
  int64_t max_big, max_huge;
  int64_t max_items;
  // unordered strategies (GT_STRATEGY_HLH / GT_STRATEGY_ATOMIC)
  int strategy;
  int32_t hdv_max, kmax;
  uint64_t seed;
  int64_t nchunks, chunk;
  // Step 3 of the unordered strategies: 0 = one chunk per workgroup, up to
  // 2048 chunks (the dispatcher balances them); 1 = static, as many chunks
  // as resident workgroups; 2 = the two-phase scheme of Section V-F (static
  // heads, tail parts claimed atomically); times: record per-chunk stamps
  int step3 = 0;
  bool step3_times = false;
  int nparts = 1;
  int64_t head = 0;
  size_t off_u_steal = 0, off_u_times = 0;
  size_t off_u_samp, off_u_hist, off_u_thr, off_u_hdv, off_u_nhdv, off_u_cnt, off_u_cur, off_u_H, off_u_sstatus,
      off_u_ticket;
  size_t ws_end;
  // sampled features (when the policy sampled the graph)
  float features[32];
  int nfeatures;
  bool learned;  // parameters chosen by the MLP
  int config;    // configuration index when chosen from the grid, else -1
};

}  // namespace gt

namespace gt {
// Per-launch HIP events recorded on the launch stream while profiling is on.
struct ProfRec {
  const char *name;
  hipEvent_t start, stop;
};
struct Profiler {
  bool on = false;
  std::vector<ProfRec> recs;   // recorded since the last read
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get();
  hipError_t begin(const char *name, hipStream_t st);
  hipError_t end(hipStream_t st);
};
}  // namespace gt

struct gt_plan_st {
  int32_t count;
  bool validate;
  std::vector<gt::GraphPlan> graphs;
  size_t ws_bytes;
  gt::Profiler prof;
  // batched launches: graphs spread over internal streams (default
  // priority), forked from and joined back into the caller's stream
  std::vector<hipStream_t> lanes;
  std::vector<hipEvent_t> lane_events;
  hipEvent_t fork_event = nullptr;
  std::vector<int> lane_of;  // graph -> lane
  // GT_FLAG_PERSISTENT: gt_transpose_batched drains one device work queue
  // with the persistent kernel.  Workspace: byte 0 the status word, bytes
  // 8..15 the queue's ticket, then one done counter per phase; after the
  // graphs' regions, the graph descriptors and the phase table (copied from
  // the pinned host staging buffer by every call).
  bool persistent = false;
  size_t off_pdesc = 0, off_pphase = 0, off_ptab = 0;
  uint64_t ptab_entries = 0;  // capacity of the ticket -> phase table
  void *pk_host = nullptr;  // hipHostMalloc'd: descriptors, then phases
  size_t pk_bytes = 0;
  hipEvent_t pk_event = nullptr;  // the last copy out of pk_host
  bool pk_pending = false;
  int pk_grid = 0;  // workgroups of the persistent launch
  size_t off_pmeta = 0;  // the queue's size: tickets, phases
  // GT_FLAG_DEVICE_PLAN: the learned choice is made on the device and kept
  // in the workspace (off_pchoice); every graph owns a region sized for any
  // choice (graph_base); each batched call lays the graphs out and builds
  // the tables on the device from the graphs' pointers (off_pgraph) and the
  // queue order (off_porder).  dp_host stages the network and the heuristic
  // choices for the planning kernels (copied once, by gt_plan).
  bool device_plan = false;
  std::vector<uint64_t> graph_base;
  std::vector<uint32_t> order;
  size_t off_ptmp = 0, off_pchoice = 0, off_pgraph = 0, off_porder = 0, off_pdp = 0, off_psamp = 0;
  void *dp_host = nullptr;
  size_t dp_bytes = 0;
  hipEvent_t dp_event = nullptr;
  ~gt_plan_st();
};

namespace gt {

void finalize_params(GraphPlan &p, size_t base);
size_t graph_workspace_bound(int64_t n, int64_t m, bool pay);
size_t plan_scratch_bytes(const gt_csr_t *graphs, int32_t count);
gt_status choose_params(gt_plan_st *plan, const gt_csr_t *graphs, int32_t count, const gt_options_t &opt,
                        void *workspace, size_t workspace_bytes, hipStream_t st);
gt_status enqueue_graph(const GraphPlan &p, const gt_csr_t &g, const gt_csc_t &out, char *ws, bool validate,
                        bool reset_status, Profiler *prof, hipStream_t st);
size_t unordered_workspace_end(GraphPlan &p, size_t base);
gt_status enqueue_unordered(const GraphPlan &p, const gt_csr_t &g, const gt_csc_t &out, char *ws, Profiler *prof,
                            hipStream_t st);
gt_status enqueue_batched(gt_plan_st *plan, const gt_csr_t *graphs, const gt_csc_t *outs, char *ws,
                          hipStream_t st);
// Persistent plans: the done counters start at this workspace byte; the
// graph regions after the counters of kPersistMaxPhases phases per graph.
constexpr size_t kPersistDoneOff = 16;
size_t persist_counters_end(int32_t count);
size_t persist_tables_bytes(int32_t count, uint64_t tab_entries);
// Device plans: the regions beyond the persistent tables (every graph's
// phases, choices, pointers, queue order, the network's staging and its
// inputs and outputs).
size_t device_plan_bytes(int32_t count);
// Device-plan staging region: network parameters, input ranges, heuristic
// choices, feature pointers, network inputs and outputs (byte offsets).
struct DevPlanStage {
  size_t params, fmin, fmax, heur, fdev, x, y, staged, total;
};
DevPlanStage dev_plan_stage(int32_t count);
// Items of all phases of a graph of n vertices and m edges, at most, for any
// parameters (sizes the ticket -> phase table before a plan exists).
uint64_t persist_item_bound(int64_t n, int64_t m);
// Device plans: stage the network and the heuristic choices, enqueue the
// sampling, the network and the choice (no host synchronisation).
gt_status device_plan_setup(gt_plan_st *plan, const gt_csr_t *graphs, const gt_options_t &opt, char *ws,
                            hipStream_t st);
// (Re)allocate a persistent plan's pinned staging buffer for its tables.
gt_status persist_staging(gt_plan_st *plan);
// Offsets of every graph's region (and of a persistent plan's tables); sets
// plan->ws_bytes.  (The per-graph layout itself: gt_layout.hpp.)
void layout_plan(gt_plan_st *plan);

}  // namespace gt
