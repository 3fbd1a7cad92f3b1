// Parameter policies of a plan.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "gt_internal.h"
#include "gt_plan.h"

namespace gt {

size_t plan_scratch_bytes(const gt_csr_t *graphs, int32_t count) {
  (void)graphs; (void)count;
  return 0;
}

// Size-only heuristic: a k_final bin should hold about one 8K-edge tile, so
// fine_bits ~ log2(4096 / average in-degree); digits of up to 10 bits.
static void heuristic(GraphPlan &p) {
  const double avg = p.n > 0 ? (double)p.m / (double)p.n : 1.0;
  int fb = (int)lround(log2(4096.0 / std::max(avg, 1.0)));
  p.fine_bits = std::min(std::max(fb, 4), kMaxFineBits);
  p.digit_bits = 10;
  p.variant = 1;
}

gt_status choose_params(gt_plan_st *plan, const gt_csr_t *graphs, int32_t count, const gt_options_t &opt,
                        void *workspace, size_t workspace_bytes, hipStream_t st) {
  (void)workspace; (void)workspace_bytes; (void)st;
  for (int32_t i = 0; i < count; ++i) {
    GraphPlan &p = plan->graphs[i];
    p = GraphPlan{};
    p.n = graphs[i].n;
    p.m = graphs[i].m;
    p.pay = graphs[i].payload != nullptr;
    heuristic(p);
    p.force_wide = (opt.flags & GT_FLAG_WIDE_STATUS) != 0;
    if (opt.policy == GT_POLICY_FIXED) {
      if (opt.fine_bits) p.fine_bits = opt.fine_bits;
      if (opt.digit_bits) p.digit_bits = opt.digit_bits;
      if (opt.variant) p.variant = opt.variant;
    }
  }
  return GT_OK;
}

gt_status enqueue_batched(gt_plan_st *plan, const gt_csr_t *graphs, const gt_csc_t *outs, char *ws,
                          hipStream_t st) {
  for (int32_t i = 0; i < plan->count; ++i) {
    gt_status s = enqueue_graph(plan->graphs[i], graphs[i], outs[i], ws, plan->validate, i == 0, &plan->prof, st);
    if (s != GT_OK) return s;
  }
  return GT_OK;
}

}  // namespace gt
