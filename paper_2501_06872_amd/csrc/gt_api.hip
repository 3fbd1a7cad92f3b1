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
  const int L = std::max(1, ceil_log2(std::max<int64_t>(p.n, 2)));
  int fb = std::min(p.fine_bits, kMaxFineBits);
  fb = std::min(fb, L - 1);
  fb = std::max(fb, 0);
  p.fine_bits = fb;
  if (L - fb > kMaxPasses * 10) fb = L - kMaxPasses * 10;  // at most 3 digits of <= 10 bits
  p.fine_bits = fb;
  const int dbits = L - fb;  // >= 1
  int maxb = std::max(1, std::min(p.digit_bits, 10));
  maxb = std::max(maxb, (dbits + kMaxPasses - 1) / kMaxPasses);  // widen digits rather than add passes
  p.passes = (dbits + maxb - 1) / maxb;
  int rem = dbits, shift = fb, maxbits = 0;
  // digits as even as possible, the wider ones first (measured: on 2^26-
  // vertex graphs 9 + 8 bits beat 8 + 9 by 1 % on natural-order R-MAT and
  // lose 0.3-0.5 % on uniform and permuted graphs)
  for (int i = 0; i < p.passes; ++i) {
    const int b = (rem + (p.passes - i) - 1) / (p.passes - i);
    p.bits[i] = b;
    p.shift[i] = shift;
    shift += b;
    rem -= b;
    maxbits = std::max(maxbits, b);
  }
  p.max_bits = maxbits;
  p.total_bits = dbits;
  // fine bits + last digit + source bits <= 48 leaves room for the fine bits
  // above the 16-bit key in the top of the 32-bit source word
  p.id_bits = L;
  p.packed = p.passes == 2 && fb + p.bits[1] + L <= 48 && p.bits[1] <= 10;
  // The 16-wave tiles have no 10-bit instance (their lane-mask tables would
  // not fit LDS): such plans use the 8-wave x 16-edge tile for every pass, so
  // that one tile size holds for the tile sources, the look-back status
  // words and every pass's grid.
  p.variant = lsd_variant_for(p.variant, maxbits);
  p.nbins_total = int64_t(1) << dbits;
  p.nbins = (p.n + (int64_t(1) << fb) - 1) >> fb;
  if (p.n == 0) p.nbins = 0;
  p.tile = lsd_tile_size(p.variant);
  p.ntiles = (p.m + p.tile - 1) / p.tile;

  size_t off = base;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  p.off_err = 0;  // one status word for the whole workspace (byte 0)
  p.off_ticket = take(sizeof(uint32_t) * kMaxPasses);
  p.off_part = take(sizeof(uint32_t) * (size_t)kHistBlocks * kMaxPasses * kMaxRadix);
  p.off_digit = take(sizeof(uint64_t) * kMaxPasses * (kMaxRadix + 1));
  p.off_dtot = take(sizeof(uint64_t) * kMaxPasses * kMaxRadix);
  p.off_bin = take(sizeof(uint64_t) * (size_t)(p.nbins_total + 1));
  p.wide_status = p.force_wide || p.m >= (int64_t(1) << 31);
  // look-back status words of the passes after the first (which places its
  // tiles with k_hist's per-tile counts)
  p.off_status = take(p.passes > 1 ? (p.wide_status ? 8 : 4) * (size_t)p.ntiles * ((size_t)1 << p.max_bits) : 0);
  p.off_tsrc = take(sizeof(int32_t) * (size_t)std::max<int64_t>(p.ntiles, 1));
  {
    const size_t r0 = (size_t)1 << p.bits[0];
    const size_t nt = (size_t)std::max<int64_t>(p.ntiles, 1);
    p.off_tcnt = take(sizeof(uint16_t) * nt * r0);
    p.off_tbsum = take(sizeof(uint32_t) * (size_t)std::max<int64_t>(tile_scan_blocks(p.ntiles), 1) * r0);
    p.off_toff = take(sizeof(uint32_t) * nt * r0);
  }
  const size_t m = (size_t)p.m;
  p.off_a_src = p.off_a_key = p.off_a_pay = 0;
  p.off_a2_src = p.off_a2_key = p.off_a2_pay = 0;
  if (p.passes >= 2) {
    p.off_a_src = take(4 * m);
    p.off_a_key = take(4 * m);
    if (p.pay) p.off_a_pay = take(4 * m);
  }
  if (p.passes >= 3) {
    p.off_a2_src = take(4 * m);
    p.off_a2_key = take(4 * m);
    if (p.pay) p.off_a2_pay = take(4 * m);
  }
  p.off_b_src = take(4 * m);
  p.off_b_key = take(2 * m);
  p.off_b_pay = p.pay ? take(4 * m) : 0;
  const size_t nb = (size_t)std::max<int64_t>(p.nbins, 1);
  p.max_items = p.nbins + (p.m + final_tile_size() - 1) / final_tile_size();
  p.off_nch = take(4 * nb);
  p.off_ibase = take(4 * nb);
  p.off_ibin = take(16 * (size_t)std::max<int64_t>(p.max_items, 1));  // item descriptors
  p.off_itotal = take(4 * 4);
  p.off_sstatus = take(8 * (size_t)((p.nbins + scan_tile_size() - 1) / scan_tile_size() + 1));
  p.off_cntab = take(4 * (size_t)std::max<int64_t>(p.max_items, 1) * ((size_t)1 << p.fine_bits));
  p.max_big = std::min<int64_t>(p.nbins, p.m / final_tile_size() + 1);
  p.off_big = take(4 * (size_t)std::max<int64_t>(p.max_big, 1));
  p.max_huge = std::min<int64_t>(p.nbins, p.m / (final_tile_size() * kHugeChunks) + 1);
  p.off_huge = take(4 * (size_t)std::max<int64_t>(p.max_huge, 1));
  p.ws_end = off;
}

size_t persist_counters_end(int32_t count) {
  return kPersistDoneOff + 4 * (size_t)count * kPersistMaxPhases;
}

size_t persist_tables_bytes(int32_t count, uint64_t tab_entries) {
  return align_up(sizeof(StableLaunch) * (size_t)count) +
         align_up(sizeof(PersistPhase) * (size_t)count * kPersistMaxPhases) + align_up(4 * (size_t)tab_entries);
}

uint64_t persist_item_bound(int64_t n, int64_t m) {
  // fixed-size phases, tiles of the passes and their scans, bins, work items
  return 8192 + 8 * ((uint64_t)m / 4096 + 1) + 4 * ((uint64_t)n + 1);
}

void persist_coerce(GraphPlan &p) {
  p.variant = 1;
  p.digit_bits = std::min(p.digit_bits, 9);
}

bool persist_eligible(const GraphPlan &p) {
  if (p.strategy != GT_STRATEGY_STABLE) return false;
  if (p.n == 0 || p.m == 0) return true;
  return p.variant == 1 && p.tile == lsd_tile_size(1) && p.max_bits <= 9 && p.passes <= 2 && !p.wide_status;
}

void layout_plan(gt_plan_st *plan) {
  size_t base = plan->persistent ? align_up(persist_counters_end(plan->count)) : kAlign;  // byte 0: status word
  for (GraphPlan &p : plan->graphs) {
    finalize_params(p, base);
    base = align_up(p.ws_end);
  }
  if (plan->persistent) {
    uint64_t items = 0;
    PersistPhase buf[kPersistMaxPhases];
    for (const GraphPlan &p : plan->graphs) {
      const int k = persist_phases(p, nullptr, nullptr, 0, plan->validate, buf);
      for (int j = 0; j < k; ++j) items += buf[j].nitems;
    }
    plan->ptab_entries = (items >> kPersistTabShift) + 2;  // tickets <= items
    plan->off_pdesc = base;
    plan->off_pphase = base + align_up(sizeof(StableLaunch) * (size_t)plan->count);
    plan->off_ptab = plan->off_pphase + align_up(sizeof(PersistPhase) * (size_t)plan->count * kPersistMaxPhases);
    base += persist_tables_bytes(plan->count, plan->ptab_entries);
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

// The arguments of every kernel of a stable transposition.
StableLaunch stable_launch(const GraphPlan &p, const gt_csr_t &g, const gt_csc_t &out, char *ws, bool validate) {
  StableLaunch L{};
  L.O = g.offsets; L.D = g.indices; L.n = p.n; L.m = p.m;
  L.ntiles = p.ntiles; L.tile = p.tile; L.nbins_total = p.nbins_total;
  L.passes = p.passes; L.radix0 = 1 << p.bits[0]; L.variant = p.variant;
  L.pay = p.pay; L.wide = p.wide_status; L.validate = validate;
  L.err = reinterpret_cast<uint32_t *>(ws);
  L.ticket = reinterpret_cast<uint32_t *>(ws + p.off_ticket);
  L.part = reinterpret_cast<uint32_t *>(ws + p.off_part);
  L.digit = reinterpret_cast<uint64_t *>(ws + p.off_digit);
  L.bins = reinterpret_cast<uint64_t *>(ws + p.off_bin);
  L.status = reinterpret_cast<uint32_t *>(ws + p.off_status);
  L.status_words = (uint64_t)p.ntiles * ((uint64_t)1 << p.max_bits) * (p.wide_status ? 2 : 1);
  L.tsrc = reinterpret_cast<int32_t *>(ws + p.off_tsrc);
  L.tcnt = reinterpret_cast<uint16_t *>(ws + p.off_tcnt);
  L.tbsum = reinterpret_cast<uint32_t *>(ws + p.off_tbsum);
  L.toff = reinterpret_cast<uint32_t *>(ws + p.off_toff);
  L.dtot = reinterpret_cast<uint64_t *>(ws + p.off_dtot);
  L.h.passes = p.passes;
  for (int i = 0; i < p.passes; ++i) { L.h.shift[i] = p.shift[i]; L.h.bits[i] = p.bits[i]; }
  // histogram workgroups take contiguous ranges of the first pass's tiles,
  // at most kHistBlocks of them: a small graph neither launches nor sums
  // partial histograms it has no edges for
  L.hist_blocks = (int)std::min<int64_t>(kHistBlocks, std::max<int64_t>(1, p.ntiles));
  const int32_t *cur_src = nullptr;
  const uint32_t *cur_key = nullptr, *cur_pay = nullptr;
  for (int pass = 0; pass < p.passes; ++pass) {
    const bool first = pass == 0, last = pass == p.passes - 1;
    LsdArgs &a = L.lsd[pass];
    a.O = g.offsets; a.D = g.indices; a.P = g.payload; a.tile_src0 = L.tsrc; a.tile_off = L.toff;
    a.in_src = cur_src; a.in_key = cur_key; a.in_pay = cur_pay;
    const bool pk = p.packed && (first != last);
    L.pk[pass] = pk;
    if (pk && last) a.in_key16 = reinterpret_cast<const uint16_t *>(cur_key);
    if (last) {
      a.out_src = reinterpret_cast<int32_t *>(ws + p.off_b_src);
      a.out_key16 = reinterpret_cast<uint16_t *>(ws + p.off_b_key);
      a.out_pay = p.pay ? reinterpret_cast<uint32_t *>(ws + p.off_b_pay) : nullptr;
    } else {
      const bool use_a2 = (pass == 1);
      a.out_src = reinterpret_cast<int32_t *>(ws + (use_a2 ? p.off_a2_src : p.off_a_src));
      a.out_key32 = reinterpret_cast<uint32_t *>(ws + (use_a2 ? p.off_a2_key : p.off_a_key));
      if (pk) a.out_key16 = reinterpret_cast<uint16_t *>(ws + p.off_a_key);
      a.out_pay = p.pay ? reinterpret_cast<uint32_t *>(ws + (use_a2 ? p.off_a2_pay : p.off_a_pay)) : nullptr;
    }
    a.shift = p.shift[pass];
    a.bits = p.bits[pass];
    a.digit_start = L.digit + pass * (kMaxRadix + 1);
    a.status = L.status;
    a.ticket = L.ticket + pass;
    a.m = p.m; a.n = p.n;
    a.fine_shift = p.fine_bits;
    a.lower_bits = p.total_bits - p.bits[p.passes - 1];
    a.fine_mask = (1u << p.fine_bits) - 1u;
    a.bin_start = L.bins;
    if (pk) {
      a.pk_lo = 16 - p.bits[1];
      a.pk_src_bits = p.id_bits;
      a.pk_dshift = p.shift[1];
      a.pk_dbits = p.bits[1];
      if (last) {  // the packed key holds the digit at bit pk_lo
        a.shift = a.pk_lo;
        a.prev_digit_start = L.digit;
        a.prev_bits = p.bits[0];
      }
    }
    cur_src = a.out_src;
    cur_key = a.out_key32;
    cur_pay = a.out_pay;
  }
  FinalArgs &f = L.f;
  f.in_src = reinterpret_cast<const int32_t *>(ws + p.off_b_src);
  f.in_key = reinterpret_cast<const uint16_t *>(ws + p.off_b_key);
  f.in_pay = p.pay ? reinterpret_cast<const uint32_t *>(ws + p.off_b_pay) : nullptr;
  f.bin_start = L.bins;
  f.T = out.offsets; f.S = out.indices; f.Q = out.payload;
  f.n = p.n; f.m = p.m; f.nbins = p.nbins; f.fine_bits = p.fine_bits;
  f.nch = reinterpret_cast<uint32_t *>(ws + p.off_nch);
  f.item_base = reinterpret_cast<uint32_t *>(ws + p.off_ibase);
  f.item_desc = reinterpret_cast<uint4 *>(ws + p.off_ibin);
  f.total_items = reinterpret_cast<uint32_t *>(ws + p.off_itotal);
  f.cntab = reinterpret_cast<uint32_t *>(ws + p.off_cntab);
  f.bigbins = reinterpret_cast<uint32_t *>(ws + p.off_big);
  f.nbig = f.total_items + 2;
  f.hugebins = reinterpret_cast<uint32_t *>(ws + p.off_huge);
  f.nhuge = f.total_items + 3;
  f.err = L.err;
  L.sstatus = reinterpret_cast<uint32_t *>(ws + p.off_sstatus);
  L.scan_tiles = (p.nbins + scan_tile_size() - 1) / scan_tile_size();
  L.max_items = p.max_items;
  L.max_big = p.max_big;
  L.max_huge = p.max_huge;
  return L;
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
  GT_TIMED("k_hist", launch_hist(L.D, L.m, L.n, L.h, L.tile, L.ntiles, L.hist_blocks, L.part, L.tcnt, L.err, st));
  GT_TIMED("k_tile_scan", launch_tile_scan(L.tcnt, L.ntiles, L.radix0, L.tbsum, L.dtot, L.toff, st));
  GT_TIMED("k_digit_scan", launch_digit_scan(L.part, L.hist_blocks, L.h, L.dtot, L.digit, L.bins, L.nbins_total,
                                             L.m, L.err, st));
  GT_TIMED("k_tile_src", launch_tile_src(L.O, L.n, L.m, L.tile, L.ntiles, L.tsrc, st));
  for (int pass = 0; pass < L.passes; ++pass) {
    const bool first = pass == 0, last = pass == L.passes - 1;
    if (!first) {  // the first pass places its tiles with k_hist's tile offsets
      GT_TIMED("k_fill_status", launch_fill(L.status, L.status_words, 0u, st));
      GT_CHK(launch_fill(L.ticket + pass, 1, 0u, st));
    }
    static const char *kLsdNames[kMaxPasses] = {"k_lsd_pass0", "k_lsd_pass1", "k_lsd_pass2"};
    GT_TIMED(kLsdNames[pass], launch_lsd(L.variant, p.bits[pass], L.lsd[pass], first, L.pay, last, L.pk[pass], L.wide,
                                         st));
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
  const size_t need = persist_tables_bytes(plan->count, plan->ptab_entries);
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
  if (pk_event) (void)hipEventSynchronize(pk_event);  // no copy still reads the staging buffer
  if (pk_event) (void)hipEventDestroy(pk_event);
  if (pk_host) (void)hipHostFree(pk_host);
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
  gt_plan_st *plan = new (std::nothrow) gt_plan_st();
  if (!plan) return GT_ERR_INVALID_ARGUMENT;
  plan->count = count;
  plan->validate = o.validate != 0;
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
