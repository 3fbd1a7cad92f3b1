// Layout arithmetic of a stable transposition, shared by the host and the
// device: every region of a graph's workspace from its parameters, the
// arguments of its kernels, and the phases of the persistent batched
// kernel.  The host plans with these functions; a plan whose parameters are
// chosen on the device (GT_FLAG_DEVICE_PLAN) runs the same functions in a
// planning kernel, so both sides lay out a graph identically.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/gt.h"
#include "gt_internal.h"
#include "gt_plan.h"

namespace gt {

constexpr size_t kLayoutAlign = 256;
__host__ __device__ inline size_t layout_align(size_t x) { return (x + kLayoutAlign - 1) & ~(kLayoutAlign - 1); }
__host__ __device__ inline int layout_ceil_log2(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x) ++b;
  return b;
}

// Parameters and workspace regions of a stable plan whose fine_bits,
// digit_bits and variant are chosen (the regions start at `base`).
__host__ __device__ inline void finalize_stable(GraphPlan &p, size_t base) {
  const int L = std::max(1, layout_ceil_log2(std::max<int64_t>(p.n, 2)));
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
  auto take = [&](size_t bytes) { size_t o = off; off = layout_align(off + bytes); return o; };
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

// The arguments of every kernel of a stable transposition.
__host__ __device__ inline StableLaunch stable_launch(const GraphPlan &p, const gt_csr_t &g, const gt_csc_t &out, char *ws, bool validate) {
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

__host__ __device__ inline void persist_coerce(GraphPlan &p) {
  p.variant = 1;
  p.digit_bits = (p.digit_bits < 9 ? p.digit_bits : 9);
}

__host__ __device__ inline bool persist_eligible(const GraphPlan &p) {
  if (p.strategy != GT_STRATEGY_STABLE) return false;
  if (p.n == 0 || p.m == 0) return true;
  return p.variant == 1 && p.tile == lsd_tile_size(1) && p.max_bits <= 9 && p.passes <= 2 && !p.wide_status;
}

__host__ __device__ inline uint32_t clamp_items(int64_t x, int64_t hi) {
  return (uint32_t)std::max<int64_t>(1, std::min<int64_t>(x, hi));
}

// The phases of one graph (at most kPersistMaxPhases), item counts from the
// plan alone; with a descriptor L, also the ranges the first phase clears.
__host__ __device__ inline int persist_phases(const GraphPlan &p, const StableLaunch *L, const gt_csc_t *out, int32_t g,
                                              bool validate, PersistPhase *ph) {
  constexpr int64_t NT = kPersistThreads;
  int k = 0;
  auto add = [&](PersistKind kind, int64_t nitems) {
    if (nitems <= 0) return;
    PersistPhase &q = ph[k++];
    q = PersistPhase{};
    q.kind = kind;
    q.graph = (uint32_t)g;
    q.nitems = (uint32_t)nitems;
    q.chunk = 1;
  };
  if (p.n == 0 || p.m == 0) {  // T = 0 everywhere
    add(kPhFill, clamp_items((2 * (p.n + 1) + NT * 16 - 1) / (NT * 16), 64));
    if (out) {
      ph[k - 1].fill[0] = reinterpret_cast<uint32_t *>(out->offsets);
      ph[k - 1].fill_words[0] = 2 * (uint64_t)(p.n + 1);
    }
    if (validate && p.n > 0) add(kPhValidate, clamp_items((p.n + NT - 1) / NT, 2048));
    return k;
  }
  const int64_t scan_tiles = (p.nbins + scan_tile_size() - 1) / scan_tile_size();
  const int64_t status_words = p.passes > 1 ? p.ntiles * ((int64_t)1 << p.max_bits) : 0;
  // counters and look-back words that start at zero
  add(kPhFill, clamp_items((status_words + scan_tiles + 3 + NT * 16 - 1) / (NT * 16), 256));
  if (L) {
    ph[k - 1].fill[0] = L->status;
    ph[k - 1].fill_words[0] = (uint64_t)status_words;
    ph[k - 1].fill[1] = L->sstatus;
    ph[k - 1].fill_words[1] = (uint64_t)scan_tiles;
    ph[k - 1].fill[2] = L->f.total_items + 1;  // scan ticket, big- and huge-bin counts
    ph[k - 1].fill_words[2] = 3;
  }
  if (validate) add(kPhValidate, clamp_items((p.n + NT - 1) / NT, 2048));
  const int64_t nblk = tile_scan_blocks(p.ntiles);
  add(kPhHist, std::min<int64_t>(kHistBlocks, std::max<int64_t>(1, p.ntiles)));
  add(kPhTileBsum, nblk);
  add(kPhTileBscan, (int64_t)1 << p.bits[0]);
  add(kPhTileOff, nblk);
  if (p.passes > 1) add(kPhDigitReduce, (int64_t)p.passes * (kMaxRadix / 64));
  add(kPhDigitScan, p.passes);
  add(kPhTileSrc, (p.ntiles + NT - 1) / NT);
  add(kPhPass0, p.ntiles);
  if (p.passes > 1) add(kPhPass1, p.ntiles);
  add(kPhBinItems, (p.nbins + NT - 1) / NT);
  add(kPhScan, scan_tiles);
  add(kPhItemMap, (p.nbins + NT - 1) / NT);
  add(kPhBigCount, p.max_items);
  add(kPhBigScan, p.max_big);
  add(kPhHugeScan, p.max_huge);
  add(kPhFinal, p.max_items);
  return k;
}

// Items per ticket: long phases hand out runs of up to 4 consecutive items
// (fewer tickets and dependency checks), as long as every resident
// workgroup still gets several tickets of the phase.  Look-back phases take
// one item per ticket: a run's last tile would hold up the next run's first.
__host__ __device__ inline uint32_t persist_chunk(uint32_t kind, uint32_t nitems, int grid) {
  if (kind == kPhPass1 || kind == kPhScan) return 1;
  const int64_t c = (int64_t)nitems / (8 * (int64_t)std::max(grid, 1));
  return (uint32_t)std::max<int64_t>(1, std::min<int64_t>(c, 4));
}

}  // namespace gt
