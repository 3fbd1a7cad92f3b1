// Work-item bodies of the transposition kernels.
//
// Every kernel's work is written as a body over one work item (`item` of
// `nitems`, NT threads) with its LDS passed in a struct.  The __global__
// kernels of gt_kernels.hip run one item per workgroup (item = blockIdx.x);
// the persistent batched kernel of gt_persistent.hip runs the same bodies on
// items it takes from its work queue.
//
// This header is compiled once per including file, into the namespace
// gt::GT_BODIES_NS, with the thread index read through GT_TID(): the
// one-item-per-workgroup kernels read threadIdx.x directly (the compiler
// knows its range), the persistent kernel through an opaque register move,
// so that no value derived from the thread index is hoisted out of its item
// loop and kept live across every body.
#pragma once
#if !defined(GT_BODIES_NS) || !defined(GT_TID)
#error "define GT_BODIES_NS and GT_TID() before including gt_bodies.hpp"
#endif
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gt_device.hpp"
#include "gt_internal.h"

namespace gt {
namespace GT_BODIES_NS {

// Zero `bytes` (a multiple of 16) of 16-byte aligned LDS with 16-byte stores.
__device__ __forceinline__ void lds_zero16(void *p, int bytes, int tid, int nt) {
  uint4 *q = static_cast<uint4 *>(p);
  for (int i = tid; i < bytes / 16; i += nt) q[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void fill_u32_body(uint32_t *p, uint64_t n, uint32_t v, int64_t item, int64_t nitems) {
  uint64_t i = (uint64_t)item * NT + GT_TID();
  const uint64_t s = (uint64_t)nitems * NT;
  for (; i < n; i += s) p[i] = v;
}
// Offsets validation: O[0] = 0, nondecreasing, O[n] = m.
template <int NT>
__device__ __forceinline__ void validate_offsets_body(const int64_t *O, int64_t n, int64_t m, uint32_t *err,
                                                      int64_t item, int64_t nitems) {
  int64_t i = item * NT + GT_TID();
  const int64_t s = nitems * NT;
  bool bad = false;
  if (i == 0) bad = (O[0] != 0) || (O[n] != m);
  for (; i < n; i += s)
    if (O[i + 1] < O[i]) bad = true;
  if (bad) atomicOr(err, kErrBadOffsets);
}
// Source of the first edge of every tile: the largest u with O[u] <= tile_base.
template <int NT>
__device__ __forceinline__ void tile_src_body(const int64_t *O, int64_t n, int64_t m, int64_t tile_size,
                                              int64_t ntiles, int32_t *out, int64_t item) {
  int64_t t = item * NT + GT_TID();
  if (t >= ntiles) return;
  const int64_t base = t * tile_size;
  int64_t lo = 0, hi = n;  // invariant: O[lo] <= base (when valid); answer in [lo, hi)
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (O[mid] <= base) lo = mid; else hi = mid;
  }
  (void)m;
  out[t] = (int32_t)lo;
}
// Step 1: digit histograms of the destinations, read in the tiles of the
// first partition pass (tile t = edges [t*TILE, (t+1)*TILE)), each workgroup
// a contiguous range of tiles.  Per tile, the counts of the first pass's
// digit (one LDS histogram for the workgroup) are written as a row of 16-bit
// counts, tilecnt[t][d]: their column prefix gives the first pass each
// tile's place within every digit, so that pass needs no look-back.  The
// digits of the later passes are summed over the workgroup's range and
// written as partial histograms (no global atomics), summed by
// k_digit_reduce.
template <int PASSES, int NT>
struct HistShared {
  static constexpr int NW = NT / kWave, LATER = PASSES > 1 ? PASSES - 1 : 1;
  uint32_t t[kMaxRadix];              // first pass, this tile (one copy)
  uint32_t h[NW][LATER * kMaxRadix];  // later passes, the workgroup's tiles
};

template <int PASSES, int TILE, int NT>
__device__ __forceinline__ void hist_body(const int32_t *__restrict__ D, int64_t m, int64_t n, const HistArgs &h,
                                          int64_t ntiles, uint32_t *__restrict__ part,
                                          uint16_t *__restrict__ tilecnt, uint32_t *err, int64_t item,
                                          int64_t nitems, HistShared<PASSES, NT> &sh_) {
  constexpr int NW = NT / kWave;
  constexpr int LATER = PASSES > 1 ? PASSES - 1 : 1;
  constexpr int V = TILE / 4 / NT;  // 16-byte loads per thread per tile
  static_assert(TILE % (4 * NT) == 0, "tile of whole 16-byte rows");
  uint32_t(&s_t)[kMaxRadix] = sh_.t;
  uint32_t(&s_h)[NW][LATER * kMaxRadix] = sh_.h;
  const int tid = GT_TID(), w = tid / kWave;
  const int b0 = h.bits[0], r0 = 1 << b0;
  for (int i = tid; i < NW * LATER * kMaxRadix; i += NT) (&s_h[0][0])[i] = 0;
  int sh[PASSES];
  uint32_t mk[PASSES];
#pragma unroll
  for (int p = 0; p < PASSES; ++p) { sh[p] = h.shift[p]; mk[p] = (1u << h.bits[p]) - 1u; }
  auto ctr = [&](int p, uint32_t d) -> uint32_t * {
    return p == 0 ? &s_t[d] : &s_h[w][(p - 1) * kMaxRadix + d];
  };
  bool bad = false;
  const uint32_t un = (uint32_t)(n > 0xFFFFFFFFll ? 0xFFFFFFFFll : n);
  auto count = [&](uint32_t u) {
    bad |= u >= un;  // also catches negative indices
#pragma unroll
    for (int p = 0; p < PASSES; ++p) atomicAdd(ctr(p, (u >> sh[p]) & mk[p]), 1u);
  };
  // Four consecutive destinations per lane.  Runs of equal digits (common
  // when destinations are close to their sources) are added once: per lane
  // when its four digits agree, per wave when every lane's do.
  auto count4 = [&](uint4 q) {
    bad |= (q.x >= un) | (q.y >= un) | (q.z >= un) | (q.w >= un);
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const uint32_t dx = (q.x >> sh[p]) & mk[p], dy = (q.y >> sh[p]) & mk[p];
      const uint32_t dz = (q.z >> sh[p]) & mk[p], dw = (q.w >> sh[p]) & mk[p];
      const bool same4 = (dx == dy) & (dy == dz) & (dz == dw);
      const uint32_t d0 = __builtin_amdgcn_readfirstlane(dx);
      const uint64_t active = __ballot(1);
      if (__all(same4 && dx == d0)) {
        if ((uint64_t)1 << (GT_TID() & 63) == (active & -active))
          atomicAdd(ctr(p, d0), 4u * (uint32_t)__popcll(active));
      } else if (same4) {
        atomicAdd(ctr(p, dx), 4u);
      } else {
        atomicAdd(ctr(p, dx), 1u);
        atomicAdd(ctr(p, dy), 1u);
        atomicAdd(ctr(p, dz), 1u);
        atomicAdd(ctr(p, dw), 1u);
      }
    }
  };
  const uint4 *D4 = reinterpret_cast<const uint4 *>(D);
  const int64_t t_beg = item * ntiles / nitems;
  const int64_t t_end = (item + 1) * ntiles / nitems;
  // the loads of the next tile are issued before the current one is counted
  uint4 q[V];
  auto load = [&](int64_t t) {
    const int64_t base = t * TILE;
    if (t < t_end && base + TILE <= m) {
#pragma unroll
      for (int v = 0; v < V; ++v) q[v] = D4[(base >> 2) + v * NT + tid];
    }
  };
  load(t_beg);
  for (int64_t t = t_beg; t < t_end; ++t) {
    for (int i = tid; i < r0; i += NT) s_t[i] = 0;
    __syncthreads();
    const int64_t base = t * TILE;
    if (base + TILE <= m) {
      uint4 c[V];
#pragma unroll
      for (int v = 0; v < V; ++v) c[v] = q[v];
      load(t + 1);
#pragma unroll
      for (int v = 0; v < V; ++v) count4(c[v]);
    } else {  // the last, ragged tile
      for (int64_t e = base + tid; e < m; e += NT) count((uint32_t)D[e]);
    }
    __syncthreads();
    uint16_t *row = tilecnt + t * r0;
    for (int d = tid; d < r0; d += NT) {
      row[d] = (uint16_t)s_t[d];
    }
    __syncthreads();
  }
  if (bad) atomicOr(err, kErrBadIndex);
  uint32_t *out = part + item * kMaxPasses * kMaxRadix;
  for (int p = 1; p < PASSES; ++p)
    for (int d = tid; d < (1 << h.bits[p]); d += NT) {
      uint32_t c = 0;
#pragma unroll
      for (int x = 0; x < NW; ++x) c += s_h[x][(p - 1) * kMaxRadix + d];
      out[p * kMaxRadix + d] = c;
    }
}
// Column prefix of the first pass's per-tile digit counts, over blocks of
// kTileBlk tiles: block sums (digit-major), an exclusive scan of each digit's
// block sums (which also yields the first pass's digit totals), then every
// tile's offset within each digit.  Offsets are kept in 32 bits: the offset
// of a tile that holds edges of digit d is below the digit's total, so below
// 2^32 for every accepted edge count.
template <int NT>
__device__ __forceinline__ void tile_bsum_body(const uint16_t *__restrict__ tilecnt, int64_t ntiles, int radix,
                                               int64_t nblk, uint32_t *__restrict__ bsum, int64_t b) {
  const int64_t t0 = b * kTileBlk, t1 = t0 + kTileBlk < ntiles ? t0 + kTileBlk : ntiles;
  for (int d = GT_TID(); d < radix; d += NT) {
    constexpr int U = 8;  // rows in flight
    uint32_t s = 0;
    int64_t t = t0;
    for (; t + U <= t1; t += U) {
      uint32_t c[U];
#pragma unroll
      for (int u = 0; u < U; ++u) c[u] = tilecnt[(t + u) * radix + d];
#pragma unroll
      for (int u = 0; u < U; ++u) s += c[u];
    }
    for (; t < t1; ++t) s += tilecnt[t * radix + d];
    bsum[(int64_t)d * nblk + b] = s;
  }
}
// One workgroup per digit: exclusive scan of its block sums, in place.
template <int NT>
struct ScanShared {
  uint64_t w[NT / kWave + 1];
};
template <int NT>
__device__ __forceinline__ void tile_bscan_body(uint32_t *bsum, int64_t nblk, uint64_t *totals0, int64_t d,
                                                ScanShared<NT> &sh) {
  constexpr int ITEMS = 8;
  uint64_t(&s_w)[NT / kWave + 1] = sh.w;
  const int tid = GT_TID(), lane = tid & (kWave - 1), w = tid / kWave;
  uint32_t *row = bsum + d * nblk;
  uint64_t carry = 0;
  for (int64_t c0 = 0; c0 < nblk; c0 += NT * ITEMS) {
    const int64_t base = c0 + (int64_t)tid * ITEMS;
    uint32_t v[ITEMS];
    uint64_t local = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      v[k] = base + k < nblk ? row[base + k] : 0u;
      local += v[k];
    }
    const uint64_t incl = wave_incl_sum64(local, lane);
    if (lane == kWave - 1) s_w[w] = incl;
    __syncthreads();
    if (tid == 0) {
      uint64_t run = 0;
      for (int i = 0; i < NT / kWave; ++i) { const uint64_t c = s_w[i]; s_w[i] = run; run += c; }
      s_w[NT / kWave] = run;
    }
    __syncthreads();
    uint64_t run = carry + s_w[w] + incl - local;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (base + k < nblk) {
        row[base + k] = (uint32_t)run;
        run += v[k];
      }
    carry += s_w[NT / kWave];
    __syncthreads();
  }
  if (tid == 0) totals0[d] = carry;
}
template <int NT>
__device__ __forceinline__ void tile_off_body(const uint16_t *__restrict__ tilecnt, int64_t ntiles, int radix,
                                              int64_t nblk, const uint32_t *__restrict__ bpre,
                                              uint32_t *__restrict__ tileoff, int64_t b) {
  const int64_t t0 = b * kTileBlk, t1 = t0 + kTileBlk < ntiles ? t0 + kTileBlk : ntiles;
  for (int d = GT_TID(); d < radix; d += NT) {
    uint32_t run = bpre[(int64_t)d * nblk + b];
    for (int64_t t = t0; t < t1; ++t) {
      tileoff[t * radix + d] = run;
      run += tilecnt[t * radix + d];
    }
  }
}
// Per-tile digit counts of a later pass, over the previous pass's output
// (tile t = positions [t*TILE, (t+1)*TILE) of its keys): one row of 16-bit
// counts per tile, as k_hist writes for the first pass, so that the pass
// places its tiles with their column prefix instead of a look-back.  Each
// thread reads a contiguous stretch of keys and adds runs of equal digits
// with one LDS atomic (a skewed graph's intermediate holds long runs of one
// destination), into an LDS histogram of its wave.
template <int NT>
struct TileHistShared {
  uint32_t c[NT / kWave][kMaxRadix];
};
template <int NT, int TILE, typename K>
__device__ __forceinline__ void tile_hist_body(const K *__restrict__ keys, int64_t m, int shift, int radix,
                                               uint16_t *__restrict__ tilecnt, int64_t t, TileHistShared<NT> &sh) {
  constexpr int NW = NT / kWave;
  constexpr int PER = 16 / (int)sizeof(K);  // keys per 16-byte load
  constexpr int V = TILE / PER / NT;        // loads per thread
  static_assert(TILE % (PER * NT) == 0, "tile of whole 16-byte rows");
  const int tid = GT_TID(), w = tid / kWave;
  const uint32_t mask = (uint32_t)radix - 1u;
  const int64_t base = t * TILE;
  uint4 q[V];
  const bool whole = base + TILE <= m;
  if (whole) {
    const uint4 *k4 = reinterpret_cast<const uint4 *>(keys + base) + (int64_t)tid * V;
#pragma unroll
    for (int v = 0; v < V; ++v) q[v] = k4[v];
  }
  const int rbits = __builtin_ctz((unsigned)radix);
  for (int i = tid; i < NW * radix; i += NT) sh.c[i >> rbits][i & (radix - 1)] = 0u;
  __syncthreads();
  uint32_t *c = sh.c[w];
  if (whole) {
    uint32_t prev = 0xFFFFFFFFu, run = 0;
    auto add = [&](uint32_t key) {
      const uint32_t d = (key >> shift) & mask;
      if (d != prev) {
        if (run) atomicAdd(&c[prev], run);
        prev = d;
        run = 0;
      }
      ++run;
    };
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const uint32_t wd[4] = {q[v].x, q[v].y, q[v].z, q[v].w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if constexpr (sizeof(K) == 2) {
          add(wd[k] & 0xFFFFu);
          add(wd[k] >> 16);
        } else {
          add(wd[k]);
        }
      }
    }
    atomicAdd(&c[prev], run);
  } else {  // the last, ragged tile
    for (int64_t e = base + tid; e < m; e += NT) atomicAdd(&c[((uint32_t)keys[e] >> shift) & mask], 1u);
  }
  __syncthreads();
  uint16_t *row = tilecnt + t * radix;
  for (int d = tid; d < radix; d += NT) {
    uint32_t sum = 0;
#pragma unroll
    for (int x = 0; x < NW; ++x) sum += sh.c[x][d];
    row[d] = (uint16_t)sum;
  }
}
// Step 2 (digit level), part 1: sum the per-workgroup partial histograms of
// the later passes.  Item (pass, 64-digit group); NT / 64 thread groups
// split the partials.
template <int NT>
struct ReduceShared {
  uint64_t sum[NT / 64][64];
};
template <int NT>
__device__ __forceinline__ void digit_reduce_body(const uint32_t *__restrict__ part, int nblocks, const HistArgs &h,
                                                  uint64_t *totals, int64_t item, ReduceShared<NT> &sh) {
  constexpr int NQ = NT / 64;
  const int p = (int)(item / (kMaxRadix / 64)), g = (int)(item % (kMaxRadix / 64));
  const int tid = GT_TID(), d = g * 64 + (tid & 63), q = tid >> 6;
  if (p == 0 || p >= h.passes) return;  // the first pass's totals come from k_tile_bscan
  const int radix = 1 << h.bits[p];
  uint64_t s = 0;
  if (d < radix) {
    // U partials in flight per thread
    constexpr int U = 8;
    constexpr int64_t kRow = (int64_t)kMaxPasses * kMaxRadix;
    const uint32_t *col = part + p * kMaxRadix + d;
    int b = q;
    for (; b + NQ * (U - 1) < nblocks; b += NQ * U) {
      uint32_t v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = col[(int64_t)(b + NQ * u) * kRow];
#pragma unroll
      for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; b < nblocks; b += NQ) s += col[(int64_t)b * kRow];
  }
  sh.sum[q][tid & 63] = s;
  __syncthreads();
  if (q == 0 && d < radix) {
    uint64_t t = 0;
#pragma unroll
    for (int x = 0; x < NQ; ++x) t += sh.sum[x][tid];
    totals[p * kMaxRadix + d] = t;
  }
}
// Step 2 (digit level), part 2: exclusive scan of the digit totals of every
// pass -> start of each digit in the partitioned stream.  Also the terminal
// bin start.  Item p = pass p.
template <int NT>
struct DigitScanShared {
  uint64_t tot[kMaxRadix];
  uint64_t wsum[NT / kWave + 1];
};
template <int NT>
__device__ __forceinline__ void digit_scan_body(const uint64_t *__restrict__ totals, const HistArgs &h,
                                                uint64_t *digit_start, uint64_t *bin_start, int64_t nbins_total,
                                                int64_t m, uint32_t *err, int p, DigitScanShared<NT> &sh) {
  const int tid = GT_TID();
  const int radix = 1 << h.bits[p];
  for (int d = tid; d < radix; d += NT) sh.tot[d] = totals[p * kMaxRadix + d];
  __syncthreads();
  const uint64_t sum = block_excl_scan<NT, uint64_t>(sh.tot, radix, sh.wsum);
  if (tid == 0 && sum != (uint64_t)m) atomicOr(err, kErrOverflow);  // every edge has one digit per pass
  for (int d = tid; d < radix; d += NT) digit_start[p * (kMaxRadix + 1) + d] = sh.tot[d];
  if (tid == 0) digit_start[p * (kMaxRadix + 1) + radix] = (uint64_t)m;
  if (p == 0 && tid == 0) bin_start[nbins_total] = (uint64_t)m;
}
// ---------------------------------------------------------------------------
// k_lsd: one stable partition pass by a destination digit.
// ---------------------------------------------------------------------------
template <int WAVES, int ITEMS, int RBITS, bool PK_IN>
struct LsdShared {
  static constexpr int NT = WAVES * kWave, TILE = NT * ITEMS, RADIX = 1 << RBITS;
  // staging buffer; during ranking it holds the per-wave lane-mask tables
  static constexpr int STAGE_WORDS = TILE > 2 * WAVES * RADIX ? TILE : 2 * WAVES * RADIX;
  alignas(16) uint32_t stage[STAGE_WORDS];
  alignas(16) uint16_t wcnt[WAVES][RADIX];
  uint32_t tot[RADIX];
  uint32_t toff[RADIX];
  uint64_t gbase[RADIX];
  uint32_t misc[NT / kWave + 1];
  int64_t tile;
  // PK_IN: positions (relative to the tile) where a digit of the first pass
  // starts inside the tile; fl = {their number, first-pass digit of the
  // tile's first edge, of the previous tile's last edge}
  uint16_t bnd[PK_IN ? kMaxRadix : 1];
  int32_t fl[3];
};

// One tile of a partition pass.  order_in: the tile's place in the pass's
// order when the caller assigns it (the persistent kernel's queue), or -1:
// the first pass runs XCD-ordered tiles by workgroup index, later passes take
// a ticket.
template <int WAVES, int ITEMS, int RBITS, bool CSR_IN, bool PAY, bool LAST, bool PACKED, typename SW>
__device__ __forceinline__ void lsd_body(const LsdArgs &a, int64_t order_in,
                                         LsdShared<WAVES, ITEMS, RBITS, PACKED && !CSR_IN && LAST> &sh) {
  // PACKED: the first pass of a two-pass plan writes the packed 6-byte
  // intermediate (PK_OUT), the last pass reads it (PK_IN)
  constexpr bool PK_OUT = PACKED && CSR_IN && !LAST;
  constexpr bool PK_IN = PACKED && !CSR_IN && LAST;
  using Sh = LsdShared<WAVES, ITEMS, RBITS, PK_IN>;
  constexpr int NT = Sh::NT;
  constexpr int TILE = Sh::TILE;
  constexpr int RADIX = Sh::RADIX;
  uint32_t(&s_stage)[Sh::STAGE_WORDS] = sh.stage;
  uint16_t(&s_wcnt)[WAVES][RADIX] = sh.wcnt;
  uint32_t(&s_tot)[RADIX] = sh.tot;
  uint32_t(&s_toff)[RADIX] = sh.toff;
  uint64_t(&s_gbase)[RADIX] = sh.gbase;
  uint32_t(&s_misc)[NT / kWave + 1] = sh.misc;
  int64_t &s_tile = sh.tile;
  uint16_t(&s_bnd)[PK_IN ? kMaxRadix : 1] = sh.bnd;
  int32_t(&s_fl)[3] = sh.fl;

  const int tid = GT_TID();
  int lane = tid & (kWave - 1), w = tid / kWave;
  const int radix = 1 << a.bits;
  const uint32_t dmask = (uint32_t)radix - 1u;

  lds_zero16(&s_wcnt[0][0], WAVES * RADIX * 2, tid, NT);
  lds_zero16(s_stage, 2 * WAVES * RADIX * 4, tid, NT);
  // A pass placed with per-tile digit offsets (the first pass always; a
  // later pass when a.placed) takes its tiles in runs of consecutive tiles
  // per XCD (their digit runs meet in one L2); a later pass with a look-back
  // takes them in ticket order.
  const bool placed = CSR_IN || a.placed;
  if (tid == 0)
    s_tile = order_in >= 0 ? order_in
                           : (placed ? xcd_item(blockIdx.x, (a.m + TILE - 1) / TILE, GT_XCD_BLOCK)
                                     : (int64_t)atomicAdd(a.ticket, 1u));
  if (PK_IN && tid < 3) s_fl[tid] = 0;
  __syncthreads();
  // The first pass takes its tiles from the end of the edge array: the
  // sources of a natural-order graph thin out towards high IDs, and a tile
  // there fills its sources from up to ~10^5 offsets, so those tiles start
  // first instead of closing the launch.  It places its tiles with the
  // per-tile digit offsets of k_hist (no look-back); a later pass either
  // places them with the offsets of k_tile_hist's counts or takes them from
  // a ticket and runs a decoupled look-back over them.
  const int64_t ntiles = (a.m + TILE - 1) / TILE;
  // position in the look-back chain; below 2^31 (a tile holds at least 4096
  // edges), read into a scalar register so the tile's bounds are scalar too
  const int64_t order = (int64_t)__builtin_amdgcn_readfirstlane((int)s_tile);
  const int64_t tile = CSR_IN ? ntiles - 1 - order : order;
  const int64_t base = tile * TILE;
  const int64_t cnt64 = a.m - base < TILE ? a.m - base : TILE;
  const int cnt = (int)cnt64;
  // rows of 64 consecutive edges; wave w owns rows [w*ITEMS, (w+1)*ITEMS)
  auto row_idx = [&](int j) { return (w * ITEMS + j) * kWave + lane; };

  // Keys first.  Without a payload, the sources of later passes are loaded
  // once the keys are staged: their latency still hides behind the look-back
  // and the ranking holds 16 registers fewer, which leaves room for three
  // workgroups per CU.  With a payload, sources and payload are loaded with
  // the keys (measured faster: the payload's latency is the longer one to
  // hide).  The first pass derives its sources from the offsets further down.
  constexpr bool kEarly = PAY;
  uint32_t key[ITEMS];
  uint32_t src_in[CSR_IN ? 1 : ITEMS];
  uint32_t pay_in[PAY ? ITEMS : 1];
  auto load_src_pay = [&]() {
    if constexpr (!CSR_IN) {
      const int32_t *sin = a.in_src + base;
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) src_in[j] = row_idx(j) < cnt ? (uint32_t)sin[row_idx(j)] : 0u;
    }
    if constexpr (PAY) {
      const uint32_t *pin = CSR_IN ? a.P + base : a.in_pay + base;
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) pay_in[j] = row_idx(j) < cnt ? pin[row_idx(j)] : 0u;
    }
  };
  if constexpr (PK_IN) {
    // 16-bit loads take a clamped index and no branch (a 16-bit load inside a
    // per-row branch is waited for before the next is issued); the edge's
    // position in the tile rides in the upper half
    const uint16_t *kin = a.in_key16 + base;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) key[j] = kin[row_idx(j) < cnt ? row_idx(j) : cnt - 1];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) key[j] = row_idx(j) < cnt ? key[j] | ((uint32_t)row_idx(j) << 16) : 0u;
    if constexpr (kEarly) load_src_pay();
  } else {
    const uint32_t *kin = CSR_IN ? reinterpret_cast<const uint32_t *>(a.D) + base : a.in_key + base;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) key[j] = row_idx(j) < cnt ? kin[row_idx(j)] : 0u;
    if constexpr (kEarly) load_src_pay();
  }
  // first pass: the source of the tile's first edge and the first offset
  // each thread inspects for the source marks (loaded after the staging)
  int64_t u0 = 0, o_first = 0;

  // In-wave stable ranking: rows in edge order, peers matched through LDS.
  // Local positions stay below the tile size: two per register.
  Packed16<ITEMS> lpos;
  {
    unsigned long long *tab = reinterpret_cast<unsigned long long *>(s_stage) + w * RADIX;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      lpos.set(j, rank_row_lds<true>((key[j] >> a.shift) & dmask, row_idx(j) < cnt, s_wcnt[w], tab, lane));
  }
  __syncthreads();

  // per digit: tile total, and exclusive prefix over waves (in place); the
  // tile's aggregate is published at once so that later tiles can use it
  for (int d = tid; d < radix; d += NT) {
    uint32_t run = 0;
#pragma unroll
    for (int x = 0; x < WAVES; ++x) run += s_wcnt[x][d];
    s_tot[d] = run;
    s_toff[d] = run;
    if (!placed) lookback_publish<SW>(static_cast<SW *>(a.status), order, radix, d, run);
  }
  // the scan below reads s_toff in blocks of radix / NT entries per thread,
  // so with more digits than threads it reads other threads' writes
  __syncthreads();
  block_excl_scan<NT, uint32_t>(s_toff, radix, s_misc);  // tile-local digit offsets (ends with a barrier)
  for (int d = tid; d < radix; d += NT) {
    uint32_t run = s_toff[d];
#pragma unroll
    for (int x = 0; x < WAVES; ++x) {
      const uint32_t c = s_wcnt[x][d];
      s_wcnt[x][d] = (uint16_t)run;
      run += c;
    }
  }
  __syncthreads();
  // first pass (no look-back wait below to bound the scheduler): the row
  // addresses of the ranking are recomputed from here on rather than kept
  // in registers across the scan, which keeps six waves per SIMD
  if constexpr (CSR_IN) {
    lane = opaque_int(lane);
    w = opaque_int(w);
  }

  // stage keys in sorted order (the keys leave registers before the wait);
  // PK_IN: with the edge's position in the tile in the upper half (its
  // first-pass digit follows from it)
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (row_idx(j) < cnt) {
      const uint32_t d = (key[j] >> a.shift) & dmask;
      const uint32_t p = lpos.get(j) + s_wcnt[w][d];
      lpos.set(j, p);
      s_stage[p] = key[j];
    }
  }
  if constexpr (PK_IN) {
    // first-pass digit of position g: the number of first-pass digits d >= 1
    // that start at or before g (digit starts are nondecreasing, so empty
    // digits are skipped).  Counted here for the tile's first edge and the
    // previous tile's last edge; the digit starts inside the tile are listed.
    const int prad = 1 << a.prev_bits;
    uint32_t le_base = 0, le_prev = 0;
    for (int d = 1 + tid; d < prad; d += NT) {
      const uint64_t ds = a.prev_digit_start[d];
      le_base += ds <= (uint64_t)base;
      le_prev += ds < (uint64_t)base;
      if (ds > (uint64_t)base && ds < (uint64_t)(base + cnt64)) s_bnd[atomicAdd(&s_fl[0], 1)] = (uint16_t)(ds - base);
    }
    le_base = wave_incl_sum(le_base, lane);
    le_prev = wave_incl_sum(le_prev, lane);
    if (lane == kWave - 1) {
      if (le_base) atomicAdd(&s_fl[1], (int32_t)le_base);
      if (le_prev) atomicAdd(&s_fl[2], (int32_t)le_prev);
    }
  }
  if constexpr (!kEarly) load_src_pay();
  if constexpr (CSR_IN) {  // loaded here, where fewer values are live
    u0 = a.tile_src0[tile];
    const int64_t u = u0 + 1 + tid;
    o_first = u < a.n ? a.O[u] : a.m;
  }
  // the tile's place within each digit (the column prefix of the per-tile
  // counts, or the look-back across tiles); staged slot i of digit d goes
  // to s_gbase[d] + i
  for (int d = tid; d < radix; d += NT) {
    if (placed) {
      s_gbase[d] = a.digit_start[d] + a.tile_off[tile * radix + d] - s_toff[d];
    } else {
      const uint64_t excl = lookback_wait<SW>(static_cast<SW *>(a.status), order, radix, d, s_tot[d]);
      s_gbase[d] = a.digit_start[d] + excl - s_toff[d];
    }
  }
  __syncthreads();

  // write keys; remember each output slot's digit (two per register).
  // PK_OUT: the slot's 16 bits also hold the fine bits that go into the
  // source word (bits 10..); PK_IN: they are the packed key itself, whose
  // fine bits are completed from the source word when it is written.
  const uint32_t pk_lomask = (1u << a.pk_lo) - 1u;
  uint32_t dpk[(ITEMS + 1) / 2];
#pragma unroll
  for (int k = 0; k < (ITEMS + 1) / 2; ++k) dpk[k] = 0u;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int i = k * NT + tid;
    if (i < cnt) {
      const uint32_t kv = s_stage[i];
      const uint32_t d = (kv >> a.shift) & dmask;
      uint32_t half = d;
      const uint64_t gp = s_gbase[d] + (uint64_t)i;
      if constexpr (PK_IN) {
        half = kv & 0xFFFFu;
      } else if constexpr (LAST) {
        a.out_key16[gp] = (uint16_t)(kv & a.fine_mask);
      } else if constexpr (PK_OUT) {
        const uint32_t fine = kv & a.fine_mask;
        const uint32_t d_last = (kv >> a.pk_dshift) & ((1u << a.pk_dbits) - 1u);
        a.out_key16[gp] = (uint16_t)((d_last << a.pk_lo) | (fine & pk_lomask));
        half = d | ((fine >> a.pk_lo) << 10);
      } else {
        a.out_key32[gp] = kv;
      }
      dpk[k >> 1] |= half << ((k & 1) * 16);
    }
  }
  auto half_of = [&](int k) -> uint32_t { return (dpk[k >> 1] >> ((k & 1) * 16)) & 0xFFFFu; };
  auto gpos_of = [&](int k, int i) -> uint64_t {
    const uint32_t h = half_of(k);
    const uint32_t d = PK_IN ? (h >> a.shift) & dmask : (PK_OUT ? h & 0x3FFu : h);
    return s_gbase[d] + (uint64_t)i;
  };

  if (LAST) {
    // Bin starts.  The tile owns the fine bins whose lower part fl lies in
    // (fl of the previous tile's last edge, fl of this tile's last edge]; for
    // every digit d the bin (d, fl) starts after the tile's edges of digit d
    // with a smaller lower part (edges of one digit are staged sorted by fl).
    const uint32_t lmask = (1u << a.lower_bits) - 1u;
    const uint32_t fl_first = PK_IN ? (uint32_t)s_fl[1] : 0u;
    const int nbnd = PK_IN ? s_fl[0] : 0;
    auto fl_of = [&](uint32_t kv) -> uint32_t {
      if constexpr (PK_IN) {
        uint32_t fl = fl_first;
        for (int b = 0; b < nbnd; ++b) fl += (uint32_t)s_bnd[b] <= (kv >> 16);
        return fl;
      } else {
        return (kv >> a.fine_shift) & lmask;
      }
    };
    int64_t fl_prev = -1;
    if (tile > 0) {
      if (PK_IN) fl_prev = s_fl[2];
      else fl_prev = CSR_IN ? (int64_t)fl_of((uint32_t)a.D[base - 1]) : (int64_t)fl_of(a.in_key[base - 1]);
    }
    int64_t fl_hi;
    if (base + cnt64 >= a.m) fl_hi = (int64_t)lmask;
    else if (PK_IN) fl_hi = (int64_t)fl_first + nbnd;
    else fl_hi = CSR_IN ? (int64_t)fl_of((uint32_t)a.D[base + cnt64 - 1]) : (int64_t)fl_of(a.in_key[base + cnt64 - 1]);
    const int64_t nown = fl_hi - fl_prev;
    for (int64_t q = tid; q < nown * radix; q += NT) {
      const uint32_t fl = (uint32_t)(fl_prev + 1 + q / radix);
      const uint32_t d = (uint32_t)(q % radix);
      int lo = (int)s_toff[d], hi = lo + (int)s_tot[d];
      while (lo < hi) {  // first staged edge of digit d with fl >= target
        const int mid = (lo + hi) >> 1;
        if (fl_of(s_stage[mid]) < fl) lo = mid + 1; else hi = mid;
      }
      a.bin_start[((uint64_t)d << a.lower_bits) | fl] = s_gbase[d] + (uint64_t)lo;
    }
  }
  __syncthreads();

  // sources
  {
    uint32_t src[ITEMS];
    if (CSR_IN) {
      // mark the first edge of every source that starts inside the tile, then
      // fill forward (sources increase along the edge array)
      lds_zero16(s_stage, TILE * 4, tid, NT);
      __syncthreads();
      if (tid == 0) s_stage[0] = (uint32_t)u0;
      // the last source that can start inside the tile: the next tile's
      // first edge's source (every later source starts after the tile).
      // Vertex IDs are below 2^31, so the walk stays in 32 bits.
      int64_t o = o_first;
      if constexpr (PK_OUT) {
        const uint32_t u_end = tile + 1 < ntiles ? (uint32_t)a.tile_src0[tile + 1] : (uint32_t)(a.n - 1);
        for (uint32_t u = (uint32_t)u0 + 1u + (uint32_t)tid; u <= u_end;) {
          if (o > base && o < base + cnt64) atomicMax(&s_stage[o - base], u);
          u += NT;
          if (u <= u_end) o = a.O[u];
        }
      } else {
        for (int64_t u = u0 + 1 + tid; u < a.n;) {
          if (o >= base + cnt64) break;
          if (o > base) atomicMax(&s_stage[o - base], (uint32_t)u);
          u += NT;
          if (u < a.n) o = a.O[u];
        }
      }
      __syncthreads();
      // running maximum along the wave's rows, kept in registers (each
      // thread reads exactly the slots of its own edges)
      uint32_t carry = 0;
#pragma unroll
      for (int r = 0; r < ITEMS; ++r) {
        uint32_t v = wave_incl_max(s_stage[row_idx(r)], lane);
        v = v > carry ? v : carry;
        src[r] = v;
        carry = wave_last(v);
      }
      if (lane == 0) s_misc[w] = carry;
      __syncthreads();  // also: every read of the marks is done before staging below
      uint32_t before = 0;
      for (int i = 0; i < w; ++i) before = before > s_misc[i] ? before : s_misc[i];
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) src[j] = src[j] > before ? src[j] : before;
    } else {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) src[j] = src_in[CSR_IN ? 0 : j];
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (row_idx(j) < cnt) s_stage[lpos.get(j)] = src[j];
  }
  __syncthreads();
  // PK_IN: the fine bits of every slot, completed from its source word, are
  // written after the sources (two per register until then)
  uint32_t fpk[PK_IN ? (ITEMS + 1) / 2 : 1];
#pragma unroll
  for (int k = 0; k < (PK_IN ? (ITEMS + 1) / 2 : 1); ++k) fpk[k] = 0u;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int i = k * NT + tid;
    if (i < cnt) {
      uint32_t sv = s_stage[i];
      if constexpr (PK_OUT) sv |= (half_of(k) >> 10) << a.pk_src_bits;
      if constexpr (PK_IN) {
        fpk[k >> 1] |= ((half_of(k) & pk_lomask) | ((sv >> a.pk_src_bits) << a.pk_lo)) << ((k & 1) * 16);
        sv &= (1u << a.pk_src_bits) - 1u;
      }
      a.out_src[gpos_of(k, i)] = (int32_t)sv;
    }
  }
  if constexpr (PK_IN) {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int i = k * NT + tid;
      if (i < cnt) a.out_key16[gpos_of(k, i)] = (uint16_t)(fpk[k >> 1] >> ((k & 1) * 16));
    }
  }
  if (PAY) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (row_idx(j) < cnt) s_stage[lpos.get(j)] = pay_in[PAY ? j : 0];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int i = k * NT + tid;
      if (i < cnt) a.out_pay[gpos_of(k, i)] = s_stage[i];
    }
  }
}

// ---------------------------------------------------------------------------
// Generic exclusive scan of a u32 array (decoupled look-back over tiles).
// ---------------------------------------------------------------------------
template <int NT>
struct ScanU32Shared {
  uint32_t w[NT / kWave + 1];
  int64_t tile;
  uint64_t excl;
};
// order_in: the tile's place in the look-back chain when the caller assigns
// it (the persistent kernel's queue), or -1: take a ticket
template <int NT, int ITEMS>
__device__ __forceinline__ void scan_u32_body(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                              int64_t len, uint32_t *status, uint32_t *ticket, uint32_t *total,
                                              int64_t order_in, ScanU32Shared<NT> &sh) {
  constexpr int TILE = NT * ITEMS;
  uint32_t(&s_w)[NT / kWave + 1] = sh.w;
  int64_t &s_tile = sh.tile;
  uint64_t &s_excl = sh.excl;
  const int tid = GT_TID(), lane = tid & (kWave - 1), w = tid / kWave;
  if (tid == 0) s_tile = order_in >= 0 ? order_in : (int64_t)atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t base = tile * TILE + (int64_t)tid * ITEMS;
  uint32_t v[ITEMS];
  uint32_t local = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    v[k] = (base + k < len) ? in[base + k] : 0u;
    local += v[k];
  }
  const uint32_t incl = wave_incl_sum(local, lane);
  if (lane == kWave - 1) s_w[w] = incl;
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (int i = 0; i < NT / kWave; ++i) { const uint32_t c = s_w[i]; s_w[i] = run; run += c; }
    s_w[NT / kWave] = run;
    s_excl = lookback_exclusive<uint32_t>(status, tile, 1, 0, run);
    if ((tile + 1) * TILE >= len) *total = (uint32_t)(s_excl + run);
  }
  __syncthreads();
  uint32_t run = (uint32_t)s_excl + s_w[w] + incl - local;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (base + k < len) { out[base + k] = run; run += v[k]; }
}
// Per bin: number of work items of k_final (bins longer than one tile are
// split into tile-sized chunks).  Also writes T[n] = m.
template <int NT>
__device__ __forceinline__ void bin_items_body(const uint64_t *bin_start, int64_t nbins, int64_t tile,
                                               uint32_t *nch, int64_t *T, int64_t n, int64_t m, int64_t item) {
  const int64_t f = item * NT + GT_TID();
  if (f >= nbins) return;
  const uint64_t N = bin_start[f + 1] - bin_start[f];
  nch[f] = N > (uint64_t)tile ? (uint32_t)((N + tile - 1) / tile) : 1u;
  if (f == nbins - 1) T[n] = m;
}
// Work-item descriptors (first edge, bin, edge count, whole-bin flag), so
// that k_big_count and k_final find their edges with one load instead of a
// chain item -> bin -> bin start; and the list of bins split into several
// chunks (its order is irrelevant: every big bin is processed independently).
template <int NT>
__device__ __forceinline__ void item_map_body(const uint32_t *nch, const uint32_t *item_base,
                                              const uint64_t *bin_start, int64_t nbins, int64_t tile,
                                              uint4 *item_desc, uint32_t *bigbins, uint32_t *nbig,
                                              uint32_t *hugebins, uint32_t *nhuge, int64_t item) {
  const int64_t f = item * NT + GT_TID();
  if (f >= nbins) return;
  const uint32_t b = item_base[f], c = nch[f];
  const uint64_t bs = bin_start[f], be = bin_start[f + 1];
  for (uint32_t k = 0; k < c; ++k) {
    const uint64_t cb = bs + (uint64_t)k * (uint64_t)tile;
    const uint32_t cnt = (uint32_t)(be - cb < (uint64_t)tile ? be - cb : (uint64_t)tile);
    item_desc[b + k] = make_uint4((uint32_t)cb, (uint32_t)(cb >> 32), (uint32_t)f, cnt | (c == 1 ? 0x80000000u : 0u));
  }
  // append to the lists with one atomic per wave and list
  const int lane = GT_TID() & (kWave - 1);
  auto push = [&](bool want, uint32_t *list, uint32_t *counter) {
    const unsigned long long mask = __ballot(want);
    if (mask == 0ull) return;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t first = 0;
    if (lane == leader) first = atomicAdd(counter, (uint32_t)__popcll(mask));
    first = (uint32_t)__shfl((int)first, leader);
    if (want) list[first + (uint32_t)__popcll(mask & lanemask_lt(lane))] = (uint32_t)f;
  };
  push(c > 1 && c <= (uint32_t)kHugeChunks, bigbins, nbig);
  push(c > (uint32_t)kHugeChunks, hugebins, nhuge);
}
// Big bins: in-degree of every vertex of the bin within each chunk.
template <int FBITS>
struct BigCountShared {
  uint32_t cnt[1 << FBITS];
};
template <int WAVES, int ITEMS, int FBITS>
__device__ __forceinline__ void big_count_body(const FinalArgs &a, int64_t item, BigCountShared<FBITS> &sh) {
  constexpr int NT = WAVES * kWave;
  constexpr int TILE = NT * ITEMS;
  constexpr int FW = 1 << FBITS;
  uint32_t(&s_cnt)[FW] = sh.cnt;
  const uint32_t total = *a.total_items;
  const uint4 dsc = a.item_desc[item];  // grid = the most items a plan can have
  if (item >= (int64_t)total || (dsc.w >> 31)) return;  // whole bins have no chunk counts
  const int tid = GT_TID();
  const int fw = 1 << a.fine_bits;
  const uint32_t vmask = (uint32_t)fw - 1u;
  const uint64_t cb = (uint64_t)dsc.x | ((uint64_t)dsc.y << 32);
  const int cnt = (int)(dsc.w & 0x7FFFFFFFu);
  for (int v = tid; v < fw; v += NT) s_cnt[v] = 0;
  __syncthreads();
  // all of the thread's keys are loaded before the first count, so the
  // loads are in flight together (clamped index, no branch around a load)
  const uint16_t *keys = a.in_key + cb;
  uint32_t kv[ITEMS];
  if (cnt > 0) {
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int i = j * NT + tid;
      kv[j] = keys[i < cnt ? i : cnt - 1];
    }
    // In a hub's chunk most lanes of a row (64 consecutive edges of one wave)
    // share one destination, and 64 lanes updating one LDS counter would be
    // serialised: a wave whose first row is dominated by lane 0's
    // destination adds, in every row, the lanes that share lane 0's
    // destination with one atomic.  Other waves count lane by lane.
    const int lane = tid & (kWave - 1);
    auto dominated = [&](int j, uint32_t &k0, unsigned long long &same) {
      const bool in = j * NT + tid < cnt;
      const uint32_t k = kv[j] & vmask;
      k0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)k);
      same = __ballot(in && k == k0);
      return __popcll(same) >= 16;
    };
    uint32_t k00;
    unsigned long long same0;
    if (dominated(0, k00, same0)) {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        const bool in = j * NT + tid < cnt;
        const uint32_t k = kv[j] & vmask;
        uint32_t k0;
        unsigned long long same;
        if (dominated(j, k0, same)) {
          if (lane == 0) atomicAdd(&s_cnt[k0], (uint32_t)__popcll(same));
          if (in && k != k0) atomicAdd(&s_cnt[k], 1u);
        } else if (in) {
          atomicAdd(&s_cnt[k], 1u);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j)
        if (j * NT + tid < cnt) atomicAdd(&s_cnt[kv[j] & vmask], 1u);
    }
  }
  __syncthreads();
  uint32_t *row = a.cntab + (uint64_t)item * fw;
  for (int v = tid; v < fw; v += NT) row[v] = s_cnt[v];
}
// Big bins, after k_big_count: per-vertex exclusive prefix over the bin's
// chunks (in place) and the bin's CSC offsets.  One workgroup per big bin.
// Bins of more than kHugeChunks chunks (a few hub regions) come in a second
// launch with one thread per vertex and more rows in flight: their chains of
// dependent round trips set the kernel's length.
template <int NT>
struct BigScanShared {
  uint64_t tot[1 << kMaxFineBits];
  uint64_t w64[NT / kWave + 1];
};
template <int NT, int B, bool HUGE>
__device__ __forceinline__ void big_scan_body(const FinalArgs &a, int64_t item, BigScanShared<NT> &sh) {
  uint64_t(&s_tot)[1 << kMaxFineBits] = sh.tot;
  uint64_t(&s_w64)[NT / kWave + 1] = sh.w64;
  if (item >= (int64_t)*(HUGE ? a.nhuge : a.nbig)) return;
  const uint32_t f = (HUGE ? a.hugebins : a.bigbins)[item];
  const uint32_t nch = a.nch[f];
  const uint32_t first_item = a.item_base[f];
  const int tid = GT_TID();
  const int fw = 1 << a.fine_bits;
  for (int v = tid; v < fw; v += NT) {
    uint64_t run = 0;
    for (uint32_t k0 = 0; k0 < nch; k0 += B) {
      uint32_t c[B];
#pragma unroll
      for (int k = 0; k < B; ++k) c[k] = (k0 + k < nch) ? a.cntab[(uint64_t)(first_item + k0 + k) * fw + v] : 0u;
#pragma unroll
      for (int k = 0; k < B; ++k)
        if (k0 + k < nch) {
          a.cntab[(uint64_t)(first_item + k0 + k) * fw + v] = (uint32_t)run;
          run += c[k];
        }
    }
    s_tot[v] = run;
  }
  __syncthreads();
  const uint64_t bin_total = block_excl_scan<NT, uint64_t>(s_tot, fw, s_w64);
  const uint64_t bs = a.bin_start[f];
  if (tid == 0 && bs + bin_total != a.bin_start[f + 1]) atomicOr(a.err, kErrOverflow);
  const int64_t v0 = (int64_t)f << a.fine_bits;
  for (int v = tid; v < fw; v += NT)
    if (v0 + v < a.n) a.T[v0 + v] = (int64_t)(bs + s_tot[v]);
}
// ---------------------------------------------------------------------------
// k_final: stable placement of one work item (a whole small bin, or one
// tile-sized chunk of a big bin) -> CSC sources/payload (+ offsets of small
// bins).
// ---------------------------------------------------------------------------
template <int WAVES, int ITEMS, int FBITS>
struct FinalShared {
  static constexpr int NT = WAVES * kWave, TILE = NT * ITEMS, FW = 1 << FBITS;
  // The per-wave lane-mask tables and counters hold one key more (FW): the
  // lanes of the item's partial row past its last edge rank under it, so no
  // row is ranked under a lane predicate.  Rows padded to 16 bytes.
  static constexpr int FWX = FW + 8;
  static constexpr int STAGE_WORDS = TILE > 2 * WAVES * FWX ? TILE : 2 * WAVES * FWX;
  alignas(16) uint32_t stage[STAGE_WORDS];
  // per wave and vertex: the wave's count, then the slot of the wave's first
  // edge of that vertex (the vertex's offset plus the earlier waves' counts)
  alignas(16) uint16_t wcnt[WAVES][FWX];
  uint32_t toff[FW];
  uint64_t cur[FW];
  uint32_t w32[NT / kWave + 1];
};
template <int WAVES, int ITEMS, int FBITS, bool PAY>
__device__ __forceinline__ void final_body(const FinalArgs &a, int64_t item, FinalShared<WAVES, ITEMS, FBITS> &sh) {
  using Sh = FinalShared<WAVES, ITEMS, FBITS>;
  constexpr int NT = Sh::NT;
  constexpr int FW = Sh::FW;
  constexpr int FWX = Sh::FWX;
  uint32_t(&s_stage)[Sh::STAGE_WORDS] = sh.stage;
  uint16_t(&s_wcnt)[WAVES][FWX] = sh.wcnt;
  uint32_t(&s_toff)[FW] = sh.toff;
  uint64_t(&s_cur)[FW] = sh.cur;
  uint32_t(&s_w32)[NT / kWave + 1] = sh.w32;
  const uint32_t total = *a.total_items;
  const uint4 dsc = a.item_desc[item];  // grid = the most items a plan can have
  if (item >= (int64_t)total) return;
  const int tid = GT_TID(), lane = tid & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(tid / kWave);
  // the item's descriptor is the workgroup's: scalar registers, so the tile's
  // base pointers are scalar and every access below takes a 32-bit offset
  const uint32_t dx = (uint32_t)__builtin_amdgcn_readfirstlane((int)dsc.x);
  const uint32_t dy = (uint32_t)__builtin_amdgcn_readfirstlane((int)dsc.y);
  const uint32_t f = (uint32_t)__builtin_amdgcn_readfirstlane((int)dsc.z);
  const uint32_t dw = (uint32_t)__builtin_amdgcn_readfirstlane((int)dsc.w);
  const bool whole = (dw >> 31) != 0u;
  const int fw = 1 << a.fine_bits;
  const uint32_t vmask = (uint32_t)fw - 1u;
  const uint64_t cb = (uint64_t)dx | ((uint64_t)dy << 32);
  const uint64_t bs = cb;  // a whole bin starts at its item's first edge
  const int cnt = (int)(dw & 0x7FFFFFFFu);
  const int64_t v0 = (int64_t)f << a.fine_bits;
  auto row_idx = [&](int j) { return (w * ITEMS + j) * kWave + lane; };

  lds_zero16(&s_wcnt[0][0], WAVES * FWX * 2, tid, NT);
  lds_zero16(s_stage, 2 * WAVES * FWX * 4, tid, NT);
  if (!whole) {
    const uint32_t *row = a.cntab + (uint64_t)item * fw;
    for (int v = tid; v < fw; v += NT) s_cur[v] = v0 + v < a.n ? (uint64_t)a.T[v0 + v] + row[v] : 0ull;
  }
  __syncthreads();
  // keys and sources at once (the sources are staged later; the payload is
  // loaded when it is staged, which keeps three workgroups per CU).  The key
  // loads take a clamped index and no branch: a 16-bit load masked inside a
  // per-row branch is waited for before the next one is issued.
  const uint16_t *kin = a.in_key + cb;
  const int32_t *sin = a.in_src + cb;
  uint32_t key[ITEMS], src[ITEMS], lpos[ITEMS];
  if (cnt > 0) {
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) key[j] = kin[row_idx(j) < cnt ? row_idx(j) : cnt - 1];
  }
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) src[j] = row_idx(j) < cnt ? (uint32_t)sin[row_idx(j)] : 0u;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) key[j] = row_idx(j) < cnt ? key[j] & vmask : (uint32_t)FW;
  {
    unsigned long long *tab = reinterpret_cast<unsigned long long *>(s_stage) + w * FWX;
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      lpos[j] = 0u;
      if ((w * ITEMS + j) * kWave < cnt)  // rows past the last edge hold none
        lpos[j] = rank_row_lds(key[j], true, s_wcnt[w], tab, lane);
    }
  }
  // the keys' LDS addresses are recomputed below instead of being kept live
  // across the scans (one register per row instead of two)
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) asm volatile("" : "+v"(key[j]));
  __syncthreads();
  // One vertex per thread (FW <= NT): the waves' counts stay in registers
  // across the scan of the vertex totals, then each wave's entry becomes the
  // slot of its first edge of the vertex.
  static_assert(FW <= NT, "one vertex per thread");
  uint32_t wc[WAVES];
  if (tid < fw) {
    uint32_t t = 0;
#pragma unroll
    for (int x = 0; x < WAVES; ++x) {
      wc[x] = s_wcnt[x][tid];
      t += wc[x];
    }
    s_toff[tid] = t;
  }
  // the extra key FW sorts after every edge: its lanes (the partial row's,
  // all in one wave) land on slots cnt, cnt + 1, ..., i.e. on their own
  if (tid < WAVES) s_wcnt[tid][FW] = (uint16_t)cnt;
  __syncthreads();
  block_excl_scan<NT, uint32_t>(s_toff, fw, s_w32);
  // A whole bin: its counts are the in-degrees of its vertices, and its
  // staged order is its final CSC order, so staged slot i goes to bs + i.
  // A chunk of a big bin: slot i of vertex v goes to s_cur[v] + i.
  if (tid < fw) {
    const uint32_t off = s_toff[tid];
    uint32_t run = off;
#pragma unroll
    for (int x = 0; x < WAVES; ++x) {
      s_wcnt[x][tid] = (uint16_t)run;
      run += wc[x];
    }
    if (whole) {
      if (v0 + tid < a.n) a.T[v0 + tid] = (int64_t)(bs + off);
    } else {
      s_cur[tid] -= off;
    }
  }
  if (cnt == 0) return;
  __syncthreads();
  // The local sorted position of every edge of this thread, in batches of G
  // rows (the reads of a batch share one wait; the scheduling barrier keeps
  // the compiler from hoisting every batch's reads at once).  Rows past the
  // last edge were not ranked and are neither placed nor staged.
  constexpr int G = 4;
  const int nrows = (cnt + kWave - 1) / kWave;  // ranked rows of the item
  auto ranked = [&](int j) { return w * ITEMS + j < nrows; };
#pragma unroll
  for (int j0 = 0; j0 < ITEMS; j0 += G) {
#pragma unroll
    for (int j = j0; j < j0 + G; ++j) lpos[j] += s_wcnt[w][key[j]];
    __builtin_amdgcn_sched_barrier(0);
  }
  uint32_t vpk[(ITEMS + 1) / 2];
#pragma unroll
  for (int k = 0; k < (ITEMS + 1) / 2; ++k) vpk[k] = 0u;
  if (!whole) {
    // the vertex of every sorted slot (for its cursor)
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (ranked(j)) s_stage[lpos[j]] = key[j] & vmask;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) vpk[k >> 1] |= (s_stage[k * NT + tid] & vmask) << ((k & 1) * 16);
  }
  // Only an invalid graph has a destination v >= n (in the last bin, below
  // the next power of two).  A whole bin keeps such edges inside its own
  // slots; in a chunk of a big bin they have no cursor (T[v] does not exist)
  // and are dropped, so no write leaves [0, m).  k_hist has already flagged
  // the graph as invalid.
  const int64_t nvalid = a.n - v0;  // vertices of the bin that exist
  // staged slot k * NT + tid of every row -> out (sources, then payload)
  auto place = [&](auto *out, const uint32_t(&val)[ITEMS]) {
    using E = typename std::remove_pointer<decltype(out)>::type;
    if (whole) {
      E *ob = out + bs;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        if (k * NT + tid < cnt) ob[k * NT + tid] = (E)val[k];
    } else {
#pragma unroll
      for (int k0 = 0; k0 < ITEMS; k0 += G) {
        uint64_t c[G];
#pragma unroll
        for (int k = 0; k < G; ++k) c[k] = s_cur[(vpk[(k0 + k) >> 1] >> (((k0 + k) & 1) * 16)) & 0xFFFFu];
#pragma unroll
        for (int k = 0; k < G; ++k) {
          const int i = (k0 + k) * NT + tid;
          const uint32_t v = (vpk[(k0 + k) >> 1] >> (((k0 + k) & 1) * 16)) & 0xFFFFu;
          if (i < cnt && (int64_t)v < nvalid) out[c[k] + (uint64_t)i] = (E)val[k0 + k];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  __syncthreads();
#pragma unroll
  for (int j = 0; j < ITEMS; ++j)
    if (ranked(j)) s_stage[lpos[j]] = src[j];
  __syncthreads();
  {
    uint32_t val[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) val[k] = s_stage[k * NT + tid];
    place(a.S, val);
  }
  if (PAY) {
    const uint32_t *pin = a.in_pay + cb;
    uint32_t pay[ITEMS];
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) pay[j] = row_idx(j) < cnt ? pin[row_idx(j)] : 0u;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (ranked(j)) s_stage[lpos[j]] = pay[j];
    __syncthreads();
    uint32_t val[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) val[k] = s_stage[k * NT + tid];
    place(a.Q, val);
  }
}

}  // namespace GT_BODIES_NS
}  // namespace gt
