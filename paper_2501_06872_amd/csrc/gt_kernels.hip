// Kernels of the stable CSR -> CSC transposition.
//
// The paper's three steps (Algorithm 2: count degrees, aggregate counters,
// write edges) are kept, but every counter lives in LDS and no edge ever
// touches a global atomic:
//
//  k_hist      Step 1.  One streaming read of the CSR edges; per-workgroup
//              LDS histograms of the destination digits used by the
//              partition passes (plus index validation).
//  k_digit_scan Step 2 at digit granularity: exclusive scan of the digit
//              totals -> start of every digit in the partitioned stream.
//  k_lsd       Step 3, part 1.  Stable partition of the edge stream by one
//              destination digit (least significant digit first), tile by
//              tile: coalesced loads, in-wave stable ranking through an LDS
//              table of lane masks, per-wave LDS counters, decoupled
//              look-back across tiles for the per-digit prefix (the first
//              pass takes its tiles from the end and sums the tiles behind
//              each one), LDS-staged coalesced writes.  The first pass reads
//              the CSR and derives each edge's source from the offsets of
//              the tile (marks in LDS, running maximum across lanes); the
//              last pass also records
//              where every fine vertex bin starts.  Between the two passes of
//              a two-pass plan an edge takes 6 bytes: a 16-bit key (last
//              digit, low fine bits) and the source word, whose unused top
//              bits carry the high fine bits; the last pass recovers the
//              first pass's digit of an edge from its position.
//  k_final     Step 3, part 2.  One workgroup per bin of 2^fine_bits
//              destinations (or per tile-sized chunk of a longer bin, whose
//              per-chunk counts k_big_count / k_big_scan turn into cursors):
//              per-vertex in-degrees counted in LDS, exclusive scan -> CSC
//              offsets of the bin, stable placement of the bin's edges
//              (ascending source) through LDS, coalesced write-out.
#include <hip/hip_runtime.h>
#include <stdint.h>

// the bodies, compiled with the thread index read directly
#define GT_BODIES_NS kb
#define GT_TID() ((int)threadIdx.x)
#include "gt_bodies.hpp"

namespace gt {
using namespace kb;

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) { fill_u32_body<256>(p, n, v, blockIdx.x, gridDim.x); }

__global__ void k_copy_u32(uint32_t *dst, const uint32_t *src, uint64_t n) {
  uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const uint64_t s = (uint64_t)gridDim.x * blockDim.x;
  for (; i < n; i += s) dst[i] = src[i];
}

__global__ void k_validate_offsets(const int64_t *O, int64_t n, int64_t m, uint32_t *err) {
  validate_offsets_body<256>(O, n, m, err, blockIdx.x, gridDim.x);
}

__global__ void k_tile_src(const int64_t *O, int64_t n, int64_t m, int64_t tile_size, int64_t ntiles,
                           int32_t *out) {
  tile_src_body<256>(O, n, m, tile_size, ntiles, out, blockIdx.x);
}

template <int PASSES, int TILE>
__global__ __launch_bounds__(256) void k_hist(const int32_t *__restrict__ D, int64_t m, int64_t n, HistArgs h,
                                              int64_t ntiles, uint32_t *__restrict__ part,
                                              uint16_t *__restrict__ tilecnt, uint32_t *err) {
  __shared__ HistShared<PASSES, 256> sh;
  hist_body<PASSES, TILE, 256>(D, m, n, h, ntiles, part, tilecnt, err, blockIdx.x, gridDim.x, sh);
}

__global__ __launch_bounds__(256) void k_tile_bsum(const uint16_t *__restrict__ tilecnt, int64_t ntiles, int radix,
                                                   int64_t nblk, uint32_t *__restrict__ bsum) {
  tile_bsum_body<256>(tilecnt, ntiles, radix, nblk, bsum, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_tile_bscan(uint32_t *bsum, int64_t nblk, uint64_t *totals0) {
  __shared__ ScanShared<256> sh;
  tile_bscan_body<256>(bsum, nblk, totals0, blockIdx.x, sh);
}

__global__ __launch_bounds__(256) void k_tile_off(const uint16_t *__restrict__ tilecnt, int64_t ntiles, int radix,
                                                  int64_t nblk, const uint32_t *__restrict__ bpre,
                                                  uint32_t *__restrict__ tileoff) {
  tile_off_body<256>(tilecnt, ntiles, radix, nblk, bpre, tileoff, blockIdx.x);
}

template <int TILE, typename K>
__global__ __launch_bounds__(256) void k_tile_hist(const K *__restrict__ keys, int64_t m, int shift, int radix,
                                                   uint16_t *__restrict__ tilecnt) {
  __shared__ TileHistShared<256> sh;
  tile_hist_body<256, TILE, K>(keys, m, shift, radix, tilecnt, blockIdx.x, sh);
}

__global__ __launch_bounds__(256) void k_digit_reduce(const uint32_t *__restrict__ part, int nblocks, HistArgs h,
                                                      uint64_t *totals) {
  __shared__ ReduceShared<256> sh;
  digit_reduce_body<256>(part, nblocks, h, totals, blockIdx.x, sh);
}

// workgroup i scans pass p0 + i
__global__ __launch_bounds__(1024) void k_digit_scan(const uint64_t *__restrict__ totals, HistArgs h,
                                                     uint64_t *digit_start, uint64_t *bin_start,
                                                     int64_t nbins_total, int64_t m, uint32_t *err, int p0) {
  __shared__ DigitScanShared<1024> sh;
  digit_scan_body<1024>(totals, h, digit_start, bin_start, nbins_total, m, err, p0 + (int)blockIdx.x, sh);
}

template <int WAVES, int ITEMS, int RBITS, bool CSR_IN, bool PAY, bool LAST, bool PACKED, typename SW>
__global__ __launch_bounds__(WAVES *kWave) void k_lsd(LsdArgs a) {
  __shared__ LsdShared<WAVES, ITEMS, RBITS, PACKED && !CSR_IN && LAST> sh;
  lsd_body<WAVES, ITEMS, RBITS, CSR_IN, PAY, LAST, PACKED, SW>(a, -1, sh);
}

template <int NT, int ITEMS>
__global__ __launch_bounds__(NT) void k_scan_u32(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                 int64_t len, uint32_t *status, uint32_t *ticket, uint32_t *total) {
  __shared__ ScanU32Shared<NT> sh;
  scan_u32_body<NT, ITEMS>(in, out, len, status, ticket, total, -1, sh);
}

__global__ void k_bin_items(const uint64_t *bin_start, int64_t nbins, int64_t tile, uint32_t *nch, int64_t *T,
                            int64_t n, int64_t m) {
  bin_items_body<256>(bin_start, nbins, tile, nch, T, n, m, blockIdx.x);
}

__global__ void k_item_map(const uint32_t *nch, const uint32_t *item_base, const uint64_t *bin_start,
                           int64_t nbins, int64_t tile, uint4 *item_desc, uint32_t *bigbins, uint32_t *nbig,
                           uint32_t *hugebins, uint32_t *nhuge) {
  item_map_body<256>(nch, item_base, bin_start, nbins, tile, item_desc, bigbins, nbig, hugebins, nhuge, blockIdx.x);
}

template <int WAVES, int ITEMS, int FBITS>
__global__ __launch_bounds__(WAVES *kWave) void k_big_count(FinalArgs a) {
  __shared__ BigCountShared<FBITS> sh;
  big_count_body<WAVES, ITEMS, FBITS>(a, blockIdx.x, sh);
}

template <int NT, int B, bool HUGE>
__global__ __launch_bounds__(NT) void k_big_scan(FinalArgs a) {
  __shared__ BigScanShared<NT> sh;
  big_scan_body<NT, B, HUGE>(a, blockIdx.x, sh);
}

template <int WAVES, int ITEMS, int FBITS, bool PAY>
__global__ __launch_bounds__(WAVES *kWave) void k_final(FinalArgs a) {
  __shared__ FinalShared<WAVES, ITEMS, FBITS> sh;
  // runs of consecutive items (neighbouring CSC windows) per XCD
  final_body<WAVES, ITEMS, FBITS, PAY>(a, xcd_item(blockIdx.x, gridDim.x, GT_XCD_BLOCK), sh);
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
template <int WAVES, int ITEMS, int RBITS, typename SW>
static hipError_t launch_lsd_w(const LsdArgs &a, bool csr_in, bool pay, bool last, bool pk, hipStream_t st) {
  const int64_t tile = (int64_t)WAVES * kWave * ITEMS;
  const unsigned grid = (unsigned)((a.m + tile - 1) / tile);
  const dim3 blk(WAVES * kWave);
#define GT_L(C, P, L, K) hipLaunchKernelGGL((k_lsd<WAVES, ITEMS, RBITS, C, P, L, K, SW>), dim3(grid), blk, 0, st, a)
  // the packed intermediate lies between a first pass that is not the last
  // and a last pass that is not the first
  if (pk && csr_in == last) return hipErrorInvalidValue;
  if (csr_in) {
    if (pay) { if (last) GT_L(true, true, true, false); else if (pk) GT_L(true, true, false, true); else GT_L(true, true, false, false); }
    else { if (last) GT_L(true, false, true, false); else if (pk) GT_L(true, false, false, true); else GT_L(true, false, false, false); }
  } else {
    if (pay) { if (!last) GT_L(false, true, false, false); else if (pk) GT_L(false, true, true, true); else GT_L(false, true, true, false); }
    else { if (!last) GT_L(false, false, false, false); else if (pk) GT_L(false, false, true, true); else GT_L(false, false, true, false); }
  }
#undef GT_L
  return hipGetLastError();
}

// status words: 32-bit when every prefix stays below 2^31, else 64-bit
template <int WAVES, int ITEMS, int RBITS>
static hipError_t launch_lsd_t(const LsdArgs &a, bool csr_in, bool pay, bool last, bool pk, bool wide,
                               hipStream_t st) {
  return wide ? launch_lsd_w<WAVES, ITEMS, RBITS, uint64_t>(a, csr_in, pay, last, pk, st)
              : launch_lsd_w<WAVES, ITEMS, RBITS, uint32_t>(a, csr_in, pay, last, pk, st);
}

// Every (variant, digit width) pair runs an instance whose tile is
// lsd_tile_size(variant); a pair without one is refused rather than run with
// another tile size than the plan sized its buffers for.
hipError_t launch_lsd(int variant, int rbits, const LsdArgs &a, bool csr_in, bool pay, bool last, bool pk, bool wide,
                      hipStream_t st) {
  if (a.m <= 0) return hipSuccess;
  if (rbits < 1 || rbits > 10 || lsd_variant_for(variant, rbits) != variant) return hipErrorInvalidValue;
  const int rb = rbits <= 8 ? 8 : (rbits <= 9 ? 9 : 10);
#define GT_V(W, I)                                                                       \
  return rb == 8 ? launch_lsd_t<W, I, 8>(a, csr_in, pay, last, pk, wide, st)                      \
                 : (rb == 9 ? launch_lsd_t<W, I, 9>(a, csr_in, pay, last, pk, wide, st)           \
                            : launch_lsd_t<W, I, 10>(a, csr_in, pay, last, pk, wide, st))
  switch (variant) {
    case 2:  // 16 waves x 8 edges, digits of up to 9 bits
      return rb == 8 ? launch_lsd_t<16, 8, 8>(a, csr_in, pay, last, pk, wide, st)
                     : launch_lsd_t<16, 8, 9>(a, csr_in, pay, last, pk, wide, st);
    case 3: GT_V(8, 8);
    case 4:  // 16 waves x 16 edges (16K-edge tiles), digits of up to 9 bits
      return rb == 8 ? launch_lsd_t<16, 16, 8>(a, csr_in, pay, last, pk, wide, st)
                     : launch_lsd_t<16, 16, 9>(a, csr_in, pay, last, pk, wide, st);
    default: GT_V(8, 16);
  }
#undef GT_V
}

hipError_t launch_bin_items(const FinalArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_items, dim3((unsigned)((a.nbins + 255) / 256)), dim3(256), 0, st, a.bin_start, a.nbins,
                     final_tile_size(), a.nch, a.T, a.n, a.m);
  return hipGetLastError();
}

hipError_t launch_item_map(const FinalArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_item_map, dim3((unsigned)((a.nbins + 255) / 256)), dim3(256), 0, st, a.nch, a.item_base,
                     a.bin_start, a.nbins, final_tile_size(), a.item_desc, a.bigbins, a.nbig, a.hugebins, a.nhuge);
  return hipGetLastError();
}

hipError_t launch_big_scan(const FinalArgs &a, int64_t max_big, int64_t max_huge, hipStream_t st) {
  if (max_big <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_big_scan<256, 16, false>), dim3((unsigned)max_big), dim3(256), 0, st, a);
  if (max_huge > 0) {
    constexpr int NT = 1 << kMaxFineBits;  // one thread per vertex of the widest bin
    hipLaunchKernelGGL((k_big_scan<NT, 32, true>), dim3((unsigned)max_huge), dim3(NT), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t len, uint32_t *status, uint32_t *ticket,
                           uint32_t *total, hipStream_t st) {
  const int64_t tiles = (len + scan_tile_size() - 1) / scan_tile_size();
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_scan_u32<256, 16>), dim3((unsigned)tiles), dim3(256), 0, st, in, out, len, status, ticket,
                     total);
  return hipGetLastError();
}

hipError_t launch_big_count(const FinalArgs &a, int64_t max_items, hipStream_t st) {
  if (max_items <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_big_count<8, 16, kMaxFineBits>), dim3((unsigned)max_items), dim3(8 * kWave), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_final(const FinalArgs &a, int64_t max_items, bool pay, hipStream_t st) {
  if (max_items <= 0) return hipSuccess;
  const dim3 grid((unsigned)max_items), blk(8 * kWave);
  if (pay) hipLaunchKernelGGL((k_final<8, 16, kMaxFineBits, true>), grid, blk, 0, st, a);
  else hipLaunchKernelGGL((k_final<8, 16, kMaxFineBits, false>), grid, blk, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_copy_u32, dim3((unsigned)blocks), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_validate_offsets(const int64_t *O, int64_t n, int64_t m, uint32_t *err, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_validate_offsets, dim3((unsigned)blocks), dim3(256), 0, st, O, n, m, err);
  return hipGetLastError();
}

hipError_t launch_tile_src(const int64_t *O, int64_t n, int64_t m, int64_t tile, int64_t ntiles, int32_t *out,
                           hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_src, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), 0, st, O, n, m, tile, ntiles,
                     out);
  return hipGetLastError();
}

template <int TILE>
static void launch_hist_t(const int32_t *D, int64_t m, int64_t n, const HistArgs &h, int64_t ntiles, int nblocks,
                          uint32_t *part, uint16_t *tilecnt, uint32_t *err, hipStream_t st) {
  switch (h.passes) {
    case 1: hipLaunchKernelGGL((k_hist<1, TILE>), dim3(nblocks), dim3(256), 0, st, D, m, n, h, ntiles, part, tilecnt,
                               err); break;
    case 2: hipLaunchKernelGGL((k_hist<2, TILE>), dim3(nblocks), dim3(256), 0, st, D, m, n, h, ntiles, part, tilecnt,
                               err); break;
    default: hipLaunchKernelGGL((k_hist<3, TILE>), dim3(nblocks), dim3(256), 0, st, D, m, n, h, ntiles, part,
                                tilecnt, err); break;
  }
}

hipError_t launch_hist(const int32_t *D, int64_t m, int64_t n, const HistArgs &h, int64_t tile, int64_t ntiles,
                       int nblocks, uint32_t *part, uint16_t *tilecnt, uint32_t *err, hipStream_t st) {
  if (ntiles <= 0 || nblocks <= 0) return hipSuccess;
  switch (tile) {
    case 4096: launch_hist_t<4096>(D, m, n, h, ntiles, nblocks, part, tilecnt, err, st); break;
    case 8192: launch_hist_t<8192>(D, m, n, h, ntiles, nblocks, part, tilecnt, err, st); break;
    case 16384: launch_hist_t<16384>(D, m, n, h, ntiles, nblocks, part, tilecnt, err, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tile_scan(const uint16_t *tilecnt, int64_t ntiles, int radix, uint32_t *bsum, uint64_t *totals0,
                            uint32_t *tileoff, hipStream_t st) {
  const int64_t nblk = tile_scan_blocks(ntiles);
  if (nblk <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_bsum, dim3((unsigned)nblk), dim3(256), 0, st, tilecnt, ntiles, radix, nblk, bsum);
  hipLaunchKernelGGL(k_tile_bscan, dim3((unsigned)radix), dim3(256), 0, st, bsum, nblk, totals0);
  hipLaunchKernelGGL(k_tile_off, dim3((unsigned)nblk), dim3(256), 0, st, tilecnt, ntiles, radix, nblk, bsum, tileoff);
  return hipGetLastError();
}

template <typename K>
static hipError_t launch_tile_hist_k(const K *keys, int64_t m, int shift, int radix, int64_t tile, int64_t ntiles,
                                     uint16_t *tilecnt, hipStream_t st) {
  const dim3 grid((unsigned)ntiles), blk(256);
  switch (tile) {
    case 4096: hipLaunchKernelGGL((k_tile_hist<4096, K>), grid, blk, 0, st, keys, m, shift, radix, tilecnt); break;
    case 8192: hipLaunchKernelGGL((k_tile_hist<8192, K>), grid, blk, 0, st, keys, m, shift, radix, tilecnt); break;
    case 16384: hipLaunchKernelGGL((k_tile_hist<16384, K>), grid, blk, 0, st, keys, m, shift, radix, tilecnt); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_tile_hist(const void *keys, bool key16, int64_t m, int shift, int radix, int64_t tile,
                            int64_t ntiles, uint16_t *tilecnt, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  if (radix < 1 || radix > kMaxRadix || ntiles != (m + tile - 1) / tile) return hipErrorInvalidValue;
  return key16 ? launch_tile_hist_k(static_cast<const uint16_t *>(keys), m, shift, radix, tile, ntiles, tilecnt, st)
               : launch_tile_hist_k(static_cast<const uint32_t *>(keys), m, shift, radix, tile, ntiles, tilecnt, st);
}

hipError_t launch_digit_scan(const uint32_t *part, int nblocks, const HistArgs &h, uint64_t *totals,
                             uint64_t *digit_start, uint64_t *bin_start, int64_t nbins_total, int64_t m,
                             uint32_t *err, hipStream_t st) {
  hipLaunchKernelGGL(k_digit_reduce, dim3(h.passes * (kMaxRadix / 64)), dim3(256), 0, st, part, nblocks, h, totals);
  hipLaunchKernelGGL(k_digit_scan, dim3(h.passes), dim3(1024), 0, st, totals, h, digit_start, bin_start,
                     nbins_total, m, err, 0);
  return hipGetLastError();
}

hipError_t launch_digit_scan_pass(const uint64_t *totals, const HistArgs &h, int pass, uint64_t *digit_start,
                                  uint64_t *bin_start, int64_t nbins_total, int64_t m, uint32_t *err,
                                  hipStream_t st) {
  if (pass < 0 || pass >= h.passes) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_digit_scan, dim3(1), dim3(1024), 0, st, totals, h, digit_start, bin_start, nbins_total, m,
                     err, pass);
  return hipGetLastError();
}

}  // namespace gt
