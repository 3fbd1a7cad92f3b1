// Internal interface between the C ABI (gt_api.hip) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

constexpr int kMaxPasses = 3;
constexpr int kMaxRadix = 1024;   // digit width <= 10 bits
constexpr int kMaxFineBits = 9;   // bins of <= 512 destinations in k_final
constexpr int kHistBlocks = 1280;

// Largest edge count a plan accepts: every per-vertex prefix over the chunks
// of a big bin (k_big_scan) stays below 2^32.
constexpr int64_t kMaxEdges = int64_t(1) << 32;

// Bits of the device status word (byte 0 of the workspace).
constexpr uint32_t kErrBadIndex = 1u;
constexpr uint32_t kErrBadOffsets = 2u;
// A count that does not add up: the digit totals of a pass differ from m, or
// the per-vertex counts of a big bin from the bin's length (only a counter
// that wrapped can cause either).
constexpr uint32_t kErrOverflow = 4u;

struct HistArgs {
  int passes;
  int shift[kMaxPasses];
  int bits[kMaxPasses];
};

struct LsdArgs {
  // CSR input (first pass)
  const int64_t *O;
  const int32_t *D;
  const uint32_t *P;
  const int32_t *tile_src0;
  // [ntiles][radix] offset of each tile within each digit: the first pass,
  // and a later pass when `placed` (else it runs a look-back)
  const uint32_t *tile_off;
  int placed;
  // partitioned input (later passes)
  const int32_t *in_src;
  const uint32_t *in_key;
  const uint16_t *in_key16;  // packed input (see below)
  const uint32_t *in_pay;
  // output
  int32_t *out_src;
  uint32_t *out_key32;
  uint16_t *out_key16;
  uint32_t *out_pay;
  // digit of this pass: (key >> shift) & ((1 << bits) - 1)
  int shift, bits;
  const uint64_t *digit_start;
  void *status;        // uint32_t words when m < 2^31, else uint64_t
  uint32_t *ticket;
  int64_t m, n;
  // Packed intermediate of a two-pass plan (6 bytes per edge instead of 8):
  // the first pass writes key16 = (last digit << pk_lo) | (fine bits mod
  // 2^pk_lo) and src | (fine bits >> pk_lo) << pk_src_bits; the last pass
  // reads it back, and takes the first pass's digit of an edge from its
  // position (prev_digit_start).  pk_dshift / pk_dbits: the last digit.
  int pk_lo, pk_src_bits, pk_dshift, pk_dbits;
  const uint64_t *prev_digit_start;
  int prev_bits;
  // last pass: bin bookkeeping
  int fine_shift;    // = fine bits
  int lower_bits;    // digit bits of the earlier passes
  uint32_t fine_mask;
  uint64_t *bin_start;
};

struct FinalArgs {
  const int32_t *in_src;
  const uint16_t *in_key;
  const uint32_t *in_pay;
  const uint64_t *bin_start;
  int64_t *T;
  int32_t *S;
  uint32_t *Q;
  int64_t n, m, nbins;
  int fine_bits;
  // work items: bins longer than one tile are split into tile-sized chunks
  uint32_t *nch;          // [nbins] chunks per bin
  uint32_t *item_base;    // [nbins] first item of each bin
  // [max items] per work item: x, y = first edge (64-bit), z = bin,
  // w = edge count | 2^31 when the item is a whole bin
  uint4 *item_desc;
  uint32_t *total_items;  // device scalar
  uint32_t *cntab;        // [max items][2^fine_bits] per-chunk vertex counts -> prefixes
  uint32_t *bigbins;      // [max big bins] bins split into 2..kHugeChunks chunks
  uint32_t *nbig;         // device scalar
  uint32_t *hugebins;     // [max huge bins] bins split into more than kHugeChunks chunks
  uint32_t *nhuge;        // device scalar
  uint32_t *err;          // device status word
};

// Everything the kernels of one stable transposition need, derived from a
// plan, the graph and the workspace (built on the host; the persistent
// batched kernel reads it from device memory).
struct StableLaunch {
  const int64_t *O;
  const int32_t *D;
  int64_t n, m, ntiles, tile, nbins_total;
  int passes, radix0, hist_blocks, variant;
  bool pay, wide, validate;
  HistArgs h;
  uint32_t *err, *part, *tbsum, *toff, *sstatus;
  uint16_t *tcnt;
  uint64_t *digit, *bins, *dtot;
  int32_t *tsrc;
  uint32_t *status;  // look-back words of the passes after the first
  uint64_t status_words;
  uint32_t *ticket;
  LsdArgs lsd[kMaxPasses];
  bool pk[kMaxPasses];
  FinalArgs f;
  int64_t scan_tiles, max_items, max_big, max_huge;
};

// ---- The persistent batched kernel: one launch drains a device work queue
// of (graph, phase, item) tickets for every graph of a batch, in dependency
// order.  Phases of one stable transposition (variant-1 tiles, digits of at
// most 9 bits, one or two passes, m < 2^31), each waiting for the previous
// phase of its graph:
enum PersistKind : uint32_t {
  kPhFill, kPhValidate, kPhHist, kPhTileBsum, kPhTileBscan, kPhTileOff, kPhDigitReduce, kPhDigitScan, kPhTileSrc,
  kPhPass0, kPhPass1, kPhBinItems, kPhScan, kPhItemMap, kPhBigCount, kPhBigScan, kPhHugeScan, kPhFinal
};
constexpr int kPersistMaxPhases = 18;  // phases of one graph, at most
constexpr int kPersistFills = 4;
struct PersistPhase {
  uint32_t kind, graph, nitems;
  uint32_t dep;    // index of the phase this one waits for, or kNoDep
  uint32_t chunk;  // items per ticket (consecutive items, run in order)
  uint64_t start;  // its first ticket (phases are stored in ticket order)
  // kPhFill: word ranges to clear
  uint32_t *fill[kPersistFills];
  uint64_t fill_words[kPersistFills];
};
constexpr uint32_t kNoDep = 0xFFFFFFFFu;
struct PersistArgs {
  const StableLaunch *graphs;
  const PersistPhase *phases;
  const uint64_t *meta;  // [0] tickets in the queue, [1] phases (written by the host or by k_persist_plan)
  // tab[i]: the phase holding ticket i << kPersistTabShift (i <= total >> shift)
  const uint32_t *tab;
  unsigned long long *ticket;  // next ticket
  uint32_t *done;              // [nphases] items finished and published
  uint32_t *err;               // device status word
};
constexpr int kPersistTabShift = 4;
// A dependency wait that has not ended after this many sleeps sets this
// status bit and gives up (the output is then undefined; no wait is endless).
constexpr uint32_t kErrStall = 8u;
// threads per workgroup of the persistent kernel, and its LDS
constexpr int kPersistThreads = 512;

// ---- Planning on the device (GT_FLAG_DEVICE_PLAN): the learned choice of
// every graph stays in the workspace, and every call lays the graphs out and
// builds the persistent kernel's tables in a planning kernel.
struct DevChoice {
  int32_t fine_bits, digit_bits, variant;
  int32_t config;  // configuration index of the learned choice, -1: the heuristic's
};
struct DevGraph {
  int64_t n, m;
  const int64_t *offsets;
  const int32_t *indices;
  const uint32_t *payload;
  int64_t *out_offsets;
  int32_t *out_indices;
  uint32_t *out_payload;
  uint64_t base;  // the graph's workspace region (sized for any choice)
};
struct DevPlanArgs {
  const DevGraph *graphs;   // [count]
  const uint32_t *order;    // [count] graphs by edge count, the largest first (ties: index)
  const DevChoice *choice;  // [count]
  int32_t count;
  bool validate;
  int32_t grid;             // workgroups of the persistent launch (items per ticket)
  char *ws;
  StableLaunch *desc;       // [count]
  PersistPhase *tmp;        // [count][kPersistMaxPhases] every graph's phases
  PersistPhase *table;      // [count * kPersistMaxPhases] the queue's phases
  uint32_t *tab;            // ticket -> phase table
  uint64_t *meta;           // tickets, phases
};
constexpr int kDevPlanMaxGraphs = 4096;
hipError_t launch_gather_features(const float *const *fdev, int32_t count, float *x, hipStream_t st);
hipError_t launch_choose(const float *x, const float *y, const float *fmin, const float *fmax, int32_t count,
                         const DevChoice *heur, DevChoice *out, hipStream_t st);
hipError_t launch_persist_plan(const DevPlanArgs &a, hipStream_t st);
size_t persistent_lds_bytes();
// workgroups of the persistent kernel one CU holds at once (0 on error)
int persistent_workgroups_per_cu();
hipError_t launch_persistent(const PersistArgs &a, int grid, hipStream_t st);

// Edges per partition tile of a tile variant (waves x edges per lane x 64).
__host__ __device__ inline int64_t lsd_tile_size(int variant) {
  switch (variant) {
    case 2: return 16 * 64 * 8;
    case 3: return 8 * 64 * 8;
    case 4: return 16 * 64 * 16;
    default: return 8 * 64 * 16;
  }
}
// The tile variant that runs digits of up to max_bits bits (variants without
// an instance for that width map to variant 1).
__host__ __device__ inline int lsd_variant_for(int variant, int max_bits) {
  if (variant < 1 || variant > 4) return 1;
  if ((variant == 2 || variant == 4) && max_bits > 9) return 1;
  return variant;
}
hipError_t launch_lsd(int variant, int rbits, const LsdArgs &a, bool csr_in, bool pay, bool last, bool packed,
                      bool wide_status,
                      hipStream_t st);
// Edges per k_final work item; entries per tile of the u32 scan.
__host__ __device__ inline int64_t final_tile_size() { return 8 * 64 * 16; }
__host__ __device__ inline int64_t scan_tile_size() { return 256 * 16; }
hipError_t launch_bin_items(const FinalArgs &a, hipStream_t st);
hipError_t launch_item_map(const FinalArgs &a, hipStream_t st);
hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t len, uint32_t *status, uint32_t *ticket,
                           uint32_t *total, hipStream_t st);
hipError_t launch_big_count(const FinalArgs &a, int64_t max_items, hipStream_t st);
// bins of more chunks than this are scanned by a wider launch of k_big_scan
constexpr int kHugeChunks = 64;
hipError_t launch_big_scan(const FinalArgs &a, int64_t max_big, int64_t max_huge, hipStream_t st);
hipError_t launch_final(const FinalArgs &a, int64_t max_items, bool pay, hipStream_t st);
hipError_t launch_fill(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st);
hipError_t launch_copy_u32(uint32_t *dst, const uint32_t *src, uint64_t n, hipStream_t st);
hipError_t launch_validate_offsets(const int64_t *O, int64_t n, int64_t m, uint32_t *err, hipStream_t st);
hipError_t launch_tile_src(const int64_t *O, int64_t n, int64_t m, int64_t tile, int64_t ntiles, int32_t *out,
                           hipStream_t st);
// Step 1 in the first pass's tiles of `tile` edges (4096, 8192 or 16384):
// per-tile 16-bit counts of the first pass's digit (tilecnt[ntiles][radix])
// and per-workgroup partial histograms of the later passes.
hipError_t launch_hist(const int32_t *D, int64_t m, int64_t n, const HistArgs &h, int64_t tile, int64_t ntiles,
                       int nblocks, uint32_t *part, uint16_t *tilecnt, uint32_t *err, hipStream_t st);
// Column prefix of tilecnt -> tileoff[ntiles][radix] (uint32) and the first
// pass's digit totals (totals0[radix]); bsum holds tile_scan_blocks(ntiles)
// * radix words.
constexpr int kTileBlk = 64;  // tiles per block of the first pass's tile prefix
__host__ __device__ inline int64_t tile_scan_blocks(int64_t ntiles) { return (ntiles + kTileBlk - 1) / kTileBlk; }
hipError_t launch_tile_scan(const uint16_t *tilecnt, int64_t ntiles, int radix, uint32_t *bsum, uint64_t *totals0,
                            uint32_t *tileoff, hipStream_t st);
// Per-tile 16-bit counts (tilecnt[ntiles][radix]) of the digit (key >> shift)
// & (radix - 1) over the keys of a later pass's input (16-bit packed keys
// when key16, else 32-bit keys), in that pass's tiles of `tile` edges.
hipError_t launch_tile_hist(const void *keys, bool key16, int64_t m, int shift, int radix, int64_t tile,
                            int64_t ntiles, uint16_t *tilecnt, hipStream_t st);
hipError_t launch_digit_scan(const uint32_t *part, int nblocks, const HistArgs &h, uint64_t *totals,
                             uint64_t *digit_start, uint64_t *bin_start, int64_t nbins_total, int64_t m,
                             uint32_t *err, hipStream_t st);
// The digit starts of one pass from its totals (totals[pass][radix]).
hipError_t launch_digit_scan_pass(const uint64_t *totals, const HistArgs &h, int pass, uint64_t *digit_start,
                                  uint64_t *bin_start, int64_t nbins_total, int64_t m, uint32_t *err,
                                  hipStream_t st);

}  // namespace gt
