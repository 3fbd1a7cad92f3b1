// Unordered strategies (Atomic GT, HLH): interface between the plan and the
// kernels of gt_unordered.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

// HDVs held in LDS per workgroup, sized by Eq. 1 (Section IV-A):
// k = |cache| / (|r| / alpha + d * t) with the 160 KB LDS of one compute unit
// as the cache (one workgroup per compute unit), |r| = 6 bytes per table slot
// (vertex ID + HDV index), alpha = 1/2, d = 2 bytes (16-bit low counter),
// t = 1 counter set per workgroup: 160 KB / 14 B = 11.7K, of which the
// largest power of two, 8192, is used (112 KB of Step 1's LDS; Step 3 holds
// 32-bit cursors instead, 144 KB).
constexpr int kHlhMaxHdv = 8192;
constexpr int kHlhLog2Slots = 14;   // table slots (load factor <= 1/2)
constexpr int kHdvHistBins = 4096;  // sampled frequencies, capped

struct UnorderedArgs {
  const int64_t *O;
  const int32_t *D;
  const uint32_t *P;
  int64_t n, m;
  int64_t chunk;      // edges per chunk (one workgroup each, same map in Steps 1 and 3)
  int64_t nchunks;
  int64_t span;       // edges Step 1 counts from the start of each chunk (chunk, or less in the probe)
  // Parts of a chunk (Section V-F, Step 3 in two phases): nparts == 1, the
  // whole chunk; else a head of `head` edges, which the chunk's own
  // workgroup scatters first, and nparts - 1 equal tail parts that any
  // workgroup claims from `steal_ticket` once its head is done.  Step 1
  // counts every part's HDVs separately, so each part has its own HDV ranges.
  int nparts;
  int64_t head;
  uint32_t *steal_ticket;
  unsigned long long *times;  // NULL, or [nchunks][3] wall-clock stamps of Step 3: start, head done, end
  const int32_t *hdv;     // [kmax] HDV list
  const uint32_t *nhdv;   // device scalar (NULL: no HDVs, Atomic GT)
  int32_t kmax;
  int log2slots;
  uint32_t *cnt;          // [n] in-degrees
  uint32_t *H;            // [nchunks * nparts][kmax] per-part HDV counts -> column prefixes
  int64_t *T;
  int32_t *S;
  uint32_t *Q;
  unsigned long long *cur;   // [n] LDV cursors
  uint32_t *err;
  uint64_t *scan_status;     // [scan tiles]
  uint32_t *scan_ticket;
};

hipError_t launch_hdv_select(const int32_t *keys, const uint32_t *counts, uint32_t mask, int32_t kmax,
                             uint32_t *hist, uint32_t *thr, int32_t *hdv, uint32_t *nhdv, hipStream_t st);
hipError_t launch_hlh_count(const UnorderedArgs &a, hipStream_t st);
hipError_t launch_hdv_colscan(const UnorderedArgs &a, hipStream_t st);
int64_t offsets_scan_tile();
hipError_t launch_scan_offsets(const UnorderedArgs &a, hipStream_t st);
hipError_t launch_hlh_scatter(const UnorderedArgs &a, hipStream_t st);
// Workgroups of k_hlh_scatter resident on the whole device at once (0 when
// the query fails): the chunk count of the static and two-phase Step 3.
int64_t hlh_resident_workgroups();
// Wall-clock ticks per second of the Step 3 time stamps.
double hlh_clock_hz();

}  // namespace gt
