// Unordered transposition: the paper's own methods, mapped to the GPU.
//
//  Atomic GT (Algorithm 1, Section II-B): in-degrees counted with global
//  atomics, exclusive prefix sum, edges scattered through atomic cursors.
//
//  HLH / PoTra (Section IV, Algorithm 2): destinations found frequent by the
//  degree sample (Step 0: 1% of |V| edge positions) are high-degree vertices
//  (HDVs).  Their counters are private to each chunk of edges and live in
//  LDS behind a per-workgroup open-addressing table (the cache-resident
//  arrays of Section IV-A); every other destination (LDV) uses a shared
//  global counter, updated once per run of equal destinations in a wave.
//  Step 2 aggregates the per-chunk HDV counters (a column prefix over chunks)
//  and scans all in-degrees.  Step 3 re-reads each chunk with the same
//  chunk -> workgroup map as Step 1, so the HDV edges of a chunk go to a
//  private range that starts at the chunk's column prefix.
//
// Neither method orders the edges inside a CSC list: as in the paper, that
// order follows the atomics.  The offsets are exact.  Atomic GT is HLH with
// no HDVs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gt_device.hpp"
#include "gt_internal.h"
#include "gt_unordered.h"

namespace gt {

namespace {

// threads per workgroup of the count / scatter kernels: one workgroup per
// compute unit (the HDV table fills most of its LDS)
constexpr int kUNT = 1024;
constexpr int kUTile = 4096;  // edges per source-staging tile of the scatter

__device__ __forceinline__ uint32_t hdv_hash(uint32_t v, int log2slots) {
  return (v * 0x9E3779B1u) >> (32 - log2slots);
}

// Per-workgroup open-addressing table of the HDVs: key = vertex ID (-1 =
// empty), value = index of the vertex in the HDV list.  At most half of the
// slots are used, so every probe sequence ends at an empty slot.
struct HdvTable {
  int32_t *key;
  uint16_t *idx;
  int log2slots;
  uint32_t nh;

  __device__ void build(const int32_t *hdv, uint32_t count, int tid, int nt) {
    nh = count;
    const int slots = 1 << log2slots;
    for (int i = tid; i < slots; i += nt) key[i] = -1;
    __syncthreads();
    for (uint32_t h = tid; h < count; h += nt) {
      const int32_t v = hdv[h];
      uint32_t s = hdv_hash((uint32_t)v, log2slots);
      while (true) {
        if (atomicCAS(&key[s], -1, v) == -1) { idx[s] = (uint16_t)h; break; }
        s = (s + 1) & (uint32_t)(slots - 1);
      }
    }
    __syncthreads();
  }
  __device__ __forceinline__ int find(uint32_t v) const {
    if (nh == 0) return -1;
    const uint32_t mask = (1u << log2slots) - 1u;
    uint32_t s = hdv_hash(v, log2slots);
    while (true) {
      const int32_t k = key[s];
      if (k == (int32_t)v) return idx[s];
      if (k == -1) return -1;
      s = (s + 1) & mask;
    }
  }
};

// Runs of equal destinations among consecutive lanes of a wave: the lowest
// lane of a run is its head; `len` is the run length at the head.
struct Run {
  bool head;
  int head_lane;
  uint32_t len;
};
__device__ __forceinline__ Run lane_runs(uint32_t v, bool ok, int lane) {
  const uint32_t prev = __shfl_up(v, 1);
  const int prev_ok = __shfl_up((int)ok, 1);
  const bool head = ok && !(lane > 0 && prev_ok && prev == v);
  const uint64_t heads = __ballot(head);
  const uint64_t oks = __ballot(ok);
  Run r;
  r.head = head;
  const uint64_t upto = heads & ((2ull << lane) - 1ull);  // lane 63: all bits
  r.head_lane = upto ? 63 - __clzll(upto) : lane;
  // a run ends at the next head or at the next lane without an edge
  const uint64_t stops = (heads | ~oks) & ~((2ull << lane) - 1ull);
  const int next = stops ? __ffsll((unsigned long long)stops) - 1 : 64;
  r.len = (uint32_t)(next - lane);
  return r;
}

// Edge range [lo, hi) of part `part` of chunk c.  One part: the chunk (Step 1
// of the probe counts only its first `span` edges).  Several: the head, then
// the tail cut into nparts - 1 near-equal parts.
__device__ __forceinline__ void part_range(const UnorderedArgs &a, int64_t c, int part, int64_t &lo, int64_t &hi) {
  const int64_t beg = c * a.chunk;
  const int64_t end = beg + a.chunk < a.m ? beg + a.chunk : a.m;
  if (a.nparts <= 1) {
    lo = beg;
    hi = beg + a.span < end ? beg + a.span : end;
    return;
  }
  const int64_t hend = beg + a.head < end ? beg + a.head : end;
  if (part == 0) {
    lo = beg;
    hi = hend;
    return;
  }
  const int64_t tl = end - hend, nt = a.nparts - 1;
  lo = hend + tl * (part - 1) / nt;
  hi = hend + tl * part / nt;
}

// Step 1's HDV counters (Algorithm 2, the narrow private counters): a 16-bit
// low counter per HDV, two per 32-bit LDS word, updated by compare-and-swap
// so that no carry reaches the neighbouring counter.  A low counter that
// wraps adds one to the HDV's high counter of the part, `high[h]` in global
// memory (once per 65536 edges of one HDV in one part).
__device__ __forceinline__ void hdv_count16(uint32_t *low, uint32_t h, uint32_t len, uint32_t *high) {
  uint32_t *wp = low + (h >> 1);
  const int sh = (int)(h & 1u) * 16;
  uint32_t old = __hip_atomic_load(wp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  while (true) {
    const uint32_t sum = ((old >> sh) & 0xFFFFu) + len;  // len <= 64
    const uint32_t nw = (old & ~(0xFFFFu << sh)) | ((sum & 0xFFFFu) << sh);
    const uint32_t seen = atomicCAS(wp, old, nw);
    if (seen == old) {
      if (sum >> 16) atomicAdd(high + h, 1u);
      return;
    }
    old = seen;
  }
}

}  // namespace

// Step 0 (selection): histogram of sampled frequencies >= 2 (capped).
__global__ __launch_bounds__(256) void k_hdv_hist(const int32_t *keys, const uint32_t *counts, uint32_t mask,
                                                  uint32_t *hist) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > (int64_t)mask || keys[i] == -1) return;
  const uint32_t c = counts[i];
  if (c >= 2) atomicAdd(&hist[c < kHdvHistBins - 1 ? c : kHdvHistBins - 1], 1u);
}

// The smallest frequency threshold t >= 2 such that at most kmax sampled
// destinations reach it (one workgroup; sequential over the capped bins).
__global__ void k_hdv_threshold(const uint32_t *hist, int32_t kmax, uint32_t *thr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint32_t above = 0, t = kHdvHistBins;
  for (int c = kHdvHistBins - 1; c >= 2; --c) {
    if (above + hist[c] > (uint32_t)kmax) break;
    above += hist[c];
    t = (uint32_t)c;
  }
  *thr = t;
}

// The HDV list: sampled destinations whose frequency reaches the threshold.
__global__ __launch_bounds__(256) void k_hdv_compact(const int32_t *keys, const uint32_t *counts, uint32_t mask,
                                                     const uint32_t *thr, int32_t *hdv, uint32_t *nhdv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > (int64_t)mask || keys[i] == -1) return;
  const uint32_t c = counts[i], t = *thr;
  const uint32_t cc = c < kHdvHistBins - 1 ? c : kHdvHistBins - 1;
  if (c >= 2 && cc >= t) hdv[atomicAdd(nhdv, 1u)] = keys[i];
}

// Step 1: in-degrees.  Workgroup c owns edges [c*chunk, (c+1)*chunk); the
// HDV counts of every part of the chunk go to a row of their own.  During a
// part the row holds the high counters (zeroed first); at the part's end it
// receives high * 65536 + low.
__global__ __launch_bounds__(kUNT) void k_hlh_count(UnorderedArgs a) {
  __shared__ int32_t s_key[1 << kHlhLog2Slots];
  __shared__ uint16_t s_idx[1 << kHlhLog2Slots];
  __shared__ uint32_t s_low[kHlhMaxHdv / 2];  // 16-bit low counters, two per word
  const int tid = threadIdx.x, lane = tid & (kWave - 1);
  HdvTable tab{s_key, s_idx, a.log2slots, 0};
  const uint32_t nh = a.nhdv ? *a.nhdv : 0u;
  for (uint32_t i = tid; i < (nh + 1) / 2; i += kUNT) s_low[i] = 0u;
  tab.build(a.hdv, nh, tid, kUNT);
  const uint32_t un = (uint32_t)a.n;
  bool bad = false;
  for (int part = 0; part < a.nparts; ++part) {
    uint32_t *row = a.H + ((int64_t)blockIdx.x * a.nparts + part) * a.kmax;
    for (uint32_t h = tid; h < nh; h += kUNT) row[h] = 0u;  // high counters of the part
    __syncthreads();
    int64_t beg, end;
    part_range(a, blockIdx.x, part, beg, end);
    for (int64_t base = beg; base < end; base += kUNT) {
      const int64_t e = base + tid;
      const bool in = e < end;
      const uint32_t v = in ? (uint32_t)a.D[e] : 0xFFFFFFFFu;
      const bool ok = in && v < un;
      bad |= in && !ok;
      const Run r = lane_runs(v, ok, lane);
      if (r.head) {
        const int h = tab.find(v);
        if (h >= 0) hdv_count16(s_low, (uint32_t)h, r.len, row);
        else atomicAdd(&a.cnt[v], r.len);
      }
    }
    __syncthreads();
    for (uint32_t h = tid; h < nh; h += kUNT) {
      const uint32_t hi = __hip_atomic_load(row + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      row[h] = (hi << 16) + ((s_low[h >> 1] >> ((h & 1u) * 16)) & 0xFFFFu);
    }
    __syncthreads();
    for (uint32_t i = tid; i < (nh + 1) / 2; i += kUNT) s_low[i] = 0u;
  }
  if (bad) atomicOr(a.err, kErrBadIndex);
}

// Step 2, HDV part: per HDV, exclusive prefix of its per-part counts over
// the parts of all chunks, in order (in place), and its total in-degree.
__global__ __launch_bounds__(256) void k_hdv_colscan(UnorderedArgs a) {
  const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t nh = a.nhdv ? *a.nhdv : 0u;
  if (h >= nh) return;
  // B rows in flight per thread: the rows are independent loads, only the
  // running sum is sequential
  constexpr int B = 16;
  const int64_t rows = a.nchunks * a.nparts;
  uint32_t run = 0;
  for (int64_t c0 = 0; c0 < rows; c0 += B) {
    uint32_t t[B];
#pragma unroll
    for (int k = 0; k < B; ++k) t[k] = c0 + k < rows ? a.H[(c0 + k) * a.kmax + h] : 0u;
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (c0 + k < rows) {
        a.H[(c0 + k) * a.kmax + h] = run;
        run += t[k];
      }
  }
  a.cnt[a.hdv[h]] = run;
}

// Step 2: exclusive scan of the in-degrees -> T[0..n] (T[n] = m) and the
// LDV cursors (decoupled look-back over tiles of NT * ITEMS vertices).
template <int NT, int ITEMS>
__global__ __launch_bounds__(NT) void k_scan_offsets(UnorderedArgs a) {
  constexpr int TILE = NT * ITEMS;
  __shared__ uint64_t s_w[NT / kWave + 1];
  __shared__ int64_t s_tile;
  __shared__ uint64_t s_excl;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  if (tid == 0) s_tile = (int64_t)atomicAdd(a.scan_ticket, 1u);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t base = tile * TILE + (int64_t)tid * ITEMS;
  uint32_t v[ITEMS];
  uint64_t local = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    v[k] = (base + k < a.n) ? a.cnt[base + k] : 0u;
    local += v[k];
  }
  const uint64_t incl = wave_incl_sum64(local, lane);
  if (lane == kWave - 1) s_w[w] = incl;
  __syncthreads();
  if (tid == 0) {
    uint64_t run = 0;
    for (int i = 0; i < NT / kWave; ++i) { const uint64_t c = s_w[i]; s_w[i] = run; run += c; }
    s_w[NT / kWave] = run;
    s_excl = lookback_exclusive<uint64_t>(a.scan_status, tile, 1, 0, run);
  }
  __syncthreads();
  uint64_t run = s_excl + s_w[w] + incl - local;
#pragma unroll
  for (int k = 0; k < ITEMS; ++k)
    if (base + k < a.n) {
      a.T[base + k] = (int64_t)run;
      a.cur[base + k] = (unsigned long long)run;
      run += v[k];
    }
  if (tile == 0 && tid == 0) a.T[a.n] = a.m;
}

// Step 3, one part [beg, end) whose HDV ranges start at row `row` of H:
// tiles of kUTile edges whose sources are derived from the offsets in LDS.
struct ScatterLds {
  uint32_t *cur;            // [kHlhMaxHdv] HDV cursors, relative to the part's HDV range
  uint32_t *src;            // [kUTile]
  uint32_t *wmax;           // [kUNT / kWave]
  int64_t *u0;
};

__device__ void scatter_part(const UnorderedArgs &a, const HdvTable &tab, uint32_t nh, int64_t row, int64_t beg,
                             int64_t end, const ScatterLds &l) {
  constexpr int ITEMS = kUTile / kUNT;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  for (uint32_t h = tid; h < nh; h += kUNT) l.cur[h] = 0u;
  const uint32_t *hrow = a.H + row * a.kmax;  // HDV h's range of this part starts at T[hdv[h]] + hrow[h]
  if (tid == 0) {  // source of the part's first edge: the largest u with O[u] <= beg
    int64_t lo = 0, hi = a.n;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (a.O[mid] <= beg) lo = mid; else hi = mid;
    }
    *l.u0 = lo;
  }
  __syncthreads();
  const uint32_t un = (uint32_t)a.n;
  for (int64_t tb = beg; tb < end; tb += kUTile) {
    const int cnt = (int)(end - tb < kUTile ? end - tb : kUTile);
    // sources: mark the first edge of every vertex starting in the tile,
    // then fill forward with a running maximum
    const int64_t u0 = *l.u0;  // source of the tile's first edge unless a vertex starts exactly there
    for (int i = tid; i < kUTile; i += kUNT) l.src[i] = i == 0 ? (uint32_t)u0 : 0u;
    __syncthreads();
    for (int64_t u = u0 + 1 + tid; u < a.n; u += kUNT) {
      const int64_t o = a.O[u];
      if (o >= tb + cnt) break;
      if (o >= tb) atomicMax(&l.src[o - tb], (uint32_t)u);
    }
    __syncthreads();
    uint32_t carry = 0;
    for (int r = 0; r < ITEMS; ++r) {  // wave w owns rows [w*ITEMS, (w+1)*ITEMS)
      const int i = (w * ITEMS + r) * kWave + lane;
      uint32_t x = wave_incl_max(l.src[i], lane);
      x = x > carry ? x : carry;
      l.src[i] = x;
      carry = wave_last(x);
    }
    if (lane == 0) l.wmax[w] = carry;
    __syncthreads();
    uint32_t before = 0;
    for (int i = 0; i < w; ++i) before = before > l.wmax[i] ? before : l.wmax[i];
    for (int r = 0; r < ITEMS; ++r) {
      const int i = (w * ITEMS + r) * kWave + lane;
      const bool in = i < cnt;
      const uint32_t v = in ? (uint32_t)a.D[tb + i] : 0xFFFFFFFFu;
      const bool ok = in && v < un;
      uint32_t src = l.src[i];
      src = src > before ? src : before;
      const uint32_t pay = (in && a.P) ? a.P[tb + i] : 0u;
      const Run run = lane_runs(v, ok, lane);
      unsigned long long pos0 = 0;
      if (run.head) {
        const int h = tab.find(v);
        pos0 = h >= 0 ? (unsigned long long)a.T[v] + hrow[h] + atomicAdd(&l.cur[h], run.len)
                      : atomicAdd(&a.cur[v], (unsigned long long)run.len);
      }
      const unsigned long long pos = __shfl(pos0, run.head_lane) + (unsigned long long)(lane - run.head_lane);
      if (ok) {
        a.S[pos] = (int32_t)src;
        if (a.Q) a.Q[pos] = pay;
      }
    }
    __syncthreads();
    if (tid == kUNT - 1) {  // carry the source of the tile's last edge
      uint32_t last = 0;
      for (int i = 0; i < kUNT / kWave; ++i) last = last > l.wmax[i] ? last : l.wmax[i];
      *l.u0 = last;
    }
    __syncthreads();
  }
}

// Step 3: scatter, with the chunk -> workgroup map of Step 1.  Phase 1:
// workgroup c scatters the head of chunk c (the whole chunk when a chunk has
// one part).  Phase 2 (Section V-F's proposal for the load imbalance of
// Step 3): every workgroup whose head is done claims tail parts, in chunk
// order, from one atomic ticket until none is left.
__global__ __launch_bounds__(kUNT) void k_hlh_scatter(UnorderedArgs a) {
  __shared__ int32_t s_key[1 << kHlhLog2Slots];
  __shared__ uint16_t s_idx[1 << kHlhLog2Slots];
  __shared__ uint32_t s_cur[kHlhMaxHdv];
  __shared__ uint32_t s_src[kUTile];
  __shared__ uint32_t s_wmax[kUNT / kWave];
  __shared__ int64_t s_u0;
  __shared__ int64_t s_claim;
  const int tid = threadIdx.x;
  const unsigned long long t_start = a.times ? wall_clock64() : 0ull;
  HdvTable tab{s_key, s_idx, a.log2slots, 0};
  const uint32_t nh = a.nhdv ? *a.nhdv : 0u;
  tab.build(a.hdv, nh, tid, kUNT);  // ends with a barrier
  const ScatterLds l{s_cur, s_src, s_wmax, &s_u0};
  const int64_t c = blockIdx.x;
  int64_t lo, hi;
  part_range(a, c, 0, lo, hi);
  if (a.nparts <= 1) hi = c * a.chunk + a.chunk < a.m ? c * a.chunk + a.chunk : a.m;  // the whole chunk
  scatter_part(a, tab, nh, c * a.nparts, lo, hi, l);
  const unsigned long long t_head = a.times ? wall_clock64() : 0ull;
  if (a.nparts > 1) {
    const int64_t ntail = a.nchunks * (a.nparts - 1);
    while (true) {
      if (tid == 0) s_claim = (int64_t)atomicAdd(a.steal_ticket, 1u);
      __syncthreads();
      const int64_t t = s_claim;
      __syncthreads();  // every thread has the claim before the next one overwrites it
      if (t >= ntail) break;
      const int64_t cc = t / (a.nparts - 1);
      const int part = 1 + (int)(t % (a.nparts - 1));
      part_range(a, cc, part, lo, hi);
      scatter_part(a, tab, nh, cc * a.nparts + part, lo, hi, l);
    }
  }
  if (a.times && tid == 0) {
    a.times[3 * c] = t_start;
    a.times[3 * c + 1] = t_head;
    a.times[3 * c + 2] = wall_clock64();
  }
}

hipError_t launch_hdv_select(const int32_t *keys, const uint32_t *counts, uint32_t mask, int32_t kmax,
                             uint32_t *hist, uint32_t *thr, int32_t *hdv, uint32_t *nhdv, hipStream_t st) {
  const unsigned blocks = (unsigned)(((uint64_t)mask + 1 + 255) / 256);
  hipError_t e = launch_fill(hist, kHdvHistBins, 0u, st);
  if (e != hipSuccess) return e;
  if ((e = launch_fill(nhdv, 1, 0u, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_hdv_hist, dim3(blocks), dim3(256), 0, st, keys, counts, mask, hist);
  hipLaunchKernelGGL(k_hdv_threshold, dim3(1), dim3(64), 0, st, hist, kmax, thr);
  hipLaunchKernelGGL(k_hdv_compact, dim3(blocks), dim3(256), 0, st, keys, counts, mask, thr, hdv, nhdv);
  return hipGetLastError();
}

hipError_t launch_hlh_count(const UnorderedArgs &a, hipStream_t st) {
  if (a.m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hlh_count, dim3((unsigned)a.nchunks), dim3(kUNT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_hdv_colscan(const UnorderedArgs &a, hipStream_t st) {
  if (a.kmax <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hdv_colscan, dim3((unsigned)((a.kmax + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

int64_t offsets_scan_tile() { return 256 * 8; }

hipError_t launch_scan_offsets(const UnorderedArgs &a, hipStream_t st) {
  const int64_t tiles = (a.n + offsets_scan_tile() - 1) / offsets_scan_tile();
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_scan_offsets<256, 8>), dim3((unsigned)tiles), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_hlh_scatter(const UnorderedArgs &a, hipStream_t st) {
  if (a.m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hlh_scatter, dim3((unsigned)a.nchunks), dim3(kUNT), 0, st, a);
  return hipGetLastError();
}

int64_t hlh_resident_workgroups() {
  static int64_t cached = -1;
  if (cached >= 0) return cached;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_hlh_scatter, kUNT, 0) != hipSuccess)
    return 0;
  cached = (int64_t)cus * per_cu;
  return cached;
}

double hlh_clock_hz() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) !=
      hipSuccess || khz <= 0)
    return 100e6;  // the 100 MHz constant clock of this GPU family
  return 1e3 * khz;
}

}  // namespace gt
