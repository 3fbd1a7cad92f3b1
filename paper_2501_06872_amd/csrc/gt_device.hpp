// Device helpers shared by the transposition kernels (wave64, gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
// A value the compiler cannot see through: expressions computed from it are
// recomputed rather than kept live from before this point.
__device__ __forceinline__ int opaque_int(int v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

// Stable in-wave ranking of one row of keys (< 2^bits) through LDS.
// Each lane ORs its lane bit into tab[key] (a per-wave table of 64-bit lane
// masks, zero between rows), so reading tab[key] back yields the lanes holding
// the same key.  The rank is the wave's running count of the key (wcnt, read
// before the lowest such lane advances it) plus the number of lower lanes
// with the key; the lowest lane then advances the count and clears the slot.
// LDS instructions of one wave execute in order, so no barrier is needed.
// PIN: compute the rank at this point (keeps register pressure low in
// callers that rank many rows while holding other per-row state).
template <bool PIN = false>
__device__ __forceinline__ uint32_t rank_row_lds(uint32_t key, bool ok, uint16_t *wcnt,
                                                 unsigned long long *tab, int lane) {
  const unsigned long long bit = 1ull << lane, lt = bit - 1ull;
  if (ok) atomicOr(&tab[key], bit);
  __builtin_amdgcn_wave_barrier();
  const unsigned long long peers = ok ? tab[key] : 0ull;
  const uint32_t old = ok ? (uint32_t)wcnt[key] : 0u;
  __builtin_amdgcn_wave_barrier();
  if (ok && (peers & lt) == 0ull) {
    wcnt[key] = (uint16_t)(old + (uint32_t)__popcll(peers));
    tab[key] = 0ull;
  }
  __builtin_amdgcn_wave_barrier();
  uint32_t rank = old + (uint32_t)__popcll(peers & lt);
  // materialise the rank here: otherwise the compiler may defer this sum
  // past the caller's unrolled rows and keep every row's 64-bit mask live
  if (PIN) asm volatile("" : "+v"(rank));
  return rank;
}

// Inclusive running maximum across the 64 lanes with DPP moves only (no
// LDS crossbar): shifts by 1, 2, 4, 8 inside each row of 16 lanes, then the
// last lane of row 0 / row 2 into rows 1 / 3 (row_bcast:15) and the last
// lane of row 1 into rows 2 and 3 (row_bcast:31).  Lanes without a source
// read 0, the identity of an unsigned maximum.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_move(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}
__device__ __forceinline__ uint32_t umax32(uint32_t a, uint32_t b) { return a > b ? a : b; }

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v, int lane) {
  (void)lane;
  v = umax32(v, dpp_move<0x111, 0xf>(v));  // row_shr:1
  v = umax32(v, dpp_move<0x112, 0xf>(v));  // row_shr:2
  v = umax32(v, dpp_move<0x114, 0xf>(v));  // row_shr:4
  v = umax32(v, dpp_move<0x118, 0xf>(v));  // row_shr:8
  v = umax32(v, dpp_move<0x142, 0xa>(v));  // row_bcast:15 -> rows 1, 3
  v = umax32(v, dpp_move<0x143, 0xc>(v));  // row_bcast:31 -> rows 2, 3
  return v;
}

// The value of lane 63 in every lane (scalar read, no LDS crossbar).
__device__ __forceinline__ uint32_t wave_last(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

// N values below 2^16 held two per 32-bit register (indices known at
// compile time after unrolling).
template <int N>
struct Packed16 {
  uint32_t w[(N + 1) / 2];
  __device__ __forceinline__ uint32_t get(int j) const { return (w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu; }
  __device__ __forceinline__ void set(int j, uint32_t v) {
    w[j >> 1] = (j & 1) ? ((w[j >> 1] & 0xFFFFu) | (v << 16)) : ((w[j >> 1] & 0xFFFF0000u) | v);
  }
};

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t v, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ uint64_t wave_incl_sum64(uint64_t v, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint64_t t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive prefix sum of s[0..len) in LDS, in place; returns the total.
// NT threads; len <= 4 * NT.  `wsum` is scratch of NT/64 + 1 entries.
// Thread t starts by reading s[t*per .. (t+1)*per) with per = ceil(len/NT),
// entries other threads may have written: callers put a barrier between
// writing s and this call.  Ends with a barrier.
template <int NT, typename T>
__device__ T block_excl_scan(T *s, int len, T *wsum) {
  constexpr int NW = NT / kWave;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int per = (len + NT - 1) / NT;
  const int beg = tid * per;
  T local = 0;
  for (int k = 0; k < per; ++k)
    if (beg + k < len) local += s[beg + k];
  T incl = local;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  if (tid == 0) {
    T run = 0;
    for (int i = 0; i < NW; ++i) { T c = wsum[i]; wsum[i] = run; run += c; }
    wsum[NW] = run;
  }
  __syncthreads();
  T run = wsum[w] + incl - local;
  for (int k = 0; k < per; ++k)
    if (beg + k < len) { T c = s[beg + k]; s[beg + k] = run; run += c; }
  T total = wsum[NW];
  __syncthreads();
  return total;
}

// Workgroup -> work-item order that keeps runs of consecutive items on one
// XCD.  Workgroups are dispatched to the 8 XCDs round-robin by index, and
// each XCD has its own L2; items that write neighbouring pieces of one output
// region (the tiles of a partition pass, the bins of the placement kernel)
// then complete each other's partial cache lines in the same L2 before the
// lines are written back.  Blocks of `blk` consecutive items go to one XCD,
// blocks round-robin over the XCDs; the item count's tail beyond whole
// rounds keeps the identity map.  A bijection on [0, count).
#ifndef GT_XCD_BLOCK
#define GT_XCD_BLOCK 64
#endif
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_item(int64_t i, int64_t count, int64_t blk) {
  if (blk <= 1) return i;
  const int64_t round = kXcds * blk;
  if (i >= (count / round) * round) return i;
  const int64_t x = i % kXcds, j = i / kXcds;  // XCD of workgroup i, its index there
  return ((j / blk) * kXcds + x) * blk + j % blk;
}

// Status words of the decoupled look-back (Merrill & Garland 2016), one per
// (tile, column): not yet published, the tile's own aggregate, or the
// inclusive prefix through the tile.
//  64-bit: bits 63..62 flag (0 none, 1 aggregate, 2 inclusive), 61..0 count.
//  32-bit (totals below 2^31): 0 none; aggregate a stored as a + 1 (bit 31
//          clear); inclusive p stored as 2^31 | p.
template <typename W> struct Status;
template <> struct Status<uint64_t> {
  static __device__ __forceinline__ uint64_t agg(uint64_t a) { return (1ull << 62) | a; }
  static __device__ __forceinline__ uint64_t incl(uint64_t p) { return (2ull << 62) | p; }
  static __device__ __forceinline__ bool ready(uint64_t s) { return (s >> 62) != 0; }
  static __device__ __forceinline__ bool is_incl(uint64_t s) { return (s >> 62) == 2; }
  static __device__ __forceinline__ uint64_t value(uint64_t s) { return s & ((1ull << 62) - 1); }
};
template <> struct Status<uint32_t> {
  static __device__ __forceinline__ uint32_t agg(uint64_t a) { return (uint32_t)a + 1u; }
  static __device__ __forceinline__ uint32_t incl(uint64_t p) { return 0x80000000u | (uint32_t)p; }
  static __device__ __forceinline__ bool ready(uint32_t s) { return s != 0u; }
  static __device__ __forceinline__ bool is_incl(uint32_t s) { return (s >> 31) != 0u; }
  static __device__ __forceinline__ uint64_t value(uint32_t s) { return (s >> 31) ? (s & 0x7FFFFFFFu) : s - 1u; }
};

template <typename W>
__device__ __forceinline__ W status_load(const W *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename W>
__device__ __forceinline__ void status_store(W *p, W v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of this tile's `count` over all earlier tiles of the same
// column (`stride` = number of columns); publishes the aggregate, then the
// inclusive prefix.  The predecessors are read kLookWin tiles per round trip,
// starting with the immediate one (a tile publishes its inclusive prefix only
// after its own look-back, so the immediate predecessor alone rarely ends the
// walk).  Each status row a window reads is another tile's row of digit
// words, mostly held in another XCD's L2; among windows of 4, 8 and 16 tiles
// the partition passes ran fastest with 4.
constexpr int kLookWin = 4;

// First half: publish this tile's aggregate (tile 0: its inclusive prefix).
template <typename W>
__device__ __forceinline__ void lookback_publish(W *status, int64_t tile, int64_t stride, int64_t col,
                                                 uint64_t count) {
  using S = Status<W>;
  status_store(status + tile * stride + col, tile == 0 ? S::incl(count) : S::agg(count));
}

// Second half: wait for the predecessors, return the exclusive prefix and
// publish the inclusive one.
template <typename W, int WIN = kLookWin>
__device__ __forceinline__ uint64_t lookback_wait(W *status, int64_t tile, int64_t stride, int64_t col,
                                                 uint64_t count) {
  using S = Status<W>;
  if (tile == 0) return 0;
  W *mine = status + tile * stride + col;
  uint64_t excl = 0;
  int64_t t = tile - 1;
  bool done = false;
  while (!done) {
    W s[WIN];
#pragma unroll
    for (int k = 0; k < WIN; ++k) s[k] = (t - k >= 0) ? status_load(status + (t - k) * stride + col) : S::incl(0);
#pragma unroll
    for (int k = 0; k < WIN; ++k) {
      if (!done) {
        const W *p = status + (t - k) * stride + col;
        while (!S::ready(s[k])) {
          __builtin_amdgcn_s_sleep(1);
          s[k] = status_load(p);
        }
        excl += S::value(s[k]);
        if (S::is_incl(s[k])) done = true;
      }
    }
    t -= WIN;
  }
  status_store(mine, S::incl(excl + count));
  return excl;
}

template <typename W>
__device__ __forceinline__ uint64_t lookback_exclusive(W *status, int64_t tile, int64_t stride, int64_t col,
                                                      uint64_t count) {
  lookback_publish(status, tile, stride, col, count);
  return lookback_wait(status, tile, stride, col, count);
}

}  // namespace gt
