// Persistent batched kernel: one launch transposes every graph of a batch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gt_device.hpp"

namespace gt {
// The thread index as the persistent kernel's bodies read it: through an
// opaque move, re-read at every use.
__device__ __forceinline__ int persist_tid() {
  int v = (int)threadIdx.x;
  asm volatile("" : "+v"(v));
  return v;
}
}  // namespace gt

#define GT_BODIES_NS pb
#define GT_TID() ::gt::persist_tid()
#include "gt_bodies.hpp"

namespace gt {
using namespace pb;

// ---------------------------------------------------------------------------
// Persistent batched kernel.  Every workgroup loops: take a ticket of the
// queue, find its phase (phases are stored in ticket order; a coarse table
// brackets the search), wait until the phase it depends on (the previous
// phase of its graph) has published all its items, run the ticket's items
// (one, or a run of up to four consecutive items of a long phase) with the
// shared bodies, count them.  Outside the look-back phases a workgroup takes
// its next ticket while it runs the current one.  Tickets are taken in queue
// order, so every item a running item waits for -- a whole earlier phase, or
// an earlier tile of its own look-back chain -- belongs to a smaller ticket,
// held by a running workgroup that runs it no later than after its current
// ticket; and a workgroup publishes what it holds before it can wait on
// anything outside its current phase: the queue always drains.  A workgroup
// publishes its finished items of a phase (its stores complete, a
// device-scope release, then one atomic add) when it moves to another phase
// and when the queue is empty.
// The L2 of an XCD is not coherent with the others': the release writes this
// XCD's dirty lines back, and the first item a workgroup runs after a phase it
// depends on has completed starts with a device-scope acquire (which drops the
// clean lines of this XCD's L2 and of the CU's L1).
// ---------------------------------------------------------------------------
constexpr uint32_t kSpinLimit = 1u << 26;  // sleeps (~50 ns each) before a wait gives up

union PersistShared {
  HistShared<1, kPersistThreads> hist1;
  HistShared<2, kPersistThreads> hist2;
  ScanShared<kPersistThreads> scan;
  ReduceShared<kPersistThreads> reduce;
  DigitScanShared<kPersistThreads> dscan;
  LsdShared<8, 16, 9, false> lsd;
  LsdShared<8, 16, 9, true> lsdp;
  ScanU32Shared<kPersistThreads> scanu;
  BigCountShared<kMaxFineBits> bigc;
  BigScanShared<kPersistThreads> bigs;
  FinalShared<8, 16, kMaxFineBits> fin;
};

// The descriptor pointer is passed through an opaque scalar move in every
// case, so that the compiler cannot hoist one case's descriptor loads above
// the switch (where they would stay live across every other case).
__device__ __forceinline__ const StableLaunch &fresh(const StableLaunch *p) {
  uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)p);
  uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uintptr_t)p >> 32));
  asm volatile("" : "+s"(lo), "+s"(hi));
  return *reinterpret_cast<const StableLaunch *>(((uintptr_t)hi << 32) | lo);
}

// One partition pass tile (variant-1 tiles, 32-bit look-back words; 9-bit
// tables also run narrower digits).
template <bool CSR_IN, bool LAST, bool PACKED>
__device__ __forceinline__ void persist_lsd(const StableLaunch &L, int pass, int64_t item, PersistShared &sh) {
  auto &lds = *reinterpret_cast<LsdShared<8, 16, 9, PACKED && !CSR_IN && LAST> *>(&sh);
  if (L.pay) lsd_body<8, 16, 9, CSR_IN, true, LAST, PACKED, uint32_t>(L.lsd[pass], item, lds);
  else lsd_body<8, 16, 9, CSR_IN, false, LAST, PACKED, uint32_t>(L.lsd[pass], item, lds);
}

__device__ __forceinline__ void persist_item(const PersistPhase &P, const StableLaunch *G, int64_t item,
                                             PersistShared &sh) {
  constexpr int NT = kPersistThreads;
  switch (P.kind) {
    case kPhFill:
#pragma unroll
      for (int r = 0; r < kPersistFills; ++r)
        if (P.fill_words[r] != 0) fill_u32_body<NT>(P.fill[r], P.fill_words[r], 0u, item, P.nitems);
      break;
    case kPhValidate: {
      const StableLaunch &L = fresh(G);
      validate_offsets_body<NT>(L.O, L.n, L.m, L.err, item, P.nitems);
      break;
    }
    case kPhHist: {
      const StableLaunch &L = fresh(G);
      if (L.passes == 1)
        hist_body<1, 8192, NT>(L.D, L.m, L.n, L.h, L.ntiles, L.part, L.tcnt, L.err, item, P.nitems, sh.hist1);
      else
        hist_body<2, 8192, NT>(L.D, L.m, L.n, L.h, L.ntiles, L.part, L.tcnt, L.err, item, P.nitems, sh.hist2);
      break;
    }
    case kPhTileBsum: {
      const StableLaunch &L = fresh(G);
      tile_bsum_body<NT>(L.tcnt, L.ntiles, L.radix0, (L.ntiles + kTileBlk - 1) / kTileBlk, L.tbsum, item);
      break;
    }
    case kPhTileBscan: {
      const StableLaunch &L = fresh(G);
      tile_bscan_body<NT>(L.tbsum, (L.ntiles + kTileBlk - 1) / kTileBlk, L.dtot, item, sh.scan);
      break;
    }
    case kPhTileOff: {
      const StableLaunch &L = fresh(G);
      tile_off_body<NT>(L.tcnt, L.ntiles, L.radix0, (L.ntiles + kTileBlk - 1) / kTileBlk, L.tbsum, L.toff, item);
      break;
    }
    case kPhDigitReduce: {
      const StableLaunch &L = fresh(G);
      digit_reduce_body<NT>(L.part, L.hist_blocks, L.h, L.dtot, item, sh.reduce);
      break;
    }
    case kPhDigitScan: {
      const StableLaunch &L = fresh(G);
      digit_scan_body<NT>(L.dtot, L.h, L.digit, L.bins, L.nbins_total, L.m, L.err, (int)item, sh.dscan);
      break;
    }
    case kPhTileSrc: {
      const StableLaunch &L = fresh(G);
      tile_src_body<NT>(L.O, L.n, L.m, L.tile, L.ntiles, L.tsrc, item);
      break;
    }
    case kPhPass0: {
      const StableLaunch &L = fresh(G);
      if (L.passes == 1) persist_lsd<true, true, false>(L, 0, item, sh);
      else if (L.pk[0]) persist_lsd<true, false, true>(L, 0, item, sh);
      else persist_lsd<true, false, false>(L, 0, item, sh);
      break;
    }
    case kPhPass1: {
      const StableLaunch &L = fresh(G);
      if (L.pk[1]) persist_lsd<false, true, true>(L, 1, item, sh);
      else persist_lsd<false, true, false>(L, 1, item, sh);
      break;
    }
    case kPhBinItems: {
      const StableLaunch &L = fresh(G);
      bin_items_body<NT>(L.f.bin_start, L.f.nbins, 8 * kWave * 16, L.f.nch, L.f.T, L.n, L.m, item);
      break;
    }
    case kPhScan: {
      const StableLaunch &L = fresh(G);
      scan_u32_body<NT, 4096 / NT>(L.f.nch, L.f.item_base, L.f.nbins, L.sstatus, L.f.total_items + 1,
                                   L.f.total_items, item, sh.scanu);
      break;
    }
    case kPhItemMap: {
      const StableLaunch &L = fresh(G);
      item_map_body<NT>(L.f.nch, L.f.item_base, L.f.bin_start, L.f.nbins, 8 * kWave * 16, L.f.item_desc,
                        L.f.bigbins, L.f.nbig, L.f.hugebins, L.f.nhuge, item);
      break;
    }
    case kPhBigCount: big_count_body<8, 16, kMaxFineBits>(fresh(G).f, item, sh.bigc); break;
    case kPhBigScan: big_scan_body<NT, 16, false>(fresh(G).f, item, sh.bigs); break;
    case kPhHugeScan: big_scan_body<NT, 16, true>(fresh(G).f, item, sh.bigs); break;
    case kPhFinal: {
      const StableLaunch &L = fresh(G);
      if (L.pay) final_body<8, 16, kMaxFineBits, true>(L.f, item, sh.fin);
      else final_body<8, 16, kMaxFineBits, false>(L.f, item, sh.fin);
      break;
    }
    default: break;
  }
}

__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// Thread 0, after every thread's stores of the counted items have completed.
__device__ __forceinline__ void persist_publish(const PersistArgs &pa, int32_t phase, uint32_t count) {
  __threadfence();  // release: this XCD's dirty L2 lines reach memory before the count
  atomicAdd(&pa.done[phase], count);
}

// The phase holding ticket t: the coarse table brackets it, a binary search
// inside the bracket (usually empty) finds it.
__device__ __forceinline__ int32_t persist_phase_of(const PersistArgs &pa, int32_t nphases, unsigned long long t) {
  const uint64_t b = t >> kPersistTabShift;
  int32_t lo = (int32_t)pa.tab[b], hi = (int32_t)pa.tab[b + 1] + 1;
  if (hi > nphases) hi = nphases;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (pa.phases[mid].start <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// 2 workgroups of 8 waves per CU: the bodies fit 128 VGPRs without spilling
__global__ __launch_bounds__(kPersistThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_persistent(
    PersistArgs pa) {
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  PersistShared &sh = *reinterpret_cast<PersistShared *>(dyn_lds);
  __shared__ unsigned long long s_ticket;
  __shared__ int32_t s_phase;
  const int tid = threadIdx.x;
  const unsigned long long total = pa.meta[0];
  const int32_t nphases = (int32_t)pa.meta[1];
  // thread 0: the next ticket (taken while the current one runs), finished
  // items not yet published, and the last phase whose completion this
  // workgroup has acquired
  unsigned long long next = 0;
  bool have_next = false;
  int32_t held_phase = -1;
  uint32_t held = 0;
  uint32_t acquired = kNoDep;
  while (true) {
    if (tid == 0) {
      if (!have_next) next = atomicAdd(pa.ticket, 1ull);
      have_next = false;
      s_ticket = next;
      if (next < total) s_phase = persist_phase_of(pa, nphases, next);
    }
    __syncthreads();
    // uniform across the workgroup: read into scalar registers, so that the
    // phase and graph descriptors are read with scalar loads
    const unsigned long long t = uniform_u64(s_ticket);
    if (t >= total) break;
    const int32_t ph = __builtin_amdgcn_readfirstlane(s_phase);
    const PersistPhase &P = pa.phases[ph];
    if (tid == 0) {
      if (held != 0 && held_phase != ph) {
        persist_publish(pa, held_phase, held);
        held = 0;
      }
      if (P.dep != kNoDep && P.dep != acquired) {
        const uint32_t need = pa.phases[P.dep].nitems;
        uint32_t spins = 0;
        while (__hip_atomic_load(&pa.done[P.dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (++spins > kSpinLimit) {
            atomicOr(pa.err, kErrStall);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();  // acquire: the phase's writes before this item's reads
        acquired = P.dep;
      }
      // the next ticket, taken now: its latency hides behind this one's
      // items.  Not in a look-back phase: a tile whose ticket waits behind
      // another tile holds up every later tile of the phase.
      if (P.kind != kPhPass1 && P.kind != kPhScan) {
        next = atomicAdd(pa.ticket, 1ull);
        have_next = true;
      }
    }
    __syncthreads();
    const uint32_t chunk = P.chunk, nitems = P.nitems;
    const uint64_t first = (t - P.start) * chunk;
    const uint32_t count = (uint32_t)(first + chunk <= nitems ? chunk : nitems - first);
    for (uint32_t c = 0; c < count; ++c) {
      persist_item(P, pa.graphs + P.graph, (int64_t)(first + c), sh);
      // every thread's stores of the item complete, then no thread uses the
      // item's LDS any more
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    if (tid == 0) {
      held_phase = ph;
      held += count;
    }
  }
  if (tid == 0 && held != 0) persist_publish(pa, held_phase, held);
}

size_t persistent_lds_bytes() { return sizeof(PersistShared); }

int persistent_workgroups_per_cu() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent, kPersistThreads, sizeof(PersistShared)) !=
      hipSuccess)
    return 0;
  return per_cu;
}

hipError_t launch_persistent(const PersistArgs &a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_persistent, dim3((unsigned)grid), dim3(kPersistThreads), sizeof(PersistShared), st, a);
  return hipGetLastError();
}

}  // namespace gt
