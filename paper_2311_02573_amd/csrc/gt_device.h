// Device helpers shared by the leaf test of the walk and the pair test of the
// exhaustive path: classification against rho and staging of candidate hits.
#pragma once
#include "gt_internal.h"

namespace gt {

// Appends up to 64 candidate hits of a wave to its LDS staging buffer and
// flushes the buffer to global memory (one atomic per flush) when it is
// nearly full or when `force` is set.  Called by the whole wave.
__device__ __forceinline__ void stage_hits(Hit* buf, int& cnt, bool have, const Hit& h,
                                           bool force, DevCounters* ctr, Hit* hits,
                                           unsigned long long hit_cap, uint32_t* band_idx,
                                           int lane) {
  const uint64_t bal = __ballot(have);
  if (have) buf[cnt + __popcll(bal & ((1ull << lane) - 1ull))] = h;
  cnt += __popcll(bal);
  if (cnt == 0 || (!force && cnt <= kHitStage - 64)) return;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(&ctr->nhits, (unsigned long long)cnt);
  base = __shfl(base, 0, 64);
  for (int i = lane; i < cnt; i += 64) {
    const Hit x = buf[i];
    const unsigned long long slot = base + i;
    if (slot < hit_cap) {
      hits[slot] = x;
      if (hit_kind(x.flag) == HIT_BAND) {
        const unsigned long long bp = atomicAdd(&ctr->nband, 1ull);
        if (bp < hit_cap) band_idx[bp] = (uint32_t)slot;
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  cnt = 0;
}

// Slot of an accepted pair among its query's results (shifted into the flag).
__device__ __forceinline__ uint32_t accept_slot(unsigned int* qcount, DevCounters* ctr) {
  const uint32_t r = atomicAdd(qcount, 1u);
  if (r >= kMaxResultsPerQuery) {
    atomicOr(&ctr->slot_over, 1u);
    return 0u;
  }
  return r << 2;
}

// Classification of a float32 cosine against rho (the float32 value is within
// 1e-6 of the canonical float64 one): accept, reject, or recheck in float64.
__device__ __forceinline__ uint32_t classify(float cs, double rho) {
  const double c64 = (double)cs;
  if (c64 >= rho + 1e-5) return HIT_ACCEPT;
  if (c64 > rho - 1e-5) return HIT_BAND;
  return 0u;
}

}  // namespace gt
