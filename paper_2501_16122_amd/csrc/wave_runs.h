// Wavefront-level segmented reduction ahead of the P^T bin atomics.
//
// Consecutive timeline samples usually fall in the same pixel, and the
// timeline-to-map kernel holds consecutive samples in consecutive lanes.
// Lanes with equal keys next to each other form a run; the run's values are
// summed across lanes (a segmented suffix sum in log2(run length) shuffle
// steps) so that one lane per run issues the atomics, instead of every lane
// of the run contending for the same LDS address.  The fused operators keep
// per-lane atomics: there the shuffles measured slower than the contention
// they remove.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mm {

// Every lane of the wavefront must call this together (no divergent exits
// before it).  key: the lane's bin key (any value for a masked sample, whose
// values are zero).  On return, the first lane of each run holds the run's
// sum in v and gets true; the other lanes get false, and their v must not be
// used.  The number of shuffle steps is the smallest that covers the longest
// run of the wavefront (none when no two neighbours share a key): it is
// decided by a ballot, so the loop is uniform over the wavefront.
template <int NC>
__device__ __forceinline__ bool wave_run_sum(int32_t key, double* v) {
  const int lane = threadIdx.x & 63;
  const int32_t next = __shfl_down(key, 1, 64);
  const int32_t prev = __shfl_up(key, 1, 64);
  const uint64_t ends = __builtin_amdgcn_ballot_w64(lane == 63 || next != key);
  // lanes after this one in its run: bit 63 of `ends` is always set
  const int dist = __builtin_ctzll(ends >> lane);
  for (int off = 1; off < 64; off <<= 1) {
    if (__builtin_amdgcn_ballot_w64(dist >= off) == 0) break;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double o = __shfl_down(v[c], off, 64);
      v[c] += dist >= off ? o : 0.0;
    }
  }
  return lane == 0 || prev != key;
}

}  // namespace mm
