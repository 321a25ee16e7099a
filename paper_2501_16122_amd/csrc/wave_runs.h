// Wavefront-level segmented reduction ahead of the P^T bin atomics.
//
// Consecutive timeline samples usually fall in the same pixel, and the
// timeline-to-map kernel holds consecutive samples in consecutive lanes.
// Lanes with equal keys next to each other form a run; the run's values are
// summed across lanes (a segmented suffix sum in log2(run length) steps of
// DPP row shifts, within each row of 16 lanes) so that one lane per run
// issues the atomics, instead of every lane of the run contending for the
// same LDS address.  The fused operators keep per-lane atomics: there the
// shuffles measured slower than the contention they remove.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mm {

// v from the lane kOff places up in the same row of 16 (DPP row_shl:kOff);
// lanes whose source is past the row end get 0.
template <int kOff>
__device__ __forceinline__ double row_down(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x100 + kOff, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x100 + kOff, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

template <int NC, int kOff>
__device__ __forceinline__ bool run_step(int dist, double* v) {
  if (__builtin_amdgcn_ballot_w64(dist >= kOff) == 0) return false;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double o = row_down<kOff>(v[c]);
    v[c] += dist >= kOff ? o : 0.0;
  }
  return true;
}

// Every lane of the wavefront must call this together (no divergent exits
// before it).  key: the lane's bin key (any value for a masked sample, whose
// values are zero).  Runs are cut at the boundaries of the 16-lane rows.  On
// return, the first lane of each run holds the run's sum in v and gets true;
// the other lanes get false, and their v must not be used.  The number of
// steps is the smallest that covers the longest run of the wavefront (none
// when no two neighbours share a key): it is decided by a ballot, so the
// steps are uniform over the wavefront.
template <int NC>
__device__ __forceinline__ bool wave_run_sum(int32_t key, double* v) {
  const int lane = threadIdx.x & 63;
  const int next = __builtin_amdgcn_update_dpp(key, key, 0x101, 0xF, 0xF, false);  // row_shl:1
  const int prev = __builtin_amdgcn_update_dpp(key, key, 0x111, 0xF, 0xF, false);  // row_shr:1
  const bool row_end = (lane & 15) == 15, row_start = (lane & 15) == 0;
  const uint64_t ends = __builtin_amdgcn_ballot_w64(row_end || next != key);
  // lanes after this one in its run: bit 15 of every row of `ends` is set
  const int dist = __builtin_ctzll(ends >> lane);
  if (run_step<NC, 1>(dist, v) && run_step<NC, 2>(dist, v) && run_step<NC, 4>(dist, v)) run_step<NC, 8>(dist, v);
  return row_start || prev != key;
}

}  // namespace mm
