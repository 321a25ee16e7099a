// Timeline-domain operators for the pointing matrix of eq. (2)/(8) and the
// diagonal (white) N^-1, plus the fused q = P^T diag(w) P x of eq. (6).
//
// Every kernel streams the per-sample compact index (int32) and angle psi
// (FP64 or FP32) once, coalesced (the intensity-only form reads no angle);
// the map x (NC values per pixel, interleaved) is gathered through the
// caches.  P^T accumulates each tile's samples into LDS bins over the tile's
// compact-index window (FP64 LDS atomics), then adds each touched bin to the
// global vector with one FP64 atomic per component.  NC = 3, 2, 1 values per
// pixel (I, Q, U; Q, U; I) selects the columns of the pointing row.
#include <algorithm>

#include "mm_internal.h"
#include "sincos2.h"
#include "stokes.h"
#include "wave_runs.h"

namespace mm {
namespace {

constexpr int kOpThreads = 256;
constexpr int kBinSlots = 2048;  // LDS bins per tile: up to 3 * 2048 doubles = 48 KiB

// (cos 2psi_t, sin 2psi_t) when the map form's row uses them
template <int NC, class S, class C>
__device__ __forceinline__ void angle(const S* __restrict__ psi, int64_t t, C* c, C* s) {
  if constexpr (Stokes<NC>::kAngle) {
    sincos2<C>(psi[t], c, s);
  } else {
    *c = C(0);
    *s = C(0);
  }
}

template <class S, class C, int NC>
__global__ __launch_bounds__(kOpThreads) void k_apply_P(const int32_t* __restrict__ sample_k,
                                                        const S* __restrict__ psi, const double* __restrict__ x,
                                                        S* __restrict__ tod, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    const int32_t k = sample_k[t];
    C y = C(0);
    if (k >= 0) {
      C c, s;
      angle<NC>(psi, t, &c, &s);
      y = Stokes<NC>::project(x + NC * (int64_t)k, c, s);
    }
    tod[t] = S(y);
  }
}

// Flush the tile's LDS bins into q (one atomic per nonzero component).
template <int NC>
__device__ __forceinline__ void flush_bins(const double* __restrict__ bins, int nb, int32_t kmin,
                                           double* __restrict__ q) {
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    double* qk = q + NC * (int64_t)(kmin + i);
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const double v = bins[j * kBinSlots + i];
      if (v != 0.0) atomicAdd(qk + j, v);
    }
  }
}

template <int NC>
__device__ __forceinline__ void bin_add(double* __restrict__ bins, int nb, int32_t kmin, int32_t k,
                                        const double* o, double* __restrict__ q) {
  const int32_t rel = k - kmin;
  if (rel < nb) {
#pragma unroll
    for (int j = 0; j < NC; ++j) atomicAdd(&bins[j * kBinSlots + rel], o[j]);
  } else {
    double* qk = q + NC * (int64_t)k;
#pragma unroll
    for (int j = 0; j < NC; ++j) atomicAdd(qk + j, o[j]);
  }
}

template <int NC>
__device__ __forceinline__ int zero_bins(double* bins, const PtTile& tl) {
  const int span = tl.kmax - tl.kmin + 1;
  const int nb = span < 0 ? 0 : (span < kBinSlots ? span : kBinSlots);
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
#pragma unroll
    for (int j = 0; j < NC; ++j) bins[j * kBinSlots + i] = 0.0;
  __syncthreads();
  return nb;
}

// q += P^T (w_det * tod)   (w = 1 for plain P^T)
template <class S, class C, bool kWeighted, int NC>
__global__ __launch_bounds__(kOpThreads) void k_bin_tod(const PtTile* __restrict__ tiles,
                                                        const int32_t* __restrict__ sample_k,
                                                        const S* __restrict__ psi, const S* __restrict__ tod,
                                                        const double* __restrict__ det_w, double* __restrict__ q) {
  __shared__ double bins[NC * kBinSlots];
  const PtTile tl = tiles[blockIdx.x];
  if (tl.kmax < tl.kmin) return;
  const int nb = zero_bins<NC>(bins, tl);
  const C w = kWeighted ? C(det_w[tl.det]) : C(1);
  // whole wavefronts per round (the tile length is uniform over the block),
  // so that runs of equal pixels are summed across lanes before the atomics
  for (int i0 = 0; i0 < tl.len; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    const int64_t t = tl.start + (i < tl.len ? i : 0);
    const int32_t kr = sample_k[t];
    const int32_t k = i < tl.len ? kr : -1;
    C c, s;
    angle<NC>(psi, t, &c, &s);
    const C z = w * C(tod[t]);
    double o[NC];
    Stokes<NC>::terms(z, c, s, o);
#pragma unroll
    for (int j = 0; j < NC; ++j) o[j] = k >= 0 ? o[j] : 0.0;
    const bool head = wave_run_sum<NC>(k, o);
    if (head && k >= 0) bin_add<NC>(bins, nb, tl.kmin, k, o, q);
  }
  __syncthreads();
  flush_bins<NC>(bins, nb, tl.kmin, q);
}

// q += P^T diag(w) P x over one pointing tile: each thread keeps its
// samples' weighted P^T terms (z times the row) in registers, and the tile's
// compact-index window is binned in LDS in passes of kBinSlots pixels (one
// pass unless the scan's footprint is wide).
template <class S, class C, int NC>
__device__ __forceinline__ void fused_white_tile(const PtTile& tl, const int32_t* __restrict__ sample_k,
                                                 const S* __restrict__ psi, const double* __restrict__ det_w,
                                                 const double* __restrict__ x, double* __restrict__ q) {
  constexpr int J = kTileSamples / kOpThreads;
  __shared__ double bins[NC * kBinSlots];
  if (tl.kmax < tl.kmin) return;
  const C w = C(det_w[tl.det]);
  int32_t kv[J];
  double v[J][NC];
  // index and angle loads first, all unconditional from in-bounds positions
  // (past the tile's end: its first sample), so that they stay in flight
  // together; masked samples gather the tile's first kept pixel and are dropped
  S ang[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int i = threadIdx.x + kOpThreads * j;
    const int64_t t = tl.start + (i < tl.len ? i : 0);
    const int32_t k = sample_k[t];
    kv[j] = i < tl.len ? k : -1;
    if constexpr (Stokes<NC>::kAngle) ang[j] = psi[t];
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int32_t k = kv[j];
    C c = C(0), s = C(0);
    if constexpr (Stokes<NC>::kAngle) sincos2<C>(ang[j], &c, &s);
    const C z = w * Stokes<NC>::project(x + NC * (int64_t)(k >= 0 ? k : tl.kmin), c, s);
    double o[NC];
    Stokes<NC>::terms(z, c, s, o);
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) v[j][cc] = k >= 0 ? o[cc] : 0.0;
    kv[j] = k >= 0 ? k - tl.kmin : -1;
  }
  const int span = tl.kmax - tl.kmin + 1;
  for (int lo = 0; lo < span; lo += kBinSlots) {
    const int nb = span - lo < kBinSlots ? span - lo : kBinSlots;
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
#pragma unroll
      for (int c = 0; c < NC; ++c) bins[c * kBinSlots + i] = 0.0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int rel = kv[j] - lo;
      if (kv[j] >= 0 && rel >= 0 && rel < nb)
#pragma unroll
        for (int c = 0; c < NC; ++c) atomicAdd(&bins[c * kBinSlots + rel], v[j][c]);
    }
    __syncthreads();
    flush_bins<NC>(bins, nb, tl.kmin + lo, q);
    __syncthreads();  // the next pass clears the bins
  }
}

// one tile per workgroup; blockIdx.y selects the right-hand side
template <class S, class C, int NC>
__global__ __launch_bounds__(kOpThreads) void k_fused_white(const PtTile* __restrict__ tiles,
                                                            const int32_t* __restrict__ sample_k,
                                                            const S* __restrict__ psi,
                                                            const double* __restrict__ det_w,
                                                            const double* __restrict__ x, double* __restrict__ q,
                                                            RhsBatch rb) {
  if (rb.done != nullptr && rb.done[(int64_t)blockIdx.y * rb.done_stride]) return;
  fused_white_tile<S, C, NC>(tiles[blockIdx.x], sample_k, psi, det_w, x + blockIdx.y * rb.vstride,
                             q + blockIdx.y * rb.vstride);
}

// Persistent form over the pointing tiles of several slots (right-hand sides
// of different solves), numbered one after the other; a slot whose done
// flag is set is skipped.
template <class S, class C, int NC>
__global__ __launch_bounds__(kOpThreads) void k_fused_white_batch(OpBatch b) {
  const int64_t n_items = b.off[b.n];
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    int sl = 0;
    for (int k = 1; k < b.n; ++k) sl = b.off[k] <= it ? k : sl;
    const OpSlot& o = b.s[sl];
    if (o.done == nullptr || *o.done == 0)
      fused_white_tile<S, C, NC>(static_cast<const PtTile*>(o.tiles)[it - b.off[sl]], o.sample_k,
                                 static_cast<const S*>(o.psi), o.det_w, o.x, o.q);
    __syncthreads();  // the next item reuses the LDS bins
  }
}

template <class S, class C>
__global__ __launch_bounds__(kOpThreads) void k_ninv_white(const PtTile* __restrict__ tiles,
                                                           const double* __restrict__ det_w,
                                                           const S* __restrict__ in, S* __restrict__ out) {
  const PtTile tl = tiles[blockIdx.x];
  const C w = C(det_w[tl.det]);
  for (int i = threadIdx.x; i < tl.len; i += blockDim.x) {
    const int64_t t = tl.start + i;
    out[t] = S(w * C(in[t]));
  }
}

// The stored pointing weight of every sample: u = tan psi_t (sin psi / cos
// psi in FP64, rounded to S), from which the kernels rebuild (cos 2psi_t,
// sin 2psi_t) by the half-angle substitution (from_tangent).
template <class S>
__global__ __launch_bounds__(kOpThreads) void k_weights(const S* __restrict__ psi, S* __restrict__ w, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) {
    double s, c;
    sincos_x(double(psi[t]), &s, &c);
    w[t] = S(s / c);
  }
}

// z = M r: the symmetric NC x NC inverse block (upper triangle, row-major)
// of each kept pixel times its NC values.
template <int NC>
__global__ void k_apply_M(const double* __restrict__ minv, const double* __restrict__ r, double* __restrict__ z,
                          int32_t n_kept) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_kept) return;
  const double* m = minv + Stokes<NC>::kBlock * k;
  const double* rk = r + NC * k;
  double* zk = z + NC * k;
  if constexpr (NC == 3) {
    const double r0 = rk[0], r1 = rk[1], r2 = rk[2];
    zk[0] = m[0] * r0 + m[1] * r1 + m[2] * r2;
    zk[1] = m[1] * r0 + m[3] * r1 + m[4] * r2;
    zk[2] = m[2] * r0 + m[4] * r1 + m[5] * r2;
  } else if constexpr (NC == 2) {
    const double r0 = rk[0], r1 = rk[1];
    zk[0] = m[0] * r0 + m[1] * r1;
    zk[1] = m[1] * r0 + m[2] * r1;
  } else {
    zk[0] = m[0] * rk[0];
  }
}

__global__ void k_expand(const int32_t* __restrict__ compact, const double* __restrict__ x,
                         double* __restrict__ full, int32_t n_pix, int32_t nc) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_pix) return;
  const int32_t k = compact[p];
  for (int c = 0; c < nc; ++c) full[nc * p + c] = k >= 0 ? x[nc * (int64_t)k + c] : 0.0;
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

inline int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

int launch_apply_P(const mm_pointing_s* pt, const double* x, void* tod, int arith, hipStream_t s) {
  const int64_t n = pt->n_samples;
  if (n == 0) return MM_OK;
  const dim3 g(grid_for(n, kOpThreads)), b(kOpThreads);
  return by_ncomp(pt->ncomp, [&]<int NC>() -> int {
    if (pt->dtype == MM_F64) {
      if (arith == MM_F64)
        hipLaunchKernelGGL((k_apply_P<double, double, NC>), g, b, 0, s, pt->sample_k, (const double*)pt->psi, x,
                           (double*)tod, n);
      else
        hipLaunchKernelGGL((k_apply_P<double, float, NC>), g, b, 0, s, pt->sample_k, (const double*)pt->psi, x,
                           (double*)tod, n);
    } else {
      if (arith == MM_F64)
        hipLaunchKernelGGL((k_apply_P<float, double, NC>), g, b, 0, s, pt->sample_k, (const float*)pt->psi, x,
                           (float*)tod, n);
      else
        hipLaunchKernelGGL((k_apply_P<float, float, NC>), g, b, 0, s, pt->sample_k, (const float*)pt->psi, x,
                           (float*)tod, n);
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
  });
}

template <bool kW>
static int launch_bin(const mm_pointing_s* pt, const double* det_w, const void* tod, double* q, int arith,
                      hipStream_t s) {
  if (pt->n_tiles == 0) return MM_OK;
  const dim3 g(pt->n_tiles), b(kOpThreads);
  return by_ncomp(pt->ncomp, [&]<int NC>() -> int {
    if (pt->dtype == MM_F64) {
      if (arith == MM_F64)
        hipLaunchKernelGGL((k_bin_tod<double, double, kW, NC>), g, b, 0, s, pt->tiles, pt->sample_k,
                           (const double*)pt->psi, (const double*)tod, det_w, q);
      else
        hipLaunchKernelGGL((k_bin_tod<double, float, kW, NC>), g, b, 0, s, pt->tiles, pt->sample_k,
                           (const double*)pt->psi, (const double*)tod, det_w, q);
    } else {
      if (arith == MM_F64)
        hipLaunchKernelGGL((k_bin_tod<float, double, kW, NC>), g, b, 0, s, pt->tiles, pt->sample_k,
                           (const float*)pt->psi, (const float*)tod, det_w, q);
      else
        hipLaunchKernelGGL((k_bin_tod<float, float, kW, NC>), g, b, 0, s, pt->tiles, pt->sample_k,
                           (const float*)pt->psi, (const float*)tod, det_w, q);
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
  });
}

int launch_apply_PT(const mm_pointing_s* pt, const void* tod, double* q, int arith, hipStream_t s) {
  return launch_bin<false>(pt, nullptr, tod, q, arith, s);
}

int launch_rhs_white(const mm_pointing_s* pt, const double* det_w, const void* tod, double* q, int arith,
                     hipStream_t s) {
  return launch_bin<true>(pt, det_w, tod, q, arith, s);
}

int launch_fused_white(const mm_pointing_s* pt, const double* det_w, const double* x, double* q, int arith,
                       const RhsBatch& rb, hipStream_t s) {
  if (pt->n_tiles == 0) return MM_OK;
  const dim3 g(pt->n_tiles, rb.nrhs), b(kOpThreads);
  return by_ncomp(pt->ncomp, [&]<int NC>() -> int {
    if (pt->dtype == MM_F64) {
      if (arith == MM_F64)
        hipLaunchKernelGGL((k_fused_white<double, double, NC>), g, b, 0, s, pt->tiles, pt->sample_k,
                           (const double*)pt->psi, det_w, x, q, rb);
      else
        hipLaunchKernelGGL((k_fused_white<double, float, NC>), g, b, 0, s, pt->tiles, pt->sample_k,
                           (const double*)pt->psi, det_w, x, q, rb);
    } else {
      if (arith == MM_F64)
        hipLaunchKernelGGL((k_fused_white<float, double, NC>), g, b, 0, s, pt->tiles, pt->sample_k,
                           (const float*)pt->psi, det_w, x, q, rb);
      else
        hipLaunchKernelGGL((k_fused_white<float, float, NC>), g, b, 0, s, pt->tiles, pt->sample_k,
                           (const float*)pt->psi, det_w, x, q, rb);
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
  });
}

int launch_white_batch(const OpBatch& b, int dtype, int arith, int ncomp, hipStream_t s) {
  if (b.n == 0) return MM_OK;
  const int64_t n_items = b.off[b.n];
  if (n_items == 0) return MM_OK;
  // up to three 48 KiB-LDS workgroups per CU on 256 CUs
  const dim3 g((unsigned)std::min<int64_t>(n_items, 3 * 256)), blk(kOpThreads);
  return by_ncomp(ncomp, [&]<int NC>() -> int {
    if (dtype == MM_F64) {
      if (arith == MM_F64) hipLaunchKernelGGL((k_fused_white_batch<double, double, NC>), g, blk, 0, s, b);
      else hipLaunchKernelGGL((k_fused_white_batch<double, float, NC>), g, blk, 0, s, b);
    } else {
      if (arith == MM_F64) hipLaunchKernelGGL((k_fused_white_batch<float, double, NC>), g, blk, 0, s, b);
      else hipLaunchKernelGGL((k_fused_white_batch<float, float, NC>), g, blk, 0, s, b);
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
  });
}

int launch_ninv_white(const mm_pointing_s* pt, const double* det_w, const void* in, void* out, int arith,
                      hipStream_t s) {
  if (pt->n_tiles == 0) return MM_OK;
  const dim3 g(pt->n_tiles), b(kOpThreads);
  if (pt->dtype == MM_F64) {
    if (arith == MM_F64)
      hipLaunchKernelGGL((k_ninv_white<double, double>), g, b, 0, s, pt->tiles, det_w, (const double*)in,
                         (double*)out);
    else
      hipLaunchKernelGGL((k_ninv_white<double, float>), g, b, 0, s, pt->tiles, det_w, (const double*)in,
                         (double*)out);
  } else {
    if (arith == MM_F64)
      hipLaunchKernelGGL((k_ninv_white<float, double>), g, b, 0, s, pt->tiles, det_w, (const float*)in,
                         (float*)out);
    else
      hipLaunchKernelGGL((k_ninv_white<float, float>), g, b, 0, s, pt->tiles, det_w, (const float*)in,
                         (float*)out);
  }
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_compute_weights(const mm_pointing_s* pt, void* weights, hipStream_t s) {
  const int64_t n = pt->n_samples;
  if (n == 0) return MM_OK;
  const dim3 g(grid_for(n, kOpThreads)), b(kOpThreads);
  if (pt->dtype == MM_F64)
    hipLaunchKernelGGL(k_weights<double>, g, b, 0, s, (const double*)pt->psi, (double*)weights, n);
  else
    hipLaunchKernelGGL(k_weights<float>, g, b, 0, s, (const float*)pt->psi, (float*)weights, n);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_apply_M(const mm_pointing_s* pt, const double* r, double* z, hipStream_t s) {
  if (pt->n_kept == 0) return MM_OK;
  return by_ncomp(pt->ncomp, [&]<int NC>() -> int {
    hipLaunchKernelGGL(k_apply_M<NC>, dim3((pt->n_kept + 255) / 256), dim3(256), 0, s, pt->minv, r, z, pt->n_kept);
    MM_HIP(hipGetLastError());
    return MM_OK;
  });
}

int launch_expand(const mm_pointing_s* pt, const double* x, double* full, hipStream_t s) {
  if (pt->n_pix == 0) return MM_OK;
  hipLaunchKernelGGL(k_expand, dim3((pt->n_pix + 255) / 256), dim3(256), 0, s, pt->compact, x, full, pt->n_pix,
                     pt->ncomp);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

int launch_fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n == 0) return MM_OK;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

}  // namespace mm
