// Template-filtered white weights: a general W of eq. (4) built from the
// filtering templates of Sec. IV.  On each interval of one detector the
// white weight w = 1/sigma_d^2 is applied after the polynomial baselines of
// degree < K are projected out:
//     W y = w (y - Pi y),   Pi = T (T^T T)^-1 T^T,
// with T the polynomials of degree < K in the sample position.  Pi does not
// depend on the basis; here it is the discrete orthogonal (Gram) polynomial
// basis of the interval's n equispaced positions, for which T^T T is
// diagonal with closed-form entries, so Pi y = sum_j (<p_j, y> / h_j) p_j.
//
// One workgroup per interval and right-hand side, in two passes over the
// interval's samples: (1) the K projections <p_j, y> (FP64 sums, reduced in
// the workgroup), (2) the filtered, weighted z = w (y - Pi y), either
// written as a timeline or scattered by P^T through LDS bins per batch of
// 2048 samples (as the white fused operator does).  With y = P x the gather
// is recomputed in the second pass instead of storing the timeline.
#include <algorithm>
#include <climits>

#include "fft_lds.h"
#include "mm_internal.h"
#include "sincos2.h"
#include "stokes.h"

namespace mm {
namespace {

constexpr int kTplThreads = 256;
constexpr int kTplJ = 8;                          // samples per thread per batch
constexpr int kTplSub = kTplJ * kTplThreads;      // samples per batch (and binning sub-tile)
constexpr int kTplBins = 2048;                    // LDS bins per pass (NC doubles each)

// Gram polynomials on the positions i = 0 .. n-1 of an interval, scaled to
// O(1): with v = (2 i - n + 1) / n,
//   p_0 = 1,  p_1 = v,  p_{k+1} = ((2k+1) v p_k - k (1 - k^2/n^2) p_{k-1}) / (k+1),
// orthogonal over the n positions with sum_i p_k(i)^2 = n prod_{j<=k} (1 - j^2/n^2) / (2k+1).
struct Gram {
  double beta[kMaxTplOrder];  // k (1 - k^2/n^2) / (k+1)
  double inv_n;
  int order;                  // effective order min(K, n)

  __device__ void init(int64_t n, int k_req) {
    order = (int64_t)k_req < n ? k_req : (int)n;
    inv_n = 1.0 / (double)n;
#pragma unroll
    for (int k = 0; k < kMaxTplOrder; ++k) {
      const double kk = (double)k * inv_n;
      beta[k] = (double)k * (1.0 - kk * kk) / (double)(k + 1);
    }
  }
  __device__ double norm(int64_t n, int k) const {
    double h = (double)n;
    for (int j = 1; j <= k; ++j) {
      const double r = (double)j * inv_n;
      h *= 1.0 - r * r;
    }
    return h / (double)(2 * k + 1);
  }
  // p_0 .. p_{order-1} at position i (entries past the order are unused)
  __device__ __forceinline__ void eval(int64_t i, double* p) const {
    const double v = (double)(2 * i + 1) * inv_n - 1.0;
    p[0] = 1.0;
#pragma unroll
    for (int k = 1; k < kMaxTplOrder; ++k) {
      if (k >= order) p[k] = 0.0;  // uniform over the workgroup
      else if (k == 1) p[1] = v;
      else p[k] = ((double)(2 * k - 1) / (double)k) * v * p[k - 1] - beta[k - 1] * p[k - 2];
    }
  }
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_minmax(T v, bool is_min) {
  for (int off = 32; off > 0; off >>= 1) {
    const T o = __shfl_down(v, off, 64);
    v = is_min ? (o < v ? o : v) : (o > v ? o : v);
  }
  return v;
}

// One interval, the whole workgroup (every return below is uniform over it).
// kIn: 1 = y = P x, 0 = y = tod_in.  kOut: 1 = q += P^T z, 0 = tod_out = z.
// kW: 1 = stream the stored (cos 2psi, sin 2psi) pairs instead of psi.
template <class S, class C, int NC, int kIn, int kOut, int kW>
__device__ __forceinline__ void templates_interval(
    const TplInterval& I, const PtTile* __restrict__ tiles, int64_t n_tiles, const double* __restrict__ det_w,
    const int32_t* __restrict__ sample_k, const S* __restrict__ psi, const S* __restrict__ wts,
    const double* __restrict__ x, const S* __restrict__ tin, S* __restrict__ tout, double* __restrict__ q) {
  constexpr int W = kTplThreads / 64;
  __shared__ double s_sum[kMaxTplOrder * W];
  __shared__ int32_t s_k[2 * W];
  __shared__ double s_w;
  __shared__ double bins[kOut == 1 ? NC * kTplBins : 1];
  const int64_t a = I.start, n = I.end - I.start;
  if (n <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // the detector weight: the pointing tile holding the interval's first sample
  if (tid == 0) {
    int64_t lo = 0, hi = n_tiles - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) / 2;
      if (tiles[mid].start <= a) lo = mid;
      else hi = mid - 1;
    }
    s_w = det_w[tiles[lo].det];
  }
  Gram g;
  g.init(n, I.order);
  const int K = g.order;

  // One batch: kTplJ samples per thread at interval positions i0 + tid +
  // kTplThreads j.  All index and angle loads are issued before the map
  // gathers and the arithmetic, so each thread keeps a batch of loads in
  // flight.  y = P x (0 for samples of masked pixels) or the input timeline;
  // k = the compact index (-1 = masked or past the end), (c, s) the angle
  // terms where the row needs them.
  constexpr bool kAng = Stokes<NC>::kAngle && (kIn == 1 || kOut == 1);
  auto load_batch = [&](int64_t i0, int32_t* kb, C* yb, C* cb, C* sb) {
    S ang[kTplJ];
    S tv[kTplJ];
    // loads past the end of the interval read its last sample instead (in
    // bounds, unconditional, then discarded)
#pragma unroll
    for (int j = 0; j < kTplJ; ++j) {
      const int64_t i = i0 + tid + (int64_t)kTplThreads * j;
      const bool ok = i < n;
      const int64_t t = a + (ok ? i : n - 1);
      kb[j] = -1;
      if constexpr (kIn == 1 || kOut == 1) {
        const int32_t kr = sample_k[t];
        kb[j] = ok ? kr : -1;
      }
      if constexpr (kAng && kW == 1) ang[j] = wts[t];
      if constexpr (kAng && kW == 0) ang[j] = psi[t];
      if constexpr (kIn == 0) tv[j] = tin[t];
    }
#pragma unroll
    for (int j = 0; j < kTplJ; ++j) {
      C c = C(0), sn = C(0);
      if constexpr (kAng && kW == 1) from_tangent<C, S>(ang[j], &c, &sn);
      if constexpr (kAng && kW == 0)
        if (kb[j] >= 0) sincos2<C>(ang[j], &c, &sn);
      cb[j] = c;
      sb[j] = sn;
      if constexpr (kIn == 1) {
        // masked samples read pixel 0 (the operator runs only with kept pixels) and are zeroed
        const C yv = Stokes<NC>::project(x + NC * (int64_t)(kb[j] >= 0 ? kb[j] : 0), c, sn);
        yb[j] = kb[j] >= 0 ? yv : C(0);
      } else {
        yb[j] = (i0 + tid + (int64_t)kTplThreads * j) < n ? C(tv[j]) : C(0);
      }
    }
  };

  // (1) projections onto the template polynomials
  double coef[kMaxTplOrder];
#pragma unroll
  for (int j = 0; j < kMaxTplOrder; ++j) coef[j] = 0.0;
  if (K > 0) {
    for (int64_t i0 = 0; i0 < n; i0 += kTplSub) {
      int32_t kb[kTplJ];
      C yb[kTplJ], cb[kTplJ], sb[kTplJ];
      load_batch(i0, kb, yb, cb, sb);
#pragma unroll
      for (int j = 0; j < kTplJ; ++j) {
        const int64_t i = i0 + tid + (int64_t)kTplThreads * j;
        if (i < n) {
          double p[kMaxTplOrder];
          g.eval(i, p);
          const double y = double(yb[j]);
#pragma unroll
          for (int o = 0; o < kMaxTplOrder; ++o)
            if (o < K) coef[o] += p[o] * y;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kMaxTplOrder; ++j) {
      if (j < K) {
        const double v = wave_sum(coef[j]);
        if (lane == 0) s_sum[j * W + wid] = v;
      }
    }
  }
  __syncthreads();
  const double w = s_w;
#pragma unroll
  for (int j = 0; j < kMaxTplOrder; ++j) {
    coef[j] = 0.0;
    if (j < K) {
      double v = 0.0;
      for (int u = 0; u < W; ++u) v += s_sum[j * W + u];
      coef[j] = v / g.norm(n, j);
    }
  }

  // (2) z = w (y - Pi y), written out or scattered by P^T per batch
  for (int64_t s0 = 0; s0 < n; s0 += kTplSub) {
    int32_t kv[kTplJ];
    C yb[kTplJ], cb[kTplJ], sb[kTplJ];
    load_batch(s0, kv, yb, cb, sb);
    double v[kTplJ][NC];
    int32_t kmin = INT_MAX, kmax = -1;
#pragma unroll
    for (int jj = 0; jj < kTplJ; ++jj) {
      const int64_t i = s0 + tid + (int64_t)kTplThreads * jj;
#pragma unroll
      for (int c = 0; c < NC; ++c) v[jj][c] = 0.0;
      if (i < n) {
        double base = 0.0;
        if (K > 0) {
          double p[kMaxTplOrder];
          g.eval(i, p);
#pragma unroll
          for (int o = 0; o < kMaxTplOrder; ++o)
            if (o < K) base += coef[o] * p[o];
        }
        const C z = C(w * (double(yb[jj]) - base));
        if constexpr (kOut == 0) {
          tout[a + i] = S(z);
        } else if (kv[jj] >= 0) {
          Stokes<NC>::terms(z, cb[jj], sb[jj], v[jj]);
          kmin = kv[jj] < kmin ? kv[jj] : kmin;
          kmax = kv[jj] > kmax ? kv[jj] : kmax;
        }
      }
    }
    if constexpr (kOut == 1) {
      kmin = wave_minmax<int32_t>(kmin, true);
      kmax = wave_minmax<int32_t>(kmax, false);
      __syncthreads();  // s_k and the bins are free
      if (lane == 0) {
        s_k[wid] = kmin;
        s_k[W + wid] = kmax;
      }
      __syncthreads();
      kmin = s_k[0];
      kmax = s_k[W];
      for (int u = 1; u < W; ++u) {
        kmin = s_k[u] < kmin ? s_k[u] : kmin;
        kmax = s_k[W + u] > kmax ? s_k[W + u] : kmax;
      }
      for (int32_t lo = kmin; lo <= kmax; lo += kTplBins) {
        const int nb = kmax - lo + 1 < kTplBins ? kmax - lo + 1 : kTplBins;
        for (int i = tid; i < nb; i += kTplThreads)
#pragma unroll
          for (int c = 0; c < NC; ++c) bins[c * kTplBins + i] = 0.0;
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < kTplJ; ++jj) {
          const int rel = kv[jj] - lo;
          if (kv[jj] >= 0 && rel >= 0 && rel < nb)
#pragma unroll
            for (int c = 0; c < NC; ++c) atomicAdd(&bins[c * kTplBins + rel], v[jj][c]);
        }
        __syncthreads();
        for (int i = tid; i < nb; i += kTplThreads) {
          double* qk = q + NC * (int64_t)(lo + i);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const double b = bins[c * kTplBins + i];
            if (b != 0.0) atomicAdd(qk + c, b);
          }
        }
        __syncthreads();  // the next pass clears the bins
      }
    }
  }
}

// One interval (blockIdx.x) of one right-hand side (blockIdx.y) per workgroup.
template <class S, class C, int NC, int kIn, int kOut, int kW>
__global__ __launch_bounds__(kTplThreads) void k_templates(
    const TplInterval* __restrict__ iv, const PtTile* __restrict__ tiles, int64_t n_tiles,
    const double* __restrict__ det_w, const int32_t* __restrict__ sample_k, const S* __restrict__ psi,
    const S* __restrict__ wts, const double* __restrict__ x, const S* __restrict__ tin, S* __restrict__ tout,
    double* __restrict__ q, RhsBatch rb) {
  if (rb.done != nullptr && rb.done[(int64_t)blockIdx.y * rb.done_stride]) return;
  if (x != nullptr) x += blockIdx.y * rb.vstride;
  if (q != nullptr) q += blockIdx.y * rb.vstride;
  templates_interval<S, C, NC, kIn, kOut, kW>(iv[blockIdx.x], tiles, n_tiles, det_w, sample_k, psi, wts, x, tin,
                                              tout, q);
}

// Persistent form of q += P^T W P x over the intervals of several slots
// (right-hand sides of different solves), numbered one after the other; a
// slot whose done flag is set is skipped.
template <class S, class C, int NC, int kW>
__global__ __launch_bounds__(kTplThreads) void k_templates_batch(OpBatch b) {
  const int64_t n_items = b.off[b.n];
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    int sl = 0;
    for (int k = 1; k < b.n; ++k) sl = b.off[k] <= it ? k : sl;
    const OpSlot& o = b.s[sl];
    if (o.done == nullptr || *o.done == 0)
      templates_interval<S, C, NC, 1, 1, kW>(static_cast<const TplInterval*>(o.iv)[it - b.off[sl]],
                                             static_cast<const PtTile*>(o.tiles), o.n_pt_tiles, o.det_w,
                                             o.sample_k, static_cast<const S*>(o.psi),
                                             static_cast<const S*>(o.wts), o.x, nullptr, nullptr, o.q);
    __syncthreads();  // the next item reuses the shared memory
  }
}

template <class S, class C, int NC, int kIn, int kOut, int kW>
int launch_one(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tin, void* tout,
               double* q, const RhsBatch& rb, hipStream_t s) {
  const dim3 g((unsigned)nz->n_chunks, rb.nrhs), b(kTplThreads);
  hipLaunchKernelGGL((k_templates<S, C, NC, kIn, kOut, kW>), g, b, 0, s, nz->tpl, pt->tiles, pt->n_tiles, nz->det_w,
                     pt->sample_k, (const S*)pt->psi, (const S*)pt->weights, x, (const S*)tin, (S*)tout, q,
                     rb);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

// Stored weights serve an arithmetic no finer than their storage; the
// intensity-only form and the timeline-out form use none.
template <int NC, int kIn, int kOut>
int launch_nc(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tin, void* tout,
              double* q, int arith, const RhsBatch& rb, hipStream_t s) {
  if (nz->n_chunks == 0 || pt->n_tiles == 0) return MM_OK;
  constexpr int kW1 = (NC == 1 || kOut == 0) ? 0 : 1;
  const bool w = kW1 == 1 && pt->weights != nullptr && (arith == MM_F32 || pt->dtype == MM_F64);
  if (pt->dtype == MM_F64) {
    if (arith == MM_F64)
      return w ? launch_one<double, double, NC, kIn, kOut, kW1>(pt, nz, x, tin, tout, q, rb, s)
               : launch_one<double, double, NC, kIn, kOut, 0>(pt, nz, x, tin, tout, q, rb, s);
    return w ? launch_one<double, float, NC, kIn, kOut, kW1>(pt, nz, x, tin, tout, q, rb, s)
             : launch_one<double, float, NC, kIn, kOut, 0>(pt, nz, x, tin, tout, q, rb, s);
  }
  if (arith == MM_F64) return launch_one<float, double, NC, kIn, kOut, 0>(pt, nz, x, tin, tout, q, rb, s);
  return w ? launch_one<float, float, NC, kIn, kOut, kW1>(pt, nz, x, tin, tout, q, rb, s)
           : launch_one<float, float, NC, kIn, kOut, 0>(pt, nz, x, tin, tout, q, rb, s);
}

}  // namespace

int launch_fused_templates(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tod,
                           double* q, int arith, const RhsBatch& rb, hipStream_t s) {
  if (pt->n_kept == 0) return MM_OK;  // nothing to gather or scatter (the kernel assumes a kept pixel)
  return by_ncomp(pt->ncomp, [&]<int NC>() -> int {
    if (x != nullptr) return launch_nc<NC, 1, 1>(pt, nz, x, nullptr, nullptr, q, arith, rb, s);
    return launch_nc<NC, 0, 1>(pt, nz, nullptr, tod, nullptr, q, arith, rb, s);
  });
}

int launch_ninv_templates(const mm_pointing_s* pt, const mm_noise_s* nz, const void* in, void* out, int arith,
                          hipStream_t s) {
  return launch_nc<3, 0, 0>(pt, nz, nullptr, in, out, nullptr, arith, RhsBatch{}, s);
}

int launch_templates_batch(const OpBatch& b, int dtype, int arith, bool weights, int ncomp, hipStream_t s) {
  if (b.n == 0) return MM_OK;
  const int64_t n_items = b.off[b.n];
  if (n_items == 0) return MM_OK;
  // up to three 48 KiB-LDS workgroups per CU on 256 CUs
  const dim3 g((unsigned)std::min<int64_t>(n_items, 3 * 256)), blk(kTplThreads);
  return by_ncomp(ncomp, [&]<int NC>() -> int {
    constexpr int kW1 = NC == 1 ? 0 : 1;  // the intensity-only form reads no angle
    const bool w = kW1 == 1 && weights;
    if (dtype == MM_F64) {
      if (arith == MM_F64) {
        if (w) hipLaunchKernelGGL((k_templates_batch<double, double, NC, kW1>), g, blk, 0, s, b);
        else hipLaunchKernelGGL((k_templates_batch<double, double, NC, 0>), g, blk, 0, s, b);
      } else {
        if (w) hipLaunchKernelGGL((k_templates_batch<double, float, NC, kW1>), g, blk, 0, s, b);
        else hipLaunchKernelGGL((k_templates_batch<double, float, NC, 0>), g, blk, 0, s, b);
      }
    } else {
      if (arith == MM_F64) hipLaunchKernelGGL((k_templates_batch<float, double, NC, 0>), g, blk, 0, s, b);
      else if (w) hipLaunchKernelGGL((k_templates_batch<float, float, NC, kW1>), g, blk, 0, s, b);
      else hipLaunchKernelGGL((k_templates_batch<float, float, NC, 0>), g, blk, 0, s, b);
    }
    MM_HIP(hipGetLastError());
    return MM_OK;
  });
}

}  // namespace mm
