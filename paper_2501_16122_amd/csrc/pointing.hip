// Pointing build: hits, the NC x NC blocks of P^T diag(N)^-1 P (eq. (7); NC
// = 3, 2 or 1 values per pixel for the IQU, QU and I map forms), their
// 2-norm conditioning, the mask, the ascending compaction of kept pixels and
// the inverse blocks of the preconditioner; then the per-sample compact index
// and each tile's compact-index window used by the hot kernels.  Blocks and
// inverses are stored as upper triangles, row-major, NC (NC + 1) / 2 doubles
// per pixel.
#include <climits>

#pragma clang fp contract(off)

#include "mm_internal.h"
#include "sincos2.h"
#include "stokes.h"

namespace mm {
namespace {



template <class T>
__device__ T block_reduce(T v, T* sh, bool is_min) {
  // 64-wide wavefronts: reduce inside the wave, then across waves in LDS.
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_down(v, off, 64);
    v = is_min ? (o < v ? o : v) : (o > v ? o : v);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    T r = sh[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = is_min ? (sh[i] < r ? sh[i] : r) : (sh[i] > r ? sh[i] : r);
    sh[0] = r;
  }
  __syncthreads();
  T r = sh[0];
  __syncthreads();
  return r;
}

// K1: per group of kHistGroup consecutive pointing tiles, bin hits and the
// upper triangle of w a a^T (a the row of P: (1, c, s), (c, s) or (1)) of
// every sample into LDS slots over the group's pixel range, then add the
// slots to the global sums with one atomic per touched pixel; samples beyond
// the LDS window go straight to global atomics.  A group spans a few scan
// rows, so each pixel it touches is hit several times before its one flush:
// grouping four tiles cuts the global atomics of the flush about 2.6-fold
// on a 512-pixel-wide scan.  An out-of-range pixel sets flags[0] (an
// unusable angle flags[0] bit 1; the intensity form reads no angle).
constexpr int kHistThreads = 1024;
constexpr int kHistGroup = 4;    // pointing tiles per workgroup
constexpr int kHistBins = 2048;  // LDS pixel slots: 2048 * (4 + 6*8) B = 104 KiB
static_assert(kHistThreads * 4 == kTileSamples, "four samples per thread and tile");

template <class S, int NC>
__global__ __launch_bounds__(kHistThreads) void k_pointing_hist(const PtTile* __restrict__ tiles, int64_t n_tiles,
                                                                const int32_t* __restrict__ pix,
                                                                const S* __restrict__ psi,
                                                                const double* __restrict__ det_w, int32_t n_pix,
                                                                int32_t* __restrict__ hits,
                                                                double* __restrict__ blocks,
                                                                int32_t* __restrict__ flags) {
  constexpr int NB = Stokes<NC>::kBlock;
  __shared__ int32_t s_hits[kHistBins];
  __shared__ double s_acc[NB * kHistBins];
  __shared__ int32_t s_red[16];
  const int64_t g0 = (int64_t)blockIdx.x * kHistGroup;
  const int ng = n_tiles - g0 < kHistGroup ? (int)(n_tiles - g0) : kHistGroup;
  int32_t lo = INT_MAX, hi = INT_MIN;
  for (int g = 0; g < ng; ++g) {
    const PtTile tl = tiles[g0 + g];
    for (int i = threadIdx.x; i < tl.len; i += blockDim.x) {
      int32_t p = pix[tl.start + i];
      lo = p < lo ? p : lo;
      hi = p > hi ? p : hi;
    }
  }
  lo = block_reduce<int32_t>(lo, s_red, true);
  hi = block_reduce<int32_t>(hi, s_red, false);
  if (lo < 0 || hi >= n_pix) {
    if (threadIdx.x == 0) atomicOr(&flags[0], 1);
  }
  const int32_t base = lo < 0 ? 0 : lo;
  for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) {
    s_hits[i] = 0;
#pragma unroll
    for (int j = 0; j < NB; ++j) s_acc[j * kHistBins + i] = 0.0;
  }
  __syncthreads();
  for (int g = 0; g < ng; ++g) {
    const PtTile tl = tiles[g0 + g];
    const double w = det_w[tl.det];
    // kB samples per thread and tile: the pixel and angle loads are issued
    // together, unconditionally (past the tile's end from its first sample,
    // then skipped)
    constexpr int kB = 4;
    int32_t pb[kB];
    S ab[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int i = threadIdx.x + kHistThreads * u;
      const int64_t t = tl.start + (i < tl.len ? i : 0);
      pb[u] = i < tl.len ? pix[t] : -1;
      if constexpr (Stokes<NC>::kAngle) ab[u] = psi[t];
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int32_t p = pb[u];
      if (p < 0 || p >= n_pix) continue;
      double a[3] = {1.0, 0.0, 0.0};  // the row of P
      if constexpr (Stokes<NC>::kAngle) {
        if (!(fabs(2.0 * double(ab[u])) < sc::kReduceMax)) {  // also NaN / inf
          atomicOr(&flags[0], 2);
          continue;
        }
        double c, s;
        sincos2<double>(ab[u], &c, &s);
        if constexpr (NC == 3) {
          a[1] = c;
          a[2] = s;
        } else {
          a[0] = c;
          a[1] = s;
        }
      }
      double v[NB];
#pragma unroll
      for (int i = 0, j = 0; i < NC; ++i)
#pragma unroll
        for (int k = i; k < NC; ++k) v[j++] = w * a[i] * a[k];
      const int32_t rel = p - base;
      if (rel < kHistBins) {
        atomicAdd(&s_hits[rel], 1);
#pragma unroll
        for (int j = 0; j < NB; ++j) atomicAdd(&s_acc[j * kHistBins + rel], v[j]);
      } else {
        atomicAdd(&hits[p], 1);
#pragma unroll
        for (int j = 0; j < NB; ++j) atomicAdd(&blocks[NB * (int64_t)p + j], v[j]);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) {
    const int32_t h = s_hits[i];
    if (h == 0) continue;
    const int64_t p = base + i;
    atomicAdd(&hits[p], h);
#pragma unroll
    for (int j = 0; j < NB; ++j) atomicAdd(&blocks[NB * p + j], s_acc[j * kHistBins + i]);
  }
}

// Eigenvalues of a symmetric 3x3 matrix by cyclic Jacobi rotations
// (Rutishauser's stable form); the diagonal converges to the eigenvalues.
__device__ void sym3_eigvals(const double b[6], double ev[3]) {
  double a00 = b[0], a01 = b[1], a02 = b[2], a11 = b[3], a12 = b[4], a22 = b[5];
  for (int sweep = 0; sweep < 32; ++sweep) {
    const double off = fabs(a01) + fabs(a02) + fabs(a12);
    const double diag = fabs(a00) + fabs(a11) + fabs(a22);
    if (off <= 1e-300 || off <= 1e-18 * diag) break;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      // rotate in plane (p, q) = (0,1), (0,2), (1,2)
      double app, aqq, apq;
      if (r == 0) { app = a00; aqq = a11; apq = a01; }
      else if (r == 1) { app = a00; aqq = a22; apq = a02; }
      else { app = a11; aqq = a22; apq = a12; }
      if (apq == 0.0) continue;
      const double theta = (aqq - app) / (2.0 * apq);
      const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      const double napp = app - t * apq, naqq = aqq + t * apq;
      if (r == 0) {
        const double x = a02, y = a12;  // entries (0,2), (1,2)
        a02 = c * x - s * y;
        a12 = s * x + c * y;
        a00 = napp; a11 = naqq; a01 = 0.0;
      } else if (r == 1) {
        const double x = a01, y = a12;  // (0,1), (2,1)
        a01 = c * x - s * y;
        a12 = s * x + c * y;
        a00 = napp; a22 = naqq; a02 = 0.0;
      } else {
        const double x = a01, y = a02;  // (1,0), (2,0)
        a01 = c * x - s * y;
        a02 = s * x + c * y;
        a11 = napp; a22 = naqq; a12 = 0.0;
      }
    }
  }
  ev[0] = a00; ev[1] = a11; ev[2] = a22;
}

// 2-norm condition number of a block (upper triangle b): lambda_max /
// lambda_min, +inf when lambda_min <= 0 (NaN propagates and masks).
template <int NC>
__device__ __forceinline__ double block_cond(const double* b) {
  if constexpr (NC == 3) {
    double ev[3];
    sym3_eigvals(b, ev);
    const double lo = fmin(ev[0], fmin(ev[1], ev[2]));
    const double hi = fmax(ev[0], fmax(ev[1], ev[2]));
    return lo > 0.0 ? hi / lo : INFINITY;
  } else if constexpr (NC == 2) {
    // [[a, c], [c, d]]: eigenvalues m -/+ r with m the mean of the diagonal
    // and r = hypot((a - d) / 2, c); the smaller one as det / the larger
    const double a = b[0], c = b[1], d = b[2];
    const double m = 0.5 * (a + d), r = hypot(0.5 * (a - d), c);
    const double hi = m + r;
    const double lo = hi > 0.0 ? (a * d - c * c) / hi : -1.0;
    return lo > 0.0 ? hi / lo : INFINITY;
  } else {
    return b[0] > 0.0 ? 1.0 : INFINITY;
  }
}

// K2a: per pixel, the keep decision (hits >= min_hits and cond <= cond_max)
// and the per-block count of kept pixels.
constexpr int kScanBlock = 1024;  // pixels per scan block (4 per thread)

template <int NC>
__global__ __launch_bounds__(256) void k_pixel_keep(const int32_t* __restrict__ hits,
                                                    const double* __restrict__ blocks, int32_t n_pix,
                                                    int32_t min_hits, double cond_max,
                                                    uint8_t* __restrict__ mask, int32_t* __restrict__ block_counts) {
  __shared__ int32_t s_cnt[4];
  int32_t cnt = 0;
  for (int j = 0; j < 4; ++j) {
    const int64_t p = (int64_t)blockIdx.x * kScanBlock + j * 256 + threadIdx.x;
    if (p >= n_pix) continue;
    bool keep = false;
    if (hits[p] >= min_hits) {
      constexpr int NB = Stokes<NC>::kBlock;
      double b[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) b[i] = blocks[NB * p + i];
      keep = block_cond<NC>(b) <= cond_max;  // NaN -> masked
    }
    mask[p] = keep ? 0 : 1;
    cnt += keep ? 1 : 0;
  }
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) block_counts[blockIdx.x] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

// K2b: exclusive scan of the block counts (one workgroup; sequential carry
// over strides of 1024) and the total number of kept pixels.
__global__ __launch_bounds__(1024) void k_scan_counts(int32_t* __restrict__ counts, int32_t n,
                                                      int32_t* __restrict__ total) {
  __shared__ int32_t sh[1024];
  int32_t carry = 0;
  for (int base = 0; base < n; base += 1024) {
    const int i = base + threadIdx.x;
    const int32_t v = i < n ? counts[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int32_t o = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
      __syncthreads();
      sh[threadIdx.x] += o;
      __syncthreads();
    }
    if (i < n) counts[i] = carry + sh[threadIdx.x] - v;
    const int32_t blk_total = sh[1023];
    __syncthreads();
    carry += blk_total;
  }
  if (threadIdx.x == 0) *total = carry;
}

// Closed-form inverse (adjugate / determinant) of a kept block, both as
// upper triangles.
template <int NC>
__device__ __forceinline__ void block_inverse(const double* m, double* o) {
  if constexpr (NC == 3) {
    const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
    // [[a b c] [b d e] [c e f]]
    const double A = d * f - e * e, B = c * e - b * f, C = b * e - c * d;
    const double det = a * A + b * B + c * C;
    const double inv = 1.0 / det;
    o[0] = A * inv;
    o[1] = B * inv;
    o[2] = C * inv;
    o[3] = (a * f - c * c) * inv;
    o[4] = (b * c - a * e) * inv;
    o[5] = (a * d - b * b) * inv;
  } else if constexpr (NC == 2) {
    const double a = m[0], b = m[1], d = m[2];  // [[a b] [b d]]
    const double inv = 1.0 / (a * d - b * b);
    o[0] = d * inv;
    o[1] = -b * inv;
    o[2] = a * inv;
  } else {
    o[0] = 1.0 / m[0];
  }
}

// K2c: compact index of every pixel (ascending), the kept list and the
// inverse of each kept block.
template <int NC>
__global__ __launch_bounds__(256) void k_compact(const uint8_t* __restrict__ mask,
                                                 const int32_t* __restrict__ block_offsets,
                                                 const double* __restrict__ blocks, int32_t n_pix,
                                                 int32_t* __restrict__ compact, int32_t* __restrict__ kept,
                                                 double* __restrict__ minv) {
  __shared__ int32_t sh[kScanBlock];
  for (int j = 0; j < 4; ++j) {
    const int64_t p = (int64_t)blockIdx.x * kScanBlock + j * 256 + threadIdx.x;
    sh[j * 256 + threadIdx.x] = (p < n_pix && mask[p] == 0) ? 1 : 0;
  }
  __syncthreads();
  // inclusive scan over 1024 flags (Hillis-Steele, 4 per thread)
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int32_t o[4];
    for (int j = 0; j < 4; ++j) {
      const int i = j * 256 + threadIdx.x;
      o[j] = i >= off ? sh[i - off] : 0;
    }
    __syncthreads();
    for (int j = 0; j < 4; ++j) sh[j * 256 + threadIdx.x] += o[j];
    __syncthreads();
  }
  const int32_t boff = block_offsets[blockIdx.x];
  for (int j = 0; j < 4; ++j) {
    const int i = j * 256 + threadIdx.x;
    const int64_t p = (int64_t)blockIdx.x * kScanBlock + i;
    if (p >= n_pix) continue;
    if (mask[p]) {
      compact[p] = -1;
      continue;
    }
    const int32_t k = boff + sh[i] - 1;
    compact[p] = k;
    kept[k] = (int32_t)p;
    constexpr int NB = Stokes<NC>::kBlock;
    double m[NB], o[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) m[j] = blocks[NB * p + j];
    block_inverse<NC>(m, o);
#pragma unroll
    for (int j = 0; j < NB; ++j) minv[NB * (int64_t)k + j] = o[j];
  }
}

// Per-sample compact index and, per tile, the window [kmin, kmax] of the
// compact indices of its kept samples.
__global__ __launch_bounds__(256) void k_sample_index(PtTile* __restrict__ tiles, const int32_t* __restrict__ pix,
                                                      const int32_t* __restrict__ compact, int32_t n_pix,
                                                      int32_t* __restrict__ sample_k) {
  __shared__ int32_t s_red[16];
  PtTile tl = tiles[blockIdx.x];
  int32_t lo = INT_MAX, hi = -1;
  for (int i = threadIdx.x; i < tl.len; i += blockDim.x) {
    const int64_t t = tl.start + i;
    const int32_t p = pix[t];
    const int32_t k = (p >= 0 && p < n_pix) ? compact[p] : -1;
    sample_k[t] = k;
    if (k >= 0) {
      lo = k < lo ? k : lo;
      hi = k > hi ? k : hi;
    }
  }
  lo = block_reduce<int32_t>(lo, s_red, true);
  hi = block_reduce<int32_t>(hi, s_red, false);
  if (threadIdx.x == 0) {
    tiles[blockIdx.x].kmin = lo;
    tiles[blockIdx.x].kmax = hi;
  }
}

// Inverse blocks as full row-major NC x NC matrices.
template <int NC>
__global__ void k_export_minv(const double* __restrict__ minv_ut, int32_t n_kept, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_kept) return;
  constexpr int NB = Stokes<NC>::kBlock;
  const double* m = minv_ut + NB * k;
  double* o = out + NC * NC * k;
#pragma unroll
  for (int i = 0, j = 0; i < NC; ++i)
#pragma unroll
    for (int c = i; c < NC; ++c, ++j) {
      o[NC * i + c] = m[j];
      o[NC * c + i] = m[j];
    }
}

template <int NC>
int build_nc(mm_pointing_s* pt, int32_t min_hits, double cond_max, hipStream_t s) {
  const int64_t nb_scan = (pt->n_pix + kScanBlock - 1) / kScanBlock;
  MM_HIP(hipMemsetAsync(pt->hits, 0, sizeof(int32_t) * pt->n_pix, s));
  MM_HIP(hipMemsetAsync(pt->blocks, 0, sizeof(double) * Stokes<NC>::kBlock * (size_t)pt->n_pix, s));
  MM_HIP(hipMemsetAsync(pt->flags, 0, sizeof(int32_t) * 4, s));
  if (pt->n_tiles > 0) {
    const dim3 hg((unsigned)((pt->n_tiles + kHistGroup - 1) / kHistGroup));
    if (pt->dtype == MM_F64)
      hipLaunchKernelGGL((k_pointing_hist<double, NC>), hg, dim3(kHistThreads), 0, s, pt->tiles, pt->n_tiles,
                         pt->pix, static_cast<const double*>(pt->psi), pt->det_w, pt->n_pix, pt->hits, pt->blocks,
                         pt->flags);
    else
      hipLaunchKernelGGL((k_pointing_hist<float, NC>), hg, dim3(kHistThreads), 0, s, pt->tiles, pt->n_tiles,
                         pt->pix, static_cast<const float*>(pt->psi), pt->det_w, pt->n_pix, pt->hits, pt->blocks,
                         pt->flags);
    MM_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_pixel_keep<NC>, dim3(nb_scan), dim3(256), 0, s, pt->hits, pt->blocks, pt->n_pix, min_hits,
                     cond_max, pt->mask, pt->scan_tmp);
  MM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, pt->scan_tmp, (int32_t)nb_scan, &pt->flags[1]);
  MM_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_compact<NC>, dim3(nb_scan), dim3(256), 0, s, pt->mask, pt->scan_tmp, pt->blocks, pt->n_pix,
                     pt->compact, pt->kept, pt->minv);
  MM_HIP(hipGetLastError());
  if (pt->n_tiles > 0) {
    hipLaunchKernelGGL(k_sample_index, dim3(pt->n_tiles), dim3(256), 0, s, pt->tiles, pt->pix, pt->compact,
                       pt->n_pix, pt->sample_k);
    MM_HIP(hipGetLastError());
  }
  return MM_OK;
}

}  // namespace

int launch_pointing_build(mm_pointing_s* pt, int32_t min_hits, double cond_max, hipStream_t s) {
  switch (pt->ncomp) {
    case 3: return build_nc<3>(pt, min_hits, cond_max, s);
    case 2: return build_nc<2>(pt, min_hits, cond_max, s);
    case 1: return build_nc<1>(pt, min_hits, cond_max, s);
    default: return fail(MM_EINVAL, "map form must have 1, 2 or 3 values per pixel");
  }
}

int launch_export(const mm_pointing_s* pt, int32_t* hits, uint8_t* mask, int32_t* compact, int32_t* kept,
                  double* minv, hipStream_t s) {
  if (hits) MM_HIP(hipMemcpyAsync(hits, pt->hits, sizeof(int32_t) * pt->n_pix, hipMemcpyDeviceToDevice, s));
  if (mask) MM_HIP(hipMemcpyAsync(mask, pt->mask, pt->n_pix, hipMemcpyDeviceToDevice, s));
  if (compact) MM_HIP(hipMemcpyAsync(compact, pt->compact, sizeof(int32_t) * pt->n_pix, hipMemcpyDeviceToDevice, s));
  if (kept && pt->n_kept)
    MM_HIP(hipMemcpyAsync(kept, pt->kept, sizeof(int32_t) * pt->n_kept, hipMemcpyDeviceToDevice, s));
  if (minv && pt->n_kept) {
    const dim3 g((pt->n_kept + 255) / 256), b(256);
    if (pt->ncomp == 3) hipLaunchKernelGGL(k_export_minv<3>, g, b, 0, s, pt->minv, pt->n_kept, minv);
    else if (pt->ncomp == 2) hipLaunchKernelGGL(k_export_minv<2>, g, b, 0, s, pt->minv, pt->n_kept, minv);
    else hipLaunchKernelGGL(k_export_minv<1>, g, b, 0, s, pt->minv, pt->n_kept, minv);
    MM_HIP(hipGetLastError());
  }
  return MM_OK;
}

}  // namespace mm
