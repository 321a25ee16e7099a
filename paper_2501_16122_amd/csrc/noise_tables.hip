// Tables of the band-Toeplitz noise weighting (the correlated N^-1 of
// eq. (5), one finite band section per stationary chunk): the overlap-save
// tiles of each FFT plan, the spectral weights (alpha_k, beta_k) of every
// filter, and the twiddle factors: the FP64 8192-point plan, the 16384-point
// plan (FP32 tables, and FP64 ones for FP64 arithmetic's longer plan), and
// the 32768-point FP32 plan.
//
// The symbol of the symmetric band filter at the L frequencies of a plan,
//   H_k = c_0 + 2 sum_{tau=1}^{lambda-1} c_tau cos(2 pi k tau / L),  k = 0..N,
// costs N * lambda multiply-adds (1e8 for both plans at lambda = 4096), so it
// is summed on the device, one frequency per thread, from a cosine table
// indexed by k tau mod L.  The weights follow from H as described in
// toeplitz.hip.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fft_lds.h"
#include "mm_internal.h"

namespace mm {
namespace {

// cos(2 pi j / kCosLen), j < kCosLen; a plan of length L reads every
// (kCosLen / L)-th entry.
constexpr int kCosLen = 2 * kFftN32L;
static_assert((kCosLen & (kCosLen - 1)) == 0, "cosine table length must be a power of two");
static_assert(kCosLen % (2 * kFftN64) == 0 && kCosLen % (2 * kFftN32) == 0, "plan lengths must divide the table");

__global__ void __launch_bounds__(256) k_symbol(const double* __restrict__ coeff, int lam,
                                                const double* __restrict__ cos_t, int step, int n,
                                                double* __restrict__ H) {
  __shared__ double c[kMaxLambda];
  const double* cf = coeff + (size_t)blockIdx.y * lam;
  for (int i = threadIdx.x; i < lam; i += blockDim.x) c[i] = cf[i];
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > n) return;
  const uint32_t dk = ((uint32_t)k * (uint32_t)step) & (kCosLen - 1);
  uint32_t idx = 0;
  // four partial sums: independent multiply-add chains
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int tau = 1;
  for (; tau + 3 < lam; tau += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      idx = (idx + dk) & (kCosLen - 1);
      acc[u] = fma(c[tau + u], cos_t[idx], acc[u]);
    }
  }
  for (; tau < lam; ++tau) {
    idx = (idx + dk) & (kCosLen - 1);
    acc[0] = fma(c[tau], cos_t[idx], acc[0]);
  }
  H[(size_t)blockIdx.y * (n + 1) + k] = c[0] + 2.0 * ((acc[0] + acc[1]) + (acc[2] + acc[3]));
}

// alpha_k = (S - D sin th) / L, beta_k = D cos th / L with S = H_k + H_{N-k},
// D = H_k - H_{N-k}, th = 2 pi k / L; sin th = cos(th - pi/2) from the table.
template <class C>
__global__ void __launch_bounds__(256) k_spectral_weights(const double* __restrict__ H,
                                                          const double* __restrict__ cos_t, int step, int n,
                                                          cpx<C>* __restrict__ ab, int regions) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double* h = H + (size_t)blockIdx.y * (n + 1);
  const double S = h[k] + h[n - k], D = h[k] - h[n - k];
  const uint32_t i = ((uint32_t)k * (uint32_t)step) & (kCosLen - 1);
  const double ct = cos_t[i];
  const double st = cos_t[(i + 3 * (kCosLen / 4)) & (kCosLen - 1)];
  const double L = 2.0 * n;
  // region-major order (the four-step plans): bin k1 + E k2 at k1 n/E + k2
  // for E = regions (a power of two)
  const int at = regions ? (k & (regions - 1)) * (n / regions) + k / regions : k;
  ab[(size_t)blockIdx.y * n + at] = cpx<C>{(C)((S - D * st) / L), (C)(D * ct / L)};
}

}  // namespace

int prepare_toeplitz_tables(mm_noise_s* nz, const double* coeff_host, void* ws, size_t ws_bytes, hipStream_t s,
                            size_t* bytes_needed) {
  const int lam = nz->lambda;
  const int nf = nz->n_filt;
  Carver cv(ws, ws_bytes);
  const int Ns[2] = {kFftN64, kFftN32};
  const int32_t wrap = nz->kind == 2 ? 1 : 0;
  std::vector<FftTile> tiles[2];
  for (int a = 0; a < 2; ++a) {
    const int64_t L = 2 * (int64_t)Ns[a];
    const int64_t V = L - 2 * (int64_t)(lam - 1);
    for (int64_t c = 0; c < nz->n_chunks; ++c) {
      const int64_t c0 = nz->chunk_offsets[c], c1 = nz->chunk_offsets[c + 1];
      for (int64_t o = c0; o < c1; o += V)
        tiles[a].push_back(FftTile{o, o + V < c1 ? o + V : c1, c0, c1, nz->chunk_filter[c], wrap});
    }
    nz->n_tiles[a] = (int64_t)tiles[a].size();
  }
  std::vector<FftTile> tiles_l;  // the 32768-point FP32 plan
  {
    const int64_t V = 2 * (int64_t)kFftN32L - 2 * (int64_t)(lam - 1);
    for (int64_t c = 0; c < nz->n_chunks; ++c) {
      const int64_t c0 = nz->chunk_offsets[c], c1 = nz->chunk_offsets[c + 1];
      for (int64_t o = c0; o < c1; o += V)
        tiles_l.push_back(FftTile{o, o + V < c1 ? o + V : c1, c0, c1, nz->chunk_filter[c], wrap});
    }
    nz->n_tiles32l = (int64_t)tiles_l.size();
  }
  // halo-carrying tiles (kCarryStride samples apart) and their segments.  Longer segments
  // gather fewer halos; the segment length is the longest (up to
  // kSegTiles) that still gives every CU a segment, and each chunk's tiles
  // are split into segments of equal length (within one tile).
  int n_cu = 256;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, nz->device) == hipSuccess && prop.multiProcessorCount > 0)
      n_cu = prop.multiProcessorCount;
  }
  std::vector<FftTile> ctiles[2];
  std::vector<CarrySeg> csegs[2];
  for (int a = 0; a < 2; ++a) {
    const int64_t stride = kCarryStride[a];
    int64_t n_ct = 0;
    for (int64_t c = 0; c < nz->n_chunks; ++c)
      n_ct += (nz->chunk_offsets[c + 1] - nz->chunk_offsets[c] + stride - 1) / stride;
    const int64_t seg_len = std::max<int64_t>(1, std::min<int64_t>(kSegTiles, n_ct / (int64_t)n_cu));
    for (int64_t c = 0; c < nz->n_chunks; ++c) {
      const int64_t c0 = nz->chunk_offsets[c], c1 = nz->chunk_offsets[c + 1];
      const int64_t nt = (c1 - c0 + stride - 1) / stride;
      if (nt == 0) continue;
      const int64_t ns = (nt + seg_len - 1) / seg_len;  // segments of this chunk
      int64_t t = 0;
      for (int64_t sgi = 0; sgi < ns; ++sgi) {
        const int64_t cnt = nt / ns + (sgi < nt % ns ? 1 : 0);
        csegs[a].push_back(CarrySeg{(int64_t)ctiles[a].size(), (int32_t)cnt, 0});
        for (int64_t u = 0; u < cnt; ++u, ++t) {
          const int64_t o = c0 + t * stride;
          ctiles[a].push_back(FftTile{o, o + stride < c1 ? o + stride : c1, c0, c1, nz->chunk_filter[c], wrap});
        }
      }
    }
    nz->n_csegs[a] = (int64_t)csegs[a].size();
  }
  FftTile* d_tiles[2];
  for (int a = 0; a < 2; ++a) d_tiles[a] = cv.take<FftTile>(tiles[a].size());
  FftTile* d_tiles_l = cv.take<FftTile>(tiles_l.size());
  FftTile* d_ctiles[2];
  CarrySeg* d_csegs[2];
  for (int a = 0; a < 2; ++a) {
    d_ctiles[a] = cv.take<FftTile>(ctiles[a].size());
    d_csegs[a] = cv.take<CarrySeg>(csegs[a].size());
  }
  void* d_ab[2];
  void* d_tw[2];
  d_ab[0] = cv.take<cpx<double>>((size_t)nf * kFftN64);
  d_ab[1] = cv.take<cpx<float>>((size_t)nf * kFftN32);
  d_tw[0] = cv.take<cpx<double>>(kFftN64);
  d_tw[1] = cv.take<cpx<float>>(kFftN32);
  void* d_abr[2];
  d_abr[0] = kHalfRegions[0] ? cv.take<cpx<double>>((size_t)nf * kFftN64) : d_ab[0];
  d_abr[1] = kHalfRegions[1] ? cv.take<cpx<float>>((size_t)nf * kFftN32) : d_ab[1];
  cpx<double>* d_ab64l = cv.take<cpx<double>>((size_t)nf * kFftN32);
  cpx<double>* d_tw64l = cv.take<cpx<double>>(kFftN32);
  cpx<float>* d_ab32l = cv.take<cpx<float>>((size_t)nf * kFftN32L);
  cpx<float>* d_tw32l = cv.take<cpx<float>>(kFftN32L);
  // build-time staging: coefficients, cosine table, symbol
  double* d_coeff = cv.take<double>((size_t)nf * lam);
  double* d_cos = cv.take<double>(kCosLen);
  double* d_H = cv.take<double>((size_t)nf * (kFftN32L + 1));
  if (bytes_needed) *bytes_needed = cv.used;
  if (ws == nullptr) return MM_OK;
  if (!cv.fits()) return fail(MM_ENOSPC, "noise workspace too small");

  std::vector<double> cos_t(kCosLen);
  for (int j = 0; j < kCosLen; ++j) cos_t[j] = std::cos(2.0 * M_PI * (double)j / (double)kCosLen);
  std::vector<cpx<double>> tw64(kFftN64);
  std::vector<cpx<float>> tw32(kFftN32);
  std::vector<cpx<double>> tw64l(kFftN32);
  std::vector<cpx<float>> tw32l(kFftN32L);
  for (int k = 0; k < kFftN64; ++k) {
    const double th = -2.0 * M_PI * (double)k / (double)kFftN64;
    tw64[k] = {std::cos(th), std::sin(th)};
  }
  for (int k = 0; k < kFftN32; ++k) {
    const double th = -2.0 * M_PI * (double)k / (double)kFftN32;
    tw64l[k] = {std::cos(th), std::sin(th)};
    tw32[k] = {(float)tw64l[k].x, (float)tw64l[k].y};
  }
  for (int k = 0; k < kFftN32L; ++k) {
    const double th = -2.0 * M_PI * (double)k / (double)kFftN32L;
    tw32l[k] = {(float)std::cos(th), (float)std::sin(th)};
  }
  for (int a = 0; a < 2; ++a) {
    if (!tiles[a].empty())
      MM_HIP(hipMemcpyAsync(d_tiles[a], tiles[a].data(), tiles[a].size() * sizeof(FftTile), hipMemcpyHostToDevice,
                            s));
    nz->tiles[a] = d_tiles[a];
    if (!ctiles[a].empty()) {
      MM_HIP(hipMemcpyAsync(d_ctiles[a], ctiles[a].data(), ctiles[a].size() * sizeof(FftTile),
                            hipMemcpyHostToDevice, s));
      MM_HIP(hipMemcpyAsync(d_csegs[a], csegs[a].data(), csegs[a].size() * sizeof(CarrySeg),
                            hipMemcpyHostToDevice, s));
    }
    nz->ctiles[a] = d_ctiles[a];
    nz->csegs[a] = d_csegs[a];
  }
  MM_HIP(hipMemcpyAsync(d_coeff, coeff_host, (size_t)nf * lam * sizeof(double), hipMemcpyHostToDevice, s));
  MM_HIP(hipMemcpyAsync(d_cos, cos_t.data(), cos_t.size() * sizeof(double), hipMemcpyHostToDevice, s));
  MM_HIP(hipMemcpyAsync(d_tw[0], tw64.data(), tw64.size() * sizeof(tw64[0]), hipMemcpyHostToDevice, s));
  MM_HIP(hipMemcpyAsync(d_tw[1], tw32.data(), tw32.size() * sizeof(tw32[0]), hipMemcpyHostToDevice, s));
  MM_HIP(hipMemcpyAsync(d_tw64l, tw64l.data(), tw64l.size() * sizeof(tw64l[0]), hipMemcpyHostToDevice, s));
  MM_HIP(hipMemcpyAsync(d_tw32l, tw32l.data(), tw32l.size() * sizeof(tw32l[0]), hipMemcpyHostToDevice, s));
  if (!tiles_l.empty())
    MM_HIP(hipMemcpyAsync(d_tiles_l, tiles_l.data(), tiles_l.size() * sizeof(FftTile), hipMemcpyHostToDevice, s));
  for (int a = 0; a < 2; ++a) {
    const int n = Ns[a];
    const int step = kCosLen / (2 * n);
    // d_H is reused by the second plan: the stream orders the two passes
    hipLaunchKernelGGL(k_symbol, dim3((n + 1 + 255) / 256, nf), dim3(256), 0, s, (const double*)d_coeff, lam,
                       (const double*)d_cos, step, n, d_H);
    MM_HIP(hipGetLastError());
    if (a == 0) {
      hipLaunchKernelGGL(k_spectral_weights<double>, dim3((n + 255) / 256, nf), dim3(256), 0, s, (const double*)d_H,
                         (const double*)d_cos, step, n, (cpx<double>*)d_ab[0], 0);
      MM_HIP(hipGetLastError());
      if (kHalfRegions[0])
        hipLaunchKernelGGL(k_spectral_weights<double>, dim3((n + 255) / 256, nf), dim3(256), 0, s,
                           (const double*)d_H, (const double*)d_cos, step, n, (cpx<double>*)d_abr[0],
                           kHalfRegions[0]);
    } else {
      hipLaunchKernelGGL(k_spectral_weights<float>, dim3((n + 255) / 256, nf), dim3(256), 0, s, (const double*)d_H,
                         (const double*)d_cos, step, n, (cpx<float>*)d_ab[1], 0);
      MM_HIP(hipGetLastError());
      if (kHalfRegions[1])
        hipLaunchKernelGGL(k_spectral_weights<float>, dim3((n + 255) / 256, nf), dim3(256), 0, s,
                           (const double*)d_H, (const double*)d_cos, step, n, (cpx<float>*)d_abr[1],
                           kHalfRegions[1]);
      MM_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_spectral_weights<double>, dim3((n + 255) / 256, nf), dim3(256), 0, s,
                         (const double*)d_H, (const double*)d_cos, step, n, d_ab64l, n / 1024);
    }
    MM_HIP(hipGetLastError());
  }
  {
    const int n = kFftN32L;
    const int step = kCosLen / (2 * n);
    hipLaunchKernelGGL(k_symbol, dim3((n + 1 + 255) / 256, nf), dim3(256), 0, s, (const double*)d_coeff, lam,
                       (const double*)d_cos, step, n, d_H);
    MM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_spectral_weights<float>, dim3((n + 255) / 256, nf), dim3(256), 0, s, (const double*)d_H,
                       (const double*)d_cos, step, n, d_ab32l, n / 1024);
    MM_HIP(hipGetLastError());
  }
  // the host staging vectors die on return: wait for the copies
  MM_HIP(hipStreamSynchronize(s));
  for (int a = 0; a < 2; ++a) {
    nz->ab[a] = d_ab[a];
    nz->abr[a] = d_abr[a];
    nz->tw[a] = d_tw[a];
  }
  nz->ab64l = d_ab64l;
  nz->tw64l = d_tw64l;
  nz->tiles32l = d_tiles_l;
  nz->ab32l = d_ab32l;
  nz->tw32l = d_tw32l;
  return MM_OK;
}

}  // namespace mm
