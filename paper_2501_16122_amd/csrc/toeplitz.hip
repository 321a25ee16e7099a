// Band-Toeplitz N^-1 per stationary chunk, applied by overlap-save FFTs in
// LDS, standalone (timeline -> timeline) and fused with the pointing
// operators (q = P^T T P x, b = P^T T d).
//
// Overlap-save: a tile reads the L-sample window starting lambda-1 samples
// before its first output (zero outside its chunk), circularly convolves it
// with the symmetric kernel h (h_0 = c_0, h_tau = h_{L-tau} = c_tau for
// 0 < tau < lambda), and keeps the V = L - 2(lambda-1) outputs whose
// circular sums never wrap: exactly the finite band section on the chunk.
//
// Real-signal trick: the L real samples u are packed as N = L/2 complex
// values z_n = u_{2n} + i u_{2n+1}; with Z = FFT_N(z) the spectrum of the
// circular convolution, repacked for the inverse, is
//   X_k = alpha_k Z_k + i beta_k conj(Z_{(N-k) mod N}),
//   alpha_k = (S_k - D_k sin th_k) / L,  beta_k = D_k cos th_k / L,
//   S_k = H_k + H_{N-k},  D_k = H_k - H_{N-k},  th_k = 2 pi k / L,
// where H is the (real, even) DFT of h, and IFFT_N(X)_n = v_{2n} + i v_{2n+1}
// is the convolved tile.  This folds the real-FFT post- and pre-processing
// and the spectral multiply into one pass over bin pairs (k, N-k).
#include <cmath>
#include <type_traits>
#include <vector>

#include "fft_lds.h"
#include "mm_internal.h"
#include "sincos2.h"

namespace mm {
namespace {

constexpr int kFftThreads = 256;

template <class C>
struct Plan;
// FP64: N = 8192 = 32 * 16 * 16, 32 elements per thread.
template <>
struct Plan<double> {
  static constexpr int N = kFftN64, R1 = 32, R2 = 16, R3 = 16;
};
// FP32: N = 16384 = 32 * 32 * 16, 64 elements per thread.
template <>
struct Plan<float> {
  static constexpr int N = kFftN32, R1 = 32, R2 = 32, R3 = 16;
};

constexpr int kLdsBytes = lds_elems<kFftN64>() * 16;  // same for both plans
static_assert(lds_elems<kFftN32>() * 8 == kLdsBytes, "plans share one LDS size");
constexpr int kTBinSlots = (kLdsBytes / 24) & ~63;    // bins reuse the FFT buffer

__device__ __forceinline__ int32_t wave_min(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_down(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const int32_t o = __shfl_down(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// kIn: 0 = timeline input tod_in; 1 = gather P x.
// kOut: 0 = timeline output tod_out; 1 = scatter q += P^T z.
template <class S, class C, int kIn, int kOut>
__global__ __launch_bounds__(kFftThreads) void k_toeplitz(const FftTile* __restrict__ tiles, int32_t lambda,
                                                          const cpx<C>* __restrict__ ab,
                                                          const cpx<C>* __restrict__ tw,
                                                          const int32_t* __restrict__ sample_k,
                                                          const S* __restrict__ psi, const double* __restrict__ x,
                                                          const S* __restrict__ tod_in, S* __restrict__ tod_out,
                                                          double* __restrict__ q, const int32_t* __restrict__ done) {
  using P = Plan<C>;
  constexpr int N = P::N, T = kFftThreads, E = N / T;
  constexpr int L = 2 * N;
  if (done != nullptr && *done) return;
  __shared__ cpx<C> buf[lds_elems<N>()];
  __shared__ int32_t s_red[8];

  const FftTile tl = tiles[blockIdx.x];
  const int64_t in0 = tl.out_start - (lambda - 1);
  const int32_t vlo = lambda - 1;                                   // first valid position
  const int32_t vhi = vlo + (int32_t)(tl.out_end - tl.out_start);  // one past the last
  const int tid = threadIdx.x;

  // ---- load the window into LDS in natural order: complex entry n packs
  // samples 2n and 2n+1 (zero outside the chunk or on masked pixels)
  int32_t kmin = INT32_MAX, kmax = -1;
#pragma unroll 2
  for (int n = tid; n < N; n += T) {
    C u[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int pos = 2 * n + h;
      const int64_t t = in0 + pos;
      C val = C(0);
      if (t >= tl.chunk_start && t < tl.chunk_end) {
        if (kIn == 0) {
          val = C(tod_in[t]);
        } else {
          const int32_t k = sample_k[t];
          if (k >= 0) {
            C c, s;
            sincos2<C>(psi[t], &c, &s);
            const double* xk = x + 3 * (int64_t)k;
            val = C(xk[0]) + c * C(xk[1]) + s * C(xk[2]);
          }
          if (kOut == 1 && k >= 0 && pos >= vlo && pos < vhi) {
            kmin = k < kmin ? k : kmin;
            kmax = k > kmax ? k : kmax;
          }
        }
        if (kIn == 0 && kOut == 1 && pos >= vlo && pos < vhi) {
          const int32_t k = sample_k[t];
          if (k >= 0) {
            kmin = k < kmin ? k : kmin;
            kmax = k > kmax ? k : kmax;
          }
        }
      }
      u[h] = val;
    }
    buf[lds_pad(n)] = cpx<C>{u[0], u[1]};
  }
  if (kOut == 1) {
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    if ((tid & 63) == 0) {
      s_red[tid >> 6] = kmin;
      s_red[4 + (tid >> 6)] = kmax;
    }
  }
  __syncthreads();

  // ---- forward FFT: passes R1, R2, R3 (spans 1, R1, R1 R2)
  cpx<C> v[E];
  pass_load<C, N, T, P::R1>(buf, v);
  pass_compute<C, N, T, P::R1, 1, true>(v, tw);
  __syncthreads();
  pass_store<C, N, T, P::R1, 1>(buf, v);
  __syncthreads();
  pass_load<C, N, T, P::R2>(buf, v);
  pass_compute<C, N, T, P::R2, P::R1, true>(v, tw);
  __syncthreads();
  pass_store<C, N, T, P::R2, P::R1>(buf, v);
  __syncthreads();
  pass_load<C, N, T, P::R3>(buf, v);
  pass_compute<C, N, T, P::R3, P::R1 * P::R2, true>(v, tw);
  __syncthreads();
  pass_store<C, N, T, P::R3, P::R1 * P::R2>(buf, v);
  __syncthreads();

  // ---- spectral multiply fused into the first inverse pass (radix R3):
  // X_k = alpha_k Z_k + i beta_k conj(Z_{N-k})
  {
    constexpr int BPT = E / P::R3;
    const cpx<C>* abf = ab + (int64_t)tl.filter * N;
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = tid + b * T;
#pragma unroll
      for (int m = 0; m < P::R3; ++m) {
        const int k = j + m * (N / P::R3);
        const cpx<C> z = buf[lds_pad(k)];
        const cpx<C> zr = buf[lds_pad((N - k) & (N - 1))];
        const cpx<C> w = abf[k];  // (alpha_k, beta_k)
        // alpha (zx + i zy) + i beta (zrx - i zry) = (alpha zx + beta zry) + i (alpha zy + beta zrx)
        v[b * P::R3 + m] = cpx<C>{w.x * z.x + w.y * zr.y, w.x * z.y + w.y * zr.x};
        if ((m & 3) == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  pass_compute<C, N, T, P::R3, 1, false>(v, tw);
  __syncthreads();
  pass_store<C, N, T, P::R3, 1>(buf, v);
  __syncthreads();
  pass_load<C, N, T, P::R2>(buf, v);
  pass_compute<C, N, T, P::R2, P::R3, false>(v, tw);
  __syncthreads();
  pass_store<C, N, T, P::R2, P::R3>(buf, v);
  __syncthreads();
  pass_load<C, N, T, P::R1>(buf, v);
  pass_compute<C, N, T, P::R1, P::R3 * P::R2, false>(v, tw);
  // v now holds, for element e, the outputs at samples 2n, 2n+1, n = tid + T e

  if (kOut == 0) {
    __syncthreads();
    pass_store<C, N, T, P::R1, P::R3 * P::R2>(buf, v);  // natural order
    __syncthreads();
#pragma unroll 2
    for (int n = tid; n < N; n += T) {
      const cpx<C> o = buf[lds_pad(n)];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int pos = 2 * n + h;
        if (pos >= vlo && pos < vhi) tod_out[in0 + pos] = S(h == 0 ? o.x : o.y);
      }
    }
    return;
  }

  // ---- P^T scatter through LDS bins over the tile's compact-index window
  __syncthreads();  // every thread is done reading buf
  kmin = s_red[0];
  kmax = s_red[4];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    kmin = s_red[w] < kmin ? s_red[w] : kmin;
    kmax = s_red[4 + w] > kmax ? s_red[4 + w] : kmax;
  }
  if (kmax < kmin) return;
  double* bins = reinterpret_cast<double*>(buf);
  const int span = kmax - kmin + 1;
  const int nb = span < kTBinSlots ? span : kTBinSlots;
  for (int i = tid; i < nb; i += T) {
    bins[i] = 0.0;
    bins[kTBinSlots + i] = 0.0;
    bins[2 * kTBinSlots + i] = 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = tid + T * e;
    const cpx<C> o = v[slot_of<N, T, P::R1>(e)];
    if ((e & 3) == 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int pos = 2 * n + h;
      if (pos < vlo || pos >= vhi) continue;
      const int64_t t = in0 + pos;
      const int32_t k = sample_k[t];
      if (k < 0) continue;
      C c, s;
      sincos2<C>(psi[t], &c, &s);
      const C z = h == 0 ? o.x : o.y;
      const int32_t rel = k - kmin;
      if (rel < nb) {
        atomicAdd(&bins[rel], double(z));
        atomicAdd(&bins[kTBinSlots + rel], double(z * c));
        atomicAdd(&bins[2 * kTBinSlots + rel], double(z * s));
      } else {
        double* qk = q + 3 * (int64_t)k;
        atomicAdd(qk + 0, double(z));
        atomicAdd(qk + 1, double(z * c));
        atomicAdd(qk + 2, double(z * s));
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < nb; i += T) {
    const double v0 = bins[i], v1 = bins[kTBinSlots + i], v2 = bins[2 * kTBinSlots + i];
    double* qk = q + 3 * (int64_t)(kmin + i);
    if (v0 != 0.0) atomicAdd(qk + 0, v0);
    if (v1 != 0.0) atomicAdd(qk + 1, v1);
    if (v2 != 0.0) atomicAdd(qk + 2, v2);
  }
}

template <class S, class C, int kIn, int kOut>
int launch_t(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tod_in, void* tod_out,
             double* q, const int32_t* done, hipStream_t s) {
  const int a = std::is_same<C, double>::value ? 0 : 1;
  if (nz->n_tiles[a] == 0) return MM_OK;
  hipLaunchKernelGGL((k_toeplitz<S, C, kIn, kOut>), dim3(nz->n_tiles[a]), dim3(kFftThreads), 0, s, nz->tiles[a],
                     nz->lambda, (const cpx<C>*)nz->ab[a], (const cpx<C>*)nz->tw[a],
                     pt ? pt->sample_k : nullptr, pt ? (const S*)pt->psi : nullptr, x, (const S*)tod_in,
                     (S*)tod_out, q, done);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

template <int kIn, int kOut>
int dispatch(const mm_pointing_s* pt, const mm_noise_s* nz, int dtype, int arith, const double* x,
             const void* tod_in, void* tod_out, double* q, const int32_t* done, hipStream_t s) {
  if (dtype == MM_F64) {
    if (arith == MM_F64) return launch_t<double, double, kIn, kOut>(pt, nz, x, tod_in, tod_out, q, done, s);
    return launch_t<double, float, kIn, kOut>(pt, nz, x, tod_in, tod_out, q, done, s);
  }
  if (arith == MM_F64) return launch_t<float, double, kIn, kOut>(pt, nz, x, tod_in, tod_out, q, done, s);
  return launch_t<float, float, kIn, kOut>(pt, nz, x, tod_in, tod_out, q, done, s);
}

}  // namespace

int launch_ninv_toeplitz(const mm_pointing_s* pt, const mm_noise_s* nz, const void* in, void* out, int arith,
                         hipStream_t s) {
  return dispatch<0, 0>(pt, nz, pt->dtype, arith, nullptr, in, out, nullptr, nullptr, s);
}

int launch_fused_toeplitz(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tod,
                          double* q, int arith, const int32_t* done, hipStream_t s) {
  if (x != nullptr) return dispatch<1, 1>(pt, nz, pt->dtype, arith, x, nullptr, nullptr, q, done, s);
  return dispatch<0, 1>(pt, nz, pt->dtype, arith, nullptr, tod, nullptr, q, done, s);
}

// Host side: overlap-save tiles per arithmetic, the spectral weights
// (alpha_k, beta_k) of every filter and the twiddle tables.
int prepare_toeplitz_tables(mm_noise_s* nz, const double* coeff_host, void* ws, size_t ws_bytes, hipStream_t s,
                            size_t* bytes_needed) {
  const int lam = nz->lambda;
  Carver cv(ws, ws_bytes);
  const int Ns[2] = {kFftN64, kFftN32};
  std::vector<FftTile> tiles[2];
  for (int a = 0; a < 2; ++a) {
    const int64_t L = 2 * (int64_t)Ns[a];
    const int64_t V = L - 2 * (int64_t)(lam - 1);
    for (int64_t c = 0; c < nz->n_chunks; ++c) {
      const int64_t c0 = nz->chunk_offsets[c], c1 = nz->chunk_offsets[c + 1];
      for (int64_t o = c0; o < c1; o += V)
        tiles[a].push_back(FftTile{o, o + V < c1 ? o + V : c1, c0, c1, nz->chunk_filter[c], 0});
    }
    nz->n_tiles[a] = (int64_t)tiles[a].size();
  }
  FftTile* d_tiles[2];
  for (int a = 0; a < 2; ++a) d_tiles[a] = cv.take<FftTile>(tiles[a].size());
  void* d_ab[2];
  void* d_tw[2];
  d_ab[0] = cv.take<cpx<double>>((size_t)nz->n_filt * kFftN64);
  d_ab[1] = cv.take<cpx<float>>((size_t)nz->n_filt * kFftN32);
  d_tw[0] = cv.take<cpx<double>>(kFftN64);
  d_tw[1] = cv.take<cpx<float>>(kFftN32);
  if (bytes_needed) *bytes_needed = cv.used;
  if (ws == nullptr) return MM_OK;
  if (!cv.fits()) return fail(MM_ENOSPC, "noise workspace too small");

  std::vector<cpx<double>> ab64((size_t)nz->n_filt * kFftN64), tw64(kFftN64);
  std::vector<cpx<float>> ab32((size_t)nz->n_filt * kFftN32), tw32(kFftN32);
  for (int a = 0; a < 2; ++a) {
    const int N = Ns[a];
    const int64_t L = 2 * (int64_t)N;
    // cos(2 pi j / L) for j in [0, L)
    std::vector<double> cosL(L);
    for (int64_t j = 0; j < L; ++j) cosL[j] = std::cos(2.0 * M_PI * (double)j / (double)L);
    for (int f = 0; f < nz->n_filt; ++f) {
      const double* c = coeff_host + (size_t)f * lam;
      // H_k = c_0 + 2 sum_{tau >= 1} c_tau cos(2 pi k tau / L), k = 0..N
      std::vector<double> H(N + 1);
      for (int k = 0; k <= N; ++k) {
        long double acc = c[0];
        int64_t idx = 0;
        for (int tau = 1; tau < lam; ++tau) {
          idx += k;
          if (idx >= L) idx -= L;
          acc += 2.0L * (long double)c[tau] * (long double)cosL[idx];
        }
        H[k] = (double)acc;
      }
      for (int k = 0; k < N; ++k) {
        const double S = H[k] + H[N - k], D = H[k] - H[N - k];
        const double th = 2.0 * M_PI * (double)k / (double)L;
        const double alpha = (S - D * std::sin(th)) / (double)L;
        const double beta = D * std::cos(th) / (double)L;
        if (a == 0)
          ab64[(size_t)f * N + k] = {alpha, beta};
        else
          ab32[(size_t)f * N + k] = {(float)alpha, (float)beta};
      }
    }
    for (int k = 0; k < N; ++k) {
      const double th = -2.0 * M_PI * (double)k / (double)N;
      if (a == 0)
        tw64[k] = {std::cos(th), std::sin(th)};
      else
        tw32[k] = {(float)std::cos(th), (float)std::sin(th)};
    }
  }
  for (int a = 0; a < 2; ++a) {
    if (!tiles[a].empty())
      MM_HIP(hipMemcpyAsync(d_tiles[a], tiles[a].data(), tiles[a].size() * sizeof(FftTile), hipMemcpyHostToDevice,
                            s));
    nz->tiles[a] = d_tiles[a];
  }
  MM_HIP(hipMemcpyAsync(d_ab[0], ab64.data(), ab64.size() * sizeof(ab64[0]), hipMemcpyHostToDevice, s));
  MM_HIP(hipMemcpyAsync(d_ab[1], ab32.data(), ab32.size() * sizeof(ab32[0]), hipMemcpyHostToDevice, s));
  MM_HIP(hipMemcpyAsync(d_tw[0], tw64.data(), tw64.size() * sizeof(tw64[0]), hipMemcpyHostToDevice, s));
  MM_HIP(hipMemcpyAsync(d_tw[1], tw32.data(), tw32.size() * sizeof(tw32[0]), hipMemcpyHostToDevice, s));
  // the host staging vectors die on return: wait for the copies
  MM_HIP(hipStreamSynchronize(s));
  for (int a = 0; a < 2; ++a) {
    nz->ab[a] = d_ab[a];
    nz->tw[a] = d_tw[a];
  }
  return MM_OK;
}

}  // namespace mm
