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
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "fft_lds.h"
#include "mm_internal.h"
#include "sincos2.h"
#include "stokes.h"

namespace mm {
namespace {

// Radix plans.
// FP64: N = 8192 = 16*16*16*2 (the radix-2 stages folded into the spectral
//   step), 512 threads x 16 elements, 136 KiB of LDS: one workgroup per CU.
// FP32: N = 16384 = 32*32*16, 512 threads x 32 elements, 136 KiB of LDS;
//   the longer tile keeps 75% of each window valid at lambda = 4096 (an
//   8192-point FP32 plan with two workgroups per CU measured slower).
template <class C>
struct Plan;
// kCarryElems: register elements a halo-carrying tile takes over from the
// previous one (its stride is (E - kCarryElems) * 2T samples, kCarryStride);
// [kKeepW0, kKeepW1): elements whose pointing weights stay in registers from
// the gather to the scatter on plain tiles (they hold most valid outputs at
// lambda = 4096; empty: none).
// kPairMerge: the scatter adds the two samples of a register element into
// one set of bin atomics when they fall in the same pixel (consecutive
// samples usually do).  kLateReduce: a halo-carrying tile reduces its
// compact-index range after the gather, so the index and weight loads are
// in flight together.  Both measured faster in FP64 only.
template <>
struct Plan<double> {
  static constexpr int N = kFftN64, T = 512, kMinBlocks = 1;
  static constexpr int kROut = 16;         // radix of the last inverse pass
  static constexpr int kGatherBatch = 8;   // entries (sample pairs) per load batch
  static constexpr int kScatterBatch = 8;
  static constexpr int kCarryElems = 8, kKeepW0 = 5, kKeepW1 = 11;
  static constexpr bool kPairMerge = true, kLateReduce = true;
};
template <>
struct Plan<float> {
  static constexpr int N = kFftN32, T = 512, kMinBlocks = 1;
  static constexpr int kROut = 32;
  static constexpr int kGatherBatch = 8;
  static constexpr int kScatterBatch = 4;
  static constexpr int kCarryElems = 8, kKeepW0 = 0, kKeepW1 = 0;
  static constexpr bool kPairMerge = false, kLateReduce = false;
};
static_assert((Plan<double>::N / Plan<double>::T - Plan<double>::kCarryElems) * 2 * Plan<double>::T ==
                  kCarryStride[0],
              "FP64 halo-carrying stride");
static_assert((Plan<float>::N / Plan<float>::T - Plan<float>::kCarryElems) * 2 * Plan<float>::T == kCarryStride[1],
              "FP32 halo-carrying stride");

// LDS reuse outside the FFT: P^T bins (NC doubles per pixel) and the staged
// map window (NC values per pixel, padded to 4 doubles for IQU so that the
// (I, Q) pair stays 16-byte aligned).
template <class C, int NC>
struct Lds {
  static constexpr int kBytes = lds_elems<Plan<C>::N>() * (int)sizeof(cpx<C>);
  static constexpr int kBinSlots = (kBytes / (8 * NC)) & ~63;
  static constexpr int kXStride = NC == 3 ? 4 : NC;
  static constexpr int kXPixels = kBytes / (8 * kXStride);
};

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

// Remaining passes of a plan: compute the pass held in registers, exchange
// through LDS, load the next pass's inputs, recurse.
template <class C, int N, int T, bool kFwd, int Ns, int R>
__device__ __forceinline__ void passes(cpx<C>* buf, cpx<C>* v, const cpx<C>* __restrict__ tw) {
  pass_compute<C, N, T, R, Ns, kFwd>(v, tw);
}
template <class C, int N, int T, bool kFwd, int Ns, int R, int R2, int... Rest>
__device__ __forceinline__ void passes(cpx<C>* buf, cpx<C>* v, const cpx<C>* __restrict__ tw) {
  pass_compute<C, N, T, R, Ns, kFwd>(v, tw);
  __syncthreads();
  pass_store<C, N, T, R, Ns>(buf, v);
  __syncthreads();
  pass_load<C, N, T, R2>(buf, v);
  passes<C, N, T, kFwd, Ns * R, R2, Rest...>(buf, v, tw);
}

// X_k = alpha_k Z_k + i beta_k conj(Z_{N-k}) for the inputs of the first
// inverse pass (radix R): slot b*R + m holds k = tid + b*T + m*N/R.
template <class C, int N, int T, int R>
__device__ __forceinline__ void spectral_load(const cpx<C>* buf, const cpx<C>* __restrict__ abf, cpx<C>* v) {
  constexpr int BPT = N / T / R;
  const int tid = fft_tid();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = tid + b * T;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int k = j + m * (N / R);
      const cpx<C> z = buf[lds_pad(k)];
      const cpx<C> zr = buf[lds_pad((N - k) & (N - 1))];
      const cpx<C> w = abf[k];  // (alpha_k, beta_k)
      // alpha (zx + i zy) + i beta (zrx - i zry) = (alpha zx + beta zry) + i (alpha zy + beta zrx)
      v[b * R + m] = cpx<C>{w.x * z.x + w.y * zr.y, w.x * z.y + w.y * zr.x};
      if (((b * R + m) & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// FP64 plan: after forward passes 16, 16, 16 the buffer holds Y, the two
// interleaved N/2-point DFTs (even / odd elements) of the packed tile.  One
// LDS round trip over bin quadruples (j, j + H, m, m + H), m = H - j, H = N/2,
// then performs the last forward radix-2 butterfly
//   Z_k = Y_k + w^k Y_{k+H},  Z_{k+H} = Y_k - w^k Y_{k+H}   (w = e^{-2 pi i/N}),
// the spectral weights X_k = alpha_k Z_k + i beta_k conj(Z_{N-k}), and the
// first inverse radix-2 pass  out_{2k} = X_k + X_{k+H},  out_{2k+1} = X_k - X_{k+H}.
__device__ __forceinline__ cpx<double> spec(cpx<double> ab, cpx<double> z, cpx<double> zr) {
  return {ab.x * z.x + ab.y * zr.y, ab.x * z.y + ab.y * zr.x};
}

template <int N, int T>
__device__ __forceinline__ void middle_r2(cpx<double>* buf, const cpx<double>* __restrict__ abf,
                                          const cpx<double>* __restrict__ tw) {
  constexpr int H = N / 2, Q = H / 2, PPT = Q / T;
  static_assert(PPT * T == Q, "quadruples must tile the threads");
  const int tid = fft_tid();
  cpx<double> o[PPT][4];
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int j = 1 + tid + T * r;  // 1..Q; j = Q is its own mirror
    const int m = H - j;
    const cpx<double> a = buf[lds_pad(j)], b = buf[lds_pad(j + H)];
    const cpx<double> c = buf[lds_pad(m)], d = buf[lds_pad(m + H)];
    const cpx<double> wb = cmul(tw[j], b), wd = cmul(tw[m], d);
    const cpx<double> zj = cadd(a, wb), zj2 = csub(a, wb), zm = cadd(c, wd), zm2 = csub(c, wd);
    const cpx<double> xj = spec(abf[j], zj, zm2), xjh = spec(abf[j + H], zj2, zm);
    const cpx<double> xm = spec(abf[m], zm, zj2), xmh = spec(abf[m + H], zm2, zj);
    o[r][0] = cadd(xj, xjh);
    o[r][1] = csub(xj, xjh);
    o[r][2] = cadd(xm, xmh);
    o[r][3] = csub(xm, xmh);
  }
  cpx<double> o0 = {0, 0}, o1 = {0, 0};
  if (tid == 0) {  // k = 0 pairs with itself and with H
    const cpx<double> a = buf[0], b = buf[lds_pad(H)];
    const cpx<double> z0 = cadd(a, b), zh = csub(a, b);
    const cpx<double> x0 = spec(abf[0], z0, z0), xh = spec(abf[H], zh, zh);
    o0 = cadd(x0, xh);
    o1 = csub(x0, xh);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int j = 1 + tid + T * r;
    const int m = H - j;
    buf[lds_pad(2 * j)] = o[r][0];
    buf[lds_pad(2 * j + 1)] = o[r][1];
    buf[lds_pad(2 * m)] = o[r][2];
    buf[lds_pad(2 * m + 1)] = o[r][3];
  }
  if (tid == 0) {
    buf[0] = o0;
    buf[lds_pad(1)] = o1;
  }
  __syncthreads();
}

template <class C>
struct Fft;
template <>
struct Fft<double> {
  static constexpr int RIn = 16, ROut = 16;  // first forward / last inverse radix
  template <int N, int T>
  static __device__ __forceinline__ void forward(cpx<double>* buf, cpx<double>* v, const cpx<double>* tw) {
    passes<double, N, T, true, 1, 16, 16, 16>(buf, v, tw);
    __syncthreads();
    pass_store<double, N, T, 16, 256>(buf, v);  // Y: two interleaved N/2-point DFTs
    __syncthreads();
  }
  template <int N, int T>
  static __device__ __forceinline__ void inverse(cpx<double>* buf, const cpx<double>* abf, cpx<double>* v,
                                                 const cpx<double>* tw) {
    middle_r2<N, T>(buf, abf, tw);
    pass_load<double, N, T, 16>(buf, v);
    passes<double, N, T, false, 2, 16, 16, 16>(buf, v, tw);
  }
};
template <>
struct Fft<float> {
  static constexpr int RIn = 32, ROut = 32;
  template <int N, int T>
  static __device__ __forceinline__ void forward(cpx<float>* buf, cpx<float>* v, const cpx<float>* tw) {
    passes<float, N, T, true, 1, 32, 32, 16>(buf, v, tw);
    __syncthreads();
    pass_store<float, N, T, 16, N / 16>(buf, v);  // natural order
    __syncthreads();
  }
  template <int N, int T>
  static __device__ __forceinline__ void inverse(cpx<float>* buf, const cpx<float>* abf, cpx<float>* v,
                                                 const cpx<float>* tw) {
    spectral_load<float, N, T, 16>(buf, abf, v);
    passes<float, N, T, false, 1, 16, 32, 32>(buf, v, tw);
  }
};

// (cos 2psi_t, sin 2psi_t) in arithmetic C: from the stored tangent
// tan psi_t when kW, else from psi.
// base[i] for a window offset i as a 32-bit unsigned byte offset from a
// wave-uniform base (one shift per load instead of a 64-bit address).  Only
// for offsets known to be >= 0: a circulant chunk's wrapped positions can
// lie before the window start (negative offsets), and those take base[i].
template <class T>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, int32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)i * (uint32_t)sizeof(T));
}

template <class C, class S, int kW>
struct Angle {
  using type = S;
  static __device__ __forceinline__ type load(const S* __restrict__ psi, const S* __restrict__ w, int32_t t) {
    if constexpr (kW == 1) return w[t];
    else return psi[t];
  }
  // the same for an offset t >= 0
  static __device__ __forceinline__ type load_nn(const S* __restrict__ psi, const S* __restrict__ w, int32_t t) {
    if constexpr (kW == 1) return ld_off(w, t);
    else return ld_off(psi, t);
  }
  static __device__ __forceinline__ type zero() { return S(0); }
  static __device__ __forceinline__ void eval(type a, C* c, C* s) {
    if constexpr (kW == 1) from_tangent<C, S>(a, c, s);
    else sincos2<C>(a, c, s);
  }
};

// P^T of one tile's outputs: q[k] += z * (the row of P: (1, cos 2psi,
// sin 2psi), or the columns the map form keeps) over the valid window
// positions [vlo, vhi), through LDS bins over the compact-index window
// [kmin, kmax].  The window is binned in passes of at most kBinSlots
// pixels (one pass for compact scans); a pass reads the indices (unless kept
// in registers: kKeepK) and weights of its own samples only, so wide windows
// (sparse or large grids) cost extra L2 reads instead of one global atomic
// per sample.  v holds the outputs in the layout of the first forward pass.
// Window position -> the (window-relative, possibly negative) position of
// the sample it holds: itself inside the chunk [ilo, ihi); for a circulant
// chunk (wrap) a position up to lam1 = lambda - 1 before or after the chunk
// holds the sample one chunk length away.  Returns false for none (zero):
// positions further out never reach a valid output.
// Branch-free (selects only), so that the loads it guards can be issued
// unconditionally from a safe position and all of a batch stay in flight.
__device__ __forceinline__ bool src_pos(int pos, int ilo, int ihi, bool wrap, int clen, int lam1, int& sp) {
  const bool in = pos >= ilo && pos < ihi;
  sp = in ? pos : (pos < ilo ? pos + clen : pos - clen);
  return in || (wrap && pos < ihi + lam1);
}

// src_pos with the wrap known at compile time, and sp always a position
// inside the chunk (the load address for a position that holds none): for a
// chunk that does not wrap, the position clamped into [ilo, ihi).
template <bool kWrap>
__device__ __forceinline__ bool win_pos(int pos, int ilo, int ihi, int clen, int lam1, int& sp) {
  if constexpr (kWrap) {
    const bool ok = src_pos(pos, ilo, ihi, true, clen, lam1, sp);
    sp = ok ? sp : ilo;
    return ok;
  } else {
    sp = max(min(pos, ihi - 1), ilo);  // >= ilo >= 0 whatever the bounds
    return (uint32_t)(pos - ilo) < (uint32_t)(ihi - ilo);
  }
}


// G: the plan whose register layout v has (N, T, last inverse radix kROut,
// kKeepW0/kKeepW1, kPairMerge).
template <class S, class C, int kW, int NC, bool kKeepK, bool kKeepW = false, int kSlots = Lds<C, NC>::kBinSlots,
          int kBatch = Plan<C>::kScatterBatch, class G = Plan<C>>
__device__ __forceinline__ void scatter_bins(const cpx<C>* v, double* bins, const int32_t* kk,
                                             const int32_t* __restrict__ sk, const S* __restrict__ ps0,
                                             const S* __restrict__ w0, int32_t vlo, int32_t vhi, int32_t kmin,
                                             int32_t kmax, double* __restrict__ q,
                                             const typename Angle<C, S, kW>::type* wk = nullptr) {
  using P = G;
  using A = Angle<C, S, kW>;
  constexpr int N = P::N, T = P::T, E = N / T, GS = kBatch;
  constexpr int kTBinSlots = kSlots;
  constexpr bool kAng = Stokes<NC>::kAngle;
  const int tid = threadIdx.x;
  for (int32_t wlo = kmin; wlo <= kmax; wlo += kTBinSlots) {
    const int nb = kmax - wlo + 1 < kTBinSlots ? kmax - wlo + 1 : kTBinSlots;
    // an opaque copy of the thread id: keeps the per-sample offsets and
    // loads inside the pass instead of 2E of them hoisted and held live
    // across all passes (the index view itself stays a global pointer, so
    // its loads stay global loads)
    int tidp = tid;
    asm volatile("" : "+v"(tidp));
    for (int i = tid; i < nb; i += T)
#pragma unroll
      for (int c = 0; c < NC; ++c) bins[c * kTBinSlots + i] = 0.0;
    __syncthreads();
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += GS) {
      // a batch whose window positions all lie outside the valid outputs
      // (the halos) has nothing to bin: skipped by every thread alike
      if (2 * T * (e0 + GS) <= vlo || 2 * T * e0 >= vhi) continue;
      __builtin_amdgcn_sched_barrier(0);  // keep one batch of loads in flight at a time
      int32_t ks[2 * GS];
      typename A::type ps[2 * GS];
#pragma unroll
      for (int i = 0; i < 2 * GS; ++i) {
        const int pos = 2 * (tidp + T * (e0 + i / 2)) + (i & 1);
        const bool valid = (uint32_t)(pos - vlo) < (uint32_t)(vhi - vlo);
        // a valid output (>= vlo >= 0): its loads are always in bounds
        const int posa = max(min(pos, vhi - 1), vlo);
        int32_t k;
        if constexpr (kKeepK) k = valid ? kk[2 * e0 + i] : -1;
        else {
          const int32_t kr = ld_off(sk, posa);  // posa >= vlo >= 0
          k = valid ? kr : -1;
        }
        const int32_t rel = k - wlo;  // k = -1 (none) gives rel < 0
        ks[i] = (uint32_t)rel < (uint32_t)nb ? rel : -1;
        const int e = e0 + i / 2;
        if (!kAng)
          ps[i] = A::zero();
        else if (kKeepW && e >= P::kKeepW0 && e < P::kKeepW1)
          ps[i] = wk[2 * (e - P::kKeepW0) + (i & 1)];
        else
          ps[i] = A::load_nn(ps0, w0, posa);  // posa >= vlo >= 0
      }
      if constexpr (P::kPairMerge) {
#pragma unroll
        for (int i = 0; i < 2 * GS; i += 2) {
          const cpx<C> o = v[slot_of<N, T, P::kROut>(e0 + i / 2)];
          C c0 = C(0), s0 = C(0), c1 = C(0), s1 = C(0);
          if constexpr (kAng) {
            A::eval(ps[i], &c0, &s0);
            A::eval(ps[i + 1], &c1, &s1);
          }
          double t0[NC], t1[NC];
          Stokes<NC>::terms(o.x, c0, s0, t0);
          Stokes<NC>::terms(o.y, c1, s1, t1);
          // the pair's second sample joins the first's atomics when both bin
          // into the same slot
          const bool same = ks[i] >= 0 && ks[i] == ks[i + 1];
#pragma unroll
          for (int j = 0; j < NC; ++j) t0[j] += same ? t1[j] : 0.0;
          if (ks[i] >= 0) {
#pragma unroll
            for (int j = 0; j < NC; ++j) atomicAdd(&bins[j * kTBinSlots + ks[i]], t0[j]);
          }
          if (ks[i + 1] >= 0 && !same) {
#pragma unroll
            for (int j = 0; j < NC; ++j) atomicAdd(&bins[j * kTBinSlots + ks[i + 1]], t1[j]);
          }
        }
      } else {
#pragma unroll
        for (int i = 0; i < 2 * GS; ++i) {
          const cpx<C> o = v[slot_of<N, T, P::kROut>(e0 + i / 2)];
          const C z = (i & 1) ? o.y : o.x;
          C c = C(0), s = C(0);
          if constexpr (kAng) A::eval(ps[i], &c, &s);
          if (ks[i] >= 0) {
            double t[NC];
            Stokes<NC>::terms(z, c, s, t);
#pragma unroll
            for (int j = 0; j < NC; ++j) atomicAdd(&bins[j * kTBinSlots + ks[i]], t[j]);
          }
        }
      }
    }
    __syncthreads();
    for (int i = tid; i < nb; i += T) {
      double* qk = q + NC * (int64_t)(wlo + i);
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const double b = bins[j * kTBinSlots + i];
        if (b != 0.0) atomicAdd(qk + j, b);
      }
    }
    __syncthreads();  // the next pass (or tile) reuses the bins
  }
}

// kIn: 0 = timeline input tod_in; 1 = gather P x.
// kOut: 0 = timeline output tod_out; 1 = scatter q += P^T z.
// kW: 1 = stream the precomputed (cos 2psi, sin 2psi) pairs instead of psi.
// NC: values per pixel of the map form (the intensity form reads no angle).
template <class S, class C, int kIn, int kOut, int kW, int NC>
__device__ __forceinline__ void toeplitz_tile(const FftTile& tl, int32_t lambda, const cpx<C>* __restrict__ abf,
                                              const cpx<C>* __restrict__ tw, const int32_t* __restrict__ sample_k,
                                              const S* __restrict__ psi, const S* __restrict__ wts,
                                              const double* __restrict__ x, const S* __restrict__ tod_in,
                                              S* __restrict__ tod_out, double* __restrict__ q, int32_t variant) {
  using P = Plan<C>;
  using F = Fft<C>;
  using A = Angle<C, S, kW>;
  constexpr int N = P::N, T = P::T, E = N / T, L = 2 * N, G = P::kGatherBatch;
  constexpr int kXPixels = Lds<C, NC>::kXPixels, kXStride = Lds<C, NC>::kXStride;
  constexpr bool kAng = Stokes<NC>::kAngle;
  static_assert(E % G == 0, "gather batches must tile the elements");
  __shared__ cpx<C> buf[lds_elems<N>()];
  __shared__ int32_t s_red[4 * (P::T / 64)];

  const int64_t in0 = tl.out_start - (lambda - 1);  // timeline index of window position 0
  const int32_t vlo = lambda - 1;                    // valid (non-wrapping) outputs: [vlo, vhi)
  const int32_t vhi = vlo + (int32_t)(tl.out_end - tl.out_start);
  // window positions inside the chunk: [ilo, ihi)
  const int32_t ilo = (int32_t)(tl.chunk_start > in0 ? tl.chunk_start - in0 : 0);
  const int32_t ihi = (int32_t)(tl.chunk_end - in0 < L ? tl.chunk_end - in0 : L);
  const bool wrap = tl.wrap != 0;
  const int32_t clen = (int32_t)(tl.chunk_end - tl.chunk_start);
  // tile-based views indexed by window position (only the chunk is read)
  const int32_t* __restrict__ sk = sample_k != nullptr ? sample_k + in0 : nullptr;
  const S* __restrict__ ps0 = (kAng && kW == 0 && psi != nullptr) ? psi + in0 : nullptr;
  const S* __restrict__ w0 = (kAng && kW == 1 && wts != nullptr) ? wts + in0 : nullptr;
  const S* __restrict__ tin = tod_in != nullptr ? tod_in + in0 : nullptr;
  S* __restrict__ tout = tod_out != nullptr ? tod_out + in0 : nullptr;
  const int tid = threadIdx.x;

  // ---- input: element e of this thread packs window samples 2n, 2n+1 with
  // n = tid + T e, which is where the first forward pass wants it
  cpx<C> v[E];
  int32_t kmin = INT32_MAX, kmax = -1;  // compact-index window of the valid outputs
  // With 16 elements per thread the compact indices stay in registers from
  // the gather to the scatter (no reload); with 32 they would not fit.
  constexpr bool kKeepK = kIn == 1 && kOut == 1 && E <= 16;
  constexpr bool kKeepW = kKeepK && kW == 1 && P::kKeepW1 > P::kKeepW0;
  int32_t kk[2 * E];
  typename A::type wk[kKeepW ? 2 * (P::kKeepW1 - P::kKeepW0) : 1];
  if constexpr (kIn == 1) {
    // (1) compact index of every window sample of this thread, one batch
#pragma unroll
    for (int i = 0; i < 2 * E; ++i) {
      const int pos = 2 * (tid + T * (i / 2)) + (i & 1);
      int sp;
      const bool ok = src_pos(pos, ilo, ihi, wrap, clen, vlo, sp);
      const int32_t kr = sk[ok ? sp : ilo];  // ilo: inside the chunk, always in bounds
      kk[i] = ok ? kr : -1;
    }
    int32_t amin = INT32_MAX, amax = -1;  // window of every kept sample (map staging)
#pragma unroll
    for (int i = 0; i < 2 * E; ++i) {
      const int pos = 2 * (tid + T * (i / 2)) + (i & 1);
      if (kk[i] >= 0) {
        amin = kk[i] < amin ? kk[i] : amin;
        amax = kk[i] > amax ? kk[i] : amax;
        if (kOut == 1 && pos >= vlo && pos < vhi) {
          kmin = kk[i] < kmin ? kk[i] : kmin;
          kmax = kk[i] > kmax ? kk[i] : kmax;
        }
      }
    }
    amin = wave_min(amin);
    amax = wave_max(amax);
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    constexpr int W = T / 64;
    if ((tid & 63) == 0) {
      s_red[tid >> 6] = kmin;
      s_red[W + (tid >> 6)] = kmax;
      s_red[2 * W + (tid >> 6)] = amin;
      s_red[3 * W + (tid >> 6)] = amax;
    }
    __syncthreads();
    amin = s_red[2 * W];
    amax = s_red[3 * W];
#pragma unroll
    for (int w = 1; w < W; ++w) {
      amin = s_red[2 * W + w] < amin ? s_red[2 * W + w] : amin;
      amax = s_red[3 * W + w] > amax ? s_red[3 * W + w] : amax;
    }
    // (2) stage the map over [amin, amax] in LDS with coalesced loads when it
    // fits (the FFT buffer is free until the first pass)
    double* xs = reinterpret_cast<double*>(buf);
    const int xspan = amax - amin + 1;
    const bool staged = amax >= amin && xspan <= kXPixels && (variant & kOpNoStaging) == 0;
    if (staged) {
      // pixel p of the window at xs[kXStride p ..]: for IQU the 32-byte
      // stride keeps the (I, Q) pair 16-byte aligned for one LDS read
      const double* xw = x + NC * (int64_t)amin;
      for (int i = tid; i < NC * xspan; i += T) {
        const int p = i / NC;
        xs[kXStride * p + (i - NC * p)] = xw[i];
      }
    }
    __syncthreads();
    // (3) pointing weights in batches, P x from the staged map
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += G) {
      __builtin_amdgcn_sched_barrier(0);  // one batch of loads in flight at a time
      typename A::type ps[2 * G];
#pragma unroll
      for (int i = 0; i < 2 * G; ++i) {
        const int pos = 2 * (tid + T * (e0 + i / 2)) + (i & 1);
        int sp;
        const bool ok = src_pos(pos, ilo, ihi, wrap, clen, vlo, sp);
        ps[i] = kAng ? A::load(ps0, w0, ok ? sp : ilo) : A::zero();
        if constexpr (kKeepW) {
          const int e = e0 + i / 2;
          if (e >= P::kKeepW0 && e < P::kKeepW1) wk[2 * (e - P::kKeepW0) + (i & 1)] = ps[i];
        }
      }
#pragma unroll
      for (int i = 0; i < 2 * G; ++i) {
        const int32_t k = kk[2 * e0 + i];
        // a masked sample reads some kept pixel (the window's first, else
        // pixel 0: the operator runs only with kept pixels) and is zeroed
        const int32_t ka = k >= 0 ? k : (amax >= amin ? amin : 0);
        C c = C(0), s = C(0);
        if constexpr (kAng) A::eval(ps[i], &c, &s);
        const double* xk = staged ? xs + kXStride * (ka - amin) : x + NC * (int64_t)ka;
        const C val = k >= 0 ? Stokes<NC>::project(xk, c, s) : C(0);
        cpx<C>& slot = v[slot_of<N, T, F::RIn>(e0 + i / 2)];
        if (i & 1) slot.y = val;
        else slot.x = val;
      }
    }
    __syncthreads();  // the FFT reuses the staging area
  } else {
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += G) {
      __builtin_amdgcn_sched_barrier(0);
      int32_t kt[2 * G];
      S tv[2 * G];
#pragma unroll
      for (int i = 0; i < 2 * G; ++i) {
        const int pos = 2 * (tid + T * (e0 + i / 2)) + (i & 1);
        int sp;
        const bool in = src_pos(pos, ilo, ihi, wrap, clen, vlo, sp);
        if (kOut == 1) {
          const bool v = pos >= ilo && pos < ihi && pos >= vlo && pos < vhi;
          const int32_t kr = sk[v ? pos : ilo];
          kt[i] = v ? kr : -1;
        }
        const S t = tin[in ? sp : ilo];
        tv[i] = in ? t : S(0);
      }
#pragma unroll
      for (int i = 0; i < 2 * G; ++i) {
        if (kOut == 1 && kt[i] >= 0) {
          kmin = kt[i] < kmin ? kt[i] : kmin;
          kmax = kt[i] > kmax ? kt[i] : kmax;
        }
        cpx<C>& slot = v[slot_of<N, T, F::RIn>(e0 + i / 2)];
        if (i & 1) slot.y = C(tv[i]);
        else slot.x = C(tv[i]);
      }
    }
    if (kOut == 1) {
      kmin = wave_min(kmin);
      kmax = wave_max(kmax);
      if ((tid & 63) == 0) {
        s_red[tid >> 6] = kmin;
        s_red[T / 64 + (tid >> 6)] = kmax;
      }
    }
  }

  // ---- forward FFT (natural order into LDS), spectral multiply fused into
  // the first inverse pass, inverse FFT (outputs stay in registers)
  F::template forward<N, T>(buf, v, tw);
  F::template inverse<N, T>(buf, abf, v, tw);
  // v[slot_of<ROut>(e)] now holds the outputs at window samples 2n, 2n+1,
  // n = tid + T e

  if (kOut == 0) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = tid + T * e;
      const cpx<C> o = v[slot_of<N, T, F::ROut>(e)];
      if (2 * n >= vlo && 2 * n < vhi) tout[2 * n] = S(o.x);
      if (2 * n + 1 >= vlo && 2 * n + 1 < vhi) tout[2 * n + 1] = S(o.y);
    }
    return;
  }

  // ---- P^T scatter through LDS bins over the tile's compact-index window
  __syncthreads();  // every thread is done reading buf
  kmin = s_red[0];
  kmax = s_red[T / 64];
#pragma unroll
  for (int w = 1; w < T / 64; ++w) {
    kmin = s_red[w] < kmin ? s_red[w] : kmin;
    kmax = s_red[T / 64 + w] > kmax ? s_red[T / 64 + w] : kmax;
  }
  if (kmax < kmin) return;
  scatter_bins<S, C, kW, NC, kKeepK, kKeepW>(v, reinterpret_cast<double*>(buf), kk, sk, ps0, w0, vlo, vhi, kmin,
                                             kmax, q, wk);
}

// One halo-carrying tile (gather P x, scatter P^T; tiles kStride = (E -
// kCarryElems) * 2T samples apart, see CarrySeg).  When `have`, the P x of
// window elements [0, kCarryElems) is this thread's carry from the previous
// tile of the segment: those window positions are the previous window's
// last kCarryElems elements, in the same thread.  On return carry holds this
// window's last kCarryElems elements, and (cmin, cmax) the compact-index
// range of their samples that are valid outputs of the next tile.  The map
// is read through L2 (no staging); indices are reloaded for the scatter.
template <class S, class C, int kW, int NC>
__device__ __forceinline__ void toeplitz_tile_carry(const FftTile& tl, int32_t lambda,
                                                    const cpx<C>* __restrict__ abf, const cpx<C>* __restrict__ tw,
                                                    const int32_t* __restrict__ sample_k, const S* __restrict__ psi,
                                                    const S* __restrict__ wts, const double* __restrict__ x,
                                                    double* __restrict__ q, cpx<C>* carry, bool have, int32_t& cmin,
                                                    int32_t& cmax) {
  using P = Plan<C>;
  using F = Fft<C>;
  using A = Angle<C, S, kW>;
  constexpr int N = P::N, T = P::T, E = N / T, L = 2 * N, G = P::kGatherBatch;
  constexpr int kCarryElems = P::kCarryElems;
  constexpr int M = E - kCarryElems;  // element shift between consecutive tiles
  constexpr int kStride = M * 2 * T;
  constexpr bool kAng = Stokes<NC>::kAngle;
  static_assert(E == F::RIn && E == F::ROut, "element e must sit in register slot e");
  static_assert(kCarryElems % G == 0 && M >= kCarryElems, "carried elements must fill whole gather batches");
  __shared__ cpx<C> buf[lds_elems<N>()];
  __shared__ int32_t s_red[4 * (P::T / 64)];

  const int64_t in0 = tl.out_start - (lambda - 1);
  const int32_t vlo = lambda - 1;
  const int32_t vhi = vlo + (int32_t)(tl.out_end - tl.out_start);
  const int32_t ilo = (int32_t)(tl.chunk_start > in0 ? tl.chunk_start - in0 : 0);
  const int32_t ihi = (int32_t)(tl.chunk_end - in0 < L ? tl.chunk_end - in0 : L);
  const bool wrap = tl.wrap != 0;
  const int32_t clen = (int32_t)(tl.chunk_end - tl.chunk_start);
  const int32_t* __restrict__ sk = sample_k + in0;
  const S* __restrict__ ps0 = (kAng && kW == 0) ? psi + in0 : nullptr;
  const S* __restrict__ w0 = (kAng && kW == 1) ? wts + in0 : nullptr;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));  // per-tile offsets: not hoisted out of the segment loop

  cpx<C> v[E];
  int32_t kk[2 * E];
#pragma unroll
  for (int i = 0; i < 2 * E; ++i) {
    const int pos = 2 * (tid + T * (i / 2)) + (i & 1);
    int sp;
    const bool ok = src_pos(pos, ilo, ihi, wrap, clen, vlo, sp);
    if (i / 2 < kCarryElems && have) {  // carried: uniform over the workgroup
      kk[i] = -1;
    } else {
      const int32_t kr = sk[ok ? sp : ilo];
      kk[i] = ok ? kr : -1;
    }
  }
  int32_t kmin = INT32_MAX, kmax = -1, nmin = INT32_MAX, nmax = -1;
  constexpr int W = T / 64;
  // the compact-index ranges of the valid outputs (this tile) and of the
  // samples that become the next tile's carried valid outputs (written out
  // at both places: as one shared lambda it compiled to a slower schedule)
  if constexpr (!P::kLateReduce) {
#pragma unroll
    for (int i = 0; i < 2 * E; ++i) {
      const int pos = 2 * (tid + T * (i / 2)) + (i & 1);
      if (kk[i] >= 0) {
        if (pos >= vlo && pos < vhi) {
          kmin = kk[i] < kmin ? kk[i] : kmin;
          kmax = kk[i] > kmax ? kk[i] : kmax;
        }
        if (pos >= vlo + kStride) {
          nmin = kk[i] < nmin ? kk[i] : nmin;
          nmax = kk[i] > nmax ? kk[i] : nmax;
        }
      }
    }
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    nmin = wave_min(nmin);
    nmax = wave_max(nmax);
    if ((tid & 63) == 0) {
      s_red[tid >> 6] = kmin;
      s_red[W + (tid >> 6)] = kmax;
      s_red[2 * W + (tid >> 6)] = nmin;
      s_red[3 * W + (tid >> 6)] = nmax;
    }
  }
  // P x of the fresh elements, in batches of pointing weights
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += G) {
    if (have && e0 < kCarryElems) {
#pragma unroll
      for (int e = e0; e < e0 + G; ++e) v[e] = carry[e];
      continue;
    }
    __builtin_amdgcn_sched_barrier(0);  // one batch of loads in flight at a time
    typename A::type ps[2 * G];
#pragma unroll
    for (int i = 0; i < 2 * G; ++i) {
      const int pos = 2 * (tid + T * (e0 + i / 2)) + (i & 1);
      int sp;
      const bool ok = src_pos(pos, ilo, ihi, wrap, clen, vlo, sp);
      ps[i] = kAng ? A::load(ps0, w0, ok ? sp : ilo) : A::zero();
    }
#pragma unroll
    for (int i = 0; i < 2 * G; ++i) {
      const int32_t k = kk[2 * e0 + i];
      C c = C(0), s = C(0);
      if constexpr (kAng) A::eval(ps[i], &c, &s);
      const C val = k >= 0 ? Stokes<NC>::project(x + NC * (int64_t)(k >= 0 ? k : 0), c, s) : C(0);
      if (i & 1) v[e0 + i / 2].y = val;
      else v[e0 + i / 2].x = val;
    }
  }
  if constexpr (P::kLateReduce) {  // the same, after the gather
#pragma unroll
    for (int i = 0; i < 2 * E; ++i) {
      const int pos = 2 * (tid + T * (i / 2)) + (i & 1);
      if (kk[i] >= 0) {
        if (pos >= vlo && pos < vhi) {
          kmin = kk[i] < kmin ? kk[i] : kmin;
          kmax = kk[i] > kmax ? kk[i] : kmax;
        }
        if (pos >= vlo + kStride) {
          nmin = kk[i] < nmin ? kk[i] : nmin;
          nmax = kk[i] > nmax ? kk[i] : nmax;
        }
      }
    }
    kmin = wave_min(kmin);
    kmax = wave_max(kmax);
    nmin = wave_min(nmin);
    nmax = wave_max(nmax);
    if ((tid & 63) == 0) {
      s_red[tid >> 6] = kmin;
      s_red[W + (tid >> 6)] = kmax;
      s_red[2 * W + (tid >> 6)] = nmin;
      s_red[3 * W + (tid >> 6)] = nmax;
    }
  }
#pragma unroll
  for (int c = 0; c < kCarryElems; ++c) carry[c] = v[M + c];
  __syncthreads();
  kmin = s_red[0];
  kmax = s_red[W];
  nmin = s_red[2 * W];
  nmax = s_red[3 * W];
#pragma unroll
  for (int w = 1; w < W; ++w) {
    kmin = s_red[w] < kmin ? s_red[w] : kmin;
    kmax = s_red[W + w] > kmax ? s_red[W + w] : kmax;
    nmin = s_red[2 * W + w] < nmin ? s_red[2 * W + w] : nmin;
    nmax = s_red[3 * W + w] > nmax ? s_red[3 * W + w] : nmax;
  }
  if (have) {  // valid outputs among the carried positions
    kmin = cmin < kmin ? cmin : kmin;
    kmax = cmax > kmax ? cmax : kmax;
  }
  cmin = nmin;
  cmax = nmax;

  F::template forward<N, T>(buf, v, tw);
  F::template inverse<N, T>(buf, abf, v, tw);
  __syncthreads();  // every thread is done reading buf
  scatter_bins<S, C, kW, NC, false>(v, reinterpret_cast<double*>(buf), nullptr, sk, ps0, w0, vlo, vhi, kmin, kmax,
                                    q);
}

// Segments of halo-carrying tiles, one segment (of one right-hand side) per
// workgroup, mapped to workgroups like k_toeplitz maps tiles.
template <class S, class C, int kW, int NC>
__global__ __launch_bounds__(Plan<C>::T, Plan<C>::kMinBlocks) void k_toeplitz_carry(
    const FftTile* __restrict__ tiles, const CarrySeg* __restrict__ segs, int64_t n_segs, int32_t lambda,
    const cpx<C>* __restrict__ ab, const cpx<C>* __restrict__ tw, const int32_t* __restrict__ sample_k,
    const S* __restrict__ psi, const S* __restrict__ wts, const double* __restrict__ x, double* __restrict__ q,
    RhsBatch rb, int32_t variant) {
  int64_t seg;
  int rhs;
  if (variant & kOpLinearOrder) {
    seg = blockIdx.x / rb.nrhs;
    rhs = (int)(blockIdx.x % rb.nrhs);
  } else {
    const int64_t per_xcd = (n_segs + 7) / 8;
    const int64_t local = blockIdx.x / 8;
    seg = (int64_t)(blockIdx.x % 8) * per_xcd + local / rb.nrhs;
    rhs = (int)(local % rb.nrhs);
  }
  if (seg >= n_segs) return;
  if (rb.done != nullptr && rb.done[(int64_t)rhs * rb.done_stride]) return;
  x += rhs * rb.vstride;
  q += rhs * rb.vstride;
  const CarrySeg sg = segs[seg];
  cpx<C> carry[Plan<C>::kCarryElems];
  int32_t cmin = INT32_MAX, cmax = -1;
  for (int t = 0; t < sg.count; ++t) {
    const FftTile tl = tiles[sg.first + t];
    toeplitz_tile_carry<S, C, kW, NC>(tl, lambda, ab + (int64_t)tl.filter * Plan<C>::N, tw, sample_k, psi, wts, x,
                                      q, carry, t > 0, cmin, cmax);
    __syncthreads();  // the next tile reuses the LDS
  }
}

// One tile of one right-hand side per workgroup.  XCD-aware mapping:
// workgroups go round-robin over the 8 XCDs, so XCD x gets a contiguous run
// of tiles; neighbouring tiles (which share their overlap-save halos) then
// run close together on one L2, and the right-hand sides of one tile are
// adjacent, so its pointing is read from HBM once.
template <class S, class C, int kIn, int kOut, int kW, int NC>
__global__ __launch_bounds__(Plan<C>::T, Plan<C>::kMinBlocks) void k_toeplitz(
    const FftTile* __restrict__ tiles, int64_t n_tiles, int32_t lambda, const cpx<C>* __restrict__ ab,
    const cpx<C>* __restrict__ tw, const int32_t* __restrict__ sample_k, const S* __restrict__ psi,
    const S* __restrict__ wts, const double* __restrict__ x, const S* __restrict__ tod_in,
    S* __restrict__ tod_out, double* __restrict__ q, RhsBatch rb, int32_t variant) {
  int64_t tile;
  int rhs;
  if (variant & kOpLinearOrder) {  // tiles in launch order
    tile = blockIdx.x / rb.nrhs;
    rhs = (int)(blockIdx.x % rb.nrhs);
  } else {
    const int64_t per_xcd = (n_tiles + 7) / 8;
    const int64_t local = blockIdx.x / 8;
    tile = (int64_t)(blockIdx.x % 8) * per_xcd + local / rb.nrhs;
    rhs = (int)(local % rb.nrhs);
  }
  if (tile >= n_tiles) return;
  if (rb.done != nullptr && rb.done[(int64_t)rhs * rb.done_stride]) return;
  if (x != nullptr) x += rhs * rb.vstride;
  q += rhs * rb.vstride;
  const FftTile tl = tiles[tile];
  toeplitz_tile<S, C, kIn, kOut, kW, NC>(tl, lambda, ab + (int64_t)tl.filter * Plan<C>::N, tw, sample_k, psi, wts, x,
                                         tod_in, tod_out, q, variant);
}

// ---------------------------------------------------------------------------
// Two workgroups per CU (operator variant bit kOpHalfLds).  The FFT state of
// a tile lives in registers, and each LDS exchange of the Stockham passes
// moves the real parts of all values first and the imaginary parts second,
// so the exchange buffer holds N scalars instead of N complex values (68 KiB
// for the FP64 plan).  Two such workgroups fit one CU's LDS, and with at
// most 128 VGPRs per thread their 16 waves fit the register file: the
// memory-bound gather and scatter of one tile overlap the FFT of the other,
// which a single 136 KiB workgroup per CU cannot do.  Plain tiles only: the
// whole window is gathered (its halo is read again through L2 by the
// neighbouring tile, which the XCD-aware order keeps on the same L2).
// ---------------------------------------------------------------------------

// padded scalar index of the half buffer (one pad scalar every 16)
__device__ __forceinline__ int hpad(int i) { return i + (i >> 4); }
template <int N>
constexpr int hlds_elems() { return N + N / 16; }
// hpad(i + d) - hpad(i) for the offsets d the exchanges use: d a multiple of
// 16, or d = q Ns with Ns dividing 16 and i mod Ns = i mod 16 < Ns (the low
// bits of i then never carry into the pad count).  With it each thread forms
// one padded address per butterfly and reaches the rest by constant offsets.
constexpr int hstep(int d) { return d + (d >> 4); }

template <class C, int kComp>
__device__ __forceinline__ C& comp(cpx<C>& a) {
  if constexpr (kComp == 0) return a.x;
  else return a.y;
}

// Component kComp of every value of pass (R, Ns) to its output position.
template <class C, int N, int T, int R, int Ns, int kComp>
__device__ __forceinline__ void hstore(C* buf, cpx<C>* v) {
  constexpr int BPT = N / T / R;
  const int tid = fft_tid();
  static_assert(Ns % 16 == 0 || (16 % Ns == 0 && (Ns * R) % 16 == 0), "offsets q Ns must keep the pad count");
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = tid + b * T;
    const int pb = hpad((j / Ns) * Ns * R + (j & (Ns - 1)));
#pragma unroll
    for (int q = 0; q < R; ++q) buf[pb + hstep(q * Ns)] = comp<C, kComp>(v[b * R + q]);
  }
}

// Component kComp of the inputs of a pass of radix R.
template <class C, int N, int T, int R, int kComp>
__device__ __forceinline__ void hload(const C* buf, cpx<C>* v) {
  constexpr int BPT = N / T / R;
  const int tid = fft_tid();
  static_assert((N / R) % 16 == 0, "input stride must keep the pad count");
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int pj = hpad(tid + b * T);
#pragma unroll
    for (int m = 0; m < R; ++m) comp<C, kComp>(v[b * R + m]) = buf[pj + hstep(m * (N / R))];
  }
}

// Every register value complete here: the compiler may not sink the
// arithmetic that produces a component past the LDS round that stores the
// other one (which would keep a pass's intermediates live instead).
template <class C, int E>
__device__ __forceinline__ void settle(cpx<C>* v) {
#pragma unroll
  for (int e = 0; e < E; ++e) asm volatile("" : "+v"(v[e].x), "+v"(v[e].y));
}

// Exchange between pass (R, Ns) and the next pass (radix R2): real parts,
// then imaginary parts, through the same half buffer.
template <class C, int N, int T, int R, int Ns, int R2>
__device__ __forceinline__ void hexchange(C* buf, cpx<C>* v) {
  settle<C, N / T>(v);
  __syncthreads();
  hstore<C, N, T, R, Ns, 0>(buf, v);
  __syncthreads();
  hload<C, N, T, R2, 0>(buf, v);
  __syncthreads();
  hstore<C, N, T, R, Ns, 1>(buf, v);
  __syncthreads();
  hload<C, N, T, R2, 1>(buf, v);
}

template <class C, int N, int T, bool kFwd, int Ns, int R>
__device__ __forceinline__ void hpasses(C* buf, cpx<C>* v, const cpx<C>* __restrict__ tw) {
  pass_compute<C, N, T, R, Ns, kFwd>(v, tw);
}
template <class C, int N, int T, bool kFwd, int Ns, int R, int R2, int... Rest>
__device__ __forceinline__ void hpasses(C* buf, cpx<C>* v, const cpx<C>* __restrict__ tw) {
  pass_compute<C, N, T, R, Ns, kFwd>(v, tw);
  hexchange<C, N, T, R, Ns, R2>(buf, v);
  hpasses<C, N, T, kFwd, Ns * R, R2, Rest...>(buf, v, tw);
}

// The FP64 middle step (see middle_r2) through the half buffer: v holds the
// outputs of the last forward pass (radix 16, span 256) on entry and the
// inputs of the first inverse pass (radix 16) on return.  Thread t takes the
// bin quadruples (j, j + H, m, m + H) with j = t + T r, m = H - j, one
// component per LDS round, computes them in registers and scatters the
// results to 2j, 2j + 1, 2m, 2m + 1.  Bins 0 and H pair with themselves:
// the slot j = 0 uses them as its own mirrors, and its m side takes the
// self-paired quadruple m = Q instead, so no thread branches.
template <int N, int T>
__device__ __forceinline__ void hmiddle(double* buf, cpx<double>* v, const cpx<double>* __restrict__ abf,
                                        const cpx<double>* __restrict__ tw) {
  constexpr int H = N / 2, Q = H / 2, PPT = Q / T;
  static_assert(PPT * T == Q && 4 * PPT == N / T, "quadruples must fill the registers");
  settle<double, N / T>(v);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    __syncthreads();
    if (c == 0) hstore<double, N, T, 16, 256, 0>(buf, v);
    else hstore<double, N, T, 16, 256, 1>(buf, v);
    __syncthreads();
    // j = t + T r and m = H - j (m = Q for j = 0): padded addresses from
    // those of t and H - t by constant offsets
    const int t = fft_tid();
    const int pj = hpad(t), pmh = hpad(H - t), pm0 = t == 0 ? hpad(Q) : pmh;
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const int aj = pj + hstep(T * r), am = r == 0 ? pm0 : pmh - hstep(T * r);
      (c == 0 ? v[4 * r + 0].x : v[4 * r + 0].y) = buf[aj];
      (c == 0 ? v[4 * r + 1].x : v[4 * r + 1].y) = buf[aj + hstep(H)];
      (c == 0 ? v[4 * r + 2].x : v[4 * r + 2].y) = buf[am];
      (c == 0 ? v[4 * r + 3].x : v[4 * r + 3].y) = buf[am + hstep(H)];
    }
  }
  const int t0 = fft_tid();
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int j = t0 + T * r;
    // bins 0 and H pair with themselves; this slot's m side takes m = Q (only
    // thread 0's first slot: r > 0 never holds j = 0)
    const bool j0 = r == 0 && t0 == 0;
    const int m = j0 ? Q : H - j;
    const cpx<double> t = tw[j];
    const cpx<double> tm = j0 ? cpx<double>{0.0, -1.0} : cpx<double>{-t.x, t.y};  // w^m
    const cpx<double> wb = cmul(t, v[4 * r + 1]), wd = cmul(tm, v[4 * r + 3]);
    const cpx<double> zj = cadd(v[4 * r], wb), zj2 = csub(v[4 * r], wb);
    const cpx<double> zm = cadd(v[4 * r + 2], wd), zm2 = csub(v[4 * r + 2], wd);
    const cpx<double> xj = spec(abf[j], zj, j0 ? zj : zm2), xjh = spec(abf[j + H], zj2, j0 ? zj2 : zm);
    const cpx<double> xm = spec(abf[m], zm, j0 ? zm2 : zj2), xmh = spec(abf[m + H], zm2, j0 ? zm : zj);
    v[4 * r + 0] = cadd(xj, xjh);
    v[4 * r + 1] = csub(xj, xjh);
    v[4 * r + 2] = cadd(xm, xmh);
    v[4 * r + 3] = csub(xm, xmh);
  }
  settle<double, N / T>(v);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    __syncthreads();
    // 2j, 2m even: 2j + 1 and 2m + 1 sit one scalar further
    const int t = fft_tid();
    const int pj = hpad(2 * t), pmh = hpad(2 * (H - t)), pm0 = t == 0 ? hpad(2 * Q) : pmh;
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const int aj = pj + hstep(2 * T * r), am = r == 0 ? pm0 : pmh - hstep(2 * T * r);
      buf[aj] = c == 0 ? v[4 * r + 0].x : v[4 * r + 0].y;
      buf[aj + 1] = c == 0 ? v[4 * r + 1].x : v[4 * r + 1].y;
      buf[am] = c == 0 ? v[4 * r + 2].x : v[4 * r + 2].y;
      buf[am + 1] = c == 0 ? v[4 * r + 3].x : v[4 * r + 3].y;
    }
    __syncthreads();
    if (c == 0) hload<double, N, T, 16, 0>(buf, v);
    else hload<double, N, T, 16, 1>(buf, v);
  }
}

// ---------------------------------------------------------------------------
// The half-buffer plans' transforms as a four-step split (Bailey's
// decomposition N = E * M with E = N/T values per thread and M = T; Van
// Loan, Sec. 3.3): with n = n2 + M n1 and k = k1 + E k2,
//   X[k1 + E k2] = sum_n2 W_M^(n2 k2) W_N^(n2 k1) sum_n1 x[n2 + M n1] W_E^(n1 k1).
// Thread t = n2 holds x[t + M n1] (the gather's layout), so the E-point
// DFTs and the twiddles W_N^(t k1) run in its registers; one transpose
// through the half buffer hands the E sequences of length M to the T/64
// waves, S = E / (T/64) sequences each, whose 64 lanes then run M-point
// Stockham transforms (radix 16, 8, 8 for M = 1024; 8, 8, 8 for M = 512)
// in the wave's own region of the buffer.  Only the transposes need the
// whole workgroup: the exchanges inside a wave's transforms order
// themselves (a wave's LDS operations complete in issue order), so the
// waves meet at 10 barriers per transform pair instead of 2 per pass.  The
// inverse runs the same steps backwards.  The spectral step pairs bin k
// with N - k through the buffer in region-major order (bin k1 + E k2 at
// sequence k1, position k2); each thread then forms its own bins' outputs
// in place.  Its weights come in the same region-major order.
// ---------------------------------------------------------------------------
template <class C, int N, int T>
struct Fs {
  static constexpr int E = N / T, M = T, W = T / 64, S = E / W, V = M / 64;
  static constexpr int MR = M + M / 16;  // one sequence's padded scalars
  static_assert(S * W == E && V == W && (M == 1024 || M == 512), "four-step shape");
  // slot of local element ln + 64 e after a wave transform's last pass
  // (radix 8)
  static constexpr int slot_out(int e) { return (e % (V / 8)) * 8 + e / (V / 8); }
};

// orders this wave's LDS operations around it (no workgroup barrier)
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One pass (radix R, span Ns) of a wave's transform of V values per lane:
// lane `ln` holds butterflies j = ln + 64 b; twiddles
// W_(Ns R)^k = W_N^(k N / (Ns R)) from the N-point table.
template <class C, int N, int V, int R, int Ns, bool kFwd>
__device__ __forceinline__ void fs_pass(cpx<C>* v, const cpx<C>* __restrict__ tw, int ln) {
  constexpr int BPT = V / R;
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    cpx<C>* a = v + b * R;
    if (Ns > 1) {
      const int k = (ln + 64 * b) & (Ns - 1);
      cpx<C> w1 = tw[k * (N / (Ns * R))];
      if (!kFwd) w1.y = -w1.y;
      cpx<C> w = w1;
#pragma unroll
      for (int m = 1; m < R; ++m) {
        a[m] = cmul(a[m], w);
        if (m + 1 < R) w = cmul(w, w1);
      }
    }
    dft_reg<C, R, kFwd>(a);
  }
}

// Exchange inside one sequence's region between pass (R, Ns) and a pass of
// radix R2, one component per round.  Ns and Ns R are powers of two, so an
// output's offset q Ns from its butterfly's first output never moves it
// across more pads than hstep counts.
template <class C, int M, int V, int R, int Ns, int R2>
__device__ __forceinline__ void fs_exchange(C* reg, cpx<C>* v, int ln) {
  static_assert(Ns % 16 == 0 || 16 % Ns == 0, "offsets q Ns must keep the pad count");
  static_assert((M / R2) % 16 == 0, "input stride must keep the pad count");
  constexpr int BPT = V / R, BPT2 = V / R2;
  settle<C, V>(v);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    wave_sync();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = ln + 64 * b;
      const int pb = hpad((j / Ns) * Ns * R + (j & (Ns - 1)));
#pragma unroll
      for (int q = 0; q < R; ++q) reg[pb + hstep(q * Ns)] = c == 0 ? v[b * R + q].x : v[b * R + q].y;
    }
    wave_sync();
#pragma unroll
    for (int b = 0; b < BPT2; ++b) {
      const int pj = hpad(ln + 64 * b);
#pragma unroll
      for (int m = 0; m < R2; ++m) (c == 0 ? v[b * R2 + m].x : v[b * R2 + m].y) = reg[pj + hstep(m * (M / R2))];
    }
  }
}

// A wave's M-point transform of one sequence, natural order in (slot e =
// element ln + 64 e) and out (slot Fs::slot_out(e)).
template <class C, int N, int M, int V, bool kFwd>
__device__ __forceinline__ void fs_wave_fft(C* reg, cpx<C>* v, const cpx<C>* __restrict__ tw, int ln) {
  if constexpr (M == 1024) {
    fs_pass<C, N, V, 16, 1, kFwd>(v, tw, ln);
    fs_exchange<C, M, V, 16, 1, 8>(reg, v, ln);
    fs_pass<C, N, V, 8, 16, kFwd>(v, tw, ln);
    fs_exchange<C, M, V, 8, 16, 8>(reg, v, ln);
    fs_pass<C, N, V, 8, 128, kFwd>(v, tw, ln);
  } else {
    fs_pass<C, N, V, 8, 1, kFwd>(v, tw, ln);
    fs_exchange<C, M, V, 8, 1, 8>(reg, v, ln);
    fs_pass<C, N, V, 8, 8, kFwd>(v, tw, ln);
    fs_exchange<C, M, V, 8, 8, 8>(reg, v, ln);
    fs_pass<C, N, V, 8, 64, kFwd>(v, tw, ln);
  }
}

// v[k1] *= W_N^(+-t k1), by powers of the thread's twiddle
template <class C, int E, bool kFwd>
__device__ __forceinline__ void fs_twiddle(cpx<C>* v, const cpx<C>* __restrict__ tw, int t) {
  cpx<C> w1 = tw[t];
  if (!kFwd) w1.y = -w1.y;
  cpx<C> w = w1;
#pragma unroll
  for (int k1 = 1; k1 < E; ++k1) {
    v[k1] = cmul(v[k1], w);
    if (k1 + 1 < E) w = cmul(w, w1);
  }
}

// Forward transform: on entry slot e of thread t holds element t + M e; on
// return slot s V + Fs::slot_out(e) of lane ln in wave w holds bin
// k1 + E (ln + 64 e) with k1 = w S + s.  The caller has synchronized the
// workgroup since the buffer's last use.
template <class C, int N, int T>
__device__ __forceinline__ void fs_forward(C* buf, cpx<C>* v, const cpx<C>* __restrict__ tw) {
  using F = Fs<C, N, T>;
  const int t = fft_tid();
  const int ln = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  dft_reg<C, F::E, true>(v);
  fs_twiddle<C, F::E, true>(v, tw, t);
  settle<C, F::E>(v);
  const int pt = hpad(t), pl = w * F::S * F::MR + hpad(ln);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (c > 0) __syncthreads();  // every wave has read the first round
#pragma unroll
    for (int k1 = 0; k1 < F::E; ++k1) buf[k1 * F::MR + pt] = c == 0 ? v[k1].x : v[k1].y;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < F::S; ++s)
#pragma unroll
      for (int m = 0; m < F::V; ++m)
        (c == 0 ? v[s * F::V + m].x : v[s * F::V + m].y) = buf[pl + s * F::MR + 68 * m];
  }
#pragma unroll
  for (int s = 0; s < F::S; ++s)
    fs_wave_fft<C, N, F::M, F::V, true>(buf + (w * F::S + s) * F::MR, v + s * F::V, tw, ln);
}

// Spectral step on the forward layout: bin k = k1 + E k2 (k2 = ln + 64 e)
// becomes X_k = alpha_k Z_k + i beta_k conj(Z_(N-k)) (the real-data
// packing's spectral step); its mirror sits in sequence E - k1 at
// position M - 1 - k2 (for k1 = 0: sequence 0, position M - k2, and bin 0
// is its own mirror).  abp holds the weights in the same region-major order.
// On return slot s V + e holds bin k1 + E (ln + 64 e), the inverse's input
// layout.
template <class C, int N, int T>
__device__ __forceinline__ void fs_middle(C* buf, cpx<C>* v, const cpx<C>* __restrict__ abp) {
  using F = Fs<C, N, T>;
  const int t = fft_tid();
  const int ln = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int pl = w * F::S * F::MR + hpad(ln);
  settle<C, F::E>(v);
  C zrx[F::E];
  cpx<C> o[F::E];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    // a wave writes only its own sequences, which no other wave has used
    // since the last barrier in the first round; in the second the mirror
    // waves must have read the first
    if (c > 0) __syncthreads();
    else wave_sync();
#pragma unroll
    for (int s = 0; s < F::S; ++s)
#pragma unroll
      for (int e = 0; e < F::V; ++e) {
        const cpx<C> z = v[s * F::V + F::slot_out(e)];
        buf[pl + s * F::MR + 68 * e] = c == 0 ? z.x : z.y;
      }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < F::S; ++s) {
      const int k1 = w * F::S + s;
      const int pm = k1 != 0 ? (F::E - k1) * F::MR + hpad(F::M - 1 - ln) : hpad(F::M - ln);
      const int pm0 = (k1 == 0 && ln == 0) ? 0 : pm;
#pragma unroll
      for (int e = 0; e < F::V; ++e) {
        const int i = s * F::V + e;
        const C zr = buf[e == 0 ? pm0 : pm - 68 * e];
        if (c == 0) {
          zrx[i] = zr;
        } else {
          const cpx<C> ab = abp[k1 * F::M + ln + 64 * e];
          const cpx<C> z = v[s * F::V + F::slot_out(e)];
          o[i] = cpx<C>{ab.x * z.x + ab.y * zr, ab.x * z.y + ab.y * zrx[i]};
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < F::E; ++i) v[i] = o[i];
  __syncthreads();  // the mirror waves have read this wave's sequences
}

// Inverse transform from the spectral step's layout; on return slot n1 of
// thread t holds element t + M n1.
template <class C, int N, int T>
__device__ __forceinline__ void fs_inverse(C* buf, cpx<C>* v, const cpx<C>* __restrict__ tw) {
  using F = Fs<C, N, T>;
  const int t = fft_tid();
  const int ln = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
#pragma unroll
  for (int s = 0; s < F::S; ++s)
    fs_wave_fft<C, N, F::M, F::V, false>(buf + (w * F::S + s) * F::MR, v + s * F::V, tw, ln);
  settle<C, F::E>(v);
  const int pt = hpad(t), pl = w * F::S * F::MR + hpad(ln);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    // the first round writes the wave's own sequences, used since the last
    // barrier by this wave alone
    if (c > 0) __syncthreads();
    else wave_sync();
#pragma unroll
    for (int s = 0; s < F::S; ++s)
#pragma unroll
      for (int e = 0; e < F::V; ++e) {
        const cpx<C> u = v[s * F::V + F::slot_out(e)];
        buf[pl + s * F::MR + 68 * e] = c == 0 ? u.x : u.y;
      }
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < F::E; ++k1) (c == 0 ? v[k1].x : v[k1].y) = buf[k1 * F::MR + pt];
  }
  fs_twiddle<C, F::E, false>(v, tw, t);
  dft_reg<C, F::E, false>(v);
}

// Plans of the half-buffer kernel.  Batches are smaller than the
// one-per-CU plan's, so that a batch of loads and the 16 register values
// fit 128 VGPRs.  kFft: 3 = the four-step split (fs_forward), its spectral
// weights in region-major order; 0 = Stockham passes through the whole
// buffer, FP64 8192 points (forward 16, 16, 16, the last radix 2 folded
// into the spectral step; weights in natural order).
template <class C>
struct HPlan {
  static constexpr int N = Plan<C>::N, T = Plan<C>::T, kROut = Plan<C>::kROut, kFft = 0;
  static constexpr bool kKeepIdx = true;   // window indices in registers from the first loads to the gather
  static constexpr int kGatherBatch = 2;   // entries (sample pairs) per load batch
  static constexpr int kScatterBatch = 2;
  static constexpr int kWavesPerEU = 4;    // two 512-thread workgroups per CU
  static constexpr int kKeepW0 = 0, kKeepW1 = 0;
  static constexpr bool kPairMerge = Plan<C>::kPairMerge;
};
// FP32: 32 values per thread, indices loaded again in the gather batches, so
// longer batches keep as many loads in flight
template <>
struct HPlan<float> {
  static constexpr int N = Plan<float>::N, T = Plan<float>::T, kROut = Plan<float>::kROut, kFft = 3;
  static constexpr bool kKeepIdx = false;
  static constexpr int kGatherBatch = 4;
  static constexpr int kScatterBatch = 2;
  static constexpr int kWavesPerEU = 4;
  static constexpr int kKeepW0 = 0, kKeepW1 = 0;
  static constexpr bool kPairMerge = Plan<float>::kPairMerge;
};
static_assert((HPlan<double>::kFft == 3 ? HPlan<double>::N / HPlan<double>::T : 0) == kHalfRegions[0] &&
                  (HPlan<float>::kFft == 3 ? HPlan<float>::N / HPlan<float>::T : 0) == kHalfRegions[1],
              "weight order of the two-per-CU plans");
// FP32 on 32768-point tiles (65536-sample windows): 1024 threads x 32
// values, one workgroup per CU, the 136 KiB half buffer.
struct HPlanL32 {
  static constexpr int N = kFftN32L, T = 1024, kROut = 32, kFft = 3;
  static constexpr bool kKeepIdx = false;
  static constexpr int kGatherBatch = 4;
  static constexpr int kScatterBatch = 4;
  static constexpr int kWavesPerEU = 4;
  static constexpr int kKeepW0 = 0, kKeepW1 = 0;
  static constexpr bool kPairMerge = false;
};
// FP64 on the 16384-point tiles: 1024 threads x 16 values, one workgroup
// (16 waves, 4 per SIMD) per CU, the 136 KiB half buffer.
struct HPlanL64 {
  static constexpr int N = kFftN32, T = 1024, kROut = 16, kFft = 3;
  static constexpr bool kKeepIdx = true;
  static constexpr int kGatherBatch = 2;
  static constexpr int kScatterBatch = 4;
  static constexpr int kWavesPerEU = 4;
  static constexpr int kKeepW0 = 0, kKeepW1 = 0;
  static constexpr bool kPairMerge = true;
};

// kIn: 1 = the timeline is P x, gathered from the map x; 0 = the timeline
// is tod (the right-hand side P^T N^-1 d).
template <class S, class C, int kW, int NC, class P, bool kWrap, int kIn = 1>
__device__ __forceinline__ void toeplitz_tile_half(const FftTile& tl, int32_t lambda, const cpx<C>* __restrict__ abf,
                                                   const cpx<C>* __restrict__ tw,
                                                   const int32_t* __restrict__ sample_k, const S* __restrict__ psi,
                                                   const S* __restrict__ wts, const double* __restrict__ x,
                                                   double* __restrict__ q, const S* __restrict__ tod = nullptr) {
  using A = Angle<C, S, kW>;
  constexpr int N = P::N, T = P::T, E = N / T, L = 2 * N, G = P::kGatherBatch;
  constexpr bool kAng = Stokes<NC>::kAngle;
  constexpr int kSlots = (hlds_elems<N>() * (int)sizeof(C) / 8) / NC / 64 * 64;
  static_assert(E % G == 0, "gather batches must tile the elements");
  static_assert((E == 16 && std::is_same<C, double>::value) || (E == 32 && std::is_same<C, float>::value),
                "the half-buffer plans: FP64 16 values per thread, FP32 32");
  // FP64 keeps every window index in registers from the first round of
  // loads to the gather; FP32 (twice the samples per thread) has no room and
  // loads them again in the gather batches
  constexpr bool kKeepIdx = P::kKeepIdx && kIn == 1;
  static_assert(!kKeepIdx || E == 16, "indices kept for 16 values per thread");
  __shared__ C buf[hlds_elems<N>()];
  __shared__ int32_t s_red[4 * (T / 64)];

  const int64_t in0 = tl.out_start - (lambda - 1);
  const int32_t vlo = lambda - 1;
  const int32_t vhi = vlo + (int32_t)(tl.out_end - tl.out_start);
  const int32_t ilo = (int32_t)(tl.chunk_start > in0 ? tl.chunk_start - in0 : 0);
  const int32_t ihi = (int32_t)(tl.chunk_end - in0 < L ? tl.chunk_end - in0 : L);
  const int32_t clen = (int32_t)(tl.chunk_end - tl.chunk_start);
  const int32_t* __restrict__ sk = sample_k + in0;
  const S* __restrict__ ps0 = (kAng && kW == 0) ? psi + in0 : nullptr;
  const S* __restrict__ w0 = (kAng && kW == 1) ? wts + in0 : nullptr;
  const int tid = threadIdx.x;

  // ---- (1) compact indices of every window sample, in rounds of 32 loads
  // per thread (element e of this thread packs window samples 2n, 2n+1,
  // n = tid + T e), and their ranges: the whole window (map staging) and
  // the valid outputs
  constexpr int kPre = kKeepIdx ? 2 * E : 1;
  int32_t kk[kPre];
  // minima as unsigned: the index -1 (no sample, or a masked pixel) is then
  // the largest value and drops out of min and max alike, without branches
  uint32_t amin_u = UINT32_MAX, kmin_u = UINT32_MAX;
  int32_t amax = -1, kmax = -1;
#pragma unroll
  for (int h = 0; h < 2 * E; h += 32) {
    int32_t kr32[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const int pos = 2 * (tid + T * ((h + i) / 2)) + (i & 1);
      int sp;
      const bool ok = win_pos<kWrap>(pos, ilo, ihi, clen, vlo, sp);
      // without wrap, sp lies in [ilo, ihi): a non-negative offset
      const int32_t kr = kWrap ? sk[sp] : ld_off(sk, sp);
      kr32[i] = ok ? kr : -1;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const int pos = 2 * (tid + T * ((h + i) / 2)) + (i & 1);
      const int32_t k = kr32[i];
      if constexpr (kKeepIdx) kk[h + i] = k;
      amin_u = min(amin_u, (uint32_t)k);
      amax = max(amax, k);
      const int32_t kv = (uint32_t)(pos - vlo) < (uint32_t)(vhi - vlo) ? k : -1;
      kmin_u = min(kmin_u, (uint32_t)kv);
      kmax = max(kmax, kv);
    }
  }
  int32_t amin = (int32_t)min(amin_u, (uint32_t)INT32_MAX), kmin = (int32_t)min(kmin_u, (uint32_t)INT32_MAX);
  constexpr int W = T / 64;
  amin = wave_min(amin);
  amax = wave_max(amax);
  kmin = wave_min(kmin);
  kmax = wave_max(kmax);
  if ((tid & 63) == 0) {
    s_red[tid >> 6] = kmin;
    s_red[W + (tid >> 6)] = kmax;
    s_red[2 * W + (tid >> 6)] = amin;
    s_red[3 * W + (tid >> 6)] = amax;
  }
  __syncthreads();
  amin = s_red[2 * W];
  amax = s_red[3 * W];
#pragma unroll
  for (int w = 1; w < W; ++w) {
    amin = s_red[2 * W + w] < amin ? s_red[2 * W + w] : amin;
    amax = s_red[3 * W + w] > amax ? s_red[3 * W + w] : amax;
  }
  // ---- (2) the map over [amin, amax] staged in the (still free) FFT
  // buffer with coalesced loads, NC doubles per pixel, when it fits
  double* xs = reinterpret_cast<double*>(buf);
  constexpr int kXPix = hlds_elems<N>() * (int)sizeof(C) / 8 / NC;
  const int xspan = amax - amin + 1;
  const bool staged = kIn == 1 && amax >= amin && xspan <= kXPix;
  if (staged) {
    const double* __restrict__ xw = x + NC * (int64_t)amin;
    const int nx = NC * xspan;
    for (int i0 = 0; i0 < nx; i0 += 4 * T) {
      double t4[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + tid + u * T;
        t4[u] = xw[i < nx ? i : 0];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + tid + u * T;
        if (i < nx) xs[i] = t4[u];
      }
    }
  }
  __syncthreads();
  // ---- (3) pointing weights in batches, P x from the staged map (or the
  // map in global memory when the window's pixels do not fit): one loop per
  // source, so that each reads its own memory directly
  cpx<C> v[E];
  const int32_t kfill = amax >= amin ? amin : 0;  // a kept pixel for masked samples (zeroed after)
  auto gather = [&](auto from_lds) {
    constexpr bool kLds = decltype(from_lds)::value;
    int tdep = tid;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += G) {
      // one batch of loads in flight at a time: the positions of a batch
      // are computed from a thread id that waits for the previous batch's
      // last value, so the compiler cannot issue the loads of several
      // batches at once and hold them beside the register values
      __builtin_amdgcn_sched_barrier(0);
      if (e0 > 0) asm volatile("" : "+v"(tdep) : "v"(v[e0 - 1].y));
      typename A::type ps[2 * G];
      int32_t kb[2 * G];
#pragma unroll
      for (int i = 0; i < 2 * G; ++i) {
        const int pos = 2 * (tdep + T * (e0 + i / 2)) + (i & 1);
        int sp;
        const bool ok = win_pos<kWrap>(pos, ilo, ihi, clen, vlo, sp);
        ps[i] = kAng ? (kWrap ? A::load(ps0, w0, sp) : A::load_nn(ps0, w0, sp)) : A::zero();
        if constexpr (kKeepIdx) {
          kb[i] = kk[2 * e0 + i];
          (void)ok;
        } else {
          const int32_t kr = kWrap ? sk[sp] : ld_off(sk, sp);
          kb[i] = ok ? kr : -1;
        }
      }
#pragma unroll
      for (int i = 0; i < 2 * G; ++i) {
        const int32_t k = kb[i];
        const int32_t ka = k >= 0 ? k : kfill;
        C c = C(0), s = C(0);
        if constexpr (kAng) A::eval(ps[i], &c, &s);
        C val;
        if constexpr (kLds) val = Stokes<NC>::project(xs + NC * (ka - amin), c, s);
        else val = Stokes<NC>::project(x + NC * (int64_t)ka, c, s);
        val = k >= 0 ? val : C(0);
        if (i & 1) v[e0 + i / 2].y = val;
        else v[e0 + i / 2].x = val;
      }
    }
  };
  if constexpr (kIn == 1) {
    if (staged) gather(std::true_type{});
    else gather(std::false_type{});
  } else {
    // the timeline itself, zero at positions that hold no sample of the chunk
    const S* __restrict__ d0 = tod + in0;
    int tdep = tid;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += G) {
      __builtin_amdgcn_sched_barrier(0);
      if (e0 > 0) asm volatile("" : "+v"(tdep) : "v"(v[e0 - 1].y));
      S dv[2 * G];
      bool okv[2 * G];
#pragma unroll
      for (int i = 0; i < 2 * G; ++i) {
        const int pos = 2 * (tdep + T * (e0 + i / 2)) + (i & 1);
        int sp;
        okv[i] = win_pos<kWrap>(pos, ilo, ihi, clen, vlo, sp);
        dv[i] = kWrap ? d0[sp] : ld_off(d0, sp);
      }
#pragma unroll
      for (int i = 0; i < 2 * G; ++i) {
        const C val = okv[i] ? C(dv[i]) : C(0);
        if (i & 1) v[e0 + i / 2].y = val;
        else v[e0 + i / 2].x = val;
      }
    }
    (void)amin;
    (void)amax;
  }
  __syncthreads();  // the FFT reuses the staging area; s_red[0, 2W) holds the valid range

  // ---- forward FFT, spectral step, inverse FFT (outputs in registers)
  static_assert(P::kFft == 3 || (P::kFft == 0 && N == 8192 && std::is_same<C, double>::value),
                "plan and length");
  if constexpr (P::kFft == 3) {
    fs_forward<C, N, T>(buf, v, tw);
    fs_middle<C, N, T>(buf, v, abf);
    fs_inverse<C, N, T>(buf, v, tw);
  } else if constexpr (P::kFft == 0) {
    hpasses<C, N, T, true, 1, 16, 16, 16>(buf, v, tw);
    hmiddle<N, T>(buf, v, abf, tw);
    hpasses<C, N, T, false, 2, 16, 16, 16>(buf, v, tw);
  }

  // ---- P^T through LDS bins in the half buffer
  __syncthreads();  // every thread is done reading buf
  kmin = s_red[0];
  kmax = s_red[W];
#pragma unroll
  for (int w = 1; w < W; ++w) {
    kmin = s_red[w] < kmin ? s_red[w] : kmin;
    kmax = s_red[W + w] > kmax ? s_red[W + w] : kmax;
  }
  if (kmax < kmin) return;
  scatter_bins<S, C, kW, NC, false, false, kSlots, P::kScatterBatch, P>(v, reinterpret_cast<double*>(buf), nullptr, sk,
                                                                     ps0, w0, vlo, vhi, kmin, kmax, q);
}

// One plain tile of one right-hand side per workgroup, two workgroups per
// CU; tiles mapped to workgroups as in k_toeplitz.
template <class S, class C, int kW, int NC, class P, bool kWrap, int kIn>
__global__ __launch_bounds__(P::T, P::kWavesPerEU) void k_toeplitz_half(
    const FftTile* __restrict__ tiles, int64_t n_tiles, int32_t lambda, const cpx<C>* __restrict__ ab,
    const cpx<C>* __restrict__ tw, const int32_t* __restrict__ sample_k, const S* __restrict__ psi,
    const S* __restrict__ wts, const double* __restrict__ x, double* __restrict__ q, RhsBatch rb,
    int32_t variant, const S* __restrict__ tod) {
  int64_t tile;
  int rhs;
  if (variant & kOpLinearOrder) {
    tile = blockIdx.x / rb.nrhs;
    rhs = (int)(blockIdx.x % rb.nrhs);
  } else {
    const int64_t per_xcd = (n_tiles + 7) / 8;
    const int64_t local = blockIdx.x / 8;
    tile = (int64_t)(blockIdx.x % 8) * per_xcd + local / rb.nrhs;
    rhs = (int)(local % rb.nrhs);
  }
  if (tile >= n_tiles) return;
  if (rb.done != nullptr && rb.done[(int64_t)rhs * rb.done_stride]) return;
  x += rhs * rb.vstride;
  q += rhs * rb.vstride;
  const FftTile tl = tiles[tile];
  toeplitz_tile_half<S, C, kW, NC, P, kWrap, kIn>(tl, lambda, ab + (int64_t)tl.filter * P::N, tw, sample_k, psi,
                                                  wts, x, q, tod);
}

// One launch over the tiles of several slots (right-hand sides of different
// solves), through the two-per-CU half-buffer tile.  Every slot's tiles are
// split into 8 contiguous parts and XCD x takes part x of every slot, one
// after the other: each XCD then gets an equal share of every solve (tiles
// of different solves differ in cost) and still walks neighbouring tiles of
// one solve together.  A slot whose done flag is set is skipped, and so is
// one whose chunks wrap differently from kWrap (circulant and band slots of
// one batch take one launch each).
template <class S, class C, int kW, int NC, bool kWrap>
__global__ __launch_bounds__(HPlan<C>::T, HPlan<C>::kWavesPerEU) void k_toeplitz_batch(OpBatch b) {
  const int x = blockIdx.x % 8;
  int64_t j = blockIdx.x / 8;  // position in XCD x's list
  int sl = -1;
  int64_t idx = 0;
  for (int k = 0; k < b.n; ++k) {
    const int64_t n = b.off[k + 1] - b.off[k];
    const int64_t per = (n + 7) / 8;
    const int64_t lo = x * per < n ? x * per : n;
    const int64_t cnt = (lo + per < n ? lo + per : n) - lo;
    if (sl < 0) {
      if (j < cnt) {
        sl = k;
        idx = lo + j;
      } else {
        j -= cnt;
      }
    }
  }
  if (sl < 0) return;
  const OpSlot& o = b.s[sl];
  if ((o.wrap != 0) != kWrap) return;
  if (o.done != nullptr && *o.done != 0) return;
  const FftTile tl = static_cast<const FftTile*>(o.tiles)[idx];
  toeplitz_tile_half<S, C, kW, NC, HPlan<C>, kWrap>(
      tl, o.lambda, static_cast<const cpx<C>*>(o.ab) + (int64_t)tl.filter * HPlan<C>::N,
      static_cast<const cpx<C>*>(o.tw), o.sample_k, static_cast<const S*>(o.psi), static_cast<const S*>(o.wts), o.x,
      o.q);
}

// A half-buffer kernel over the given tiles; circulant chunks (their tiles
// wrap) take the instantiation with the wrap-around positions.
template <class S, class C, int kW, int NC, class P, int kIn = 1>
int launch_half(const mm_pointing_s* pt, const mm_noise_s* nz, const FftTile* tiles, int64_t n_tiles,
                const void* ab, const void* tw, const double* x, double* q, const RhsBatch& rb, hipStream_t s,
                int32_t variant, const void* tod = nullptr) {
  if (n_tiles == 0) return MM_OK;
  const int64_t g = 8 * ((n_tiles + 7) / 8) * rb.nrhs;
  if (nz->kind == 2)
    hipLaunchKernelGGL((k_toeplitz_half<S, C, kW, NC, P, true, kIn>), dim3(g), dim3(P::T), 0, s, tiles, n_tiles,
                       nz->lambda, (const cpx<C>*)ab, (const cpx<C>*)tw, pt->sample_k, (const S*)pt->psi,
                       (const S*)pt->weights, x, q, rb, variant, (const S*)tod);
  else
    hipLaunchKernelGGL((k_toeplitz_half<S, C, kW, NC, P, false, kIn>), dim3(g), dim3(P::T), 0, s, tiles, n_tiles,
                       nz->lambda, (const cpx<C>*)ab, (const cpx<C>*)tw, pt->sample_k, (const S*)pt->psi,
                       (const S*)pt->weights, x, q, rb, variant, (const S*)tod);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

template <class S, class C, int kIn, int kOut, int kW, int NC>
int launch_t(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tod_in, void* tod_out,
             double* q, const RhsBatch& rb, hipStream_t s, int32_t variant) {
  const int a = std::is_same<C, double>::value ? 0 : 1;
  if (nz->n_tiles[a] == 0) return MM_OK;
  // the right-hand side P^T N^-1 d: plain tiles through the half buffer;
  // in FP64 the 16384-point four-step plan (its windows keep 75 % of their
  // samples at lambda = 4096 against 50 %), in FP32 the two-per-CU plan
  if constexpr (kIn == 0 && kOut == 1) {
    if constexpr (std::is_same<C, double>::value)
      return launch_half<S, C, kW, NC, HPlanL64, 0>(pt, nz, nz->tiles[1], nz->n_tiles[1], nz->ab64l, nz->tw64l,
                                                     nullptr, q, rb, s, variant, tod_in);
    else
      return launch_half<S, C, kW, NC, HPlan<C>, 0>(pt, nz, nz->tiles[a], nz->n_tiles[a], nz->abr[a], nz->tw[a],
                                                    nullptr, q, rb, s, variant, tod_in);
  }
  // the longer plan of the arithmetic (bit kOpLongPlan) before any other bit
  if constexpr (kIn == 1 && kOut == 1) {
    if (variant & kOpLongPlan) {
      if constexpr (std::is_same<C, double>::value)
        return launch_half<S, C, kW, NC, HPlanL64>(pt, nz, nz->tiles[1], nz->n_tiles[1], nz->ab64l, nz->tw64l, x, q,
                                                   rb, s, variant);
      else
        return launch_half<S, C, kW, NC, HPlanL32>(pt, nz, nz->tiles32l, nz->n_tiles32l, nz->ab32l, nz->tw32l, x, q,
                                                   rb, s, variant);
    }
  }
  // the halo-carrying form streams stored weights (with psi it spills), or
  // no angle at all (intensity only)
  if constexpr (kIn == 1 && kOut == 1 && (kW == 1 || NC == 1)) {
    if (variant & kOpCarry) {
      if (nz->n_csegs[a] == 0) return MM_OK;
      const int64_t g = 8 * ((nz->n_csegs[a] + 7) / 8) * rb.nrhs;
      hipLaunchKernelGGL((k_toeplitz_carry<S, C, kW, NC>), dim3(g), dim3(Plan<C>::T), 0, s, nz->ctiles[a],
                         nz->csegs[a], nz->n_csegs[a], nz->lambda, (const cpx<C>*)nz->ab[a],
                         (const cpx<C>*)nz->tw[a], pt->sample_k, (const S*)pt->psi,
                         (const S*)pt->weights, x, q, rb, variant);
      MM_HIP(hipGetLastError());
      return MM_OK;
    }
  }
  const int64_t grid = 8 * ((nz->n_tiles[a] + 7) / 8) * rb.nrhs;
  if constexpr (kIn == 1 && kOut == 1) {
    if (variant & kOpHalfLds)
      return launch_half<S, C, kW, NC, HPlan<C>>(pt, nz, nz->tiles[a], nz->n_tiles[a], nz->abr[a], nz->tw[a], x, q, rb,
                                                 s, variant);
  }
  hipLaunchKernelGGL((k_toeplitz<S, C, kIn, kOut, kW, NC>), dim3(grid), dim3(Plan<C>::T), 0, s, nz->tiles[a],
                     nz->n_tiles[a], nz->lambda, (const cpx<C>*)nz->ab[a], (const cpx<C>*)nz->tw[a],
                     pt ? pt->sample_k : nullptr, pt ? (const S*)pt->psi : nullptr,
                     pt ? (const S*)pt->weights : nullptr, x, (const S*)tod_in, (S*)tod_out, q, rb, variant);
  MM_HIP(hipGetLastError());
  return MM_OK;
}

// Stored weights serve an arithmetic no finer than their storage; the
// intensity-only form needs none.
inline bool use_weights(const mm_pointing_s* pt, int arith) {
  return pt != nullptr && pt->ncomp != 1 && pt->weights != nullptr && (arith == MM_F32 || pt->dtype == MM_F64);
}

template <int kIn, int kOut, int NC>
int dispatch_nc(const mm_pointing_s* pt, const mm_noise_s* nz, int dtype, int arith, const double* x,
                const void* tod_in, void* tod_out, double* q, const RhsBatch& rb, hipStream_t s, int32_t variant) {
  const bool w = kOut == 1 && use_weights(pt, arith);
  constexpr int kW1 = NC == 1 ? 0 : 1;  // no weights without an angle
  if (dtype == MM_F64) {
    if (arith == MM_F64)
      return w ? launch_t<double, double, kIn, kOut, kW1, NC>(pt, nz, x, tod_in, tod_out, q, rb, s, variant)
               : launch_t<double, double, kIn, kOut, 0, NC>(pt, nz, x, tod_in, tod_out, q, rb, s, variant);
    return w ? launch_t<double, float, kIn, kOut, kW1, NC>(pt, nz, x, tod_in, tod_out, q, rb, s, variant)
             : launch_t<double, float, kIn, kOut, 0, NC>(pt, nz, x, tod_in, tod_out, q, rb, s, variant);
  }
  if (arith == MM_F64)
    return launch_t<float, double, kIn, kOut, 0, NC>(pt, nz, x, tod_in, tod_out, q, rb, s, variant);
  return w ? launch_t<float, float, kIn, kOut, kW1, NC>(pt, nz, x, tod_in, tod_out, q, rb, s, variant)
           : launch_t<float, float, kIn, kOut, 0, NC>(pt, nz, x, tod_in, tod_out, q, rb, s, variant);
}

// The map form matters only where the pointing is applied (kIn or kOut).
template <int kIn, int kOut>
int dispatch(const mm_pointing_s* pt, const mm_noise_s* nz, int dtype, int arith, const double* x,
             const void* tod_in, void* tod_out, double* q, const RhsBatch& rb, hipStream_t s, int32_t variant) {
  if constexpr (kIn == 0 && kOut == 0) {
    return dispatch_nc<0, 0, 3>(pt, nz, dtype, arith, x, tod_in, tod_out, q, rb, s, variant);
  } else {
    return by_ncomp(pt->ncomp, [&]<int NC>() -> int {
      return dispatch_nc<kIn, kOut, NC>(pt, nz, dtype, arith, x, tod_in, tod_out, q, rb, s, variant);
    });
  }
}

template <int NC>
int launch_batch_nc(const OpBatch& b, dim3 grid, int dtype, int arith, bool weights, bool wrap, hipStream_t s) {
  const int T = arith == MM_F64 ? HPlan<double>::T : HPlan<float>::T;
  constexpr int kW1 = NC == 1 ? 0 : 1;  // no weights without an angle
  auto go = [&]<class S, class C, int kW>() {
    if (wrap) hipLaunchKernelGGL((k_toeplitz_batch<S, C, kW, NC, true>), grid, dim3(T), 0, s, b);
    else hipLaunchKernelGGL((k_toeplitz_batch<S, C, kW, NC, false>), grid, dim3(T), 0, s, b);
  };
  if (dtype == MM_F64) {
    if (arith == MM_F64) {
      if (weights) go.template operator()<double, double, kW1>();
      else go.template operator()<double, double, 0>();
    } else {
      if (weights) go.template operator()<double, float, kW1>();
      else go.template operator()<double, float, 0>();
    }
  } else {
    if (arith == MM_F64) {
      go.template operator()<float, double, 0>();
    } else {
      if (weights) go.template operator()<float, float, kW1>();
      else go.template operator()<float, float, 0>();
    }
  }
  MM_HIP(hipGetLastError());
  return MM_OK;
}

}  // namespace

int launch_toeplitz_batch(const OpBatch& b, int dtype, int arith, bool weights, int ncomp, hipStream_t s) {
  if (b.n == 0) return MM_OK;
  // XCD x's list holds up to ceil(n_s / 8) tiles of every slot s
  int64_t per_xcd = 0;
  for (int k = 0; k < b.n; ++k) per_xcd += (b.off[k + 1] - b.off[k] + 7) / 8;
  if (per_xcd == 0) return MM_OK;
  const dim3 grid((unsigned)(8 * per_xcd));
  bool any_wrap = false, any_band = false;
  for (int k = 0; k < b.n; ++k) (b.s[k].wrap ? any_wrap : any_band) = true;
  for (const bool wrap : {false, true}) {
    if (!(wrap ? any_wrap : any_band)) continue;
    if (int rc = by_ncomp(ncomp, [&]<int NC>() -> int {
          return launch_batch_nc<NC>(b, grid, dtype, arith, weights, wrap, s);
        }))
      return rc;
  }
  return MM_OK;
}

int launch_ninv_toeplitz(const mm_pointing_s* pt, const mm_noise_s* nz, const void* in, void* out, int arith,
                         hipStream_t s) {
  return dispatch<0, 0>(pt, nz, pt->dtype, arith, nullptr, in, out, nullptr, RhsBatch{}, s, 0);
}

int launch_fused_toeplitz(const mm_pointing_s* pt, const mm_noise_s* nz, const double* x, const void* tod,
                          double* q, int arith, const RhsBatch& rb, hipStream_t s, int32_t variant) {
  if (pt->n_kept == 0) return MM_OK;  // nothing to gather or scatter (the kernels assume a kept pixel)
  if (x != nullptr) return dispatch<1, 1>(pt, nz, pt->dtype, arith, x, nullptr, nullptr, q, rb, s, variant);
  return dispatch<0, 1>(pt, nz, pt->dtype, arith, nullptr, tod, nullptr, q, rb, s, variant);
}

}  // namespace mm
