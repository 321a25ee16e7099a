// Workgroup-wide complex FFT of compile-time length N held in LDS and
// registers (Stockham autosort: natural order in and out, one LDS exchange
// per pass).  Each of T threads keeps E = N/T elements in registers; thread
// `tid` always owns elements tid + T*e, e = 0..E-1, before the first pass
// and after the last one, so producers and consumers of the timeline can
// address their samples directly.
//
// Pass with radix R and span Ns (product of the radices before it): for each
// butterfly j in [0, N/R), with k = j mod Ns, the inputs a_m = in[j + m N/R]
// are multiplied by w^(m k) with w = exp(-+2 pi i / (Ns R)), transformed by
// an R-point DFT, and output q goes to out[(j / Ns) Ns R + k + q Ns]
// (the decimation-in-time Stockham formulation, e.g. Van Loan, "Computational
// Frameworks for the Fast Fourier Transform", Sec. 1.7).
#pragma once
#include <hip/hip_runtime.h>

namespace mm {

template <class C>
struct cpx {
  C x, y;
};

template <class C>
__device__ __forceinline__ cpx<C> cadd(cpx<C> a, cpx<C> b) { return {a.x + b.x, a.y + b.y}; }
template <class C>
__device__ __forceinline__ cpx<C> csub(cpx<C> a, cpx<C> b) { return {a.x - b.x, a.y - b.y}; }
template <class C>
__device__ __forceinline__ cpx<C> cmul(cpx<C> a, cpx<C> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// cos(2 pi i / 64) for i = 0..16 (quarter wave; entry 16 is exactly 0).
__device__ constexpr double kCos64[17] = {
    1.0,
    0.99518472667219693,
    0.98078528040323043,
    0.95694033573220882,
    0.92387953251128674,
    0.88192126434835505,
    0.83146961230254524,
    0.77301045336273699,
    0.70710678118654757,
    0.63439328416364549,
    0.55557023301960218,
    0.47139673682599764,
    0.38268343236508978,
    0.29028467725446233,
    0.19509032201612828,
    0.098017140329560604,
    0.0};

// a * exp(sign * 2 pi i * idx / 64), sign = -1 forward, +1 inverse.  idx is a
// compile-time constant after unrolling, so the quarter-turn cases fold to
// swaps and sign flips and the eighth-turn cases to two multiplies.
template <class C, bool kFwd>
__device__ __forceinline__ cpx<C> rot64(cpx<C> a, int idx) {
  idx &= 63;
  const int q = idx >> 4, r = idx & 15;
  if (r == 0) {
    // multiply by (-i)^q forward, i^q inverse
    const int qq = kFwd ? q : (4 - q) & 3;
    if (qq == 0) return a;
    if (qq == 1) return {a.y, -a.x};   // * (-i)
    if (qq == 2) return {-a.x, -a.y};  // * (-1)
    return {-a.y, a.x};                // * (+i)
  }
  if (r == 8) {
    // eighth turns: rotate by -+pi/4 with two multiplies, then by the
    // remaining quarter turns ((-i)^q forward, i^q inverse)
    const C h = C(0.70710678118654757);
    const cpx<C> t = kFwd ? cpx<C>{(a.x + a.y) * h, (a.y - a.x) * h} : cpx<C>{(a.x - a.y) * h, (a.x + a.y) * h};
    const int qt = kFwd ? (4 - q) & 3 : q;  // number of +i rotations
    if (qt == 0) return t;
    if (qt == 1) return {-t.y, t.x};
    if (qt == 2) return {-t.x, -t.y};
    return {t.y, -t.x};
  }
  C c = C(kCos64[r]), s = C(kCos64[16 - r]);
  // rotate (c, s) by q quarter turns: angle 2 pi idx / 64
  C cc, ss;
  if (q == 0) { cc = c; ss = s; }
  else if (q == 1) { cc = -s; ss = c; }
  else if (q == 2) { cc = -c; ss = -s; }
  else { cc = s; ss = -c; }
  if (kFwd) ss = -ss;
  return cmul(a, cpx<C>{cc, ss});
}

// In-register R-point DFT (R a power of two <= 32), natural order in/out:
// radix-2 decimation in time after a compile-time bit reversal.
template <int R>
__device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

template <class C, int R, bool kFwd>
__device__ __forceinline__ void dft_reg(cpx<C>* a) {
  cpx<C> t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[bitrev<R>(i)] = a[i];
#pragma unroll
  for (int len = 2; len <= R; len <<= 1) {
    const int half = len >> 1;
#pragma unroll
    for (int g = 0; g < R; g += len) {
#pragma unroll
      for (int j = 0; j < half; ++j) {
        const cpx<C> u = t[g + j];
        const cpx<C> v = rot64<C, kFwd>(t[g + j + half], j * (64 / len));
        t[g + j] = cadd(u, v);
        t[g + j + half] = csub(u, v);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = t[i];
}

// Thread index as an opaque value: each pass derives its LDS addresses from
// it afresh, so the compiler cannot hoist (and keep live, or spill) the
// addresses of every pass when the FFT runs inside a loop over tiles.
__device__ __forceinline__ int fft_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// LDS index with one pad element every 16, which staggers the strided
// accesses of the passes across banks.
__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }
template <int N>
constexpr int lds_elems() { return N + N / 16; }
// lds_pad(i + d) - lds_pad(i) for d a multiple of 16, or d = q Ns with Ns
// dividing 16 and i mod 16 < Ns: one padded address per butterfly, the other
// inputs or outputs at constant offsets from it.
constexpr int lds_step(int d) { return d + (d >> 4); }

// Twiddle by w^(m k), then DFT, for the BPT butterflies held in v.
template <class C, int N, int T, int R, int Ns, bool kFwd>
__device__ __forceinline__ void pass_compute(cpx<C>* v, const cpx<C>* __restrict__ tw) {
  constexpr int E = N / T;
  constexpr int BPT = E / R;
  static_assert(BPT * R == E, "radix must divide the elements per thread");
  const int tid = fft_tid();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    cpx<C>* a = v + b * R;
    if (Ns > 1) {
      const int j = tid + b * T;
      const int k = j & (Ns - 1);
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

template <class C, int N, int T, int R, int Ns>
__device__ __forceinline__ void pass_store(cpx<C>* buf, const cpx<C>* v) {
  constexpr int BPT = N / T / R;
  static_assert(Ns % 16 == 0 || (16 % Ns == 0 && (Ns * R) % 16 == 0), "offsets q Ns must keep the pad count");
  const int tid = fft_tid();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = tid + b * T;
    const int pb = lds_pad((j / Ns) * Ns * R + (j & (Ns - 1)));
#pragma unroll
    for (int q = 0; q < R; ++q) buf[pb + lds_step(q * Ns)] = v[b * R + q];
  }
}

template <class C, int N, int T, int R>
__device__ __forceinline__ void pass_load(const cpx<C>* buf, cpx<C>* v) {
  constexpr int BPT = N / T / R;
  static_assert((N / R) % 16 == 0, "input stride must keep the pad count");
  const int tid = fft_tid();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int pj = lds_pad(tid + b * T);
#pragma unroll
    for (int m = 0; m < R; ++m) v[b * R + m] = buf[pj + lds_step(m * (N / R))];
  }
}

// Register slot of element tid + T*e before a first pass / after a last
// pass of radix R: butterfly b = e mod BPT, input/output m = e / BPT.
template <int N, int T, int R>
__device__ constexpr int slot_of(int e) {
  constexpr int BPT = N / T / R;
  return (e % BPT) * R + e / BPT;
}

}  // namespace mm
