// (cos 2psi, sin 2psi) of eq. (2) from a stored angle psi (FP64 or FP32) in a
// chosen arithmetic C.
//
// Argument reduction x = 2 psi = j pi/2 + r, |r| <= pi/4, in FP64 with pi/2
// split into four parts (Cody & Waite, "Software Manual for the Elementary
// Functions", 1980): the first three carry 25 significant bits, so j times
// each of them is exact for |j| < 2^28, and the reduction error stays near
// one ulp of r for |x| < kReduceMax.  sin r and cos r come from their Taylor
// series in Horner form (truncation below 1e-19 relative on |r| <= pi/4 in
// FP64, below 2e-9 in FP32), and the quadrant j mod 4 permutes and negates
// them.  There is no slow path: the pointing build rejects angles with
// |2 psi| >= kReduceMax (or non-finite), so every kernel stays call-free.
#pragma once
#include <hip/hip_runtime.h>

namespace mm {

namespace sc {
constexpr double kPio2A = 1.5707963109016418;      // 0x1.921fb5p+0
constexpr double kPio2B = 1.5893254712295857e-08;  // 0x1.110b46p-26
constexpr double kPio2C = 6.123233932053594e-17;   // 0x1.1a6263p-54
constexpr double kPio2D = 6.36831716351095e-25;    // 0x1.8a2e03707344ap-81
constexpr double kTwoOverPi = 0.63661977236758134308;
constexpr double kReduceMax = 4.0e8;  // < 2^28 * pi/2

// x = j pi/2 + r; returns r and j mod 4
__device__ __forceinline__ double reduce(double x, int* q) {
  const double j = rint(x * kTwoOverPi);
  double r = fma(-j, kPio2A, x);
  r = fma(-j, kPio2B, r);
  r = fma(-j, kPio2C, r);
  r = fma(-j, kPio2D, r);
  *q = (int)(long long)j & 3;
  return r;
}

template <class C>
__device__ __forceinline__ void quadrant(int q, C sr, C cr, C* s, C* c) {
  const C s0 = (q & 1) ? cr : sr;
  const C c0 = (q & 1) ? sr : cr;
  *s = (q & 2) ? -s0 : s0;
  *c = ((q + 1) & 2) ? -c0 : c0;
}

__device__ __forceinline__ void poly_f64(double r, double* sr, double* cr) {
  const double u = r * r;
  double ps = 2.8114572543455206e-15;        // 1/17!
  ps = fma(ps, u, -7.647163731819816e-13);   // -1/15!
  ps = fma(ps, u, 1.6059043836821613e-10);   // 1/13!
  ps = fma(ps, u, -2.505210838544172e-08);   // -1/11!
  ps = fma(ps, u, 2.7557319223985893e-06);   // 1/9!
  ps = fma(ps, u, -0.0001984126984126984);   // -1/7!
  ps = fma(ps, u, 0.008333333333333333);     // 1/5!
  ps = fma(ps, u, -0.16666666666666666);     // -1/3!
  *sr = fma(r * u, ps, r);
  double pc = -1.5619206968586225e-16;       // -1/18!
  pc = fma(pc, u, 4.779477332387385e-14);    // 1/16!
  pc = fma(pc, u, -1.1470745597729725e-11);  // -1/14!
  pc = fma(pc, u, 2.08767569878681e-09);     // 1/12!
  pc = fma(pc, u, -2.755731922398589e-07);   // -1/10!
  pc = fma(pc, u, 2.48015873015873e-05);     // 1/8!
  pc = fma(pc, u, -0.001388888888888889);    // -1/6!
  pc = fma(pc, u, 0.041666666666666664);     // 1/4!
  pc = fma(pc, u, -0.5);                     // -1/2!
  *cr = fma(u, pc, 1.0);
}

__device__ __forceinline__ void poly_f32(float r, float* sr, float* cr) {
  const float u = r * r;
  float ps = 2.7557319e-06f;          // 1/9!
  ps = fmaf(ps, u, -1.9841270e-04f);  // -1/7!
  ps = fmaf(ps, u, 8.3333333e-03f);   // 1/5!
  ps = fmaf(ps, u, -1.6666667e-01f);  // -1/3!
  *sr = fmaf(r * u, ps, r);
  float pc = -2.7557319e-07f;         // -1/10!
  pc = fmaf(pc, u, 2.4801587e-05f);   // 1/8!
  pc = fmaf(pc, u, -1.3888889e-03f);  // -1/6!
  pc = fmaf(pc, u, 4.1666667e-02f);   // 1/4!
  pc = fmaf(pc, u, -0.5f);            // -1/2!
  *cr = fmaf(u, pc, 1.0f);
}
}  // namespace sc

// sin and cos of an FP64 argument with |x| < kReduceMax
__device__ __forceinline__ void sincos_x(double x, double* s, double* c) {
  int q;
  const double r = sc::reduce(x, &q);
  double sr, cr;
  sc::poly_f64(r, &sr, &cr);
  sc::quadrant<double>(q, sr, cr, s, c);
}

// the same to FP32 accuracy
__device__ __forceinline__ void sincos_x(double x, float* s, float* c) {
  int q;
  const float r = float(sc::reduce(x, &q));
  float sr, cr;
  sc::poly_f32(r, &sr, &cr);
  sc::quadrant<float>(q, sr, cr, s, c);
}

template <class C, class S>
__device__ __forceinline__ void sincos2(S psi, C* c, C* s) {
  sincos_x(2.0 * double(psi), s, c);
}

// 1 / d for d >= 1: the hardware estimate refined by Newton steps
// r <- r + r (1 - d r), each of which squares the relative error.
__device__ __forceinline__ double recip_ge1(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  r = fma(r, fma(-d, r, 1.0), r);
  return r;
}
__device__ __forceinline__ float recip_ge1(float d) {
  float r = __builtin_amdgcn_rcpf(d);
  return fmaf(r, fmaf(-d, r, 1.0f), r);
}

// (cos 2psi, sin 2psi) from the stored tangent u = tan psi, by the
// half-angle (Weierstrass) substitution: cos 2psi = (1 - u^2) / (1 + u^2),
// sin 2psi = 2u / (1 + u^2).  u is finite for every stored angle (no FP64 or
// FP32 number is an odd multiple of pi/2), a relative error e in u moves the
// angle 2psi by at most e, and 1 + u^2 >= 1 keeps the reciprocal well
// conditioned: a few multiplies instead of a reduction and two polynomials.
template <class C, class S>
__device__ __forceinline__ void from_tangent(S u, C* c, C* s) {
  const C v = C(u);
  const C v2 = v * v;
  const C r = recip_ge1(C(1) + v2);
  *c = (C(1) - v2) * r;
  *s = (v + v) * r;
}

}  // namespace mm
