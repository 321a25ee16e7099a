// Map forms: the columns of the pointing row a sample sees, per number of
// unknowns per pixel NC.  IQU (NC = 3): (1, cos 2psi, sin 2psi) of eq. (8);
// QU (NC = 2): the two angle columns; I (NC = 1): the constant column.  The
// reduced pixel-domain vector then holds NC values per kept pixel, the two-
// or three-fold size Sec. III-B names.
#pragma once
#include <hip/hip_runtime.h>

namespace mm {

template <int NC>
struct Stokes {
  static_assert(NC >= 1 && NC <= 3, "1, 2 or 3 values per pixel");
  static constexpr bool kAngle = NC != 1;  // the row needs cos/sin of 2 psi
  static constexpr int kBlock = NC * (NC + 1) / 2;

  // P x at one sample: the row times the pixel's NC values.
  template <class C>
  static __device__ __forceinline__ C project(const double* __restrict__ xk, C c, C s) {
    if constexpr (NC == 3) return C(xk[0]) + c * C(xk[1]) + s * C(xk[2]);
    else if constexpr (NC == 2) return c * C(xk[0]) + s * C(xk[1]);
    else return C(xk[0]);
  }

  // The P^T terms of one sample with timeline value z: z times the row.
  template <class C>
  static __device__ __forceinline__ void terms(C z, C c, C s, double* o) {
    if constexpr (NC == 3) {
      o[0] = double(z);
      o[1] = double(z * c);
      o[2] = double(z * s);
    } else if constexpr (NC == 2) {
      o[0] = double(z * c);
      o[1] = double(z * s);
    } else {
      o[0] = double(z);
    }
  }
};

}  // namespace mm
