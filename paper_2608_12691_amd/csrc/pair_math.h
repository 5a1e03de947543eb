// Device math shared by the kernels: the fitted erfc of the FP32 pair
// arithmetic and the LBF switching functions of eqs. 7-10.
#pragma once
#include <hip/hip_runtime.h>

#include "erfc_coeffs.h"

namespace anb {

// erfc(x) and exp(-x^2) for 0 <= x <= ANB_ERFC_XMAX: in FP32 from the fit of
// erfc_coeffs.h (relative error 1.5e-8), in FP64 from the library
__device__ inline void erfc_exp(float x, float& ec, float& ex) {
  const float t = __builtin_amdgcn_rcpf(fmaf(ANB_ERFC_P, x, 1.0f));
  float p = kErfcCoef[ANB_ERFC_DEG];
#pragma unroll
  for (int k = ANB_ERFC_DEG - 1; k >= 0; --k) p = fmaf(p, t, kErfcCoef[k]);
  ex = __builtin_amdgcn_exp2f((x * x) * -1.4426950408889634f);
  ec = t * p * ex;
}
__device__ inline void erfc_exp(double x, double& ec, double& ex) {
  ex = exp(-x * x);
  ec = erfc(x);
}

// hA = S32((l - 0.35)/0.65) and hB = S22(l) - hA with their l-derivatives
// (the paper's eqs. 7-10; l in [0, 1])
__host__ __device__ inline void lbf_switch(double l, double& hA, double& hB, double& dhA, double& dhB) {
  const double x = (l - 0.35) / 0.65;
  hA = 0.0;
  dhA = 0.0;
  if (x > 0.0) {
    const double xc = x < 1.0 ? x : 1.0;
    hA = xc * xc * xc * xc * (15.0 + xc * (-24.0 + 10.0 * xc));
    dhA = x < 1.0 ? 60.0 * xc * xc * xc * (1.0 - xc) * (1.0 - xc) / 0.65 : 0.0;
  }
  const double s22 = l * l * l * (10.0 + l * (-15.0 + 6.0 * l));
  const double ds22 = 30.0 * l * l * (1.0 - l) * (1.0 - l);
  hB = s22 - hA;
  dhB = ds22 - dhA;
}

}  // namespace anb
