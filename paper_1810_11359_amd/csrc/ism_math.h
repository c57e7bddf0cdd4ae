// Device math shared by the HIP sources of the library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace ism {

// pi^k / k!, the Taylor coefficients of sin(pi r) (odd k) and cos(pi r) (even k).
constexpr double kPiPow1 = 3.14159265358979323846;
constexpr double kPiPow2 = kPiPow1 * kPiPow1;
constexpr double kPiPow3 = kPiPow2 * kPiPow1;
constexpr double kPiPow4 = kPiPow3 * kPiPow1;
constexpr double kPiPow5 = kPiPow4 * kPiPow1;
constexpr double kPiPow6 = kPiPow5 * kPiPow1;
constexpr double kPiPow7 = kPiPow6 * kPiPow1;
constexpr double kPiPow8 = kPiPow7 * kPiPow1;
constexpr double kPiPow9 = kPiPow8 * kPiPow1;
constexpr double kPiPow10 = kPiPow9 * kPiPow1;

// sin(pi x) and cos(pi x) in FP32 for |x| < 2^22, to a few ulp. x is reduced
// exactly to r = x - n/2 with n = rint(2x) (|r| <= 1/4); sin(pi r) and
// cos(pi r) are summed from their Taylor series to degree 9 and 10 (the first
// omitted terms are below 2e-10 at |pi r| <= pi/4), with coefficients
// pi^k / k! rounded to FP32, and rotated by the quadrant n mod 4.
__device__ __forceinline__ void sincospi_acc(float x, float &s, float &c) {
  const float n = __builtin_rintf(2.0f * x);
  const float r = __builtin_fmaf(n, -0.5f, x);  // exact
  const float r2 = r * r;
  constexpr float S1 = (float)kPiPow1, S3 = (float)(-kPiPow3 / 6.0), S5 = (float)(kPiPow5 / 120.0),
                  S7 = (float)(-kPiPow7 / 5040.0), S9 = (float)(kPiPow9 / 362880.0);
  constexpr float C2 = (float)(-kPiPow2 / 2.0), C4 = (float)(kPiPow4 / 24.0), C6 = (float)(-kPiPow6 / 720.0),
                  C8 = (float)(kPiPow8 / 40320.0), C10 = (float)(-kPiPow10 / 3628800.0);
  float ps = __builtin_fmaf(r2, S9, S7);
  ps = __builtin_fmaf(r2, ps, S5);
  ps = __builtin_fmaf(r2, ps, S3);
  ps = __builtin_fmaf(r2, ps, S1);
  const float sr = r * ps;
  float pc = __builtin_fmaf(r2, C10, C8);
  pc = __builtin_fmaf(r2, pc, C6);
  pc = __builtin_fmaf(r2, pc, C4);
  pc = __builtin_fmaf(r2, pc, C2);
  const float cr = __builtin_fmaf(r2, pc, 1.0f);
  const int q = ((int)n) & 3;
  s = q == 0 ? sr : q == 1 ? cr : q == 2 ? -sr : -cr;
  c = q == 0 ? cr : q == 1 ? -sr : q == 2 ? -cr : sr;
}

}  // namespace ism
