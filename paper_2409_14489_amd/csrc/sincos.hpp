// sin and cos of a nonlinear phase (the rotation of eq. (3)) in FP32.
//
// Cody-Waite reduction x = k pi/2 + r with pi/2 in three FP32 parts (products
// by FMA), |r| <= pi/4, then polynomials in r^2 fitted by least squares on
// Chebyshev nodes of [0, pi/4] (gen_sincos.py writes the constants and the
// worst error: 4.2e-8 for sin, 6.5e-8 for cos, under one FP32 ulp of 1), and
// the quadrant k mod 4.  Accurate for |x| < 2^22 pi/2; beyond that the
// reduction loses accuracy but the result keeps s^2 + c^2 close to 1.  It
// takes a few registers, where the general-purpose sincosf keeps its
// large-argument path live in many.
#pragma once

#include <hip/hip_runtime.h>

namespace cbessfm {

__device__ __forceinline__ void phase_sincos(float x, float& s, float& c) {
  constexpr float kTwoOverPi = 0.636619772367581343f;
  constexpr float kPio2Hi = 1.5707963705062866f;
  constexpr float kPio2Mid = -4.371138828673793e-08f;
  constexpr float kPio2Lo = -1.7763568394002505e-15f;
  constexpr float S0 = -0.1666666716337204f, S1 = 0.008333329111337662f, S2 = -0.00019839353626593947f,
                  S3 = 2.7184505597688258e-06f;
  constexpr float C0 = -0.5f, C1 = 0.04166662320494652f, C2 = -0.0013886808883398771f,
                  C3 = 2.439408672216814e-05f;
  const float k = rintf(x * kTwoOverPi);
  float r = fmaf(-k, kPio2Hi, x);
  r = fmaf(-k, kPio2Mid, r);
  r = fmaf(-k, kPio2Lo, r);
  const float r2 = r * r;
  const float ps = fmaf(fmaf(fmaf(S3, r2, S2), r2, S1), r2, S0);
  const float pc = fmaf(fmaf(fmaf(C3, r2, C2), r2, C1), r2, C0);
  const float sr = fmaf(r * r2, ps, r);
  const float cr = fmaf(r2, pc, 1.0f);
  const int q = (int)k & 3;  // quadrant of x; two's complement keeps k mod 4 for negative k
  // sin x = sr, cr, -sr, -cr and cos x = cr, -sr, -cr, sr for q = 0, 1, 2, 3
  const float s0 = (q & 1) ? cr : sr;
  const float c0 = (q & 1) ? sr : cr;
  s = (q & 2) ? -s0 : s0;
  c = ((q + 1) & 2) ? -c0 : c0;
}

}  // namespace cbessfm
