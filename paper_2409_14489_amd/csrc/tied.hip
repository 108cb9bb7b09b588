// Tied coefficients of the paper's fitting protocol (Sec. III-B, assumptions
// (i)-(iii)): one row c_h of applied coefficients per subband distance h,
// shared by all subband pairs at that distance (eq. (23)), mirrored for the
// pairs below the diagonal (eq. (24)), even for h = 0 (eq. (25)), and scaled
// by a weight w_s per step:
//   C[s][i][l][m] = w_s c_{l-i}[m]  (l >= i),   C[s][i][l][m] = w_s c_{i-l}[-m]  (l < i),
// zero where |m| > Nc(|l - i|).  Of row 0 only the taps m >= 0 are read.
//
// tie_expand_kernel writes the applied tensor; tie_reduce_kernel is its
// transpose (the gradient of a loss with respect to the rows, given its
// gradient with respect to the tensor), summed in FP64 in a fixed order.
#include <hip/hip_runtime.h>

#include "cbessfm.h"
#include "internal.hpp"

namespace cbessfm {
namespace {

struct TieShape {
  int steps, n_sb, n_taps;
  int half[kMaxSubbands];  // Nc(h)
};

// Row-major index into params of the coefficient that C[.][i][l][t] reads, or -1.
__device__ __forceinline__ int tie_source(const TieShape& sh, int i, int l, int t) {
  const int nc = sh.n_taps / 2;
  const int h = l >= i ? l - i : i - l;
  int m = t - nc;
  if (l < i) m = -m;
  if (h == 0 && m < 0) m = -m;
  if (m > sh.half[h] || -m > sh.half[h]) return -1;
  return h * sh.n_taps + m + nc;
}

__global__ __launch_bounds__(256) void tie_expand_kernel(const float* __restrict__ params,
                                                         const float* __restrict__ w, TieShape sh,
                                                         float* __restrict__ out) {
  const int per_step = sh.n_sb * sh.n_sb * sh.n_taps;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)sh.steps * per_step) return;
  const int s = (int)(idx / per_step);
  int r = (int)(idx - (long long)s * per_step);
  const int t = r % sh.n_taps;
  r /= sh.n_taps;
  const int l = r % sh.n_sb;
  const int i = r / sh.n_sb;
  const int src = tie_source(sh, i, l, t);
  out[idx] = src < 0 ? 0.0f : w[s] * params[src];
}

// One thread per parameter (h, tt).  Its pre-image in C: for h > 0 the pairs
// (i, i + h) at tap tt and (i + h, i) at the mirrored tap; for h = 0 the
// diagonal at tap tt and, unless m = 0, at the mirrored tap.
__global__ __launch_bounds__(256) void tie_reduce_kernel(const float* __restrict__ g,
                                                         const float* __restrict__ w, TieShape sh,
                                                         float* __restrict__ gp) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= sh.n_sb * sh.n_taps) return;
  const int h = idx / sh.n_taps, tt = idx - h * sh.n_taps;
  const int nc = sh.n_taps / 2, m = tt - nc;
  const int nsb = sh.n_sb, taps = sh.n_taps;
  if ((h == 0 && m < 0) || m > sh.half[h] || -m > sh.half[h]) {
    gp[idx] = 0.0f;
    return;
  }
  const int mirror = nc - m;  // tap of -m
  const bool two = h > 0 || m != 0;
  double acc = 0.0;
  for (int s = 0; s < sh.steps; ++s) {
    const float* gs = g + (size_t)s * nsb * nsb * taps;
    double part = 0.0;
    for (int i = 0; i + h < nsb; ++i) {
      part += (double)gs[((size_t)i * nsb + i + h) * taps + tt];
      if (two) part += (double)gs[((size_t)(i + h) * nsb + i) * taps + mirror];
    }
    acc += (double)w[s] * part;
  }
  gp[idx] = (float)acc;
}

int tie_shape(int steps, int n_sb, int n_taps, const int32_t* half_taps, TieShape& sh) {
  if (steps < 1 || n_sb < 1 || n_sb > kMaxSubbands || n_taps < 1 || (n_taps & 1) == 0 || n_taps > kMaxTaps)
    return CBESSFM_EINVAL;
  sh.steps = steps;
  sh.n_sb = n_sb;
  sh.n_taps = n_taps;
  for (int h = 0; h < kMaxSubbands; ++h) {
    sh.half[h] = -1;
    if (h >= n_sb) continue;
    const int v = half_taps ? half_taps[h] : n_taps / 2;
    if (v < 0 || v > n_taps / 2) return CBESSFM_EINVAL;
    sh.half[h] = v;
  }
  return CBESSFM_OK;
}

}  // namespace
}  // namespace cbessfm

using cbessfm::TieShape;

int cbessfm_tie_expand(const float* params, const float* weights, int32_t steps, int32_t n_sb, int32_t n_taps,
                       const int32_t* half_taps, float* coeffs, void* stream) {
  TieShape sh;
  const int rc = cbessfm::tie_shape(steps, n_sb, n_taps, half_taps, sh);
  if (rc) return rc;
  if (!params || !weights || !coeffs) return CBESSFM_EINVAL;
  const long long total = (long long)steps * n_sb * n_sb * n_taps;
  hipLaunchKernelGGL(cbessfm::tie_expand_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), params, weights, sh, coeffs);
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

int cbessfm_tie_reduce(const float* grad_c, const float* weights, int32_t steps, int32_t n_sb, int32_t n_taps,
                       const int32_t* half_taps, float* grad_params, void* stream) {
  TieShape sh;
  const int rc = cbessfm::tie_shape(steps, n_sb, n_taps, half_taps, sh);
  if (rc) return rc;
  if (!grad_c || !weights || !grad_params) return CBESSFM_EINVAL;
  const int total = n_sb * n_taps;
  hipLaunchKernelGGL(cbessfm::tie_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), grad_c, weights, sh, grad_params);
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}
