// CB-ESSFM forward kernel for gfx950 (MI355X).
//
// One persistent launch processes every overlap-and-save block of every batch
// instance (Sec. III-A).  A "team" of N_sb workgroups handles one block at a
// time; workgroup i of the team owns subband i (and, at the block's input and
// output, the polyphase component i of the size-N DFT).  Within a workgroup the
// subband's two polarisations live in registers for the whole step loop
// (layout contract of fft_lds.hpp); LDS is only used for the FFT pass
// exchanges and the coupled-intensity filter.  HBM is touched when the block
// is read and written; team members exchange intensities (once per step) and
// spectra (at the block's input and output) through tagged words that stay in
// the caches (team.hpp).
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "internal.hpp"
#include "team.hpp"

namespace cbessfm {

// Coupled intensity filter of eq. (15) for subband `me`, circular over N':
//   theta[k] = sum_l sum_tau C[s][me][l][tau] p_l[(k - tau + nc) mod N'].
// p_own holds this workgroup's intensities at positions t + NT o; on return
// theta holds the phase at the same positions.  For n_sb > 1 the team's rows
// come from the tagged exchange row `xrow` ([n_sb][N'], round `tag`).
template <int N>
__device__ __forceinline__ void coupled_fir(const FwdArgs& a, const float* __restrict__ crow, int me,
                                           uint64_t* xrow, unsigned tag, const float (&p_own)[FftShape<N>::RR],
                                           float (&theta)[FftShape<N>::RR], float* lf) {
  using S = FftShape<N>;
  constexpr int RR = S::RR, NT = S::NT;
  const int t = opaque_tid();
  const int nsb = a.n_sb;
  const int nc = a.nc;
  const int tap_pad = kTapChunk * a.n_chunks;
  const int hl = tap_pad - 1 - nc;  // left halo of the circular extension
  constexpr int PB = NlprLds<N>::PB;  // row l lives at lf + (l & 1) * PB
  float* th = lf + 2 * PB;

  if (nsb > 1) {
#pragma unroll
    for (int o = 0; o < RR; ++o) xput(xrow + (size_t)me * N + t + NT * o, p_own[o], tag);
  }
  __syncthreads();  // the LDS rows alias the FFT exchange buffers
  {
    float v[RR];
    if (nsb > 1 && me != 0) {
      xget<RR>(xrow, t, NT, tag, a.ctl, v);
      stage_row<N, RR, NT>(lf, v, t, hl, nc);
    } else {
      stage_row<N, RR, NT>(lf, p_own, t, hl, nc);
    }
  }
  __syncthreads();

  float acc[RR];
#pragma unroll
  for (int q = 0; q < RR; ++q) acc[q] = 0.0f;
  for (int l = 0; l < nsb; ++l) {
    const float* cur = lf + (l & 1) * PB;
    const bool fetch = (l + 1 < nsb) && (l + 1 != me);  // next row is remote
    uint64_t w[RR];
    if (fetch) xissue<RR>(xrow + (size_t)(l + 1) * N, t, NT, w);  // in flight during the filter
    const float* cl = crow + (size_t)l * tap_pad;
    for (int c = 0; c < a.n_chunks; ++c) {
      // window w in [0, RR + 7): p index t RR + w - 7 - 8 c + nc, stored at + hl
      float win[RR + kTapChunk - 1];
      const int base = t * RR - (kTapChunk - 1) - kTapChunk * c + nc + hl;
#pragma unroll
      for (int i = 0; i < RR + kTapChunk - 1; ++i) win[i] = cur[pad_f(base + i)];
#pragma unroll
      for (int tt = 0; tt < kTapChunk; ++tt) {
        const float cf = cl[kTapChunk * c + tt];
#pragma unroll
        for (int q = 0; q < RR; ++q) acc[q] = fmaf(cf, win[q - tt + kTapChunk - 1], acc[q]);
      }
    }
    if (l + 1 < nsb) {
      if (fetch) {
        float v[RR];
        xcomplete<RR>(xrow + (size_t)(l + 1) * N, t, NT, tag, a.ctl, w, v);
        stage_row<N, RR, NT>(lf + ((l + 1) & 1) * PB, v, t, hl, nc);
      } else {
        stage_row<N, RR, NT>(lf + ((l + 1) & 1) * PB, p_own, t, hl, nc);
      }
    }
    __syncthreads();
  }
  // block mapping (t RR + q) -> owned positions (t + NT o)
#pragma unroll
  for (int q = 0; q < RR; ++q) th[pad_f(t * RR + q)] = acc[q];
  __syncthreads();
#pragma unroll
  for (int o = 0; o < RR; ++o) theta[o] = th[pad_f(t + NT * o)];
}

// Publishes this member's four spectrum components (x.re, x.im, y.re, y.im) at
// positions t + NT o, for round `tag`.
template <int RR, int NT, int N>
__device__ __forceinline__ void put_spectrum(uint64_t* dst, const float2 (&x)[RR], const float2 (&y)[RR],
                                             unsigned tag, int t) {
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    const int k = t + NT * o;
    xput(dst + 0 * N + k, x[o].x, tag);
    xput(dst + 1 * N + k, x[o].y, tag);
    xput(dst + 2 * N + k, y[o].x, tag);
    xput(dst + 3 * N + k, y[o].y, tag);
  }
}

// ax / ay = sum over members n2 of w_n2 * (member n2's spectrum), where
// w_n2 = wsb[(n2 * me) mod n_sb], conjugated when CONJ.
template <int RR, int NT, int N, bool CONJ>
__device__ __forceinline__ void combine_spectra(const uint64_t* src, int nsb, int me, const float2* wsb,
                                                unsigned tag, const XchgCtl& ctl, int t, float2 (&ax)[RR],
                                                float2 (&ay)[RR]) {
#pragma unroll
  for (int o = 0; o < RR; ++o) ax[o] = ay[o] = make_float2(0.f, 0.f);
  for (int n2 = 0; n2 < nsb; ++n2) {
    const float2 w = wsb[(n2 * me) % nsb];
    const uint64_t* row = src + (size_t)n2 * 4 * N;
#pragma unroll
    for (int comp = 0; comp < 2; ++comp) {  // polarisation x, then y
      float re[RR], im[RR];
      xget<RR>(row + (2 * comp) * N, t, NT, tag, ctl, re);
      xget<RR>(row + (2 * comp + 1) * N, t, NT, tag, ctl, im);
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const float2 v = make_float2(re[o], im[o]);
        const float2 prod = CONJ ? cmulc(v, w) : cmul(v, w);
        if (comp == 0) ax[o] = cadd(ax[o], prod);
        else ay[o] = cadd(ay[o], prod);
      }
    }
  }
}

template <int LOGN>
__global__ __launch_bounds__(FftShape<(1 << LOGN)>::NT) void fwd_kernel(FwdArgs a) {
  constexpr int N = 1 << LOGN;  // N'
  using S = FftShape<N>;
  constexpr int RR = S::RR, NT = S::NT;
  __shared__ __align__(16) float lf[lds_floats<N>()];
  float2* lx = reinterpret_cast<float2*>(lf);
  float2* ly = lx + S::LDS_C;

  const int nsb = a.n_sb;
  // XCD-aware mapping: the n_sb members of a team share blockIdx mod 8
  const int xcd = blockIdx.x % kXcds;
  const int r = blockIdx.x / kXcds;
  const int me = r % nsb;
  const int team = (r / nsb) * kXcds + xcd;
  if (team >= a.n_teams) return;

  const float2* tw = a.tab.tw;

  const int T = a.T;
  const int tap_pad = kTapChunk * a.n_chunks;
  const unsigned rounds_per_item = (unsigned)a.steps + 2u;
  uint64_t* xs_in = a.xspec + ((size_t)team * 2 + 0) * nsb * 4 * N;
  uint64_t* xs_out = a.xspec + ((size_t)team * 2 + 1) * nsb * 4 * N;
  unsigned iter = 0;
  for (int item = team; item < a.n_items; item += a.n_teams, ++iter) {
    int t = opaque_tid();
    const unsigned round0 = a.tag_base + iter * rounds_per_item;
    const int inst = item / a.nblk;
    const int blk = item - inst * a.nblk;
    const float2* in_x = a.in + (size_t)inst * 2 * T;
    const float2* in_y = in_x + T;
    float2 x[RR], y[RR];

    // ---- gather polyphase component `me` (n = n_sb n1 + me), times (-1)^n
    {
      const int first = frame_first(blk, a.hop, a.n_ov, T, a.boundary);
      const bool short_seq = T < nsb * N;
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const int n = nsb * (t + NT * o) + me;
        const int pos = frame_pos(first, n, T, a.boundary, short_seq);
        float2 vx = make_float2(0.f, 0.f), vy = vx;
        if (pos >= 0) {
          vx = in_x[pos];
          vy = in_y[pos];
        }
        const float sg = (n & 1) ? -1.0f : 1.0f;
        x[o] = cscale(vx, sg);
        y[o] = cscale(vy, sg);
      }
    }
    fft<N, false>(x, y, lx, ly, tw, t);

    // ---- size-n_sb DFT across the team: subband `me` of the block spectrum
    if (nsb > 1) {
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const float2 w = a.tab.poly_tw[(size_t)me * N + t + NT * o];
        x[o] = cmul(x[o], w);
        y[o] = cmul(y[o], w);
      }
      put_spectrum<RR, NT, N>(xs_in + (size_t)me * 4 * N, x, y, round0, t);
      combine_spectra<RR, NT, N, false>(xs_in, nsb, me, a.tab.wsb, round0, a.ctl, t, x, y);
    }

    // ---- step loop (Fig. "scheme_CB-ESSFM"), spectra in subband order
    for (int s = 0; s < a.steps; ++s) {
      t = opaque_tid();
      const float2* h = (s == 0 ? a.tab.h_first : a.tab.h_mid) + (size_t)me * N;
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const float2 hv = h[t + NT * o];
        x[o] = cmul(x[o], hv);
        y[o] = cmul(y[o], hv);
      }
      fft<N, true>(x, y, lx, ly, tw, t);  // lowpass-equivalent subband samples
      float p[RR], theta[RR];
#pragma unroll
      for (int o = 0; o < RR; ++o) p[o] = x[o].x * x[o].x + x[o].y * x[o].y + y[o].x * y[o].x + y[o].y * y[o].y;
      const unsigned round = round0 + 1u + (unsigned)s;
      uint64_t* xrow = a.xp + ((size_t)team * 2 + (round & 1u)) * nsb * N;
      const float* crow = a.tab.cpad + ((size_t)(s * nsb + me) * nsb) * tap_pad;
      coupled_fir<N>(a, crow, me, xrow, round, p, theta, lf);
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        float sn, cs;
        sincosf(theta[o], &sn, &cs);
        const float2 rot = make_float2(cs, -sn);  // exp(-j theta)
        x[o] = cmul(x[o], rot);
        y[o] = cmul(y[o], rot);
      }
      fft<N, false>(x, y, lx, ly, tw, t);
    }

    // ---- final GVD, recombination, inverse size-N DFT
    t = opaque_tid();
    {
      const float2* h = a.tab.h_last + (size_t)me * N;
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const float2 hv = h[t + NT * o];
        x[o] = cmul(x[o], hv);
        y[o] = cmul(y[o], hv);
      }
    }
    if (nsb > 1) {
      const unsigned round = round0 + rounds_per_item - 1u;
      put_spectrum<RR, NT, N>(xs_out + (size_t)me * 4 * N, x, y, round, t);
      combine_spectra<RR, NT, N, true>(xs_out, nsb, me, a.tab.wsb, round, a.ctl, t, x, y);
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const float2 w = a.tab.poly_tw[(size_t)me * N + t + NT * o];
        x[o] = cmulc(x[o], w);
        y[o] = cmulc(y[o], w);
      }
    }
    fft<N, true>(x, y, lx, ly, tw, t);

    // ---- keep samples [N_ov/2, N - N_ov/2) of the block
    float2* out_x = a.out + (size_t)inst * 2 * T;
    float2* out_y = out_x + T;
    const int keep_lo = a.n_ov / 2, keep_hi = nsb * N - a.n_ov / 2;
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      const int n = nsb * (t + NT * o) + me;
      const int pos = blk * a.hop + n - keep_lo;
      if (n >= keep_lo && n < keep_hi && pos < T) {
        const float sg = (n & 1) ? -1.0f : 1.0f;
        out_x[pos] = cscale(x[o], sg);
        out_y[pos] = cscale(y[o], sg);
      }
    }
  }
}

// ------------------------------------------------------------------ tables
// FP32 rounding of (c, s) keeping the magnitude (see round_pair in plan.cpp).
__device__ float2 round_pair_dev(double c, double s) {
  const float c0 = (float)c, s0 = (float)s;
  const float c1 = (double)c0 < c ? nextafterf(c0, 2.0f) : nextafterf(c0, -2.0f);
  const float s1 = (double)s0 < s ? nextafterf(s0, 2.0f) : nextafterf(s0, -2.0f);
  const double target = c * c + s * s;
  float2 best = make_float2(c0, s0);
  double err = fabs((double)c0 * c0 + (double)s0 * s0 - target);
  const float2 cand[3] = {make_float2(c0, s1), make_float2(c1, s0), make_float2(c1, s1)};
  for (int i = 0; i < 3; ++i) {
    const double e = fabs((double)cand[i].x * cand[i].x + (double)cand[i].y * cand[i].y - target);
    if (e < err) {
      err = e;
      best = cand[i];
    }
  }
  return best;
}

// h tables from the FP64 phase-per-km table and the current split ratio.
__global__ void tables_kernel(const double* __restrict__ phase, const double* __restrict__ rho_p, double L,
                              double inv_n, double inv_np, int n, float2* __restrict__ h) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double rho = *rho_p;
  const double ph = phase[q];
  double s, c;
  sincos(ph * (1.0 - rho) * L, &s, &c);
  h[q] = round_pair_dev(c * inv_n, s * inv_n);
  sincos(ph * L, &s, &c);
  h[n + q] = round_pair_dev(c * inv_np, s * inv_np);
  sincos(ph * rho * L, &s, &c);
  h[2 * n + q] = round_pair_dev(c * inv_np, s * inv_np);
}

__global__ void pad_coeffs_kernel(const float* __restrict__ src, float* __restrict__ dst, int rows, int n_taps,
                                  int tap_pad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * tap_pad) return;
  const int row = i / tap_pad, tau = i % tap_pad;
  dst[i] = tau < n_taps ? src[(size_t)row * n_taps + tau] : 0.0f;
}

__global__ void copy_rho_kernel(const float* __restrict__ src, double* __restrict__ dst) { *dst = (double)*src; }

// ------------------------------------------------------------------ launchers
template <int LOGN>
static int launch_fwd_t(const FwdArgs& args, int grid, hipStream_t s) {
  void* kargs[] = {(void*)&args};
  hipError_t e = hipLaunchCooperativeKernel((const void*)fwd_kernel<LOGN>, dim3(grid),
                                            dim3(FftShape<(1 << LOGN)>::NT), kargs, 0, s);
  return e == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

int threads_for(int log_np) {
  switch (log_np) {
    case 8: return FftShape<256>::NT;
    case 9: return FftShape<512>::NT;
    case 10: return FftShape<1024>::NT;
    case 11: return FftShape<2048>::NT;
    case 12: return FftShape<4096>::NT;
    case 13: return FftShape<8192>::NT;
    default: return 0;
  }
}

template <int LOGN>
static int occ_t(int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fwd_kernel<LOGN>, FftShape<(1 << LOGN)>::NT, 0) ==
                 hipSuccess
             ? CBESSFM_OK
             : CBESSFM_EHIP;
}

int occupancy_per_cu(int log_np, int* blocks) {
  switch (log_np) {
    case 8: return occ_t<8>(blocks);
    case 9: return occ_t<9>(blocks);
    case 10: return occ_t<10>(blocks);
    case 11: return occ_t<11>(blocks);
    case 12: return occ_t<12>(blocks);
    case 13: return occ_t<13>(blocks);
    default: return CBESSFM_EUNSUPPORTED;
  }
}

void fill_tables(const cbessfm_plan_t* p, Tables& tb) {
  tb.h_first = p->d_h;
  tb.h_mid = p->d_h + p->N;
  tb.h_last = p->d_h + 2 * (size_t)p->N;
  tb.tw = p->d_tw;
  tb.poly_tw = p->d_poly;
  tb.cpad = p->d_cpad;
  for (int i = 0; i < kMaxSubbands; ++i) tb.wsb[i] = p->wsb[i];
}

int launch_forward(cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, hipStream_t s) {
  FwdArgs a;
  a.in = static_cast<const float2*>(in);
  a.out = static_cast<float2*>(out);
  a.T = (int)T;
  a.nblk = (int)((T + p->hop - 1) / p->hop);
  a.n_items = batch * a.nblk;
  a.n_sb = p->sb.n_sb;
  a.steps = p->steps;
  a.n_chunks = p->n_chunks;
  a.nc = p->n_taps / 2;
  a.n_ov = p->sb.overlap;
  a.hop = p->hop;
  a.boundary = p->sb.boundary;
  a.n_teams = a.n_items < p->team_capacity ? a.n_items : p->team_capacity;
  fill_tables(p, a.tab);
  a.xspec = p->d_xspec;
  a.xp = p->d_xp;
  a.ctl.abort = p->d_abort;
  a.ctl.err = p->d_err;
  a.ctl.spin_limit = 1u << 22;
  const unsigned per_team = (unsigned)((a.n_items + a.n_teams - 1) / a.n_teams);
  a.tag_base = take_tags(p, per_team * (unsigned)(a.steps + 2), s);
  if (a.tag_base == 0u) return CBESSFM_EHIP;
  const int groups = (a.n_teams + kXcds - 1) / kXcds;
  const int grid = groups * kXcds * a.n_sb;
  switch (p->log_np) {
    case 8: return launch_fwd_t<8>(a, grid, s);
    case 9: return launch_fwd_t<9>(a, grid, s);
    case 10: return launch_fwd_t<10>(a, grid, s);
    case 11: return launch_fwd_t<11>(a, grid, s);
    case 12: return launch_fwd_t<12>(a, grid, s);
    case 13: return launch_fwd_t<13>(a, grid, s);
    default: return CBESSFM_EUNSUPPORTED;
  }
}

int launch_tables(cbessfm_plan_t* p, hipStream_t s) {
  const int n = p->N;
  tables_kernel<<<(n + 255) / 256, 256, 0, s>>>(p->d_phase, p->d_rho, p->step_km, 1.0 / (double)n,
                                                1.0 / (double)p->Np, n, p->d_h);
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

int launch_pad_coeffs(cbessfm_plan_t* p, const float* src, hipStream_t s) {
  const int rows = p->steps * p->sb.n_sb * p->sb.n_sb;
  const int total = rows * p->tap_pad;
  pad_coeffs_kernel<<<(total + 255) / 256, 256, 0, s>>>(src, p->d_cpad, rows, p->n_taps, p->tap_pad);
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

int launch_copy_rho(cbessfm_plan_t* p, const float* src, hipStream_t s) {
  copy_rho_kernel<<<1, 1, 0, s>>>(src, p->d_rho);
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

}  // namespace cbessfm
