// CB-ESSFM forward kernel for gfx950 (MI355X).
//
// One persistent launch processes every overlap-and-save block of every batch
// instance (Sec. III-A).  A "team" of N_sb workgroups handles one block at a
// time; workgroup i of the team owns subband i (and, at the block's input and
// output, the polyphase component i of the size-N DFT).  Within a workgroup the
// subband's two polarisations live in registers for the whole step loop
// (FFT layout contract of fft_lds.hpp); LDS is only used for the FFT pass
// exchanges and the coupled-intensity filter.  HBM is touched when the block
// is read and written and, between team members, for the per-step intensity
// exchange of eq. (15), which stays in L2 / MALL.
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "internal.hpp"

namespace cbessfm {

// ------------------------------------------------------------------ team barrier
// All n_sb workgroups of a team must be resident (cooperative launch).  The
// wait is bounded: on timeout the sticky error flag is set and every later
// barrier of the launch falls through, so the grid always drains.
// `abort` is zeroed with the counters at every launch; `err` is sticky until
// cbessfm_status() reads it.
__device__ __forceinline__ void team_sync(unsigned* ctr, unsigned target, unsigned* abort, int* err,
                                          unsigned spin_limit) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned n = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
      if (++n > spin_limit) {
        __hip_atomic_store(abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(err, (int)CBESSFM_ESYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
  __threadfence();
}

// Input position of block sample n, or -1 for a zero.  `first` is the
// position of sample 0: already reduced mod T for the circular boundary (so a
// single subtraction wraps it unless T < N), raw for the zero boundary.
__device__ __forceinline__ int in_pos(int first, int n, int T, int boundary, bool short_seq) {
  if (boundary == 0) {
    int pos = first + n;
    if (short_seq) return pos % T;
    return pos >= T ? pos - T : pos;
  }
  const int pos = first + n;
  return (pos < 0 || pos >= T) ? -1 : pos;
}

// LDS of the nonlinear stage (aliases the FFT exchange buffers): two rows of
// circularly extended intensities and one row of phases, in floats.
template <int N>
struct NlprLds {
  static constexpr int PB = pad_f_size(N + kMaxTaps + 2 * kTapChunk);
  static constexpr int TH = pad_f_size(N);
  static constexpr int FLOATS = 2 * PB + TH;
};
template <int N>
constexpr int lds_floats() {
  return 4 * FftShape<N>::LDS_C > NlprLds<N>::FLOATS ? 4 * FftShape<N>::LDS_C : NlprLds<N>::FLOATS;
}

// Coupled intensity filter of eq. (15) for subband `me`, circular over N':
//   theta[k] = sum_l sum_tau C[s][me][l][tau] p_l[(k - tau + nc) mod N'].
// p_own holds this workgroup's intensities at positions t + NT o; on return
// theta holds the phase at the same positions.  For n_sb > 1 the team's
// intensities are exchanged through `xp` (global, one barrier).
template <int N>
__device__ __forceinline__ void coupled_fir(const FwdArgs& a, int s, int me, int team, int slot,
                                           const float (&p_own)[FftShape<N>::RR], float (&theta)[FftShape<N>::RR],
                                           float* lf, unsigned* bar, unsigned& nbar) {
  using S = FftShape<N>;
  constexpr int RR = S::RR, NT = S::NT;
  const int t = threadIdx.x;
  const int nsb = a.n_sb;
  const int nc = a.nc;
  const int hl = kTapChunk * a.n_chunks - 1 - nc;  // left halo
  float* pb0 = lf;
  float* pb1 = lf + NlprLds<N>::PB;
  float* th = lf + 2 * NlprLds<N>::PB;
  const int tap_pad = kTapChunk * a.n_chunks;
  const float* crow = a.tab.cpad + ((size_t)(s * nsb + me) * nsb) * tap_pad;

  // stores p (positions t + NT o) into a circularly extended LDS row
  auto stage = [&](float* dst, const float* src_glob, const float (&src_reg)[RR], bool from_reg) {
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      const int k = t + NT * o;
      const float v = from_reg ? src_reg[o] : src_glob[k];
      dst[pad_f(k + hl)] = v;
      if (k >= N - hl) dst[pad_f(k - N + hl)] = v;
      if (k < nc) dst[pad_f(k + N + hl)] = v;
    }
  };

  float* xp = nullptr;
  __syncthreads();  // the LDS rows alias the FFT exchange buffers
  if (nsb == 1) {
    stage(pb0, nullptr, p_own, true);
  } else {
    xp = a.xp + ((size_t)team * 2 + slot) * nsb * N;
#pragma unroll
    for (int o = 0; o < RR; ++o) xp[(size_t)me * N + t + NT * o] = p_own[o];
    team_sync(bar, (++nbar) * (unsigned)nsb, a.abort, a.err, a.spin_limit);
    stage(pb0, xp, p_own, false);
  }
  __syncthreads();

  float acc[RR];
#pragma unroll
  for (int q = 0; q < RR; ++q) acc[q] = 0.0f;
  for (int l = 0; l < nsb; ++l) {
    float* cur = (l & 1) ? pb1 : pb0;
    if (l + 1 < nsb) stage((l & 1) ? pb0 : pb1, xp + (size_t)(l + 1) * N, p_own, false);
    const float* cl = crow + (size_t)l * tap_pad;
    for (int c = 0; c < a.n_chunks; ++c) {
      // window w in [0, RR + 7): p index t RR + w - 7 - 8 c + nc, stored at + hl
      float win[RR + kTapChunk - 1];
      const int base = t * RR - (kTapChunk - 1) - kTapChunk * c + nc + hl;
#pragma unroll
      for (int w = 0; w < RR + kTapChunk - 1; ++w) win[w] = cur[pad_f(base + w)];
#pragma unroll
      for (int tt = 0; tt < kTapChunk; ++tt) {
        const float cf = cl[kTapChunk * c + tt];
#pragma unroll
        for (int q = 0; q < RR; ++q) acc[q] = fmaf(cf, win[q - tt + kTapChunk - 1], acc[q]);
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

template <int LOGN>
__global__ __launch_bounds__(FftShape<(1 << LOGN)>::NT) void fwd_kernel(FwdArgs a) {
  constexpr int N = 1 << LOGN;  // N'
  using S = FftShape<N>;
  constexpr int RR = S::RR, NT = S::NT;
  __shared__ __align__(16) float lf[lds_floats<N>()];
  float2* lx = reinterpret_cast<float2*>(lf);
  float2* ly = lx + S::LDS_C;

  const int t = threadIdx.x;
  const int nsb = a.n_sb;
  // XCD-aware mapping: the n_sb members of a team share blockIdx mod 8
  const int xcd = blockIdx.x % kXcds;
  const int r = blockIdx.x / kXcds;
  const int me = r % nsb;
  const int team = (r / nsb) * kXcds + xcd;
  if (team >= a.n_teams) return;
  unsigned* bar = a.bar + (size_t)team * kBarStride;
  unsigned nbar = 0;

  float2 tw[S::TWC > 0 ? S::TWC : 1];
  load_twiddles<N>(tw, a.tab.tw, t);

  const long long T = a.T;
  int step_ctr = 0;
  for (int item = team; item < a.n_items; item += a.n_teams) {
    const int inst = item / a.nblk;
    const int blk = item - inst * a.nblk;
    const float2* in_x = a.in + (size_t)inst * 2 * T;
    const float2* in_y = in_x + T;
    float2 x[RR], y[RR];

    // ---- gather polyphase component `me` (n = n_sb n1 + me), times (-1)^n
    int first = blk * a.hop - a.n_ov / 2;
    if (a.boundary == 0) first = ((first % (int)T) + (int)T) % (int)T;
    const bool short_seq = T < (long long)nsb * N;
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      const int n = nsb * (t + NT * o) + me;
      const int pos = in_pos(first, n, (int)T, a.boundary, short_seq);
      float2 vx = make_float2(0.f, 0.f), vy = vx;
      if (pos >= 0) {
        vx = in_x[pos];
        vy = in_y[pos];
      }
      const float sg = (n & 1) ? -1.0f : 1.0f;
      x[o] = cscale(vx, sg);
      y[o] = cscale(vy, sg);
    }
    fft<N, false>(x, y, lx, ly, tw, t);

    // ---- size-n_sb DFT across the team: subband `me` of the block spectrum
    if (nsb > 1) {
      float2* xs = a.xspec + ((size_t)team * 2 + 0) * nsb * 2 * N;
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const int k = t + NT * o;
        const float2 w = a.tab.poly_tw[(size_t)me * N + k];
        xs[(size_t)(2 * me) * N + k] = cmul(x[o], w);
        xs[(size_t)(2 * me + 1) * N + k] = cmul(y[o], w);
      }
      team_sync(bar, (++nbar) * (unsigned)nsb, a.abort, a.err, a.spin_limit);
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const int k = t + NT * o;
        float2 ax = make_float2(0.f, 0.f), ay = ax;
        for (int n2 = 0; n2 < nsb; ++n2) {
          const float2 w = a.tab.wsb[(n2 * me) % nsb];
          ax = cadd(ax, cmul(xs[(size_t)(2 * n2) * N + k], w));
          ay = cadd(ay, cmul(xs[(size_t)(2 * n2 + 1) * N + k], w));
        }
        x[o] = ax;
        y[o] = ay;
      }
    }

    // ---- step loop (Fig. "scheme_CB-ESSFM"), spectra in subband order
    for (int s = 0; s < a.steps; ++s, ++step_ctr) {
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
      coupled_fir<N>(a, s, me, team, step_ctr & 1, p, theta, lf, bar, nbar);
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        float sn, cs;
        sincosf(theta[o], &sn, &cs);
        const float2 r = make_float2(cs, -sn);  // exp(-j theta)
        x[o] = cmul(x[o], r);
        y[o] = cmul(y[o], r);
      }
      fft<N, false>(x, y, lx, ly, tw, t);
    }

    // ---- final GVD, recombination, inverse size-N DFT
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
      float2* xs = a.xspec + ((size_t)team * 2 + 1) * nsb * 2 * N;
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const int k = t + NT * o;
        xs[(size_t)(2 * me) * N + k] = x[o];
        xs[(size_t)(2 * me + 1) * N + k] = y[o];
      }
      team_sync(bar, (++nbar) * (unsigned)nsb, a.abort, a.err, a.spin_limit);
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const int k = t + NT * o;
        float2 ax = make_float2(0.f, 0.f), ay = ax;
        for (int k2 = 0; k2 < nsb; ++k2) {
          const float2 w = a.tab.wsb[(k2 * me) % nsb];
          ax = cadd(ax, cmulc(xs[(size_t)(2 * k2) * N + k], w));
          ay = cadd(ay, cmulc(xs[(size_t)(2 * k2 + 1) * N + k], w));
        }
        const float2 w = a.tab.poly_tw[(size_t)me * N + k];
        x[o] = cmulc(ax, w);
        y[o] = cmulc(ay, w);
      }
    }
    fft<N, true>(x, y, lx, ly, tw, t);

    // ---- keep samples [N_ov/2, N - N_ov/2) of the block
    float2* out_x = a.out + (size_t)inst * 2 * T;
    float2* out_y = out_x + T;
    const int n_full = nsb * N;
    const int keep_lo = a.n_ov / 2, keep_hi = n_full - a.n_ov / 2;
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
// h tables from the FP64 phase-per-km table and the current split ratio.
__global__ void tables_kernel(const double* __restrict__ phase, const double* __restrict__ rho_p, double L,
                              double inv_n, double inv_np, int n, float2* __restrict__ h) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double rho = *rho_p;
  const double ph = phase[q];
  double s, c;
  sincos(ph * (1.0 - rho) * L, &s, &c);
  h[q] = make_float2((float)(c * inv_n), (float)(s * inv_n));
  sincos(ph * L, &s, &c);
  h[n + q] = make_float2((float)(c * inv_np), (float)(s * inv_np));
  sincos(ph * rho * L, &s, &c);
  h[2 * n + q] = make_float2((float)(c * inv_np), (float)(s * inv_np));
}

__global__ void pad_coeffs_kernel(const float* __restrict__ src, float* __restrict__ dst, int rows, int n_taps,
                                  int tap_pad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * tap_pad) return;
  const int row = i / tap_pad, tau = i % tap_pad;
  dst[i] = tau < n_taps ? src[(size_t)row * n_taps + tau] : 0.0f;
}

__global__ void copy_rho_kernel(const float* __restrict__ src, double* __restrict__ dst) { *dst = (double)*src; }

__global__ void zero_u32_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------------ launchers
template <int LOGN>
static int launch_fwd_t(cbessfm_plan_t* p, const FwdArgs& args, int grid, hipStream_t s) {
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

static void fill_tables(const cbessfm_plan_t* p, Tables& tb) {
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
  a.T = T;
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
  a.bar = p->d_bar;
  a.err = p->d_err;
  a.spin_limit = 1u << 24;
  a.abort = p->d_bar + (size_t)a.n_teams * kBarStride;
  const int nbar = a.n_teams * kBarStride + 1;
  zero_u32_kernel<<<(nbar + 255) / 256, 256, 0, s>>>(p->d_bar, nbar);
  if (hipGetLastError() != hipSuccess) return CBESSFM_EHIP;
  const int groups = (a.n_teams + kXcds - 1) / kXcds;
  const int grid = groups * kXcds * a.n_sb;
  switch (p->log_np) {
    case 8: return launch_fwd_t<8>(p, a, grid, s);
    case 9: return launch_fwd_t<9>(p, a, grid, s);
    case 10: return launch_fwd_t<10>(p, a, grid, s);
    case 11: return launch_fwd_t<11>(p, a, grid, s);
    case 12: return launch_fwd_t<12>(p, a, grid, s);
    case 13: return launch_fwd_t<13>(p, a, grid, s);
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
