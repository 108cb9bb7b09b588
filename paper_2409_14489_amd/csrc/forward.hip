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
#include "stages.hpp"
#include "team.hpp"

namespace cbessfm {

// Exchange rounds per step: one, or two for the dual-polarisation NLPR when
// its two filters cannot share a round (their rows do not fit the LDS).
template <int N, bool DUAL>
__host__ __device__ constexpr unsigned dual_rounds() {
  return DUAL && !DualFir<N>::fits ? 2u : 1u;
}

// One overlap-and-save block of one instance, as member c.me of a team.
// sub = batch entry * nblk + block; the team's exchange rounds for this block
// are round0 .. round0 + fwd_rounds - 1: two for the input DEMUX (one per
// polarisation), the steps' rounds, two for the output MUX.  Every round goes
// through xp_team, the team's two slots of n_sb x 2 N' words (intensity rows,
// or one polarisation's spectra), slot = round & 1, so a block touches
// 2 n_sb x 2 N' words of exchange memory and more of it stays in the L2.
// FIR: 0 time-domain coupled filter, 1 frequency domain, 2 as the instance's
// tables say (batches mixing instances of both kinds).
template <int N, bool DUAL, int FIR>
__device__ __forceinline__ void fwd_item(TeamCtx& c, const Inst& d, int sub, unsigned round0, uint64_t* xp_team,
                                         float* lf) {
  using S = FftShape<N>;
  constexpr int RR = S::RR;
  float4* lxy = reinterpret_cast<float4*>(lf);
  const int nsb = c.nsb, me = c.me;
  const float2* tw = d.tab.tw;
  const int T = d.T;
  const int tap_pad = kTapChunk * d.n_chunks;
  const int inst = sub / d.nblk;
  const int blk = sub - inst * d.nblk;
  const float2* in_x = d.in + (size_t)inst * 2 * T;
  int t = opaque_tid();
  float2 x[RR], y[RR];

  // ---- block input: size-N DFT as N_sb polyphase FFTs + N_sb-point DFT
  gather_block<N, false>(in_x, in_x + T, blk, d.hop, d.n_ov, T, d.boundary, nsb, me, t, x, y);
  fft<N, false>(x, y, lxy, tw, t);
  polyphase_to_subband_xp<N>(c, xp_team, round0, t, x, y);

  // ---- step loop (Fig. "scheme_CB-ESSFM"), spectra in subband order
  for (int s = 0; s < d.steps; ++s) {
    t = opaque_tid();
    apply_diag<N, false>(x, y, step_gvd(d.tab, s) + (size_t)me * N, t);
    fft<N, true>(x, y, lxy, tw, t);  // lowpass-equivalent subband samples
    float p[RR], theta[RR];
    intensity<N>(x, y, p);
    const size_t crow = ((size_t)(s * nsb + me) * nsb) * tap_pad;
    const unsigned round = round0 + 2u + (unsigned)s * dual_rounds<N, DUAL>();
    uint64_t* xrow = xp_team + (size_t)(round & 1u) * nsb * 2 * N;
    if constexpr (DUAL) {
      // theta^{x,y} = theta +- phi, phi_i = (1/3) sum_{l != i} C_il (*) (|x_l|^2 - |y_l|^2)
      float phi[RR], pd[RR];
      intensity_diff<N>(x, y, pd);
      if constexpr (DualFir<N>::fits) {
        coupled_fir_dual<N>(c, d.tab.cpad + crow, d.tab.cdpad + crow, xrow, round, p, pd, theta, phi, lf);
      } else {
        coupled_fir<N>(c, d.tab.cpad + crow, xrow, round, p, theta, lf);
        uint64_t* drow = xp_team + (size_t)((round + 1u) & 1u) * nsb * 2 * N;
        coupled_fir<N>(c, d.tab.cdpad + crow, drow, round + 1u, pd, phi, lf);
      }
      rotate_dual<N>(x, y, theta, phi);
    } else {
      if (FIR == 1 || (FIR == 2 && d.tab.chat != nullptr))
        coupled_fir_freq<N>(c, d.tab.chat + ((size_t)(s * nsb + me) * nsb) * N, xrow, round, p, theta, lf);
      else
        coupled_fir<N>(c, d.tab.cpad + crow, xrow, round, p, theta, lf);
      rotate<N, -1>(x, y, theta);
    }
    fft<N, false>(x, y, lxy, tw, t);
  }

  // ---- final GVD, recombination, inverse size-N DFT, kept samples
  t = opaque_tid();
  apply_diag<N, false>(x, y, d.tab.h_last + (size_t)me * N, t);
  subband_to_polyphase_xp<N>(c, xp_team, round0 + fwd_rounds(d.steps, dual_rounds<N, DUAL>()) - 2u, t, x, y);
  fft<N, true>(x, y, lxy, tw, t);
  float2* out_x = d.out + (size_t)inst * 2 * T;
  scatter_block<N>(out_x, out_x + T, blk, d.hop, d.n_ov, T, nsb, me, t, x, y);
}

// Single plan: team j takes blocks j, j + n_teams, ...  The n_sb members of a
// team share blockIdx mod 8, i.e. one XCD and its L2 (workgroups are dispatched
// round-robin over the 8 XCDs).
template <int LOGN, bool DUAL, int FIR>
__global__ __launch_bounds__(FftShape<(1 << LOGN)>::NT) void fwd_kernel(FwdArgs a) {
  constexpr int N = 1 << LOGN;  // N'
  __shared__ __align__(16) float lf[lds_floats<N>()];
  __shared__ unsigned epoch_word;

  TeamCtx c;
  c.nsb = a.inst.n_sb;
  const int r = blockIdx.x / kXcds;
  c.me = r % c.nsb;
  c.team = (r / c.nsb) * kXcds + blockIdx.x % kXcds;
  if (c.team >= a.n_teams) return;
  c.n_chunks = a.inst.n_chunks;
  c.nc = a.inst.nc;
  c.ctl = a.ctl;
  c.tab = &a.inst.tab;
  const int nsb = c.nsb;
  const unsigned rounds_per_item = fwd_rounds(a.inst.steps, dual_rounds<N, DUAL>());
  uint64_t* xp_team = a.xp + (size_t)c.team * 2 * nsb * 2 * N;
  const unsigned first = epoch_begin(a.epoch + c.team, &epoch_word);
  unsigned iter = 0;
  for (int item = c.team; item < a.n_items; item += a.n_teams, ++iter)
    fwd_item<N, DUAL, FIR>(c, a.inst, item, first + iter * rounds_per_item, xp_team, lf);
  epoch_end(a.epoch + c.team, first, iter * rounds_per_item, c.me);
}

// Batch: workgroup -> (team, member) and team -> items come from a schedule
// built on the host; the instances of one team all have the team's n_sb and
// this kernel's N'.
template <int LOGN>
__global__ __launch_bounds__(FftShape<(1 << LOGN)>::NT) void fwd_batch_kernel(BatchArgs a) {
  constexpr int N = 1 << LOGN;
  __shared__ __align__(16) float lf[lds_floats<N>()];
  __shared__ unsigned epoch_word;

  const int2 wg = a.wg[blockIdx.x];
  if (wg.x < 0) return;
  const BatchTeam& tm = a.teams[wg.x];
  TeamCtx c;
  c.nsb = tm.width;
  c.me = wg.y;
  c.team = wg.x;
  c.ctl = a.ctl;
  uint64_t* xp_team = a.xp + tm.xp_off;
  unsigned* epoch = a.epoch + tm.epoch_slot;
  const unsigned first = epoch_begin(epoch, &epoch_word);
  for (int k = 0; k < tm.count; ++k) {
    const BatchItem it = a.items[tm.first + k];
    const Inst& d = a.insts[it.inst];
    c.n_chunks = d.n_chunks;
    c.nc = d.nc;
    c.tab = &d.tab;
    fwd_item<N, false, 2>(c, d, it.sub, first + it.round_off, xp_team, lf);
  }
  epoch_end(epoch, first, tm.rounds, c.me);
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

// Explicit dispersion segments: table j = exp(+j phi len[j]), scaled by 1 / N
// for j = 0 (after the unscaled size-N input DFT) and 1 / N' otherwise.
__global__ void gvd_tables_kernel(const double* __restrict__ phase, const double* __restrict__ len, int n_seg,
                                  double inv_n, double inv_np, int n, float2* __restrict__ h) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n_seg * n) return;
  const int j = (int)(idx / n), q = (int)(idx - (long long)j * n);
  const double scale = j == 0 ? inv_n : inv_np;
  double sn, cs;
  sincos(phase[q] * len[j], &sn, &cs);
  h[idx] = round_pair_dev(cs * scale, sn * scale);
}

// dst[s][i][l][tau] = C[s][i][l][tau] (zero for tau >= n_taps);
// dstt[s][l][i][tau] = C[s][i][l][n_taps - 1 - tau] (the adjoint's correlation);
// dstd[s][i][l][tau] = C[s][i][l][tau] / 3 for l != i, 0 on the diagonal.
__global__ void pad_coeffs_kernel(const float* __restrict__ src, float* __restrict__ dst, float* __restrict__ dstt,
                                  float* __restrict__ dstd, int steps, int nsb, int n_taps, int tap_pad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int rows = steps * nsb * nsb;
  if (i >= rows * tap_pad) return;
  const int row = i / tap_pad, tau = i % tap_pad;
  const float v = tau < n_taps ? src[(size_t)row * n_taps + tau] : 0.0f;
  dst[i] = v;
  dstd[i] = ((row / nsb) % nsb == row % nsb) ? 0.0f : v / 3.0f;
  const int s = row / (nsb * nsb), l = (row / nsb) % nsb, ii = row % nsb;  // row of dstt = (s, l, ii)
  dstt[i] = tau < n_taps ? src[(((size_t)s * nsb + ii) * nsb + l) * n_taps + (n_taps - 1 - tau)] : 0.0f;
}

__global__ void copy_rho_kernel(const float* __restrict__ src, double* __restrict__ dst) { *dst = (double)*src; }

// chat[row][k] = sum_t c[row][t] exp(-j 2 pi k (t - Nc) / N'): the DFT of a
// coefficient row placed circularly (tap t at position t - Nc mod N'), from
// the plan's twiddle table tw[n] = exp(-j 2 pi n / N'), summed in FP64.
__global__ void row_dft_kernel(const float* __restrict__ c, const float2* __restrict__ tw, float2* __restrict__ chat,
                               int rows, int n_taps, int np) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)rows * np) return;
  const int row = (int)(idx / np), k = (int)(idx - (long long)row * np);
  const int nc = n_taps / 2;
  double re = 0.0, im = 0.0;
  for (int t = 0; t < n_taps; ++t) {
    const int m = ((t - nc) % np + np) % np;
    const float2 w = tw[(int)(((long long)k * m) % np)];
    const double cv = (double)c[(size_t)row * n_taps + t];
    re += cv * (double)w.x;
    im += cv * (double)w.y;
  }
  chat[idx] = make_float2((float)re, (float)im);
}

// ------------------------------------------------------------------ launchers
// True when `s` is recording a graph.  Cooperative launches guarantee that
// the whole grid is resident; inside a capture an ordinary launch of the same
// (resident-sized) grid is recorded instead.
bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return st != hipStreamCaptureStatusNone;
}

template <typename K, typename A>
static int launch_persistent(K kernel, const A& args, int grid, int threads, hipStream_t s) {
  void* kargs[] = {(void*)&args};
  hipError_t e;
  if (stream_capturing(s))
    e = hipLaunchKernel((const void*)kernel, dim3(grid), dim3(threads), kargs, 0, s);
  else
    e = hipLaunchCooperativeKernel((const void*)kernel, dim3(grid), dim3(threads), kargs, 0, s);
  return e == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

template <int LOGN>
static int launch_fwd_t(const FwdArgs& args, bool dual, int grid, hipStream_t s) {
  constexpr int NT = FftShape<(1 << LOGN)>::NT;
  if (dual) return launch_persistent(fwd_kernel<LOGN, true, 0>, args, grid, NT, s);
  return args.inst.tab.chat != nullptr ? launch_persistent(fwd_kernel<LOGN, false, 1>, args, grid, NT, s)
                                       : launch_persistent(fwd_kernel<LOGN, false, 0>, args, grid, NT, s);
}

template <int LOGN>
static int launch_batch_t(const BatchArgs& args, int grid, hipStream_t s) {
  return launch_persistent(fwd_batch_kernel<LOGN>, args, grid, FftShape<(1 << LOGN)>::NT, s);
}

int launch_batch(int log_np, const BatchArgs& a, int grid, hipStream_t s) {
  switch (log_np) {
    case 8: return launch_batch_t<8>(a, grid, s);
    case 9: return launch_batch_t<9>(a, grid, s);
    case 10: return launch_batch_t<10>(a, grid, s);
    case 11: return launch_batch_t<11>(a, grid, s);
    case 12: return launch_batch_t<12>(a, grid, s);
    case 13: return launch_batch_t<13>(a, grid, s);
    default: return CBESSFM_EUNSUPPORTED;
  }
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

// Resident workgroups per CU; for the averaged NLPR the smaller of the time-
// and frequency-domain filter kernels (the plan's teams fit either).
template <int LOGN>
static int occ_t(bool dual, int* blocks) {
  constexpr int NT = FftShape<(1 << LOGN)>::NT;
  if (dual)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fwd_kernel<LOGN, true, 0>, NT, 0) == hipSuccess
               ? CBESSFM_OK
               : CBESSFM_EHIP;
  int bt = 0, bf = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bt, fwd_kernel<LOGN, false, 0>, NT, 0) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&bf, fwd_kernel<LOGN, false, 1>, NT, 0) != hipSuccess)
    return CBESSFM_EHIP;
  *blocks = bt < bf ? bt : bf;
  return CBESSFM_OK;
}

template <int LOGN>
static int bocc_t(int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fwd_batch_kernel<LOGN>, FftShape<(1 << LOGN)>::NT,
                                                      0) == hipSuccess
             ? CBESSFM_OK
             : CBESSFM_EHIP;
}

int batch_occupancy_per_cu(int log_np, int* blocks) {
  switch (log_np) {
    case 8: return bocc_t<8>(blocks);
    case 9: return bocc_t<9>(blocks);
    case 10: return bocc_t<10>(blocks);
    case 11: return bocc_t<11>(blocks);
    case 12: return bocc_t<12>(blocks);
    case 13: return bocc_t<13>(blocks);
    default: return CBESSFM_EUNSUPPORTED;
  }
}

int occupancy_per_cu(int log_np, bool dual, int* blocks) {
  switch (log_np) {
    case 8: return occ_t<8>(dual, blocks);
    case 9: return occ_t<9>(dual, blocks);
    case 10: return occ_t<10>(dual, blocks);
    case 11: return occ_t<11>(dual, blocks);
    case 12: return occ_t<12>(dual, blocks);
    case 13: return occ_t<13>(dual, blocks);
    default: return CBESSFM_EUNSUPPORTED;
  }
}

void fill_tables(const cbessfm_plan_t* p, Tables& tb) {
  tb.h_first = p->d_h;
  tb.h_mid = p->d_h + p->N;
  tb.h_last = p->d_h + (size_t)(p->gvd_explicit ? p->steps : 2) * p->N;
  tb.h_stride = p->gvd_explicit ? p->N : 0;
  tb.tw = p->d_tw;
  tb.poly_tw = p->d_poly;
  tb.cpad = p->d_cpad;
  tb.cdpad = p->d_cdpad;
  tb.chat = p->fir_freq ? p->d_chat : nullptr;
  for (int i = 0; i < kMaxSubbands; ++i) tb.wsb[i] = p->wsb[i];
}

void fill_inst(const cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, Inst& d) {
  (void)batch;
  d.in = static_cast<const float2*>(in);
  d.out = static_cast<float2*>(out);
  d.T = (int)T;
  d.nblk = (int)((T + p->hop - 1) / p->hop);
  d.n_sb = p->sb.n_sb;
  d.steps = p->steps;
  d.n_chunks = p->n_chunks;
  d.nc = p->n_taps / 2;
  d.n_ov = p->sb.overlap;
  d.hop = p->hop;
  d.boundary = p->sb.boundary;
  fill_tables(p, d.tab);
}

int launch_forward(cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, hipStream_t s) {
  FwdArgs a;
  fill_inst(p, in, out, T, batch, a.inst);
  a.n_items = batch * a.inst.nblk;
  const bool dual = p->nlpr == CBESSFM_NLPR_DUAL_POL;
  const int capacity = dual ? p->team_capacity_dual : p->team_capacity;
  a.n_teams = a.n_items < capacity ? a.n_items : capacity;
  a.epoch = p->d_epoch;
  a.xp = p->d_xp;
  a.ctl.abort = p->d_abort;
  a.ctl.err = p->d_err;
  a.ctl.spin_limit = p->wait_limit;
  const int groups = (a.n_teams + kXcds - 1) / kXcds;
  const int grid = groups * kXcds * a.inst.n_sb;
  switch (p->log_np) {
    case 8: return launch_fwd_t<8>(a, dual, grid, s);
    case 9: return launch_fwd_t<9>(a, dual, grid, s);
    case 10: return launch_fwd_t<10>(a, dual, grid, s);
    case 11: return launch_fwd_t<11>(a, dual, grid, s);
    case 12: return launch_fwd_t<12>(a, dual, grid, s);
    case 13: return launch_fwd_t<13>(a, dual, grid, s);
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
  pad_coeffs_kernel<<<(total + 255) / 256, 256, 0, s>>>(src, p->d_cpad, p->d_ctpad, p->d_cdpad, p->steps,
                                                       p->sb.n_sb, p->n_taps, p->tap_pad);
  if (p->fir_freq) {
    const long long cells = (long long)rows * p->Np;
    row_dft_kernel<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(src, p->d_tw, p->d_chat, rows, p->n_taps,
                                                                  p->Np);
  }
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

int launch_gvd_tables(cbessfm_plan_t* p, const double* lengths, hipStream_t s) {
  const int n_seg = p->steps + 1;
  if (hipMemcpyAsync(p->d_len, lengths, sizeof(double) * n_seg, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return CBESSFM_EHIP;
  const long long total = (long long)n_seg * p->N;
  gvd_tables_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(p->d_phase, p->d_len, n_seg, 1.0 / (double)p->N,
                                                                    1.0 / (double)p->Np, p->N, p->d_h);
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

int launch_copy_rho(cbessfm_plan_t* p, const float* src, hipStream_t s) {
  copy_rho_kernel<<<1, 1, 0, s>>>(src, p->d_rho);
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

}  // namespace cbessfm
