// CB-ESSFM adjoint (reverse-mode) kernel for gfx950 (MI355X).
//
// Gives dL/dC (the per-step coupled-filter coefficients), dL/drho and,
// optionally, dL/dfield_in from dL/dfield_out, by running the forward map of
// Sec. III-A / III-C backwards.  The paper fits its coefficients offline with
// finite-difference gradients and names automatic differentiation as future
// work (Sec. III-B, Sec. V); this is that derivative, hand-written.
//
// Per block, with the forward quantities of step s (1-based) written
//   A = h_s S_{s-1},  v = IDFT(A),  p = |v_x|^2 + |v_y|^2,  theta = C_s (*) p,
//   w = v exp(-j theta),  S_s = DFT(w)        (unscaled size-N' transforms),
// and g_X the cotangent of X (PyTorch convention dL/dRe + j dL/dIm):
//   g_w = IDFT(g_S),  theta_bar = sum_pol Im(conj(g_w) w),
//   p_bar_l = sum_i C_s[i][l] (x) theta_bar_i   (correlation: taps reversed),
//   g_v = g_w exp(+j theta) + 2 p_bar v,  g_A = DFT(g_v),  g_{S_{s-1}} = conj(h_s) g_A,
//   dL/dC_s[i][l][tau] = sum_k theta_bar_i[k] p_l[(k - tau + Nc) mod N'].
// Dispersion segment j (lengths d_0 = (1 - rho) L, d_1 .. d_{N_st-1} = L,
// d_{N_st} = rho L, Sec. III-C) contributes dL/dd_j = -G_j with
// G_j = sum_q phi_q Im(conj(g_{A_j}) A_j), phi_q = 2 pi^2 beta2 f_q^2 per km and
// A_j the spectrum after segment j.  The split ratio moves length from the
// first segment to the last, dL/drho = L (G_0 - G_{N_st}); G_0 and G_{N_st}
// are each up to hundreds of times larger than their difference, which FP32
// state cannot resolve.  Telescoping over the steps instead, with
// e = exp(-j theta) - 1 (formed as (-2 sin^2(theta/2), -sin theta)),
// D = DFT(e v) and E = DFT(dg), dg = conj(e) g_w + 2 p_bar v:
//   G_s - G_{s-1} = sum_q phi'_q [Im(conj(g_S) D) - Im(conj(E) A)],
// over both polarisations and the subbands, phi'_q = phi_q - phi(f_i) (a
// constant per subband changes nothing: the rotation commutes with it).  This
// is the commutator of the dispersion operator with the step's rotation, in
// the frequency domain (Parseval); D and E are transforms of the small
// differences w - v = e v and g_v - g_w = dg, so both terms scale with the
// nonlinear phase and vanish with C, and
//   dL/drho = -L sum_s (G_s - G_{s-1})
// keeps the relative accuracy of the FP32 state.  The reverse step then needs
// no extra transform: g_A = DFT(g_w + dg) = N' g_S + E.  With free dispersion
// segments dL/dd_j is written as well: A_j for 0 < j < N_st is the stored A
// of step j + 1.  The block's output stage (MUX, inverse size-N DFT) is
// adjoint to its input stage and vice versa, so both are reused.
//
// The reverse step needs v, theta, A and D of its forward step.  The forward
// sweep stores the spectrum S_s at the start of every segment of `ck_every`
// steps, and (A, theta, D) of every step of the last segment; the reverse
// step makes v = IDFT(A) again, bit for bit, which costs one transform and
// keeps the record at 9 N' floats instead of 13.  The reverse sweep
// recomputes each earlier segment once from its spectrum, storing the records
// per step, and then runs that segment's reverse steps on them (one level of
// Griewank-style checkpointing; with a single segment nothing is recomputed).
// Coefficient and split-ratio partials are written per block and reduced over
// blocks in FP64 by a second kernel, in a fixed order.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fft_lds.hpp"
#include "internal.hpp"
#include "stages.hpp"
#include "team.hpp"

namespace cbessfm {

template <int N>
__device__ __forceinline__ void store_state(float2* st, const float2 (&x)[FftShape<N>::RR],
                                            const float2 (&y)[FftShape<N>::RR], int t) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    st[t + NT * o] = x[o];
    st[N + t + NT * o] = y[o];
  }
}

template <int N>
__device__ __forceinline__ void load_state(const float2* st, float2 (&x)[FftShape<N>::RR],
                                           float2 (&y)[FftShape<N>::RR], int t) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    x[o] = st[t + NT * o];
    y[o] = st[N + t + NT * o];
  }
}

// Stored record of one step, kVtFloats N' floats: the spectra A_x, A_y
// (N' complex each), theta (N' floats), the spectra D_x, D_y.
constexpr int kVtFloats = 9;
constexpr int kVtTheta = 4;  // offsets in N' floats
constexpr int kVtD = 5;

template <int N>
__device__ __forceinline__ void store_theta(float* st, const float (&th)[FftShape<N>::RR], int t) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
#pragma unroll
  for (int o = 0; o < RR; ++o) st[kVtTheta * N + t + NT * o] = th[o];
}

// A (into x, y) and theta of a stored record.
template <int N>
__device__ __forceinline__ void load_atheta(const float* st, float2 (&x)[FftShape<N>::RR],
                                            float2 (&y)[FftShape<N>::RR], float (&th)[FftShape<N>::RR], int t) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  const float2* a = reinterpret_cast<const float2*>(st);
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    x[o] = a[t + NT * o];
    y[o] = a[N + t + NT * o];
    th[o] = st[kVtTheta * N + t + NT * o];
  }
}

// Sum over the 64 lanes of a wave of eight values per lane.  On return the
// lanes 8 i .. 8 i + 7 hold the total of value i.
__device__ __forceinline__ float wave_sum8(const float (&v)[8], int lane) {
  const bool b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1;
  float u[4], w[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float send = b5 ? v[i] : v[i + 4];
    const float keep = b5 ? v[i + 4] : v[i];
    u[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float send = b4 ? u[i] : u[i + 2];
    const float keep = b4 ? u[i + 2] : u[i];
    w[i] = keep + __shfl_xor(send, 16, 64);
  }
  float z = (b3 ? w[1] : w[0]) + __shfl_xor(b3 ? w[0] : w[1], 8, 64);
  z += __shfl_xor(z, 4, 64);
  z += __shfl_xor(z, 2, 64);
  z += __shfl_xor(z, 1, 64);
  return z;
}

// dL/dC_s[me][l][tau] for this block: sum_k tb[k] p_l[(k - tau + nc) mod N']
// with tb = theta_bar of member `me` (positions t + NT o).  The p rows of
// the step are re-read from the exchange (round `tag`, still untouched
// because this member has not yet published a later round).  Writes
// n_sb x n_taps floats at `dst`.
template <int N>
__device__ __forceinline__ void coeff_grad(const TeamCtx& c, uint64_t* xrow, unsigned tag,
                                           const float (&p_own)[FftShape<N>::RR], const float (&tb_own)[FftShape<N>::RR],
                                           int n_taps, float* __restrict__ dst, float* lf) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT, NW = NT / 64;
  constexpr int PB = NlprLds<N>::PB;
  const int t = opaque_tid();
  const int lane = t & 63, wave = t >> 6;
  const int nsb = c.nsb, me = c.me, nc = c.nc;
  const int tap_pad = kTapChunk * c.n_chunks;
  const int hl = tap_pad - 1 - nc;
  float* th = lf + 2 * PB;
  float* red = th + NlprLds<N>::TH;  // [tap_pad][NW]

  __syncthreads();
#pragma unroll
  for (int o = 0; o < RR; ++o) th[pad_r(t + NT * o)] = tb_own[o];
  stage_row<N, RR, NT>(lf, p_own, t, hl, nc);  // rows in the order me, me + 1, ... (mod n_sb)
  __syncthreads();
  float tb[RR];  // block mapping t RR + q
#pragma unroll
  for (int q = 0; q < RR; ++q) tb[q] = th[pad_r(t * RR + q)];

  for (int j = 0; j < nsb; ++j) {
    const float* cur = lf + (j & 1) * PB;
    const int l = me + j < nsb ? me + j : me + j - nsb;  // the row used now
    const int ln = l + 1 < nsb ? l + 1 : 0;                // the next one (remote)
    const bool more = j + 1 < nsb;
    uint64_t w[RR];
    if (more) xissue<RR>(xrow + (size_t)ln * N, t, NT, w);
    // window W[i] = cur[t RR + i]; chunk ch of taps reads W[tap_pad - 8 ch - 8 + i]
    float win[RR + kTapChunk];
    int start = t * RR;
    load_row4<RR + kTapChunk, 0>(cur, start, win);
    for (int ch = c.n_chunks - 1; ch >= 0; --ch) {
      float part[kTapChunk];
#pragma unroll
      for (int tt = 0; tt < kTapChunk; ++tt) {
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q < RR; ++q) acc = fmaf(tb[q], win[q - tt + kTapChunk - 1], acc);
        part[tt] = acc;
      }
      const float z = wave_sum8(part, lane);
      if ((lane & 7) == 0) red[(kTapChunk * ch + (lane >> 3)) * NW + wave] = z;
      if (ch > 0) {
#pragma unroll
        for (int i = 0; i < RR; ++i) win[i] = win[i + kTapChunk];
        start += kTapChunk;
        load_row4<kTapChunk, RR>(cur, start + RR, win);
      }
    }
    if (more) {
      float v[RR];
      xcomplete<RR>(xrow + (size_t)ln * N, t, NT, tag, c.ctl, w, v);
      stage_row<N, RR, NT>(lf + ((j + 1) & 1) * PB, v, t, hl, nc);
    }
    __syncthreads();
    for (int tau = t; tau < n_taps; tau += NT) {
      float sum = 0.0f;
      for (int wv = 0; wv < NW; ++wv) sum += red[tau * NW + wv];
      dst[(size_t)l * n_taps + tau] = sum;
    }
    __syncthreads();
  }
}

// Sum over the workgroup (NW waves) of one double per thread; the total is
// returned to thread 0.  red: NW doubles of LDS.
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* red, int t) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  __syncthreads();
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double sum = 0.0;
  if (t == 0)
    for (int wv = 0; wv < NW; ++wv) sum += red[wv];
  return sum;
}

// rho partial: sum over owned bins of phi_q L Im(conj(g) a), both polarisations.
template <int N>
__device__ __forceinline__ double rho_term(const double* __restrict__ phase_km, double L, int t,
                                           const float2 (&gx)[FftShape<N>::RR], const float2 (&gy)[FftShape<N>::RR],
                                           const float2 (&ax)[FftShape<N>::RR], const float2 (&ay)[FftShape<N>::RR]) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  double acc = 0.0;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    const double ph = phase_km[t + NT * o] * L;
    const float im = (gx[o].x * ax[o].y - gx[o].y * ax[o].x) + (gy[o].x * ay[o].y - gy[o].y * ay[o].x);
    acc += ph * (double)im;
  }
  return acc;
}

// exp(-j theta) - 1 with both parts accurate for small theta:
// cos theta - 1 = -2 sin^2(theta / 2), sin theta = 2 sin(theta / 2) cos(theta / 2).
__device__ __forceinline__ float2 rot_minus_one(float th) {
  float sh, ch;
  phase_sincos(0.5f * th, sh, ch);
  return make_float2(-2.0f * sh * sh, -2.0f * sh * ch);
}

// phi'_q = phi_q - phi(f_i) of owned bin t + NT o: the member's phase table
// relative to its centre bin N'/2.
template <int N>
__device__ __forceinline__ float phase_rel(const double* __restrict__ phase_km, int t, int o) {
  return (float)(phase_km[t + FftShape<N>::NT * o] - phase_km[N / 2]);
}

__device__ __forceinline__ float im_conj_mul(float2 a, float2 b) { return fmaf(a.x, b.y, -a.y * b.x); }

template <int LOGN>
__global__ __launch_bounds__(FftShape<(1 << LOGN)>::NT, 2) void bwd_kernel(BwdArgs a) {
  constexpr int N = 1 << LOGN;  // N'
  using S = FftShape<N>;
  constexpr int RR = S::RR, NT = S::NT, NW = NT / 64;
  __shared__ __align__(16) float lf[lds_floats<N>()];
  __shared__ double rho_red[NW];
  __shared__ unsigned epoch_word;
  float4* lxy = reinterpret_cast<float4*>(lf);

  TeamCtx c;
  c.nsb = a.n_sb;
  const int r = blockIdx.x / kXcds;
  c.me = r % c.nsb;
  c.team = (r / c.nsb) * kXcds + blockIdx.x % kXcds;
  if (c.team >= a.n_teams) return;
  c.n_chunks = a.n_chunks;
  c.nc = a.nc;
  c.ctl = a.ctl;
  c.tab = &a.tab;
  const int nsb = c.nsb, me = c.me;
  const float2* tw = a.tab.tw;
  const int T = a.T;
  const int tap_pad = kTapChunk * a.n_chunks;
  const int k = a.ck_every;
  const size_t spec_sz = (size_t)2 * N;  // one member's spectra, two polarisations (float2)
  const size_t vt_sz = (size_t)kVtFloats * N;  // one member's step record (A, theta, D), floats
  float2* team_spec = a.spec + (size_t)c.team * a.n_ck * nsb * spec_sz;
  float* team_vt = a.vtheta + (size_t)c.team * k * nsb * vt_sz;
  auto sp = [&](int slot) { return team_spec + ((size_t)slot * nsb + me) * spec_sz; };
  auto vt = [&](int slot) { return team_vt + ((size_t)slot * nsb + me) * vt_sz; };
  float2* gsv = a.gsave + ((size_t)c.team * nsb + me) * 2 * N;  // reused by every reverse step
  const int last0 = (a.n_ck - 1) * k;  // first step of the last segment
  uint64_t* xs_team = a.xspec + (size_t)c.team * 2 * nsb * 4 * N;
  // the team's intensity slots (n_sb x N' words each) at the start of the
  // region the forward kernel's team of the same index uses (2 x n_sb x 2 N'
  // words): a word of it is only ever written by this team's rounds, which
  // take their tags from this team's round counter
  uint64_t* xp_team = a.xp + (size_t)c.team * 2 * nsb * 2 * N;
  const double* phase_km = a.phase + (size_t)me * N;
  const unsigned first = epoch_begin(a.epoch + c.team, &epoch_word);

  unsigned iter = 0;
  for (int item = c.team; item < a.n_items; item += a.n_teams, ++iter) {
    int t = opaque_tid();
    unsigned rnd = first + iter * a.rounds_per_item;
    unsigned np = 0, nq = 0;  // p- and theta_bar-rounds so far (slot parity)
    // one spectrum slot for the three spectrum rounds of this block (the step
    // rounds between them keep the exchange's reuse rule); the next block
    // takes the other slot
    uint64_t* xs = xs_team + (size_t)(iter & 1u) * nsb * 4 * N;
    const int inst = item / a.nblk;
    const int blk = item - inst * a.nblk;
    float2 x[RR], y[RR], gx[RR], gy[RR];
    double rho_acc = 0.0;

    // Forward step s (0-based) on x / y with its intensity exchange round;
    // stores (A, theta, D) at `dst` if given, and stops after theta if !tail.
    auto forward_step = [&](int s, float* dst, bool tail) {
      t = opaque_tid();
      apply_diag<N, false>(x, y, step_gvd(a.tab, s) + (size_t)me * N, t);
      float2* rec = dst != nullptr ? reinterpret_cast<float2*>(dst) : nullptr;  // A
      if (dst != nullptr) {
#pragma unroll
        for (int o = 0; o < RR; ++o) {
          rec[t + NT * o] = x[o];
          rec[N + t + NT * o] = y[o];
        }
      }
      fft<N, true>(x, y, lxy, tw, t);
      float p[RR], theta[RR];
      intensity<N>(x, y, p);
      uint64_t* xrow = xp_team + (size_t)(np & 1u) * nsb * N;
      coupled_fir<N>(c, a.tab.cpad + ((size_t)(s * nsb + me) * nsb) * tap_pad, xrow, rnd, p, theta, lf);
      ++rnd;
      ++np;
      if (dst != nullptr) {
        t = opaque_tid();
        store_theta<N>(dst, theta, t);
        // D = DFT(e v), the transform of w - v
        float2 dx[RR], dy[RR];
#pragma unroll
        for (int o = 0; o < RR; ++o) {
          const float2 e = rot_minus_one(theta[o]);
          dx[o] = cmul(e, x[o]);
          dy[o] = cmul(e, y[o]);
        }
        fft<N, false>(dx, dy, lxy, tw, t);
#pragma unroll
        for (int o = 0; o < RR; ++o) {
          rec[kVtD * N / 2 + t + NT * o] = dx[o];
          rec[kVtD * N / 2 + N + t + NT * o] = dy[o];
        }
      }
      if (tail) {
        rotate<N, -1>(x, y, theta);
        fft<N, false>(x, y, lxy, tw, t);
      }
    };

    // ---- A: forward sweep
    const float2* in_x = a.in + (size_t)inst * 2 * T;
    gather_block<N, false>(in_x, in_x + T, blk, a.hop, a.n_ov, T, a.boundary, nsb, me, t, x, y);
    fft<N, false>(x, y, lxy, tw, t);
    polyphase_to_subband<N>(c, xs, rnd++, t, x, y);
    for (int s = 0; s < a.steps; ++s) {
      if (s % k == 0) store_state<N>(sp(s / k), x, y, opaque_tid());
      forward_step(s, s >= last0 ? vt(s - last0) : nullptr, true);
    }

    // ---- B: adjoint of the output stage
    t = opaque_tid();
    apply_diag<N, false>(x, y, a.tab.h_last + (size_t)me * N, t);  // B
    const float2* go_x = a.gout + (size_t)inst * 2 * T;
    gather_block<N, true>(go_x, go_x + T, blk, a.hop, a.n_ov, T, a.boundary, nsb, me, t, gx, gy);
    fft<N, false>(gx, gy, lxy, tw, t);
    polyphase_to_subband<N>(c, xs, rnd++, t, gx, gy);  // g_B
    if (a.lpart != nullptr) {
      // dL/d(length of the last dispersion segment) = -sum phi Im(conj(g_B) B)
      const double tb = rho_term<N>(phase_km, 1.0, t, gx, gy, x, y);
      const double tot = block_sum<NW>(-tb, rho_red, t);
      if (t == 0) a.lpart[((size_t)item * nsb + me) * (a.steps + 1) + a.steps] = tot;
    }
    apply_diag<N, true>(gx, gy, a.tab.h_last + (size_t)me * N, t);  // g_{S_Nst}

    // ---- C: reverse sweep, segment by segment
    for (int seg = a.n_ck - 1; seg >= 0; --seg) {
      const int s0 = seg * k;
      const int s1 = min(s0 + k, a.steps);
      if (seg != a.n_ck - 1) {  // recompute (v, theta) of the segment's steps
        load_state<N>(sp(seg), x, y, opaque_tid());
        for (int j = 0; j < s1 - s0; ++j) forward_step(s0 + j, vt(j), j + 1 < s1 - s0);
      }
      for (int s = s1; s > s0; --s) {  // 1-based step s
        t = opaque_tid();
        const float2* hs = step_gvd(a.tab, s - 1) + (size_t)me * N;
        float p[RR], theta[RR], tbar[RR];
        const float2* rec = reinterpret_cast<const float2*>(vt(s - 1 - s0));  // A, then D at kVtD N' floats
        // keep g_S for g_A = N' g_S + E and the split-ratio terms
#pragma unroll
        for (int o = 0; o < RR; ++o) {
          gsv[t + NT * o] = gx[o];
          gsv[N + t + NT * o] = gy[o];
        }
        load_atheta<N>(vt(s - 1 - s0), x, y, theta, t);  // A, theta of step s
        fft<N, true>(x, y, lxy, tw, t);                   // v = IDFT(A), as in the forward sweep
        intensity<N>(x, y, p);
        // republish p for the coefficient gradient of the other members
        const unsigned tag_p = rnd++;
        uint64_t* prow = xp_team + (size_t)(np & 1u) * nsb * N;
        ++np;
        if (nsb > 1) {
#pragma unroll
          for (int o = 0; o < RR; ++o) xput(prow + (size_t)me * N + t + NT * o, p[o], tag_p);
        }
        // g_w, theta_bar
        fft<N, true>(gx, gy, lxy, tw, t);
#pragma unroll
        for (int o = 0; o < RR; ++o) {
          float sn, cs;
          phase_sincos(theta[o], sn, cs);
          const float2 rot = make_float2(cs, -sn);
          const float2 wx = cmul(x[o], rot), wy = cmul(y[o], rot);
          tbar[o] = (gx[o].x * wx.y - gx[o].y * wx.x) + (gy[o].x * wy.y - gy[o].y * wy.x);
        }
        coeff_grad<N>(c, prow, tag_p, p, tbar, a.n_taps,
                      a.cpart + ((((size_t)item * a.steps + (s - 1)) * nsb + me) * nsb) * a.n_taps, lf);
        // p_bar: transposed filter over the team's theta_bar rows
        float pbar[RR];
        uint64_t* qrow = a.xq + ((size_t)c.team * 2 + (nq & 1u)) * nsb * N;
        ++nq;
        coupled_fir<N>(c, a.ctpad + ((size_t)((s - 1) * nsb + me) * nsb) * tap_pad, qrow, rnd++, tbar, pbar, lf);
        // g_v = g_w exp(+j theta) + 2 p_bar v = g_w + dg, dg = conj(e) g_w + 2 p_bar v
#pragma unroll
        for (int o = 0; o < RR; ++o) {
          const float2 e = rot_minus_one(theta[o]);
          const float p2 = 2.0f * pbar[o];
          gx[o] = make_float2(fmaf(p2, x[o].x, fmaf(e.x, gx[o].x, e.y * gx[o].y)),
                              fmaf(p2, x[o].y, fmaf(e.x, gx[o].y, -e.y * gx[o].x)));
          gy[o] = make_float2(fmaf(p2, y[o].x, fmaf(e.x, gy[o].x, e.y * gy[o].y)),
                              fmaf(p2, y[o].y, fmaf(e.x, gy[o].y, -e.y * gy[o].x)));
        }
        fft<N, false>(gx, gy, lxy, tw, t);  // E = DFT(dg)
        // split-ratio terms sum phi' [Im(conj(g_S) D) - Im(conj(E) A)]; g_A = N' g_S + E
#pragma unroll
        for (int o = 0; o < RR; ++o) {
          const float w = phase_rel<N>(phase_km, t, o);
          const float2 sx = gsv[t + NT * o], sy = gsv[N + t + NT * o];
          const float im = im_conj_mul(sx, rec[kVtD * N / 2 + t + NT * o]) +
                           im_conj_mul(sy, rec[kVtD * N / 2 + N + t + NT * o]) -
                           im_conj_mul(gx[o], rec[t + NT * o]) - im_conj_mul(gy[o], rec[N + t + NT * o]);
          rho_acc -= a.L * (double)(w * im);
          gx[o] = make_float2(fmaf((float)N, sx.x, gx[o].x), fmaf((float)N, sx.y, gx[o].y));
          gy[o] = make_float2(fmaf((float)N, sy.x, gy[o].x), fmaf((float)N, sy.y, gy[o].y));
        }
        if (a.lpart != nullptr) {  // dL/d(length of segment s - 1) = -sum phi Im(conj(g_A) A)
          float2 ax[RR], ay[RR];
#pragma unroll
          for (int o = 0; o < RR; ++o) {
            ax[o] = rec[t + NT * o];
            ay[o] = rec[N + t + NT * o];
          }
          const double ta = rho_term<N>(phase_km, 1.0, t, gx, gy, ax, ay);
          const double tot = block_sum<NW>(-ta, rho_red, t);
          if (t == 0) a.lpart[((size_t)item * nsb + me) * (a.steps + 1) + (s - 1)] = tot;
        }
        apply_diag<N, true>(gx, gy, hs, t);  // g_{S_{s-1}}
      }
    }

    // ---- D: adjoint of the input stage (optional)
    if (a.gin_blk != nullptr) {
      t = opaque_tid();
      subband_to_polyphase<N>(c, xs, rnd++, t, gx, gy);
      fft<N, true>(gx, gy, lxy, tw, t);
      float2* dst = a.gin_blk + (size_t)item * 2 * nsb * N;
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const int n = nsb * (t + NT * o) + me;
        const float sg = (n & 1) ? -1.0f : 1.0f;
        dst[n] = cscale(gx[o], sg);
        dst[(size_t)nsb * N + n] = cscale(gy[o], sg);
      }
    }

    // ---- split-ratio partial of this member
    {
      t = opaque_tid();
      double v = rho_acc;
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
      __syncthreads();
      if ((t & 63) == 0) rho_red[t >> 6] = v;
      __syncthreads();
      if (t == 0) {
        double sum = 0.0;
        for (int wv = 0; wv < NW; ++wv) sum += rho_red[wv];
        a.rpart[(size_t)item * nsb + me] = sum;
      }
    }
  }
  epoch_end(a.epoch + c.team, first, iter * a.rounds_per_item, me);
}

// ------------------------------------------------------------------ reductions
// out[j] = sum over items of part[item][j] in FP64.  Thread (jj, g) of a
// 64 x 16 block sums items g, g + 16, ... in order; the 16 partial sums are
// then added in a fixed tree order, so the result does not depend on timing.
constexpr int kRedJ = 64, kRedG = 16;
__global__ __launch_bounds__(kRedJ * kRedG) void reduce_items_kernel(const float* __restrict__ part,
                                                                     float* __restrict__ out, int n_items,
                                                                     int per_item) {
  __shared__ double buf[kRedG][kRedJ];
  const int jj = threadIdx.x % kRedJ, g = threadIdx.x / kRedJ;
  const int j = blockIdx.x * kRedJ + jj;
  double acc = 0.0;
  if (j < per_item)
    for (int it = g; it < n_items; it += kRedG) acc += (double)part[(size_t)it * per_item + j];
  buf[g][jj] = acc;
  __syncthreads();
  for (int w = kRedG / 2; w > 0; w >>= 1) {
    if (g < w) buf[g][jj] += buf[g + w][jj];
    __syncthreads();
  }
  if (g == 0 && j < per_item) out[j] = (float)buf[0][jj];
}

// out[j] = sum over k of part[k][j], k < n (items x members), for j < m: block j
// sums a strided share per thread and adds the shares in a fixed tree.
__global__ void reduce_len_kernel(const double* __restrict__ part, double* __restrict__ out, int n, int m) {
  __shared__ double buf[256];
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) acc += part[(size_t)k * m + j];
  buf[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = buf[0];
}

__global__ void reduce_rho_kernel(const double* __restrict__ part, float* __restrict__ out, int n) {
  __shared__ double buf[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  buf[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = (float)buf[0];
}

__device__ __forceinline__ long long floor_div(long long a, long long h) {
  return a >= 0 ? a / h : -((-a + h - 1) / h);
}
__device__ __forceinline__ long long ceil_div(long long a, long long h) { return -floor_div(-a, h); }

// grad_in[inst][pol][pos] = sum over the blocks that read input sample pos of
// their input cotangents (blocks in order, FP64 accumulation).
__global__ void gather_gin_kernel(const float2* __restrict__ blk_g, float2* __restrict__ gin, int T, int N, int hop,
                                  int n_ov, int nblk, int batch, int boundary) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)batch * 2 * T) return;
  const int pos = (int)(idx % T);
  const int pol = (int)((idx / T) % 2);
  const int inst = (int)(idx / (2LL * T));
  double ax = 0.0, ay = 0.0;
  auto add = [&](int b, int n) {
    const float2 v = blk_g[((size_t)(inst * nblk + b) * 2 + pol) * N + n];
    ax += v.x;
    ay += v.y;
  };
  const int off = n_ov / 2;
  if (boundary == 1 || T >= N) {
    const int m_lo = boundary == 1 ? 0 : -1, m_hi = boundary == 1 ? 0 : 2;
    for (int m = m_lo; m <= m_hi; ++m) {
      const long long P = (long long)pos + (long long)m * T;  // unwrapped position
      // blocks b with start b hop - off <= P < start + N
      long long b_lo = ceil_div(P + off - N + 1, hop);
      long long b_hi = floor_div(P + off, hop);
      if (b_lo < 0) b_lo = 0;
      if (b_hi > nblk - 1) b_hi = nblk - 1;
      for (long long b = b_lo; b <= b_hi; ++b) {
        const long long n = P - (b * hop - off);
        if (n >= 0 && n < N) add((int)b, (int)n);
      }
    }
  } else {  // sequence shorter than a block: a block wraps over it several times
    for (int b = 0; b < nblk; ++b) {
      const long long start = (long long)b * hop - off;
      long long n0 = ((long long)pos - start) % T;
      if (n0 < 0) n0 += T;
      for (long long n = n0; n < N; n += T) add(b, (int)n);
    }
  }
  gin[((size_t)inst * 2 + pol) * T + pos] = make_float2((float)ax, (float)ay);
}

// ------------------------------------------------------------------ launchers
template <int LOGN>
static int launch_bwd_t(const BwdArgs& args, int grid, hipStream_t s) {
  void* kargs[] = {(void*)&args};
  const dim3 threads(FftShape<(1 << LOGN)>::NT);
  hipError_t e = stream_capturing(s)
                     ? hipLaunchKernel((const void*)bwd_kernel<LOGN>, dim3(grid), threads, kargs, 0, s)
                     : hipLaunchCooperativeKernel((const void*)bwd_kernel<LOGN>, dim3(grid), threads, kargs, 0, s);
  return e == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

template <int LOGN>
static int bwd_occ_t(int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, bwd_kernel<LOGN>, FftShape<(1 << LOGN)>::NT, 0) ==
                 hipSuccess
             ? CBESSFM_OK
             : CBESSFM_EHIP;
}

int bwd_occupancy_per_cu(int log_np, int* blocks) {
  switch (log_np) {
    case 8: return bwd_occ_t<8>(blocks);
    case 9: return bwd_occ_t<9>(blocks);
    case 10: return bwd_occ_t<10>(blocks);
    case 11: return bwd_occ_t<11>(blocks);
    case 12: return bwd_occ_t<12>(blocks);
    case 13: return bwd_occ_t<13>(blocks);
    default: return CBESSFM_EUNSUPPORTED;
  }
}

BwdLayout bwd_layout(const cbessfm_plan_t* p, long long T, int batch, int ck_every) {
  BwdLayout L;
  // one segment (nothing recomputed) for ck_every <= 1 or >= steps
  L.k = (ck_every <= 1 || ck_every > p->steps) ? p->steps : ck_every;
  L.n_ck = (p->steps + L.k - 1) / L.k;
  L.nblk = (int)((T + p->hop - 1) / p->hop);
  L.n_items = batch * L.nblk;
  L.n_teams = L.n_items < p->bwd_team_capacity ? L.n_items : p->bwd_team_capacity;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t nsb = p->sb.n_sb;
  L.spec_off = 0;
  L.vtheta_off = up(L.spec_off + sizeof(float2) * (size_t)L.n_teams * L.n_ck * nsb * 2 * p->Np);
  L.gsave_off = up(L.vtheta_off + sizeof(float) * (size_t)L.n_teams * L.k * nsb * kVtFloats * p->Np);
  L.cpart_off = up(L.gsave_off + sizeof(float2) * (size_t)L.n_teams * nsb * 2 * p->Np);
  L.rpart_off = up(L.cpart_off + sizeof(float) * (size_t)L.n_items * p->steps * nsb * nsb * p->n_taps);
  L.lpart_off = up(L.rpart_off + sizeof(double) * (size_t)L.n_items * nsb);
  L.gin_off = up(L.lpart_off + sizeof(double) * (size_t)L.n_items * nsb * (p->steps + 1));
  L.bytes = up(L.gin_off + sizeof(float2) * (size_t)L.n_items * 2 * p->N);
  return L;
}

int launch_backward(cbessfm_plan_t* p, const void* field_in, const void* grad_out, void* grad_in, float* grad_c,
                    float* grad_rho, double* grad_gvd, long long T, int batch, int ck_every, void* workspace,
                    size_t ws_bytes, hipStream_t s) {
  const BwdLayout L = bwd_layout(p, T, batch, ck_every);
  if (ws_bytes < L.bytes) return CBESSFM_EWORKSPACE;
  char* ws = static_cast<char*>(workspace);
  BwdArgs a;
  a.in = static_cast<const float2*>(field_in);
  a.gout = static_cast<const float2*>(grad_out);
  a.T = (int)T;
  a.nblk = L.nblk;
  a.n_items = L.n_items;
  a.n_sb = p->sb.n_sb;
  a.steps = p->steps;
  a.n_chunks = p->n_chunks;
  a.nc = p->n_taps / 2;
  a.n_taps = p->n_taps;
  a.n_ov = p->sb.overlap;
  a.hop = p->hop;
  a.boundary = p->sb.boundary;
  a.n_teams = L.n_teams;
  a.ck_every = L.k;
  a.n_ck = L.n_ck;
  fill_tables(p, a.tab);
  a.ctpad = p->d_ctpad;
  a.phase = p->d_phase;
  a.L = p->step_km;
  a.xspec = p->d_xspec;
  a.xp = p->d_xp;
  a.xq = p->d_xq;
  a.spec = reinterpret_cast<float2*>(ws + L.spec_off);
  a.vtheta = reinterpret_cast<float*>(ws + L.vtheta_off);
  a.gsave = reinterpret_cast<float2*>(ws + L.gsave_off);
  a.cpart = reinterpret_cast<float*>(ws + L.cpart_off);
  a.rpart = reinterpret_cast<double*>(ws + L.rpart_off);
  a.lpart = grad_gvd ? reinterpret_cast<double*>(ws + L.lpart_off) : nullptr;
  a.gin_blk = grad_in ? reinterpret_cast<float2*>(ws + L.gin_off) : nullptr;
  a.ctl.abort = p->d_abort;
  a.ctl.err = p->d_err;
  a.ctl.spin_limit = p->wait_limit;
  a.rounds_per_item = 4u * (unsigned)p->steps + 4u;
  a.epoch = p->d_epoch;
  const int groups = (a.n_teams + kXcds - 1) / kXcds;
  const int grid = groups * kXcds * a.n_sb;
  int rc;
  switch (p->log_np) {
    case 8: rc = launch_bwd_t<8>(a, grid, s); break;
    case 9: rc = launch_bwd_t<9>(a, grid, s); break;
    case 10: rc = launch_bwd_t<10>(a, grid, s); break;
    case 11: rc = launch_bwd_t<11>(a, grid, s); break;
    case 12: rc = launch_bwd_t<12>(a, grid, s); break;
    case 13: rc = launch_bwd_t<13>(a, grid, s); break;
    default: rc = CBESSFM_EUNSUPPORTED;
  }
  if (rc) return rc;
  const int per_item = p->steps * a.n_sb * a.n_sb * p->n_taps;
  reduce_items_kernel<<<(per_item + kRedJ - 1) / kRedJ, kRedJ * kRedG, 0, s>>>(a.cpart, grad_c, a.n_items, per_item);
  reduce_rho_kernel<<<1, 256, 0, s>>>(a.rpart, grad_rho, a.n_items * a.n_sb);
  if (grad_gvd)
    reduce_len_kernel<<<p->steps + 1, 256, 0, s>>>(a.lpart, grad_gvd, a.n_items * a.n_sb, p->steps + 1);
  if (hipGetLastError() != hipSuccess) return CBESSFM_EHIP;
  if (grad_in)
    return launch_gather_gin(a.gin_blk, static_cast<float2*>(grad_in), T, p->N, p->hop, p->sb.overlap, a.nblk, batch,
                             p->sb.boundary, s);
  return CBESSFM_OK;
}

int launch_gather_gin(const float2* blk_g, float2* gin, long long T, int N, int hop, int n_ov, int nblk, int batch,
                      int boundary, hipStream_t s) {
  const long long total = (long long)batch * 2 * T;
  gather_gin_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(blk_g, gin, (int)T, N, hop, n_ov, nblk, batch,
                                                                     boundary);
  return hipGetLastError() == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

// ------------------------------------------------------------------ fixed scratch
// Device memory of cbessfm_backward_static: one array per device, held until
// the process ends, shared by every such call on that device (calls that
// overlap in time on one device race on it).  The kernels write every part
// of the workspace they later read (the FP64 accumulators of the streaming
// path are cleared by a kernel at the start of each call), so nothing is
// cleared here.  In host code `scratch` is only a stand-in for the symbol:
// its device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[CBESSFM_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};
}  // namespace

int static_scratch(int device, void** ptr) {
  if (device < 0 || device >= kMaxScratchDevices) return CBESSFM_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return CBESSFM_EHIP;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return CBESSFM_OK;
}

}  // namespace cbessfm
