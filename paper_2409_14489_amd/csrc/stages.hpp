// Block stages shared by the forward and adjoint kernels.
//
// Conventions (see fft_lds.hpp for the register layout): a workgroup is
// member `me` of a team of n_sb workgroups processing one overlap-and-save
// block; x / y hold the member's two polarisations at positions t + NT o.
// In the frequency domain the member holds subband `me` in subband order
// (bin j of subband i is the block bin i N' + j - N/2); at the block's input
// and output it holds the polyphase component n = n_sb n1 + me.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "internal.hpp"
#include "sincos.hpp"
#include "team.hpp"

namespace cbessfm {

// What a member needs to know about its team and block.
struct TeamCtx {
  int nsb, me, team;
  int n_chunks, nc;
  XchgCtl ctl;
  const Tables* tab;
};

template <int N>
struct Regs {
  static constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
};

// x / y *= h[t + NT o] (h already offset to the member's subband).
template <int N, bool CONJ>
__device__ __forceinline__ void apply_diag(float2 (&x)[FftShape<N>::RR], float2 (&y)[FftShape<N>::RR],
                                           const float2* __restrict__ h, int t) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    const float2 hv = h[t + NT * o];
    x[o] = CONJ ? cmulc(x[o], hv) : cmul(x[o], hv);
    y[o] = CONJ ? cmulc(y[o], hv) : cmul(y[o], hv);
  }
}

// Gathers the polyphase component `me` of a block of a sequence (both
// polarisations), times (-1)^n.  Forward use: every sample of the block
// (framing of Sec. III-A).  KEEP_ONLY: only samples in [n_ov/2, N - n_ov/2)
// that fall inside [0, T) after the hop offset (the adjoint of the output
// write); all others read as zero.
template <int N, bool KEEP_ONLY>
__device__ __forceinline__ void gather_block(const float2* __restrict__ sx, const float2* __restrict__ sy,
                                             int blk, int hop, int n_ov, int T, int boundary, int nsb, int me,
                                             int t, float2 (&x)[FftShape<N>::RR], float2 (&y)[FftShape<N>::RR]) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  const int first = KEEP_ONLY ? 0 : frame_first(blk, hop, n_ov, T, boundary);
  const bool short_seq = T < nsb * N;
  const int keep_lo = n_ov / 2, keep_hi = nsb * N - n_ov / 2;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    const int n = nsb * (t + NT * o) + me;
    int pos;
    if (KEEP_ONLY) {
      pos = blk * hop + n - keep_lo;
      if (n < keep_lo || n >= keep_hi || pos >= T) pos = -1;
    } else {
      pos = frame_pos(first, n, T, boundary, short_seq);
    }
    float2 vx = make_float2(0.f, 0.f), vy = vx;
    if (pos >= 0) {
      vx = sx[pos];
      vy = sy[pos];
    }
    const float sg = (n & 1) ? -1.0f : 1.0f;
    x[o] = cscale(vx, sg);
    y[o] = cscale(vy, sg);
  }
}

// Writes the kept samples [n_ov/2, N - n_ov/2) of the block's polyphase
// component `me` (times (-1)^n) to the output sequence.
template <int N>
__device__ __forceinline__ void scatter_block(float2* __restrict__ dx, float2* __restrict__ dy, int blk, int hop,
                                              int n_ov, int T, int nsb, int me, int t,
                                              const float2 (&x)[FftShape<N>::RR], const float2 (&y)[FftShape<N>::RR]) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  const int keep_lo = n_ov / 2, keep_hi = nsb * N - n_ov / 2;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    const int n = nsb * (t + NT * o) + me;
    const int pos = blk * hop + n - keep_lo;
    if (n >= keep_lo && n < keep_hi && pos < T) {
      const float sg = (n & 1) ? -1.0f : 1.0f;
      dx[pos] = cscale(x[o], sg);
      dy[pos] = cscale(y[o], sg);
    }
  }
}

// Publishes this member's four spectrum components (x.re, x.im, y.re, y.im).
template <int N>
__device__ __forceinline__ void put_spectrum(uint64_t* dst, const float2 (&x)[FftShape<N>::RR],
                                             const float2 (&y)[FftShape<N>::RR], unsigned tag, int t) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    const int k = t + NT * o;
    xput(dst + 0 * N + k, x[o].x, tag);
    xput(dst + 1 * N + k, x[o].y, tag);
    xput(dst + 2 * N + k, y[o].x, tag);
    xput(dst + 3 * N + k, y[o].y, tag);
  }
}

// x / y = sum over members n2 of w_n2 * (member n2's spectrum),
// w_n2 = wsb[(n2 me) mod n_sb], conjugated when CONJ.  On entry x / y hold
// this member's own spectrum (already published), which is used from the
// registers; the other members' spectra come from the exchange.
template <int N, bool CONJ>
__device__ __forceinline__ void combine_spectra(const uint64_t* src, const TeamCtx& c, unsigned tag, int t,
                                                float2 (&x)[FftShape<N>::RR], float2 (&y)[FftShape<N>::RR]) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  {
    const float2 w = c.tab->wsb[(c.me * c.me) % c.nsb];
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      x[o] = CONJ ? cmulc(x[o], w) : cmul(x[o], w);
      y[o] = CONJ ? cmulc(y[o], w) : cmul(y[o], w);
    }
  }
  for (int n2 = 0; n2 < c.nsb; ++n2) {
    if (n2 == c.me) continue;
    const float2 w = c.tab->wsb[(n2 * c.me) % c.nsb];
    const uint64_t* row = src + (size_t)n2 * 4 * N;
    // all four components of the member in flight at once when they fit the
    // register file, else one at a time
    constexpr bool ALL4 = RR <= 8;
    float re[RR], im[RR];
    if constexpr (ALL4) {
      uint64_t wxr[RR], wxi[RR], wyr[RR], wyi[RR];
      xissue<RR>(row, t, NT, wxr);
      xissue<RR>(row + N, t, NT, wxi);
      xissue<RR>(row + 2 * N, t, NT, wyr);
      xissue<RR>(row + 3 * N, t, NT, wyi);
      xcomplete<RR>(row, t, NT, tag, c.ctl, wxr, re);
      xcomplete<RR>(row + N, t, NT, tag, c.ctl, wxi, im);
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const float2 v = make_float2(re[o], im[o]);
        x[o] = cadd(x[o], CONJ ? cmulc(v, w) : cmul(v, w));
      }
      xcomplete<RR>(row + 2 * N, t, NT, tag, c.ctl, wyr, re);
      xcomplete<RR>(row + 3 * N, t, NT, tag, c.ctl, wyi, im);
    } else {
      xget<RR>(row, t, NT, tag, c.ctl, re);
      xget<RR>(row + N, t, NT, tag, c.ctl, im);
#pragma unroll
      for (int o = 0; o < RR; ++o) {
        const float2 v = make_float2(re[o], im[o]);
        x[o] = cadd(x[o], CONJ ? cmulc(v, w) : cmul(v, w));
      }
      xget<RR>(row + 2 * N, t, NT, tag, c.ctl, re);
      xget<RR>(row + 3 * N, t, NT, tag, c.ctl, im);
    }
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      const float2 v = make_float2(re[o], im[o]);
      y[o] = cadd(y[o], CONJ ? cmulc(v, w) : cmul(v, w));
    }
  }
}

// Polyphase spectra -> subband spectrum: multiply by exp(-j 2 pi me k / N),
// exchange, n_sb-point DFT across the team (the input DEMUX of
// Fig. "scheme_CB-ESSFM").  No-op for one subband.
template <int N>
__device__ __forceinline__ void polyphase_to_subband(const TeamCtx& c, uint64_t* xs, unsigned tag, int t,
                                                     float2 (&x)[FftShape<N>::RR], float2 (&y)[FftShape<N>::RR]) {
  if (c.nsb == 1) return;
  apply_diag<N, false>(x, y, c.tab->poly_tw + (size_t)c.me * N, t);
  put_spectrum<N>(xs + (size_t)c.me * 4 * N, x, y, tag, t);
  combine_spectra<N, false>(xs, c, tag, t, x, y);
}

// Subband spectra -> polyphase spectra: the inverse direction (the MUX),
// conjugate weights and twiddles.  No-op for one subband.
template <int N>
__device__ __forceinline__ void subband_to_polyphase(const TeamCtx& c, uint64_t* xs, unsigned tag, int t,
                                                     float2 (&x)[FftShape<N>::RR], float2 (&y)[FftShape<N>::RR]) {
  if (c.nsb == 1) return;
  put_spectrum<N>(xs + (size_t)c.me * 4 * N, x, y, tag, t);
  combine_spectra<N, true>(xs, c, tag, t, x, y);
  apply_diag<N, true>(x, y, c.tab->poly_tw + (size_t)c.me * N, t);
}

// The DEMUX and MUX one polarisation at a time, through the team's two
// intensity-row slots (n_sb x 2 N' words each; a member's spectrum takes its
// 2 N' words, real parts then imaginary parts): x in round `round` in slot
// round & 1, y in round + 1 in the other slot.  A member publishes y only
// after it has consumed every member's x, which keeps the exchange's reuse
// rule (two uses of a slot are separated by another round); the two rounds
// touch n_sb x 2 N' words of the team's memory where one round of both
// polarisations would need a slot of n_sb x 4 N'.
template <int N>
__device__ __forceinline__ void put_pol(uint64_t* dst, const float2 (&v)[FftShape<N>::RR], unsigned tag, int t) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    const int k = t + NT * o;
    xput(dst + k, v[o].x, tag);
    xput(dst + N + k, v[o].y, tag);
  }
}

// v = sum over members n2 of w_n2 * (member n2's spectrum of this
// polarisation), w_n2 = wsb[(n2 me) mod n_sb], conjugated when CONJ; the
// member's own spectrum comes from v.
template <int N, bool CONJ>
__device__ __forceinline__ void combine_pol(const uint64_t* src, const TeamCtx& c, unsigned tag, int t,
                                            float2 (&v)[FftShape<N>::RR]) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  {
    const float2 w = c.tab->wsb[(c.me * c.me) % c.nsb];
#pragma unroll
    for (int o = 0; o < RR; ++o) v[o] = CONJ ? cmulc(v[o], w) : cmul(v[o], w);
  }
  for (int n2 = 0; n2 < c.nsb; ++n2) {
    if (n2 == c.me) continue;
    const float2 w = c.tab->wsb[(n2 * c.me) % c.nsb];
    const uint64_t* row = src + (size_t)n2 * 2 * N;
    uint64_t wr[RR], wi[RR];
    float re[RR], im[RR];
    xissue<RR>(row, t, NT, wr);
    xissue<RR>(row + N, t, NT, wi);
    xcomplete<RR>(row, t, NT, tag, c.ctl, wr, re);
    xcomplete<RR>(row + N, t, NT, tag, c.ctl, wi, im);
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      const float2 u = make_float2(re[o], im[o]);
      v[o] = cadd(v[o], CONJ ? cmulc(u, w) : cmul(u, w));
    }
  }
}

// polyphase_to_subband through the intensity-row slots xp (rounds round and
// round + 1).
template <int N>
__device__ __forceinline__ void polyphase_to_subband_xp(const TeamCtx& c, uint64_t* xp, unsigned round, int t,
                                                        float2 (&x)[FftShape<N>::RR],
                                                        float2 (&y)[FftShape<N>::RR]) {
  if (c.nsb == 1) return;
  apply_diag<N, false>(x, y, c.tab->poly_tw + (size_t)c.me * N, t);
  uint64_t* s0 = xp + (size_t)(round & 1u) * c.nsb * 2 * N;
  put_pol<N>(s0 + (size_t)c.me * 2 * N, x, round, t);
  combine_pol<N, false>(s0, c, round, t, x);
  uint64_t* s1 = xp + (size_t)((round + 1u) & 1u) * c.nsb * 2 * N;
  put_pol<N>(s1 + (size_t)c.me * 2 * N, y, round + 1u, t);
  combine_pol<N, false>(s1, c, round + 1u, t, y);
}

// subband_to_polyphase through the intensity-row slots xp (rounds round and
// round + 1).
template <int N>
__device__ __forceinline__ void subband_to_polyphase_xp(const TeamCtx& c, uint64_t* xp, unsigned round, int t,
                                                        float2 (&x)[FftShape<N>::RR],
                                                        float2 (&y)[FftShape<N>::RR]) {
  if (c.nsb == 1) return;
  uint64_t* s0 = xp + (size_t)(round & 1u) * c.nsb * 2 * N;
  put_pol<N>(s0 + (size_t)c.me * 2 * N, x, round, t);
  combine_pol<N, true>(s0, c, round, t, x);
  uint64_t* s1 = xp + (size_t)((round + 1u) & 1u) * c.nsb * 2 * N;
  put_pol<N>(s1 + (size_t)c.me * 2 * N, y, round + 1u, t);
  combine_pol<N, true>(s1, c, round + 1u, t, y);
  apply_diag<N, true>(x, y, c.tab->poly_tw + (size_t)c.me * N, t);
}

// A pointer every lane of the wave holds the same value of, made visible as
// such to the compiler (so that loads through it become scalar loads).
template <typename T>
__device__ __forceinline__ const T* uniform_ptr(const T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

// acc[q] += sum_{tau < 8 NCH} cl[tau] W[q - tau + 8 NCH - 1], q < QB, with the
// window W[i] = cur[pad_r(start + i)], i < QB + 8 NCH - 1, read once; the
// taps are compile-time, so every window index is static (no register moves)
// and the coefficients are scalar operands.
template <int NCH, int QB>
__device__ __forceinline__ void fir_row_fixed(const float* cur, int start, const float* __restrict__ cl,
                                              float* acc) {
  constexpr int TP = kTapChunk * NCH;
  constexpr int WN = (QB + TP - 1 + 3) & ~3;
  float win[WN];
  load_row4<WN, 0>(cur, start, win);
#pragma unroll
  for (int tau = 0; tau < TP; ++tau) {
    const float cv = cl[tau];
#pragma unroll
    for (int q = 0; q < QB; ++q) acc[q] = fmaf(cv, win[q - tau + TP - 1], acc[q]);
  }
}

// acc[q] += the filter of row `cur` (LDS, circularly extended) with the
// member's coefficient row cl (8 n_chunks taps, zero padded) at outputs
// start + q, q < QB: compile-time taps up to 32 (the window read once), a
// chunk loop beyond.
template <int QB>
__device__ __forceinline__ void fir_row(int n_chunks, const float* cur, int start, const float* __restrict__ cl,
                                        float* acc) {
  switch (n_chunks) {  // up to 32 taps: compile-time taps, window read once
    case 1: fir_row_fixed<1, QB>(cur, start, cl, acc); break;
    case 2: fir_row_fixed<2, QB>(cur, start, cl, acc); break;
    case 3: fir_row_fixed<3, QB>(cur, start, cl, acc); break;
    case 4: fir_row_fixed<4, QB>(cur, start, cl, acc); break;
    default: {
      float win[QB + kTapChunk];
      load_row4<QB + kTapChunk, 0>(cur, start, win);
      // the chunk's 8 coefficients, fetched one chunk ahead
      float cf[kTapChunk];
#pragma unroll
      for (int tt = 0; tt < kTapChunk; ++tt) cf[tt] = cl[kTapChunk * (n_chunks - 1) + tt];
      for (int ch = n_chunks - 1; ch >= 0; --ch) {
        float cf_next[kTapChunk];
        const int ch_next = ch > 0 ? ch - 1 : 0;
#pragma unroll
        for (int tt = 0; tt < kTapChunk; ++tt) cf_next[tt] = cl[kTapChunk * ch_next + tt];
#pragma unroll
        for (int tt = 0; tt < kTapChunk; ++tt) {
#pragma unroll
          for (int q = 0; q < QB; ++q)
            acc[q] = fmaf(cf[tt], win[q - tt + kTapChunk - 1], acc[q]);
        }
        if (ch > 0) {
#pragma unroll
          for (int i = 0; i < QB; ++i) win[i] = win[i + kTapChunk];
          start += kTapChunk;
          load_row4<kTapChunk, QB>(cur, start + QB, win);
        }
#pragma unroll
        for (int tt = 0; tt < kTapChunk; ++tt) cf[tt] = cf_next[tt];
      }
    }
  }
}

// Coupled intensity filter of eq. (15) for member `me`, circular over N':
//   out[k] = sum_l sum_tau crow[l][tau] in_l[(k - tau + nc) mod N'],
// crow = the member's coefficient rows ([n_sb][8 n_chunks], zero padded).
// own: this member's row at positions t + NT o; the other rows come from the
// tagged exchange `xrow` ([n_sb][N'], round `tag`).  Result at t + NT o.
// Rows are taken in the order me, me + 1, ... (mod n_sb): the member's own
// row needs no exchange, so the other members' rows travel while it is
// filtered.
template <int N>
__device__ __forceinline__ void coupled_fir(const TeamCtx& c, const float* __restrict__ crow, uint64_t* xrow,
                                           unsigned tag, const float (&own)[FftShape<N>::RR],
                                           float (&out)[FftShape<N>::RR], float* lf) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  constexpr int PB = NlprLds<N>::PB;  // row l lives at lf + (l & 1) * PB
  const int t = opaque_tid();
  const int nsb = c.nsb, me = c.me, nc = c.nc;
  const int tap_pad = kTapChunk * c.n_chunks;
  const int hl = tap_pad - 1 - nc;  // left halo of the circular extension
  float* th = lf + 2 * PB;

  if (nsb > 1) {
#pragma unroll
    for (int o = 0; o < RR; ++o) xput(xrow + (size_t)me * N + t + NT * o, own[o], tag);
  }
  __syncthreads();  // the LDS rows alias the FFT exchange buffers
  stage_row<N, RR, NT>(lf, own, t, hl, nc);
  __syncthreads();

  // The row of member l, circularly extended, is W[i] = cur[t RR + i] for this
  // thread's outputs k = t RR + q:  out[q] += sum_tau c[tau] W[q - tau + tap_pad - 1].
  // Outputs go in groups of QB <= 8; for each group the next row's matching
  // part is in flight while the group is filtered.  Taps go in chunks of 8
  // from the last chunk down; chunk ch reads W[g QB + tap_pad - 8 ch - 8 + i],
  // i < QB + 8, so each next chunk's window is the previous one moved by 8 (QB
  // floats are kept, 8 are read).
  constexpr int QB = RR < 8 ? RR : 8;
  constexpr int G = RR / QB;
  float acc[RR];
#pragma unroll
  for (int q = 0; q < RR; ++q) acc[q] = 0.0f;
  for (int j = 0; j < nsb; ++j) {
    const float* cur = lf + (j & 1) * PB;
    float* nxt = lf + ((j + 1) & 1) * PB;
    const int l = me + j < nsb ? me + j : me + j - nsb;  // the row filtered now
    const int ln = l + 1 < nsb ? l + 1 : 0;                // the next one (remote)
    const bool more = j + 1 < nsb;
    const uint64_t* nrow = xrow + (size_t)ln * N;
    const float* cl = uniform_ptr(crow + (size_t)l * tap_pad);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      uint64_t w[QB];
      if (more) xissue<QB>(nrow + NT * QB * g, t, NT, w);  // in flight during the filter
      int start = t * RR + g * QB;  // = t RR + g QB + tap_pad - 8 n_chunks
      fir_row<QB>(c.n_chunks, cur, start, cl, acc + g * QB);
      if (more) {  // this part of the next row into the other buffer (last read before the previous barrier)
        float v[QB];
        xcomplete<QB>(nrow + NT * QB * g, t, NT, tag, c.ctl, w, v);
        stage_row<N, QB, NT>(nxt, v, t + NT * QB * g, hl, nc);
      }
    }
    __syncthreads();
  }
  // block mapping (t RR + q) -> owned positions (t + NT o)
#pragma unroll
  for (int q = 0; q < RR; q += 4)
    *reinterpret_cast<float4*>(th + pad_r(t * RR + q)) = make_float4(acc[q], acc[q + 1], acc[q + 2], acc[q + 3]);
  __syncthreads();
#pragma unroll
  for (int o = 0; o < RR; ++o) out[o] = th[pad_r(t + NT * o)];
}

// The two filters of the dual-polarisation NLPR (eqs. (20)-(21)) in one
// exchange round: theta over the rows p_l = |x_l|^2 + |y_l|^2 with the
// coefficient rows crow, phi over d_l = |x_l|^2 - |y_l|^2 with drow (both
// [n_sb][8 n_chunks], zero padded).  Member l's two rows travel together in
// the round's slot (p at 2 N' l, d at 2 N' l + N'), so the filter costs one
// exchange latency instead of two.  LDS: the p rows double buffered at lf,
// the d rows at lf + 2 PB, the output staging at lf + 4 PB.  DualFir<N>::fits
// takes it where that fits the kernel's LDS and N' >= 4096: below, the
// second row set pushes the kernel to one wave per SIMD, and two rounds at
// two waves per SIMD are the better trade.  (At N' = 4096 the dual forward of
// the 5-channel workload went from 432 to 421 us.)
template <int N>
struct DualFir {
  static constexpr bool fits = N >= 4096 && 4 * NlprLds<N>::PB + NlprLds<N>::TH <= lds_floats<N>();
};

template <int N>
__device__ __forceinline__ void coupled_fir_dual(const TeamCtx& c, const float* __restrict__ crow,
                                                const float* __restrict__ drow, uint64_t* xrow, unsigned tag,
                                                const float (&own_p)[FftShape<N>::RR],
                                                const float (&own_d)[FftShape<N>::RR],
                                                float (&theta)[FftShape<N>::RR], float (&phi)[FftShape<N>::RR],
                                                float* lf) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  constexpr int PB = NlprLds<N>::PB;
  static_assert(DualFir<N>::fits, "LDS of the one-round dual filter");
  const int t = opaque_tid();
  const int nsb = c.nsb, me = c.me, nc = c.nc;
  const int tap_pad = kTapChunk * c.n_chunks;
  const int hl = tap_pad - 1 - nc;
  float* th = lf + 4 * PB;

  if (nsb > 1) {
    uint64_t* mine = xrow + (size_t)me * 2 * N;
#pragma unroll
    for (int o = 0; o < RR; ++o) xput(mine + t + NT * o, own_p[o], tag);
#pragma unroll
    for (int o = 0; o < RR; ++o) xput(mine + N + t + NT * o, own_d[o], tag);
  }
  __syncthreads();  // the LDS rows alias the FFT exchange buffers
  stage_row<N, RR, NT>(lf, own_p, t, hl, nc);
  stage_row<N, RR, NT>(lf + 2 * PB, own_d, t, hl, nc);
  __syncthreads();

  constexpr int QB = RR < 8 ? RR : 8;
  constexpr int G = RR / QB;
  float ap[RR], ad[RR];
#pragma unroll
  for (int q = 0; q < RR; ++q) {
    ap[q] = 0.0f;
    ad[q] = 0.0f;
  }
  for (int j = 0; j < nsb; ++j) {  // rows me, me + 1, ... (mod n_sb), as in coupled_fir
    const float* cur_p = lf + (j & 1) * PB;
    const float* cur_d = lf + (2 + (j & 1)) * PB;
    float* nxt_p = lf + ((j + 1) & 1) * PB;
    float* nxt_d = lf + (2 + ((j + 1) & 1)) * PB;
    const int l = me + j < nsb ? me + j : me + j - nsb;
    const int ln = l + 1 < nsb ? l + 1 : 0;
    const bool more = j + 1 < nsb;
    const uint64_t* nrow = xrow + (size_t)ln * 2 * N;
    const float* cl = uniform_ptr(crow + (size_t)l * tap_pad);
    const float* dl = uniform_ptr(drow + (size_t)l * tap_pad);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      // one row's words in flight at a time: the next p row's during this
      // p filter, the next d row's during this d filter
      const int start = t * RR + g * QB;
      {
        uint64_t w[QB];
        if (more) xissue<QB>(nrow + NT * QB * g, t, NT, w);
        fir_row<QB>(c.n_chunks, cur_p, start, cl, ap + g * QB);
        if (more) {
          float v[QB];
          xcomplete<QB>(nrow + NT * QB * g, t, NT, tag, c.ctl, w, v);
          stage_row<N, QB, NT>(nxt_p, v, t + NT * QB * g, hl, nc);
        }
      }
      {
        uint64_t w[QB];
        if (more) xissue<QB>(nrow + N + NT * QB * g, t, NT, w);
        fir_row<QB>(c.n_chunks, cur_d, start, dl, ad + g * QB);
        if (more) {
          float v[QB];
          xcomplete<QB>(nrow + N + NT * QB * g, t, NT, tag, c.ctl, w, v);
          stage_row<N, QB, NT>(nxt_d, v, t + NT * QB * g, hl, nc);
        }
      }
    }
    __syncthreads();
  }
  // block mapping (t RR + q) -> owned positions (t + NT o), one row after the other
#pragma unroll
  for (int q = 0; q < RR; q += 4)
    *reinterpret_cast<float4*>(th + pad_r(t * RR + q)) = make_float4(ap[q], ap[q + 1], ap[q + 2], ap[q + 3]);
  __syncthreads();
#pragma unroll
  for (int o = 0; o < RR; ++o) theta[o] = th[pad_r(t + NT * o)];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < RR; q += 4)
    *reinterpret_cast<float4*>(th + pad_r(t * RR + q)) = make_float4(ad[q], ad[q + 1], ad[q + 2], ad[q + 3]);
  __syncthreads();
#pragma unroll
  for (int o = 0; o < RR; ++o) phi[o] = th[pad_r(t + NT * o)];
}

// The coupled filter of eq. (15) in the frequency domain (the paper's form,
// Sec. III-A and Fig. "scheme_NLPR"): the member's intensity row is
// transformed (P_me = DFT(p), a complex transform of the real row), the
// spectra are exchanged, and
//   theta_me = (1/N') IDFT( sum_l chat[me][l] P_l ),
// chat[me][l] = DFT of coefficient row (me, l) placed circularly.  The same
// circular map as coupled_fir.  xrow: the team's exchange slot, member l's
// spectrum at xrow + 2 N' l (real parts, then imaginary parts); chat_me: the
// member's N_sb rows of N' bins for this step.  Result at t + NT o.
template <int N>
__device__ __forceinline__ void coupled_fir_freq(const TeamCtx& c, const float2* __restrict__ chat_me,
                                                uint64_t* xrow, unsigned tag, const float (&own)[FftShape<N>::RR],
                                                float (&out)[FftShape<N>::RR], float* lf) {
  constexpr int RR = FftShape<N>::RR, NT = FftShape<N>::NT;
  const int nsb = c.nsb, me = c.me;
  const float2* tw = c.tab->tw;
  float2* lx = reinterpret_cast<float2*>(lf);
  int t = opaque_tid();
  float2 z[RR];
#pragma unroll
  for (int o = 0; o < RR; ++o) z[o] = make_float2(own[o], 0.0f);
  fft1<N, false>(z, lx, tw, t);  // P_me at bins t + NT o
  t = opaque_tid();
  if (nsb > 1) {
    uint64_t* row = xrow + (size_t)me * 2 * N;
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      xput(row + t + NT * o, z[o].x, tag);
      xput(row + N + t + NT * o, z[o].y, tag);
    }
  }
  float2 acc[RR];
  {
    const float2* cm = chat_me + (size_t)me * N;
#pragma unroll
    for (int o = 0; o < RR; ++o) acc[o] = cmul(cm[t + NT * o], z[o]);
  }
  for (int l = 0; l < nsb; ++l) {
    if (l == me) continue;
    const uint64_t* row = xrow + (size_t)l * 2 * N;
    uint64_t wr[RR], wi[RR];
    xissue<RR>(row, t, NT, wr);
    xissue<RR>(row + N, t, NT, wi);
    float re[RR], im[RR];
    xcomplete<RR>(row, t, NT, tag, c.ctl, wr, re);
    xcomplete<RR>(row + N, t, NT, tag, c.ctl, wi, im);
    const float2* cl = chat_me + (size_t)l * N;
#pragma unroll
    for (int o = 0; o < RR; ++o) acc[o] = cadd(acc[o], cmul(cl[t + NT * o], make_float2(re[o], im[o])));
  }
  fft1<N, true>(acc, lx, tw, t);
  constexpr float inv_n = 1.0f / (float)N;
#pragma unroll
  for (int o = 0; o < RR; ++o) out[o] = acc[o].x * inv_n;
}

// x / y *= exp(-+ j theta): '-' (SIGN = -1) is the rotation of eq. (3).
template <int N, int SIGN>
__device__ __forceinline__ void rotate(float2 (&x)[FftShape<N>::RR], float2 (&y)[FftShape<N>::RR],
                                       const float (&theta)[FftShape<N>::RR]) {
  constexpr int RR = FftShape<N>::RR;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    float sn, cs;
    phase_sincos(theta[o], sn, cs);
    const float2 r = make_float2(cs, SIGN < 0 ? -sn : sn);
    x[o] = cmul(x[o], r);
    y[o] = cmul(y[o], r);
  }
}

template <int N>
__device__ __forceinline__ void intensity(const float2 (&x)[FftShape<N>::RR], const float2 (&y)[FftShape<N>::RR],
                                          float (&p)[FftShape<N>::RR]) {
#pragma unroll
  for (int o = 0; o < FftShape<N>::RR; ++o)
    p[o] = x[o].x * x[o].x + x[o].y * x[o].y + y[o].x * y[o].x + y[o].y * y[o].y;
}

// Dispersion table before the NLPR of step s (0-based).
__device__ __forceinline__ const float2* step_gvd(const Tables& tb, int s) {
  return s == 0 ? tb.h_first : tb.h_mid + (size_t)(s - 1) * tb.h_stride;
}

// Dual-polarisation NLPR (eqs. (20)-(21)): d = |x|^2 - |y|^2, the input of
// the extra cross-band filter.
template <int N>
__device__ __forceinline__ void intensity_diff(const float2 (&x)[FftShape<N>::RR],
                                               const float2 (&y)[FftShape<N>::RR], float (&d)[FftShape<N>::RR]) {
#pragma unroll
  for (int o = 0; o < FftShape<N>::RR; ++o)
    d[o] = (x[o].x * x[o].x + x[o].y * x[o].y) - (y[o].x * y[o].x + y[o].y * y[o].y);
}

// x *= exp(-j (theta + phi)), y *= exp(-j (theta - phi)).
template <int N>
__device__ __forceinline__ void rotate_dual(float2 (&x)[FftShape<N>::RR], float2 (&y)[FftShape<N>::RR],
                                            const float (&theta)[FftShape<N>::RR],
                                            const float (&phi)[FftShape<N>::RR]) {
  constexpr int RR = FftShape<N>::RR;
#pragma unroll
  for (int o = 0; o < RR; ++o) {
    float sn, cs;
    phase_sincos(theta[o] + phi[o], sn, cs);
    x[o] = cmul(x[o], make_float2(cs, -sn));
    phase_sincos(theta[o] - phi[o], sn, cs);
    y[o] = cmul(y[o], make_float2(cs, -sn));
  }
}

}  // namespace cbessfm
