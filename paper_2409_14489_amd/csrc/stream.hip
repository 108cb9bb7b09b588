// Streaming CB-ESSFM forward for overlap-and-save blocks larger than one CU
// holds (N' = 2^14 .. 2^17 per subband), as long links need: the overlap must
// cover the group-delay spread of the whole backpropagated link (Sec. III-A),
// which reaches 1.8e5 full-field samples for 40 x 80 km at 640 GS/s.
//
// The block state lives in device memory, one array of N' complex samples
// per subband (or polyphase component) and polarisation, and each stage of a
// step is a kernel over all blocks of a wave:
//
//   size-N' DFT = N1 x N2 (N1 = 4096, N2 = N' / 4096), four-step form:
//     column pass: N1 DFTs of size N2 over samples n1 + N1 n2, one per
//                  thread in registers, times exp(-+j 2 pi n1 k2 / N');
//     row pass:    N2 DFTs of size N1 over contiguous rows, one per
//                  workgroup (the register-resident FFT of fft_lds.hpp).
//   A forward transform of time samples in natural order leaves bin
//   k2 + N2 k1 at position k1 + N1 k2; the inverse takes that order back to
//   natural time order.  Spectra are only ever multiplied pointwise (the
//   dispersion filters, the DEMUX twiddles), so the plan keeps those tables
//   in the same permuted order and no transposition is ever done.
//
//   per step (Fig. "scheme_CB-ESSFM"): row kernel [forward row pass of the
//   previous step's FFT, dispersion filter, inverse row pass]; intensity
//   kernel [inverse column pass, |x|^2 + |y|^2]; filter kernel [coupled FIR of
//   eq. (15), circular over N']; rotation kernel [inverse column pass again,
//   exp(-j theta) of eq. (3), forward column pass].
//
// Every kernel reads and writes whole coalesced rows or columns-across-lanes;
// nothing here is resident across steps, so the path is bound by HBM (and the
// 256 MB last-level cache) rather than by the persistent kernel's LDS.
#include <hip/hip_runtime.h>

#include "fft_lds.hpp"
#include "internal.hpp"
#include "sincos.hpp"
#include "team.hpp"

namespace cbessfm {

namespace {

constexpr int kRow = kStreamRow;                  // N1
constexpr int kRowNT = FftShape<kRow>::NT;        // 512 threads per row workgroup
constexpr int kRowRR = FftShape<kRow>::RR;        // 8 samples per thread
constexpr int kColThreads = 256;

// cos(2 pi k / 32) as an FP32 leading part and an FP32 remainder (the
// products add the remainder by FMA, as the radix-16 constants do).
__host__ __device__ constexpr float cos32(int k) {
  constexpr float c[32] = {
      1.0f, 0.9807852506637573f, 0.9238795042037964f, 0.8314695954322815f, 0.7071067690849304f,
      0.5555702447891235f, 0.3826834261417389f, 0.19509032368659973f, 0.0f, -0.19509032368659973f,
      -0.3826834261417389f, -0.5555702447891235f, -0.7071067690849304f, -0.8314695954322815f,
      -0.9238795042037964f, -0.9807852506637573f, -1.0f, -0.9807852506637573f, -0.9238795042037964f,
      -0.8314695954322815f, -0.7071067690849304f, -0.5555702447891235f, -0.3826834261417389f,
      -0.19509032368659973f, 0.0f, 0.19509032368659973f, 0.3826834261417389f, 0.5555702447891235f,
      0.7071067690849304f, 0.8314695954322815f, 0.9238795042037964f, 0.9807852506637573f};
  return c[k & 31];
}
__host__ __device__ constexpr float cos32_lo(int k) {
  constexpr float c[32] = {
      0.0f, 2.9739473106360492e-08f, 2.830748968563057e-08f, 1.687026340846387e-08f, 1.2101617485882343e-08f,
      -1.1769521357507529e-08f, 6.2233507236442165e-09f, -1.670471427850373e-09f, 0.0f,
      1.670471427850373e-09f, -6.2233507236442165e-09f, 1.1769521357507529e-08f, -1.2101617485882343e-08f,
      -1.687026340846387e-08f, -2.830748968563057e-08f, -2.9739473106360492e-08f, 0.0f,
      -2.9739473106360492e-08f, -2.830748968563057e-08f, -1.687026340846387e-08f, -1.2101617485882343e-08f,
      1.1769521357507529e-08f, -6.2233507236442165e-09f, 1.670471427850373e-09f, 0.0f,
      -1.670471427850373e-09f, 6.2233507236442165e-09f, -1.1769521357507529e-08f, 1.2101617485882343e-08f,
      1.687026340846387e-08f, 2.830748968563057e-08f, 2.9739473106360492e-08f};
  return c[k & 31];
}

// a * exp(-+ j 2 pi K / 32)
template <int K, bool INV>
__device__ __forceinline__ float2 w32(float2 a) {
  if constexpr ((K & 1) == 0) {
    return w16<K / 2, INV>(a);
  } else {
    constexpr float c = cos32(K), s = cos32(K + 24), cl = cos32_lo(K), sl = cos32_lo(K + 24);
    const float ss = INV ? -s : s, ssl = INV ? -sl : sl;
    const float re_lo = fmaf(a.x, cl, a.y * ssl);
    const float im_lo = fmaf(a.y, cl, -a.x * ssl);
    return make_float2(fmaf(a.x, c, fmaf(a.y, ss, re_lo)), fmaf(a.y, c, fmaf(-a.x, ss, im_lo)));
  }
}

template <int K, bool INV>
__device__ __forceinline__ void w32_all(float2 (&b)[16]) {
  if constexpr (K < 16) {
    b[K] = w32<K, INV>(b[K]);
    w32_all<K + 1, INV>(b);
  }
}

// 32-point DFT, natural order in and out: two 16-point DFTs of the even and
// odd samples, a twiddle, and 16 butterflies.
template <bool INV>
__device__ __forceinline__ void dft32(float2 (&v)[32]) {
  float2 e[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft16<INV>(e);
  dft16<INV>(o);
  w32_all<0, INV>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 16] = csub(e[k], o[k]);
  }
}

template <int R, bool INV>
__device__ __forceinline__ void col_dft(float2 (&v)[R]) {
  if constexpr (R == 32)
    dft32<INV>(v);
  else
    dft<R, INV>(v);
}

// Column n1 of one array: v[k2] = a[n1 + N1 k2].
template <int N2>
__device__ __forceinline__ void load_col(const float2* __restrict__ a, int n1, float2 (&v)[N2]) {
#pragma unroll
  for (int k = 0; k < N2; ++k) v[k] = a[n1 + kRow * k];
}
template <int N2>
__device__ __forceinline__ void store_col(float2* __restrict__ a, int n1, const float2 (&v)[N2]) {
#pragma unroll
  for (int k = 0; k < N2; ++k) a[n1 + kRow * k] = v[k];
}

// Inverse column pass of column n1: undo the twiddle, size-N2 inverse DFT.
template <int N2>
__device__ __forceinline__ void col_inverse(const float2* __restrict__ tw2, int n1, float2 (&v)[N2]) {
#pragma unroll
  for (int k = 1; k < N2; ++k) v[k] = cmulc(v[k], tw2[kRow * k + n1]);
  col_dft<N2, true>(v);
}
// Forward column pass: size-N2 DFT, then the twiddle exp(-j 2 pi n1 k2 / N').
template <int N2>
__device__ __forceinline__ void col_forward(const float2* __restrict__ tw2, int n1, float2 (&v)[N2]) {
  col_dft<N2, false>(v);
#pragma unroll
  for (int k = 1; k < N2; ++k) v[k] = cmul(v[k], tw2[kRow * k + n1]);
}

}  // namespace

// ------------------------------------------------------------------ kernels
// Block input: framing (Sec. III-A), (-1)^n (so that bin k of the size-N DFT
// is frequency k - N/2), polyphase split n = n_sb m + a, forward column pass
// of every polyphase component.  Thread g: a = g mod n_sb, n1 = g / n_sb, so
// neighbouring threads read neighbouring input samples.
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_head_kernel(StreamArgs a) {
  constexpr int NP = kRow * N2;
  const int g = blockIdx.x * kColThreads + threadIdx.x;
  if (g >= a.n_sb * kRow) return;
  const int w = blockIdx.y;
  const int item = a.item0 + w;
  const int inst = item / a.nblk, blk = item - inst * a.nblk;
  const int nsb = a.n_sb, ap = g % nsb, n1 = g / nsb;
  const int T = a.T;
  const float2* sx = a.in + (size_t)inst * 2 * T;
  const int first = frame_first(blk, a.hop, a.n_ov, T, a.boundary);
  const bool short_seq = T < nsb * NP;
  float2* base = a.st + ((size_t)w * nsb + ap) * 2 * NP;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const int n = ap + nsb * (n1 + kRow * k);
      const int pos = frame_pos(first, n, T, a.boundary, short_seq);
      float2 u = make_float2(0.f, 0.f);
      if (pos >= 0) u = sx[(size_t)pol * T + pos];
      v[k] = cscale(u, (n & 1) ? -1.0f : 1.0f);
    }
    col_forward<N2>(a.tw2, n1, v);
    store_col<N2>(base + (size_t)pol * NP, n1, v);
  }
}

// Row pass of row k2 of array (block w, subband i): optional forward size-N1
// DFT, optional pointwise filter h (permuted order, subband i at i N'),
// optional inverse size-N1 DFT.  blockIdx.x = i N2 + k2.
template <bool FWD, bool GVD, bool INV>
__global__ __launch_bounds__(kRowNT, 4) void st_row_kernel(float2* __restrict__ st, const float2* __restrict__ h,
                                                        const float2* __restrict__ twr, int nsb, int n2,
                                                        int np) {
  __shared__ __align__(16) float4 lxy[FftShape<kRow>::LDS_C];
  const int i = blockIdx.x / n2, k2 = blockIdx.x - (blockIdx.x / n2) * n2;
  const int w = blockIdx.y;
  float2* bx = st + ((size_t)w * nsb + i) * 2 * np + (size_t)k2 * kRow;
  float2* by = bx + np;
  const int t = threadIdx.x;
  float2 x[kRowRR], y[kRowRR];
#pragma unroll
  for (int o = 0; o < kRowRR; ++o) {
    x[o] = bx[t + kRowNT * o];
    y[o] = by[t + kRowNT * o];
  }
  if constexpr (FWD) fft<kRow, false>(x, y, lxy, twr, t);
  if constexpr (GVD) {
    const float2* hr = h + (size_t)i * np + (size_t)k2 * kRow;
#pragma unroll
    for (int o = 0; o < kRowRR; ++o) {
      const float2 hv = hr[t + kRowNT * o];
      x[o] = cmul(x[o], hv);
      y[o] = cmul(y[o], hv);
    }
  }
  if constexpr (INV) fft<kRow, true>(x, y, lxy, twr, t);
#pragma unroll
  for (int o = 0; o < kRowRR; ++o) {
    bx[t + kRowNT * o] = x[o];
    by[t + kRowNT * o] = y[o];
  }
}

// DEMUX (INV = false): polyphase spectra P_a -> subband spectra
//   V_c = sum_a wsb[a c] poly[a] P_a;
// MUX (INV = true): P_a = conj(poly[a]) sum_c conj(wsb[a c]) V_c.
// Pointwise over the (permuted) bin position, in place.
template <bool INV>
__global__ __launch_bounds__(256) void st_mix_kernel(float2* __restrict__ st, const float2* __restrict__ poly,
                                                     StreamWsb wsb, int nsb, int np) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= np) return;
  float2* base = st + (size_t)blockIdx.y * nsb * 2 * np + q;
  float2 vx[kMaxSubbands], vy[kMaxSubbands];
#pragma unroll
  for (int a = 0; a < kMaxSubbands; ++a) {
    if (a < nsb) {
      vx[a] = base[(size_t)(2 * a) * np];
      vy[a] = base[(size_t)(2 * a + 1) * np];
      if (!INV) {
        const float2 pw = poly[(size_t)a * np + q];
        vx[a] = cmul(vx[a], pw);
        vy[a] = cmul(vy[a], pw);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kMaxSubbands; ++c) {
    if (c < nsb) {
      float2 sx = make_float2(0.f, 0.f), sy = sx;
#pragma unroll
      for (int a = 0; a < kMaxSubbands; ++a) {
        if (a < nsb) {
          const float2 wv = wsb.w[(a * c) % nsb];
          sx = cadd(sx, INV ? cmulc(vx[a], wv) : cmul(vx[a], wv));
          sy = cadd(sy, INV ? cmulc(vy[a], wv) : cmul(vy[a], wv));
        }
      }
      if (INV) {
        const float2 pw = poly[(size_t)c * np + q];
        sx = cmulc(sx, pw);
        sy = cmulc(sy, pw);
      }
      base[(size_t)(2 * c) * np] = sx;
      base[(size_t)(2 * c + 1) * np] = sy;
    }
  }
}

// Intensity p_i[n] = |x_i[n]|^2 + |y_i[n]|^2 of subband i (Sec. II-C): inverse
// column pass of column n1, time samples n = n1 + N1 n2 in natural order.
// blockIdx.x = i (N1 / 256) + column group.
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_intensity_kernel(const float2* __restrict__ st,
                                                                   float* __restrict__ pb,
                                                                   const float2* __restrict__ tw2, int nsb) {
  constexpr int NP = kRow * N2;
  constexpr int GROUPS = kRow / kColThreads;
  const int i = blockIdx.x / GROUPS;
  const int n1 = (blockIdx.x - i * GROUPS) * kColThreads + threadIdx.x;
  const size_t arr = (size_t)blockIdx.y * nsb + i;
  float p[N2];
#pragma unroll
  for (int k = 0; k < N2; ++k) p[k] = 0.0f;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
    load_col<N2>(st + (arr * 2 + pol) * NP, n1, v);
    col_inverse<N2>(tw2, n1, v);
#pragma unroll
    for (int k = 0; k < N2; ++k) p[k] = fmaf(v[k].x, v[k].x, fmaf(v[k].y, v[k].y, p[k]));
  }
  float* dst = pb + arr * NP + n1;
#pragma unroll
  for (int k = 0; k < N2; ++k) dst[kRow * k] = p[k];
}

// Coupled filter of eq. (15), circular over N':
//   theta_i[n] = sum_l sum_tau C_s[i][l][tau] p_l[(n - tau + nc) mod N'].
// A workgroup filters kFirOut consecutive n of one block for every subband i;
// each thread takes kFirQ consecutive outputs.  The rows p_l, extended
// circularly by tap_pad - 1 - nc on the left and nc on the right, are staged
// in LDS once.  Taps go in chunks of 8 over the zero-padded coefficient rows
// (uniform across the workgroup, so they are scalar loads of 8 words); for
// each chunk a thread reads a window of kFirQ + 7 intensities and does
// 8 kFirQ multiply-adds per output subband.
constexpr int kFirQ = 4;
constexpr int kFirOut = 256 * kFirQ;

__global__ __launch_bounds__(256) void st_fir_kernel(const float* __restrict__ pb, float* __restrict__ th,
                                                     const float* __restrict__ cs, int nsb, int np, int nc,
                                                     int tap_pad) {
  constexpr int W = kFirOut + 256;  // >= kFirOut + tap_pad - 1, tap_pad <= 256
  __shared__ float tile[kMaxSubbands][W];
  const int n0 = blockIdx.x * kFirOut;
  const size_t arr0 = (size_t)blockIdx.y * nsb;
  const int hl = tap_pad - 1 - nc;
  const int span = kFirOut + tap_pad - 1;
  for (int l = 0; l < nsb; ++l) {
    const float* row = pb + (arr0 + l) * np;
    for (int j = threadIdx.x; j < span; j += 256) {
      int q = n0 - hl + j;
      q = q < 0 ? q + np : (q >= np ? q - np : q);
      tile[l][j] = row[q];
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  float acc[kMaxSubbands][kFirQ];
#pragma unroll
  for (int i = 0; i < kMaxSubbands; ++i)
#pragma unroll
    for (int q = 0; q < kFirQ; ++q) acc[i][q] = 0.0f;
  const int n_chunks = tap_pad / kTapChunk;
  for (int l = 0; l < nsb; ++l) {
    const float* tl = tile[l] + t * kFirQ + tap_pad - 1 - (kTapChunk - 1);
    for (int ch = 0; ch < n_chunks; ++ch) {
      // taps tau = 8 ch + u use win[q + 7 - u] for output q
      float win[kFirQ + kTapChunk - 1];
#pragma unroll
      for (int m = 0; m < kFirQ + kTapChunk - 1; ++m) win[m] = tl[m - kTapChunk * ch];
#pragma unroll
      for (int i = 0; i < kMaxSubbands; ++i) {
        if (i < nsb) {
          const float* ci = cs + ((size_t)i * nsb + l) * tap_pad + kTapChunk * ch;
#pragma unroll
          for (int u = 0; u < kTapChunk; ++u) {
            const float cv = ci[u];
#pragma unroll
            for (int q = 0; q < kFirQ; ++q) acc[i][q] = fmaf(cv, win[q + kTapChunk - 1 - u], acc[i][q]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kMaxSubbands; ++i)
    if (i < nsb)
      *reinterpret_cast<float4*>(th + (arr0 + i) * np + n0 + t * kFirQ) =
          make_float4(acc[i][0], acc[i][1], acc[i][2], acc[i][3]);
}

// Rotation of eq. (3): inverse column pass, x, y *= exp(-j theta_i[n]),
// forward column pass, in place.
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_rotate_kernel(float2* __restrict__ st,
                                                                const float* __restrict__ th,
                                                                const float2* __restrict__ tw2, int nsb) {
  constexpr int NP = kRow * N2;
  constexpr int GROUPS = kRow / kColThreads;
  const int i = blockIdx.x / GROUPS;
  const int n1 = (blockIdx.x - i * GROUPS) * kColThreads + threadIdx.x;
  const size_t arr = (size_t)blockIdx.y * nsb + i;
  float theta[N2];
  const float* src = th + arr * NP + n1;
#pragma unroll
  for (int k = 0; k < N2; ++k) theta[k] = src[kRow * k];
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2* a = st + (arr * 2 + pol) * NP;
    float2 v[N2];
    load_col<N2>(a, n1, v);
    col_inverse<N2>(tw2, n1, v);
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      float sn, cs;
      phase_sincos(theta[k], sn, cs);
      v[k] = cmul(v[k], make_float2(cs, -sn));
    }
    col_forward<N2>(tw2, n1, v);
    store_col<N2>(a, n1, v);
  }
}

// Block output: inverse column pass of polyphase component a, (-1)^n, kept
// samples [n_ov/2, N - n_ov/2) that fall inside [0, T).
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_tail_kernel(StreamArgs a) {
  constexpr int NP = kRow * N2;
  const int g = blockIdx.x * kColThreads + threadIdx.x;
  if (g >= a.n_sb * kRow) return;
  const int w = blockIdx.y;
  const int item = a.item0 + w;
  const int inst = item / a.nblk, blk = item - inst * a.nblk;
  const int nsb = a.n_sb, ap = g % nsb, n1 = g / nsb;
  const int T = a.T;
  const int keep_lo = a.n_ov / 2, keep_hi = nsb * NP - a.n_ov / 2;
  float2* dx = a.out + (size_t)inst * 2 * T;
  const float2* base = a.st + ((size_t)w * nsb + ap) * 2 * NP;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
    load_col<N2>(base + (size_t)pol * NP, n1, v);
    col_inverse<N2>(a.tw2, n1, v);
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const int n = ap + nsb * (n1 + kRow * k);
      const int pos = blk * a.hop + n - keep_lo;
      if (n >= keep_lo && n < keep_hi && pos < T) dx[(size_t)pol * T + pos] = cscale(v[k], (n & 1) ? -1.0f : 1.0f);
    }
  }
}

// ------------------------------------------------------------------ launcher
namespace {

bool ok_launch() { return hipGetLastError() == hipSuccess; }

template <bool FWD, bool GVD, bool INV>
bool row(const StreamArgs& a, const float2* h, hipStream_t s) {
  st_row_kernel<FWD, GVD, INV><<<dim3(a.n_sb * a.n2, a.nb), kRowNT, 0, s>>>(a.st, h, a.twr, a.n_sb, a.n2, a.np);
  return ok_launch();
}

template <int N2>
int run_wave(const StreamArgs& a, const Tables& tb, const float* cpad, int steps, int n_taps, int tap_pad,
             hipStream_t s) {
  const int nsb = a.n_sb;
  const dim3 col_grid((nsb * kRow + kColThreads - 1) / kColThreads, a.nb);
  const dim3 sb_grid(nsb * (kRow / kColThreads), a.nb);
  const dim3 mix_grid(a.np / 256, a.nb);
  StreamWsb wsb;
  for (int k = 0; k < kMaxSubbands; ++k) wsb.w[k] = tb.wsb[k];
  const int nc = n_taps / 2;
  bool ok = true;
  st_head_kernel<N2><<<col_grid, kColThreads, 0, s>>>(a);
  ok = ok && ok_launch();
  if (nsb > 1) {
    ok = ok && row<true, false, false>(a, nullptr, s);
    st_mix_kernel<false><<<mix_grid, 256, 0, s>>>(a.st, tb.poly_tw, wsb, nsb, a.np);
    ok = ok && ok_launch();
  }
  for (int st = 0; st < steps && ok; ++st) {
    const float2* h = st == 0 ? tb.h_first : tb.h_mid + (size_t)(st - 1) * tb.h_stride;
    if (st == 0 && nsb > 1)
      ok = ok && row<false, true, true>(a, h, s);
    else
      ok = ok && row<true, true, true>(a, h, s);
    st_intensity_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(a.st, a.pb, a.tw2, nsb);
    ok = ok && ok_launch();
    st_fir_kernel<<<dim3(a.np / kFirOut, a.nb), 256, 0, s>>>(a.pb, a.th, cpad + (size_t)st * nsb * nsb * tap_pad,
                                                             nsb, a.np, nc, tap_pad);
    ok = ok && ok_launch();
    st_rotate_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(a.st, a.th, a.tw2, nsb);
    ok = ok && ok_launch();
  }
  if (nsb > 1) {
    ok = ok && row<true, true, false>(a, tb.h_last, s);
    st_mix_kernel<true><<<mix_grid, 256, 0, s>>>(a.st, tb.poly_tw, wsb, nsb, a.np);
    ok = ok && ok_launch();
    ok = ok && row<false, false, true>(a, nullptr, s);
  } else {
    ok = ok && row<true, true, true>(a, tb.h_last, s);
  }
  st_tail_kernel<N2><<<col_grid, kColThreads, 0, s>>>(a);
  ok = ok && ok_launch();
  return ok ? CBESSFM_OK : CBESSFM_EHIP;
}

}  // namespace

int launch_stream_forward(cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, hipStream_t s) {
  if (p->nlpr != CBESSFM_NLPR_AVERAGED) return CBESSFM_EUNSUPPORTED;
  Tables tb;
  fill_tables(p, tb);
  StreamArgs a;
  a.in = static_cast<const float2*>(in);
  a.out = static_cast<float2*>(out);
  a.T = (int)T;
  a.nblk = (int)((T + p->hop - 1) / p->hop);
  a.n_sb = p->sb.n_sb;
  a.np = p->Np;
  a.n2 = p->Np / kRow;
  a.n_ov = p->sb.overlap;
  a.hop = p->hop;
  a.boundary = p->sb.boundary;
  a.st = p->d_st;
  a.pb = p->d_pb;
  a.th = p->d_th;
  a.tw2 = p->d_tw;
  a.twr = p->d_tw + p->Np;
  const int items = batch * a.nblk;
  for (int item0 = 0; item0 < items; item0 += p->st_blocks) {
    a.item0 = item0;
    a.nb = items - item0 < p->st_blocks ? items - item0 : p->st_blocks;
    int rc;
    switch (p->log_np) {
      case 14: rc = run_wave<4>(a, tb, p->d_cpad, p->steps, p->n_taps, p->tap_pad, s); break;
      case 15: rc = run_wave<8>(a, tb, p->d_cpad, p->steps, p->n_taps, p->tap_pad, s); break;
      case 16: rc = run_wave<16>(a, tb, p->d_cpad, p->steps, p->n_taps, p->tap_pad, s); break;
      case 17: rc = run_wave<32>(a, tb, p->d_cpad, p->steps, p->n_taps, p->tap_pad, s); break;
      default: rc = CBESSFM_EUNSUPPORTED;
    }
    if (rc) return rc;
  }
  return CBESSFM_OK;
}

}  // namespace cbessfm
