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
//
// The second half of the file is the reverse-mode derivative of the same
// chain (dL/dC, dL/drho, dL/d(segment lengths), dL/dfield_in): a forward
// sweep that keeps the block state at every checkpoint segment start, then
// per segment (recomputed from its start) the adjoint stages in reverse
// order, built from the same column/row passes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fft_lds.hpp"
#include "internal.hpp"
#include "sincos.hpp"
#include "team.hpp"

namespace cbessfm {

namespace {

constexpr int kRow = kStreamRow;  // N1
// Row transforms hold 16 samples per thread (three radix-16 passes, two LDS
// exchanges) and use one LDS exchange buffer: two workgroups of 74 KB share a
// CU, where two buffers each would leave room for one.
constexpr int kRowRR = 16;
using RowShape = FftShape<kRow, kRowRR>;
constexpr int kRowNT = RowShape::NT;  // 256 threads per row workgroup
constexpr bool kRowDB = false;
constexpr int kRowLds = kRowDB ? RowShape::LDS_ENTRIES : RowShape::LDS_C;
// The dispersion-derivative kernel holds two row states at once and keeps 8
// samples per thread (512 threads), which fits its registers.
constexpr int kGvdRR = 8;
constexpr int kGvdNT = FftShape<kRow, kGvdRR>::NT;
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

// Column twiddle exp(-j 2 pi n1 k / N') for k < N2: read directly for
// k < 8 and k multiple of 8, else as the product of the k mod 8 and the
// 8 floor(k / 8) entries (10 reads instead of 31 at N2 = 32).
template <int N2>
__device__ __forceinline__ void col_twiddles(const float2* __restrict__ tw2, int n1, float2 (&a)[8],
                                             float2 (&b)[(N2 + 7) / 8]) {
#pragma unroll
  for (int j = 1; j < 8 && j < N2; ++j) a[j] = tw2[kRow * j + n1];
#pragma unroll
  for (int m = 1; m < (N2 + 7) / 8; ++m) b[m] = tw2[kRow * 8 * m + n1];
}
template <int N2>
__device__ __forceinline__ float2 col_tw(const float2 (&a)[8], const float2 (&b)[(N2 + 7) / 8], int k) {
  const int j = k & 7, m = k >> 3;
  if (m == 0) return a[j];
  if (j == 0) return b[m];
  return cmul(a[j], b[m]);
}
// Inverse column pass of column n1: undo the twiddle, size-N2 inverse DFT.
template <int N2>
__device__ __forceinline__ void col_inverse(const float2* __restrict__ tw2, int n1, float2 (&v)[N2]) {
  float2 a[8], b[(N2 + 7) / 8];
  col_twiddles<N2>(tw2, n1, a, b);
#pragma unroll
  for (int k = 1; k < N2; ++k) v[k] = cmulc(v[k], col_tw<N2>(a, b, k));
  col_dft<N2, true>(v);
}
// Forward column pass: size-N2 DFT, then the twiddle exp(-j 2 pi n1 k2 / N').
template <int N2>
__device__ __forceinline__ void col_forward(const float2* __restrict__ tw2, int n1, float2 (&v)[N2]) {
  col_dft<N2, false>(v);
  float2 a[8], b[(N2 + 7) / 8];
  col_twiddles<N2>(tw2, n1, a, b);
#pragma unroll
  for (int k = 1; k < N2; ++k) v[k] = cmul(v[k], col_tw<N2>(a, b, k));
}

}  // namespace

// ------------------------------------------------------------------ kernels
// Block input: framing (Sec. III-A), (-1)^n (so that bin k of the size-N DFT
// is frequency k - N/2), polyphase split n = n_sb m + a, forward column pass
// of every polyphase component.  Thread g: a = g mod n_sb, n1 = g / n_sb, so
// neighbouring threads read neighbouring input samples.
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_head_kernel(StreamArgs a, const StreamBlk* __restrict__ tab) {
  constexpr int NP = kRow * N2;
  const int g = blockIdx.x * kColThreads + threadIdx.x;
  if (g >= a.n_sb * kRow) return;
  const int nsb = a.n_sb, ap = g % nsb, n1 = g / nsb;
  const float2* sx;
  float2* base;
  const float2* tw2 = a.tw2;
  int T, first, boundary;
  if (tab != nullptr) {  // blockIdx.y = entry of the block table
    const StreamBlk& e = tab[blockIdx.y];
    T = e.T;
    boundary = e.boundary;
    sx = e.in;
    first = frame_first(e.blk, e.hop, e.n_ov, T, boundary);
    base = e.st + (size_t)ap * 2 * NP;
    tw2 = e.tw2;
  } else {
    const int w = blockIdx.y;
    const int item = a.item0 + w;
    const int inst = item / a.nblk, blk = item - inst * a.nblk;
    T = a.T;
    boundary = a.boundary;
    sx = a.in + (size_t)inst * 2 * T;
    first = frame_first(blk, a.hop, a.n_ov, T, boundary);
    base = a.st + ((size_t)w * nsb + ap) * 2 * NP;
  }
  const bool short_seq = T < nsb * NP;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const int n = ap + nsb * (n1 + kRow * k);
      const int pos = frame_pos(first, n, T, boundary, short_seq);
      float2 u = make_float2(0.f, 0.f);
      if (pos >= 0) u = sx[(size_t)pol * T + pos];
      v[k] = cscale(u, (n & 1) ? -1.0f : 1.0f);
    }
    col_forward<N2>(tw2, n1, v);
    store_col<N2>(base + (size_t)pol * NP, n1, v);
  }
}

// Row pass of row k2 of array (block w, subband i): optional forward size-N1
// DFT, optional pointwise filter h (permuted order, subband i at i N'; conj(h)
// when CONJ, the adjoint's filter), optional inverse size-N1 DFT.  Reads src,
// writes dst (the same array for an in-place pass).  blockIdx.x = i N2 + k2,
// blockIdx.y = block of the wave, or, with a block table `blk`, the entry of
// that table (in place on its state, with the filter of step `step`, or of
// the last segment for step < 0).
template <bool FWD, bool GVD, bool INV, bool CONJ = false>
__global__ __launch_bounds__(kRowNT, 2) void st_row_kernel(const float2* src, float2* dst,
                                                        const float2* __restrict__ h,
                                                        const float2* __restrict__ twr, int nsb, int n2,
                                                        int np, const StreamBlk* __restrict__ blk, int step) {
  __shared__ __align__(16) float4 lxy[kRowLds];
  const int i = blockIdx.x / n2, k2 = blockIdx.x - (blockIdx.x / n2) * n2;
  size_t wb = blockIdx.y;
  if (blk != nullptr) {
    const StreamBlk& e = blk[blockIdx.y];
    src = e.st;
    dst = e.st;
    h = step < 0 ? e.h_last : step == 0 ? e.h_first : e.h_mid + (size_t)(step - 1) * e.h_stride;
    twr = e.twr;
    wb = 0;
  }
  const size_t off = (wb * nsb + i) * 2 * np + (size_t)k2 * kRow;
  const float2* bx = src + off;
  const float2* by = bx + np;
  const int t = threadIdx.x;
  float2 x[kRowRR], y[kRowRR];
#pragma unroll
  for (int o = 0; o < kRowRR; ++o) {
    x[o] = bx[t + kRowNT * o];
    y[o] = by[t + kRowNT * o];
  }
  if constexpr (FWD) fft<kRow, false, kRowDB, kRowRR>(x, y, lxy, twr, t);
  if constexpr (GVD) {
    const float2* hr = h + (size_t)i * np + (size_t)k2 * kRow;
#pragma unroll
    for (int o = 0; o < kRowRR; ++o) {
      const float2 hv = hr[t + kRowNT * o];
      x[o] = CONJ ? cmulc(x[o], hv) : cmul(x[o], hv);
      y[o] = CONJ ? cmulc(y[o], hv) : cmul(y[o], hv);
    }
  }
  if constexpr (INV) fft<kRow, true, kRowDB, kRowRR>(x, y, lxy, twr, t);
  float2* ox = dst + off;
  float2* oy = ox + np;
#pragma unroll
  for (int o = 0; o < kRowRR; ++o) {
    ox[t + kRowNT * o] = x[o];
    oy[t + kRowNT * o] = y[o];
  }
}

// DEMUX (INV = false): polyphase spectra P_a -> subband spectra
//   V_c = sum_a wsb[a c] poly[a] P_a;
// MUX (INV = true): P_a = conj(poly[a]) sum_c conj(wsb[a c]) V_c.
// Pointwise over the (permuted) bin position, in place.
template <bool INV>
__global__ __launch_bounds__(256) void st_mix_kernel(float2* __restrict__ st, const float2* __restrict__ poly,
                                                     StreamWsb wsb, int nsb, int np,
                                                     const StreamBlk* __restrict__ tab) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= np) return;
  size_t wb = blockIdx.y;
  if (tab != nullptr) {  // blockIdx.y = entry of the block table
    const StreamBlk& e = tab[blockIdx.y];
    st = e.st;
    poly = e.poly;
    wb = 0;
  }
  float2* base = st + wb * nsb * 2 * np + q;
  // every load before the first store (a load issued after a store waits for it)
  float2 vx[kMaxSubbands], vy[kMaxSubbands], pw[kMaxSubbands];
#pragma unroll
  for (int a = 0; a < kMaxSubbands; ++a) {
    if (a < nsb) {
      vx[a] = base[(size_t)(2 * a) * np];
      vy[a] = base[(size_t)(2 * a + 1) * np];
      pw[a] = poly[(size_t)a * np + q];
    }
  }
  if (!INV) {
#pragma unroll
    for (int a = 0; a < kMaxSubbands; ++a) {
      if (a < nsb) {
        vx[a] = cmul(vx[a], pw[a]);
        vy[a] = cmul(vy[a], pw[a]);
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
        sx = cmulc(sx, pw[c]);
        sy = cmulc(sy, pw[c]);
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
                                                                   const float2* __restrict__ tw2, int nsb,
                                                                   const StreamBlk* __restrict__ blk) {
  constexpr int NP = kRow * N2;
  constexpr int GROUPS = kRow / kColThreads;
  const int i = blockIdx.x / GROUPS;
  const int n1 = (blockIdx.x - i * GROUPS) * kColThreads + threadIdx.x;
  size_t arr = (size_t)blockIdx.y * nsb + i;
  if (blk != nullptr) {  // blockIdx.y = entry of the block table
    const StreamBlk& e = blk[blockIdx.y];
    st = e.st;
    pb = e.pb;
    tw2 = e.tw2;
    arr = i;
  }
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

typedef float fir_v4 __attribute__((ext_vector_type(4)));

// Coupled filter of eq. (15), circular over N':
//   theta_i[n] = sum_l sum_tau C_s[i][l][tau] p_l[(n - tau + nc) mod N'].
// A workgroup filters kFirOut consecutive n of one block for every subband i;
// each thread takes kFirQ consecutive outputs.  The rows p_l, extended
// circularly by tap_pad - 1 - nc on the left and nc on the right, are staged
// in LDS once.  Taps go in chunks of 8 over the zero-padded coefficient rows
// (uniform across the workgroup, so they are scalar loads of 8 words); for
// each chunk a thread reads a window of kFirQ + 7 intensities and does
// 8 kFirQ multiply-adds per output subband.  The LDS rows (dynamic, n_sb of
// them, fir_lds_bytes) are only as many as the plan has subbands, so more
// workgroups fit a CU at small n_sb.
constexpr int kFirQ = 4;
constexpr int kFirOut = 256 * kFirQ;

// LDS row width in float4: the window of kFirOut + tap_pad - 1 samples from
// the float4 group that holds its first sample (shift < 4)
__host__ __device__ inline int fir_row_w4(int tap_pad) { return (kFirOut + tap_pad + 6) / 4; }
__host__ inline size_t fir_lds_bytes(int nsb, int tap_pad) { return 16 * (size_t)nsb * fir_row_w4(tap_pad); }

// NCH: the number of 8-tap chunks when known at compile time (1 .. 4, up to
// 32 taps), else 0.
template <int NSB, int NCH>
__global__ __launch_bounds__(256) void st_fir_kernel(const float* __restrict__ pb, float* __restrict__ th,
                                                     const float* __restrict__ cs, int np, int nc, int tap_pad,
                                                     const StreamBlk* __restrict__ blk, int step) {
  constexpr int nsb = NSB;
  extern __shared__ __align__(16) float fir_lds[];
  const int w4 = fir_row_w4(tap_pad), W = 4 * w4;
  const int n0 = blockIdx.x * kFirOut;
  size_t arr0 = (size_t)blockIdx.y * nsb;
  if (blk != nullptr) {  // blockIdx.y = entry of the block table; coefficients of step `step`
    const StreamBlk& e = blk[blockIdx.y];
    pb = e.pb;
    th = e.th;
    cs = e.cpad + (size_t)step * nsb * nsb * tap_pad;
    arr0 = 0;
  }
  const int hl = tap_pad - 1 - nc;
  const int t = threadIdx.x;
  // row l: fir_lds[l][j] = p_l[(4 g0 + j) mod N'], sample n0 - hl at j = sh;
  // aligned float4 loads with clamped indices, all issued before the stores
  const int sh = ((n0 - hl) % 4 + 4) % 4;
  const int g0 = (n0 - hl - sh) / 4, np4 = np / 4;
  {
    constexpr int CNT = (NSB * ((kFirOut + kMaxTaps + 1 + 6) / 4) + 255) / 256;
    const int nall = nsb * w4;
    fir_v4 v[CNT];
#pragma unroll
    for (int c = 0; c < CNT; ++c) {
      const int idx = t + 256 * c < nall ? t + 256 * c : nall - 1;
      const int l = idx / w4;
      int g = g0 + idx - l * w4;
      g = g < 0 ? g + np4 : (g >= np4 ? g - np4 : g);
      v[c] = reinterpret_cast<const fir_v4*>(pb + (arr0 + l) * np)[g];
    }
    fir_v4* lv = reinterpret_cast<fir_v4*>(fir_lds);
#pragma unroll
    for (int c = 0; c < CNT; ++c)
      if (t + 256 * c < nall) lv[t + 256 * c] = v[c];
  }
  __syncthreads();
  float acc[kMaxSubbands][kFirQ];
#pragma unroll
  for (int i = 0; i < kMaxSubbands; ++i)
#pragma unroll
    for (int q = 0; q < kFirQ; ++q) acc[i][q] = 0.0f;
  const int n_chunks = NCH > 0 ? NCH : tap_pad / kTapChunk;
  for (int l = 0; l < nsb; ++l) {
    const float* tl = fir_lds + l * W + sh + t * kFirQ + tap_pad - 1 - (kTapChunk - 1);
#pragma unroll
    for (int ch = 0; ch < (NCH > 0 ? NCH : n_chunks); ++ch) {
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

// The same filter on the matrix cores (FP32 MFMA, 16x16x4), for up to 32
// taps.  With R = 16 / NSB, the 16 rows of a tile are R consecutive outputs
// of each subband (row m = R i + r; rows from NSB R on are idle) and its 16
// columns step the output position by R, so a tile holds
// theta_i[nb + R q + r], q < 16.  Over the window index u = r + TAPS - 1 - tau,
//   theta_i[nb + R q + r] = sum_l sum_u A_l[R i + r][u] B_l[u][q],
//   A_l[R i + r][u] = C[i][l][r + TAPS - 1 - u]   (zero off the taps),
//   B_l[u][q]       = p_l[(nb + R q + u - hl) mod N'],
// a product over K = R + TAPS - 1 (rounded up to 4) per input row l.  A is
// the same for every tile of the step and stays in registers (NSB K / 4 per
// lane); B is read from the LDS rows.  FP32 MFMA does twice the
// multiply-adds per clock of the unpacked vector ALU that bounds the kernel
// above; the zero corners of the Toeplitz A cost (R + TAPS - 1) / TAPS of the
// direct form.  Operand layouts of v_mfma_f32_16x16x4f32 for lane j:
// A[j mod 16][j / 16], B[j / 16][j mod 16], D[4 (j / 16) + e][j mod 16], e < 4.
template <int NSB>
struct FirMfma {
  static constexpr int R = 16 / NSB;               // outputs per subband in a tile row group
  static constexpr int TILE = 16 * R;              // output positions per tile
  static constexpr int TW = (1024 + 4 * TILE - 1) / (4 * TILE);  // tiles per wave
  static constexpr int OUT = 4 * TW * TILE;        // output positions per workgroup (4 waves)
};
__host__ inline int fir_mfma_out(int nsb) { return 4 * ((1024 + 64 * (16 / nsb) - 1) / (64 * (16 / nsb))) * 16 * (16 / nsb); }
template <int NSB, int NCH>
struct FirMfmaShape {
  static constexpr int TAPS = kTapChunk * NCH;
  static constexpr int KP = (FirMfma<NSB>::R + TAPS - 1 + 3) & ~3;  // window per row, in k-steps of 4
  static constexpr int S = KP / 4;
  static constexpr int W4 = (FirMfma<NSB>::OUT + KP + 3 + 3) / 4;  // LDS row width in float4 (3 for the shift)
  static constexpr int CNT = (NSB * W4 + 255) / 256;               // float4 loads per thread
};
__host__ inline size_t fir_mfma_lds_bytes(int nsb, int tap_pad) {
  const int R = 16 / nsb, kp = (R + tap_pad - 1 + 3) & ~3;
  const int w4 = (fir_mfma_out(nsb) + kp + 6) / 4;
  return 16 * (size_t)256 * ((nsb * w4 + 255) / 256);
}

template <int NSB, int NCH>
__global__ __launch_bounds__(256) void st_fir_mfma_kernel(const float* __restrict__ pb, float* __restrict__ th,
                                                          const float* __restrict__ cs, int np, int nc,
                                                          const StreamBlk* __restrict__ blk, int step) {
  using F = FirMfma<NSB>;
  using G = FirMfmaShape<NSB, NCH>;
  constexpr int R = F::R, TAPS = G::TAPS, S = G::S, W4 = G::W4, OUT = F::OUT;
  extern __shared__ float4 fir_lds4[];
  float* fir_lds = reinterpret_cast<float*>(fir_lds4);
  const int n0 = blockIdx.x * OUT;
  size_t arr0 = (size_t)blockIdx.y * NSB;
  if (blk != nullptr) {  // blockIdx.y = entry of the block table; coefficients of step `step`
    const StreamBlk& e = blk[blockIdx.y];
    pb = e.pb;
    th = e.th;
    cs = e.cpad + (size_t)step * NSB * NSB * TAPS;
    arr0 = 0;
  }
  const int t = threadIdx.x;
  const int hl = TAPS - 1 - nc;
  // this lane's A entries: row m = lane mod 16, window index u = 4 s + lane / 16
  const int lane = t & 63, lq = lane & 15, kq = lane >> 4;  // lq: row of A, column of B and D
  const int ai = lq / R, ar = lq - (lq / R) * R;
  float a[NSB][S];
#pragma unroll
  for (int l = 0; l < NSB; ++l)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int tau = ar + TAPS - 1 - (4 * s + kq);
      const bool on = lq < NSB * R && tau >= 0 && tau < TAPS;
      // a clamped, always valid index, so that the loads carry no branch
      const int ic = ai < NSB ? ai : NSB - 1, tc = tau < 0 ? 0 : (tau < TAPS ? tau : TAPS - 1);
      const float cv = cs[((size_t)ic * NSB + l) * TAPS + tc];
      a[l][s] = on ? cv : 0.0f;
    }
  // LDS row l holds p_l[(4 g0 + j) mod N'], j < 4 W4, read as aligned float4
  // (N' is a multiple of 4), all loads in flight at once; sample n0 - hl of
  // the window is at j = sh.
  const int sh = ((n0 - hl) % 4 + 4) % 4;
  const int g0 = (n0 - hl - sh) / 4, np4 = np / 4;
  // (the slots past NSB W4 take more of the last row, so that every thread
  // has the same loads, all without a branch; g0 + W4 + 255 < 2 np4)
  {
    fir_v4 v[G::CNT];  // loaded first, stored after: the stores must not hold the loads back
#pragma unroll
    for (int c = 0; c < G::CNT; ++c) {
      const int idx = t + 256 * c;
      const int l = idx / W4 < NSB ? idx / W4 : NSB - 1;
      int g = g0 + idx - l * W4;
      g = g < 0 ? g + np4 : (g >= np4 ? g - np4 : g);
      v[c] = reinterpret_cast<const fir_v4*>(pb + (arr0 + l) * np)[g];
    }
    fir_v4* lv = reinterpret_cast<fir_v4*>(fir_lds4);
#pragma unroll
    for (int c = 0; c < G::CNT; ++c) lv[t + 256 * c] = v[c];
  }
  __syncthreads();
  const int wave = t >> 6;
  fir_v4 res[F::TW];
#pragma unroll
  for (int tw = 0; tw < F::TW; ++tw) {
    const int off = (wave * F::TW + tw) * F::TILE;
    fir_v4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;  // two chains, even and odd k-steps
#pragma unroll
    for (int l = 0; l < NSB; ++l) {
      const float* b = fir_lds + l * 4 * W4 + sh + off + R * lq + kq;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        if (s & 1)
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[l][s], b[4 * s], acc1, 0, 0, 0);
        else
          acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[l][s], b[4 * s], acc0, 0, 0, 0);
      }
    }
    res[tw] = acc0 + acc1;
  }
  __syncthreads();  // every wave is done with the rows; the outputs take their place
  float* out = fir_lds;  // [NSB][OUT]
#pragma unroll
  for (int tw = 0; tw < F::TW; ++tw) {
    const int off = (wave * F::TW + tw) * F::TILE;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int m = 4 * kq + e;
      if (m < NSB * R) {
        const int i = m / R, r = m - (m / R) * R;
        out[i * OUT + off + R * lq + r] = res[tw][e];
      }
    }
  }
  __syncthreads();
  constexpr int Q4 = OUT / 4;
  for (int idx = t; idx < NSB * Q4; idx += 256) {
    const int i = idx / Q4, c4 = idx - (idx / Q4) * Q4;
    const int n = n0 + 4 * c4;
    if (n < np)
      *reinterpret_cast<float4*>(th + (arr0 + i) * np + n) =
          *reinterpret_cast<const float4*>(out + i * OUT + 4 * c4);
  }
}

// Rotation of eq. (3): inverse column pass of src, x, y *= exp(-j theta_i[n]),
// forward column pass into dst (the same array for an in-place pass).
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_rotate_kernel(const float2* src, float2* dst,
                                                                const float* __restrict__ th,
                                                                const float2* __restrict__ tw2, int nsb,
                                                                const StreamBlk* __restrict__ blk) {
  constexpr int NP = kRow * N2;
  constexpr int GROUPS = kRow / kColThreads;
  const int i = blockIdx.x / GROUPS;
  const int n1 = (blockIdx.x - i * GROUPS) * kColThreads + threadIdx.x;
  size_t arr = (size_t)blockIdx.y * nsb + i;
  if (blk != nullptr) {  // blockIdx.y = entry of the block table, in place
    const StreamBlk& e = blk[blockIdx.y];
    src = e.st;
    dst = e.st;
    th = e.th;
    tw2 = e.tw2;
    arr = i;
  }
  float theta[N2];
  const float* tsrc = th + arr * NP + n1;
#pragma unroll
  for (int k = 0; k < N2; ++k) theta[k] = tsrc[kRow * k];
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
    load_col<N2>(src + (arr * 2 + pol) * NP, n1, v);
    col_inverse<N2>(tw2, n1, v);
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      float sn, cs;
      phase_sincos(theta[k], sn, cs);
      v[k] = cmul(v[k], make_float2(cs, -sn));
    }
    col_forward<N2>(tw2, n1, v);
    store_col<N2>(dst + (arr * 2 + pol) * NP, n1, v);
  }
}

// Block output: inverse column pass of polyphase component a, (-1)^n, kept
// samples [n_ov/2, N - n_ov/2) that fall inside [0, T).
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_tail_kernel(StreamArgs a, const StreamBlk* __restrict__ tab) {
  constexpr int NP = kRow * N2;
  const int g = blockIdx.x * kColThreads + threadIdx.x;
  if (g >= a.n_sb * kRow) return;
  const int nsb = a.n_sb, ap = g % nsb, n1 = g / nsb;
  int T, blk, hop, n_ov;
  float2* dx;
  const float2* base;
  const float2* tw2 = a.tw2;
  if (tab != nullptr) {  // blockIdx.y = entry of the block table
    const StreamBlk& e = tab[blockIdx.y];
    T = e.T;
    blk = e.blk;
    hop = e.hop;
    n_ov = e.n_ov;
    dx = e.out;
    base = e.st + (size_t)ap * 2 * NP;
    tw2 = e.tw2;
  } else {
    const int w = blockIdx.y;
    const int item = a.item0 + w;
    const int inst = item / a.nblk;
    blk = item - inst * a.nblk;
    T = a.T;
    hop = a.hop;
    n_ov = a.n_ov;
    dx = a.out + (size_t)inst * 2 * T;
    base = a.st + ((size_t)w * nsb + ap) * 2 * NP;
  }
  const int keep_lo = n_ov / 2, keep_hi = nsb * NP - n_ov / 2;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
    load_col<N2>(base + (size_t)pol * NP, n1, v);
    col_inverse<N2>(tw2, n1, v);
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const int n = ap + nsb * (n1 + kRow * k);
      const int pos = blk * hop + n - keep_lo;
      if (n >= keep_lo && n < keep_hi && pos < T) dx[(size_t)pol * T + pos] = cscale(v[k], (n & 1) ? -1.0f : 1.0f);
    }
  }
}

// ------------------------------------------------------------------ adjoint
// Reverse-mode derivative of the streaming forward (the same map as the
// persistent kernels differentiate).  Every linear stage is unitary up to a
// real scale or is an unnormalised DFT, so its adjoint is a stage the
// forward already has: the adjoint of a forward column pass is the inverse
// column pass and vice versa, the adjoint of a row pass [F1, h, G1] is
// [F1, conj(h), G1], the adjoint of the MUX is the DEMUX.  The adjoint state
// G (the cotangent dL/dRe + j dL/dIm of the forward state) lives in arrays of
// the same layout.

// Adjoint of st_tail_kernel: the cotangent of every kept output sample goes
// back to its block position ((-1)^n, polyphase split, forward column pass);
// samples the block does not keep get zero.
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_adj_tail_kernel(StreamArgs a, const float2* __restrict__ gout) {
  constexpr int NP = kRow * N2;
  const int g = blockIdx.x * kColThreads + threadIdx.x;
  if (g >= a.n_sb * kRow) return;
  const int w = blockIdx.y;
  const int item = a.item0 + w;
  const int inst = item / a.nblk, blk = item - inst * a.nblk;
  const int nsb = a.n_sb, ap = g % nsb, n1 = g / nsb;
  const int T = a.T;
  const int keep_lo = a.n_ov / 2, keep_hi = nsb * NP - a.n_ov / 2;
  const float2* src = gout + (size_t)inst * 2 * T;
  float2* base = a.st + ((size_t)w * nsb + ap) * 2 * NP;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const int n = ap + nsb * (n1 + kRow * k);
      const int pos = blk * a.hop + n - keep_lo;
      float2 u = make_float2(0.f, 0.f);
      if (n >= keep_lo && n < keep_hi && pos < T) u = src[(size_t)pol * T + pos];
      v[k] = cscale(u, (n & 1) ? -1.0f : 1.0f);
    }
    col_forward<N2>(a.tw2, n1, v);
    store_col<N2>(base + (size_t)pol * NP, n1, v);
  }
}

// Adjoint of st_head_kernel up to the framing: inverse column pass of the
// polyphase component, (-1)^n; writes the block's input cotangent
// gin_blk[item][pol][n] for every block sample n (summed over overlapping
// blocks afterwards).
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_adj_head_kernel(StreamArgs a, float2* __restrict__ gin_blk) {
  constexpr int NP = kRow * N2;
  const int g = blockIdx.x * kColThreads + threadIdx.x;
  if (g >= a.n_sb * kRow) return;
  const int w = blockIdx.y;
  const int item = a.item0 + w;
  const int nsb = a.n_sb, ap = g % nsb, n1 = g / nsb;
  const size_t N = (size_t)nsb * NP;
  float2* dst = gin_blk + (size_t)item * 2 * N;
  const float2* base = a.st + ((size_t)w * nsb + ap) * 2 * NP;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
    load_col<N2>(base + (size_t)pol * NP, n1, v);
    col_inverse<N2>(a.tw2, n1, v);
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      const int n = ap + nsb * (n1 + kRow * k);
      dst[(size_t)pol * N + n] = cscale(v[k], (n & 1) ? -1.0f : 1.0f);
    }
  }
}

// Phase cotangent of the rotation v' = v exp(-j theta) (eq. (3)):
//   theta_bar_i[n] = sum_pol Im(conj(g'[n]) v'[n]),
// with g' the inverse column pass of the adjoint state g (the adjoint of the
// forward column pass) and v' = inverse column pass of the stored forward
// state sf / N2 (the unnormalised pair multiplies by N2); also
// p_i[n] = sum_pol |v'[n]|^2 (the rotation keeps |v|).  v' is written to vt
// (time samples n = n1 + N1 k2 at position n1 + N1 k2, the state layout) and
// g' over g (same layout) for st_adj_comm_kernel; only one column of 32
// samples is live at a time.
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_adj_phase_kernel(float2* __restrict__ g,
                                                                   const float2* __restrict__ sf,
                                                                   float2* __restrict__ vt,
                                                                   float* __restrict__ tbar, float* __restrict__ pb,
                                                                   const float2* __restrict__ tw2, int nsb) {
  constexpr int NP = kRow * N2;
  constexpr int GROUPS = kRow / kColThreads;
  const int i = blockIdx.x / GROUPS;
  const int n1 = (blockIdx.x - i * GROUPS) * kColThreads + threadIdx.x;
  const size_t arr = (size_t)blockIdx.y * nsb + i;
  // v' and g' of a polarisation in one pass: both columns in flight, then
  // both inverse column passes, the sums, and the stores
  float p[N2], q[N2];
#pragma unroll
  for (int k = 0; k < N2; ++k) p[k] = q[k] = 0.0f;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 vf[N2], vg[N2];
    load_col<N2>(sf + (arr * 2 + pol) * NP, n1, vf);
    load_col<N2>(g + (arr * 2 + pol) * NP, n1, vg);
    col_inverse<N2>(tw2, n1, vf);
    col_inverse<N2>(tw2, n1, vg);
#pragma unroll
    for (int k = 0; k < N2; ++k) {
      vf[k] = cscale(vf[k], 1.0f / N2);
      p[k] = fmaf(vf[k].x, vf[k].x, fmaf(vf[k].y, vf[k].y, p[k]));
      q[k] = fmaf(vg[k].x, vf[k].y, fmaf(-vg[k].y, vf[k].x, q[k]));
    }
    store_col<N2>(vt + (arr * 2 + pol) * NP, n1, vf);
    store_col<N2>(g + (arr * 2 + pol) * NP, n1, vg);  // g' in place of g
  }
  float* dp = pb + arr * NP + n1;
#pragma unroll
  for (int k = 0; k < N2; ++k) dp[kRow * k] = p[k];
  float* dq = tbar + arr * NP + n1;
#pragma unroll
  for (int k = 0; k < N2; ++k) dq[kRow * k] = q[k];
}

// Forward column pass of every column of src (time samples in the state
// layout) into dst.
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_col_forward_kernel(const float2* __restrict__ src,
                                                                     float2* __restrict__ dst,
                                                                     const float2* __restrict__ tw2, int nsb) {
  constexpr int NP = kRow * N2;
  constexpr int GROUPS = kRow / kColThreads;
  const int i = blockIdx.x / GROUPS;
  const int n1 = (blockIdx.x - i * GROUPS) * kColThreads + threadIdx.x;
  const size_t arr = (size_t)blockIdx.y * nsb + i;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    float2 v[N2];
    load_col<N2>(src + (arr * 2 + pol) * NP, n1, v);
    col_forward<N2>(tw2, n1, v);
    store_col<N2>(dst + (arr * 2 + pol) * NP, n1, v);
  }
}

// Split-ratio derivative (the telescoped form of the persistent adjoint):
// with v the time samples before step st's rotation, w after it, g' the
// cotangent of w, p_bar the intensity cotangent, e = exp(-j theta) - 1 and K
// the filter phi'_q = phi_q - phi(f_i) (phi_q = 2 pi^2 beta2 f_q^2 per km,
// phi(f_i) at the subband centre) applied to a time signal,
//   G_{st+1} - G_{st} = sum_n Im(conj(K g') e v) - Im(conj(e* g' + 2 p_bar v) K v)
// over both polarisations and the subbands, where G_j = sum_q phi_q
// Im(conj(g_{A_j}) A_j) over the spectrum after dispersion segment j; then
// dL/drho = L (G_0 - G_{N_st}) = -L sum over steps.  Both terms scale with the
// nonlinear phase, where G_0 and G_{N_st} are each many times their
// difference.
//
// st_kweight_kernel: row pass [optional forward size-N1 DFT, times
// scale phi' (and h when GVD), inverse size-N1 DFT] of row k2 of array
// (block w, subband i).  Its inverse column pass is K applied to the time
// samples of the state (K v from S(st) with h the step's filter, K g' from G
// with scale 1 / N1, the gain of the unnormalised row pair).
template <bool FWD, bool GVD>
__global__ __launch_bounds__(kRowNT, 2) void st_kweight_kernel(const float2* __restrict__ src,
                                                              float2* __restrict__ dst,
                                                              const float2* __restrict__ h,
                                                              const double* __restrict__ phase, float scale,
                                                              const float2* __restrict__ twr, int nsb, int n2,
                                                              int np) {
  __shared__ __align__(16) float4 lxy[kRowLds];
  const int i = blockIdx.x / n2, k2 = blockIdx.x - (blockIdx.x / n2) * n2;
  const size_t off = ((size_t)blockIdx.y * nsb + i) * 2 * np + (size_t)k2 * kRow;
  const int t = threadIdx.x;
  float2 x[kRowRR], y[kRowRR];
#pragma unroll
  for (int o = 0; o < kRowRR; ++o) {
    x[o] = src[off + t + kRowNT * o];
    y[o] = src[off + np + t + kRowNT * o];
  }
  if constexpr (FWD) fft<kRow, false, kRowDB, kRowRR>(x, y, lxy, twr, t);
  const size_t hoff = (size_t)i * np + (size_t)k2 * kRow;
  const double centre = phase[(size_t)i * np + kRow / 2];  // bin N'/2 sits at position N1/2
#pragma unroll
  for (int o = 0; o < kRowRR; ++o) {
    float2 w = make_float2((float)(phase[hoff + t + kRowNT * o] - centre) * scale, 0.0f);
    if constexpr (GVD) w = cscale(h[hoff + t + kRowNT * o], w.x);
    x[o] = GVD ? cmul(x[o], w) : cscale(x[o], w.x);
    y[o] = GVD ? cmul(y[o], w) : cscale(y[o], w.x);
  }
  fft<kRow, true, kRowDB, kRowRR>(x, y, lxy, twr, t);
#pragma unroll
  for (int o = 0; o < kRowRR; ++o) {
    dst[off + t + kRowNT * o] = x[o];
    dst[off + np + t + kRowNT * o] = y[o];
  }
}

// Adjoint of the rotation and intensity with the split-ratio sum: per column
// n1, K g' and K v are the inverse column passes of kg and kv; g', w (as
// written by st_adj_phase_kernel in gt and vt), theta and p_bar are read per
// sample.  g_v = g' + e* g' + 2 p_bar v (= g' exp(+j theta) + 2 p_bar v, v =
// w exp(+j theta)) overwrites w in vt, for st_col_forward_kernel.  Each
// workgroup writes its FP64 share of the sum above to part.
template <int N2>
__global__ __launch_bounds__(kColThreads) void st_adj_comm_kernel(const float2* __restrict__ gt,
                                                                  float2* __restrict__ vt,
                                                                  const float2* __restrict__ kg,
                                                                  const float2* __restrict__ kv,
                                                                  const float* __restrict__ th,
                                                                  const float* __restrict__ pbar,
                                                                  const float2* __restrict__ tw2, int nsb,
                                                                  double* __restrict__ part) {
  constexpr int NP = kRow * N2;
  constexpr int GROUPS = kRow / kColThreads;
  __shared__ double red[kColThreads / 64];
  const int i = blockIdx.x / GROUPS;
  const int n1 = (blockIdx.x - i * GROUPS) * kColThreads + threadIdx.x;
  const size_t arr = (size_t)blockIdx.y * nsb + i;
  const float* tc = th + arr * NP + n1;
  const float* pc = pbar + arr * NP + n1;
  double acc = 0.0;
#pragma unroll 1
  for (int pol = 0; pol < 2; ++pol) {
    const size_t base = (arr * 2 + pol) * NP;
    float2 a[N2], b[N2];
    load_col<N2>(kg + base, n1, a);
    col_inverse<N2>(tw2, n1, a);
    load_col<N2>(kv + base, n1, b);
    col_inverse<N2>(tw2, n1, b);
    const float2* gc = gt + base + n1;
    float2* vc = vt + base + n1;
    // Samples in chunks: a chunk's loads all precede its stores.  (Stores
    // count in the same in-order memory counter as loads, so a load issued
    // after a store waits for it; sample by sample, every load waited for
    // the previous sample's store.)
    constexpr int CH = N2 < 8 ? N2 : 8;
#pragma unroll
    for (int k0 = 0; k0 < N2; k0 += CH) {
      float tv[CH], pv[CH];
      float2 wv[CH], gv[CH];
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        tv[j] = tc[kRow * (k0 + j)];
        pv[j] = pc[kRow * (k0 + j)];
        wv[j] = vc[kRow * (k0 + j)];
        gv[j] = gc[kRow * (k0 + j)];
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const int k = k0 + j;
        float sh, ch;
        phase_sincos(0.5f * tv[j], sh, ch);
        const float2 e = make_float2(-2.0f * sh * sh, -2.0f * sh * ch);  // exp(-j theta) - 1
        const float2 w = wv[j], g = gv[j];
        const float2 ew = cmulc(w, e);                                   // conj(e) w = v - w
        const float2 v = cadd(w, ew);
        const float2 ge = cmulc(g, e);                                   // conj(e) g'
        const float p2 = 2.0f * pv[j];
        const float2 dg = make_float2(fmaf(p2, v.x, ge.x), fmaf(p2, v.y, ge.y));
        // Im(conj(K g') e v) with e v = w - v = -conj(e) w; Im(conj(dg) K v)
        const float t1 = -fmaf(a[k].x, ew.y, -a[k].y * ew.x);
        const float t2 = fmaf(dg.x, b[k].y, -dg.y * b[k].x);
        acc += (double)t1 - (double)t2;
        wv[j] = cadd(g, dg);
      }
#pragma unroll
      for (int j = 0; j < CH; ++j) vc[kRow * (k0 + j)] = wv[j];
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int wv = 0; wv < kColThreads / 64; ++wv) sum += red[wv];
    part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sum;
  }
}

// Coefficient cotangent of eq. (15) over one block's kCgOut consecutive
// samples n0 .. n0 + kCgOut - 1:
//   part[i][l][tau] = sum_n theta_bar_i[n] p_l[(n - tau + nc) mod N'].
// Thread work items are (l, tau) pairs, each over a contiguous share of the
// samples (pairs x shares <= 256); the shares are added in LDS in a fixed
// order.  Per 4 samples a thread reads theta_bar of every subband as one
// 128-bit word (the same for all lanes of a share) and 4 intensities.  LDS
// (dynamic): p rows with a halo of nc each side, read as aligned float4 from
// the float4 group holding sample n0 - nc (row width rounded up to 4 floats,
// the window starting at the shift psh < 4), theta_bar rows, the share
// partials.  Every row load is issued before the first LDS store, with
// clamped (always valid) indices, so the loads carry no branch and wait once.
constexpr int kCgOut = 512;

__host__ __device__ inline int cg_shares(int npair) {
  int sh = 1;
  while (2 * sh * npair <= 256 && sh < 64) sh *= 2;
  return sh;
}
__host__ __device__ inline int cg_pw4(int n_taps) { return (kCgOut + n_taps + 6) / 4; }  // p row, float4
__host__ __device__ inline int cg_pw(int n_taps) { return 4 * cg_pw4(n_taps); }
__host__ inline size_t cg_lds_bytes(int nsb, int n_taps) {
  const int npair = nsb * n_taps;
  const int sh = npair > 256 ? 1 : cg_shares(npair);
  return sizeof(float) * ((size_t)nsb * cg_pw(n_taps) + (size_t)nsb * kCgOut +
                          (npair > 256 ? 0 : (size_t)sh * npair * nsb));
}

template <int NSB>
__global__ __launch_bounds__(256) void st_cgrad_kernel(const float* __restrict__ tbar, const float* __restrict__ pb,
                                                       float* __restrict__ part, int np, int n_taps) {
  constexpr int nsb = NSB;
  extern __shared__ __align__(16) float cg_lds[];
  const int nc = n_taps / 2;
  const int pw = cg_pw(n_taps);
  float* ptile = cg_lds;
  float* ttile = cg_lds + (size_t)nsb * pw;  // 16-byte aligned: pw is a multiple of 4
  float* red = ttile + (size_t)nsb * kCgOut;
  const int n0 = blockIdx.x * kCgOut;
  const size_t arr0 = (size_t)blockIdx.y * nsb;
  const int t = threadIdx.x;
  // p row l: ptile[l][j] = p_l[(4 pg0 + j) mod N'], sample n0 - nc at j = psh
  const int psh = ((n0 - nc) % 4 + 4) % 4;
  const int pg0 = (n0 - nc - psh) / 4, np4 = np / 4, pw4 = pw / 4;
  {
    constexpr int PCNT = (NSB * ((kCgOut + kMaxTaps + 6) / 4) + 255) / 256;
    constexpr int TCNT = (NSB * (kCgOut / 4) + 255) / 256;
    const int pn = nsb * pw4;
    fir_v4 pv[PCNT], tv[TCNT];
#pragma unroll
    for (int c = 0; c < PCNT; ++c) {
      const int idx = t + 256 * c < pn ? t + 256 * c : pn - 1;
      const int l = idx / pw4;
      int g = pg0 + idx - l * pw4;
      g = g < 0 ? g + np4 : (g >= np4 ? g - np4 : g);
      pv[c] = reinterpret_cast<const fir_v4*>(pb + (arr0 + l) * np)[g];
    }
#pragma unroll
    for (int c = 0; c < TCNT; ++c) {
      const int idx = t + 256 * c < nsb * (kCgOut / 4) ? t + 256 * c : nsb * (kCgOut / 4) - 1;
      const int l = idx / (kCgOut / 4);
      tv[c] = reinterpret_cast<const fir_v4*>(tbar + (arr0 + l) * np + n0)[idx - l * (kCgOut / 4)];
    }
    fir_v4* p4 = reinterpret_cast<fir_v4*>(ptile);
    fir_v4* q4 = reinterpret_cast<fir_v4*>(ttile);
#pragma unroll
    for (int c = 0; c < PCNT; ++c)
      if (t + 256 * c < pn) p4[t + 256 * c] = pv[c];
#pragma unroll
    for (int c = 0; c < TCNT; ++c)
      if (t + 256 * c < nsb * (kCgOut / 4)) q4[t + 256 * c] = tv[c];
  }
  __syncthreads();
  const int npair = nsb * n_taps;
  const bool wide = npair > 256;
  const int sh = wide ? 1 : cg_shares(npair);
  const int len = kCgOut / sh;  // a multiple of 8
  const size_t out0 = ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * nsb * npair;
  const int items = wide ? npair : sh * npair;
  const float4* t4 = reinterpret_cast<const float4*>(ttile);
  for (int wi = t; wi < items; wi += 256) {
    const int pr = wide ? wi : wi % npair;
    const int sp = wide ? 0 : wi / npair;
    const int l = pr / n_taps, tau = pr - (pr / n_taps) * n_taps;
    // p_l[n - tau + nc] sits at ptile[l][psh + n - n0 - tau + 2 nc]
    const float* prow = ptile + l * pw + psh + 2 * nc - tau;
    float acc[kMaxSubbands];
#pragma unroll
    for (int i = 0; i < kMaxSubbands; ++i) acc[i] = 0.0f;
    for (int n = sp * len; n < (sp + 1) * len; n += 4) {
      const float p0 = prow[n], p1 = prow[n + 1], p2 = prow[n + 2], p3 = prow[n + 3];
#pragma unroll
      for (int i = 0; i < kMaxSubbands; ++i) {
        if (i < nsb) {
          const float4 tv = t4[(i * kCgOut + n) >> 2];
          acc[i] = fmaf(tv.x, p0, fmaf(tv.y, p1, fmaf(tv.z, p2, fmaf(tv.w, p3, acc[i]))));
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kMaxSubbands; ++i) {
      if (i < nsb) {
        if (wide)
          part[out0 + ((size_t)i * nsb + l) * n_taps + tau] = acc[i];
        else
          red[((size_t)sp * npair + pr) * nsb + i] = acc[i];
      }
    }
  }
  if (!wide) {
    __syncthreads();
    for (int j = t; j < npair * nsb; j += 256) {
      const int pr = j / nsb, i = j - (j / nsb) * nsb;
      float sum = 0.0f;
      for (int sp = 0; sp < sh; ++sp) sum += red[((size_t)sp * npair + pr) * nsb + i];
      const int l = pr / n_taps, tau = pr - (pr / n_taps) * n_taps;
      part[out0 + ((size_t)i * nsb + l) * n_taps + tau] = sum;
    }
  }
}

// Adjoint row pass across a dispersion filter Y = h X, with the derivative of
// h = exp(j phi dz) / scale in its segment length dz (Sec. III-C):
//   part[row] = sum phi Im(conj(Gy) Y)   (dL/d dz = -sum over rows),
// Gy = F1(g) (G_FWD) or g, X = F1(xs) (X_FWD) or xs.  STORE writes
// conj(h) Gy back to g, through the inverse row DFT when INV.
template <bool G_FWD, bool X_FWD, bool STORE, bool INV>
__global__ __launch_bounds__(kGvdNT, 2) void st_gvd_adj_kernel(float2* g, const float2* __restrict__ xs,
                                                              const float2* __restrict__ h,
                                                              const double* __restrict__ phase,
                                                              double* __restrict__ part,
                                                              const float2* __restrict__ twr, int nsb, int n2,
                                                              int np) {
  __shared__ __align__(16) float4 lxy[kRowLds];
  __shared__ double red[kGvdNT / 64];
  const int i = blockIdx.x / n2, k2 = blockIdx.x - (blockIdx.x / n2) * n2;
  const size_t off = ((size_t)blockIdx.y * nsb + i) * 2 * np + (size_t)k2 * kRow;
  const int t = threadIdx.x;
  float2 gx[kGvdRR], gy[kGvdRR];
#pragma unroll
  for (int o = 0; o < kGvdRR; ++o) {
    gx[o] = g[off + t + kGvdNT * o];
    gy[o] = g[off + np + t + kGvdNT * o];
  }
  if constexpr (G_FWD) fft<kRow, false, kRowDB, kGvdRR>(gx, gy, lxy, twr, t);
  double acc = 0.0;
  {
    float2 x[kGvdRR], y[kGvdRR];
#pragma unroll
    for (int o = 0; o < kGvdRR; ++o) {
      x[o] = xs[off + t + kGvdNT * o];
      y[o] = xs[off + np + t + kGvdNT * o];
    }
    if constexpr (X_FWD) fft<kRow, false, kRowDB, kGvdRR>(x, y, lxy, twr, t);
    const size_t hoff = (size_t)i * np + (size_t)k2 * kRow;
#pragma unroll
    for (int o = 0; o < kGvdRR; ++o) {
      const float2 hv = h[hoff + t + kGvdNT * o];
      const float2 yx = cmul(x[o], hv), yy = cmul(y[o], hv);
      const float im = fmaf(gx[o].x, yx.y, fmaf(-gx[o].y, yx.x, fmaf(gy[o].x, yy.y, -gy[o].y * yy.x)));
      acc += phase[hoff + t + kGvdNT * o] * (double)im;
      if constexpr (STORE) {
        gx[o] = cmulc(gx[o], hv);
        gy[o] = cmulc(gy[o], hv);
      }
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if ((t & 63) == 0) red[t >> 6] = acc;
  __syncthreads();
  if (t == 0) {
    double sum = 0.0;
    for (int wv = 0; wv < kGvdNT / 64; ++wv) sum += red[wv];
    part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = sum;
  }
  if constexpr (STORE) {
    if constexpr (INV) fft<kRow, true, kRowDB, kGvdRR>(gx, gy, lxy, twr, t);
#pragma unroll
    for (int o = 0; o < kGvdRR; ++o) {
      g[off + t + kGvdNT * o] = gx[o];
      g[off + np + t + kGvdNT * o] = gy[o];
    }
  }
}

// acc[j] += sum over r < n_rows of part[r][j] (FP64, fixed order), in two
// launches: st_sum_rows_kernel gives the sum of every chunk of rows
// (chunk c = rows c, c + kAccC, ...; thread (jj, g) of a 64 x 16 block sums
// every 16th of them, then a fixed tree), st_add_chunks_kernel adds the
// kAccC chunk sums in order.
constexpr int kAccJ = 64, kAccG = 16, kAccC = 32;
__global__ __launch_bounds__(kAccJ * kAccG) void st_sum_rows_kernel(const float* __restrict__ part, int n_rows,
                                                                   int per_row, double* __restrict__ csum) {
  __shared__ double buf[kAccG][kAccJ];
  const int jj = threadIdx.x % kAccJ, gg = threadIdx.x / kAccJ;
  const int j = blockIdx.x * kAccJ + jj;
  const int c = blockIdx.y;
  double s = 0.0;
  if (j < per_row)
    for (int r = c + kAccC * gg; r < n_rows; r += kAccC * kAccG) s += (double)part[(size_t)r * per_row + j];
  buf[gg][jj] = s;
  __syncthreads();
  for (int w = kAccG / 2; w > 0; w >>= 1) {
    if (gg < w) buf[gg][jj] += buf[gg + w][jj];
    __syncthreads();
  }
  if (gg == 0 && j < per_row) csum[(size_t)c * per_row + j] = buf[0][jj];
}
__global__ void st_add_chunks_kernel(const double* __restrict__ csum, int per_row, double* __restrict__ acc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= per_row) return;
  double s = 0.0;
  for (int c = 0; c < kAccC; ++c) s += csum[(size_t)c * per_row + j];
  acc[j] += s;
}

// *acc += sum of part[0 .. n) (FP64, fixed order).
__global__ __launch_bounds__(256) void st_acc_sum_kernel(const double* __restrict__ part, int n,
                                                        double* __restrict__ acc) {
  __shared__ double buf[256];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += part[k];
  buf[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *acc += buf[0];
}

__global__ void st_zero_kernel(double* __restrict__ p, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0.0;
}

// Final gradients: dL/dC from the FP64 sums; acc_t[j] = sum phi Im(conj(Gy) Y)
// over dispersion segment j, so dL/d(length j) = -acc_t[j]; acc_t[steps + 1]
// is the sum over steps of G_{st+1} - G_{st} (st_adj_comm_kernel), so with
// the first and last segments (1 - rho) L and rho L,
// dL/drho = L (G_0 - G_{N_st}) = -L acc_t[steps + 1].
__global__ void st_bwd_finish_kernel(const double* __restrict__ acc_c, int n_c, const double* __restrict__ acc_t,
                                     int steps, double L, float* __restrict__ grad_c, float* __restrict__ grad_rho,
                                     double* __restrict__ grad_gvd) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n_c) grad_c[k] = (float)acc_c[k];
  if (k == 0) *grad_rho = (float)(-L * acc_t[steps + 1]);
  if (grad_gvd != nullptr && k <= steps) grad_gvd[k] = -acc_t[k];
}

// ------------------------------------------------------------------ launcher
namespace {

bool ok_launch() { return hipGetLastError() == hipSuccess; }

// The coupled-filter kernels take the subband count as a template argument,
// so their per-subband loops have no branches and their loads batch.
template <int NSB>
void fir_t(int ny, hipStream_t s, const float* pb, float* th, const float* cs, int np, int nc, int tap_pad,
           const StreamBlk* blk, int step) {
  // up to 32 taps: the matrix-core kernel, taps a compile-time count
  const dim3 gm((np + FirMfma<NSB>::OUT - 1) / FirMfma<NSB>::OUT, ny);
  const size_t lm = fir_mfma_lds_bytes(NSB, tap_pad);
  switch (tap_pad / kTapChunk) {
    case 1: st_fir_mfma_kernel<NSB, 1><<<gm, 256, lm, s>>>(pb, th, cs, np, nc, blk, step); break;
    case 2: st_fir_mfma_kernel<NSB, 2><<<gm, 256, lm, s>>>(pb, th, cs, np, nc, blk, step); break;
    case 3: st_fir_mfma_kernel<NSB, 3><<<gm, 256, lm, s>>>(pb, th, cs, np, nc, blk, step); break;
    case 4: st_fir_mfma_kernel<NSB, 4><<<gm, 256, lm, s>>>(pb, th, cs, np, nc, blk, step); break;
    default:
      st_fir_kernel<NSB, 0><<<dim3(np / kFirOut, ny), 256, fir_lds_bytes(NSB, tap_pad), s>>>(pb, th, cs, np, nc,
                                                                                          tap_pad, blk, step);
  }
}
bool launch_fir(int nsb, int ny, hipStream_t s, const float* pb, float* th, const float* cs, int np, int nc,
                int tap_pad, const StreamBlk* blk = nullptr, int step = 0) {
  switch (nsb) {
    case 1: fir_t<1>(ny, s, pb, th, cs, np, nc, tap_pad, blk, step); break;
    case 2: fir_t<2>(ny, s, pb, th, cs, np, nc, tap_pad, blk, step); break;
    case 3: fir_t<3>(ny, s, pb, th, cs, np, nc, tap_pad, blk, step); break;
    case 4: fir_t<4>(ny, s, pb, th, cs, np, nc, tap_pad, blk, step); break;
    case 5: fir_t<5>(ny, s, pb, th, cs, np, nc, tap_pad, blk, step); break;
    case 6: fir_t<6>(ny, s, pb, th, cs, np, nc, tap_pad, blk, step); break;
    case 7: fir_t<7>(ny, s, pb, th, cs, np, nc, tap_pad, blk, step); break;
    case 8: fir_t<8>(ny, s, pb, th, cs, np, nc, tap_pad, blk, step); break;
    default: return false;
  }
  return ok_launch();
}
template <int NSB>
void cgrad_t(dim3 grid, size_t lds, hipStream_t s, const float* tbar, const float* pb, float* part, int np,
             int n_taps) {
  st_cgrad_kernel<NSB><<<grid, 256, lds, s>>>(tbar, pb, part, np, n_taps);
}
bool launch_cgrad(int nsb, dim3 grid, hipStream_t s, const float* tbar, const float* pb, float* part, int np,
                  int n_taps) {
  const size_t lds = cg_lds_bytes(nsb, n_taps);
  switch (nsb) {
    case 1: cgrad_t<1>(grid, lds, s, tbar, pb, part, np, n_taps); break;
    case 2: cgrad_t<2>(grid, lds, s, tbar, pb, part, np, n_taps); break;
    case 3: cgrad_t<3>(grid, lds, s, tbar, pb, part, np, n_taps); break;
    case 4: cgrad_t<4>(grid, lds, s, tbar, pb, part, np, n_taps); break;
    case 5: cgrad_t<5>(grid, lds, s, tbar, pb, part, np, n_taps); break;
    case 6: cgrad_t<6>(grid, lds, s, tbar, pb, part, np, n_taps); break;
    case 7: cgrad_t<7>(grid, lds, s, tbar, pb, part, np, n_taps); break;
    case 8: cgrad_t<8>(grid, lds, s, tbar, pb, part, np, n_taps); break;
    default: return false;
  }
  return ok_launch();
}

template <bool FWD, bool GVD, bool INV, bool CONJ = false>
bool row(const StreamArgs& a, const float2* src, float2* dst, const float2* h, hipStream_t s) {
  st_row_kernel<FWD, GVD, INV, CONJ>
      <<<dim3(a.n_sb * a.n2, a.nb), kRowNT, 0, s>>>(src, dst, h, a.twr, a.n_sb, a.n2, a.np, nullptr, 0);
  return ok_launch();
}

const float2* step_filter(const Tables& tb, int st) {
  return st == 0 ? tb.h_first : tb.h_mid + (size_t)(st - 1) * tb.h_stride;
}

// Block input: framing, polyphase column pass and (n_sb > 1) row pass and
// DEMUX into the subband spectra, in a.st.
template <int N2>
bool wave_input(const StreamArgs& a, const Tables& tb, hipStream_t s) {
  const int nsb = a.n_sb;
  const dim3 col_grid((nsb * kRow + kColThreads - 1) / kColThreads, a.nb);
  st_head_kernel<N2><<<col_grid, kColThreads, 0, s>>>(a, nullptr);
  bool ok = ok_launch();
  if (nsb > 1) {
    StreamWsb wsb;
    for (int k = 0; k < kMaxSubbands; ++k) wsb.w[k] = tb.wsb[k];
    ok = ok && row<true, false, false>(a, a.st, a.st, nullptr, s);
    st_mix_kernel<false><<<dim3(a.np / 256, a.nb), 256, 0, s>>>(a.st, tb.poly_tw, wsb, nsb, a.np, nullptr);
    ok = ok && ok_launch();
  }
  return ok;
}

// Step st (0-based) from state src to state dst: row pass with the step's
// dispersion filter into work, intensity, coupled filter into theta,
// rotation from work into dst.
template <int N2>
bool wave_step(const StreamArgs& a, const Tables& tb, const float* cpad, int st, int n_taps, int tap_pad,
               const float2* src, float2* work, float* theta, float2* dst, hipStream_t s) {
  const int nsb = a.n_sb;
  const dim3 sb_grid(nsb * (kRow / kColThreads), a.nb);
  const float2* h = step_filter(tb, st);
  bool ok = (st == 0 && nsb > 1) ? row<false, true, true>(a, src, work, h, s) : row<true, true, true>(a, src, work, h, s);
  st_intensity_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(work, a.pb, a.tw2, nsb, nullptr);
  ok = ok && ok_launch();
  ok = ok && launch_fir(nsb, a.nb, s, a.pb, theta,
                        cpad + (size_t)st * nsb * nsb * tap_pad, a.np, n_taps / 2, tap_pad);
  ok = ok && ok_launch();
  st_rotate_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(work, dst, theta, a.tw2, nsb, nullptr);
  return ok && ok_launch();
}

// Block output: final dispersion segment, MUX, inverse column pass, kept
// samples.
template <int N2>
bool wave_output(const StreamArgs& a, const Tables& tb, hipStream_t s) {
  const int nsb = a.n_sb;
  bool ok = true;
  if (nsb > 1) {
    StreamWsb wsb;
    for (int k = 0; k < kMaxSubbands; ++k) wsb.w[k] = tb.wsb[k];
    ok = ok && row<true, true, false>(a, a.st, a.st, tb.h_last, s);
    st_mix_kernel<true><<<dim3(a.np / 256, a.nb), 256, 0, s>>>(a.st, tb.poly_tw, wsb, nsb, a.np, nullptr);
    ok = ok && ok_launch();
    ok = ok && row<false, false, true>(a, a.st, a.st, nullptr, s);
  } else {
    ok = ok && row<true, true, true>(a, a.st, a.st, tb.h_last, s);
  }
  st_tail_kernel<N2><<<dim3((nsb * kRow + kColThreads - 1) / kColThreads, a.nb), kColThreads, 0, s>>>(a, nullptr);
  return ok && ok_launch();
}

template <int N2>
int run_wave(const StreamArgs& a, const Tables& tb, const float* cpad, int steps, int n_taps, int tap_pad,
             hipStream_t s) {
  bool ok = wave_input<N2>(a, tb, s);
  for (int st = 0; st < steps && ok; ++st)
    ok = wave_step<N2>(a, tb, cpad, st, n_taps, tap_pad, a.st, a.st, a.th, a.st, s);
  ok = ok && wave_output<N2>(a, tb, s);
  return ok ? CBESSFM_OK : CBESSFM_EHIP;
}

// Step `step` of every block in the table blks[0 .. nb) (instances of one
// class: same N', n_sb and taps; each entry names its own state, phase and
// intensity arrays and its plan's tables).  The same kernels as wave_step.
template <int N2>
bool class_step(int nsb, int n_taps, int tap_pad, int step, const StreamBlk* blks, int nb, hipStream_t s) {
  constexpr int NP = kRow * N2;
  const dim3 row_grid(nsb * N2, nb), sb_grid(nsb * (kRow / kColThreads), nb);
  if (step == 0 && nsb > 1)
    st_row_kernel<false, true, true>
        <<<row_grid, kRowNT, 0, s>>>(nullptr, nullptr, nullptr, nullptr, nsb, N2, NP, blks, step);
  else
    st_row_kernel<true, true, true><<<row_grid, kRowNT, 0, s>>>(nullptr, nullptr, nullptr, nullptr, nsb, N2, NP, blks, step);
  bool ok = ok_launch();
  st_intensity_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(nullptr, nullptr, nullptr, nsb, blks);
  ok = ok && ok_launch();
  ok = ok && launch_fir(nsb, nb, s, nullptr, nullptr, nullptr, NP, n_taps / 2, tap_pad, blks,
                        step);
  st_rotate_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(nullptr, nullptr, nullptr, nullptr, nsb, blks);
  return ok && ok_launch();
}

// Block input and output of every block in the table: the kernels of
// wave_input and wave_output, each one launch over all the blocks.
template <int N2>
bool class_input(int nsb, const StreamWsb& wsb, const StreamBlk* blks, int nb, hipStream_t s) {
  constexpr int NP = kRow * N2;
  StreamArgs a{};
  a.n_sb = nsb;
  st_head_kernel<N2><<<dim3((nsb * kRow + kColThreads - 1) / kColThreads, nb), kColThreads, 0, s>>>(a, blks);
  bool ok = ok_launch();
  if (nsb > 1) {
    st_row_kernel<true, false, false>
        <<<dim3(nsb * N2, nb), kRowNT, 0, s>>>(nullptr, nullptr, nullptr, nullptr, nsb, N2, NP, blks, 0);
    ok = ok && ok_launch();
    st_mix_kernel<false><<<dim3(NP / 256, nb), 256, 0, s>>>(nullptr, nullptr, wsb, nsb, NP, blks);
    ok = ok && ok_launch();
  }
  return ok;
}

template <int N2>
bool class_output(int nsb, const StreamWsb& wsb, const StreamBlk* blks, int nb, hipStream_t s) {
  constexpr int NP = kRow * N2;
  const dim3 row_grid(nsb * N2, nb);
  bool ok;
  if (nsb > 1) {
    st_row_kernel<true, true, false><<<row_grid, kRowNT, 0, s>>>(nullptr, nullptr, nullptr, nullptr, nsb, N2, NP, blks, -1);
    ok = ok_launch();
    st_mix_kernel<true><<<dim3(NP / 256, nb), 256, 0, s>>>(nullptr, nullptr, wsb, nsb, NP, blks);
    ok = ok && ok_launch();
    st_row_kernel<false, false, true><<<row_grid, kRowNT, 0, s>>>(nullptr, nullptr, nullptr, nullptr, nsb, N2, NP, blks, 0);
    ok = ok && ok_launch();
  } else {
    st_row_kernel<true, true, true><<<row_grid, kRowNT, 0, s>>>(nullptr, nullptr, nullptr, nullptr, nsb, N2, NP, blks, -1);
    ok = ok_launch();
  }
  StreamArgs a{};
  a.n_sb = nsb;
  st_tail_kernel<N2><<<dim3((nsb * kRow + kColThreads - 1) / kColThreads, nb), kColThreads, 0, s>>>(a, blks);
  return ok && ok_launch();
}

void fill_stream_args(const cbessfm_plan_t* p, const void* in, void* out, long long T, StreamArgs& a) {
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
}

}  // namespace

int stream_single_wave(const cbessfm_plan_t* p, long long T, int batch) {
  const long long items = (long long)batch * ((T + p->hop - 1) / p->hop);
  return p->stream && p->nlpr == CBESSFM_NLPR_AVERAGED && items <= p->st_blocks;
}

void stream_blocks(const cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, StreamBlk* out_blk) {
  Tables tb;
  fill_tables(p, tb);
  const int nsb = p->sb.n_sb;
  const size_t np = (size_t)p->Np;
  const int nblk = (int)((T + p->hop - 1) / p->hop);
  for (long long b = 0; b < (long long)batch * nblk; ++b) {
    StreamBlk& e = out_blk[b];
    e.st = p->d_st + (size_t)b * nsb * 2 * np;
    e.pb = p->d_pb + (size_t)b * nsb * np;
    e.th = p->d_th + (size_t)b * nsb * np;
    e.h_first = tb.h_first;
    e.h_mid = tb.h_mid;
    e.h_last = tb.h_last;
    e.h_stride = tb.h_stride;
    e.cpad = p->d_cpad;
    e.tw2 = p->d_tw;
    e.twr = p->d_tw + p->Np;
    e.poly = tb.poly_tw;
    const long long entry = b / nblk;  // batch entry
    e.in = static_cast<const float2*>(in) + (size_t)entry * 2 * T;
    e.out = static_cast<float2*>(out) + (size_t)entry * 2 * T;
    e.T = (int)T;
    e.blk = (int)(b - entry * nblk);
    e.hop = p->hop;
    e.n_ov = p->sb.overlap;
    e.boundary = p->sb.boundary;
  }
}

int stream_class_input(const cbessfm_plan_t* p0, const StreamBlk* d_blks, int nb, hipStream_t s) {
  if (nb < 1) return CBESSFM_OK;
  Tables tb;
  fill_tables(p0, tb);
  StreamWsb wsb;
  for (int k = 0; k < kMaxSubbands; ++k) wsb.w[k] = tb.wsb[k];
  const int nsb = p0->sb.n_sb;
  bool ok;
  switch (p0->log_np) {
    case 14: ok = class_input<4>(nsb, wsb, d_blks, nb, s); break;
    case 15: ok = class_input<8>(nsb, wsb, d_blks, nb, s); break;
    case 16: ok = class_input<16>(nsb, wsb, d_blks, nb, s); break;
    case 17: ok = class_input<32>(nsb, wsb, d_blks, nb, s); break;
    default: return CBESSFM_EUNSUPPORTED;
  }
  return ok ? CBESSFM_OK : CBESSFM_EHIP;
}

int stream_class_output(const cbessfm_plan_t* p0, const StreamBlk* d_blks, int nb, hipStream_t s) {
  if (nb < 1) return CBESSFM_OK;
  Tables tb;
  fill_tables(p0, tb);
  StreamWsb wsb;
  for (int k = 0; k < kMaxSubbands; ++k) wsb.w[k] = tb.wsb[k];
  const int nsb = p0->sb.n_sb;
  bool ok;
  switch (p0->log_np) {
    case 14: ok = class_output<4>(nsb, wsb, d_blks, nb, s); break;
    case 15: ok = class_output<8>(nsb, wsb, d_blks, nb, s); break;
    case 16: ok = class_output<16>(nsb, wsb, d_blks, nb, s); break;
    case 17: ok = class_output<32>(nsb, wsb, d_blks, nb, s); break;
    default: return CBESSFM_EUNSUPPORTED;
  }
  return ok ? CBESSFM_OK : CBESSFM_EHIP;
}

int stream_class_step(int log_np, int n_sb, int n_taps, int tap_pad, int step, const StreamBlk* d_blks, int nb,
                      hipStream_t s) {
  if (nb < 1) return CBESSFM_OK;
  bool ok;
  switch (log_np) {
    case 14: ok = class_step<4>(n_sb, n_taps, tap_pad, step, d_blks, nb, s); break;
    case 15: ok = class_step<8>(n_sb, n_taps, tap_pad, step, d_blks, nb, s); break;
    case 16: ok = class_step<16>(n_sb, n_taps, tap_pad, step, d_blks, nb, s); break;
    case 17: ok = class_step<32>(n_sb, n_taps, tap_pad, step, d_blks, nb, s); break;
    default: return CBESSFM_EUNSUPPORTED;
  }
  return ok ? CBESSFM_OK : CBESSFM_EHIP;
}

int stream_launches(const cbessfm_plan_t* p, int steps) {
  const bool multi = p->sb.n_sb > 1;
  const int in = multi ? 3 : 1;   // head [, row pass, DEMUX]
  const int out = multi ? 4 : 2;  // [row pass, MUX,] row pass, tail
  return in + out + 4 * steps;    // each step: row pass, intensity, filter, rotation
}

int launch_stream_forward(cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, hipStream_t s) {
  if (p->nlpr != CBESSFM_NLPR_AVERAGED) return CBESSFM_EUNSUPPORTED;
  Tables tb;
  fill_tables(p, tb);
  StreamArgs a;
  fill_stream_args(p, in, out, T, a);
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

// ---- adjoint launcher
// Workspace of one adjoint call, for waves of up to st_blocks blocks:
//   ck     [n_ck] states S_{c k} at every segment start (S_0 = subband spectra)
//   slot   [k] states after the steps of the current segment
//   work   one state (row-pass output of a forward step)
//   g      one state (the adjoint state)
//   v      one state-sized array of time samples (v' of the step being undone)
//   theta  [k] phase arrays of the segment's steps
//   kg     one state (K g' of the step being undone, before its column pass;
//          K v goes to work)
//   tbar   one phase-cotangent array
//   cpart  coefficient partials of one step, [N' / kCgOut x nb][n_sb][n_sb][n_taps]
//   rpart  dispersion and split-ratio partials of one pass, [n_sb max(N2, N1 / 256) nb]
//   acc_c  FP64 [steps][n_sb][n_sb][n_taps], acc_t FP64 [steps + 2] (segment
//          derivatives, then the split-ratio sum)
//   csum   FP64 [kAccC][n_sb][n_sb][n_taps] chunk sums of the partials
//   gin    [batch nblk][2][N] block input cotangents (only with grad_in)
// A state is [nb][n_sb][2][N'] complex; p and p_bar use the plan's arrays.
StreamBwdLayout stream_bwd_layout(const cbessfm_plan_t* p, long long T, int batch, int ck_every, bool gin) {
  StreamBwdLayout L;
  L.k = (ck_every <= 1 || ck_every > p->steps) ? p->steps : ck_every;
  L.n_ck = (p->steps + L.k - 1) / L.k;
  L.nblk = (int)((T + p->hop - 1) / p->hop);
  const int items = batch * L.nblk;
  L.nb = items < p->st_blocks ? items : p->st_blocks;
  const size_t nsb = p->sb.n_sb, cells = (size_t)L.nb * nsb * p->Np;
  L.state = cells * 2;
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t sbytes = up(sizeof(float2) * L.state);
  L.ck_off = 0;
  L.slot_off = L.ck_off + sbytes * L.n_ck;
  L.work_off = L.slot_off + sbytes * L.k;
  L.g_off = L.work_off + sbytes;
  L.v_off = L.g_off + sbytes;
  L.kg_off = L.v_off + sbytes;
  L.theta_off = L.kg_off + sbytes;
  L.tbar_off = L.theta_off + up(sizeof(float) * cells) * L.k;
  L.cpart_off = L.tbar_off + up(sizeof(float) * cells);
  const size_t n_cg = (size_t)(p->Np / kCgOut) * L.nb;
  L.rpart_off = L.cpart_off + up(sizeof(float) * n_cg * nsb * nsb * p->n_taps);
  const size_t rows = (size_t)std::max(p->Np / kRow, kRow / kColThreads);
  L.accc_off = L.rpart_off + up(sizeof(double) * nsb * rows * L.nb);
  L.acct_off = L.accc_off + up(sizeof(double) * (size_t)p->steps * nsb * nsb * p->n_taps);
  L.csum_off = L.acct_off + up(sizeof(double) * (size_t)(p->steps + 2));
  L.gin_off = L.csum_off + up(sizeof(double) * kAccC * nsb * nsb * p->n_taps);
  L.bytes = L.gin_off + (gin ? up(sizeof(float2) * (size_t)items * 2 * p->N) : 0);
  return L;
}

namespace {

struct StreamBwdCall {
  const cbessfm_plan_t* p;
  Tables tb;
  StreamBwdLayout L;
  char* ws;
  const float2* gout;
  bool want_gvd, want_gin;
  hipStream_t s;
  size_t sbytes() const { return (sizeof(float2) * L.state + 255) & ~(size_t)255; }
  size_t tbytes() const { return (sizeof(float) * (L.state / 2) + 255) & ~(size_t)255; }
  float2* ck(int c) const { return reinterpret_cast<float2*>(ws + L.ck_off + sbytes() * c); }
  // state after q steps
  float2* S(int q) const {
    if (q % L.k == 0 && q / L.k < L.n_ck) return ck(q / L.k);
    return reinterpret_cast<float2*>(ws + L.slot_off + sbytes() * ((q - 1) % L.k));
  }
  float* TH(int st) const { return reinterpret_cast<float*>(ws + L.theta_off + tbytes() * (st % L.k)); }
  float2* work() const { return reinterpret_cast<float2*>(ws + L.work_off); }
  float2* G() const { return reinterpret_cast<float2*>(ws + L.g_off); }
  float2* V() const { return reinterpret_cast<float2*>(ws + L.v_off); }
  float2* KG() const { return reinterpret_cast<float2*>(ws + L.kg_off); }
  double* csum() const { return reinterpret_cast<double*>(ws + L.csum_off); }
  float* tbar() const { return reinterpret_cast<float*>(ws + L.tbar_off); }
  float* cpart() const { return reinterpret_cast<float*>(ws + L.cpart_off); }
  double* rpart() const { return reinterpret_cast<double*>(ws + L.rpart_off); }
  double* acc_c() const { return reinterpret_cast<double*>(ws + L.accc_off); }
  double* acc_t() const { return reinterpret_cast<double*>(ws + L.acct_off); }
  float2* gin() const { return reinterpret_cast<float2*>(ws + L.gin_off); }
};

// Row pass of the adjoint across filter h with the segment-length derivative
// summed into acc_t[seg].
template <bool G_FWD, bool X_FWD, bool STORE, bool INV>
bool gvd_adj(const StreamBwdCall& c, const StreamArgs& a, const float2* xs, const float2* h, int seg) {
  const dim3 grid(a.n_sb * a.n2, a.nb);
  st_gvd_adj_kernel<G_FWD, X_FWD, STORE, INV>
      <<<grid, kGvdNT, 0, c.s>>>(c.G(), xs, h, c.p->d_phase, c.rpart(), a.twr, a.n_sb, a.n2, a.np);
  bool ok = ok_launch();
  st_acc_sum_kernel<<<1, 256, 0, c.s>>>(c.rpart(), (int)(grid.x * grid.y), c.acc_t() + seg);
  return ok && ok_launch();
}

template <int N2>
int bwd_wave(const StreamBwdCall& c, StreamArgs a) {
  const cbessfm_plan_t* p = c.p;
  const Tables& tb = c.tb;
  const int nsb = a.n_sb, steps = p->steps, k = c.L.k;
  const int n_taps = p->n_taps, tap_pad = p->tap_pad;
  const int per_step = nsb * nsb * n_taps;
  const dim3 col_grid((nsb * kRow + kColThreads - 1) / kColThreads, a.nb);
  const dim3 sb_grid(nsb * (kRow / kColThreads), a.nb);
  const dim3 cg_grid(a.np / kCgOut, a.nb);
  StreamWsb wsb;
  for (int j = 0; j < kMaxSubbands; ++j) wsb.w[j] = tb.wsb[j];
  hipStream_t s = c.s;
  // forward sweep: S_0 into ck(0), every step, segment starts kept
  a.st = c.ck(0);
  bool ok = wave_input<N2>(a, tb, s);
  for (int st = 0; st < steps && ok; ++st)
    ok = wave_step<N2>(a, tb, p->d_cpad, st, n_taps, tap_pad, c.S(st), c.work(), c.TH(st), c.S(st + 1), s);
  // adjoint of the output stage, into G = dL/dS_steps
  a.st = c.G();
  st_adj_tail_kernel<N2><<<col_grid, kColThreads, 0, s>>>(a, c.gout);
  ok = ok && ok_launch();
  if (nsb > 1) {
    ok = ok && row<true, false, false>(a, c.G(), c.G(), nullptr, s);
    st_mix_kernel<false><<<dim3(a.np / 256, a.nb), 256, 0, s>>>(c.G(), tb.poly_tw, wsb, nsb, a.np, nullptr);
    ok = ok && ok_launch();
    ok = ok && gvd_adj<false, true, true, true>(c, a, c.S(steps), tb.h_last, steps);
  } else {
    ok = ok && gvd_adj<true, true, true, true>(c, a, c.S(steps), tb.h_last, steps);
  }
  // reverse sweep, segment by segment
  for (int seg = c.L.n_ck - 1; seg >= 0 && ok; --seg) {
    const int s0 = seg * k, s1 = s0 + k < steps ? s0 + k : steps;
    if (seg != c.L.n_ck - 1)
      for (int st = s0; st < s1 && ok; ++st)
        ok = wave_step<N2>(a, tb, p->d_cpad, st, n_taps, tap_pad, c.S(st), c.work(), c.TH(st), c.S(st + 1), s);
    for (int st = s1 - 1; st >= s0 && ok; --st) {
      // K g' (row domain, from G) and K v (from the state before the step)
      const dim3 row_grid(nsb * a.n2, a.nb);
      st_kweight_kernel<true, false><<<row_grid, kRowNT, 0, s>>>(c.G(), c.KG(), nullptr, p->d_phase,
                                                                 1.0f / (float)kRow, a.twr, nsb, a.n2, a.np);
      if (st == 0 && nsb > 1)
        st_kweight_kernel<false, true><<<row_grid, kRowNT, 0, s>>>(c.S(st), c.work(), step_filter(tb, st),
                                                                   p->d_phase, 1.0f, a.twr, nsb, a.n2, a.np);
      else
        st_kweight_kernel<true, true><<<row_grid, kRowNT, 0, s>>>(c.S(st), c.work(), step_filter(tb, st),
                                                                  p->d_phase, 1.0f, a.twr, nsb, a.n2, a.np);
      ok = ok && ok_launch();
      st_adj_phase_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(c.G(), c.S(st + 1), c.V(), c.tbar(), a.pb, a.tw2,
                                                              nsb);
      ok = ok && ok_launch();
      // p_bar = C^T applied to theta_bar (transposed, tap-reversed rows)
      ok = ok && launch_fir(nsb, a.nb, s, c.tbar(), a.th,
                            p->d_ctpad + (size_t)st * per_step / n_taps * tap_pad, a.np, n_taps / 2, tap_pad);
      ok = ok && ok_launch();
      ok = ok && launch_cgrad(nsb, cg_grid, s, c.tbar(), a.pb, c.cpart(), a.np, n_taps);
      ok = ok && ok_launch();
      st_sum_rows_kernel<<<dim3((per_step + kAccJ - 1) / kAccJ, kAccC), kAccJ * kAccG, 0, s>>>(
          c.cpart(), (int)(cg_grid.x * cg_grid.y), per_step, c.csum());
      st_add_chunks_kernel<<<(per_step + 255) / 256, 256, 0, s>>>(c.csum(), per_step,
                                                                  c.acc_c() + (size_t)st * per_step);
      ok = ok && ok_launch();
      st_adj_comm_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(c.G(), c.V(), c.KG(), c.work(), c.TH(st), a.th,
                                                             a.tw2, nsb, c.rpart());
      st_acc_sum_kernel<<<1, 256, 0, s>>>(c.rpart(), (int)(sb_grid.x * sb_grid.y), c.acc_t() + steps + 1);
      st_col_forward_kernel<N2><<<sb_grid, kColThreads, 0, s>>>(c.V(), c.G(), a.tw2, nsb);
      ok = ok && ok_launch();
      if (st > 0) {
        if (c.want_gvd)
          ok = ok && gvd_adj<true, true, true, true>(c, a, c.S(st), step_filter(tb, st), st);
        else
          ok = ok && row<true, true, true, true>(a, c.G(), c.G(), step_filter(tb, st), s);
      } else if (nsb > 1) {
        ok = ok && gvd_adj<true, false, true, false>(c, a, c.S(0), tb.h_first, 0);
      } else {
        ok = ok && gvd_adj<true, true, true, true>(c, a, c.S(0), tb.h_first, 0);
      }
    }
  }
  // adjoint of the input stage: block input cotangents
  if (c.want_gin && ok) {
    if (nsb > 1) {
      st_mix_kernel<true><<<dim3(a.np / 256, a.nb), 256, 0, s>>>(c.G(), tb.poly_tw, wsb, nsb, a.np, nullptr);
      ok = ok_launch() && row<false, false, true>(a, c.G(), c.G(), nullptr, s);
    }
    st_adj_head_kernel<N2><<<col_grid, kColThreads, 0, s>>>(a, c.gin());
    ok = ok && ok_launch();
  }
  return ok ? CBESSFM_OK : CBESSFM_EHIP;
}

}  // namespace

int launch_stream_backward(cbessfm_plan_t* p, const void* field_in, const void* grad_out, void* grad_in,
                           float* grad_c, float* grad_rho, double* grad_gvd, long long T, int batch, int ck_every,
                           void* workspace, size_t ws_bytes, hipStream_t s) {
  if (p->nlpr != CBESSFM_NLPR_AVERAGED) return CBESSFM_EUNSUPPORTED;
  StreamBwdCall c;
  c.p = p;
  fill_tables(p, c.tb);
  c.L = stream_bwd_layout(p, T, batch, ck_every, grad_in != nullptr);
  if (ws_bytes < c.L.bytes) return CBESSFM_EWORKSPACE;
  c.ws = static_cast<char*>(workspace);
  c.gout = static_cast<const float2*>(grad_out);
  c.want_gvd = grad_gvd != nullptr;
  c.want_gin = grad_in != nullptr;
  c.s = s;
  const int n_c = p->steps * p->sb.n_sb * p->sb.n_sb * p->n_taps;
  st_zero_kernel<<<(n_c + 255) / 256, 256, 0, s>>>(c.acc_c(), n_c);
  st_zero_kernel<<<(p->steps + 2 + 255) / 256, 256, 0, s>>>(c.acc_t(), p->steps + 2);
  if (!ok_launch()) return CBESSFM_EHIP;
  StreamArgs a;
  fill_stream_args(p, field_in, nullptr, T, a);
  const int items = batch * a.nblk;
  for (int item0 = 0; item0 < items; item0 += p->st_blocks) {
    a.item0 = item0;
    a.nb = items - item0 < p->st_blocks ? items - item0 : p->st_blocks;
    int rc;
    switch (p->log_np) {
      case 14: rc = bwd_wave<4>(c, a); break;
      case 15: rc = bwd_wave<8>(c, a); break;
      case 16: rc = bwd_wave<16>(c, a); break;
      case 17: rc = bwd_wave<32>(c, a); break;
      default: rc = CBESSFM_EUNSUPPORTED;
    }
    if (rc) return rc;
  }
  const int n_fin = n_c > p->steps + 1 ? n_c : p->steps + 1;
  st_bwd_finish_kernel<<<(n_fin + 255) / 256, 256, 0, s>>>(c.acc_c(), n_c, c.acc_t(), p->steps, p->step_km, grad_c,
                                                           grad_rho, grad_gvd);
  if (!ok_launch()) return CBESSFM_EHIP;
  if (grad_in != nullptr)
    return launch_gather_gin(c.gin(), static_cast<float2*>(grad_in), T, p->N, p->hop, p->sb.overlap, a.nblk, batch,
                             p->sb.boundary, s);
  return CBESSFM_OK;
}

}  // namespace cbessfm
