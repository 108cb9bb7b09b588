// Register-resident radix-16/8/4/2 complex FP32 FFT of one subband block, with
// LDS used only to exchange data between Stockham passes.
//
// Layout contract (the whole kernel is built around it): a workgroup of NT
// threads handles an N-point transform; thread t owns the RR = N / NT
// samples at positions t + NT * o, o in [0, RR), both on input and output.
// The first pass reads its butterfly inputs straight from those registers and
// the last pass leaves its outputs in them, so pointwise work before and
// after a transform (GVD filter, intensity, rotation) never touches LDS.
#pragma once

#include <hip/hip_runtime.h>

namespace cbessfm {

// ---------------------------------------------------------------- complex ops
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// a * (-j) for the forward transform, a * (+j) for the inverse
template <bool INV>
__device__ __forceinline__ float2 mul_mj(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
template <bool INV>
__device__ __forceinline__ float2 twmul(float2 a, float2 w) {  // a * w (fwd) or a * conj(w) (inv)
  return INV ? cmulc(a, w) : cmul(a, w);
}

// cos / sin of 2 pi k / 16 split into an FP32 leading part and an FP32
// remainder.  Every leading pair has |w| slightly below 1; since every
// butterfly reuses the same constants, that shortfall would compound into a
// systematic loss of amplitude over the many transforms of a step loop, so
// the products below add the remainder term with an FMA.
__host__ __device__ constexpr float cos16(int k) {
  constexpr float c[16] = {1.0f, 0.92387950420379638671875f, 0.707106769084930419921875f,
                           0.3826834261417388916015625f, 0.0f, -0.3826834261417388916015625f,
                           -0.707106769084930419921875f, -0.92387950420379638671875f, -1.0f,
                           -0.92387950420379638671875f, -0.707106769084930419921875f,
                           -0.3826834261417388916015625f, 0.0f, 0.3826834261417388916015625f,
                           0.707106769084930419921875f, 0.92387950420379638671875f};
  return c[k & 15];
}
__host__ __device__ constexpr float cos16_lo(int k) {
  constexpr float c[16] = {0.0f, 2.830748968563057e-08f, 1.2101617485882343e-08f, 6.2233507236442165e-09f,
                           0.0f, -6.2233507236442165e-09f, -1.2101617485882343e-08f, -2.830748968563057e-08f,
                           0.0f, -2.830748968563057e-08f, -1.2101617485882343e-08f, -6.2233507236442165e-09f,
                           0.0f, 6.2233507236442165e-09f, 1.2101617485882343e-08f, 2.830748968563057e-08f};
  return c[k & 15];
}
__host__ __device__ constexpr float sin16(int k) { return cos16(k + 12); }
__host__ __device__ constexpr float sin16_lo(int k) { return cos16_lo(k + 12); }

// a * exp(-+ j 2 pi K / 16): '-' forward, '+' inverse
template <int K, bool INV>
__device__ __forceinline__ float2 w16(float2 a) {
  constexpr int k = K & 15;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (k == 4) {
    return mul_mj<INV>(a);
  } else if constexpr (k == 8) {
    return make_float2(-a.x, -a.y);
  } else if constexpr (k == 12) {
    return mul_mj<!INV>(a);
  } else {
    constexpr float c = cos16(k), s = sin16(k), cl = cos16_lo(k), sl = sin16_lo(k);
    // forward: (x c + y s, y c - x s); inverse: (x c - y s, y c + x s)
    const float ss = INV ? -s : s, ssl = INV ? -sl : sl;
    const float re_lo = fmaf(a.x, cl, a.y * ssl);
    const float im_lo = fmaf(a.y, cl, -a.x * ssl);
    return make_float2(fmaf(a.x, c, fmaf(a.y, ss, re_lo)), fmaf(a.y, c, fmaf(-a.x, ss, im_lo)));
  }
}

// ------------------------------------------------------------- small DFTs
template <bool INV>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
  float2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = mul_mj<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// 8-point DFT, natural order in and out (n = 2 n1 + n2, k = k1 + 4 k2)
template <bool INV>
__device__ __forceinline__ void dft8(float2 (&v)[8]) {
  dft4<INV>(v[0], v[2], v[4], v[6]);
  dft4<INV>(v[1], v[3], v[5], v[7]);
  v[3] = w16<2, INV>(v[3]);
  v[5] = w16<4, INV>(v[5]);
  v[7] = w16<6, INV>(v[7]);
  dft2<INV>(v[0], v[1]);
  dft2<INV>(v[2], v[3]);
  dft2<INV>(v[4], v[5]);
  dft2<INV>(v[6], v[7]);
  // v[2 k1 + k2] = X[k1 + 4 k2]
  float2 o[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    o[k1] = v[2 * k1];
    o[k1 + 4] = v[2 * k1 + 1];
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = o[i];
}

// 16-point DFT, natural order in and out (n = 4 n1 + n2, k = k1 + 4 k2)
template <bool INV>
__device__ __forceinline__ void dft16(float2 (&v)[16]) {
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<INV>(v[n2], v[4 + n2], v[8 + n2], v[12 + n2]);
  // v[4 k1 + n2] = A_n2[k1]; multiply by W16^(n2 k1)
  v[5] = w16<1, INV>(v[5]);
  v[6] = w16<2, INV>(v[6]);
  v[7] = w16<3, INV>(v[7]);
  v[9] = w16<2, INV>(v[9]);
  v[10] = w16<4, INV>(v[10]);
  v[11] = w16<6, INV>(v[11]);
  v[13] = w16<3, INV>(v[13]);
  v[14] = w16<6, INV>(v[14]);
  v[15] = w16<9, INV>(v[15]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // v[4 k1 + k2] = X[k1 + 4 k2]
  float2 o[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) o[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <int R, bool INV>
__device__ __forceinline__ void dft(float2 (&v)[R]) {
  if constexpr (R == 2) {
    dft2<INV>(v[0], v[1]);
  } else if constexpr (R == 4) {
    dft4<INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    dft8<INV>(v);
  } else {
    static_assert(R == 16, "radix");
    dft16<INV>(v);
  }
}

// ------------------------------------------------------------- plan (constexpr)
// LDS placement of entry i of an N-point FFT exchange buffer (entries of 16
// bytes), chosen per N by measurement (every placement gives the same bits):
// at N = 2048 and 4096 an XOR swizzle within groups of 16 entries (bits 0-3
// of i with bits 4-7), no padding; at 8192 one entry of padding after every
// 16; below 2048 one after every 8, which keeps the 8 lanes served together
// on distinct banks for consecutive positions and for the stride-R writes
// of the first pass.  Forward times against one entry after every 8
// everywhere: 0.315 against 0.319 ms at N' = 4096 (5 subbands), 0.595
// against 0.601 ms at 8192; at 1024 the swizzle made the adjoint of the
// gradient workload 2.7% slower.
template <int N>
__device__ __forceinline__ int pad_c(int i) {
  if constexpr (N == 2048 || N == 4096)
    return i ^ ((i >> 4) & 15);
  else if constexpr (N == 8192)
    return i + (i >> 4);
  else
    return i + (i >> 3);
}
template <int N>
__host__ __device__ constexpr int pad_c_size() {
  return (N == 2048 || N == 4096) ? N : N == 8192 ? N + (N >> 4) + 1 : N + (N >> 3) + 1;
}
__device__ __forceinline__ int pad_f(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int pad_f_size(int n) { return n + (n >> 4) + 1; }

// Samples per thread per polarisation of the persistent kernels.
__host__ __device__ constexpr int default_rr(int n) { return n >= 8192 ? 16 : (n >= 512 ? 8 : n / 64); }

// Shape of an N-point transform over N / RR threads, RR samples each.
template <int N, int RRX = default_rr(N)>
struct FftShape {
  static_assert(N >= 256 && N <= 8192 && (N & (N - 1)) == 0, "N' must be a power of two in [256, 8192]");
  static_assert((RRX == 4 || RRX == 8 || RRX == 16) && N / RRX <= 1024, "samples per thread");
  static constexpr int SIZE = N;
  static constexpr int RR = RRX;   // samples per thread per polarisation
  static constexpr int NT = N / RR;  // threads per workgroup
  static constexpr int radix(int p) {
    int rem = N;
    for (int q = 0; q < p; ++q) rem /= (rem < RR ? rem : RR);
    return rem < RR ? rem : RR;
  }
  static constexpr int stride(int p) {  // L_p = product of the radices before pass p
    int l = 1;
    for (int q = 0; q < p; ++q) l *= radix(q);
    return l;
  }
  static constexpr int passes() {
    int p = 0, rem = N;
    while (rem > 1) {
      rem /= (rem < RR ? rem : RR);
      ++p;
    }
    return p;
  }
  static constexpr int LDS_C = pad_c_size<N>();  // float2 entries per polarisation (float4 entries in all)
  // Two exchange buffers (passes alternate between them, so a pass needs no
  // barrier between its reads and its writes) where they fit the LDS beside
  // one workgroup's other use: N' <= 4096 (2 x 64 KB at 4096).
  static constexpr bool DB = N <= 4096;
  static constexpr int LDS_ENTRIES = DB ? 2 * LDS_C : LDS_C;  // float4 entries of the exchange
};

// Twiddle registers of pass P: NB butterflies x (R - 1) factors (one dummy
// for passes without twiddles).
template <class S, int P>
struct PassTw {
  static constexpr int R = S::radix(P);
  static constexpr int NB = S::RR / R;
  static constexpr int C = (P == 0 || P >= S::passes() || R < 2) ? 1 : NB * (R - 1);
};
template <class S, int P>
using PassTwRegs = float2[PassTw<S, P>::C];

// Loads the twiddles W_{L R}^{k m} = table[k m N / (L R)], k = j mod L, of
// pass P.  They depend only on the thread, so they are issued one pass ahead.
template <class S, int P>
__device__ __forceinline__ void load_pass_tw(PassTwRegs<S, P>& w, const float2* __restrict__ twt, int t) {
  constexpr int N = S::SIZE;
  if constexpr (P > 0 && P < S::passes()) {
    constexpr int R = S::radix(P);
    constexpr int L = S::stride(P);
    constexpr int NB = S::RR / R;
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      const int k = (t + S::NT * a) % L;
#pragma unroll
      for (int m = 1; m < R; ++m) w[a * (R - 1) + m - 1] = twt[(k * m * (N / (L * R))) % N];
    }
  }
}

// One Stockham pass p of radix R over both polarisations.  The exchange
// buffer holds (x.re, x.im, y.re, y.im) per position, so each value moves
// through LDS with one 128-bit access.
//   FIRST: inputs come from the owned registers (positions t + NT o)
//   LAST : outputs go to the owned registers
// Otherwise inputs are read from / outputs written to LDS.  With DB, pass p
// writes buffer p mod 2 and reads buffer (p - 1) mod 2: every reader of the
// buffer a pass writes has passed the barrier that ended the previous pass.
template <class S, int P, bool INV, bool DB>
__device__ __forceinline__ void fft_pass(float2 (&x)[S::RR], float2 (&y)[S::RR], float4* __restrict__ lxy,
                                         const PassTwRegs<S, P>& w, int t) {
  constexpr int N = S::SIZE;
  const float4* rd = DB ? lxy + ((P + 1) & 1) * S::LDS_C : lxy;
  float4* wr = DB ? lxy + (P & 1) * S::LDS_C : lxy;
  constexpr int R = S::radix(P);
  constexpr int L = S::stride(P);
  constexpr int NB = S::RR / R;           // butterflies per thread
  constexpr bool FIRST = (P == 0);
  constexpr bool LAST = (P == S::passes() - 1);
  constexpr int NR = N / R;
  // gather inputs: vx[a][m] = x[j + m N/R], j = t + NT a
  float2 vx[NB][R], vy[NB][R];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if constexpr (FIRST) {
        vx[a][m] = x[a + m * NB];
        vy[a][m] = y[a + m * NB];
      } else {
        const float4 v = rd[pad_c<S::SIZE>(t + S::NT * a + m * NR)];
        vx[a][m] = make_float2(v.x, v.y);
        vy[a][m] = make_float2(v.z, v.w);
      }
    }
  if constexpr (!DB && !FIRST && !LAST) __syncthreads();  // everyone has read before anyone writes
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    if constexpr (!FIRST) {
#pragma unroll
      for (int m = 1; m < R; ++m) {
        vx[a][m] = twmul<INV>(vx[a][m], w[a * (R - 1) + m - 1]);
        vy[a][m] = twmul<INV>(vy[a][m], w[a * (R - 1) + m - 1]);
      }
    }
    dft<R, INV>(vx[a]);
    dft<R, INV>(vy[a]);
  }
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const int j = t + S::NT * a;
    const int k = j % L;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if constexpr (LAST) {  // j < L here, so the output position is j + m L
        x[a + m * NB] = vx[a][m];
        y[a + m * NB] = vy[a][m];
      } else {
        wr[pad_c<S::SIZE>((j - k) * R + k + m * L)] = make_float4(vx[a][m].x, vx[a][m].y, vy[a][m].x, vy[a][m].y);
      }
    }
  }
  if constexpr (!LAST) __syncthreads();
}

template <class S, int P, bool INV, bool DB>
__device__ __forceinline__ void fft_passes(float2 (&x)[S::RR], float2 (&y)[S::RR], float4* lxy, const float2* twt,
                                           const PassTwRegs<S, P>& w, int t) {
  if constexpr (P < S::passes()) {
    PassTwRegs<S, P + 1> w_next;
    load_pass_tw<S, P + 1>(w_next, twt, t);  // in flight during this pass
    fft_pass<S, P, INV, DB>(x, y, lxy, w, t);
    fft_passes<S, P + 1, INV, DB>(x, y, lxy, twt, w_next, t);
  }
}

// Unnormalised size-N DFT (INV = false: exp(-j...), INV = true: exp(+j...))
// of the two owned register sets; twt[n] = exp(-j 2 pi n / N) (FP64 values
// rounded once, read through the caches one pass ahead of their use).
// Starts with a barrier so that earlier LDS readers are done before the first
// pass overwrites the exchange buffer(s): lxy holds DB ? 2 LDS_C : LDS_C
// float4 entries (FftShape::LDS_ENTRIES); a caller with room for one buffer
// only passes DB = false.  RRX: samples per thread (N / RRX threads).
template <int N, bool INV, bool DB = FftShape<N>::DB, int RRX = default_rr(N)>
__device__ __forceinline__ void fft(float2 (&x)[RRX], float2 (&y)[RRX], float4* lxy, const float2* twt, int t) {
  using S = FftShape<N, RRX>;
  PassTwRegs<S, 0> w0;
  __syncthreads();
  fft_passes<S, 0, INV, DB>(x, y, lxy, twt, w0, t);
}

// ------------------------------------------------------------- one array
// The same Stockham transform of a single owned register set (a real
// intensity or phase row of the frequency-domain coupled filter): identical
// radices, twiddles and layout contract, with two exchange buffers of one
// float2 per position (the space of one float4 buffer), alternated as in
// fft_pass.
template <class S, int P, bool INV>
__device__ __forceinline__ void fft1_pass(float2 (&x)[S::RR], float2* __restrict__ lx, const PassTwRegs<S, P>& w,
                                          int t) {
  constexpr int N = S::SIZE;
  const float2* rd = lx + ((P + 1) & 1) * S::LDS_C;
  float2* wr = lx + (P & 1) * S::LDS_C;
  constexpr int R = S::radix(P);
  constexpr int L = S::stride(P);
  constexpr int NB = S::RR / R;
  constexpr bool FIRST = (P == 0);
  constexpr bool LAST = (P == S::passes() - 1);
  constexpr int NR = N / R;
  float2 vx[NB][R];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if constexpr (FIRST)
        vx[a][m] = x[a + m * NB];
      else
        vx[a][m] = rd[pad_c<S::SIZE>(t + S::NT * a + m * NR)];
    }
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    if constexpr (!FIRST) {
#pragma unroll
      for (int m = 1; m < R; ++m) vx[a][m] = twmul<INV>(vx[a][m], w[a * (R - 1) + m - 1]);
    }
    dft<R, INV>(vx[a]);
  }
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    const int j = t + S::NT * a;
    const int k = j % L;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      if constexpr (LAST)
        x[a + m * NB] = vx[a][m];
      else
        wr[pad_c<S::SIZE>((j - k) * R + k + m * L)] = vx[a][m];
    }
  }
  if constexpr (!LAST) __syncthreads();
}

template <class S, int P, bool INV>
__device__ __forceinline__ void fft1_passes(float2 (&x)[S::RR], float2* lx, const float2* twt,
                                            const PassTwRegs<S, P>& w, int t) {
  if constexpr (P < S::passes()) {
    PassTwRegs<S, P + 1> w_next;
    load_pass_tw<S, P + 1>(w_next, twt, t);
    fft1_pass<S, P, INV>(x, lx, w, t);
    fft1_passes<S, P + 1, INV>(x, lx, twt, w_next, t);
  }
}

// Unnormalised size-N DFT of one owned register set; same conventions as fft.
template <int N, bool INV>
__device__ __forceinline__ void fft1(float2 (&x)[FftShape<N>::RR], float2* lx, const float2* twt, int t) {
  using S = FftShape<N>;
  PassTwRegs<S, 0> w0;
  __syncthreads();
  fft1_passes<S, 0, INV>(x, lx, twt, w0, t);
}

}  // namespace cbessfm
