// Team-level helpers shared by the forward and adjoint kernels: the tagged
// exchange between the workgroups of a team, and the overlap-and-save framing.
//
// Exchange protocol.  Every exchanged float travels in its own 64-bit word
// whose high half is a round tag; words are single-copy atomic, written with
// relaxed workgroup-scope atomic stores and read with relaxed device-scope
// atomic loads.  The members of a team are workgroups with the same blockIdx
// mod 8, which the dispatcher places on one XCD (workgroups go to the XCDs
// round-robin, from a launch-dependent start), so the exchange only has to
// be coherent within that XCD's L2: the stores go through the CU's
// write-through L1 into the L2 and are not written through to memory, and
// the loads miss the L1 and read the L2.  A reader polls a word until it
// carries the tag of the round it needs, so it can never consume stale data,
// and no cache write-back / invalidate fences are needed.  Were the members
// of a team ever on different XCDs, the bounded waits would give up and the
// launch would report CBESSFM_ESYNC; a stale word cannot be mistaken for a
// new one.
//
// Tags come from a per-team round counter kept in device memory (the team's
// "epoch"): a launch reads it once at the start, numbers its rounds after it,
// and member 0 stores the advanced value at the end.  Nothing on the host has
// to number rounds, so a launch recorded in a HIP graph stays correct on every
// replay.  Member 0 finishes only after consuming a round from every member,
// and each member reads the counter before its first write, so the update can
// never be seen by a member of the same launch.
//
// Reuse of a buffer slot is safe when two uses of the same slot are separated
// by at least one other all-to-all round: a member writes round r + 1 only
// after it has consumed round r, so a member that has consumed round r + 1 from
// everybody knows that everybody is done reading round r.  A word therefore
// holds either the tag a reader expects or the tag of an earlier use of that
// slot a few rounds back; tags are compared modulo 2^32, so the counter may
// wrap.  Buffers start zeroed and the first tag of a team is 1, and every slot
// has been written before its team's tags can come back around to 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"
#include "internal.hpp"

namespace cbessfm {

// The thread index, hidden from the optimiser so that index arithmetic derived
// from it is recomputed where it is used instead of being hoisted into
// long-lived registers.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

__device__ __forceinline__ void xput(uint64_t* dst, float v, unsigned tag) {
  const uint64_t w = ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v);
  __hip_atomic_store(dst, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint64_t xload(const uint64_t* src) {
  return __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reads the team's round counter into LDS (one load per workgroup) and
// returns the first tag of this launch.
__device__ __forceinline__ unsigned epoch_begin(const unsigned* epoch, unsigned* lds_word) {
  if (threadIdx.x == 0) *lds_word = __hip_atomic_load(epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return *lds_word + 1u;
}

// Member 0 stores the counter advanced by the rounds of this launch.
__device__ __forceinline__ void epoch_end(unsigned* epoch, unsigned first_tag, unsigned rounds, int me) {
  if (me == 0 && threadIdx.x == 0)
    __hip_atomic_store(epoch, first_tag - 1u + rounds, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Issues the CNT loads row[t + stride * o].
template <int CNT>
__device__ __forceinline__ void xissue(const uint64_t* row, int t, int stride, uint64_t (&w)[CNT]) {
#pragma unroll
  for (int o = 0; o < CNT; ++o) w[o] = xload(row + t + stride * o);
}

// Re-polls every word (straight-line code), keeping the ones that already
// carry `tag`.
template <int O, int CNT>
__device__ __forceinline__ void repoll(const uint64_t* row, int t, int stride, unsigned tag, uint64_t (&w)[CNT]) {
  if constexpr (O < CNT) {
    const uint64_t nw = xload(row + t + stride * O);
    w[O] = ((unsigned)(w[O] >> 32) == tag) ? w[O] : nw;
    repoll<O + 1, CNT>(row, t, stride, tag, w);
  }
}

// Completes reads started with xissue(): re-polls the words that do not yet
// carry `tag` until all do, then returns the payloads.  Bounded: on timeout
// the sticky abort word and the error flag are set and every later wait falls
// through (results are then invalid until cbessfm_status() clears the flag).
template <int CNT>
__device__ __forceinline__ void xcomplete(const uint64_t* row, int t, int stride, unsigned tag, const XchgCtl& c,
                                          uint64_t (&w)[CNT], float (&v)[CNT]) {
  unsigned n = 0;
  while (true) {
    unsigned bad = 0u;
#pragma unroll
    for (int o = 0; o < CNT; ++o) bad |= (unsigned)(w[o] >> 32) ^ tag;
    if (bad == 0u) break;
    if (__hip_atomic_load(c.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
    if (++n > c.spin_limit) {
      __hip_atomic_store(c.abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(c.err, (int)CBESSFM_ESYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
    repoll<0, CNT>(row, t, stride, tag, w);
  }
#pragma unroll
  for (int o = 0; o < CNT; ++o) v[o] = __uint_as_float((unsigned)w[o]);
}

// Reads the CNT words row[t + stride * o] of round `tag`.
template <int CNT>
__device__ __forceinline__ void xget(const uint64_t* row, int t, int stride, unsigned tag, const XchgCtl& c,
                                     float (&v)[CNT]) {
  uint64_t w[CNT];
  xissue<CNT>(row, t, stride, w);
  xcomplete<CNT>(row, t, stride, tag, c, w, v);
}

// Position in [0, T) of block sample n, or -1 for a zero.  `first` is the
// position of sample 0: reduced mod T for the circular boundary (a single
// subtraction then wraps unless the sequence is shorter than the block), raw
// for the zero boundary.
__device__ __forceinline__ int frame_pos(int first, int n, int T, int boundary, bool short_seq) {
  const int pos = first + n;
  if (boundary == 0) {
    if (short_seq) return pos % T;
    return pos >= T ? pos - T : pos;
  }
  return (pos < 0 || pos >= T) ? -1 : pos;
}

__device__ __forceinline__ int frame_first(int blk, int hop, int n_ov, int T, int boundary) {
  int first = blk * hop - n_ov / 2;
  if (boundary == 0) first = ((first % T) + T) % T;
  return first;
}

// LDS of the nonlinear stage (aliases the FFT exchange buffers): two rows of
// circularly extended intensities, one row of phases and the per-wave tap
// sums of the coefficient gradient, in floats.  Rows use the layout pad_r:
// four floats of padding after every 32, so aligned groups of four stay
// contiguous (128-bit reads) and lanes reading 4, 8 or 16 floats apart fall
// on different banks.
__device__ __forceinline__ int pad_r(int i) { return i + ((i >> 5) << 2); }
__host__ __device__ constexpr int pad_r_size(int n) { return ((n + ((n >> 5) << 2) + 8) + 3) & ~3; }

template <int N>
struct NlprLds {
  static constexpr int PB = pad_r_size(N + kMaxTaps + 3 * kTapChunk + FftShape<N>::RR);
  static constexpr int TH = pad_r_size(N);
  static constexpr int RED = (kMaxTaps + 1) * (FftShape<N>::NT / 64);  // per-wave tap sums (adjoint)
  static constexpr int FLOATS = 2 * PB + TH + RED;
};
template <int N>
constexpr int lds_floats() {
  return 4 * FftShape<N>::LDS_ENTRIES > NlprLds<N>::FLOATS ? 4 * FftShape<N>::LDS_ENTRIES : NlprLds<N>::FLOATS;
}

// Writes values held at positions t + NT o (o < RR; t may include an offset
// of whole NT RR' groups) into a circularly extended LDS row:
// row[pad_r(k + hl)] = v[k], plus the wrapped copies for the left halo (hl
// samples) and the right halo (hr samples).
template <int N, int RR, int NT>
__device__ __forceinline__ void stage_row(float* row, const float (&v)[RR], int t, int hl, int hr) {
#pragma unroll
  for (int o = 0; o < RR; ++o) row[pad_r(t + NT * o + hl)] = v[o];
  if constexpr (NT >= 256) {
    // halos are shorter than NT (both at most 255), so only the last value
    // can fall in the left one and only the first in the right one
    const int k_last = t + NT * (RR - 1);
    if (k_last >= N - hl) row[pad_r(k_last - N + hl)] = v[RR - 1];
    if (t < hr) row[pad_r(t + N + hl)] = v[0];
  } else {
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      const int k = t + NT * o;
      if (k >= N - hl) row[pad_r(k - N + hl)] = v[o];
      if (k < hr) row[pad_r(k + N + hl)] = v[o];
    }
  }
}

// CNT (a multiple of 4) consecutive floats of a pad_r row from index `start`
// (a multiple of 4) into w[OFF ..), by 128-bit reads.
template <int CNT, int OFF, int W>
__device__ __forceinline__ void load_row4(const float* row, int start, float (&w)[W]) {
  static_assert(CNT % 4 == 0 && OFF + CNT <= W, "window");
#pragma unroll
  for (int i = 0; i < CNT; i += 4) {
    const float4 v = *reinterpret_cast<const float4*>(row + pad_r(start + i));
    w[OFF + i] = v.x;
    w[OFF + i + 1] = v.y;
    w[OFF + i + 2] = v.z;
    w[OFF + i + 3] = v.w;
  }
}

}  // namespace cbessfm
