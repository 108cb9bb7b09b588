// Internal plan layout and kernel-argument blocks shared by the host code and
// the HIP kernels of libcbessfm.  Nothing here crosses the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cbessfm.h"

namespace cbessfm {

constexpr int kMaxSubbands = 8;
constexpr int kTapChunk = 8;          // FIR taps are processed in chunks of 8
constexpr int kMaxTaps = 255;
constexpr int kXcds = 8;              // MI355X: 8 accelerator complex dies, round-robin dispatch

// Device tables of one plan (all FP32 values are FP64 results rounded once).
struct Tables {
  const float2* h_first;  // [N] exp(+j phi (1 - rho) L) / N,  phi = 2 pi^2 beta2 f^2, subband order
  const float2* h_mid;    // [N] exp(+j phi L) / N'
  const float2* h_last;   // [N] exp(+j phi rho L) / N'
  int h_stride;           // 0: every middle step uses h_mid; N: step s (1-based, >= 2) uses h_mid + (s - 2) N
  const float2* tw;       // [N'] exp(-j 2 pi n / N')
  const float2* poly_tw;  // [n_sb][N'] exp(-j 2 pi i k / N)
  const float* cpad;      // [steps][n_sb][n_sb][tap_pad] applied coefficients, zero padded
  const float* cdpad;     // the same with a zero diagonal, divided by 3 (dual-polarisation NLPR)
  const float2* chat;     // [steps][n_sb][n_sb][N'] DFT of each coefficient row placed circularly
                          // (tap t at position t - Nc mod N'), natural bin order; NULL: time-domain filter
  float2 wsb[kMaxSubbands];  // exp(-j 2 pi a / n_sb)
};

struct XchgCtl {
  unsigned* abort;      // sticky: some exchange wait of this plan gave up
  int* err;             // sticky error code for cbessfm_status()
  unsigned spin_limit;  // polls before a wait gives up
};

// One forward instance: a plan's tables and geometry and the fields it runs on.
struct Inst {
  const float2* in;   // [batch][2][T]
  float2* out;        // [batch][2][T]
  int T;
  int nblk;           // overlap-and-save blocks per batch entry
  int n_sb, steps, n_chunks, nc, n_ov, hop, boundary;
  Tables tab;
};

// Exchange rounds of one forward block: input DEMUX (two, one per
// polarisation), per_step per step, output MUX (two).
__host__ __device__ inline unsigned fwd_rounds(int steps, unsigned per_step) {
  return (unsigned)steps * per_step + 4u;
}

// Everything a single-plan forward launch needs.
struct FwdArgs {
  Inst inst;
  int n_items;        // batch * blocks per batch entry
  int n_teams;        // persistent teams of n_sb workgroups
  unsigned* epoch;    // [teams] exchange rounds completed so far by each team (device)
  uint64_t* xp;       // [team_capacity][2 slots][n_sb][2 N'] tagged words per member: intensity rows
                      // (N' words; two rows for the dual NLPR), the filter's intensity spectra or one
                      // polarisation's block spectrum (re then im, 2 N' words)
  XchgCtl ctl;
};

// Batched forward: a static schedule of teams of varying width.
struct BatchItem {
  int inst;            // index into the instance table
  int sub;             // batch entry * nblk + block
  unsigned round_off;  // exchange rounds of the team's earlier items in this launch
};
struct BatchTeam {
  int width;           // n_sb of every instance the team runs
  int first, count;    // its items: items[first, first + count)
  unsigned rounds;     // exchange rounds of all its items
  int epoch_slot;      // index into the epoch array
  long long xp_off;    // word offset of its exchange slots
};
struct BatchArgs {
  const Inst* insts;
  const int2* wg;            // per workgroup: (team, member), team < 0 = idle
  const BatchTeam* teams;
  const BatchItem* items;
  unsigned* epoch;
  uint64_t* xp;
  XchgCtl ctl;
};

// Streaming forward of blocks larger than one CU holds (stream.hip): the
// size-N' DFT is split into N1 = kStreamRow columns of N' / N1 samples and
// N' / N1 rows of N1 samples.
constexpr int kStreamRow = 4096;
constexpr int kStreamMinLog = 14;
constexpr int kStreamMaxLog = 17;
constexpr size_t kStreamBudget = size_t(512) << 20;  // bytes of block state a plan keeps
constexpr int kStreamMaxBlocks = 256;

struct StreamWsb {
  float2 w[kMaxSubbands];
};

// One wave of blocks of a streaming forward call.
struct StreamArgs {
  const float2* in;    // [batch][2][T]
  float2* out;         // [batch][2][T]
  int T, nblk;         // sequence length, blocks per batch entry
  int item0, nb;       // first item (batch entry * nblk + block) of the wave, items in it
  int n_sb, np, n2;    // subbands, N', N' / N1
  int n_ov, hop, boundary;
  float2* st;          // [nb][n_sb][2][N'] block state
  float* pb;           // [nb][n_sb][N'] intensities
  float* th;           // [nb][n_sb][N'] filtered phases
  const float2* tw2;   // [N2][N1] exp(-j 2 pi n1 k2 / N')
  const float2* twr;   // [N1] exp(-j 2 pi n / N1)
};

// One block of one streamed batch instance, for the step kernels that take
// every such block of a class of instances (same N', n_sb and taps) in one
// launch: the block's state, intensity and phase arrays and its plan's
// tables.  A launch over a table of these takes blockIdx.y as the entry.
struct StreamBlk {
  float2* st;             // [n_sb][2][N'] block state
  float* pb;              // [n_sb][N'] intensities
  float* th;              // [n_sb][N'] phases
  const float2* h_first;  // dispersion filter of step 0, [n_sb][N'] (permuted order)
  const float2* h_mid;    // of step s >= 1: h_mid + (s - 1) h_stride
  const float2* h_last;   // of the last segment (step -1 below)
  long long h_stride;
  const float* cpad;      // [steps][n_sb][n_sb][tap_pad] zero-padded coefficients
  const float2* tw2;      // column twiddles
  const float2* twr;      // row twiddles
  const float2* poly;     // [n_sb][N'] polyphase twiddles of the DEMUX / MUX
  const float2* in;       // the block's batch entry of the input [2][T]
  float2* out;            // and of the output
  int T, blk, hop, n_ov, boundary;  // length, block index in the entry, framing
};

// Workspace layout of one streaming adjoint call (stream.hip): byte offsets
// of its arrays; k steps per checkpoint segment, n_ck segments, waves of nb
// blocks, `state` complex words per block state.
struct StreamBwdLayout {
  int k, n_ck, nblk, nb;
  size_t state;
  size_t ck_off, slot_off, work_off, g_off, v_off, kg_off, theta_off, tbar_off, cpart_off, rpart_off, accc_off, acct_off,
      csum_off, gin_off, bytes;
};

// Everything an adjoint launch needs.
struct BwdArgs {
  const float2* in;    // [batch][2][T] forward input
  const float2* gout;  // [batch][2][T] cotangent of the forward output
  int T, n_items, nblk;
  int n_sb, steps, n_chunks, nc, n_taps, n_ov, hop, boundary;
  int n_teams;
  int ck_every, n_ck;  // segments of ck_every steps, n_ck of them
  unsigned rounds_per_item;
  unsigned* epoch;     // [teams] exchange rounds completed so far by each team (device)
  Tables tab;
  const float* ctpad;   // [steps][n_sb][n_sb][tap_pad]: ctpad[s][l][i][t] = C[s][i][l][n_taps - 1 - t]
  const double* phase;  // [N] 2 pi^2 beta2 f^2 per km, subband order
  double L;             // step length, km
  uint64_t* xspec;
  uint64_t* xp;         // tagged intensity rows
  uint64_t* xq;         // tagged theta_bar rows, [team_capacity][2][n_sb][N']
  float2* spec;         // [n_teams][n_ck][n_sb][2][N'] spectrum at each segment start
  float* vtheta;        // [n_teams][ck_every][n_sb][13 N'] (v_x, v_y, theta, A, D) of a segment's steps
  float2* gsave;        // [n_teams][n_sb][2 N'] the incoming g_S of the reverse step
  float* cpart;         // [n_items][steps][n_sb][n_sb][n_taps]
  double* rpart;        // [n_items][n_sb]
  double* lpart;        // [n_items][n_sb][steps + 1] dispersion-segment partials, or null
  float2* gin_blk;      // [n_items][2][N] or null
  XchgCtl ctl;
};

// Workspace layout of one adjoint call.
struct BwdLayout {
  int k, n_ck, nblk, n_items, n_teams;
  size_t spec_off, vtheta_off, gsave_off, cpart_off, rpart_off, lpart_off, gin_off, bytes;
};

}  // namespace cbessfm

// Default bound of an exchange wait: 2^22 polls about 64 cycles apart
// (about 0.1 s), far beyond any wait of a healthy launch.
constexpr unsigned kDefaultWaitLimit = 1u << 22;

struct cbessfm_plan {
  cbessfm_link link;
  cbessfm_subbands sb;
  int steps;
  int n_taps, tap_pad, n_chunks;
  int N, Np, hop, log_np;
  double step_km, rho;
  int device;
  int cu_count;
  int threads;
  int team_capacity;      // forward teams whose workgroups can all be resident at once
  int team_capacity_dual; // the same for the dual-polarisation forward kernel
  int nlpr;               // CBESSFM_NLPR_AVERAGED or CBESSFM_NLPR_DUAL_POL
  int gvd_explicit;       // 1: dispersion segment lengths from d_len, else (1 - rho) L, L, ..., rho L
  int bwd_team_capacity;  // the same for the adjoint kernel
  int fir_freq;           // 1: the forward evaluates the coupled filter in the frequency domain
  int xchg_teams;         // teams the exchange buffers are sized for
  unsigned wait_limit;    // polls before an exchange wait gives up (cbessfm_set_wait_limit)
  // device memory
  double* d_phase;    // [N] 2 pi^2 beta2 f^2 per km, subband order (FP64); streaming plans keep
                      // each subband's N' entries in the permuted order of stream.hip
  float2* d_h;        // [3][N] (same order as d_phase)
  float2* d_tw;       // [N'] exp(-j 2 pi n / N'); streaming plans: [N2][N1] column twiddles, then [N1]
  float2* d_poly;     // [n_sb][N'] (streaming plans: permuted order)
  float* d_c;         // [steps][n_sb][n_sb][n_taps] as given
  float* d_cpad;      // padded copy used by the kernels
  float* d_ctpad;     // transposed, tap-reversed padded copy (adjoint)
  float* d_cdpad;     // padded copy with zero diagonal, / 3 (dual-polarisation NLPR)
  float2* d_chat;     // [steps][n_sb][n_sb][N'] row DFTs (frequency-domain filter only)
  double* d_rho;      // current split ratio
  double* d_len;      // [steps + 1] explicit dispersion segment lengths, km
  uint64_t* d_xspec;  // tagged exchange words
  uint64_t* d_xp;
  uint64_t* d_xq;
  unsigned* d_epoch;  // [xchg_teams] exchange rounds completed per team
  unsigned* d_abort;  // sticky exchange-timeout word
  int* d_err;
  float2 wsb[cbessfm::kMaxSubbands];
  // streaming forward (N' > 8192): block state of st_blocks blocks
  int stream;
  int st_blocks;
  float2* d_st;
  float* d_pb;
  float* d_th;
};

namespace cbessfm {
// forward.hip
int launch_forward(cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, hipStream_t s);
int launch_tables(cbessfm_plan_t* p, hipStream_t s);
int launch_pad_coeffs(cbessfm_plan_t* p, const float* src, hipStream_t s);
int launch_copy_rho(cbessfm_plan_t* p, const float* src, hipStream_t s);
int launch_gvd_tables(cbessfm_plan_t* p, const double* lengths, hipStream_t s);
int occupancy_per_cu(int log_np, bool dual, int* blocks);
int bwd_occupancy_per_cu(int log_np, int* blocks);
void fill_tables(const cbessfm_plan_t* p, Tables& tb);
BwdLayout bwd_layout(const cbessfm_plan_t* p, long long T, int batch, int ck_every);
int launch_backward(cbessfm_plan_t* p, const void* field_in, const void* grad_out, void* grad_in, float* grad_c,
                    float* grad_rho, double* grad_gvd, long long T, int batch, int ck_every, void* workspace,
                    size_t ws_bytes, hipStream_t s);
int threads_for(int log_np);
bool stream_capturing(hipStream_t s);
int batch_occupancy_per_cu(int log_np, int* blocks);
int launch_batch(int log_np, const BatchArgs& a, int grid, hipStream_t s);
void fill_inst(const cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, Inst& d);
// stream.hip
int launch_stream_forward(cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, hipStream_t s);
// A streaming forward whose blocks fit one wave (batch instances), over a
// table of blocks of any number of instances of one class (same N', n_sb and
// taps): block input, one step, block output.  p0: any plan of the class
// (for N', n_sb and the DEMUX weights).
int stream_single_wave(const cbessfm_plan_t* p, long long T, int batch);
void stream_blocks(const cbessfm_plan_t* p, const void* in, void* out, long long T, int batch, StreamBlk* out_blk);
int stream_class_input(const cbessfm_plan_t* p0, const StreamBlk* d_blks, int nb, hipStream_t s);
int stream_class_step(int log_np, int n_sb, int n_taps, int tap_pad, int step, const StreamBlk* d_blks, int nb,
                      hipStream_t s);
int stream_class_output(const cbessfm_plan_t* p0, const StreamBlk* d_blks, int nb, hipStream_t s);
// Kernel launches of one wave of a streaming forward with `steps` steps (0:
// its block input and output only).
int stream_launches(const cbessfm_plan_t* p, int steps);
StreamBwdLayout stream_bwd_layout(const cbessfm_plan_t* p, long long T, int batch, int ck_every, bool gin);
int launch_stream_backward(cbessfm_plan_t* p, const void* field_in, const void* grad_out, void* grad_in,
                           float* grad_c, float* grad_rho, double* grad_gvd, long long T, int batch, int ck_every,
                           void* workspace, size_t ws_bytes, hipStream_t s);
// backward.hip: device address of the fixed scratch array on `device` (which
// must be current), looked up once per device and kept.
int static_scratch(int device, void** ptr);
// backward.hip: grad_in[inst][pol][pos] = sum of the block input cotangents
// blk_g[inst nblk + b][pol][n] of every block position that reads pos.
int launch_gather_gin(const float2* blk_g, float2* gin, long long T, int N, int hop, int n_ov, int nblk, int batch,
                      int boundary, hipStream_t s);
}  // namespace cbessfm
