/*
 * cbessfm.h -- C ABI of the MI355X (gfx950) coupled-band enhanced split-step
 * Fourier method (CB-ESSFM) digital backpropagation library.
 *
 * The operation (Sec. III-A and III-C of Civelli, Jana, Forestieri, Secondini,
 * "A New Twist on Low-Complexity Digital Backpropagation"):
 *
 *   A dual-polarisation field sampled at rate R is cut into overlap-and-save
 *   blocks of N = N_sb * N' samples with N_ov samples of overlap.  Each block is
 *   transformed (two size-N DFTs), split into N_sb contiguous subbands of N'
 *   bins, and then goes through N_st steps of
 *       GVD compensation  h = exp(+j 2 pi^2 beta2 dz f^2)       (Sec. III-A)
 *       size-N' inverse DFT per subband and polarisation
 *       intensity p_i = |x_i|^2 + |y_i|^2                       (Sec. II-C)
 *       theta_i[k] = sum_l sum_m C_s[i][l][m] p_l[(k - m) mod N']  (eq. (15))
 *       rotation x_i, y_i *= exp(-j theta_i)                    (eq. (3))
 *       size-N' forward DFT
 *   with dz = (1 - rho) L in the first step and L afterwards, a final GVD of
 *   rho L (Sec. III-C), recombination and two inverse size-N DFTs.  Samples
 *   [N_ov/2, N - N_ov/2) of every block are kept.
 *
 *   Subband i holds the bins q_i + delta, q_i = -N/2 + i N' + N'/2,
 *   delta in [-N'/2, N'/2) (equal contiguous partition of the sampled band);
 *   its time samples are the lowpass-equivalent samples of App. B at rate
 *   R / N_sb.  The coefficient tensor C is the *applied* one: it already holds
 *   the 3/2 cross-band factor of eq. (15) and the backpropagation sign.
 *
 * Conventions for every entry point:
 *   - Return 0 on success or a negative CBESSFM_E* code.  Nothing prints,
 *     throws or aborts across this boundary.
 *   - "device" pointers are HIP device allocations owned by the caller;
 *     "host" pointers are ordinary host memory owned by the caller.
 *   - Fields are interleaved complex float32 (re, im), laid out
 *     [batch][2 polarisations][T], in sqrt(W).
 *   - stream is a hipStream_t passed as void* (NULL = default stream).  run
 *     and backward are asynchronous on that stream and allocate nothing.
 *   - A plan may be used by one stream at a time; calls that overlap on one
 *     plan race on its exchange buffers.
 *   - run and backward keep no host-side state between calls (the exchange
 *     round counters live in device memory), so they may be recorded in a HIP
 *     graph and replayed.
 */
#ifndef CBESSFM_H
#define CBESSFM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CBESSFM_OK = 0,
  CBESSFM_EINVAL = -1,      /* an argument is out of its documented range */
  CBESSFM_EUNSUPPORTED = -2,/* a size this build does not implement */
  CBESSFM_ENOMEM = -3,      /* device or host allocation failed */
  CBESSFM_EHIP = -4,        /* a HIP runtime call failed */
  CBESSFM_ESYNC = -5,       /* a device-side exchange wait gave up */
  CBESSFM_EWORKSPACE = -6   /* caller workspace too small */
};

/* Fibre link (Sec. IV-A): span_km * n_spans is the backpropagated length. */
typedef struct {
  double alpha_db_km;    /* attenuation, dB/km (analytic coefficients only) */
  double beta2_ps2_km;   /* dispersion beta2, ps^2/km (negative for SMF) */
  double gamma_w_km;     /* Kerr coefficient, 1/(W km) (analytic coefficients) */
  double span_km;        /* amplifier spacing, km */
  int32_t n_spans;       /* number of spans, >= 1 */
  double sample_rate_hz; /* full-field sampling rate R, Hz, > 0 */
  int32_t manakov_8_9;   /* nonzero: scale gamma by 8/9 in analytic coefficients */
} cbessfm_link;

/* Block and subband layout (Sec. III-A). */
typedef struct {
  int32_t n_sb;      /* N_sb, 1..8 */
  int32_t block_sb;  /* N' = N / N_sb, power of two in [256, 8192] (one CU per
                        subband block) or [2^14, 2^17] (streamed block state) */
  int32_t overlap;   /* N_ov, full-field samples, even, 0 <= N_ov < N */
  int32_t fir_mode;  /* how the forward evaluates the coupled filter of eq. (15),
                        circular over N' (the same map either way):
                        CBESSFM_FIR_TIME: direct sum over the taps;
                        CBESSFM_FIR_FREQ: the paper's frequency-domain form
                        (Sec. III-A, Fig. "scheme_NLPR"): DFT of each subband's
                        intensity, the N_sb x N_sb matrix of the coefficient
                        rows' DFTs per bin, inverse DFT (N' <= 8192 only);
                        CBESSFM_FIR_AUTO: frequency domain above 64 taps.
                        The adjoint and the dual-polarisation NLPR evaluate the
                        filter in the time domain. */
  int32_t boundary;  /* 0: circular sequence; 1: zeros outside [0, T) */
} cbessfm_subbands;
enum { CBESSFM_FIR_AUTO = 0, CBESSFM_FIR_TIME = 1, CBESSFM_FIR_FREQ = 2 };

/* Coefficients of the coupled intensity filter, eq. (15). */
typedef struct {
  int32_t n_taps;    /* 2 Nc + 1: odd, 1 <= n_taps <= min(N', 255) */
  const float* c;    /* host, [steps][n_sb][n_sb][n_taps], rad/W, tap t <-> m = t - Nc;
                        NULL: analytic coefficients (eqs. (13), (22), Sec. III-C) */
  int32_t grid_m;    /* analytic only: odd frequency grid size >= n_taps, 0 = n_taps */
} cbessfm_coeffs;

typedef struct cbessfm_plan cbessfm_plan_t;

/* Geometry of a plan, for callers that size buffers or report throughput. */
typedef struct {
  int32_t n_sb, block_sb, block, overlap, hop, steps, n_taps;
  int32_t threads_per_group; /* workgroup size of the main kernels */
  int32_t team_capacity;     /* teams (of n_sb workgroups) that can be resident */
  double step_km, split_ratio;
} cbessfm_info;

/* Checks every argument of cbessfm_plan on the host, touching no device.
 * Order of checks: link (n_spans >= 1, span_km > 0, sample_rate_hz > 0,
 * finite beta2), n_sb in 1..8, N' supported, overlap even and in [0, N),
 * fir_mode in {0, 1, 2} (CBESSFM_EUNSUPPORTED for 2 with N' >= 2^14),
 * boundary in {0, 1}, n_taps odd and in range, grid_m, split_ratio in [0, 1],
 * steps >= 1.  Returns CBESSFM_EINVAL or CBESSFM_EUNSUPPORTED on the first
 * failure. */
int cbessfm_plan_check(const cbessfm_link* link, const cbessfm_subbands* sb,
                       int32_t steps, double split_ratio, const cbessfm_coeffs* coeffs);

/* Creates a plan on the current HIP device: validates as cbessfm_plan_check,
 * builds the dispersion filters and DFT twiddles in FP64 (rounded once to
 * FP32), copies or computes the coefficients, and allocates every device
 * table and exchange buffer the kernels need.  Synchronises the device.
 * *out receives the plan (NULL on failure); release it with cbessfm_destroy. */
int cbessfm_plan(cbessfm_plan_t** out, const cbessfm_link* link, const cbessfm_subbands* sb,
                 int32_t steps, double split_ratio, const cbessfm_coeffs* coeffs);

/* Replaces coefficients and/or split ratio from device memory, on stream:
 * dev_c (nullable = keep) has the layout of cbessfm_coeffs.c with the plan's
 * n_taps; dev_rho (nullable = keep) points to one float in [0, 1] (not
 * checked on the device).  Asynchronous; no allocation. */
int cbessfm_set_coeffs(cbessfm_plan_t* plan, const float* dev_c, const float* dev_rho,
                       void* stream);

/* Host-side form of the split-ratio update (validated; asynchronous). */
int cbessfm_set_split_ratio(cbessfm_plan_t* plan, double split_ratio, void* stream);

/* Nonlinear phase rotation used by cbessfm_run.
 *   CBESSFM_NLPR_AVERAGED (the default): one phase per subband from the total
 *     intensity |x|^2 + |y|^2 of every subband, eq. (15);
 *   CBESSFM_NLPR_DUAL_POL: separate phases for the two polarisations,
 *     eqs. (20)-(21): other subbands act twice as strongly on the co-polarised
 *     component (weights 2 and 1 instead of the averaged 3/2), the same
 *     coefficients C (whose 3/2 cross-band factor is then divided out).  It
 *     costs a second filter and exchange per step.  cbessfm_backward and
 *     cbessfm_batch_create return CBESSFM_EUNSUPPORTED for such a plan.
 * CBESSFM_EINVAL for another mode.  Host only; takes effect at the next run. */
enum { CBESSFM_NLPR_AVERAGED = 0, CBESSFM_NLPR_DUAL_POL = 1 };
int cbessfm_set_nlpr(cbessfm_plan_t* plan, int32_t mode);

/* Forward backpropagation of batch fields of T samples per polarisation.
 * field_in, field_out: device, complex float32 [batch][2][T], must not
 * overlap.  T >= 1, batch >= 1.  Asynchronous on stream. */
int cbessfm_run(cbessfm_plan_t* plan, const void* field_in, void* field_out,
                int64_t T, int32_t batch, void* stream);

/* Bytes of device workspace cbessfm_backward needs for (T, batch,
 * checkpoint_every); see cbessfm_backward for checkpoint_every. */
int cbessfm_backward_workspace(const cbessfm_plan_t* plan, int64_t T, int32_t batch,
                               int32_t checkpoint_every, size_t* bytes);

/* Reverse-mode derivative of L with respect to the coefficients, the split
 * ratio and (optionally) the input field, given grad_out = dL/dRe(out) +
 * j dL/dIm(out) for the output of cbessfm_run on field_in.
 *   grad_in   device complex float32 [batch][2][T] or NULL (not computed)
 *   grad_c    device float [steps][n_sb][n_sb][n_taps], overwritten
 *   grad_rho  device float, overwritten
 * checkpoint_every <= 1 (or >= steps): the forward sweep stores every step's
 * intermediate field and phase and nothing is recomputed.  1 < k < steps:
 * only the spectrum at the start of every k-th step is stored, and each
 * segment of k steps is recomputed once during the reverse sweep (less
 * workspace, about one more forward pass of work).  workspace: device, at
 * least cbessfm_backward_workspace() bytes.  Asynchronous on stream.
 * Plans with N' >= 2^14 (streamed block state) run the same derivative as a
 * sequence of per-stage kernels over waves of blocks; their workspace holds,
 * per wave, the block state at every segment start and after every step of
 * one segment, so it grows with steps / k + k.  Every checkpoint spacing
 * gives the same result bit for bit.  Errors: CBESSFM_EINVAL (NULL required
 * pointer, T or batch out of range), CBESSFM_EWORKSPACE, CBESSFM_EUNSUPPORTED
 * (dual-polarisation NLPR plan), CBESSFM_EHIP. */
int cbessfm_backward(cbessfm_plan_t* plan, const void* field_in, const void* grad_out,
                     void* grad_in, float* grad_c, float* grad_rho, int64_t T, int32_t batch,
                     int32_t checkpoint_every, void* workspace, size_t workspace_bytes,
                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): cbessfm_backward
 * with the library's own fixed device scratch as its workspace.  The scratch
 * is one array of CBESSFM_STATIC_SCRATCH_BYTES per device, held until the
 * process ends and shared by every call on that device: calls that overlap in
 * time on one device race on it.  It calls no allocating routine; the plan
 * (created beforehand) still owns its tables and exchange buffers.  Same
 * arguments, results and errors as cbessfm_backward without the workspace;
 * also CBESSFM_EWORKSPACE when the call would need more than
 * CBESSFM_STATIC_SCRATCH_BYTES (cbessfm_backward_workspace gives the need;
 * a checkpoint spacing between 1 and steps, or a smaller T or batch, lowers
 * it), CBESSFM_EINVAL when the current device is not the plan's.
 * Asynchronous on stream. */
#define CBESSFM_STATIC_SCRATCH_BYTES (64u << 20)
int cbessfm_backward_static(cbessfm_plan_t* plan, const void* field_in, const void* grad_out, void* grad_in,
                            float* grad_c, float* grad_rho, int64_t T, int32_t batch, int32_t checkpoint_every,
                            void* stream);

/* Complexity model of Sec. III-D (host): real multiplications *rm and real
 * additions *ra per 2D symbol of a method processing blocks of N samples with
 * overlap N_ov at n_sps samples per symbol.
 *   CBESSFM_CX_FREQ: CB-ESSFM with n_sb subbands and a frequency-domain
 *     NLPR, eqs. (28)-(29) (n_c ignored; n_sb must divide N);
 *   CBESSFM_CX_TIME: single-band ESSFM with a time-domain NLPR of 2 n_c + 1
 *     coefficients, eqs. (30)-(31) (n_sb ignored); the SSFM and OSSFM are
 *     n_c = 0, EDC is steps = 0.
 * CBESSFM_EINVAL for N < 2, N_ov outside [0, N), steps < 0, n_c < 0,
 * n_sps <= 0, an unknown kind or a NULL output. */
enum { CBESSFM_CX_FREQ = 0, CBESSFM_CX_TIME = 1 };
int cbessfm_complexity(int32_t kind, double n_sps, int64_t N, int64_t N_ov, int32_t steps, int32_t n_sb,
                       int32_t n_c, double* rm, double* ra);

/* ---- Tied coefficients of the fitting protocol (Sec. III-B) ----
 * params: device float [n_sb][n_taps]; row h is c_h, the applied coefficients
 * (rad/W) between subbands l and l + h, tap t <-> m = t - Nc; of row 0 only
 * the taps m >= 0 are read (c_0 is even, eq. (25)).  weights: device float
 * [steps], w_s of assumption (i).  half_taps: host int32 [n_sb] with
 * 0 <= Nc(h) <= Nc (assumption (iii)), or NULL for Nc everywhere.
 * cbessfm_tie_expand writes the applied tensor, device float
 * [steps][n_sb][n_sb][n_taps]:
 *   C[s][i][l][m] = w_s c_{l-i}[m] (l >= i),  w_s c_{i-l}[-m] (l < i)
 * (eqs. (23), (24)), zero where |m| > Nc(|l - i|).
 * cbessfm_tie_reduce is its transpose: grad_params [n_sb][n_taps] from
 * grad_c of that shape, summed in FP64 in a fixed order (unused entries of
 * row 0 get 0).  Both return CBESSFM_EINVAL for n_sb outside 1..8, n_taps not
 * odd in 1..255, steps < 1, a bad half_taps entry or a NULL pointer;
 * asynchronous on stream; the caller owns every buffer. */
int cbessfm_tie_expand(const float* params, const float* weights, int32_t steps, int32_t n_sb,
                       int32_t n_taps, const int32_t* half_taps, float* coeffs, void* stream);
int cbessfm_tie_reduce(const float* grad_c, const float* weights, int32_t steps, int32_t n_sb,
                       int32_t n_taps, const int32_t* half_taps, float* grad_params, void* stream);

/* Host FP64 weights of assumption (i) of Sec. III-B, in backpropagation step
 * order: the effective length of the physical step each backpropagation step
 * undoes, divided by the mean over steps (for equal steps within a span, the
 * ratio of the signal powers at the step inputs).  mean_leff_km (may be NULL)
 * receives that mean, so gamma * mean_leff_km is the nonlinear phase per
 * watt of an average step. */
int cbessfm_step_weights(const cbessfm_link* link, int32_t steps, double* weights, double* mean_leff_km);

/* Host: half lengths Nc(h), h = 0..n_sb-1, of assumption (iii) of Sec. III-B:
 * 2 Nc(h) + 1 is the odd integer nearest to pi L |beta2| R'^2 (h + 1), L the
 * step length, R' = R / n_sb, capped at n_taps / 2. */
int cbessfm_tied_half_taps(const cbessfm_link* link, int32_t n_sb, int32_t steps, int32_t n_taps,
                           int32_t* half_taps);

/* Free dispersion segments (Sec. III-C; the step-size distribution and
 * per-step split ratio left to future work in Sec. V).  dev_lengths: device
 * double [steps + 1], km: the dispersion compensated before the first NLPR,
 * between NLPR s and s + 1, and after the last NLPR (by default (1 - rho) L,
 * L, ..., L, rho L; their sum is normally the link length).  The plan uses
 * these from the next run or backward on; NULL, cbessfm_set_split_ratio or a
 * cbessfm_set_coeffs call with a split ratio return to the uniform steps.
 * Asynchronous on stream (graph-capturable); the lengths are copied. */
int cbessfm_set_gvd_lengths(cbessfm_plan_t* plan, const double* dev_lengths, void* stream);

/* cbessfm_backward that also writes grad_gvd (device double [steps + 1], or
 * NULL): dL/d(length of each dispersion segment), in the plan's current
 * segment layout.  Costs one more size-N' transform per step and member.
 * Same workspace and errors as cbessfm_backward. */
int cbessfm_backward_gvd(cbessfm_plan_t* plan, const void* field_in, const void* grad_out,
                         void* grad_in, float* grad_c, float* grad_rho, double* grad_gvd, int64_t T,
                         int32_t batch, int32_t checkpoint_every, void* workspace, size_t workspace_bytes,
                         void* stream);

/* Analytic applied coefficients (host FP64), [steps][n_sb][n_sb][n_taps]:
 * c_il[m] of eq. (13) on an odd grid_m x grid_m midpoint grid (0 = n_taps)
 * with the kernel of eq. (6) integrated exactly between amplifiers (eq. (22)
 * for symmetric whole-span steps); DBP step s undoes physical step
 * N_st - s + 1 with its NLPR at rho L from that step's start; the returned
 * tensor is -c_ii on the diagonal and -(3/2) c_il off it. */
int cbessfm_analytic_coeffs(const cbessfm_link* link, const cbessfm_subbands* sb,
                            int32_t steps, double split_ratio, int32_t n_taps, int32_t grid_m,
                            double* out_host);

/* Plan geometry. */
int cbessfm_plan_info(const cbessfm_plan_t* plan, cbessfm_info* out);

/* Synchronises the plan's device, returns and clears the sticky device error
 * flag (CBESSFM_ESYNC if an exchange wait gave up since the last call; the
 * plan's exchange state is then reset as well). */
int cbessfm_status(cbessfm_plan_t* plan);

/* Bound of the device-side exchange waits of the plan's persistent kernels
 * (cbessfm_run, cbessfm_backward): a wait polls at most `polls` times, about
 * 64 cycles apart, then gives up: it sets the plan's sticky error
 * (CBESSFM_ESYNC from cbessfm_status) and every later wait of the launch
 * falls through, so the launch still ends, with invalid results.  A healthy
 * launch never comes near the default of 2^22 polls (about 0.1 s); 0 restores
 * it.  Lowering it exercises the give-up path (tests).  Host only; takes
 * effect at the next run or backward.  CBESSFM_EINVAL for a NULL plan. */
int cbessfm_set_wait_limit(cbessfm_plan_t* plan, uint32_t polls);

/* Releases the plan and all its device memory (NULL is a no-op). */
void cbessfm_destroy(cbessfm_plan_t* plan);

/* Static description of an error code. */
const char* cbessfm_strerror(int code);

/* ------------------------------------------------------------------ batches
 * Many instances in one persistent launch per distinct N' up to 8192 (one
 * launch when all instances share N'); instances with N' >= 2^14 (streamed
 * block state) run on the streaming kernels after those launches,
 * concurrently on up to four side streams of the batch (default priority)
 * that fork from and join back to the caller's stream.  An instance is a plan -- its own link, subband
 * count, steps, split ratio and coefficients -- with its own fields, length
 * and batch count; the batch computes for every instance exactly what
 * cbessfm_run would (Sec. III-A / III-C).  Workgroups form static teams of the
 * width (n_sb) of the instances they run; every team is placed on one XCD,
 * the number of teams of each width balances the predicted work, and blocks
 * are dealt to teams longest first (cbessfm_schedule).  A run allocates
 * nothing and keeps no host-side state between launches, so it may be
 * recorded in a HIP graph and replayed.
 */
typedef struct {
  cbessfm_plan_t* plan;    /* the instance's plan, on the current device; must outlive the batch */
  const void* field_in;    /* device complex float32 [batch][2][T] */
  void* field_out;         /* device, same shape; may not overlap any field of the batch */
  int64_t T;               /* samples per polarisation, 1 <= T < 2^31 */
  int32_t batch;           /* >= 1 */
} cbessfm_instance;

typedef struct cbessfm_batch cbessfm_batch_t;

typedef struct {
  int32_t launches;        /* persistent launches per run (distinct N' <= 8192) */
  int32_t teams;           /* teams over all launches */
  int32_t workgroups;      /* summed grid sizes */
  int64_t items;           /* overlap-and-save blocks over all instances */
  double makespan_s;       /* predicted run time: summed over launches, max over teams,
                              plus the streamed instances */
  double lower_bound_s;    /* a lower bound of makespan_s for the same item costs */
  int32_t streamed;        /* instances with N' >= 2^14, run by the streaming kernels */
  int64_t streamed_items;  /* their blocks (included in items) */
  int32_t stream_classes;  /* classes of streamed instances (same N', n_sb, taps) whose
                              steps run as one launch per stage over all their blocks */
  int32_t stream_lone;     /* streamed instances run one by one (more than one wave, or a
                              plan shared with another instance) */
  int32_t kernel_launches; /* kernels one run launches in all (persistent launches, the
                              streamed instances' input and output stages, class steps) */
} cbessfm_batch_info;

/* Builds the schedule and the device tables of a batch on the current
 * device (synchronous).  Field pointers are bound now: every run reads and
 * writes the same buffers.  Item costs come from the autotuner's device
 * timings when cbessfm_autotune(..., CBESSFM_TUNE_MEASURE, ...) has run for
 * the shape, else from an operation-count model.  Errors: CBESSFM_EINVAL for
 * null or out-of-range arguments, a plan of another device or overlapping
 * fields; CBESSFM_ENOMEM; CBESSFM_EHIP.  *out is NULL on failure. */
int cbessfm_batch_create(cbessfm_batch_t** out, const cbessfm_instance* inst, int32_t n);

/* Runs every instance of the batch: asynchronous on stream, no allocation,
 * graph-capturable (inside a capture the launches are recorded as ordinary
 * kernel nodes of resident-sized grids).  Runs of one batch that overlap in
 * time race on its exchange buffers. */
int cbessfm_batch_run(cbessfm_batch_t* b, void* stream);

/* Schedule summary of a batch. */
int cbessfm_batch_describe(const cbessfm_batch_t* b, cbessfm_batch_info* out);

/* As cbessfm_status, for the batch's own exchange state. */
int cbessfm_batch_status(cbessfm_batch_t* b);

/* Releases the batch (not its plans or fields; NULL is a no-op). */
void cbessfm_batch_destroy(cbessfm_batch_t* b);

/* The batch scheduler on its own (host only, no device).  Job j has n_items
 * blocks of predicted cost `cost` each, run by teams of `width` workgroups.
 * slots_per_xcd: resident workgroups per XCD.  Outputs (caller-allocated):
 * wg_team / wg_member [max_wg] give each workgroup's team and member index
 * (-1: idle) for workgroups 0 .. grid - 1, workgroup w running on XCD w mod 8;
 * item_team / item_rank [sum of n_items] give each block's team and its
 * position in that team's sequence (blocks numbered job by job).  Either pair
 * may be NULL.  Errors: CBESSFM_EINVAL (bad job, no blocks, grid > max_wg),
 * CBESSFM_EUNSUPPORTED (a width that does not fit one XCD). */
typedef struct {
  int32_t width;
  int64_t n_items;
  double cost;
} cbessfm_sched_job;

typedef struct {
  int32_t grid;            /* workgroups to launch */
  int32_t n_teams;
  double makespan;         /* max over teams of the summed cost of its blocks */
  double lower_bound;      /* max(largest block cost, total cost x width / workgroup slots) */
} cbessfm_sched_stats;

int cbessfm_schedule(const cbessfm_sched_job* jobs, int32_t n_jobs, int32_t slots_per_xcd, int32_t max_wg,
                     int32_t* wg_team, int32_t* wg_member, int32_t* item_team, int32_t* item_rank,
                     cbessfm_sched_stats* stats);

/* ------------------------------------------------------------------ autotuner
 * Picks N' and N_ov for one instance.  The overlap must cover the memory of
 * the accumulated dispersion of the backpropagated link, taken as
 * 2 pi |beta2| L R^2 full-field samples (the group-delay spread of a band R
 * over L; Sec. III-A), rounded up to even.  Among the N' in [256, 8192] whose
 * block N = n_sb N' exceeds it, the one with the least predicted time for the
 * instance (blocks / resident teams, rounded up, times the time of one block)
 * is the persistent candidate.  The smallest streamed block N' in
 * [2^14, 2^17] that covers the memory is the streamed candidate (its time:
 * blocks times the time of one streamed block).  The streamed candidate is
 * returned if no persistent block covers the memory, or if it is predicted
 * faster; only if even N' = 2^17 does not cover the memory (and no
 * persistent block does), N' = 2^17 with N_ov = min(memory, N / 2) and
 * covered = 0.  A streamed instance needs its own plan's block-state buffers
 * (cbessfm_plan sizes them, at most 512 MB).  flags: CBESSFM_TUNE_MEASURE
 * times each candidate block shape on the current device (persistent: probe
 * launches of one block per resident team; streamed: as many blocks as
 * 256 MB of block state holds; both at 1 and 4 steps, linear in the step
 * count, cached per device and shape for the process); 0 uses
 * operation-count models and touches no device.  Errors: CBESSFM_EINVAL,
 * CBESSFM_EHIP. */
enum { CBESSFM_TUNE_MEASURE = 1 };

typedef struct {
  int32_t block_sb;        /* chosen N' */
  int32_t overlap;         /* chosen N_ov, full-field samples, even */
  int32_t memory;          /* dispersion memory, full-field samples */
  int32_t covered;         /* 1 if overlap >= memory */
  int32_t measured;        /* 1 if the prediction uses device timings */
  double predicted_s;      /* predicted time of one cbessfm_run of the instance */
} cbessfm_tuning;

int cbessfm_autotune(const cbessfm_link* link, int32_t n_sb, int32_t steps, int32_t n_taps, int64_t T,
                     int32_t batch, int32_t flags, cbessfm_tuning* out);

#ifdef __cplusplus
}
#endif

#endif /* CBESSFM_H */
