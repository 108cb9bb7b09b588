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
  CBESSFM_ESYNC = -5,       /* a device-side team barrier gave up waiting */
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
  int32_t block_sb;  /* N' = N / N_sb, power of two in [256, 8192] */
  int32_t overlap;   /* N_ov, full-field samples, even, 0 <= N_ov < N */
  int32_t boundary;  /* 0: circular sequence; 1: zeros outside [0, T) */
} cbessfm_subbands;

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

/* Forward backpropagation of batch fields of T samples per polarisation.
 * field_in, field_out: device, complex float32 [batch][2][T], must not
 * overlap.  T >= 1, batch >= 1.  Asynchronous on stream. */
int cbessfm_run(cbessfm_plan_t* plan, const void* field_in, void* field_out,
                int64_t T, int32_t batch, void* stream);

/* Bytes of device workspace cbessfm_backward needs for (T, batch,
 * checkpoint_every); checkpoint_every <= 0 means "store every step". */
int cbessfm_backward_workspace(const cbessfm_plan_t* plan, int64_t T, int32_t batch,
                               int32_t checkpoint_every, size_t* bytes);

/* Reverse-mode derivative of L with respect to the coefficients, the split
 * ratio and (optionally) the input field, given grad_out = dL/dRe(out) +
 * j dL/dIm(out) for the output of cbessfm_run on field_in.
 *   grad_in   device complex float32 [batch][2][T] or NULL (not computed)
 *   grad_c    device float [steps][n_sb][n_sb][n_taps], overwritten
 *   grad_rho  device float, overwritten
 * The forward trajectory is recomputed from states stored every
 * checkpoint_every steps (<= 0: every step).  workspace: device, at least
 * cbessfm_backward_workspace() bytes.  Asynchronous on stream. */
int cbessfm_backward(cbessfm_plan_t* plan, const void* field_in, const void* grad_out,
                     void* grad_in, float* grad_c, float* grad_rho, int64_t T, int32_t batch,
                     int32_t checkpoint_every, void* workspace, size_t workspace_bytes,
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
 * flag (CBESSFM_ESYNC if a team barrier gave up since the last call). */
int cbessfm_status(cbessfm_plan_t* plan);

/* Releases the plan and all its device memory (NULL is a no-op). */
void cbessfm_destroy(cbessfm_plan_t* plan);

/* Static description of an error code. */
const char* cbessfm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CBESSFM_H */
