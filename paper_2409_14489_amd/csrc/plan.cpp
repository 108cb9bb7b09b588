// Host side of libcbessfm: argument validation, plan construction (FP64
// tables rounded once to FP32), analytic coefficients, error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "cbessfm.h"
#include "internal.hpp"

using cbessfm::kMaxSubbands;
using cbessfm::kMaxTaps;
using cbessfm::kTapChunk;
using cd = std::complex<double>;

namespace {

constexpr double kPi = 3.14159265358979323846;

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

int check_link(const cbessfm_link* link) {
  if (!link) return CBESSFM_EINVAL;
  if (link->n_spans < 1 || !(link->span_km > 0.0) || !std::isfinite(link->span_km)) return CBESSFM_EINVAL;
  if (!(link->sample_rate_hz > 0.0) || !std::isfinite(link->sample_rate_hz)) return CBESSFM_EINVAL;
  if (!std::isfinite(link->beta2_ps2_km) || !std::isfinite(link->alpha_db_km) ||
      !std::isfinite(link->gamma_w_km) || link->alpha_db_km < 0.0)
    return CBESSFM_EINVAL;
  return CBESSFM_OK;
}

int check_layout(const cbessfm_subbands* sb) {
  if (!sb) return CBESSFM_EINVAL;
  if (sb->n_sb < 1 || sb->n_sb > kMaxSubbands) return CBESSFM_EINVAL;
  if (!is_pow2(sb->block_sb) || sb->block_sb < 256 || sb->block_sb > (1 << cbessfm::kStreamMaxLog))
    return CBESSFM_EUNSUPPORTED;
  if (sb->block_sb > 8192 && sb->block_sb < (1 << cbessfm::kStreamMinLog)) return CBESSFM_EUNSUPPORTED;
  const long long n = (long long)sb->n_sb * sb->block_sb;
  if (sb->overlap < 0 || sb->overlap >= n || (sb->overlap & 1)) return CBESSFM_EINVAL;
  if (sb->fir_mode < CBESSFM_FIR_AUTO || sb->fir_mode > CBESSFM_FIR_FREQ) return CBESSFM_EINVAL;
  if (sb->fir_mode == CBESSFM_FIR_FREQ && sb->block_sb > 8192) return CBESSFM_EUNSUPPORTED;
  if (sb->boundary != 0 && sb->boundary != 1) return CBESSFM_EINVAL;
  return CBESSFM_OK;
}

int check_taps(int n_taps, int grid_m, int block_sb) {
  if (n_taps < 1 || (n_taps & 1) == 0) return CBESSFM_EINVAL;
  if (n_taps > block_sb) return CBESSFM_EINVAL;
  if (n_taps > kMaxTaps) return CBESSFM_EUNSUPPORTED;
  if (grid_m != 0 && (grid_m < n_taps || (grid_m & 1) == 0)) return CBESSFM_EINVAL;
  return CBESSFM_OK;
}

// ---------------------------------------------------------------- analytic coefficients
// Kernel of eq. (6) in the form of App. C (eq. kernel_b):
//   K(b) = gamma int_{z_lo}^{z_hi} g(z) exp(-j 2 b (z - z0)) dz,
// g(z) = exp(-alpha (z - position of the last amplifier)).  Each piece between
// amplifiers integrates in closed form: exp(-(alpha + j 2 b) l) terms.
cd step_kernel(double b, double z_lo, double z_hi, double z0, double alpha, double span, double gamma) {
  const cd kappa(alpha, 2.0 * b);
  cd acc(0.0, 0.0);
  double a = z_lo;
  const double tol = 1e-12 * std::max(1.0, std::fabs(z_hi));
  while (a < z_hi - tol) {
    const double amp = std::floor(a / span + 1e-12) * span;  // last amplifier
    const double c = std::min(z_hi, amp + span);
    const double len = c - a;
    const cd x = kappa * len;
    cd frac;  // (1 - exp(-kappa len)) / kappa
    if (std::abs(x) < 1e-6)
      frac = len * (1.0 - x / 2.0 + x * x / 6.0);
    else
      frac = (1.0 - std::exp(-x)) / kappa;
    acc += std::exp(-alpha * (a - amp)) * std::exp(cd(0.0, -2.0 * b * (a - z0))) * frac;
    a = c;
  }
  return gamma * acc;
}

}  // namespace

namespace cbessfm {
// FP32 rounding of (c, s) that keeps the magnitude: of the (at most) four
// pairs of FP32 neighbours of c and s, the one whose squared magnitude is
// closest to c^2 + s^2.  Unit-magnitude tables reused by every transform and
// step would otherwise bias the signal amplitude.
float2 round_pair(double c, double s) {
  const float c0 = (float)c, s0 = (float)s;
  const float cs[2] = {c0, (double)c0 < c ? std::nextafter(c0, 2.0f) : std::nextafter(c0, -2.0f)};
  const float ss[2] = {s0, (double)s0 < s ? std::nextafter(s0, 2.0f) : std::nextafter(s0, -2.0f)};
  const double target = c * c + s * s;
  float2 best = make_float2(c0, s0);
  double err = 1e300;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const double m = (double)cs[i] * cs[i] + (double)ss[j] * ss[j];
      const double e = std::fabs(m - target);
      if (e < err) {
        err = e;
        best = make_float2(cs[i], ss[j]);
      }
    }
  return best;
}
}  // namespace cbessfm

namespace {

size_t xspec_bytes(const cbessfm_plan_t* p) {
  return sizeof(uint64_t) * (size_t)p->xchg_teams * 2 * p->sb.n_sb * 4 * p->Np;
}
size_t xp_bytes(const cbessfm_plan_t* p) {  // room for the spectra of the frequency-domain filter
  return sizeof(uint64_t) * (size_t)p->xchg_teams * 2 * p->sb.n_sb * 2 * p->Np;
}

}  // namespace

extern "C" {

const char* cbessfm_strerror(int code) {
  switch (code) {
    case CBESSFM_OK: return "success";
    case CBESSFM_EINVAL: return "invalid argument";
    case CBESSFM_EUNSUPPORTED: return "unsupported size";
    case CBESSFM_ENOMEM: return "out of memory";
    case CBESSFM_EHIP: return "HIP runtime error";
    case CBESSFM_ESYNC: return "device team barrier timed out";
    case CBESSFM_EWORKSPACE: return "workspace too small";
    default: return "unknown error";
  }
}

int cbessfm_plan_check(const cbessfm_link* link, const cbessfm_subbands* sb, int32_t steps, double split_ratio,
                       const cbessfm_coeffs* coeffs) {
  int rc = check_link(link);
  if (rc) return rc;
  rc = check_layout(sb);
  if (rc) return rc;
  if (!coeffs) return CBESSFM_EINVAL;
  rc = check_taps(coeffs->n_taps, coeffs->grid_m, sb->block_sb);
  if (rc) return rc;
  if (!(split_ratio >= 0.0 && split_ratio <= 1.0)) return CBESSFM_EINVAL;
  if (steps < 1) return CBESSFM_EINVAL;
  return CBESSFM_OK;
}

// Weights of assumption (i) of Sec. III-B: the effective length of the
// physical step each backpropagation step undoes (K of eq. (6) at b = 0, over
// gamma), divided by their mean.  For equal steps within a span this is the
// ratio of the signal powers at the step inputs.
int cbessfm_step_weights(const cbessfm_link* link, int32_t steps, double* weights, double* mean_leff_km) {
  const int rc = check_link(link);
  if (rc) return rc;
  if (steps < 1 || !weights) return CBESSFM_EINVAL;
  const double alpha = link->alpha_db_km * std::log(10.0) / 10.0;
  const double step = link->span_km * link->n_spans / steps;
  double sum = 0.0;
  for (int s = 0; s < steps; ++s) {
    const int j = steps - 1 - s;  // physical step, 0-based
    weights[s] = step_kernel(0.0, j * step, (j + 1) * step, 0.0, alpha, link->span_km, 1.0).real();
    sum += weights[s];
  }
  const double mean = sum / steps;
  for (int s = 0; s < steps; ++s) weights[s] /= mean;
  if (mean_leff_km) *mean_leff_km = mean;
  return CBESSFM_OK;
}

// Assumption (iii) of Sec. III-B: 2 Nc(h) + 1 is the odd integer nearest to
// pi L |beta2| R'^2 (h + 1) (L the step length, R' the subband rate), capped
// at n_taps.
int cbessfm_tied_half_taps(const cbessfm_link* link, int32_t n_sb, int32_t steps, int32_t n_taps,
                           int32_t* half_taps) {
  const int rc = check_link(link);
  if (rc) return rc;
  if (n_sb < 1 || n_sb > kMaxSubbands || steps < 1 || n_taps < 1 || (n_taps & 1) == 0 || !half_taps)
    return CBESSFM_EINVAL;
  const double step = link->span_km * link->n_spans / steps;
  const double rp = link->sample_rate_hz / n_sb;
  const double b2 = std::fabs(link->beta2_ps2_km) * 1e-24;
  for (int h = 0; h < n_sb; ++h) {
    const double x = kPi * step * b2 * rp * rp * (h + 1);
    const double nc = std::floor((x - 1.0) / 2.0 + 0.5);
    half_taps[h] = (int32_t)std::min<double>(n_taps / 2, std::max(0.0, nc));
  }
  return CBESSFM_OK;
}

// Complexity model of Sec. III-D, per 2D symbol: a block of N 4D samples
// keeps N - N_ov of them, each carrying two 2D symbols at n samples per
// symbol.  Frequency-domain CB-ESSFM: 4 size-N CFFTs, 4 N_sb N_st size-N'
// CFFTs (split radix: N log2 N - 3N + 4 RM, 3 N log2 N - 3N + 4 RA), N_st + 1
// dispersion steps (6N RM, 6N RA) and N_st NLPRs (N log2 N' + N (3 N_sb + 13) / 2
// + 4 N_sb RM, 3 N log2 N' + N (5 N_sb + 11) / 2 + 4 N_sb RA).  Time-domain
// ESSFM: N_st + 1 dispersion steps of 4 size-N CFFTs each and N_st NLPRs of
// (11 + Nc) N RM and (11 + 2 Nc) N RA.
int cbessfm_complexity(int32_t kind, double n_sps, int64_t N, int64_t N_ov, int32_t steps, int32_t n_sb,
                       int32_t n_c, double* rm, double* ra) {
  if (!(n_sps > 0.0) || N < 2 || N_ov < 0 || N_ov >= N || steps < 0 || n_c < 0 || !rm || !ra)
    return CBESSFM_EINVAL;
  const double n = (double)N;
  const double per = n_sps / 2.0 / (double)(N - N_ov);  // per 2D symbol, per block
  auto cfft_rm = [](double m) { return m * std::log2(m) - 3.0 * m + 4.0; };
  auto cfft_ra = [](double m) { return 3.0 * m * std::log2(m) - 3.0 * m + 4.0; };
  if (kind == CBESSFM_CX_FREQ) {
    if (n_sb < 1 || N % n_sb) return CBESSFM_EINVAL;
    const double np = n / n_sb, lg = std::log2(np);
    const double m = 4.0 * cfft_rm(n) + 4.0 * n_sb * steps * cfft_rm(np) + 6.0 * n * (steps + 1) +
                     steps * (n * lg + n * (3.0 * n_sb + 13.0) / 2.0 + 4.0 * n_sb);
    const double a = 4.0 * cfft_ra(n) + 4.0 * n_sb * steps * cfft_ra(np) + 6.0 * n * (steps + 1) +
                     steps * (3.0 * n * lg + n * (5.0 * n_sb + 11.0) / 2.0 + 4.0 * n_sb);
    *rm = per * m;
    *ra = per * a;
    return CBESSFM_OK;
  }
  if (kind == CBESSFM_CX_TIME) {
    const double m = (steps + 1) * (4.0 * cfft_rm(n) + 6.0 * n) + steps * (11.0 + n_c) * n;
    const double a = (steps + 1) * (4.0 * cfft_ra(n) + 6.0 * n) + steps * (11.0 + 2.0 * n_c) * n;
    *rm = per * m;
    *ra = per * a;
    return CBESSFM_OK;
  }
  return CBESSFM_EINVAL;
}

int cbessfm_analytic_coeffs(const cbessfm_link* link, const cbessfm_subbands* sb, int32_t steps,
                            double split_ratio, int32_t n_taps, int32_t grid_m, double* out_host) {
  int rc = check_link(link);
  if (rc) return rc;
  if (!sb || sb->n_sb < 1 || sb->n_sb > kMaxSubbands || !out_host) return CBESSFM_EINVAL;
  if (n_taps < 1 || (n_taps & 1) == 0 || (grid_m != 0 && (grid_m < n_taps || (grid_m & 1) == 0)))
    return CBESSFM_EINVAL;
  if (!(split_ratio >= 0.0 && split_ratio <= 1.0) || steps < 1) return CBESSFM_EINVAL;
  const int nsb = sb->n_sb;
  const int m_grid = grid_m ? grid_m : n_taps;
  const int half = m_grid / 2, nc = n_taps / 2;
  const double alpha = link->alpha_db_km * std::log(10.0) / 10.0;  // power, 1/km
  const double beta2 = link->beta2_ps2_km * 1e-24;                  // s^2/km
  const double gamma = link->gamma_w_km * (link->manakov_8_9 ? 8.0 / 9.0 : 1.0);
  const double step = link->span_km * link->n_spans / steps;
  const double rp = link->sample_rate_hz / nsb;                      // subband rate R'
  // phase factors exp(j 2 pi m d / M) for d = p - q in [-(M-1), M-1]
  std::vector<cd> kgrid((size_t)m_grid * m_grid);
  for (int s = 0; s < steps; ++s) {
    const int j = steps - s;  // physical step undone by DBP step s (1-based)
    const double z_lo = (j - 1) * step, z_hi = j * step, z0 = z_lo + split_ratio * step;
    for (int i = 0; i < nsb; ++i)
      for (int l = 0; l < nsb; ++l) {
        const double f_il = (l - i) * rp;  // f_l - f_i for equally spaced subbands
        for (int p = 0; p < m_grid; ++p)
          for (int q = 0; q < m_grid; ++q) {
            const double mu = f_il + (p - half) * rp / m_grid;
            const double nu = f_il + (q - half) * rp / m_grid;
            const double b = 2.0 * kPi * kPi * beta2 * nu * (mu - nu);
            kgrid[(size_t)p * m_grid + q] = step_kernel(b, z_lo, z_hi, z0, alpha, link->span_km, gamma);
          }
        const double xpm = (i == l) ? 1.0 : 1.5;
        for (int tau = 0; tau < n_taps; ++tau) {
          const int m = tau - nc;
          // c[m] = Re (1/M^2) sum_{p,q} K(mu_p, nu_q) exp(j 2 pi m (p - q) / M)
          cd acc(0.0, 0.0);
          for (int p = 0; p < m_grid; ++p) {
            cd row(0.0, 0.0);
            for (int q = 0; q < m_grid; ++q) {
              const double ang = 2.0 * kPi * (double)m * (double)(p - q) / m_grid;
              row += kgrid[(size_t)p * m_grid + q] * cd(std::cos(ang), std::sin(ang));
            }
            acc += row;
          }
          const double c = acc.real() / ((double)m_grid * m_grid);
          out_host[(((size_t)s * nsb + i) * nsb + l) * n_taps + tau] = -xpm * c;
        }
      }
  }
  return CBESSFM_OK;
}

void cbessfm_destroy(cbessfm_plan_t* p) {
  if (!p) return;
  // a void release path: HIP errors are not reportable here
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(p->device);
  void* bufs[] = {p->d_phase, p->d_h,     p->d_tw,    p->d_poly, p->d_c,     p->d_cpad,  p->d_ctpad,
                  p->d_cdpad, p->d_chat,  p->d_rho,   p->d_len,   p->d_xspec, p->d_xp,  p->d_xq,
                  p->d_epoch, p->d_abort, p->d_err,   p->d_st,    p->d_pb,    p->d_th};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  (void)hipSetDevice(prev);
  delete p;
}

int cbessfm_plan(cbessfm_plan_t** out, const cbessfm_link* link, const cbessfm_subbands* sb, int32_t steps,
                 double split_ratio, const cbessfm_coeffs* coeffs) {
  if (!out) return CBESSFM_EINVAL;
  *out = nullptr;
  int rc = cbessfm_plan_check(link, sb, steps, split_ratio, coeffs);
  if (rc) return rc;
  cbessfm_plan_t* p = new (std::nothrow) cbessfm_plan_t();
  if (!p) return CBESSFM_ENOMEM;
  std::memset(p, 0, sizeof(*p));
  p->link = *link;
  p->sb = *sb;
  p->steps = steps;
  p->n_taps = coeffs->n_taps;
  p->n_chunks = (coeffs->n_taps + kTapChunk - 1) / kTapChunk;
  p->tap_pad = p->n_chunks * kTapChunk;
  p->Np = sb->block_sb;
  p->N = sb->n_sb * sb->block_sb;
  p->hop = p->N - sb->overlap;
  p->log_np = log2i(p->Np);
  p->step_km = link->span_km * link->n_spans / steps;
  p->rho = split_ratio;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return CBESSFM_EHIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->device) != hipSuccess) {
    delete p;
    return CBESSFM_EHIP;
  }
  p->cu_count = prop.multiProcessorCount;
  p->stream = p->log_np >= cbessfm::kStreamMinLog;
  if (p->stream) {
    // block state of as many blocks as the budget holds, up to a cap
    const size_t per_block = (size_t)sb->n_sb * p->Np * (sizeof(float2) * 2 + sizeof(float) * 2);
    p->st_blocks = (int)std::max<size_t>(1, std::min<size_t>(cbessfm::kStreamBudget / per_block,
                                                              (size_t)cbessfm::kStreamMaxBlocks));
    p->threads = cbessfm::kStreamRow / 8;
    p->team_capacity = p->st_blocks;
  } else {
  p->threads = cbessfm::threads_for(p->log_np);
  int per_cu = 0, per_cu_dual = 0;
  if (cbessfm::occupancy_per_cu(p->log_np, false, &per_cu) != CBESSFM_OK || per_cu < 1 ||
      cbessfm::occupancy_per_cu(p->log_np, true, &per_cu_dual) != CBESSFM_OK || per_cu_dual < 1) {
    delete p;
    return CBESSFM_EHIP;
  }
  // teams are placed as groups of n_sb workgroups per XCD; keep the whole
  // (padded) grid resident
  int bwd_per_cu = 0;
  if (cbessfm::bwd_occupancy_per_cu(p->log_np, &bwd_per_cu) != CBESSFM_OK || bwd_per_cu < 1) {
    delete p;
    return CBESSFM_EHIP;
  }
  p->team_capacity = (per_cu * p->cu_count / (cbessfm::kXcds * sb->n_sb)) * cbessfm::kXcds;
  p->team_capacity_dual = (per_cu_dual * p->cu_count / (cbessfm::kXcds * sb->n_sb)) * cbessfm::kXcds;
  p->bwd_team_capacity = (bwd_per_cu * p->cu_count / (cbessfm::kXcds * sb->n_sb)) * cbessfm::kXcds;
  if (p->team_capacity < 1 || p->team_capacity_dual < 1 || p->bwd_team_capacity < 1) {
    delete p;
    return CBESSFM_EUNSUPPORTED;
  }
  p->xchg_teams = std::max(std::max(p->team_capacity, p->team_capacity_dual), p->bwd_team_capacity);
  }
  p->nlpr = CBESSFM_NLPR_AVERAGED;
  p->wait_limit = kDefaultWaitLimit;
  // auto: the frequency-domain filter costs about two single-array transforms
  // per step whatever the tap count; the direct sum grows with n_sb x n_taps
  // and is cheaper up to 64 taps (measured crossover 45..100 taps)
  p->fir_freq = !p->stream && (sb->fir_mode == CBESSFM_FIR_FREQ ||
                               (sb->fir_mode == CBESSFM_FIR_AUTO && coeffs->n_taps > 8 * kTapChunk));

  const int N = p->N, Np = p->Np, nsb = sb->n_sb;
  const size_t crows = (size_t)steps * nsb * nsb;
  // Streaming plans hold spectra with bin k2 + N2 k1 of a subband at position
  // k1 + N1 k2 (the order the four-step transform leaves them in); every
  // per-bin table follows that order.
  const int n1 = cbessfm::kStreamRow, n2 = p->stream ? Np / n1 : 1;
  auto bin_of = [&](int pos) { return p->stream ? (pos % n1) * n2 + pos / n1 : pos; };
  // ---- host tables in FP64
  std::vector<double> phase(N);
  const double beta2 = link->beta2_ps2_km * 1e-24;
  for (int q = 0; q < N; ++q) {  // subband order: q' = i N' + j  <->  bin q' - N/2
    const int qb = (q / Np) * Np + bin_of(q % Np);
    const double f = (double)(qb - N / 2) * link->sample_rate_hz / N;
    phase[q] = 2.0 * kPi * kPi * beta2 * f * f;
  }
  const int n_tw = p->stream ? Np + n1 : Np;
  std::vector<float2> tw(n_tw), poly((size_t)nsb * Np);
  if (p->stream) {
    for (int k = 0; k < n2; ++k)  // column twiddles exp(-j 2 pi n1 k2 / N')
      for (int j = 0; j < n1; ++j) {
        const double a = -2.0 * kPi * (double)((long long)j * k % Np) / Np;
        tw[(size_t)k * n1 + j] = cbessfm::round_pair(std::cos(a), std::sin(a));
      }
    for (int n = 0; n < n1; ++n) {  // row transform table
      const double a = -2.0 * kPi * n / n1;
      tw[(size_t)Np + n] = cbessfm::round_pair(std::cos(a), std::sin(a));
    }
  } else {
    for (int n = 0; n < Np; ++n) {
      const double a = -2.0 * kPi * n / Np;
      tw[n] = cbessfm::round_pair(std::cos(a), std::sin(a));
    }
  }
  for (int i = 0; i < nsb; ++i)
    for (int q = 0; q < Np; ++q) {
      const int k = bin_of(q);
      const double a = -2.0 * kPi * (double)((long long)i * k % N) / N;
      poly[(size_t)i * Np + q] = cbessfm::round_pair(std::cos(a), std::sin(a));
    }
  for (int a = 0; a < kMaxSubbands; ++a) {
    const double ang = -2.0 * kPi * a / nsb;
    p->wsb[a] = cbessfm::round_pair(std::cos(ang), std::sin(ang));
  }
  std::vector<float> c(crows * p->n_taps);
  if (coeffs->c) {
    std::memcpy(c.data(), coeffs->c, c.size() * sizeof(float));
  } else {
    std::vector<double> cd64(c.size());
    rc = cbessfm_analytic_coeffs(link, sb, steps, split_ratio, p->n_taps, coeffs->grid_m, cd64.data());
    if (rc) {
      delete p;
      return rc;
    }
    for (size_t k = 0; k < c.size(); ++k) c[k] = (float)cd64[k];
  }

  // ---- device memory
  bool ok = true;
  auto alloc = [&](void** ptr, size_t bytes) {
    if (ok && hipMalloc(ptr, bytes) != hipSuccess) ok = false;
  };
  alloc((void**)&p->d_phase, sizeof(double) * N);
  alloc((void**)&p->d_h, sizeof(float2) * (size_t)std::max(3, steps + 1) * N);
  alloc((void**)&p->d_tw, sizeof(float2) * n_tw);
  alloc((void**)&p->d_poly, sizeof(float2) * nsb * Np);
  alloc((void**)&p->d_c, sizeof(float) * crows * p->n_taps);
  alloc((void**)&p->d_cpad, sizeof(float) * crows * p->tap_pad);
  alloc((void**)&p->d_ctpad, sizeof(float) * crows * p->tap_pad);
  alloc((void**)&p->d_cdpad, sizeof(float) * crows * p->tap_pad);
  if (p->fir_freq) alloc((void**)&p->d_chat, sizeof(float2) * crows * Np);
  alloc((void**)&p->d_rho, sizeof(double));
  alloc((void**)&p->d_len, sizeof(double) * (size_t)(steps + 1));
  if (p->stream) {
    const size_t cells = (size_t)p->st_blocks * nsb * Np;
    alloc((void**)&p->d_st, sizeof(float2) * 2 * cells);
    alloc((void**)&p->d_pb, sizeof(float) * cells);
    alloc((void**)&p->d_th, sizeof(float) * cells);
  } else {
    alloc((void**)&p->d_xspec, xspec_bytes(p));
    alloc((void**)&p->d_xp, xp_bytes(p));
    alloc((void**)&p->d_xq, xp_bytes(p));
    alloc((void**)&p->d_epoch, sizeof(unsigned) * p->xchg_teams);
  }
  alloc((void**)&p->d_abort, sizeof(unsigned));
  alloc((void**)&p->d_err, sizeof(int));
  if (!ok) {
    cbessfm_destroy(p);
    return CBESSFM_ENOMEM;
  }
  bool hip_ok = hipMemcpy(p->d_phase, phase.data(), sizeof(double) * N, hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(p->d_tw, tw.data(), sizeof(float2) * n_tw, hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(p->d_poly, poly.data(), sizeof(float2) * nsb * Np, hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(p->d_c, c.data(), sizeof(float) * c.size(), hipMemcpyHostToDevice) == hipSuccess &&
                hipMemcpy(p->d_rho, &split_ratio, sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
                hipMemset(p->d_err, 0, sizeof(int)) == hipSuccess &&
                hipMemset(p->d_abort, 0, sizeof(unsigned)) == hipSuccess &&
                (p->stream || (hipMemset(p->d_xspec, 0, xspec_bytes(p)) == hipSuccess &&
                               hipMemset(p->d_xp, 0, xp_bytes(p)) == hipSuccess &&
                               hipMemset(p->d_xq, 0, xp_bytes(p)) == hipSuccess &&
                               hipMemset(p->d_epoch, 0, sizeof(unsigned) * p->xchg_teams) == hipSuccess));
  if (!hip_ok || cbessfm::launch_tables(p, nullptr) || cbessfm::launch_pad_coeffs(p, p->d_c, nullptr) ||
      hipDeviceSynchronize() != hipSuccess) {
    cbessfm_destroy(p);
    return CBESSFM_EHIP;
  }
  *out = p;
  return CBESSFM_OK;
}

int cbessfm_set_coeffs(cbessfm_plan_t* p, const float* dev_c, const float* dev_rho, void* stream) {
  if (!p) return CBESSFM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dev_c) {
    const size_t bytes = sizeof(float) * (size_t)p->steps * p->sb.n_sb * p->sb.n_sb * p->n_taps;
    if (hipMemcpyAsync(p->d_c, dev_c, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) return CBESSFM_EHIP;
    int rc = cbessfm::launch_pad_coeffs(p, p->d_c, s);
    if (rc) return rc;
  }
  if (dev_rho) {
    int rc = cbessfm::launch_copy_rho(p, dev_rho, s);
    if (rc) return rc;
    rc = cbessfm::launch_tables(p, s);
    if (rc) return rc;
    p->gvd_explicit = 0;
  }
  return CBESSFM_OK;
}

int cbessfm_set_gvd_lengths(cbessfm_plan_t* p, const double* dev_lengths, void* stream) {
  if (!p) return CBESSFM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int rc = dev_lengths ? cbessfm::launch_gvd_tables(p, dev_lengths, s) : cbessfm::launch_tables(p, s);
  if (rc) return rc;
  p->gvd_explicit = dev_lengths ? 1 : 0;
  return CBESSFM_OK;
}

int cbessfm_set_split_ratio(cbessfm_plan_t* p, double split_ratio, void* stream) {
  if (!p) return CBESSFM_EINVAL;
  if (!(split_ratio >= 0.0 && split_ratio <= 1.0)) return CBESSFM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  p->rho = split_ratio;
  p->gvd_explicit = 0;
  // the value is staged through the plan-owned host copy, so wait for it
  if (hipMemcpyAsync(p->d_rho, &p->rho, sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
    return CBESSFM_EHIP;
  int rc = cbessfm::launch_tables(p, s);
  if (rc) return rc;
  return hipStreamSynchronize(s) == hipSuccess ? CBESSFM_OK : CBESSFM_EHIP;
}

int cbessfm_run(cbessfm_plan_t* p, const void* field_in, void* field_out, int64_t T, int32_t batch,
                void* stream) {
  if (!p || !field_in || !field_out || T < 1 || batch < 1 || T >= (1LL << 31)) return CBESSFM_EINVAL;
  const char* a = static_cast<const char*>(field_in);
  const char* b = static_cast<const char*>(field_out);
  const long long bytes = (long long)batch * 2 * T * 8;
  if (a < b + bytes && b < a + bytes) return CBESSFM_EINVAL;  // in and out must not overlap
  if (p->stream)
    return cbessfm::launch_stream_forward(p, field_in, field_out, T, batch, static_cast<hipStream_t>(stream));
  return cbessfm::launch_forward(p, field_in, field_out, T, batch, static_cast<hipStream_t>(stream));
}

int cbessfm_plan_info(const cbessfm_plan_t* p, cbessfm_info* out) {
  if (!p || !out) return CBESSFM_EINVAL;
  out->n_sb = p->sb.n_sb;
  out->block_sb = p->Np;
  out->block = p->N;
  out->overlap = p->sb.overlap;
  out->hop = p->hop;
  out->steps = p->steps;
  out->n_taps = p->n_taps;
  out->threads_per_group = p->threads;
  out->team_capacity = p->team_capacity;
  out->step_km = p->step_km;
  out->split_ratio = p->rho;
  return CBESSFM_OK;
}

int cbessfm_status(cbessfm_plan_t* p) {
  if (!p) return CBESSFM_EINVAL;
  if (hipSetDevice(p->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return CBESSFM_EHIP;
  int err = 0;
  if (hipMemcpy(&err, p->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return CBESSFM_EHIP;
  if (err && !p->stream) {
    // An exchange wait gave up.  Workgroups of that launch may have written
    // words with tags a later launch would reuse, so the exchange state is
    // reset along with the sticky words.
    if (hipMemset(p->d_err, 0, sizeof(int)) != hipSuccess ||
        hipMemset(p->d_abort, 0, sizeof(unsigned)) != hipSuccess ||
        hipMemset(p->d_xspec, 0, xspec_bytes(p)) != hipSuccess || hipMemset(p->d_xp, 0, xp_bytes(p)) != hipSuccess ||
        hipMemset(p->d_xq, 0, xp_bytes(p)) != hipSuccess ||
        hipMemset(p->d_epoch, 0, sizeof(unsigned) * p->xchg_teams) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess)
      return CBESSFM_EHIP;
  }
  return err;
}

int cbessfm_set_wait_limit(cbessfm_plan_t* p, uint32_t polls) {
  if (!p) return CBESSFM_EINVAL;
  p->wait_limit = polls ? polls : kDefaultWaitLimit;
  return CBESSFM_OK;
}

int cbessfm_set_nlpr(cbessfm_plan_t* p, int32_t mode) {
  if (!p || (mode != CBESSFM_NLPR_AVERAGED && mode != CBESSFM_NLPR_DUAL_POL)) return CBESSFM_EINVAL;
  if (p->stream && mode != CBESSFM_NLPR_AVERAGED) return CBESSFM_EUNSUPPORTED;  // streaming runs eq. (15)
  p->nlpr = mode;
  return CBESSFM_OK;
}

int cbessfm_backward_workspace(const cbessfm_plan_t* p, int64_t T, int32_t batch, int32_t checkpoint_every,
                               size_t* bytes) {
  if (!p || !bytes || T < 1 || batch < 1 || T >= (1LL << 31)) return CBESSFM_EINVAL;
  *bytes = p->stream ? cbessfm::stream_bwd_layout(p, T, batch, checkpoint_every, true).bytes
                     : cbessfm::bwd_layout(p, T, batch, checkpoint_every).bytes;
  return CBESSFM_OK;
}

int cbessfm_backward(cbessfm_plan_t* p, const void* field_in, const void* grad_out, void* grad_in, float* grad_c,
                     float* grad_rho, int64_t T, int32_t batch, int32_t checkpoint_every, void* workspace,
                     size_t workspace_bytes, void* stream) {
  if (!p || !field_in || !grad_out || !grad_c || !grad_rho || !workspace || T < 1 || batch < 1 ||
      T >= (1LL << 31))
    return CBESSFM_EINVAL;
  return cbessfm_backward_gvd(p, field_in, grad_out, grad_in, grad_c, grad_rho, nullptr, T, batch,
                              checkpoint_every, workspace, workspace_bytes, stream);
}

int cbessfm_backward_gvd(cbessfm_plan_t* p, const void* field_in, const void* grad_out, void* grad_in,
                         float* grad_c, float* grad_rho, double* grad_gvd, int64_t T, int32_t batch,
                         int32_t checkpoint_every, void* workspace, size_t workspace_bytes, void* stream) {
  if (!p || !field_in || !grad_out || !grad_c || !grad_rho || !workspace || T < 1 || batch < 1 ||
      T >= (1LL << 31))
    return CBESSFM_EINVAL;
  if (p->nlpr != CBESSFM_NLPR_AVERAGED) return CBESSFM_EUNSUPPORTED;  // the adjoint covers eq. (15)
  if (p->stream)
    return cbessfm::launch_stream_backward(p, field_in, grad_out, grad_in, grad_c, grad_rho, grad_gvd, T, batch,
                                           checkpoint_every, workspace, workspace_bytes,
                                           static_cast<hipStream_t>(stream));
  return cbessfm::launch_backward(p, field_in, grad_out, grad_in, grad_c, grad_rho, grad_gvd, T, batch,
                                  checkpoint_every, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int cbessfm_backward_static(cbessfm_plan_t* p, const void* field_in, const void* grad_out, void* grad_in,
                            float* grad_c, float* grad_rho, int64_t T, int32_t batch, int32_t checkpoint_every,
                            void* stream) {
  if (!p || !field_in || !grad_out || !grad_c || !grad_rho || T < 1 || batch < 1 || T >= (1LL << 31))
    return CBESSFM_EINVAL;
  if (p->nlpr != CBESSFM_NLPR_AVERAGED) return CBESSFM_EUNSUPPORTED;
  const size_t need = p->stream ? cbessfm::stream_bwd_layout(p, T, batch, checkpoint_every, grad_in != nullptr).bytes
                                : cbessfm::bwd_layout(p, T, batch, checkpoint_every).bytes;
  if (need > (size_t)CBESSFM_STATIC_SCRATCH_BYTES) return CBESSFM_EWORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return CBESSFM_EHIP;
  if (dev != p->device) return CBESSFM_EINVAL;
  void* ws = nullptr;
  const int rc = cbessfm::static_scratch(dev, &ws);
  if (rc) return rc;
  return cbessfm_backward_gvd(p, field_in, grad_out, grad_in, grad_c, grad_rho, nullptr, T, batch, checkpoint_every,
                              ws, (size_t)CBESSFM_STATIC_SCRATCH_BYTES, stream);
}

}  // extern "C"
