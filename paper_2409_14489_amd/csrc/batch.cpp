// Host side of batched execution: the static team schedule, the batch object
// and the block-length autotuner.
//
// A batch runs many instances (plans with their own link, subband count,
// steps, coefficients, fields and length) in one persistent launch per
// distinct N' up to 8192; instances whose blocks exceed one CU (N' = 2^14 ..
// 2^17, streamed block state) run on the streaming kernels after those
// launches, concurrently on a few side streams forked from and joined back
// to the caller's stream (so the whole run stays graph-capturable); those
// that fit one wave are grouped into classes (N', n_sb, taps) whose steps
// run as one launch per stage over all their blocks.  The persistent
// launches' workgroups form static teams; a team has the width
// (n_sb) of the instances it runs and keeps that width for the whole launch,
// so the exchange protocol of the single-plan kernel carries over unchanged:
// a team owns its exchange slots and round counter and runs its items one
// after the other.  The schedule decides how many teams of each width to
// form (balancing the predicted work per team across widths), puts every team
// on one XCD, and deals items to teams longest-first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <queue>
#include <tuple>
#include <vector>

#include "cbessfm.h"
#include "internal.hpp"

using cbessfm::BatchArgs;
using cbessfm::BatchItem;
using cbessfm::BatchTeam;
using cbessfm::Inst;
using cbessfm::kXcds;

namespace {

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- schedule
struct Job {
  int width;
  long long n_items;
  double cost;  // of one item
};

struct Schedule {
  int grid = 0;
  std::vector<int> wg_team, wg_member;      // per workgroup
  std::vector<int> team_width, team_xcd;    // per team
  std::vector<double> team_load;
  std::vector<std::vector<long long>> team_items;  // global item ids (job-major) in run order
  std::vector<int> item_team, item_rank;           // per global item
  double makespan = 0.0, lower_bound = 0.0;
};

// Builds the schedule; returns 0 or a CBESSFM_E* code.
int build_schedule(const std::vector<Job>& jobs, int slots_per_xcd, Schedule& s) {
  if (slots_per_xcd < 1) return CBESSFM_EINVAL;
  long long total_items = 0;
  double total_area = 0.0, max_item = 0.0;
  std::map<int, double> work;          // width -> summed item cost
  std::map<int, long long> items_of;   // width -> item count
  for (const Job& j : jobs) {
    if (j.width < 1 || j.width > cbessfm::kMaxSubbands || j.n_items < 0 || !(j.cost >= 0.0))
      return CBESSFM_EINVAL;
    if (j.n_items == 0) continue;
    if (j.width > slots_per_xcd) return CBESSFM_EUNSUPPORTED;
    total_items += j.n_items;
    work[j.width] += j.cost * (double)j.n_items;
    items_of[j.width] += j.n_items;
    total_area += j.cost * (double)j.n_items * j.width;
    max_item = std::max(max_item, j.cost);
  }
  if (total_items == 0) return CBESSFM_EINVAL;
  if (total_items >= (1LL << 31)) return CBESSFM_EUNSUPPORTED;

  // ---- teams per width: start with one each (widest first), then keep giving
  // a team to the width with the largest predicted load per team
  std::vector<int> free_slots(kXcds, slots_per_xcd);
  std::map<int, int> teams_of;
  s.team_width.clear();
  s.team_xcd.clear();
  auto place = [&](int w) {
    int best = -1;
    for (int x = 0; x < kXcds; ++x)
      if (free_slots[x] >= w && (best < 0 || free_slots[x] > free_slots[best])) best = x;
    if (best < 0) return false;
    free_slots[best] -= w;
    s.team_width.push_back(w);
    s.team_xcd.push_back(best);
    ++teams_of[w];
    return true;
  };
  for (auto it = work.rbegin(); it != work.rend(); ++it)
    if (!place(it->first)) return CBESSFM_EUNSUPPORTED;
  std::map<int, bool> saturated;
  while (true) {
    int pick = -1;
    double worst = -1.0;
    for (const auto& kv : work) {
      const int w = kv.first;
      if (saturated[w] || teams_of[w] >= items_of[w]) continue;
      const double per_team = kv.second / teams_of[w];
      if (per_team > worst) {
        worst = per_team;
        pick = w;
      }
    }
    if (pick < 0) break;
    if (!place(pick)) saturated[pick] = true;
  }

  // ---- workgroup numbering: XCD x owns workgroups x, x + 8, x + 16, ...
  const int n_teams = (int)s.team_width.size();
  std::vector<int> next_k(kXcds, 0);
  std::vector<std::vector<int>> team_wgs(n_teams);
  int max_wg = -1;
  for (int tm = 0; tm < n_teams; ++tm) {
    const int x = s.team_xcd[tm];
    for (int m = 0; m < s.team_width[tm]; ++m) {
      const int wg = x + kXcds * next_k[x]++;
      team_wgs[tm].push_back(wg);
      max_wg = std::max(max_wg, wg);
    }
  }
  s.grid = max_wg + 1;
  s.wg_team.assign(s.grid, -1);
  s.wg_member.assign(s.grid, -1);
  for (int tm = 0; tm < n_teams; ++tm)
    for (int m = 0; m < s.team_width[tm]; ++m) {
      s.wg_team[team_wgs[tm][m]] = tm;
      s.wg_member[team_wgs[tm][m]] = m;
    }

  // ---- items to teams: longest first onto the least loaded team of the width
  s.team_load.assign(n_teams, 0.0);
  s.team_items.assign(n_teams, {});
  s.item_team.assign(total_items, -1);
  s.item_rank.assign(total_items, -1);
  std::vector<int> order(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) order[j] = (int)j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return jobs[a].cost > jobs[b].cost; });
  std::vector<long long> first_item(jobs.size(), 0);
  for (size_t j = 1; j < jobs.size(); ++j) first_item[j] = first_item[j - 1] + jobs[j - 1].n_items;
  using Entry = std::pair<double, int>;  // (load, team)
  std::map<int, std::priority_queue<Entry, std::vector<Entry>, std::greater<Entry>>> heaps;
  for (int tm = 0; tm < n_teams; ++tm) heaps[s.team_width[tm]].push({0.0, tm});
  for (int j : order) {
    auto& h = heaps[jobs[j].width];
    for (long long k = 0; k < jobs[j].n_items; ++k) {
      Entry e = h.top();
      h.pop();
      const long long id = first_item[j] + k;
      s.item_team[id] = e.second;
      s.item_rank[id] = (int)s.team_items[e.second].size();
      s.team_items[e.second].push_back(id);
      e.first += jobs[j].cost;
      s.team_load[e.second] = e.first;
      h.push(e);
    }
  }
  s.makespan = 0.0;
  for (double l : s.team_load) s.makespan = std::max(s.makespan, l);
  s.lower_bound = std::max(max_item, total_area / ((double)kXcds * slots_per_xcd));
  return CBESSFM_OK;
}

// ---------------------------------------------------------------- item cost
// Predicted time of one block (seconds) for one persistent team.  With a
// device, measured: a probe plan with the given shape runs exactly one block
// per resident team, at 1 and 4 steps, and the time is taken as linear in the
// step count.  Without one, a rough operation-count model.
struct CostKey {
  int device, log_np, nsb, n_chunks;
  bool operator<(const CostKey& o) const {
    return std::tie(device, log_np, nsb, n_chunks) < std::tie(o.device, o.log_np, o.nsb, o.n_chunks);
  }
};
std::mutex g_cost_mu;
std::map<CostKey, std::pair<double, double>> g_cost;  // (time at 0 steps, time per step)

double model_cost(int log_np, int nsb, int n_chunks, int steps) {
  const double np = (double)(1 << log_np);
  const double per_transform = np * log_np * 2.5e-12;
  const double per_step = 4.0 * per_transform * (1.0 + 0.15 * nsb * n_chunks) + 2.0e-6;
  return 3.0 * per_transform + 4.0e-6 + steps * per_step;
}

int team_capacity(int log_np, int nsb, int* teams, int* slots_per_xcd) {
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return CBESSFM_EHIP;
  if (cbessfm::batch_occupancy_per_cu(log_np, &per_cu) != CBESSFM_OK || per_cu < 1) return CBESSFM_EHIP;
  const int spx = per_cu * prop.multiProcessorCount / kXcds;
  if (slots_per_xcd) *slots_per_xcd = spx;
  if (teams) *teams = (spx / nsb) * kXcds;
  return CBESSFM_OK;
}

int probe_time(const cbessfm_link* link, int log_np, int nsb, int n_taps, int steps, double* out_s) {
  int teams = 0;
  int rc = team_capacity(log_np, nsb, &teams, nullptr);
  if (rc) return rc;
  cbessfm_subbands sb{nsb, 1 << log_np, 0, CBESSFM_FIR_AUTO, 0};
  std::vector<float> c((size_t)steps * nsb * nsb * n_taps, 0.0f);
  for (int s = 0; s < steps; ++s)
    for (int i = 0; i < nsb; ++i)
      for (int l = 0; l < nsb; ++l) c[(((size_t)s * nsb + i) * nsb + l) * n_taps + n_taps / 2] = 30.0f;
  cbessfm_coeffs co{n_taps, c.data(), 0};
  cbessfm_plan_t* p = nullptr;
  rc = cbessfm_plan(&p, link, &sb, steps, 0.5, &co);
  if (rc) return rc;
  const long long T = (long long)teams * nsb * (1 << log_np);  // one block per team
  void* buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 1e30;
  rc = CBESSFM_EHIP;
  if (hipMalloc(&buf, (size_t)2 * 2 * T * sizeof(float2)) == hipSuccess &&
      hipMemset(buf, 0, (size_t)2 * 2 * T * sizeof(float2)) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
      hipEventCreate(&e1) == hipSuccess) {
    char* in = static_cast<char*>(buf);
    char* out = in + (size_t)2 * T * sizeof(float2);
    rc = cbessfm_run(p, in, out, T, 1, nullptr);  // warm-up
    for (int r = 0; r < 3 && rc == CBESSFM_OK; ++r) {
      float ms = 0.0f;
      if (hipEventRecord(e0, nullptr) != hipSuccess) rc = CBESSFM_EHIP;
      if (!rc) rc = cbessfm_run(p, in, out, T, 1, nullptr);
      if (!rc && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = CBESSFM_EHIP;
      if (!rc) best = std::min(best, 1e-3 * ms);
    }
    if (!rc) rc = cbessfm_status(p);
  }
  // release: failures here cannot change the measurement
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) (void)hipFree(buf);
  cbessfm_destroy(p);
  if (!rc) *out_s = best;
  return rc;
}

enum CostMode { kModel, kMeasure, kCachedOrModel };

int item_cost(const cbessfm_link* link, int log_np, int nsb, int n_taps, int steps, CostMode mode, double* out) {
  const int n_chunks = (n_taps + cbessfm::kTapChunk - 1) / cbessfm::kTapChunk;
  if (mode == kModel) {
    *out = model_cost(log_np, nsb, n_chunks, steps);
    return CBESSFM_OK;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CBESSFM_EHIP;
  const CostKey key{dev, log_np, nsb, n_chunks};
  {
    std::lock_guard<std::mutex> g(g_cost_mu);
    auto it = g_cost.find(key);
    if (it != g_cost.end()) {
      *out = it->second.first + steps * it->second.second;
      return CBESSFM_OK;
    }
  }
  if (mode == kCachedOrModel) {
    *out = model_cost(log_np, nsb, n_chunks, steps);
    return CBESSFM_OK;
  }
  double t1 = 0.0, t4 = 0.0;
  const int taps = n_chunks * cbessfm::kTapChunk - 1 < (1 << log_np) ? n_chunks * cbessfm::kTapChunk - 1 : 1;
  int rc = probe_time(link, log_np, nsb, taps, 1, &t1);
  if (!rc) rc = probe_time(link, log_np, nsb, taps, 4, &t4);
  if (rc) return rc;
  const double per_step = std::max(0.0, (t4 - t1) / 3.0);
  const double base = std::max(0.0, t1 - per_step);
  {
    std::lock_guard<std::mutex> g(g_cost_mu);
    g_cost[key] = {base, per_step};
  }
  *out = base + steps * per_step;
  return CBESSFM_OK;
}

// Operation-count model of one streamed block (seconds): each step moves the
// block state through device memory about six times (row pass in and out,
// intensity, filter, rotation in and out) at an assumed 4 TB/s, plus the
// input and output stages and a small per-step share of launch latency.
double stream_block_cost(int log_np, int nsb, int steps) {
  const double state = (double)nsb * (double)(1 << log_np) * 2.0 * sizeof(float2);
  return (6.0 * steps + 4.0) * state / 4e12 + 2e-6 * steps;
}

// Measured time of one streamed block (seconds), linear in the step count: a
// probe plan runs as many blocks as 256 MB of block state holds (at most one
// wave) at 1 and 4 steps.  Cached per device and shape like item_cost.
std::map<CostKey, std::pair<double, double>> g_stream_cost;

int stream_probe_time(const cbessfm_link* link, int log_np, int nsb, int n_taps, int steps, double* out_s) {
  cbessfm_subbands sb{nsb, 1 << log_np, 0, CBESSFM_FIR_AUTO, 0};
  std::vector<float> c((size_t)steps * nsb * nsb * n_taps, 0.0f);
  for (int s = 0; s < steps; ++s)
    for (int i = 0; i < nsb; ++i)
      for (int l = 0; l < nsb; ++l) c[(((size_t)s * nsb + i) * nsb + l) * n_taps + n_taps / 2] = 30.0f;
  cbessfm_coeffs co{n_taps, c.data(), 0};
  cbessfm_plan_t* p = nullptr;
  int rc = cbessfm_plan(&p, link, &sb, steps, 0.5, &co);
  if (rc) return rc;
  const long long N = (long long)nsb << log_np;
  const double state = (double)N * 2.0 * sizeof(float2);
  const int blocks = std::max(1, std::min<int>(p->st_blocks, (int)(256.0 * (1 << 20) / state)));
  const long long T = (long long)blocks * N;  // no overlap: one block per N samples
  void* buf = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 1e30;
  rc = CBESSFM_EHIP;
  if (hipMalloc(&buf, (size_t)2 * 2 * T * sizeof(float2)) == hipSuccess &&
      hipMemset(buf, 0, (size_t)2 * 2 * T * sizeof(float2)) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
      hipEventCreate(&e1) == hipSuccess) {
    char* in = static_cast<char*>(buf);
    char* out = in + (size_t)2 * T * sizeof(float2);
    rc = cbessfm_run(p, in, out, T, 1, nullptr);  // warm-up
    for (int r = 0; r < 3 && rc == CBESSFM_OK; ++r) {
      float ms = 0.0f;
      if (hipEventRecord(e0, nullptr) != hipSuccess) rc = CBESSFM_EHIP;
      if (!rc) rc = cbessfm_run(p, in, out, T, 1, nullptr);
      if (!rc && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                  hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = CBESSFM_EHIP;
      if (!rc) best = std::min(best, 1e-3 * ms);
    }
    if (!rc) rc = cbessfm_status(p);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (buf) (void)hipFree(buf);
  cbessfm_destroy(p);
  if (!rc) *out_s = best / blocks;
  return rc;
}

int stream_item_cost(const cbessfm_link* link, int log_np, int nsb, int n_taps, int steps, bool measure,
                     double* out) {
  if (!measure) {
    *out = stream_block_cost(log_np, nsb, steps);
    return CBESSFM_OK;
  }
  const int n_chunks = (n_taps + cbessfm::kTapChunk - 1) / cbessfm::kTapChunk;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CBESSFM_EHIP;
  const CostKey key{dev, log_np, nsb, n_chunks};
  {
    std::lock_guard<std::mutex> g(g_cost_mu);
    auto it = g_stream_cost.find(key);
    if (it != g_stream_cost.end()) {
      *out = it->second.first + steps * it->second.second;
      return CBESSFM_OK;
    }
  }
  const int taps = n_chunks * cbessfm::kTapChunk - 1;
  double t1 = 0.0, t4 = 0.0;
  int rc = stream_probe_time(link, log_np, nsb, taps, 1, &t1);
  if (!rc) rc = stream_probe_time(link, log_np, nsb, taps, 4, &t4);
  if (rc) return rc;
  const double per_step = std::max(0.0, (t4 - t1) / 3.0);
  const double base = std::max(0.0, t1 - per_step);
  {
    std::lock_guard<std::mutex> g(g_cost_mu);
    g_stream_cost[key] = {base, per_step};
  }
  *out = base + steps * per_step;
  return CBESSFM_OK;
}

long long dispersion_memory(const cbessfm_link* link) {
  const double beta2 = std::fabs(link->beta2_ps2_km) * 1e-24;  // s^2/km
  const double L = link->span_km * link->n_spans;
  const double R = link->sample_rate_hz;
  const double m = 2.0 * kPi * beta2 * L * R * R;
  long long v = (long long)std::ceil(m);
  if (v & 1) ++v;
  return v;
}

}  // namespace

// ---------------------------------------------------------------- batch object
struct cbessfm_batch {
  int device = 0;
  struct Launch {
    int log_np = 0, grid = 0;
    BatchArgs args{};
  };
  std::vector<Launch> launches;
  // instances whose plans stream their block state (N' >= 2^14): run by the
  // streaming kernels after the persistent launches
  std::vector<cbessfm_instance> streamed;
  // Streamed instances whose blocks fit one wave of their own plan (and whose
  // plan no other instance uses) are grouped into classes of equal N', n_sb
  // and taps: the block input and output of a class, and each of its steps,
  // are one launch per stage over the blocks of all its instances (for a
  // step, those still stepping: members by step count, descending, so their
  // blocks are a prefix of the block table).  The other streamed instances
  // run one by one.
  struct StreamClass {
    int log_np = 0, n_sb = 0, n_taps = 0, tap_pad = 0, max_steps = 0;
    std::vector<int> members;     // indices into streamed
    std::vector<int> active;      // [max_steps] blocks taking part in step s
    cbessfm::StreamBlk* d_blks = nullptr;
  };
  std::vector<StreamClass> classes;
  // units run on the side streams: a class (k < classes.size()) or the lone
  // streamed instance k - classes.size()
  std::vector<int> lone;     // indices into streamed
  std::vector<int> unit_side;
  // side streams (default priority) and fork / join events: the units run
  // concurrently, instances of one plan on one stream
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  cbessfm_batch_info info{};
  std::vector<void*> allocs;
  unsigned* d_abort = nullptr;
  int* d_err = nullptr;
  uint64_t* d_xp = nullptr;
  unsigned* d_epoch = nullptr;
  size_t xp_words = 0, n_epoch = 0;
};

namespace {

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + nb && pb < pa + na;
}

int reset_exchange(cbessfm_batch_t* b) {
  if (hipMemset(b->d_err, 0, sizeof(int)) != hipSuccess || hipMemset(b->d_abort, 0, sizeof(unsigned)) != hipSuccess ||
      hipMemset(b->d_xp, 0, b->xp_words * sizeof(uint64_t)) != hipSuccess ||
      hipMemset(b->d_epoch, 0, b->n_epoch * sizeof(unsigned)) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return CBESSFM_EHIP;
  return CBESSFM_OK;
}

}  // namespace

extern "C" {

int cbessfm_schedule(const cbessfm_sched_job* jobs, int32_t n_jobs, int32_t slots_per_xcd, int32_t max_wg,
                     int32_t* wg_team, int32_t* wg_member, int32_t* item_team, int32_t* item_rank,
                     cbessfm_sched_stats* stats) {
  if (!jobs || n_jobs < 1 || !stats) return CBESSFM_EINVAL;
  std::vector<Job> js(n_jobs);
  for (int j = 0; j < n_jobs; ++j) js[j] = Job{jobs[j].width, jobs[j].n_items, jobs[j].cost};
  Schedule s;
  int rc = build_schedule(js, slots_per_xcd, s);
  if (rc) return rc;
  if (s.grid > max_wg) return CBESSFM_EINVAL;
  stats->grid = s.grid;
  stats->n_teams = (int32_t)s.team_width.size();
  stats->makespan = s.makespan;
  stats->lower_bound = s.lower_bound;
  if (wg_team && wg_member)
    for (int w = 0; w < s.grid; ++w) {
      wg_team[w] = s.wg_team[w];
      wg_member[w] = s.wg_member[w];
    }
  if (item_team && item_rank)
    for (size_t i = 0; i < s.item_team.size(); ++i) {
      item_team[i] = s.item_team[i];
      item_rank[i] = s.item_rank[i];
    }
  return CBESSFM_OK;
}

int cbessfm_autotune(const cbessfm_link* link, int32_t n_sb, int32_t steps, int32_t n_taps, int64_t T,
                     int32_t batch, int32_t flags, cbessfm_tuning* out) {
  if (!link || !out || n_sb < 1 || n_sb > cbessfm::kMaxSubbands || steps < 1 || n_taps < 1 || !(n_taps & 1) ||
      n_taps > cbessfm::kMaxTaps || T < 1 || batch < 1 || (flags & ~CBESSFM_TUNE_MEASURE))
    return CBESSFM_EINVAL;
  if (!(link->span_km > 0.0) || link->n_spans < 1 || !(link->sample_rate_hz > 0.0) ||
      !std::isfinite(link->beta2_ps2_km))
    return CBESSFM_EINVAL;
  const bool measure = (flags & CBESSFM_TUNE_MEASURE) != 0;
  const long long mem = dispersion_memory(link);
  std::memset(out, 0, sizeof(*out));
  out->memory = mem > 0x7fffffff ? 0x7fffffff : (int32_t)mem;
  out->measured = measure ? 1 : 0;
  double best = 1e300;
  for (int log_np = 8; log_np <= 13; ++log_np) {
    const int np = 1 << log_np;
    if (n_taps > np) continue;
    const long long N = (long long)n_sb * np;
    const bool covers = mem < N;
    const bool last = log_np == 13;
    if (!covers && !(last && out->block_sb == 0)) continue;
    long long ov = covers ? mem : std::min(mem, N / 2);
    ov &= ~1LL;
    const long long hop = N - ov;
    const long long items = (long long)batch * ((T + hop - 1) / hop);
    int teams = 0;
    if (measure) {
      int rc = team_capacity(log_np, n_sb, &teams, nullptr);
      if (rc) return rc;
    } else {
      teams = (256 * (log_np <= 12 ? 2 : 1) / (kXcds * n_sb)) * kXcds;
    }
    if (teams < 1) continue;
    double t_item = 0.0;
    int rc = item_cost(link, log_np, n_sb, n_taps, steps, measure ? kMeasure : kModel, &t_item);
    if (rc) return rc;
    const double pred = (double)((items + teams - 1) / teams) * t_item;
    if (pred < best) {
      best = pred;
      out->block_sb = np;
      out->overlap = (int32_t)ov;
      out->covered = covers ? 1 : 0;
      out->predicted_s = pred;
    }
  }
  // The smallest streamed block (N' = 2^14 .. 2^17) that covers the memory,
  // else the largest with N_ov = min(memory, N / 2): taken when no persistent
  // block covers the memory, or when it covers it and is predicted faster
  // (a persistent block whose overlap is most of it does little useful work
  // per block).
  const bool have = out->block_sb && out->covered;
  for (int log_np = cbessfm::kStreamMinLog; log_np <= cbessfm::kStreamMaxLog; ++log_np) {
    const long long N = (long long)n_sb << log_np;
    const bool covers = mem < N;
    if (!covers && log_np < cbessfm::kStreamMaxLog) continue;
    if (have && !covers) break;
    if (n_taps > (1 << log_np)) break;
    long long ov = covers ? mem : std::min(mem, N / 2);
    ov &= ~1LL;
    const long long items = (long long)batch * ((T + (N - ov) - 1) / (N - ov));
    double t_blk = 0.0;
    const int rc = stream_item_cost(link, log_np, n_sb, n_taps, steps, measure, &t_blk);
    if (rc) return rc;
    const double pred = (double)items * t_blk;
    if (!have || pred < best) {
      out->block_sb = 1 << log_np;
      out->overlap = (int32_t)ov;
      out->covered = covers ? 1 : 0;
      out->predicted_s = pred;
    }
    break;
  }
  return out->block_sb ? CBESSFM_OK : CBESSFM_EUNSUPPORTED;
}

void cbessfm_batch_destroy(cbessfm_batch_t* b) {
  if (!b) return;
  // a void release path: HIP errors are not reportable here
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(b->device);
  for (void* p : b->allocs) (void)hipFree(p);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipStream_t st : b->side) (void)hipStreamDestroy(st);
  (void)hipSetDevice(prev);
  delete b;
}

int cbessfm_batch_create(cbessfm_batch_t** out, const cbessfm_instance* inst, int32_t n) {
  if (!out) return CBESSFM_EINVAL;
  *out = nullptr;
  if (!inst || n < 1) return CBESSFM_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CBESSFM_EHIP;
  // ---- validation
  for (int i = 0; i < n; ++i) {
    const cbessfm_instance& a = inst[i];
    if (!a.plan || !a.field_in || !a.field_out || a.T < 1 || a.batch < 1 || a.T >= (1LL << 31))
      return CBESSFM_EINVAL;
    if (a.plan->device != dev) return CBESSFM_EINVAL;
    if (a.plan->nlpr != CBESSFM_NLPR_AVERAGED) return CBESSFM_EUNSUPPORTED;  // batches run eq. (15)
    const size_t bytes = (size_t)a.batch * 2 * a.T * sizeof(float2);
    if (overlaps(a.field_in, bytes, a.field_out, bytes)) return CBESSFM_EINVAL;
    for (int j = 0; j < i; ++j) {
      const size_t bj = (size_t)inst[j].batch * 2 * inst[j].T * sizeof(float2);
      if (overlaps(a.field_out, bytes, inst[j].field_out, bj) || overlaps(a.field_out, bytes, inst[j].field_in, bj) ||
          overlaps(a.field_in, bytes, inst[j].field_out, bj))
        return CBESSFM_EINVAL;
    }
  }
  cbessfm_batch_t* b = new (std::nothrow) cbessfm_batch_t();
  if (!b) return CBESSFM_ENOMEM;
  b->device = dev;

  // ---- one launch per N' of the persistent kernels; streamed plans apart
  std::map<int, std::vector<int>> by_np;
  long long stream_items = 0;
  double stream_time = 0.0;
  for (int i = 0; i < n; ++i) {
    const cbessfm_plan_t* p = inst[i].plan;
    if (p->stream) {
      b->streamed.push_back(inst[i]);
      const long long nblk = (inst[i].T + p->hop - 1) / p->hop;
      stream_items += (long long)inst[i].batch * nblk;
      stream_time += (double)inst[i].batch * nblk * stream_block_cost(p->log_np, p->sb.n_sb, p->steps);
    } else {
      by_np[p->log_np].push_back(i);
    }
  }
  struct Built {
    int log_np;
    Schedule s;
    std::vector<int> members;  // instance ids of this launch
    std::vector<Inst> insts;
  };
  std::vector<Built> built;
  size_t xp_words = 0, n_epoch = 0;
  int rc = CBESSFM_OK;
  for (auto& kv : by_np) {
    Built bt;
    bt.log_np = kv.first;
    bt.members = kv.second;
    int spx = 0;
    rc = team_capacity(bt.log_np, 1, nullptr, &spx);
    if (rc) break;
    std::vector<Job> jobs;
    for (int i : bt.members) {
      const cbessfm_instance& a = inst[i];
      const cbessfm_plan_t* p = a.plan;
      Inst d;
      cbessfm::fill_inst(p, a.field_in, a.field_out, a.T, a.batch, d);
      bt.insts.push_back(d);
      double cost = 0.0;
      rc = item_cost(&p->link, p->log_np, p->sb.n_sb, p->n_taps, p->steps, kCachedOrModel, &cost);
      if (rc) break;
      jobs.push_back(Job{p->sb.n_sb, (long long)a.batch * d.nblk, cost});
    }
    if (rc) break;
    rc = build_schedule(jobs, spx, bt.s);
    if (rc) break;
    const int np = 1 << bt.log_np;
    for (size_t tm = 0; tm < bt.s.team_width.size(); ++tm) {
      xp_words += (size_t)2 * bt.s.team_width[tm] * 2 * np;
      ++n_epoch;
    }
    built.push_back(std::move(bt));
  }
  if (rc) {
    delete b;
    return rc;
  }

  // ---- device memory: exchange pool, counters, schedule tables
  bool ok = true;
  auto alloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (ok && hipMalloc(&p, bytes) != hipSuccess) {
      ok = false;
      p = nullptr;
    }
    if (p) b->allocs.push_back(p);
    return p;
  };
  b->xp_words = xp_words;
  b->n_epoch = n_epoch;
  b->d_xp = static_cast<uint64_t*>(alloc(std::max<size_t>(1, xp_words) * sizeof(uint64_t)));
  b->d_epoch = static_cast<unsigned*>(alloc(std::max<size_t>(1, n_epoch) * sizeof(unsigned)));
  b->d_abort = static_cast<unsigned*>(alloc(sizeof(unsigned)));
  b->d_err = static_cast<int*>(alloc(sizeof(int)));
  if (!ok || reset_exchange(b)) {
    cbessfm_batch_destroy(b);
    return ok ? CBESSFM_EHIP : CBESSFM_ENOMEM;
  }
  size_t xp_off = 0, ep_off = 0;
  long long total_items = 0;
  int total_teams = 0, total_wg = 0;
  double makespan = 0.0, bound = 0.0;
  for (Built& bt : built) {
    const int np = 1 << bt.log_np;
    const Schedule& s = bt.s;
    const int n_teams = (int)s.team_width.size();
    std::vector<int2> wg(s.grid);
    for (int w = 0; w < s.grid; ++w) wg[w] = make_int2(s.wg_team[w], s.wg_member[w]);
    // items in team order; item ids are job-major over this launch's members
    std::vector<long long> first_item(bt.members.size(), 0);
    for (size_t j = 1; j < bt.members.size(); ++j)
      first_item[j] = first_item[j - 1] + (long long)inst[bt.members[j - 1]].batch * bt.insts[j - 1].nblk;
    std::vector<BatchTeam> teams(n_teams);
    std::vector<BatchItem> items;
    for (int tm = 0; tm < n_teams; ++tm) {
      BatchTeam& t = teams[tm];
      t.width = s.team_width[tm];
      t.first = (int)items.size();
      t.count = (int)s.team_items[tm].size();
      t.epoch_slot = (int)(ep_off + tm);
      t.xp_off = (long long)xp_off;
      xp_off += (size_t)2 * t.width * 2 * np;
      unsigned rounds = 0;
      for (long long id : s.team_items[tm]) {
        const size_t j = std::upper_bound(first_item.begin(), first_item.end(), id) - first_item.begin() - 1;
        BatchItem it;
        it.inst = (int)j;
        it.sub = (int)(id - first_item[j]);
        it.round_off = rounds;
        rounds += cbessfm::fwd_rounds(bt.insts[j].steps, 1u);
        items.push_back(it);
      }
      t.rounds = rounds;
    }
    ep_off += n_teams;
    Inst* d_insts = static_cast<Inst*>(alloc(sizeof(Inst) * bt.insts.size()));
    int2* d_wg = static_cast<int2*>(alloc(sizeof(int2) * wg.size()));
    BatchTeam* d_teams = static_cast<BatchTeam*>(alloc(sizeof(BatchTeam) * teams.size()));
    BatchItem* d_items = static_cast<BatchItem*>(alloc(sizeof(BatchItem) * items.size()));
    if (!ok || hipMemcpy(d_insts, bt.insts.data(), sizeof(Inst) * bt.insts.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(d_wg, wg.data(), sizeof(int2) * wg.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(d_teams, teams.data(), sizeof(BatchTeam) * teams.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice)) {
      cbessfm_batch_destroy(b);
      return ok ? CBESSFM_EHIP : CBESSFM_ENOMEM;
    }
    cbessfm_batch::Launch L;
    L.log_np = bt.log_np;
    L.grid = s.grid;
    L.args.insts = d_insts;
    L.args.wg = d_wg;
    L.args.teams = d_teams;
    L.args.items = d_items;
    L.args.epoch = b->d_epoch;
    L.args.xp = b->d_xp;
    L.args.ctl.abort = b->d_abort;
    L.args.ctl.err = b->d_err;
    L.args.ctl.spin_limit = 1u << 22;
    b->launches.push_back(L);
    total_items += (long long)items.size();
    total_teams += n_teams;
    total_wg += s.grid;
    makespan += s.makespan;
    bound += s.lower_bound;
  }
  // ---- streamed instances: classes, lone instances, side streams (units
  // longest first onto the least loaded stream, lone instances sharing a plan
  // on the same stream)
  if (!b->streamed.empty()) {
    const size_t ns = b->streamed.size();
    std::vector<double> cost(ns);
    std::map<const cbessfm_plan_t*, int> uses;
    for (size_t k = 0; k < ns; ++k) {
      const cbessfm_instance& a = b->streamed[k];
      const cbessfm_plan_t* p = a.plan;
      cost[k] = (double)a.batch * ((a.T + p->hop - 1) / p->hop) * stream_block_cost(p->log_np, p->sb.n_sb, p->steps);
      ++uses[p];
    }
    std::map<std::array<int, 4>, int> class_of;
    for (size_t k = 0; k < ns; ++k) {
      const cbessfm_instance& a = b->streamed[k];
      const cbessfm_plan_t* p = a.plan;
      if (uses[p] != 1 || !cbessfm::stream_single_wave(p, a.T, a.batch)) {
        b->lone.push_back((int)k);
        continue;
      }
      const std::array<int, 4> key{p->log_np, p->sb.n_sb, p->n_taps, p->tap_pad};
      auto it = class_of.find(key);
      if (it == class_of.end()) {
        it = class_of.emplace(key, (int)b->classes.size()).first;
        cbessfm_batch::StreamClass c;
        c.log_np = key[0];
        c.n_sb = key[1];
        c.n_taps = key[2];
        c.tap_pad = key[3];
        b->classes.push_back(c);
      }
      b->classes[it->second].members.push_back((int)k);
    }
    std::vector<double> unit_cost;
    for (auto& c : b->classes) {
      std::stable_sort(c.members.begin(), c.members.end(), [&](int x, int y) {
        return b->streamed[x].plan->steps > b->streamed[y].plan->steps;
      });
      c.max_steps = b->streamed[c.members.front()].plan->steps;
      std::vector<cbessfm::StreamBlk> blks;
      std::vector<int> nb_of;
      double uc = 0.0;
      for (int k : c.members) {
        const cbessfm_instance& a = b->streamed[k];
        const long long nb = (long long)a.batch * ((a.T + a.plan->hop - 1) / a.plan->hop);
        const size_t at = blks.size();
        blks.resize(at + (size_t)nb);
        cbessfm::stream_blocks(a.plan, a.field_in, a.field_out, a.T, a.batch, blks.data() + at);
        nb_of.push_back((int)nb);
        uc += cost[k];
      }
      c.active.assign(c.max_steps, 0);
      for (size_t j = 0; j < c.members.size(); ++j)
        for (int st = 0; st < b->streamed[c.members[j]].plan->steps; ++st) c.active[st] += nb_of[j];
      c.d_blks = static_cast<cbessfm::StreamBlk*>(alloc(blks.size() * sizeof(cbessfm::StreamBlk)));
      if (ok && hipMemcpy(c.d_blks, blks.data(), blks.size() * sizeof(cbessfm::StreamBlk), hipMemcpyHostToDevice) !=
                    hipSuccess)
        ok = false;
      unit_cost.push_back(uc);
    }
    for (int k : b->lone) unit_cost.push_back(cost[k]);
    if (!ok) {
      cbessfm_batch_destroy(b);
      return CBESSFM_EHIP;
    }
    constexpr int kSideStreams = 4;
    const int n_units = (int)unit_cost.size();
    const int n_side = std::min<int>(kSideStreams, n_units);
    std::vector<double> load(n_side, 0.0);
    std::vector<int> order(n_units);
    for (int u = 0; u < n_units; ++u) order[u] = u;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return unit_cost[x] > unit_cost[y]; });
    b->unit_side.assign(n_units, 0);
    std::map<const cbessfm_plan_t*, int> plan_side;
    const int n_cls = (int)b->classes.size();
    for (int u : order) {
      const cbessfm_plan_t* lp = u >= n_cls ? b->streamed[b->lone[u - n_cls]].plan : nullptr;
      auto it = lp ? plan_side.find(lp) : plan_side.end();
      int sd;
      if (it != plan_side.end()) {
        sd = it->second;
      } else {
        sd = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        if (lp) plan_side[lp] = sd;
      }
      b->unit_side[u] = sd;
      load[sd] += unit_cost[u];
    }
    bool sok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < n_side && sok; ++k) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      sok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
      if (sok) b->side.push_back(st);
      sok = sok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
      if (sok) b->join.push_back(ev);
    }
    if (!sok) {
      cbessfm_batch_destroy(b);
      return CBESSFM_EHIP;
    }
    stream_time = *std::max_element(load.begin(), load.end());
  }
  b->info.launches = (int32_t)b->launches.size();
  b->info.teams = total_teams;
  b->info.workgroups = total_wg;
  b->info.items = total_items + stream_items;
  b->info.makespan_s = makespan + stream_time;
  b->info.lower_bound_s = bound + stream_time;
  b->info.streamed = (int32_t)b->streamed.size();
  b->info.streamed_items = stream_items;
  b->info.stream_classes = (int32_t)b->classes.size();
  b->info.stream_lone = (int32_t)b->lone.size();
  {
    long long k = (long long)b->launches.size();
    for (const auto& c : b->classes)
      k += cbessfm::stream_launches(b->streamed[c.members.front()].plan, c.max_steps);
    for (int m : b->lone) {
      const cbessfm_instance& a = b->streamed[m];
      const long long items = (long long)a.batch * ((a.T + a.plan->hop - 1) / a.plan->hop);
      const long long waves = (items + a.plan->st_blocks - 1) / a.plan->st_blocks;
      k += waves * cbessfm::stream_launches(a.plan, a.plan->steps);
    }
    b->info.kernel_launches = (int32_t)std::min<long long>(k, 0x7fffffff);
  }
  *out = b;
  return CBESSFM_OK;
}

int cbessfm_batch_run(cbessfm_batch_t* b, void* stream) {
  if (!b) return CBESSFM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (const auto& L : b->launches) {
    const int rc = cbessfm::launch_batch(L.log_np, L.args, L.grid, s);
    if (rc) return rc;
  }
  if (b->streamed.empty()) return CBESSFM_OK;
  // streamed instances: fork to the side streams after the persistent
  // launches, join back (under graph capture this records a fork / join of
  // kernel nodes)
  if (hipEventRecord(b->fork, s) != hipSuccess) return CBESSFM_EHIP;
  for (hipStream_t st : b->side)
    if (hipStreamWaitEvent(st, b->fork, 0) != hipSuccess) return CBESSFM_EHIP;
  int rc = CBESSFM_OK;
  const int n_cls = (int)b->classes.size();
  for (int u = 0; u < (int)b->unit_side.size() && !rc; ++u) {
    hipStream_t st = b->side[b->unit_side[u]];
    if (u >= n_cls) {
      const cbessfm_instance& a = b->streamed[b->lone[u - n_cls]];
      rc = cbessfm::launch_stream_forward(a.plan, a.field_in, a.field_out, a.T, a.batch, st);
      continue;
    }
    const auto& c = b->classes[u];
    const cbessfm_plan_t* p0 = b->streamed[c.members.front()].plan;
    rc = cbessfm::stream_class_input(p0, c.d_blks, c.active.front(), st);
    for (int step = 0; step < c.max_steps && !rc; ++step)
      rc = cbessfm::stream_class_step(c.log_np, c.n_sb, c.n_taps, c.tap_pad, step, c.d_blks, c.active[step], st);
    if (!rc) rc = cbessfm::stream_class_output(p0, c.d_blks, c.active.front(), st);
  }
  // join every side stream even after a failed launch
  for (size_t k = 0; k < b->side.size(); ++k)
    if (hipEventRecord(b->join[k], b->side[k]) != hipSuccess || hipStreamWaitEvent(s, b->join[k], 0) != hipSuccess)
      rc = rc ? rc : CBESSFM_EHIP;
  return rc;
}

int cbessfm_batch_describe(const cbessfm_batch_t* b, cbessfm_batch_info* out) {
  if (!b || !out) return CBESSFM_EINVAL;
  *out = b->info;
  return CBESSFM_OK;
}

int cbessfm_batch_status(cbessfm_batch_t* b) {
  if (!b) return CBESSFM_EINVAL;
  if (hipSetDevice(b->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) return CBESSFM_EHIP;
  int err = 0;
  if (hipMemcpy(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return CBESSFM_EHIP;
  if (err && reset_exchange(b)) return CBESSFM_EHIP;
  return err;
}

}  // extern "C"
