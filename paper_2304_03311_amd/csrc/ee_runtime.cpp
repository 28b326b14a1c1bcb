// ee_runtime.cpp -- host runtime of the C ABI declared in include/ee.h.
//
// Validates job descriptions, builds the geometry constants and the uint32
// Metropolis threshold tables on the host (FP64 libm exp; compiled with
// -ffp-contract=off so the expression is evaluated exactly as written),
// lays the job out in the caller's arena, runs the job state machine and
// launches the kernels of ee_kernels.hip.  The batch path keeps a plan per
// job set (device work queue + job table + a HIP graph of the launches).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <unordered_map>
#include <mutex>
#include <string>
#include <vector>

#include "ee_internal.hpp"

namespace {

thread_local std::string g_err;

ee_status fail(ee_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(EE_EHIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, \
                  __LINE__);                                                            \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

enum State { CREATED = 0, SERVED = 1, DONE = 2 };  // SERVED: submitted to a server, not yet done

struct Layout {
  size_t off_jobdev, off_selfptr, off_result, off_ramp, off_work, off_spins, total;
  int H, G, R, traj_words, packed_words;
  size_t storage_words_per_traj;
};

// Metropolis threshold of an energy cost K (units of beta/N): accept iff
// u <= U with u a uint32 uniform, so P(accept) = (U+1)/2^32 ~ exp(-2 beta K/N).
uint32_t threshold(double beta, int64_t K, int32_t N) {
  if (beta * (double)K <= 0.0) return 0xFFFFFFFFu;
  const double x = (2.0 * beta * (double)K) / (double)N;
  const double p = std::exp(-x);
  double f = std::floor(std::ldexp(p, 32));
  if (f >= 4294967296.0) return 0xFFFFFFFFu;
  if (f < 1.0) f = 1.0;
  return (uint32_t)(f - 1.0);
}

ee_status validate(const ee_job_desc* d) {
  if (!d) return fail(EE_EINVAL, "desc is NULL");
  if (d->dim != 2 && d->dim != 3) return fail(EE_EINVAL, "dim must be 2 or 3 (got %d)", d->dim);
  if (d->lt < 2 || (d->lt & 1)) return fail(EE_EINVAL, "lt must be even and >= 2 (got %d)", d->lt);
  if (d->lx < 2 || (d->lx & 1)) return fail(EE_EINVAL, "lx must be even and >= 2 (got %d)", d->lx);
  if (d->dim == 2 && d->ly != 1) return fail(EE_EINVAL, "ly must be 1 in 2D (got %d)", d->ly);
  if (d->dim == 3 && (d->ly < 2 || (d->ly & 1)))
    return fail(EE_EINVAL, "ly must be even and >= 2 in 3D (got %d)", d->ly);
  if (d->n_replicas < 2 || d->n_replicas > (1 << 20))
    return fail(EE_EINVAL, "n_replicas must be in [2, 2^20] (got %d)", d->n_replicas);
  if (!(d->beta >= 0.0) || !std::isfinite(d->beta))
    return fail(EE_EINVAL, "beta must be finite and >= 0");
  if (d->flags & EE_FLAG_WHOLE) {
    if (d->l < 1 || d->l > d->lx)
      return fail(EE_EINVAL, "the whole-region protocol needs 1 <= l <= lx (got %d)", d->l);
    if (d->flags & EE_FLAG_SUBSETS) return fail(EE_EINVAL, "EE_FLAG_WHOLE and EE_FLAG_SUBSETS exclude each other");
  } else if (d->l < 0 || d->l >= d->lx) {
    return fail(EE_EINVAL, "l must satisfy 0 <= l < lx (got %d)", d->l);
  }
  if (d->n_step < 1) return fail(EE_EINVAL, "n_step must be >= 1 (got %d)", d->n_step);
  if (d->n_traj < 1 || d->n_traj > 65535)
    return fail(EE_EINVAL, "n_traj must be in [1, 65535] (got %d)", d->n_traj);
  if (d->spin_format != EE_SPINS_INT8 && d->spin_format != EE_SPINS_BITPACKED)
    return fail(EE_EINVAL, "unknown spin_format %d", d->spin_format);
  if (d->flags & ~(EE_FLAG_REVERSE | EE_FLAG_SUBSETS | EE_FLAG_WHOLE))
    return fail(EE_EINVAL, "unknown flags 0x%x", d->flags);
  if ((d->flags & EE_FLAG_SUBSETS) && d->n_step % d->ly)
    return fail(EE_EINVAL, "the subset protocol needs n_step divisible by ly (%d %% %d)", d->n_step, d->ly);
  // |I| <= 2 n ly N (2 n ly l N with the whole-region protocol, which ramps
  // the l columns x < l) must fit the int32 accumulators
  const double ramped_cols = (d->flags & EE_FLAG_WHOLE) ? (double)d->l : 1.0;
  if (2.0 * d->n_replicas * d->ly * ramped_cols * (double)d->n_step >= 2147483647.0)
    return fail(EE_EINVAL, "the work bound 2*n*ly*(ramped columns)*n_step exceeds the int32 range");
  if ((double)d->lt * d->ly * d->lx > 1e8) return fail(EE_EINVAL, "lattice too large");
  return EE_OK;
}

Layout layout_of(const ee_job_desc* d) {
  Layout L{};
  L.H = d->lx / 2;
  L.G = (L.H + 3) / 4;
  L.R = d->lt * d->ly;
  L.traj_words = 2 * d->n_replicas * L.R * L.G;
  L.packed_words = 2 * d->n_replicas * L.R * ((L.H + 31) / 32);
  L.storage_words_per_traj =
      (d->spin_format == EE_SPINS_INT8) ? (size_t)L.traj_words : (size_t)L.packed_words;
  size_t off = 0;
  L.off_jobdev = off; off = align_up(off + sizeof(ee::JobDev));
  L.off_selfptr = off; off = align_up(off + sizeof(void*));
  L.off_result = off; off = align_up(off + sizeof(ee_result));
  L.off_ramp = off; off = align_up(off + (size_t)(d->n_step + 1) * 8 * d->dim * sizeof(uint32_t));
  L.off_work = off; off = align_up(off + 3 * (size_t)d->n_traj * sizeof(int64_t));  // I_j + estimator scratch
  L.off_spins = off; off = align_up(off + (size_t)d->n_traj * L.storage_words_per_traj * 4);
  L.total = off;
  return L;
}

struct DeviceInfo {
  int cus = 0;
  int max_lds = 0;
};

DeviceInfo device_info() {
  static std::mutex mu;
  static std::vector<DeviceInfo> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lk(mu);
  if ((int)cache.size() <= dev) cache.resize(dev + 1);
  if (cache[dev].cus == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess) cache[dev].cus = v;
    if (cache[dev].cus <= 0) cache[dev].cus = 256;
    cache[dev].max_lds = ee_k_max_lds_bytes();
  }
  return cache[dev];
}

constexpr int kDefaultBlock = 1024;
constexpr int kMaxBlock = 1024;

// The on-chip sweep needs one lane per word of a row in every workgroup:
// threads >= G, rounded up to whole waves.
int min_block(const Layout& L) { return (L.G + 63) / 64 * 64; }

// Default block for a job when the caller gives none: about one lane per
// four row-words of a trajectory (n * R * G words in a colour plane), so
// that small lattices do not leave most lanes of a 1024-thread block idle,
// within [min_block, kDefaultBlock].
int default_block(const Layout& L, int n_rep) {
  const long words = (long)n_rep * L.R * L.G;
  const long want = (words + 3) / 4;
  int b = (int)std::min<long>(kDefaultBlock, (want + 63) / 64 * 64);
  return std::max(b, std::max(64, min_block(L)));
}

// Default block of a job launched alone (per-job path): when its
// trajectories cannot fill the GPU's threads with one lane per row-word,
// take that many lanes per trajectory (every lane one row: lowest
// latency); otherwise share the GPU's threads out over the trajectories.
int job_block(const Layout& L, const ee_job_desc& d) {
  const long words = (long)d.n_replicas * L.R * L.G;
  const long capacity = (long)device_info().cus * 2048;
  const long per_traj = std::max(64L, std::min(words, capacity / std::max(1, d.n_traj)));
  const int b = (int)std::min<long>(kDefaultBlock, (per_traj + 63) / 64 * 64);
  return std::max(b, min_block(L));
}

// A job runs on chip when one trajectory fits a workgroup's LDS and one row
// fits a workgroup's lanes; otherwise it is streamed from HBM.
bool fits_on_chip(const Layout& L) {
  return L.traj_words * 4 <= ee_k_max_lds_bytes() && min_block(L) <= kMaxBlock;
}
constexpr int kDefaultLdsBudget = 80 * 1024;  // two workgroups per CU

// Trajectories per workgroup that maximise the trajectories finished per
// unit of workgroup time, within the LDS budget.
// min_groups > 0 (per-job launches): keep at least that many workgroups so
// that one job alone fills the GPU.
int choose_slots(const Layout& L, int n_rep, int block, int lds_budget, int n_traj, int min_groups = 0) {
  const int traj_bytes = L.traj_words * 4;
  int kmax = std::min(ee::kMaxSlots, std::max(1, lds_budget / traj_bytes));
  kmax = std::min(kmax, std::max(1, block / L.G));
  kmax = std::min(kmax, std::max(1, n_traj));
  if (min_groups > 0) kmax = std::min(kmax, std::max(1, n_traj / min_groups));
  const int nrows = n_rep * L.R;
  // ties go to the larger k: more rows per lane between workgroup barriers
  int best_k = 1;
  double best = -1.0;
  for (int k = kmax; k >= 1; --k) {
    const int T = block / k;
    const int nrg = T / L.G;
    if (nrg < 1) continue;
    const int iters = (nrows + nrg - 1) / nrg;
    const double rate = (double)k / iters;
    if (rate > best * 1.0001) {
      best = rate;
      best_k = k;
    }
  }
  return best_k;
}

}  // namespace

struct ee_job {
  ee_job_desc d;
  Layout L;
  hipStream_t stream;
  uint8_t* arena;
  size_t arena_bytes;
  ee::JobDev host_jobdev;  // kept alive for the asynchronous upload
  const ee::JobDev* host_selfptr;
  std::vector<uint32_t> host_ramp;
  int state;
  bool spins_exist;
  int64_t g;
  int64_t n_therm_total;
  bool est_enqueued;
  hipStream_t est_stream;
  ee_launch_cfg cfg;
  bool streaming;  // spins stay in HBM (one launch per half-sweep)
  ee::JobDev* dev_jobdev() const { return reinterpret_cast<ee::JobDev*>(arena + L.off_jobdev); }
  const ee::JobDev* const* dev_selfptr() const {
    return reinterpret_cast<const ee::JobDev* const*>(arena + L.off_selfptr);
  }
  ee_result* dev_result() const { return reinterpret_cast<ee_result*>(arena + L.off_result); }
};

namespace {

// ---------------------------------------------------------------------------
// Batch plans: device queue + job table + units, and a HIP graph of
// [queue reset] -> [event] -> [persistent sweep kernel] -> [event] -> [estimator]
// ---------------------------------------------------------------------------
struct Plan {
  std::vector<ee_job*> jobs;
  int n_therm = 0;
  ee_launch_cfg cfg{};
  int dim = 0;
  int block = 0, lds = 0, grid = 0, n_units = 0;
  void* dev_buf = nullptr;
  int* dev_queue = nullptr;
  const ee::JobDev** dev_jobtab = nullptr;
  ee::Unit* dev_units = nullptr;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev_start) (void)hipEventDestroy(ev_start);
    if (ev_stop) (void)hipEventDestroy(ev_stop);
    if (dev_buf) (void)hipFree(dev_buf);
  }
};

std::mutex g_plan_mu;
std::list<Plan*> g_plans;  // most recent first
constexpr size_t kMaxPlans = 16;
thread_local Plan* g_last_plan = nullptr;

void drop_plans_with(ee_job* j) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  for (auto it = g_plans.begin(); it != g_plans.end();) {
    Plan* p = *it;
    if (std::find(p->jobs.begin(), p->jobs.end(), j) != p->jobs.end()) {
      if (g_last_plan == p) g_last_plan = nullptr;
      (void)hipDeviceSynchronize();
      delete p;
      it = g_plans.erase(it);
    } else {
      ++it;
    }
  }
}

bool same_cfg(const ee_launch_cfg& a, const ee_launch_cfg& b) {
  return a.block_threads == b.block_threads && a.lds_bytes == b.lds_bytes &&
         a.grid_blocks == b.grid_blocks && a.use_graph == b.use_graph && a.flags == b.flags;
}

// Lanes per trajectory of the streaming path: every lane walks about 4 rows
// (measured on 96^3: 4% faster than 8 rows, and faster than 2).  W: the
// words per lane the streaming kernel takes for these rows (four for a
// multiple of 16 sites per colour, three for rows of 12, two for a
// multiple of 8, else one).
int stream_lanes(const ee_job* j) {
  const int nrows = j->d.n_replicas * j->L.R;
  const int H = j->L.H;
  const int W = ((H & 15) == 0) ? 4 : (H == 12) ? 3 : ((H & 7) == 0) ? 2 : 1;
  const int GW = j->L.G / W;
  const int nrg = std::max(1, (nrows + 3) / 4);
  return nrg * GW;
}

// Words of one plane of the plane-marching kernel (one replica, one t,
// both colours, all y): a slot of its LDS ring.
int plane_words(const ee_job* j) { return 2 * j->d.ly * j->L.G; }

// Workgroup size of the marching kernel: a lane per row group of up to four
// words of one colour, and enough lanes that each prefetches at most four
// transfer units (4 words, or 1 word for rows of other lengths) of a plane.
int march_block(const ee_job* j) {
  const long items = (long)j->d.ly * ((j->L.G + 3) / 4);
  const long units = (j->L.G % 4 == 0) ? plane_words(j) / 4 : plane_words(j);
  const long lanes = std::max(items, (units + 3) / 4);
  return (int)std::max(64L, std::min(1024L, (lanes + 63) / 64 * 64));
}

// Segments per trajectory of the plane-marching kernel for this job, or 0 if
// the two-pass kernel runs it.  The march reads and writes each plane once
// per sweep (2 B per site against the two-pass kernel's 3 B), but both
// kernels are bound by their issue rate and latency rather than by HBM,
// and the march, with one row per lane between barriers, runs slower
// (96^3, n = 2, 256 trajectories: 828 attempts/ns against 1213), so it runs
// only when EE_LAUNCH_MARCH asks for it.  A workgroup marches one segment of
// one replica of one trajectory, and each segment boundary costs a fix-up
// pass over two planes; without a segment count in grid_blocks the count
// minimises rounds x (planes per segment + 3) over the workgroups resident
// at once (by LDS and by 16 waves per CU).
int march_segments(const ee_job* j) {
  if (j->cfg.flags & EE_LAUNCH_TWO_PASS) return 0;
  const int lds = ee_k_march_lds_bytes(plane_words(j));
  if (lds > ee_k_max_lds_bytes()) return (j->cfg.flags & EE_LAUNCH_MARCH) ? -1 : 0;
  if (!(j->cfg.flags & EE_LAUNCH_MARCH)) return 0;
  const int max_seg = std::max(1, j->d.lt / 2);
  if (j->cfg.grid_blocks > 0) return std::min(j->cfg.grid_blocks, max_seg);
  const int waves = (march_block(j) + 63) / 64;
  const int per_cu = std::max(1, std::min(160 * 1024 / lds, 16 / waves));
  const long slots = (long)device_info().cus * per_cu;
  const long pairs = (long)j->d.n_traj * j->d.n_replicas;
  int best = 1;
  double best_cost = 1e300;
  for (int k = 1; k <= std::min(max_seg, 64); ++k) {
    const double rounds = (double)((pairs * k + slots - 1) / slots);
    const double cost = rounds * ((double)j->d.lt / k + 3.0);
    if (cost < best_cost * 0.999) {
      best_cost = cost;
      best = k;
    }
  }
  return best;
}

ee_status stream_sweeps(ee_job* j, int n_sweeps, bool protocol) {
  const int lanes = stream_lanes(j);
  const int nt = j->d.n_traj;
  const int nseg = march_segments(j);
  if (nseg < 0)
    return fail(EE_EUNSUPPORTED, "EE_LAUNCH_MARCH: a plane ring of %d bytes exceeds the %d bytes of LDS",
                ee_k_march_lds_bytes(plane_words(j)), ee_k_max_lds_bytes());
  int rc = 0;
  if (protocol) rc = ee_k_launch_zero_work(j->dev_jobdev(), nt, j->stream);
  uint32_t g = (uint32_t)j->g;
  const int N = j->d.n_step;
  const bool rev = (j->d.flags & EE_FLAG_REVERSE) != 0;
  const int dpos = protocol ? (rev ? -1 : 1) : 0;
  for (int s = 0; s < n_sweeps && rc == 0; ++s, ++g) {
    const int pos = protocol ? (rev ? N - 1 - s : s + 1) : (rev ? N : 0);
    if (nseg > 0) {
      rc = ee_k_launch_march(j->dev_jobdev(), nt, j->d.n_replicas, nseg, march_block(j), plane_words(j), g, pos,
                             dpos, protocol ? 1 : 0, j->stream);
      continue;
    }
    rc = ee_k_launch_stream_sweep(j->dev_jobdev(), nt, lanes, 0, g, pos, dpos, protocol ? 1 : 0, j->stream);
    if (rc == 0) rc = ee_k_launch_stream_sweep(j->dev_jobdev(), nt, lanes, 1, g, pos, dpos, 0, j->stream);
  }
  if (rc) return fail(EE_EHIP, "streaming sweep launch failed: %s", hipGetErrorString((hipError_t)rc));
  return EE_OK;
}

ee_status launch_sweep_for_job(ee_job* j, uint32_t flags, int n_therm) {
  if (j->streaming) {
    if (flags & ee::kFlagInit) {
      const int rc = ee_k_launch_stream_init(j->dev_jobdev(), j->d.n_traj, stream_lanes(j), j->stream);
      if (rc) return fail(EE_EHIP, "streaming init launch failed: %s", hipGetErrorString((hipError_t)rc));
    }
    if (flags & ee::kFlagProto) return stream_sweeps(j, j->d.n_step, true);
    return stream_sweeps(j, n_therm, false);
  }
  const int block = std::max(j->cfg.block_threads > 0 ? j->cfg.block_threads : job_block(j->L, j->d), min_block(j->L));
  const int budget = j->cfg.lds_bytes > 0 ? j->cfg.lds_bytes : kDefaultLdsBudget;
  const int k = choose_slots(j->L, j->d.n_replicas, block, std::max(budget, j->L.traj_words * 4), j->d.n_traj,
                             2 * device_info().cus);
  const int grid = (j->d.n_traj + k - 1) / k;
  const int lds = k * j->L.traj_words * 4;
  const int rc = ee_k_launch_sweep(j->dev_jobdev(), k, nullptr, 0, nullptr, nullptr, flags, n_therm, (int)j->g, grid,
                                   block, lds, j->stream);
  if (rc != 0) return fail(EE_EHIP, "sweep kernel launch failed: %s", hipGetErrorString((hipError_t)rc));
  return EE_OK;
}

ee_status check_cfg(const ee_launch_cfg* cfg) {
  if (!cfg) return EE_OK;
  if (cfg->block_threads != 0 &&
      (cfg->block_threads < 64 || cfg->block_threads > 1024 || (cfg->block_threads % 64)))
    return fail(EE_EINVAL, "block_threads must be a multiple of 64 in [64, 1024]");
  if (cfg->lds_bytes < 0 || cfg->lds_bytes > ee_k_max_lds_bytes())
    return fail(EE_EINVAL, "lds_bytes must be in [0, %d]", ee_k_max_lds_bytes());
  if (cfg->grid_blocks < 0) return fail(EE_EINVAL, "grid_blocks must be >= 0");
  if (cfg->flags & ~(EE_LAUNCH_STREAMING | EE_LAUNCH_MARCH | EE_LAUNCH_TWO_PASS))
    return fail(EE_EINVAL, "unknown launch flags 0x%x", cfg->flags);
  if ((cfg->flags & EE_LAUNCH_MARCH) && (cfg->flags & EE_LAUNCH_TWO_PASS))
    return fail(EE_EINVAL, "EE_LAUNCH_MARCH and EE_LAUNCH_TWO_PASS exclude each other");
  return EE_OK;
}

// Block size of a persistent launch over these jobs: the config's, else the
// largest default block of the jobs; at least one lane per row word of
// every job.
int launch_block(ee_job* const* jobs, int count, const ee_launch_cfg& cfg) {
  int block = 64;
  if (cfg.block_threads > 0) {
    block = cfg.block_threads;
  } else {
    for (int i = 0; i < count; ++i) block = std::max(block, default_block(jobs[i]->L, jobs[i]->d.n_replicas));
  }
  for (int i = 0; i < count; ++i) block = std::max(block, min_block(jobs[i]->L));
  return block;
}

// LDS budget per workgroup: the config's (else the default), at least one
// trajectory of every job.
int lds_budget(ee_job* const* jobs, int count, const ee_launch_cfg& cfg) {
  int budget = cfg.lds_bytes > 0 ? cfg.lds_bytes : kDefaultLdsBudget;
  for (int i = 0; i < count; ++i) budget = std::max(budget, jobs[i]->L.traj_words * 4);
  return budget;
}

// Relative cost of one unit of job j (k trajectories per workgroup of
// `block` lanes): row iterations per half-sweep times sweeps.
double unit_cost(const ee_job* j, int block, int k, int n_therm) {
  const int T = block / k;
  const int nrg = std::max(1, T / j->L.G);
  const double iters = std::ceil((double)j->d.n_replicas * j->L.R / nrg);
  return iters * (double)(n_therm + j->d.n_step);
}

// Persistent grid: as many workgroups of this shape as fit on the GPU at
// once (or the config's count), at most one per unit.
ee_status persistent_grid(int block, int lds, int n_units, const ee_launch_cfg& cfg, int* grid) {
  const void* fn = nullptr;
  const int rc = ee_k_sweep_kernel_ptr(&fn);
  if (rc != 0) return fail(EE_EHIP, "kernel attribute: %s", hipGetErrorString((hipError_t)rc));
  int per_cu = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block, lds + ee::kSweepTailBytes);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const int g = cfg.grid_blocks > 0 ? cfg.grid_blocks : device_info().cus * per_cu;
  *grid = std::max(1, std::min(g, n_units));
  return EE_OK;
}

// The work units of a persistent launch over these jobs: per job, blocks
// of k trajectories (k LDS slots within the budget), sorted longest first.
struct UnitPlan {
  int block = 0, lds = 0, grid = 0;
  std::vector<ee::Unit> units;
};

ee_status plan_units(ee_job* const* jobs, int count, int n_therm, const ee_launch_cfg& cfg, UnitPlan* out) {
  out->block = launch_block(jobs, count, cfg);
  const int budget = lds_budget(jobs, count, cfg);
  struct U { ee::Unit u; double cost; };
  std::vector<U> units;
  int lds_need = 0;
  for (int i = 0; i < count; ++i) {
    ee_job* j = jobs[i];
    const int k = choose_slots(j->L, j->d.n_replicas, out->block, budget, j->d.n_traj);
    lds_need = std::max(lds_need, k * j->L.traj_words * 4);
    const double cost = unit_cost(j, out->block, k, n_therm);
    for (int j0 = 0; j0 < j->d.n_traj; j0 += k)
      units.push_back({ee::Unit{i, j0, std::min(k, j->d.n_traj - j0), k}, cost});
  }
  std::stable_sort(units.begin(), units.end(), [](const U& a, const U& b) { return a.cost > b.cost; });
  out->lds = lds_need;
  out->units.resize(units.size());
  for (size_t i = 0; i < units.size(); ++i) out->units[i] = units[i].u;
  return persistent_grid(out->block, out->lds, (int)units.size(), cfg, &out->grid);
}

ee_status build_plan(ee_job* const* jobs, int count, int n_therm, const ee_launch_cfg& cfg,
                     hipStream_t stream, Plan** out) {
  UnitPlan up;
  ee_status st = plan_units(jobs, count, n_therm, cfg, &up);
  if (st) return st;
  auto P = new Plan();
  P->jobs.assign(jobs, jobs + count);
  P->n_therm = n_therm;
  P->cfg = cfg;
  P->dim = jobs[0]->d.dim;
  P->block = up.block;
  P->lds = up.lds;
  P->grid = up.grid;
  P->n_units = (int)up.units.size();
  const std::vector<ee::Unit>& units = up.units;
  const void* fn = nullptr;
  int rc = ee_k_sweep_kernel_ptr(&fn);
  if (rc != 0) { delete P; return fail(EE_EHIP, "kernel attribute: %s", hipGetErrorString((hipError_t)rc)); }
  hipError_t e = hipSuccess;
  // device metadata
  const size_t off_tab = kAlign;
  const size_t off_units = align_up(off_tab + sizeof(void*) * count);
  const size_t bytes = off_units + sizeof(ee::Unit) * units.size();
  e = hipMalloc(&P->dev_buf, bytes);
  if (e != hipSuccess) { delete P; return fail(EE_EHIP, "hipMalloc(batch plan): %s", hipGetErrorString(e)); }
  P->dev_queue = reinterpret_cast<int*>(P->dev_buf);
  P->dev_jobtab = reinterpret_cast<const ee::JobDev**>((uint8_t*)P->dev_buf + off_tab);
  P->dev_units = reinterpret_cast<ee::Unit*>((uint8_t*)P->dev_buf + off_units);
  std::vector<uint8_t> host(bytes, 0);
  for (int i = 0; i < count; ++i)
    reinterpret_cast<const ee::JobDev**>(host.data() + off_tab)[i] = jobs[i]->dev_jobdev();
  for (size_t i = 0; i < units.size(); ++i)
    reinterpret_cast<ee::Unit*>(host.data() + off_units)[i] = units[i];
  e = hipMemcpy(P->dev_buf, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) { delete P; return fail(EE_EHIP, "upload of batch plan: %s", hipGetErrorString(e)); }
  if (hipEventCreate(&P->ev_start) != hipSuccess || hipEventCreate(&P->ev_stop) != hipSuccess) {
    delete P;
    return fail(EE_EHIP, "hipEventCreate failed");
  }
  if (cfg.use_graph) {
    hipGraph_t g;
    e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) { delete P; return fail(EE_EHIP, "hipGraphCreate: %s", hipGetErrorString(e)); }
    P->graph = g;
    const void* f_reset = nullptr;
    const void* f_est = nullptr;
    ee_k_queue_reset_ptr(&f_reset);
    ee_k_estimate_ptr(&f_est);
    hipGraphNode_t n_reset, n_ev0, n_sweep, n_ev1, n_est;
    int* q = P->dev_queue;
    void* a_reset[] = {&q};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(f_reset);
    kp.gridDim = dim3(1);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = a_reset;
    e = hipGraphAddKernelNode(&n_reset, g, nullptr, 0, &kp);
    if (e == hipSuccess) e = hipGraphAddEventRecordNode(&n_ev0, g, &n_reset, 1, P->ev_start);
    const ee::JobDev* sj = nullptr;
    int sk = 0;
    const ee::Unit* un = P->dev_units;
    int nu = P->n_units;
    const ee::JobDev* const* jt = P->dev_jobtab;
    uint32_t fl = ee::kFlagInit | ee::kFlagProto;
    int nt = n_therm, g0 = 0;
    int tail = ee::sweep_tail_words(P->lds);
    void* a_sweep[] = {&sj, &sk, &un, &nu, &q, &jt, &fl, &nt, &g0, &tail};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = dim3(P->grid);
    kp.blockDim = dim3(P->block);
    kp.sharedMemBytes = P->lds + ee::kSweepTailBytes;
    kp.kernelParams = a_sweep;
    if (e == hipSuccess) e = hipGraphAddKernelNode(&n_sweep, g, &n_ev0, 1, &kp);
    if (e == hipSuccess) e = hipGraphAddEventRecordNode(&n_ev1, g, &n_sweep, 1, P->ev_stop);
    void* a_est[] = {&jt};
    kp.func = const_cast<void*>(f_est);
    kp.gridDim = dim3(count);
    kp.blockDim = dim3(ee::kEstimateThreads);
    kp.sharedMemBytes = 0;
    kp.kernelParams = a_est;
    if (e == hipSuccess) e = hipGraphAddKernelNode(&n_est, g, &n_ev1, 1, &kp);
    if (e == hipSuccess) e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { delete P; return fail(EE_EHIP, "building the batch graph: %s", hipGetErrorString(e)); }
  }
  (void)stream;
  *out = P;
  return EE_OK;
}

// Checks shared by the batch entry points: every job freshly created, on
// chip, listed once; the sweep counters fit.
ee_status check_batch(ee_job* const* jobs, int count, int n_therm, const ee_launch_cfg* cfg) {
  if (!jobs || count < 1) return fail(EE_EINVAL, "need at least one job");
  if (n_therm < 0) return fail(EE_EINVAL, "n_therm must be >= 0");
  ee_status s = check_cfg(cfg);
  if (s) return s;
  for (int i = 0; i < count; ++i) {
    if (!jobs[i]) return fail(EE_EINVAL, "jobs[%d] is NULL", i);
    if (jobs[i]->state != CREATED || jobs[i]->spins_exist)
      return fail(EE_ESTATE, "jobs[%d] is not freshly created (use ee_job_reset)", i);
    if (jobs[i]->streaming)
      return fail(EE_EUNSUPPORTED, "jobs[%d] is too large for the on-chip batch kernel; run it with "
                  "ee_thermalize / ee_run_protocol", i);
    for (int k = 0; k < i; ++k)
      if (jobs[k] == jobs[i]) return fail(EE_EINVAL, "jobs[%d] appears twice", i);
    if ((int64_t)n_therm + jobs[i]->d.n_step > 0x7FFFFFFF) return fail(EE_EINVAL, "sweep counter overflow");
  }
  return EE_OK;
}

// Host state of jobs whose batch (sweeps + estimator) is enqueued on stream.
void mark_batch_done(ee_job* const* jobs, int count, int n_therm, hipStream_t stream) {
  for (int i = 0; i < count; ++i) {
    ee_job* j = jobs[i];
    j->spins_exist = true;
    j->g = (int64_t)n_therm + j->d.n_step;
    j->n_therm_total = n_therm;
    j->state = DONE;
    j->est_enqueued = true;
    j->est_stream = stream;
  }
}

ee_status run_plan(Plan* P, hipStream_t stream) {
  if (P->exec) {
    HIP_TRY(hipGraphLaunch(P->exec, stream));
  } else {
    int rc = ee_k_launch_queue_reset(P->dev_queue, stream);
    if (rc) return fail(EE_EHIP, "queue reset launch: %s", hipGetErrorString((hipError_t)rc));
    HIP_TRY(hipEventRecord(P->ev_start, stream));
    rc = ee_k_launch_sweep(nullptr, 0, P->dev_units, P->n_units, P->dev_queue, P->dev_jobtab,
                           ee::kFlagInit | ee::kFlagProto, P->n_therm, 0, P->grid, P->block, P->lds, stream);
    if (rc) return fail(EE_EHIP, "persistent sweep launch: %s", hipGetErrorString((hipError_t)rc));
    HIP_TRY(hipEventRecord(P->ev_stop, stream));
    rc = ee_k_launch_estimate(P->dev_jobtab, (int)P->jobs.size(), stream);
    if (rc) return fail(EE_EHIP, "estimator launch: %s", hipGetErrorString((hipError_t)rc));
  }
  return EE_OK;
}

}  // namespace

extern "C" {

const char* ee_last_error(void) { return g_err.c_str(); }
const char* ee_version(void) { return "ee-mi355x 0.2 (gfx950)"; }

#ifndef EE_SOURCE_HASH
#define EE_SOURCE_HASH "unknown"
#endif
const char* ee_build_id(void) { return EE_SOURCE_HASH; }

ee_status ee_job_footprint(const ee_job_desc* desc, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(EE_EINVAL, "bytes is NULL");
  ee_status s = validate(desc);
  if (s) return s;
  Layout L = layout_of(desc);
  if (!fits_on_chip(L) && desc->spin_format != EE_SPINS_INT8)
    return fail(EE_EUNSUPPORTED,
                "a trajectory of %d bytes with rows of %d words exceeds the on-chip tile (%d bytes, %d words "
                "per row); such lattices are streamed from HBM and need EE_SPINS_INT8 storage",
                L.traj_words * 4, L.G, ee_k_max_lds_bytes(), kMaxBlock);
  *bytes = L.total;
  return EE_OK;
}

ee_status ee_job_on_chip(const ee_job_desc* desc, int32_t* on_chip) {
  g_err.clear();
  if (!on_chip) return fail(EE_EINVAL, "on_chip is NULL");
  ee_status s = validate(desc);
  if (s) return s;
  *on_chip = fits_on_chip(layout_of(desc)) ? 1 : 0;
  return EE_OK;
}

ee_status ee_job_create(const ee_job_desc* desc, void* dev_arena, size_t arena_bytes, void* hip_stream,
                        ee_job** out) {
  g_err.clear();
  if (!out) return fail(EE_EINVAL, "out is NULL");
  size_t need = 0;
  ee_status s = ee_job_footprint(desc, &need);
  if (s) return s;
  if (!dev_arena) return fail(EE_EINVAL, "arena is NULL");
  if (reinterpret_cast<uintptr_t>(dev_arena) % kAlign) return fail(EE_EINVAL, "arena must be 256-byte aligned");
  if (arena_bytes < need) return fail(EE_ENOMEM, "arena has %zu bytes, the job needs %zu", arena_bytes, need);
  ee_job* j = new ee_job();
  j->d = *desc;
  j->L = layout_of(desc);
  j->stream = reinterpret_cast<hipStream_t>(hip_stream);
  j->arena = reinterpret_cast<uint8_t*>(dev_arena);
  j->arena_bytes = arena_bytes;
  j->state = CREATED;
  j->spins_exist = false;
  j->g = 0;
  j->n_therm_total = 0;
  j->est_enqueued = false;
  j->est_stream = j->stream;
  j->cfg = ee_launch_cfg{0, 0, 0, 1, 0};
  j->streaming = !fits_on_chip(j->L);
  const int dim = desc->dim, N = desc->n_step;
  const bool subsets = (desc->flags & EE_FLAG_SUBSETS) != 0;
  const int S = subsets ? N / desc->ly : N;  // weights in units of beta/S
  // thresholds
  ee::JobDev& D = j->host_jobdev;
  std::memset(&D, 0, sizeof(D));
  D.dim = dim; D.lt = desc->lt; D.lx = desc->lx; D.ly = desc->ly; D.n = desc->n_replicas;
  D.l = desc->l; D.N = N; D.n_traj = desc->n_traj;
  D.H = j->L.H; D.G = j->L.G; D.R = j->L.R; D.traj_words = j->L.traj_words;
  D.packed_words = j->L.packed_words;
  D.key0 = (uint32_t)(desc->seed & 0xFFFFFFFFu);
  D.key1 = (uint32_t)(desc->seed >> 32);
  D.S = S;
  D.subsets = subsets ? 1 : 0;
  D.whole = (desc->flags & EE_FLAG_WHOLE) ? 1 : 0;
  for (int a = 0; a < dim; ++a) D.thr_bulk[a] = threshold(desc->beta, (int64_t)S * (2 * dim - 2 * a), S);
  D.reverse = (desc->flags & EE_FLAG_REVERSE) ? 1u : 0u;
  D.spin_format = (uint32_t)desc->spin_format;
  ee::Magic mr = ee::make_magic((uint32_t)j->L.R), my = ee::make_magic((uint32_t)desc->ly);
  D.magic_R = mr.mul; D.shift_R = mr.shift; D.magic_Ly = my.mul; D.shift_Ly = my.shift;
  D.beta = desc->beta;
  D.ramp_thr = reinterpret_cast<const uint32_t*>(j->arena + j->L.off_ramp);
  D.spins = reinterpret_cast<uint32_t*>(j->arena + j->L.off_spins);
  D.work = reinterpret_cast<int64_t*>(j->arena + j->L.off_work);
  D.result = j->dev_result();
  // ramped-site thresholds U_m[fa][b][c], K = S(2dim-1-2fa) + (S-m)(1-2b) + m(1-2c)
  j->host_ramp.resize((size_t)(S + 1) * 8 * dim);
  for (int m = 0; m <= S; ++m)
    for (int fa = 0; fa < 2 * dim; ++fa)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
          const int64_t K = (int64_t)S * (2 * dim - 1 - 2 * fa) + (int64_t)(S - m) * (1 - 2 * b) +
                            (int64_t)m * (1 - 2 * c);
          j->host_ramp[(size_t)m * 8 * dim + fa * 4 + b * 2 + c] = threshold(desc->beta, K, S);
        }
  j->host_selfptr = j->dev_jobdev();
  hipError_t e = hipMemcpyAsync(j->dev_jobdev(), &j->host_jobdev, sizeof(ee::JobDev), hipMemcpyHostToDevice, j->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(j->arena + j->L.off_selfptr, &j->host_selfptr, sizeof(void*), hipMemcpyHostToDevice, j->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(j->arena + j->L.off_ramp, j->host_ramp.data(), j->host_ramp.size() * 4,
                       hipMemcpyHostToDevice, j->stream);
  if (e != hipSuccess) {
    delete j;
    return fail(EE_EHIP, "upload of job tables: %s", hipGetErrorString(e));
  }
  *out = j;
  return EE_OK;
}

ee_status ee_job_set_launch(ee_job* job, const ee_launch_cfg* cfg) {
  g_err.clear();
  if (!job) return fail(EE_EINVAL, "job is NULL");
  ee_status s = check_cfg(cfg);
  if (s) return s;
  if (job->state == SERVED) return fail(EE_ESTATE, "the job is on a server that has not reported it done");
  const bool force_stream = cfg && (cfg->flags & (EE_LAUNCH_STREAMING | EE_LAUNCH_MARCH | EE_LAUNCH_TWO_PASS));
  if (force_stream && job->d.spin_format != EE_SPINS_INT8)
    return fail(EE_EUNSUPPORTED, "the streaming path needs EE_SPINS_INT8 storage");
  if (force_stream && job->spins_exist && !job->streaming)
    return fail(EE_ESTATE, "switch to the streaming path before the first ee_thermalize");
  if (cfg && (cfg->flags & EE_LAUNCH_MARCH) && ee_k_march_lds_bytes(plane_words(job)) > ee_k_max_lds_bytes())
    return fail(EE_EUNSUPPORTED, "EE_LAUNCH_MARCH: a plane ring of %d bytes exceeds the %d bytes of LDS",
                ee_k_march_lds_bytes(plane_words(job)), ee_k_max_lds_bytes());
  job->cfg = cfg ? *cfg : ee_launch_cfg{0, 0, 0, 1, 0};
  job->streaming = force_stream || !fits_on_chip(job->L);
  return EE_OK;
}

ee_status ee_thermalize(ee_job* job, int32_t n_sweeps) {
  g_err.clear();
  if (!job) return fail(EE_EINVAL, "job is NULL");
  if (n_sweeps < 0) return fail(EE_EINVAL, "n_sweeps must be >= 0");
  if (job->state != CREATED) return fail(EE_ESTATE, "ee_thermalize after the protocol");
  if (job->g + n_sweeps > 0x7FFFFFFF - (int64_t)job->d.n_step) return fail(EE_EINVAL, "sweep counter overflow");
  uint32_t flags = job->spins_exist ? 0u : ee::kFlagInit;
  if (n_sweeps == 0 && job->spins_exist) return EE_OK;
  ee_status s = launch_sweep_for_job(job, flags, n_sweeps);
  if (s) return s;
  job->spins_exist = true;
  job->g += n_sweeps;
  job->n_therm_total += n_sweeps;
  return EE_OK;
}

ee_status ee_run_protocol(ee_job* job) {
  g_err.clear();
  if (!job) return fail(EE_EINVAL, "job is NULL");
  if (job->state != CREATED) return fail(EE_ESTATE, "the protocol runs once per job");
  if (!job->spins_exist) return fail(EE_ESTATE, "call ee_thermalize (possibly with 0 sweeps) first");
  ee_status s = launch_sweep_for_job(job, ee::kFlagProto, 0);
  if (s) return s;
  job->g += job->d.n_step;
  job->state = DONE;
  job->est_enqueued = false;
  return EE_OK;
}

ee_status ee_estimate(ee_job* job, ee_result* out) {
  g_err.clear();
  if (!job || !out) return fail(EE_EINVAL, "NULL argument");
  if (job->state != DONE) return fail(EE_ESTATE, "ee_estimate before the protocol");
  if (!job->est_enqueued) {
    int rc = ee_k_launch_estimate(job->dev_selfptr(), 1, job->stream);
    if (rc) return fail(EE_EHIP, "estimator launch: %s", hipGetErrorString((hipError_t)rc));
    job->est_enqueued = true;
    job->est_stream = job->stream;
  }
  ee_result r;
  HIP_TRY(hipMemcpyAsync(&r, job->dev_result(), sizeof(r), hipMemcpyDeviceToHost, job->est_stream));
  HIP_TRY(hipStreamSynchronize(job->est_stream));
  r.n_traj = job->d.n_traj;
  r.attempts = (int64_t)job->d.n_traj * job->d.n_replicas * job->d.lt * job->d.ly * job->d.lx *
               (job->n_therm_total + job->d.n_step);
  r.reserved = 0;
  *out = r;
  return EE_OK;
}

ee_status ee_job_read_work(ee_job* job, int64_t* host_I, int32_t count) {
  g_err.clear();
  if (!job || (!host_I && count > 0)) return fail(EE_EINVAL, "NULL argument");
  if (job->state != DONE) return fail(EE_ESTATE, "no works before the protocol");
  if (count < 0 || count > job->d.n_traj) return fail(EE_EINVAL, "count must be in [0, n_traj]");
  if (count == 0) return EE_OK;
  HIP_TRY(hipMemcpyAsync(host_I, job->arena + job->L.off_work, sizeof(int64_t) * count,
                         hipMemcpyDeviceToHost, job->est_stream));
  HIP_TRY(hipStreamSynchronize(job->est_stream));
  return EE_OK;
}

ee_status ee_job_read_spins(ee_job* job, int8_t* host, size_t count) {
  g_err.clear();
  if (!job || (!host && count > 0)) return fail(EE_EINVAL, "NULL argument");
  if (job->state == SERVED) return fail(EE_ESTATE, "the job is on a server that has not reported it done");
  if (!job->spins_exist) return fail(EE_ESTATE, "no spins before ee_thermalize");
  const ee_job_desc& d = job->d;
  const size_t per = (size_t)d.n_replicas * d.lt * d.ly * d.lx;
  if (count % per || count / per > (size_t)d.n_traj)
    return fail(EE_EINVAL, "count must be a multiple of %zu and at most n_traj of them", per);
  const size_t nt = count / per;
  if (nt == 0) return EE_OK;
  const size_t words = job->L.storage_words_per_traj;
  std::vector<uint32_t> raw(nt * words);
  HIP_TRY(hipMemcpyAsync(raw.data(), job->arena + job->L.off_spins, raw.size() * 4, hipMemcpyDeviceToHost,
                         job->est_stream));
  HIP_TRY(hipStreamSynchronize(job->est_stream));
  const int n = d.n_replicas, R = job->L.R, G = job->L.G, H = job->L.H;
  const int PW = (H + 31) / 32;
  for (size_t j = 0; j < nt; ++j) {
    const uint32_t* tw = raw.data() + j * words;
    for (int c = 0; c < 2; ++c)
      for (int r = 0; r < n; ++r)
        for (int t = 0; t < d.lt; ++t)
          for (int y = 0; y < d.ly; ++y) {
            const int rho = t * d.ly + y;
            const size_t rowg = ((size_t)c * n + r) * R + rho;
            for (int h = 0; h < H; ++h) {
              int bit;
              if (d.spin_format == EE_SPINS_INT8)
                bit = (tw[rowg * G + (h >> 2)] >> (8 * (h & 3))) & 1;
              else
                bit = (tw[rowg * PW + (h >> 5)] >> (h & 31)) & 1;
              const int x = 2 * h + ((c + t + y) & 1);
              host[(((j * n + r) * d.lt + t) * d.ly + y) * d.lx + x] = bit ? 1 : -1;
            }
          }
  }
  return EE_OK;
}

ee_status ee_job_reset(ee_job* job) {
  g_err.clear();
  if (!job) return fail(EE_EINVAL, "job is NULL");
  if (job->state == SERVED) return fail(EE_ESTATE, "the job is on a server that has not reported it done");
  job->state = CREATED;
  job->spins_exist = false;
  job->g = 0;
  job->n_therm_total = 0;
  job->est_enqueued = false;
  return EE_OK;
}

ee_status ee_batch_run_cfg(ee_job* const* jobs, int32_t count, int32_t n_therm, const ee_launch_cfg* cfg,
                           void* hip_stream) {
  g_err.clear();
  ee_status s = check_batch(jobs, count, n_therm, cfg);
  if (s) return s;
  ee_launch_cfg c = cfg ? *cfg : ee_launch_cfg{0, 0, 0, 1, 0};
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  // the job tables must be uploaded before the batch reads them
  for (int i = 0; i < count; ++i)
    if (jobs[i]->stream != stream) HIP_TRY(hipStreamSynchronize(jobs[i]->stream));
  Plan* P = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it) {
      Plan* q = *it;
      if (q->n_therm == n_therm && same_cfg(q->cfg, c) && (int)q->jobs.size() == count &&
          std::equal(q->jobs.begin(), q->jobs.end(), jobs)) {
        P = q;
        g_plans.erase(it);
        g_plans.push_front(P);
        break;
      }
    }
  }
  if (!P) {
    s = build_plan(jobs, count, n_therm, c, stream, &P);
    if (s) return s;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans.push_front(P);
    while (g_plans.size() > kMaxPlans) {
      Plan* old = g_plans.back();
      g_plans.pop_back();
      if (g_last_plan == old) g_last_plan = nullptr;
      (void)hipDeviceSynchronize();
      delete old;
    }
  }
  s = run_plan(P, stream);
  if (s) return s;
  g_last_plan = P;
  mark_batch_done(jobs, count, n_therm, stream);
  return EE_OK;
}

ee_status ee_batch_run(ee_job* const* jobs, int32_t count, int32_t n_therm, void* hip_stream) {
  return ee_batch_run_cfg(jobs, count, n_therm, nullptr, hip_stream);
}

ee_status ee_batch_run_noalloc(ee_job* const* jobs, int32_t count, int32_t n_therm, const ee_launch_cfg* cfg,
                               void* hip_stream) {
  g_err.clear();
  ee_status s = check_batch(jobs, count, n_therm, cfg);
  if (s) return s;
  const ee_launch_cfg c = cfg ? *cfg : ee_launch_cfg{0, 0, 0, 1, 0};
  hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
  UnitPlan up;
  s = plan_units(jobs, count, n_therm, c, &up);
  if (s) return s;
  // the tables in the fixed scratch array: [queue counter][job table][units]
  const size_t off_tab = kAlign;
  const size_t off_units = align_up(off_tab + sizeof(void*) * count);
  const size_t bytes = off_units + sizeof(ee::Unit) * up.units.size();
  if (bytes > ee_k_scratch_bytes())
    return fail(EE_EINVAL, "the batch needs %zu bytes of tables (%d jobs, %zu work units), more than the %zu-byte "
                "scratch of the allocation-free entry point", bytes, count, up.units.size(), ee_k_scratch_bytes());
  void* scr = nullptr;
  int rc = ee_k_scratch_ptr(&scr);
  if (rc) return fail(EE_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString((hipError_t)rc));
  for (int i = 0; i < count; ++i)
    if (jobs[i]->stream != stream) HIP_TRY(hipStreamSynchronize(jobs[i]->stream));
  std::vector<uint8_t> host(bytes - off_tab);
  for (int i = 0; i < count; ++i) reinterpret_cast<const ee::JobDev**>(host.data())[i] = jobs[i]->dev_jobdev();
  std::memcpy(host.data() + (off_units - off_tab), up.units.data(), sizeof(ee::Unit) * up.units.size());
  uint8_t* base = reinterpret_cast<uint8_t*>(scr);
  int* queue = reinterpret_cast<int*>(base);
  const ee::JobDev* const* jobtab = reinterpret_cast<const ee::JobDev* const*>(base + off_tab);
  const ee::Unit* units = reinterpret_cast<const ee::Unit*>(base + off_units);
  // stream-ordered after the previous user of the array on this stream; the
  // host buffer must outlive the copy, so the call waits for it
  HIP_TRY(hipMemcpyAsync(base + off_tab, host.data(), host.size(), hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  rc = ee_k_launch_queue_reset(queue, stream);
  if (rc == 0)
    rc = ee_k_launch_sweep(nullptr, 0, units, (int)up.units.size(), queue, jobtab, ee::kFlagInit | ee::kFlagProto,
                           n_therm, 0, up.grid, up.block, up.lds, stream);
  if (rc == 0) rc = ee_k_launch_estimate(jobtab, count, stream);
  if (rc) return fail(EE_EHIP, "allocation-free batch launch: %s", hipGetErrorString((hipError_t)rc));
  mark_batch_done(jobs, count, n_therm, stream);
  return EE_OK;
}

ee_status ee_batch_kernel_ms(double* ms) {
  g_err.clear();
  if (!ms) return fail(EE_EINVAL, "ms is NULL");
  Plan* P = g_last_plan;
  if (!P) return fail(EE_ESTATE, "no batch has run on this thread");
  HIP_TRY(hipEventSynchronize(P->ev_stop));
  float f = 0.0f;
  HIP_TRY(hipEventElapsedTime(&f, P->ev_start, P->ev_stop));
  *ms = (double)f;
  return EE_OK;
}

ee_status ee_job_destroy(ee_job* job) {
  g_err.clear();
  if (!job) return EE_OK;
  if (job->state == SERVED) return fail(EE_ESTATE, "the job is on a server that has not reported it done");
  drop_plans_with(job);
  (void)hipStreamSynchronize(job->stream);
  if (job->est_stream != job->stream) (void)hipStreamSynchronize(job->est_stream);
  delete job;
  return EE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Continuous batching (serving): the chunk scheduler behind ee_server_*.
//
// A submitted job is split into work units (blocks of k trajectories, as in
// a batch) of its launch class: the job's own launch shape (ee_job_set_launch)
// or the server's.  Units queue on the host per class, in submission order.
// Whenever one of the server's launch slots is free and units are waiting,
// the class whose oldest unit is the oldest overall fills a chunk (at most
// its chunk size) and one persistent sweep kernel of that class's shape runs
// it on the slot's stream.  Several slots keep chunks in flight, so a
// chunk's workgroups fill the CUs the previous chunk's tail leaves idle,
// and units of jobs submitted while others run start as soon as a slot
// frees.  A job's table upload (on its own stream) is awaited on the device
// by the chunks that need it, not on the host.  When every unit of a job has
// run (the host sees its chunks' events), the job's estimator is launched on
// the server's service stream; ee_server_poll reports the job once that
// launch has completed.
// ---------------------------------------------------------------------------
namespace {

struct SrvJob {
  ee_job* job = nullptr;
  int units_left = 0;
  hipEvent_t uploaded = nullptr;  // recorded on the job's stream at submission
  bool upload_seen = false;       // the host has seen that event complete
};

struct SrvUnit {
  int id;  // index into ee_server::jobs
  int j0, count, k;
  double cost;
  uint64_t seq;  // submission order
};

struct SrvClass {
  int block = 0, budget = 0, chunk_units = 0;
  std::deque<SrvUnit> pending;
};

struct SrvSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t* dev = nullptr;   // [queue counter][job table][units]
  uint8_t* host = nullptr;  // pinned staging of the same bytes
  bool busy = false;
  std::vector<std::pair<int, int>> per_job;  // (job id, units of it in the chunk)
};

struct SrvEst {
  hipEvent_t ev;
  std::vector<int> ids;
};

}  // namespace

struct ee_server {
  ee_launch_cfg cfg{};
  int n_therm = 0;
  int max_chunk = 0;  // units per chunk at most (slot buffer capacity)
  size_t off_tab = 0, off_units = 0, bytes = 0;
  std::vector<SrvSlot> slots;
  std::vector<SrvClass> classes;
  uint64_t seq = 0;
  std::vector<SrvJob> jobs;  // by id; ids of reported jobs are reused
  std::vector<int> free_ids;
  hipStream_t est_stream = nullptr;
  std::deque<SrvEst> est;  // estimator launches in flight, in order
  std::vector<hipEvent_t> spare_events;
  std::deque<int> ready;  // done, not yet returned by ee_server_poll
  int open_jobs = 0;      // submitted, not yet returned
};

namespace {

ee_status server_event(ee_server* S, hipEvent_t* ev) {
  if (!S->spare_events.empty()) {
    *ev = S->spare_events.back();
    S->spare_events.pop_back();
    return EE_OK;
  }
  HIP_TRY(hipEventCreateWithFlags(ev, hipEventDisableTiming));
  return EE_OK;
}

void server_free(ee_server* S) {
  for (SrvSlot& sl : S->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.host) (void)hipHostFree(sl.host);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  if (S->est_stream) (void)hipStreamSynchronize(S->est_stream);
  for (SrvEst& e : S->est) (void)hipEventDestroy(e.ev);
  for (hipEvent_t e : S->spare_events) (void)hipEventDestroy(e);
  for (SrvJob& sj : S->jobs)
    if (sj.uploaded) (void)hipEventDestroy(sj.uploaded);
  if (S->est_stream) (void)hipStreamDestroy(S->est_stream);
  delete S;
}

// Launch the next chunk on a free slot: units of the class holding the
// oldest waiting unit, longest first within the chunk.
ee_status server_launch(ee_server* S, SrvSlot& sl) {
  SrvClass* C = nullptr;
  for (SrvClass& c : S->classes)
    if (!c.pending.empty() && (!C || c.pending.front().seq < C->pending.front().seq)) C = &c;
  if (!C) return EE_OK;
  const int take = std::min<int>(C->chunk_units, (int)C->pending.size());
  std::vector<SrvUnit> chunk(C->pending.begin(), C->pending.begin() + take);
  C->pending.erase(C->pending.begin(), C->pending.begin() + take);
  std::stable_sort(chunk.begin(), chunk.end(), [](const SrvUnit& a, const SrvUnit& b) { return a.cost > b.cost; });
  std::unordered_map<int, int> local;  // job id -> index in the chunk's job table
  sl.per_job.clear();
  std::memset(sl.host, 0, S->off_tab);  // queue counter = 0
  const ee::JobDev** tab = reinterpret_cast<const ee::JobDev**>(sl.host + S->off_tab);
  ee::Unit* units = reinterpret_cast<ee::Unit*>(sl.host + S->off_units);
  int block = C->block, lds = 0;
  for (int i = 0; i < take; ++i) {
    const SrvUnit& u = chunk[i];
    SrvJob& sj = S->jobs[u.id];
    auto it = local.find(u.id);
    if (it == local.end()) {
      it = local.emplace(u.id, (int)sl.per_job.size()).first;
      tab[it->second] = sj.job->dev_jobdev();
      sl.per_job.emplace_back(u.id, 0);
      block = std::max(block, min_block(sj.job->L));
      if (!sj.upload_seen) {
        const hipError_t q = hipEventQuery(sj.uploaded);
        if (q == hipSuccess) {
          sj.upload_seen = true;
        } else if (q == hipErrorNotReady) {
          HIP_TRY(hipStreamWaitEvent(sl.stream, sj.uploaded, 0));
        } else {
          return fail(EE_EHIP, "job upload: %s", hipGetErrorString(q));
        }
      }
    }
    sl.per_job[it->second].second += 1;
    units[i] = ee::Unit{it->second, u.j0, u.count, u.k};
    lds = std::max(lds, u.k * sj.job->L.traj_words * 4);
  }
  int grid = 0;
  ee_status s = persistent_grid(block, lds, take, S->cfg, &grid);
  if (s) return s;
  int* queue = reinterpret_cast<int*>(sl.dev);
  HIP_TRY(hipMemcpyAsync(sl.dev, sl.host, S->off_units + sizeof(ee::Unit) * take, hipMemcpyHostToDevice, sl.stream));
  const int rc = ee_k_launch_sweep(nullptr, 0, reinterpret_cast<const ee::Unit*>(sl.dev + S->off_units), take, queue,
                                   reinterpret_cast<const ee::JobDev* const*>(sl.dev + S->off_tab),
                                   ee::kFlagInit | ee::kFlagProto, S->n_therm, 0, grid, block, lds, sl.stream);
  if (rc) return fail(EE_EHIP, "server chunk launch: %s", hipGetErrorString((hipError_t)rc));
  HIP_TRY(hipEventRecord(sl.done, sl.stream));
  sl.busy = true;
  return EE_OK;
}

bool server_has_pending(const ee_server* S) {
  for (const SrvClass& c : S->classes)
    if (!c.pending.empty()) return true;
  return false;
}

// Collect finished chunks, launch the estimators of jobs whose last unit
// ran, move finished estimators to the ready list, and refill free slots.
ee_status server_progress(ee_server* S) {
  std::vector<int> finished;
  for (SrvSlot& sl : S->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail(EE_EHIP, "server chunk: %s", hipGetErrorString(q));
    for (const auto& pj : sl.per_job) {
      SrvJob& sj = S->jobs[pj.first];
      sj.units_left -= pj.second;
      if (sj.units_left == 0) finished.push_back(pj.first);
    }
    sl.busy = false;
  }
  if (!finished.empty()) {
    for (int id : finished) {
      ee_job* j = S->jobs[id].job;
      const int rc = ee_k_launch_estimate(j->dev_selfptr(), 1, S->est_stream);
      if (rc) return fail(EE_EHIP, "server estimator launch: %s", hipGetErrorString((hipError_t)rc));
      // the job stays SERVED until a poll returns it
      j->spins_exist = true;
      j->g = (int64_t)S->n_therm + j->d.n_step;
      j->n_therm_total = S->n_therm;
      j->est_enqueued = true;
    }
    hipEvent_t ev = nullptr;
    ee_status s = server_event(S, &ev);
    if (s) return s;
    HIP_TRY(hipEventRecord(ev, S->est_stream));
    S->est.push_back(SrvEst{ev, finished});
  }
  while (!S->est.empty()) {
    const hipError_t q = hipEventQuery(S->est.front().ev);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) return fail(EE_EHIP, "server estimator: %s", hipGetErrorString(q));
    for (int id : S->est.front().ids) S->ready.push_back(id);
    S->spare_events.push_back(S->est.front().ev);
    S->est.pop_front();
  }
  for (SrvSlot& sl : S->slots) {
    if (!server_has_pending(S)) break;
    if (sl.busy) continue;
    ee_status s = server_launch(S, sl);
    if (s) return s;
  }
  return EE_OK;
}

// The launch class of a job: its own shape if ee_job_set_launch gave block
// and LDS, else the server's.
ee_status server_class(ee_server* S, const ee_job* job, SrvClass** out) {
  int block = S->cfg.block_threads > 0 ? S->cfg.block_threads : 256;
  int budget = S->cfg.lds_bytes > 0 ? S->cfg.lds_bytes : kDefaultLdsBudget;
  if (job->cfg.block_threads > 0) block = job->cfg.block_threads;
  if (job->cfg.lds_bytes > 0) budget = job->cfg.lds_bytes;
  for (SrvClass& c : S->classes)
    if (c.block == block && c.budget == budget) {
      *out = &c;
      return EE_OK;
    }
  SrvClass c;
  c.block = block;
  c.budget = budget;
  int grid = 0;
  ee_status s = persistent_grid(block, budget, 1 << 30, S->cfg, &grid);
  if (s) return s;
  c.chunk_units = std::min(S->max_chunk, 2 * grid);
  S->classes.push_back(c);
  *out = &S->classes.back();
  return EE_OK;
}

}  // namespace

extern "C" {

ee_status ee_server_create(const ee_launch_cfg* cfg, int32_t n_therm, int32_t max_inflight, int32_t chunk_units,
                           ee_server** out) {
  g_err.clear();
  if (!out) return fail(EE_EINVAL, "out is NULL");
  ee_status s = check_cfg(cfg);
  if (s) return s;
  if (n_therm < 0) return fail(EE_EINVAL, "n_therm must be >= 0");
  if (max_inflight < 1 || max_inflight > 8) return fail(EE_EINVAL, "max_inflight must be in [1, 8]");
  if (chunk_units < 0 || chunk_units > (1 << 20)) return fail(EE_EINVAL, "chunk_units must be in [0, 2^20]");
  ee_server* S = new ee_server();
  S->cfg = cfg ? *cfg : ee_launch_cfg{0, 0, 0, 1, 0};
  S->n_therm = n_therm;
  S->max_chunk = chunk_units > 0 ? chunk_units : 8192;
  S->off_tab = kAlign;
  S->off_units = align_up(S->off_tab + sizeof(void*) * S->max_chunk);
  S->bytes = S->off_units + sizeof(ee::Unit) * S->max_chunk;
  S->slots.resize(max_inflight);
  for (SrvSlot& sl : S->slots) {
    hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&sl.dev), S->bytes);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&sl.host), S->bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      server_free(S);
      return fail(EE_EHIP, "server set-up: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = hipStreamCreateWithFlags(&S->est_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    server_free(S);
    return fail(EE_EHIP, "server set-up: %s", hipGetErrorString(e));
  }
  *out = S;
  return EE_OK;
}

ee_status ee_server_submit(ee_server* S, ee_job* job) {
  g_err.clear();
  if (!S || !job) return fail(EE_EINVAL, "NULL argument");
  ee_job* one[1] = {job};
  ee_status s = check_batch(one, 1, S->n_therm, nullptr);
  if (s) return s;
  SrvClass* C = nullptr;
  s = server_class(S, job, &C);
  if (s) return s;
  const int block = std::max(C->block, min_block(job->L));
  const int k = choose_slots(job->L, job->d.n_replicas, block, std::max(C->budget, job->L.traj_words * 4),
                             job->d.n_traj);
  const double cost = unit_cost(job, block, k, S->n_therm);
  hipEvent_t ev = nullptr;
  s = server_event(S, &ev);
  if (s) return s;
  // the chunks that run the job wait (on the device) for its table upload
  const hipError_t e = hipEventRecord(ev, job->stream);
  if (e != hipSuccess) {
    S->spare_events.push_back(ev);
    return fail(EE_EHIP, "hipEventRecord: %s", hipGetErrorString(e));
  }
  int id;
  if (!S->free_ids.empty()) {
    id = S->free_ids.back();
    S->free_ids.pop_back();
  } else {
    id = (int)S->jobs.size();
    S->jobs.emplace_back();
  }
  SrvJob& sj = S->jobs[id];
  sj.job = job;
  sj.units_left = (job->d.n_traj + k - 1) / k;
  sj.uploaded = ev;
  sj.upload_seen = false;
  for (int j0 = 0; j0 < job->d.n_traj; j0 += k)
    C->pending.push_back(SrvUnit{id, j0, std::min(k, job->d.n_traj - j0), k, cost, S->seq++});
  job->state = SERVED;
  S->open_jobs += 1;
  return server_progress(S);
}

ee_status ee_server_poll(ee_server* S, ee_job** done, int32_t cap, int32_t* n_done) {
  g_err.clear();
  if (!S || !n_done || (cap > 0 && !done)) return fail(EE_EINVAL, "NULL argument");
  *n_done = 0;
  ee_status s = server_progress(S);
  if (s) return s;
  while (*n_done < cap && !S->ready.empty()) {
    const int id = S->ready.front();
    S->ready.pop_front();
    // its estimate has completed: later reads use the job's own stream, not
    // the server's (which ee_server_destroy frees)
    SrvJob& sj = S->jobs[id];
    ee_job* j = sj.job;
    j->state = DONE;
    j->est_stream = j->stream;
    done[(*n_done)++] = j;
    S->spare_events.push_back(sj.uploaded);
    sj = SrvJob{};
    S->free_ids.push_back(id);
    S->open_jobs -= 1;
  }
  return EE_OK;
}

ee_status ee_server_stream(ee_server* S, void** stream) {
  g_err.clear();
  if (!S || !stream) return fail(EE_EINVAL, "NULL argument");
  *stream = reinterpret_cast<void*>(S->est_stream);
  return EE_OK;
}

ee_status ee_server_open_jobs(ee_server* S, int32_t* n) {
  g_err.clear();
  if (!S || !n) return fail(EE_EINVAL, "NULL argument");
  *n = S->open_jobs;
  return EE_OK;
}

ee_status ee_server_destroy(ee_server* S) {
  g_err.clear();
  if (!S) return EE_OK;
  for (SrvSlot& sl : S->slots)
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  if (S->est_stream) (void)hipStreamSynchronize(S->est_stream);
  // jobs not yet reported: those whose estimator was launched (it has now
  // completed) are DONE; the others go back to CREATED (their partial device
  // state is redrawn by the next run).  None keeps the server's stream.
  for (SrvJob& sj : S->jobs) {
    ee_job* j = sj.job;
    if (!j || j->state != SERVED) continue;
    if (sj.uploaded) (void)hipEventSynchronize(sj.uploaded);
    if (j->est_enqueued) {
      j->state = DONE;
    } else {
      j->state = CREATED;
      j->spins_exist = false;
      j->g = 0;
      j->n_therm_total = 0;
    }
    j->est_stream = j->stream;
  }
  server_free(S);
  return EE_OK;
}

}  // extern "C"
