// ee_internal.hpp -- structures shared by the host runtime and the gfx950
// kernels of the non-equilibrium Renyi-entropy estimator.
//
// Device data layout of one job (all inside the caller's arena):
//
//   [jobdev]     ee_jobdev descriptor (read by every kernel)
//   [selfptr]    one pointer to the descriptor (a 1-entry job table)
//   [result]     ee_result written by the estimator kernel
//   [ramp_thr]   (S+1) x (8*dim) uint32 Metropolis thresholds of the ramped
//                sites (S = N, or N/ly for the subset protocol), indexed
//                [m][fa][b][c]: fa = anti-aligned fixed
//                neighbours (0..2dim-1), b = intra partner anti-aligned,
//                c = inter partner anti-aligned
//   [work]       n_traj x int64 integer works I_j, then 2 n_traj doubles of
//                estimator scratch (the exponentials e_j and the
//                leave-one-out estimates)
//   [spins]      n_traj trajectories, each two colour planes
//                [colour][replica][row = t*ly + y][word], where a row of one
//                colour holds the lx/2 sites x = 2h + ((colour+t+y)&1),
//                h = 0..lx/2-1.  INT8: G = ceil(lx/8) 32-bit words per row,
//                one byte per site (bit 0 = 1 for spin +1), pad bytes 0.
//                BITPACKED: ceil(lx/64) words per row, bit h%32 of word h/32.
//
// On chip (LDS) a trajectory is always held in the INT8 layout.
#pragma once
#include <stdint.h>

#include "../../include/ee.h"

namespace ee {

constexpr int kMaxSlots = 16;  // trajectories per workgroup at most
// The sweep kernels' small tables (unit index, per-slot work sums, threshold
// table) follow the trajectory slots in dynamic LDS: a launch whose slots
// take lds_bytes asks for lds_bytes + kSweepTailBytes and passes the
// tables' word offset.
constexpr int kSweepTailBytes = 128;
static_assert((4 + kMaxSlots + 8) * 4 <= kSweepTailBytes, "sweep LDS tables");
inline int sweep_tail_words(int lds_bytes) { return (lds_bytes + 15) / 16 * 4; }
constexpr int kEstimateThreads = 1024;  // workgroup size of the estimator kernel
constexpr uint32_t kFlagInit = 1u;   // draw the initial spins (else load them)
constexpr uint32_t kFlagProto = 2u;  // run the N protocol sweeps after n_therm sweeps

struct alignas(256) JobDev {
  int32_t dim, lt, lx, ly, n, l, N, n_traj;
  int32_t H;            // sites per colour row = lx/2
  int32_t G;            // int8 words per colour row = ceil(H/4) = Philox groups per row
  int32_t R;            // rows per replica = lt*ly
  int32_t traj_words;   // int8 words per trajectory = 2*n*R*G
  int32_t packed_words; // bit-packed words per trajectory = 2*n*R*ceil(H/32)
  int32_t S;            // weight unit beta/S: N, or N/ly for the subset protocol
  int32_t subsets;      // EE_FLAG_SUBSETS: rows of the ramped column moved one at a time
  int32_t whole;        // EE_FLAG_WHOLE: every cut link of x < l ramped, none glued
  uint32_t key0, key1;  // Philox key
  uint32_t thr_bulk[4]; // U for a = 0..dim-1 anti-aligned neighbours (bulk/glued sites)
  uint32_t reverse;     // EE_FLAG_REVERSE
  uint32_t spin_format; // ee_spin_format
  uint32_t magic_R, shift_R, magic_Ly, shift_Ly;  // unsigned division by R and ly
  double beta;
  const uint32_t* ramp_thr;
  uint32_t* spins;
  int64_t* work;
  ee_result* result;
};

struct Unit {      // one work unit of the batch queue
  int32_t job;     // index into the job table
  int32_t j0;      // first trajectory
  int32_t count;   // trajectories in this unit (<= slots)
  int32_t slots;   // trajectories per workgroup for this job (LDS slots)
};

// q = n / d for n < 2^31 with (magic, shift) from make_magic (round-up method
// of Granlund & Montgomery, PLDI'94).
struct Magic {
  uint32_t mul, shift;
};
inline Magic make_magic(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return Magic{(uint32_t)m, l};
}

}  // namespace ee

// Launch helpers implemented in ee_kernels.hip.
extern "C" {
int ee_k_launch_sweep(const ee::JobDev* single_job, int single_k, const ee::Unit* units, int n_units, int* queue,
                      const ee::JobDev* const* jobtab, uint32_t flags, int n_therm, int g0, int grid, int block,
                      int lds_bytes, void* stream);
int ee_k_launch_queue_reset(int* queue, void* stream);
int ee_k_launch_estimate(const ee::JobDev* const* jobtab, int count, void* stream);
int ee_k_sweep_kernel_ptr(const void** fn);
int ee_k_queue_reset_ptr(const void** fn);
int ee_k_estimate_ptr(const void** fn);
int ee_k_max_lds_bytes();
int ee_k_launch_stream_sweep(const ee::JobDev* job, int n_traj, int lanes, int c, uint32_t g, int pos, int dpos,
                             int work, void* stream);
int ee_k_launch_stream_init(const ee::JobDev* job, int n_traj, int lanes, void* stream);
int ee_k_launch_zero_work(const ee::JobDev* job, int n_traj, void* stream);
// Plane-marching kernel: LDS bytes of a workgroup whose plane (one
// replica, both colours) has plane_words words; one sweep (main pass over
// n_traj * n_replicas * nseg workgroups, then the fix-up pass).
int ee_k_march_lds_bytes(int plane_words);
int ee_k_launch_march(const ee::JobDev* job, int n_traj, int n_replicas, int nseg, int block, int plane_words,
                      uint32_t g, int pos, int dpos, int work, void* stream);
size_t ee_k_scratch_bytes();
int ee_k_scratch_ptr(void** out);
}
