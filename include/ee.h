/*
 * ee.h -- C ABI of the MI355X (gfx950) implementation of the non-equilibrium
 * Monte Carlo estimator of Renyi-entropy increments of Bulgarelli & Panero,
 * "Entanglement entropy from non-equilibrium Monte Carlo simulations"
 * (arXiv:2304.03311).
 *
 * One "job" is one increment Delta S_n(l) = S_n(l+1) - S_n(l) of an Ising
 * model (D = 2 or 3) on n replicas glued along region A (Sec. 3): n_traj
 * independent non-equilibrium trajectories, each thermalised at lambda = 0
 * (geometry A(l)) and then driven to lambda = 1 (geometry A(l+1)) in N
 * checkerboard-Metropolis sweeps while the couplings of the column x = l are
 * ramped linearly (Sec. 3, linear protocol).  The work of each trajectory is
 * kept as an exact integer I_j, W_j = -(beta/N) I_j, and
 * Delta F = -log <exp(-W)> (App. A, Jarzynski's equality) gives
 * Delta S_n = Delta F / (n-1) (Sec. 2, derivative of the Renyi entropy).
 *
 * Conventions (the paper is silent on them; they make results bit-exact
 * between the GPU path and any other implementation that follows them):
 *   sites (r,t,y,x): replica r < n, Euclidean time t < lt, y < ly (ly = 1 in
 *   2D), x < lx; periodic in t, y, x.  The cut lies on the temporal links
 *   from t = 0 to t = 1.  Columns x < l are glued: (r,0,y,x) couples to
 *   ((r+1)%n,1,y,x).  The ramped column x = l couples (r,0,y,l) to (r,1,y,l)
 *   with beta(1 - m/N) and to ((r+1)%n,1,y,l) with beta m/N.  Colour =
 *   (t+y+x) mod 2; a sweep updates colour 0, then colour 1.  A flip is
 *   accepted iff u <= U, u a uint32 from Philox4x32-10 keyed by the seed,
 *   U = max(floor(2^32 exp(-(2 beta K)/N)), 1) - 1 for K > 0 (K = the
 *   integer energy cost in units of beta/N) and U = 2^32-1 otherwise.
 *   The work is measured on the configuration before each sweep, and the
 *   sweep runs at the new coupling (App. A, work in one Monte Carlo step).
 *
 * Every call returns an ee_status (0 = EE_OK, < 0 = error).  No exception
 * crosses the ABI.  On error the call has no effect on the job and
 * ee_last_error() describes the failure (thread-local, valid until the next
 * call on the same thread).
 *
 * Memory: the caller owns all device memory.  A job lives in one
 * caller-provided device "arena" of ee_job_footprint() bytes that must stay
 * allocated until ee_job_destroy().  The library keeps only host state per
 * job, plus one small internal device buffer per device for batch metadata.
 *
 * Streams: every device operation of a job is enqueued on the HIP stream
 * given to ee_job_create (a hipStream_t passed as void*; NULL = the null
 * stream).  Calls are asynchronous unless stated otherwise.  One job must not
 * be used from two threads at the same time.
 */
#ifndef EE_H
#define EE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EE_OK = 0,
  EE_EINVAL = -1,        /* invalid argument or job description            */
  EE_ENOMEM = -2,        /* arena smaller than ee_job_footprint()          */
  EE_EHIP = -3,          /* a HIP runtime call failed (text in last error) */
  EE_ESTATE = -4,        /* call not allowed in the job's current state    */
  EE_EUNSUPPORTED = -5   /* valid description this build cannot run        */
} ee_status;

/* Device storage format of the spins between calls. */
typedef enum {
  EE_SPINS_INT8 = 0,      /* one byte per site, colour-separated rows       */
  EE_SPINS_BITPACKED = 1  /* one bit per site, colour-separated rows        */
} ee_spin_format;

/* ee_job_desc.flags */
#define EE_FLAG_REVERSE 1u /* ramp lambda 1 -> 0: start from A(l+1) and remove
                              column l (the paper's "direct" realisation,
                              App. A direct/reverse equality).  The estimate
                              is then Delta F = -log Z_n(l)/Z_n(l+1).       */
#define EE_FLAG_SUBSETS 2u /* protocol 2 of App. B: the ly rows of the ramped
                              column move one after the other, row y during
                              steps [y S, (y+1) S) with S = n_step / ly
                              (n_step must be divisible by ly).  Couplings
                              are then in units of beta/S and
                              W_j = -(beta/S) I_j.  Identical to the default
                              protocol in 2D.                               */
#define EE_FLAG_WHOLE 4u   /* the whole-region protocol reviewed in Sec. 3:
                              start from n decoupled replicas and ramp every
                              cut link of A = {x < l} at once (intra
                              beta (1 - m/N), inter beta m/N) to A(l)
                              glued, so Delta F = (n-1) S_n(l) directly.
                              Needs 1 <= l <= lx; not with EE_FLAG_SUBSETS.
                              With EE_FLAG_REVERSE it starts from A(l).    */

/*
 * Problem statement of one job, in the paper's terms (Sec. 3; Sec. 4 and 5
 * conventions: lattice extents, replica number n, beta, region size l,
 * protocol length N, trajectory count n_t).
 * Constraints: dim in {2,3}; lt, lx even >= 2; ly == 1 for dim 2, even >= 2
 * for dim 3; n_replicas >= 2; beta finite >= 0; 0 <= l < lx (1 <= l <= lx
 * with EE_FLAG_WHOLE); n_step >= 1;
 * 1 <= n_traj <= 65535.  Violations return EE_EINVAL.
 */
typedef struct {
  int32_t dim;          /* D = 2 or 3                                        */
  int32_t lt, lx, ly;   /* L_tau, L_x, L_y (ly = 1 in 2D)                    */
  int32_t n_replicas;   /* n                                                 */
  int32_t l;            /* |A| before the ramp; column x = l is ramped       */
  int32_t n_step;       /* N: protocol sweeps, lambda_m = m/N                */
  int32_t n_traj;       /* n_t: independent trajectories                     */
  double beta;          /* inverse temperature of the bulk couplings         */
  uint64_t seed;        /* Philox key of the job                             */
  int32_t spin_format;  /* ee_spin_format                                    */
  uint32_t flags;       /* EE_FLAG_* bits; 0 = the forward (add-column) ramp */
} ee_job_desc;

/*
 * Result of one job (App. A estimator; Sec. 2 for dS).
 *   dF      = -log( (1/n_t) sum_j exp(-W_j) ),  W_j = -(beta/S) I_j with
 *             S = N (S = N/ly with EE_FLAG_SUBSETS)
 *   dS      = dF / (n-1)
 *   dF_err  delete-one jackknife standard error of dF (NaN if n_t < 2)
 *   w_mean, w_var  mean and population variance of W
 *   ess     (sum e_j)^2 / sum e_j^2, e_j = exp(-W_j)
 *   i_min, i_max  extreme integer works
 *   attempts      n_t * n * lt*ly*lx * (thermalisation sweeps + N)
 */
typedef struct {
  double dF, dS, dF_err, w_mean, w_var, ess;
  int64_t i_min, i_max, attempts;
  int32_t n_traj;
  int32_t reserved;
} ee_result;

typedef struct ee_job ee_job; /* opaque host-side handle */

/* Device bytes a job needs (spins of every trajectory, works, threshold
 * tables, result).  No device work.  EE_EINVAL for a bad description,
 * EE_EUNSUPPORTED for a bit-packed job that cannot run on chip: its
 * trajectory exceeds one workgroup's LDS, or a row has more than 1024
 * words (lx/2 > 4096 sites).  Such lattices are streamed from HBM in INT8. */
ee_status ee_job_footprint(const ee_job_desc* desc, size_t* bytes);

/* *on_chip = 1 if the job's trajectories run on chip (one trajectory fits
 * a workgroup's LDS and a row has at most 1024 words), 0 if they are
 * streamed from HBM (per-job path only).  No device work. */
ee_status ee_job_on_chip(const ee_job_desc* desc, int32_t* on_chip);

/* Validate desc, build the geometry and the uint32 threshold tables on the
 * host (FP64 libm exp, Sec. 3 couplings), and enqueue their upload into the
 * arena on hip_stream.  arena: device pointer, 256-byte aligned, at least
 * ee_job_footprint() bytes; borrowed (not freed by the library).  The
 * description is copied.  State after success: CREATED. */
ee_status ee_job_create(const ee_job_desc* desc, void* dev_arena, size_t arena_bytes,
                        void* hip_stream, ee_job** out);

/* Thermalisation (Sec. 4 conventions: sweeps at fixed lambda = 0 before the
 * protocol).  The first call also draws the initial spins (Philox, each
 * spin +1 with probability 1/2).  Runs n_sweeps >= 0 sweeps at the starting
 * coupling; several calls add up.  Allowed in CREATED state only. Async. */
ee_status ee_thermalize(ee_job* job, int32_t n_sweeps);

/* The non-equilibrium protocol (Sec. 3 linear protocol; App. A): for
 * k = 0..N-1, I_j += D_k(phi_k), then one sweep at lambda_{k+1}.  Exactly
 * once per job, after at least one ee_thermalize call (which may be 0
 * sweeps).  State after: DONE.  Async. */
ee_status ee_run_protocol(ee_job* job);

/* Jarzynski estimator (App. A) over the job's n_t works, computed on the
 * device (integer max, FP64 sum of exponentials, log-sum-exp, jackknife);
 * copies the result to *out.  DONE state only.  Synchronises the stream. */
ee_status ee_estimate(ee_job* job, ee_result* out);

/* Copy I_j for j < count (count <= n_traj) to host memory.  DONE state
 * only.  Synchronises the stream. */
ee_status ee_job_read_work(ee_job* job, int64_t* host_I, int32_t count);

/* Copy the spins of trajectories j < count / (n*lt*ly*lx) as +-1 bytes in
 * canonical order idx = ((((j*n + r)*lt + t)*ly + y)*lx + x).  count must be
 * a multiple of n*lt*ly*lx and at most n_traj of them.  Allowed once spins
 * exist (after the first ee_thermalize).  Synchronises the stream. */
ee_status ee_job_read_spins(ee_job* job, int8_t* host, size_t count);

/* Return the job to CREATED state (spins and works are redrawn by the next
 * run; results are bit-identical to the first run).  Async-safe: only host
 * state changes. */
ee_status ee_job_reset(ee_job* job);

/* Persistent fused path (many jobs of uneven shape and protocol length).
 * Every job must be CREATED.  One persistent launch runs, for every
 * trajectory of every job: the initial spins, n_therm sweeps at the starting
 * coupling and the N protocol sweeps with the work; then one launch computes
 * every job's estimate.  Work units (job, block of trajectories) are drawn
 * from a device queue, longest first.  The launch sequence is recorded in a
 * HIP graph and replayed when the same jobs are run again.  All jobs end in
 * DONE; their results are then read with ee_estimate.  Results are
 * bit-identical to the per-job path (ee_thermalize + ee_run_protocol).
 * Jobs on the HBM-streaming path are rejected with EE_EUNSUPPORTED.
 * hip_stream: stream of the batch (the jobs' own streams are not used). */
ee_status ee_batch_run(ee_job* const* jobs, int32_t count, int32_t n_therm, void* hip_stream);

/* Launch shape of the sweep kernel (what the autotuner varies). */
typedef struct {
  int32_t block_threads;   /* threads per workgroup: 64..1024, multiple of 64; 0 = about
                              one thread per four words of a trajectory's colour plane
                              (n*lt*ly*ceil(lx/8)/4, rounded up to 64, at most 1024);
                              raised to ceil(lx/8) rounded up to 64 when smaller (one lane
                              per word of a row)                                           */
  int32_t lds_bytes;       /* LDS budget per workgroup (bytes); 0 = default               */
  int32_t grid_blocks;     /* persistent workgroups; 0 = one wave of the whole GPU (with
                              EE_LAUNCH_MARCH: segments per trajectory, 0 = the runtime's) */
  int32_t use_graph;       /* 1 = record/replay a HIP graph (default), 0 = direct launches  */
  uint32_t flags;          /* EE_LAUNCH_* bits                                            */
} ee_launch_cfg;

/* ee_launch_cfg.flags: run a job on the HBM-streaming path even if its
 * trajectories fit on chip (per-job path only; needs EE_SPINS_INT8).  Jobs
 * whose trajectory exceeds one workgroup's LDS always use that path: the
 * spins stay in HBM and every half-sweep is one launch over all
 * trajectories, with bit-identical results. */
#define EE_LAUNCH_STREAMING 1u
/* Kernel of the HBM-streaming path (either flag implies EE_LAUNCH_STREAMING).
 * Streamed jobs run the two-pass kernel (one launch per colour: 3 B of HBM
 * traffic per site and sweep) unless EE_LAUNCH_MARCH selects the
 * plane-marching kernel: each workgroup marches the t-planes of one segment
 * of one replica of one trajectory through a five-slot LDS ring (a plane:
 * both colours, all y, 2 ly G words), updating colour 0 of plane p and
 * colour 1 of plane p-1 at each step, so each plane is read and written once
 * per sweep (2 B per site); colour 1 of each segment's first and last plane
 * (planes t = 0 and 1 among them) follows in a second launch.  grid_blocks
 * > 0 then sets the segments per trajectory (at most lt/2), else the
 * runtime picks them; ee_job_set_launch returns EE_EUNSUPPORTED if the ring
 * does not fit LDS.  EE_LAUNCH_TWO_PASS names the default explicitly.
 * Results are bit-identical either way. */
#define EE_LAUNCH_MARCH 2u
#define EE_LAUNCH_TWO_PASS 4u
/* ee_batch_run with an explicit launch shape (NULL = defaults). */
ee_status ee_batch_run_cfg(ee_job* const* jobs, int32_t count, int32_t n_therm,
                           const ee_launch_cfg* cfg, void* hip_stream);

/* Allocation-free variant of ee_batch_run_cfg, for callers that cannot
 * allocate device memory (code that must not call hipMalloc: under graph
 * capture, in tight serving loops, in harnesses that forbid it).  Same
 * kernels and bit-identical results.  The queue counter, job table and
 * unit table go into a fixed static device array of 2 MiB per GPU, held
 * until the process ends; a batch whose tables need more (256 + 8 count
 * rounded up to 256, plus 16 bytes per work unit) returns EE_EINVAL before
 * any device work.  It calls no hipMalloc or hipFree, records no graph and
 * creates no event (cfg->use_graph is ignored; ee_batch_kernel_ms does not
 * time it).  The unit table is copied from host memory on hip_stream, and
 * the call waits for that copy (and so for the work queued before it).
 * Every call on one GPU uses the same array: calls on one stream are
 * ordered, but calls that overlap on one GPU (other streams, other
 * threads) race and must not be made. */
ee_status ee_batch_run_noalloc(ee_job* const* jobs, int32_t count, int32_t n_therm, const ee_launch_cfg* cfg,
                               void* hip_stream);

/*
 * Continuous batching (serving).  A server runs the persistent sweep kernel
 * over the work units (blocks of trajectories) of the jobs submitted to it,
 * in chunks.  A job's units belong to its launch class: the job's own shape
 * if ee_job_set_launch gave block_threads and lds_bytes, else the server's.
 * Units queue per class in submission order; whenever one of the server's
 * max_inflight launch slots is free, the class holding the oldest waiting
 * unit fills a chunk (at most chunk_units, or twice the workgroups of its
 * shape that fit on the GPU at once) that runs in one persistent launch on
 * that slot's stream.  Chunks overlap on the device, so jobs submitted while
 * others run start as soon as a slot frees, and each chunk's workgroups fill
 * the CUs the previous chunk's tail leaves idle.  When every unit of a job
 * has run, its estimator runs on the server's service stream, and
 * ee_server_poll then reports the job DONE (its result is read with
 * ee_estimate).  Results are bit-identical to the per-job and batch paths,
 * whatever else is on the server.  The server owns its streams (default
 * priority, non-blocking), one device table buffer and one pinned staging
 * buffer per slot.  One server must not be used from two threads at once.
 */
typedef struct ee_server ee_server;

/* cfg: the default block_threads (0 = 256) and lds_bytes (0 = default) of
 * chunk launches, grid_blocks as for ee_batch_run_cfg; use_graph is
 * ignored.  n_therm: thermalisation sweeps of every job.  max_inflight:
 * launch slots (1..8).  chunk_units: work units per launch at most (0 =
 * 8192, and per class twice its workgroups that fit on the GPU at once). */
ee_status ee_server_create(const ee_launch_cfg* cfg, int32_t n_therm, int32_t max_inflight, int32_t chunk_units,
                           ee_server** out);

/* Queue a CREATED job (fresh, on chip; EE_EUNSUPPORTED for jobs on the
 * HBM-streaming path), then launch chunks on free slots.  Does not wait on
 * the host: the chunks that run the job wait on the device for its table
 * upload on its own stream.  The job is then SERVED: every other call on it
 * returns EE_ESTATE (ee_job_destroy included) until a poll has reported
 * it. */
ee_status ee_server_submit(ee_server* srv, ee_job* job);

/* Non-blocking progress: collect finished chunks, launch estimators of jobs
 * whose units have all run, refill free slots.  Writes up to cap jobs
 * whose estimate has completed to done[] (in completion order) and their
 * number to *n_done; those jobs are DONE, and later reads of them run on
 * their own streams. */
ee_status ee_server_poll(ee_server* srv, ee_job** done, int32_t cap, int32_t* n_done);

/* The server's service stream (a hipStream_t), on which it launches the
 * estimators.  Creating the jobs for a server on this stream (ee_job_create)
 * keeps their table uploads off the chunk streams: with more streams than
 * the device has hardware queues, streams share in-order queues, and an
 * upload queued behind a long chunk kernel would hold up ee_server_submit.
 * Owned by the server. */
ee_status ee_server_stream(ee_server* srv, void** stream);

/* Jobs submitted and not yet returned by ee_server_poll. */
ee_status ee_server_open_jobs(ee_server* srv, int32_t* n);

/* Wait for the server's device work and free it.  Jobs not yet returned by
 * a poll become DONE if their estimator was launched (it has completed),
 * else go back to CREATED. */
ee_status ee_server_destroy(ee_server* srv);

/* Per-job launch shape for ee_thermalize / ee_run_protocol (NULL = default). */
ee_status ee_job_set_launch(ee_job* job, const ee_launch_cfg* cfg);

/* Device time (ms, HIP events on the batch stream) of the persistent sweep
 * kernel of the most recent ee_batch_run* on this thread.  Waits for it. */
ee_status ee_batch_kernel_ms(double* ms);

/* Destroy the host handle.  Does not free the arena.  Waits for the job's
 * outstanding device work first. */
ee_status ee_job_destroy(ee_job* job);

/* Text of the last error on this thread ("" if none).  Never NULL. */
const char* ee_last_error(void);

/* Library version string. */
const char* ee_version(void);

/* Hash of the sources the library was built from (the build script passes
 * it in; the Python binding refuses a library whose hash differs from that
 * of the sources next to it).  Never NULL. */
const char* ee_build_id(void);

#ifdef __cplusplus
}
#endif

#endif /* EE_H */
