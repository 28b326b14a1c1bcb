/*
 * ee_oracle.c -- reference CPU implementation.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this file's library.  The product path (HIP kernels + C ABI in
 * paper_2304_03311_amd/) shares no code with it and never calls it.
 *
 * A plain, slow, single-threaded simulator of the non-equilibrium
 * (Jarzynski) estimator of the Renyi-entropy increment of Bulgarelli &
 * Panero, "Entanglement entropy from non-equilibrium Monte Carlo
 * simulations" (arXiv:2304.03311):
 *
 *   - n-replica Ising lattice with a cut orthogonal to Euclidean time
 *     (Sec. 3, replica Hamiltonian with beta^(k,k) and beta^(k,k+1));
 *   - region A = slab of columns x < l, glued lower-side(replica r) to
 *     upper-side(replica r+1) (Sec. 3; cyclic gluing of Sec. 2);
 *   - the c-function protocol: the couplings of the column x = l are ramped
 *     linearly, beta^(k,k) = beta (1 - m/N), beta^(k,k+1) = beta m/N
 *     (Sec. 3, linear protocol), so lambda = 0 is A(l) and lambda = 1 is
 *     A(l+1);
 *   - the whole-region protocol reviewed in Sec. 3 (flag bit 2): every cut
 *     link of A = {x < l} is ramped at once, intra beta (1 - m/N), inter
 *     beta m/N, from n decoupled replicas (lambda = 0) to A(l) glued
 *     (lambda = 1), so Delta F = (n-1) S_n(l) directly;
 *   - work on phi_k, then an update at lambda_{k+1} (App. A, eq. for the
 *     work in one Monte Carlo step and the discretised average);
 *   - exp(-W) averaged over trajectories (App. A, Jarzynski's equality),
 *     Delta F = -log <exp(-W)> = (n-1) [S_n(l+1) - S_n(l)] (Sec. 2, eq. for
 *     the derivative of the Renyi entropy).
 *
 * The Monte Carlo update is checkerboard Metropolis (the paper uses
 * Swendsen-Wang; App. A only needs a transition kernel that satisfies
 * detailed balance at fixed lambda).  The paper is silent on the random
 * numbers; the conventions below are this project's reading and are the
 * contract that makes the GPU path bit-comparable:
 *
 *   Lattice   sites (r,t,y,x), r<n, t<Lt, y<Ly, x<Lx, periodic; Ly = 1 in
 *             2D.  Each site owns its +x, +y (3D) and +t bonds.
 *   Cut       the +t bond of (r,0,y,x): x <  l -> ((r+1)%n, 1, y, x)
 *                                       x == l -> ramped (intra + inter)
 *                                       x >  l -> (r, 1, y, x)
 *             whole-region protocol:    x <  l -> ramped (intra + inter)
 *                                       x >= l -> (r, 1, y, x)
 *   Weights   integer, in units of beta/N: bulk N, ramped intra N-m,
 *             ramped inter m.  H/T = -(beta/N) sum_b w_b s_a s_b.  (With
 *             subsets, below, N is replaced by S everywhere.)
 *   Colour    (t+y+x) mod 2; a sweep = colour 0 then colour 1.
 *   Accept    K = s_i * sum_b w_b s_nb; accept iff u <= U(K) with
 *             U(K) = 2^32-1 if beta*K <= 0, else
 *             max(floor(2^32 exp(-(2 beta K)/N)), 1) - 1, evaluated in
 *             FP64 exactly as (2.0*beta*(double)K)/(double)N, and u a
 *             uniform 32-bit integer u = 2^16 v + w (below).
 *   RNG       Philox4x32-10 (Salmon et al., SC'11), key = (seed lo, seed
 *             hi).  Site with colour c, half-index h = x>>1, row rho =
 *             t*Ly+y.
 *             Initial spin (phase 0, g = 0): with G4 = ceil((Lx/2)/4),
 *               counter = (rho*G4 + (h>>2), 0, j, (r<<1)|c), +1 iff output
 *               word (h & 3) < 2^31.
 *             Sweep g (thermalisation sweeps first, then the protocol):
 *             with G8 = ceil((Lx/2)/8), one call serves the 8 sites of a
 *             row with the same h>>3:
 *               counter = (rho*G8 + (h>>3), g, j, (phase<<28)|(r<<1)|c),
 *               field(phase) = 16-bit half (h & 1) (low half first) of
 *               output word ((h & 7) >> 1);
 *             v = field(1); w = field(2) is drawn only when v = U >> 16,
 *             the only case in which u <= U depends on it.  So u is uniform
 *             on [0, 2^32) and P(accept) = (U+1)/2^32 exactly.
 *   Work      D_k = sum over ramped bonds of (w(m_{k+1}) - w(m_k)) s s,
 *             I = sum_k D_k, W = -(beta/N) I   (exact integer).
 *   Reverse   flag bit 0: start at lambda = 1 (geometry A(l+1)) and ramp
 *             to lambda = 0 (the paper's "direct" realisation, App. A
 *             direct/reverse equality).
 *   Subsets   flag bit 1 (App. B, protocol 2): the Ly rows of the ramped
 *             column are ramped one after the other, row y during steps
 *             [y S, (y+1) S) with S = N / Ly; all weights are then in units
 *             of beta/S (bulk S, intra S - m_y, inter m_y) and W = -(beta/S) I.
 *             Without the flag S = N and every row has m_y = m.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EO_OK 0
#define EO_EINVAL -1
#define EO_ENOMEM -2

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon, Moraes, Dror, */
/* Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).        */
/* ------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n1 = lo1;
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  uint32_t n3 = lo0;
  c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void eo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k[0] += 0x9E3779B9u; /* Weyl key schedule */
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* ------------------------------------------------------------------ */
/* Metropolis threshold (acceptance as an integer compare).            */
/* ------------------------------------------------------------------ */
uint32_t eo_threshold(double beta, int64_t K, int32_t N) {
  if (beta * (double)K <= 0.0) return 0xFFFFFFFFu;
  double x = (2.0 * beta * (double)K) / (double)N; /* Delta(H/T) of the flip */
  double p = exp(-x);
  double f = floor(ldexp(p, 32));
  if (f >= 4294967296.0) return 0xFFFFFFFFu;
  if (f < 1.0) f = 1.0;
  return (uint32_t)(f - 1.0);
}

/* ------------------------------------------------------------------ */
/* Geometry: an explicit bond list of the replica lattice.             */
/* ------------------------------------------------------------------ */
enum { BOND_BULK = 0, BOND_INTRA = 1, BOND_INTER = 2 };

typedef struct {
  int dim, lt, lx, ly, n;
  double beta;
  int l, N, n_traj;
  uint64_t seed;
  int reverse;
  int subsets;     /* protocol 2 of App. B */
  int S;           /* weight unit: beta/S (S = N, or N/Ly with subsets) */
  int64_t V;       /* sites per replica */
  int64_t nsites;  /* n * V */
  /* bonds */
  int64_t nb;
  int64_t *ba, *bb;
  int8_t *bk;
  int32_t *by;     /* y of each bond (the ramped row it belongs to) */
  /* per-site adjacency in CSR form */
  int64_t *adj_off;
  int64_t *adj_nbr;
  int8_t *adj_kind;
  int32_t *adj_y;
} geom;

static int64_t site_index(const geom* G, int r, int t, int y, int x) {
  return (((int64_t)r * G->lt + t) * G->ly + y) * G->lx + x;
}

static void add_bond(geom* G, int64_t a, int64_t b, int kind, int y) {
  G->ba[G->nb] = a; G->bb[G->nb] = b; G->bk[G->nb] = (int8_t)kind; G->by[G->nb] = y; G->nb++;
}

static void geom_free(geom* G) {
  free(G->ba); free(G->bb); free(G->bk); free(G->by);
  free(G->adj_off); free(G->adj_nbr); free(G->adj_kind); free(G->adj_y);
  memset(G, 0, sizeof(*G));
}

static int geom_build(geom* G, int dim, int lt, int lx, int ly, int n, double beta, int l, int N,
                      int n_traj, uint64_t seed, int flags) {
  memset(G, 0, sizeof(*G));
  if (dim != 2 && dim != 3) return EO_EINVAL;
  if (dim == 2 && ly != 1) return EO_EINVAL;
  if (lt < 2 || lx < 2 || ly < 1 || (lt & 1) || (lx & 1) || (dim == 3 && ((ly & 1) || ly < 2))) return EO_EINVAL;
  const int whole = (flags >> 2) & 1;
  if (n < 2 || !(beta >= 0.0) || N < 1 || n_traj < 0) return EO_EINVAL;
  if (whole ? (l < 1 || l > lx || (flags & 2)) : (l < 0 || l >= lx)) return EO_EINVAL;
  G->dim = dim; G->lt = lt; G->lx = lx; G->ly = ly; G->n = n; G->beta = beta;
  G->l = l; G->N = N; G->n_traj = n_traj; G->seed = seed; G->reverse = flags & 1;
  G->subsets = (flags >> 1) & 1;
  if (G->subsets && N % ly) return EO_EINVAL;
  G->S = G->subsets ? N / ly : N;
  G->V = (int64_t)lt * ly * lx;
  G->nsites = (int64_t)n * G->V;
  /* a ramped column adds one bond per (r,y) */
  int64_t maxb = G->nsites * dim + (int64_t)n * ly * (whole ? l : 1);
  G->ba = (int64_t*)malloc(sizeof(int64_t) * maxb);
  G->bb = (int64_t*)malloc(sizeof(int64_t) * maxb);
  G->bk = (int8_t*)malloc(maxb);
  G->by = (int32_t*)malloc(sizeof(int32_t) * maxb);
  if (!G->ba || !G->bb || !G->bk || !G->by) { geom_free(G); return EO_ENOMEM; }
  for (int r = 0; r < n; ++r)
    for (int t = 0; t < lt; ++t)
      for (int y = 0; y < ly; ++y)
        for (int x = 0; x < lx; ++x) {
          int64_t s = site_index(G, r, t, y, x);
          add_bond(G, s, site_index(G, r, t, y, (x + 1) % lx), BOND_BULK, y);          /* +x */
          if (dim == 3) add_bond(G, s, site_index(G, r, t, (y + 1) % ly, x), BOND_BULK, y); /* +y */
          if (whole && t == 0 && x < l) {                                             /* ramped */
            add_bond(G, s, site_index(G, r, 1, y, x), BOND_INTRA, y);
            add_bond(G, s, site_index(G, (r + 1) % n, 1, y, x), BOND_INTER, y);
          } else if (whole) {                                                         /* +t */
            add_bond(G, s, site_index(G, r, (t + 1) % lt, y, x), BOND_BULK, y);
          } else if (t == 0 && x < l) {                                               /* glued */
            add_bond(G, s, site_index(G, (r + 1) % n, 1, y, x), BOND_BULK, y);
          } else if (t == 0 && x == l) {                                              /* ramped */
            add_bond(G, s, site_index(G, r, 1, y, x), BOND_INTRA, y);
            add_bond(G, s, site_index(G, (r + 1) % n, 1, y, x), BOND_INTER, y);
          } else {                                                                    /* +t */
            add_bond(G, s, site_index(G, r, (t + 1) % lt, y, x), BOND_BULK, y);
          }
        }
  /* adjacency */
  G->adj_off = (int64_t*)calloc((size_t)G->nsites + 1, sizeof(int64_t));
  G->adj_nbr = (int64_t*)malloc(sizeof(int64_t) * 2 * G->nb);
  G->adj_kind = (int8_t*)malloc(2 * G->nb);
  G->adj_y = (int32_t*)malloc(sizeof(int32_t) * 2 * G->nb);
  if (!G->adj_off || !G->adj_nbr || !G->adj_kind || !G->adj_y) { geom_free(G); return EO_ENOMEM; }
  for (int64_t b = 0; b < G->nb; ++b) { G->adj_off[G->ba[b] + 1]++; G->adj_off[G->bb[b] + 1]++; }
  for (int64_t s = 0; s < G->nsites; ++s) G->adj_off[s + 1] += G->adj_off[s];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * G->nsites);
  if (!fill) { geom_free(G); return EO_ENOMEM; }
  memcpy(fill, G->adj_off, sizeof(int64_t) * G->nsites);
  for (int64_t b = 0; b < G->nb; ++b) {
    int64_t a = G->ba[b], c = G->bb[b];
    G->adj_nbr[fill[a]] = c; G->adj_kind[fill[a]] = G->bk[b]; G->adj_y[fill[a]] = G->by[b]; fill[a]++;
    G->adj_nbr[fill[c]] = a; G->adj_kind[fill[c]] = G->bk[b]; G->adj_y[fill[c]] = G->by[b]; fill[c]++;
  }
  free(fill);
  return EO_OK;
}

/* Ramp position of row y when the protocol stands at position pos (0..N):
 * every row follows pos, or (subsets) row y moves during [y S, (y+1) S). */
static int row_m(const geom* G, int y, int pos) {
  if (!G->subsets) return pos;
  int m = pos - y * G->S;
  return m < 0 ? 0 : (m > G->S ? G->S : m);
}

/* bond weight in units of beta/S at protocol position pos */
static int64_t bond_weight(const geom* G, int kind, int y, int pos) {
  if (kind == BOND_INTRA) return (int64_t)(G->S - row_m(G, y, pos));
  if (kind == BOND_INTER) return (int64_t)row_m(G, y, pos);
  return (int64_t)G->S;
}

/* protocol position after step k (k = -1 is the starting point) */
static int ramp_pos(const geom* G, int k) {
  int forward = k + 1;
  return G->reverse ? G->N - forward : forward;
}

/* ------------------------------------------------------------------ */
/* Random numbers of one site                                          */
/* ------------------------------------------------------------------ */
static void site_philox(const geom* G, int group_size, uint32_t phase, uint32_t g, uint32_t j, int r, int t,
                        int y, int x, uint32_t out[4]) {
  int c = (t + y + x) & 1;
  int h = x >> 1;
  int groups = (G->lx / 2 + group_size - 1) / group_size;
  int rho = t * G->ly + y;
  uint32_t ctr[4] = {(uint32_t)(rho * groups + h / group_size), g, j,
                     (phase << 28) | ((uint32_t)r << 1) | (uint32_t)c};
  uint32_t key[2] = {(uint32_t)(G->seed & 0xFFFFFFFFu), (uint32_t)(G->seed >> 32)};
  eo_philox4x32_10(ctr, key, out);
}

/* uniform 32-bit word of the initial spin (4 sites per call) */
static uint32_t init_uniform(const geom* G, uint32_t j, int r, int t, int y, int x) {
  uint32_t out[4];
  site_philox(G, 4, 0, 0, j, r, t, y, x, out);
  return out[(x >> 1) & 3];
}

/* 16-bit field of a sweep's random numbers (8 sites per call) */
static uint32_t sweep_field(const geom* G, uint32_t phase, uint32_t g, uint32_t j, int r, int t, int y, int x) {
  uint32_t out[4];
  site_philox(G, 8, phase, g, j, r, t, y, x, out);
  int h = x >> 1;
  uint32_t word = out[(h & 7) >> 1];
  return (h & 1) ? (word >> 16) : (word & 0xFFFFu);
}

/* Metropolis decision u <= U with u = 2^16 v + w uniform on [0, 2^32) */
static int accept(const geom* G, uint32_t U, uint32_t g, uint32_t j, int r, int t, int y, int x) {
  uint32_t v = sweep_field(G, 1, g, j, r, t, y, x);
  uint32_t u_hi = U >> 16;
  if (v != u_hi) return v < u_hi;
  uint32_t w = sweep_field(G, 2, g, j, r, t, y, x);
  return w <= (U & 0xFFFFu);
}

/* ------------------------------------------------------------------ */
/* One trajectory                                                      */
/* ------------------------------------------------------------------ */
static void init_spins(const geom* G, uint32_t j, int8_t* s) {
  for (int r = 0; r < G->n; ++r)
    for (int t = 0; t < G->lt; ++t)
      for (int y = 0; y < G->ly; ++y)
        for (int x = 0; x < G->lx; ++x) {
          uint32_t u = init_uniform(G, j, r, t, y, x);
          s[site_index(G, r, t, y, x)] = (u < 0x80000000u) ? 1 : -1;
        }
}

/* One Metropolis sweep at protocol position pos: colour 0 over all replicas, then colour 1. */
static void sweep(const geom* G, int pos, uint32_t g, uint32_t j, int8_t* s) {
  for (int colour = 0; colour < 2; ++colour)
    for (int r = 0; r < G->n; ++r)
      for (int t = 0; t < G->lt; ++t)
        for (int y = 0; y < G->ly; ++y)
          for (int x = 0; x < G->lx; ++x) {
            if (((t + y + x) & 1) != colour) continue;
            int64_t i = site_index(G, r, t, y, x);
            int64_t field = 0;
            for (int64_t e = G->adj_off[i]; e < G->adj_off[i + 1]; ++e)
              field += bond_weight(G, G->adj_kind[e], G->adj_y[e], pos) * s[G->adj_nbr[e]];
            int64_t K = (int64_t)s[i] * field;
            uint32_t U = eo_threshold(G->beta, K, G->S);
            if (accept(G, U, g, j, r, t, y, x)) s[i] = (int8_t)(-s[i]);
          }
}

/* Integer energy in units of beta/S:  H/T = (beta/S) * energy_units. */
static int64_t energy_units(const geom* G, int pos, const int8_t* s) {
  int64_t e = 0;
  for (int64_t b = 0; b < G->nb; ++b)
    e -= bond_weight(G, G->bk[b], G->by[b], pos) * s[G->ba[b]] * s[G->bb[b]];
  return e;
}

/*
 * Run trajectories j0 <= j < j1 of one job: initial state, n_therm sweeps at
 * the starting ramp position, then the N protocol sweeps.  I_out[j - j0]
 * receives I_j (W_j = -(beta/S) I_j).  spins_out (nullable) receives the
 * final +-1 spins in the order ((((j-j0)*n + r)*Lt + t)*Ly + y)*Lx + x.
 * If n_step_run < N only the first n_step_run protocol sweeps are run (a
 * partial protocol, used to check resumption).
 */
int eo_run(int dim, int lt, int lx, int ly, int n, double beta, int l, int N, int n_traj,
           uint64_t seed, int flags, int n_therm, int j0, int j1, int n_step_run, int64_t* I_out,
           int8_t* spins_out) {
  geom G;
  int rc = geom_build(&G, dim, lt, lx, ly, n, beta, l, N, n_traj, seed, flags);
  if (rc) return rc;
  if (j0 < 0 || j1 < j0 || j1 > n_traj || n_therm < 0 || n_step_run < 0 || n_step_run > N) {
    geom_free(&G);
    return EO_EINVAL;
  }
  int8_t* s = (int8_t*)malloc((size_t)G.nsites);
  if (!s) { geom_free(&G); return EO_ENOMEM; }
  for (int j = j0; j < j1; ++j) {
    init_spins(&G, (uint32_t)j, s);
    uint32_t g = 0;
    int m0 = ramp_pos(&G, -1);
    for (int k = 0; k < n_therm; ++k) sweep(&G, m0, g++, (uint32_t)j, s);
    int64_t work_units = 0; /* sum_k [E(pos_{k+1}) - E(pos_k)](phi_k), units of beta/S */
    for (int k = 0; k < n_step_run; ++k) {
      int m_now = ramp_pos(&G, k - 1), m_next = ramp_pos(&G, k);
      work_units += energy_units(&G, m_next, s) - energy_units(&G, m_now, s);
      sweep(&G, m_next, g++, (uint32_t)j, s);
    }
    if (I_out) I_out[j - j0] = -work_units;
    if (spins_out) memcpy(spins_out + (int64_t)(j - j0) * G.nsites, s, (size_t)G.nsites);
  }
  free(s);
  geom_free(&G);
  return EO_OK;
}

/* The two 16-bit fields (v, w) of one site in sweep g and the lazy
 * decision for threshold U (test hook for the decision rule). */
int eo_site_fields(int dim, int lt, int lx, int ly, int n, uint64_t seed, uint32_t g, uint32_t j, int r, int t,
                   int y, int x, uint32_t U, uint32_t* v, uint32_t* w, int* decision) {
  geom G;
  int rc = geom_build(&G, dim, lt, lx, ly, n, 1.0, 0, 1, 1, seed, 0);
  if (rc) return rc;
  *v = sweep_field(&G, 1, g, j, r, t, y, x);
  *w = sweep_field(&G, 2, g, j, r, t, y, x);
  *decision = accept(&G, U, g, j, r, t, y, x);
  geom_free(&G);
  return EO_OK;
}

/* Number of bonds whose coupling the protocol varies (2 n Lx^(D-2)... per ramped column). */
int eo_count_ramped_bonds(int dim, int lt, int lx, int ly, int n, int l) {
  geom G;
  if (geom_build(&G, dim, lt, lx, ly, n, 1.0, l, 1, 1, 0, 0)) return -1;
  int c = 0;
  for (int64_t b = 0; b < G.nb; ++b) c += (G.bk[b] != BOND_BULK);
  geom_free(&G);
  return c;
}

/* Integer energy (units of beta/S) of a +-1 configuration at protocol position m. */
int eo_energy_units(int dim, int lt, int lx, int ly, int n, int l, int N, int m, int flags, const int8_t* s,
                    int64_t* out) {
  geom G;
  int rc = geom_build(&G, dim, lt, lx, ly, n, 1.0, l, N, 1, 0, flags);
  if (rc) return rc;
  if (m < 0 || m > N) { geom_free(&G); return EO_EINVAL; }
  *out = energy_units(&G, m, s);
  geom_free(&G);
  return EO_OK;
}

/* ------------------------------------------------------------------ */
/* Estimator (App. A, Jarzynski's equality)                            */
/* ------------------------------------------------------------------ */
/*
 * out[0] dF      = -log < exp(-W) >,  W_j = -(beta/N) I_j
 * out[1] dS      = dF / (n-1)
 * out[2] dF_err  delete-one jackknife error of dF (NaN if n_t < 2)
 * out[3] w_mean  mean of W
 * out[4] w_var   population variance of W
 * out[5] ess     (sum e)^2 / sum e^2, e_j = exp(-W_j)
 * out[6] i_min, out[7] i_max (as doubles; also returned exactly in imm[2])
 */
int eo_estimate(const int64_t* I, int n_t, double beta, int N, int n_rep, double* out, int64_t* imm) {
  if (n_t < 1 || N < 1 || n_rep < 2) return EO_EINVAL;
  int64_t imax = I[0], imin = I[0];
  for (int j = 1; j < n_t; ++j) {
    if (I[j] > imax) imax = I[j];
    if (I[j] < imin) imin = I[j];
  }
  double s = 0.0, s2 = 0.0;
  for (int j = 0; j < n_t; ++j) {
    double e = exp((beta * (double)(I[j] - imax)) / (double)N);
    s += e;
    s2 += e * e;
  }
  double shift = (beta * (double)imax) / (double)N;
  double dF = -(shift + log(s) - log((double)n_t));
  double err = NAN;
  if (n_t >= 2) {
    double* loo = (double*)malloc(sizeof(double) * n_t);
    if (!loo) return EO_ENOMEM;
    double mean = 0.0;
    for (int i = 0; i < n_t; ++i) {
      double si = 0.0;
      for (int j = 0; j < n_t; ++j)
        if (j != i) si += exp((beta * (double)(I[j] - imax)) / (double)N);
      loo[i] = -(shift + log(si) - log((double)(n_t - 1)));
      mean += loo[i];
    }
    mean /= n_t;
    double acc = 0.0;
    for (int i = 0; i < n_t; ++i) acc += (loo[i] - mean) * (loo[i] - mean);
    err = sqrt((double)(n_t - 1) / (double)n_t * acc);
    free(loo);
  }
  double wm = 0.0;
  for (int j = 0; j < n_t; ++j) wm += -(beta / (double)N) * (double)I[j];
  wm /= n_t;
  double wv = 0.0;
  for (int j = 0; j < n_t; ++j) {
    double d = -(beta / (double)N) * (double)I[j] - wm;
    wv += d * d;
  }
  wv /= n_t;
  out[0] = dF;
  out[1] = dF / (double)(n_rep - 1);
  out[2] = err;
  out[3] = wm;
  out[4] = wv;
  out[5] = s * s / s2;
  out[6] = (double)imin;
  out[7] = (double)imax;
  if (imm) { imm[0] = imin; imm[1] = imax; }
  return EO_OK;
}
