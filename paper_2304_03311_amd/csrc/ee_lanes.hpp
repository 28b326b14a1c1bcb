// ee_lanes.hpp -- how the lanes of a sweep workgroup enumerate the rows of a
// trajectory's colour planes (the lane-map and parity-major orders), where a
// row's glued partner across the cut lies, and the launch-shape choices that
// depend on them.  Pure index arithmetic on the job constants, compiled into
// the kernels and, for the tests of the enumeration, into host code.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define EE_HDI __host__ __device__ __forceinline__
#else
#define EE_HDI inline
#endif

namespace ee {
namespace lanes {

// q = n / d for n < 2^31 with (mul, shift) from make_magic: the high word
// of n * mul plus n, shifted (it stays below 2^32 for such n).
EE_HDI uint32_t fdiv(uint32_t n, uint32_t mul, uint32_t shift) {
  return ((uint32_t)(((uint64_t)n * mul) >> 32) + n) >> shift;
}

// Per-job constants, held in scalar registers.
struct JP {
  int dim, n, lt, ly, l, N, S, subsets, whole, H, G, G8, R, traj_words, packed_row_words;
  uint32_t key0, key1, thr0, thr1, thr2, reverse, spin_format;
  uint32_t pt_hi0, pt_hi1, pt_lo0, pt_lo1;  // byte tables of (thr[a] >> 16) ^ 0x8000, a = 0..7
  uint32_t mR, sR, mLy, sLy;
  const uint32_t* ramp;
  uint32_t* spins;
  int64_t* work;
};


// Per-lane iteration state of one work unit (the same for every sweep): the
// lane owns words w .. w+W-1 of the rows numbered kstart, kstart + kstep,
// ... below kend; wl / wr are the words left and right of that group
// (periodic in x).  The first row is (r0, t0, y0) at word offset rowbase0;
// each next row is dr replicas, dt time slices and dy rows of y further
// on, step words further in storage; when t wraps, r moves by rinc and the
// offset back by wrapadj.
struct Lane {
  int w, wl, wr;
  int kstart, kstep, kend, rowbase0, step;
  int r0, t0, y0;
  int dr, dt, dy;
  int rinc, wrapadj;
};

// Lane map of the rows of one colour plane (n replicas x R = lt*ly rows of G
// words) over T lanes, GW = G/W lanes per row, S = T/GW row slots.
//  * groups and S >= n: slot s takes replica s / B, B = S/n, and rows k, k+B, ... of
//    that replica in the order rho = (k + 2 ly) mod R, so that the rows
//    next to the cut (t = 0, 1) come last: one iteration of the lane's loop
//    meets them instead of one per replica.
//  * otherwise: slot s takes rows s, s+S, ... of the planes in storage order.
//    The streaming kernel keeps this order: its rows come from HBM through
//    the caches, and it measured 11% faster than the grouped order.
// The rows of a colour are independent within a half-sweep, so the order
// does not change any result.  Divisions by R and ly use the job's magic
// multipliers (the streaming kernel builds this map at every launch).
EE_HDI Lane make_lane(const JP& P, int lt_, int T, int W, bool groups) {
  const int GW = P.G / W;
  const int S = T / GW;
  const int slot = lt_ / GW;
  const auto div_ly = [&](int v) { return (int)fdiv((uint32_t)v, P.mLy, P.sLy); };
  const auto div_R = [&](int v) { return (int)fdiv((uint32_t)v, P.mR, P.sR); };
  Lane ln;
  ln.w = (lt_ - slot * GW) * W;
  ln.wl = (ln.w == 0) ? P.G - 1 : ln.w - 1;
  ln.wr = (ln.w + W == P.G) ? 0 : ln.w + W;
  if (groups && S >= P.n) {
    const int B = S / P.n;
    ln.r0 = slot / B;
    const int k0 = slot - ln.r0 * B;
    ln.kstart = k0;
    ln.kstep = B;
    ln.kend = (ln.r0 < P.n) ? P.R : 0;
    int rho = k0 + 2 * P.ly;
    if (rho >= P.R) rho -= P.R;
    ln.t0 = div_ly(rho);
    ln.y0 = rho - ln.t0 * P.ly;
    ln.rowbase0 = (ln.r0 * P.R + rho) * P.G;
    ln.step = B * P.G;
    const int b = B - div_R(B) * P.R;  // B mod R
    ln.dr = 0;
    ln.dt = div_ly(b);
    ln.dy = b - ln.dt * P.ly;
    ln.rinc = 0;
    ln.wrapadj = P.R * P.G;
  } else {
    ln.kstart = slot;
    ln.kstep = S;
    ln.kend = (slot < S) ? P.n * P.R : 0;
    ln.r0 = div_R(slot);
    const int rho = slot - ln.r0 * P.R;
    ln.t0 = div_ly(rho);
    ln.y0 = rho - ln.t0 * P.ly;
    ln.rowbase0 = slot * P.G;
    ln.step = S * P.G;
    ln.dr = div_R(S);
    const int b = S - ln.dr * P.R;
    ln.dt = div_ly(b);
    ln.dy = b - ln.dt * P.ly;
    ln.rinc = 1;
    ln.wrapadj = 0;
  }
  return ln;
}


// Row (in the lane's own trajectory) of the glued partner across the cut of
// row (r, t, y), t in {0, 1}: replica r+1 at t = 1 for t = 0, replica r-1 at
// t = 0 for t = 1.
EE_HDI int glued_row(const JP& P, int r, int t, int y) {
  const int rgl = (t == 0) ? ((r + 1 == P.n) ? 0 : r + 1) : ((r == 0) ? P.n - 1 : r - 1);
  return rgl * P.R + (1 - t) * P.ly + y;
}

// Byte mask of the glued sites (x < l) of a word whose first site has
// x = l - v: bytes i with 2i < v.
EE_HDI uint32_t glued_mask(int v) {
  const int ng = (v <= 0) ? 0 : ((v + 1) >> 1);
  return (ng >= 4) ? 0xFFFFFFFFu : ((1u << (8 * ng)) - 1u);
}


// Parity-major row order (grouped lane map, rows of whole words).  The rows
// (t, y) of a replica fall into two classes by the parity q of t + y, and in
// a half-sweep of colour c the sites of the class-q rows have x parity
// p = c ^ q.  Slot k0 of the B slots of its replica takes the class-q rows
// m = k0, k0 + B, ... below R/2 of both classes, one row of each class per
// step: the lanes of a wave meet rows of one class at a time, so p is a
// compile-time constant of each row's code, and the next rows are a fixed
// stride further on.
//   2D: t = 2m + q, so the class-1 row is the row after the class-0 one.
//   3D, ly dividing B: t = m / (ly/2) and y = 2 (m mod ly/2) + ((t + q) & 1):
//   both rows share t, their y differ in bit 0, and t moves by 2B/ly (even)
//   from step to step, so both y stay fixed per lane.
// The rows of one colour are independent within a half-sweep, so the order
// changes no result.  LanePM holds what is fixed for a work unit: the
// lane's first class-0 row (t, word offset rw, Philox counter word 0, y),
// the offsets d_rw, d_c0 of its class-1 partner, the y of both rows and
// their y-neighbour offsets; dt is the t stride (uniform).
// For the lane's rows next to the cut (if any) it also holds their glued
// rows' word offsets og and the byte masks gm[p] of the glued columns x < l
// of its words for x parity p.
struct LanePM {
  int w, wl, wr, r0, dt;
  uint32_t c3;  // Philox counter word 3 without the colour bit
  int t, rw, d_rw;
  uint32_t c0, d_c0;
  int y[2], ymo[2], ypo[2];
  int og[2];
  uint32_t gm[2][4];
};

template <int DIM, int W>
EE_HDI LanePM make_lane_pm(const JP& P, int lt_, int T) {
  const int GW = P.G / W;
  const int slot = lt_ / GW;
  const int B = (T / GW) / P.n;
  LanePM L;
  L.w = (lt_ - slot * GW) * W;
  L.wl = (L.w == 0) ? P.G - 1 : L.w - 1;
  L.wr = (L.w + W == P.G) ? 0 : L.w + W;
  L.r0 = slot / B;
  const int k0 = slot - L.r0 * B;
  L.dt = (DIM == 2) ? 2 * B : (int)fdiv((uint32_t)(2 * B), P.mLy, P.sLy);
  L.c3 = (1u << 28) | ((uint32_t)L.r0 << 1);
  int t, y0, y1;
  if (DIM == 2) {
    t = 2 * k0;
    y0 = y1 = 0;
  } else {
    t = (int)fdiv((uint32_t)(2 * k0), P.mLy, P.sLy);
    y0 = 2 * (k0 - t * (P.ly >> 1)) + (t & 1);
    y1 = y0 ^ 1;
  }
  const int rho0 = t * P.ly + y0;
  const int rho1 = (DIM == 2) ? rho0 + 1 : t * P.ly + y1;
  L.t = (L.r0 < P.n) ? t : P.lt;  // a slot past the last replica has no rows
  L.rw = (L.r0 * P.R + rho0) * P.G + L.w;
  L.d_rw = (rho1 - rho0) * P.G;
  L.c0 = (uint32_t)(rho0 * P.G8 + (L.w >> 1));
  L.d_c0 = (uint32_t)((rho1 - rho0) * P.G8);
  L.y[0] = y0;
  L.y[1] = y1;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    L.ymo[q] = (L.y[q] == 0) ? (P.ly - 1) * P.G : -P.G;
    L.ypo[q] = (L.y[q] == P.ly - 1) ? -(P.ly - 1) * P.G : P.G;
    // the class-q row of the lane's first step (2D: t = q, 3D: t), if next to the cut
    const int tq = (DIM == 2) ? t + q : t;
    L.og[q] = (L.t <= 1) ? glued_row(P, L.r0, tq, L.y[q]) * P.G + L.w : 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) L.gm[q][i] = (i < W) ? glued_mask(P.l - q - 8 * (L.w + i)) : 0u;
  }
  return L;
}


// Words per lane for a job and slot size of T lanes.  The widest W <= 4
// that divides the row's words and still gives every row a lane group
// (rows of exactly three words take W = 3) needs the fewest passes of the
// slot's lanes over its row groups; of the W that need as many passes, the
// narrowest is taken: each pass is then a shorter instruction chain, and a
// slot with more lanes than wide row groups (a small, latency-bound
// lattice) spreads its rows over all of its lanes.
EE_HDI int words_per_lane(const JP& P, int T) {
  const int nrows = P.n * P.R;  // rows of one colour of a trajectory
  const auto passes = [&](int W) { return (nrows * (P.G / W) + T - 1) / T; };
  int W = 1;
  if ((P.H & 15) == 0 && T / (P.G / 4) >= 1) W = 4;
  else if (P.H == 12) W = 3;
  else if ((P.H & 7) == 0 && T / (P.G / 2) >= 1) W = 2;
  const int p = passes(W);
  if (W == 4 && passes(2) == p) W = 2;
  if (W > 1 && passes(1) == p) W = 1;
  return W;
}

// Whether the rows of a unit go in parity-major order: the grouped lane map
// (at least one row slot per replica), fewer row slots B per replica than
// rows (else half of them would idle there, while the lane-map order gives
// every row its own lane), and, in 3D, ly dividing B.  Uniform over the
// workgroup.
EE_HDI bool use_pm(const JP& P, int T, int W) {
  const int S = T / (P.G / W);
  if (S < P.n) return false;
  const int B = S / P.n;
  return B < P.R && (P.dim == 2 || B % P.ly == 0);
}

}  // namespace lanes
}  // namespace ee
